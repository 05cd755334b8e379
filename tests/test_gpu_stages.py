"""Step-by-step parity: the matrix-core GEMM on random data, and every
intermediate array of the right-hand side (U^f, C^f, Q~, Q, Q^f, F~, D~)
against the oracle's recorded intermediates."""
import numpy as np
import pytest

import frcases as C
from oracle import Discretisation

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("M,K1,K2,N", [(16, 4, 0, 16), (16, 16, 0, 1600), (96, 64, 0, 320),
                                       (192, 96, 64, 640), (125, 150, 375, 96), (150, 125, 0, 48),
                                       (7, 3, 5, 32), (375, 150, 125, 64)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_gemm_random(M, K1, K2, N, prec):
    import torch
    import paper_1312_1638_amd as P
    rng = np.random.default_rng(M + K1 + K2 + N)
    A = rng.standard_normal((M, K1 + K2))
    B1 = rng.standard_normal((K1, N))
    B2 = rng.standard_normal((K2, N)) if K2 else None
    dB1 = torch.from_numpy(B1).cuda()
    dB2 = torch.from_numpy(B2).cuda() if K2 else None
    got = P.binding.debug_gemm(A, dB1, dB2, prec).double().cpu().numpy()
    B = B1 if not K2 else np.concatenate([B1, B2])
    ref = A @ B
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"gemm {M}x{K1}+{K2}x{N} {prec}: max rel {err:.2e}")
    assert err < {"fp64": 1e-14, "fp32": 2e-6, "bf16x3": 6e-5}[prec]


SHAPES = [(1, 1), (1, 2), (1, 4), (2, 1), (2, 2), (2, 4), (3, 1), (3, 2), (3, 4), (4, 1),
          (4, 2), (4, 4), (6, 1), (6, 2), (6, 4), (8, 1), (8, 2), (12, 1), (12, 2)]


TOL = {"fp64": 1e-14, "fp32": 2e-6, "bf16x3": 6e-5}


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_gemm_every_tile_shape(prec):
    """Every instantiated (row blocks, column strips) shape, with a ragged M,
    ragged K in both panels and a column count not divisible by the strip
    width."""
    import torch
    import paper_1312_1638_amd as P
    rng = np.random.default_rng(11)
    M, K1, K2, N = 150, 37, 22, 16 * 13
    A = rng.standard_normal((M, K1 + K2))
    B1 = rng.standard_normal((K1, N))
    B2 = rng.standard_normal((K2, N))
    ref = A @ np.concatenate([B1, B2])
    dB1, dB2 = torch.from_numpy(B1).cuda(), torch.from_numpy(B2).cuda()
    MB = (M + 15) // 16
    for mbw, nc in SHAPES:
        wm = -(-MB // mbw)
        got = P.binding.debug_gemm(A, dB1, dB2, prec, (mbw, nc, wm)).double().cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err < TOL[prec], (mbw, nc, wm, err)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sparse_row_kernel(prec):
    """The sparse-row operator kernel: a random operator with a few non-zeros
    per row (ragged M, both panels, columns in a ragged last workgroup) and
    the library's own line-structured hex operators, for several rows per
    workgroup; it must equal the dense product."""
    import torch
    import paper_1312_1638_amd as P
    rng = np.random.default_rng(13)
    cases = []
    M, K1, K2, N = 151, 40, 23, 16 * 21
    A = rng.standard_normal((M, K1 + K2)) * (rng.random((M, K1 + K2)) < 0.1)
    cases.append((A, K1, N))
    m0 = P.binding.reference_operator("hex", 4, 0)
    m3 = P.binding.reference_operator("hex", 4, 1)
    m1p = P.binding.reference_operator("hex", 4, 4)
    cases.append((m0, m0.shape[1], 16 * 40))
    cases.append((np.concatenate([m1p, m3], 1), m1p.shape[1], 16 * 17))
    for A, K1, N in cases:
        M, K = A.shape
        B = rng.standard_normal((K, N))
        ref = A @ B
        dB1 = torch.from_numpy(B[:K1].copy()).cuda()
        dB2 = torch.from_numpy(B[K1:].copy()).cuda() if K > K1 else None
        for rpg in (1, 4, 7, 16, 64):
            got = P.binding.debug_gemm(A, dB1, dB2, prec, (0, rpg, 0)).double().cpu().numpy()
            err = np.abs(got - ref).max() / np.abs(ref).max()
            assert err < TOL[prec], (A.shape, rpg, err)


@pytest.mark.parametrize("plan", [(0, 0, 0), (0, 1, 0), (0, 5, 0), (2, 2, 2)])
def test_operands_with_a_row_stride_beyond_n(plan):
    """B1 and B2 as column slices of wider arrays (row stride ldb > N): the
    sparse-row kernel's byte offsets and the matrix-core loads follow ldb."""
    import torch
    import paper_1312_1638_amd as P
    rng = np.random.default_rng(17)
    m1p = P.binding.reference_operator("hex", 3, 4)
    m3 = P.binding.reference_operator("hex", 3, 1)
    A = np.concatenate([m3, m1p], 1)
    K1 = m3.shape[1]
    K2 = m1p.shape[1]
    N, ldb = 16 * 9, 16 * 9 + 40
    W1 = rng.standard_normal((K1, ldb))
    W2 = rng.standard_normal((K2, ldb))
    dB1 = torch.from_numpy(W1).cuda()[:, :N]
    dB2 = torch.from_numpy(W2).cuda()[:, :N]
    assert dB1.stride(0) == ldb and dB2.stride(0) == ldb
    ref = A @ np.concatenate([W1[:, :N], W2[:, :N]])
    got = P.binding.debug_gemm(A, dB1, dB2, "fp64", plan).cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"strided operands, plan {plan}: max rel {err:.2e}")
    assert err < TOL["fp64"]


def test_row_stride_below_n_is_rejected():
    """Overlapping rows (ldb < N) are refused before any launch."""
    import torch
    import paper_1312_1638_amd as P
    A = np.eye(16)
    base = torch.zeros(16 * 64, dtype=torch.float64, device="cuda")
    B = base.as_strided((16, 32), (16, 1))
    with pytest.raises(P.binding.FRError) as e:
        P.binding.debug_gemm(A, B, None, "fp64", (0, 1, 0))
    assert e.value.status == P.binding.FR_EINVAL


def test_sparse_plan_rejected_for_dense_operator():
    import torch
    import paper_1312_1638_amd as P
    A = np.ones((32, 16))
    B = torch.ones((16, 32), dtype=torch.float64, device="cuda")
    with pytest.raises(P.binding.FRError):
        P.binding.debug_gemm(A, B, None, "fp64", (0, 8, 0))


def _split(s, flat, rows_per_block, nvars):
    """Internal scratch array -> per-block [rows, alpha, n] (padding removed)."""
    out, off = [], 0
    for blk, rows in zip(s.blocks, rows_per_block):
        ld, ne = blk["ld"], blk["nelem"]
        a = flat[off:off + rows * nvars * ld].reshape(rows, nvars, ld)[:, :, :ne]
        out.append(a)
        off += rows * nvars * ld
    return out


@pytest.mark.parametrize("name", ["vortex7_p3", "mixed6_p3_euler", "tgv4_p1", "tgv3_p4",
                                  "mixed5_p2_ns", "curved3_p2_ns"])
def test_stage_parity(name):
    import paper_1312_1638_amd as P
    w = C.SMALL[name]()
    d = Discretisation(w)
    u = C.perturbed(d, d.initial_state(w))
    rec = {}
    ref_out = d.rhs(u, rec)
    s = C.solver_for(w)
    t = s.pack(u)
    D, NV = d.ndims, d.nvars
    nf = [r.nfpts for r in d.refs]
    nu = [r.nupts for r in d.refs]
    stages = [(1, "uf", nf, None)]
    if w.system == "ns":
        stages += [(2, "cf", nf, None), (3, "qt", [D * n for n in nu], D),
                   (4, "q", [D * n for n in nu], D), (5, "qf", [D * n for n in nf], D)]
    stages += [(6, "ft", [D * n for n in nu], D), (7, "df", nf, None)]
    for st, key, rows, vec in stages:
        flat = s.debug_stage(t, st).cpu().numpy()
        if st == 2:
            # C^f lives in the first N^f rows of each block's Q^f region
            parts, off = [], 0
            for blk, r in zip(s.blocks, nf):
                ld, ne = blk["ld"], blk["nelem"]
                parts.append(flat[off:off + r * NV * ld].reshape(r, NV, ld)[:, :, :ne])
                off += D * r * NV * ld
            got = parts
        else:
            got = _split(s, flat, rows, NV)
        ref = rec[key]
        if vec:
            ref = [x.reshape((-1,) + x.shape[2:]) for x in ref]
        err = C.rel_l2(got, ref)
        print(f"{name} stage {st} ({key}): rel L2 {err:.3e}", flush=True)
        assert err < 1e-12, (name, key, err)
    err = C.rel_l2(s.unpack(s.rhs(t)), ref_out)
    assert err < 1e-12
