"""CPU-only checks of the HIP library: it loads, exports the declared ABI,
and its host set-up (operators, metrics, pairing, error paths) agrees with
the oracle's independent construction.  No device call is made."""
import os
import re

import numpy as np
import pytest

from oracle import reference as oref
from workloads import configs, meshes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

P = pytest.importorskip("paper_1312_1638_amd")


def _lib():
    try:
        return P.load_library()
    except FileNotFoundError:
        pytest.skip("libfr.so not built")


def test_exports_every_declared_symbol():
    L = _lib()
    with open(os.path.join(ROOT, "include", "fr.h")) as fh:
        hdr = fh.read()
    declared = set(re.findall(r"\b(fr_[a-z0-9_]+)\s*\(", hdr))
    assert len(declared) >= 12
    for name in declared:
        assert hasattr(L, name), name
    assert set(P.binding.EXPORTS) <= declared


CASES = [("quad", p) for p in (1, 2, 3, 4, 6)] + [("tri", p) for p in (1, 2, 3, 4, 5)] + \
        [("hex", p) for p in (1, 2, 3, 4)]


@pytest.mark.parametrize("etype,p", CASES)
def test_operators_match_oracle(etype, p):
    _lib()
    r = oref.ref_element(etype, p)
    D, Nu = r.ndims, r.nupts
    assert np.allclose(P.reference_operator(etype, p, 5), r.upts, atol=1e-14)
    assert np.allclose(P.reference_operator(etype, p, 0), r.L_f, atol=1e-13)
    assert np.allclose(P.reference_operator(etype, p, 1), r.divg, atol=5e-13)
    M4 = np.concatenate([r.D_u[i] for i in range(D)], 0)
    assert np.allclose(P.reference_operator(etype, p, 10), M4, atol=1e-12)
    assert np.allclose(P.reference_operator(etype, p, 8)[:, 0], r.W, atol=1e-14)
    assert np.allclose(P.reference_operator(etype, p, 9)[:, 0], r.fweight, atol=1e-14)


@pytest.mark.parametrize("scheme", ["sd", "hu"])
@pytest.mark.parametrize("etype,p", [("quad", p) for p in range(1, 7)]
                         + [("hex", p) for p in range(1, 5)])
def test_sd_hu_correction_matches_oracle(etype, p, scheme):
    """The library's SD/HU correction divergence (VCJH closed form through
    the Legendre recurrences) against the oracle's (Legendre series and
    Lagrange factors); the other operators are those of DG."""
    _lib()
    r = oref.ref_element(etype, p, scheme)
    M3 = P.reference_operator(etype, p, 1, scheme)
    assert np.max(np.abs(M3 - r.divg)) < 1e-13 * max(1.0, np.max(np.abs(r.divg)))
    assert np.allclose(P.reference_operator(etype, p, 0, scheme), P.reference_operator(etype, p, 0))
    assert np.allclose(P.reference_operator(etype, p, 10, scheme),
                       P.reference_operator(etype, p, 10))


def test_sd_hu_rejected_on_triangles():
    _lib()
    with pytest.raises(P.FRError) as e:
        P.reference_operator("tri", 3, 1, "sd")
    assert e.value.status == P.binding.FR_EUNSUPPORTED
    L = P.binding.load_library()
    import ctypes
    assert L.fr_reference_operator(0, 3, 7, 1, None, 0, None, None) == P.binding.FR_EINVAL


@pytest.mark.parametrize("scheme", ["dg", "sd", "hu"])
@pytest.mark.parametrize("etype,p", [("quad", 3), ("tri", 3), ("hex", 3), ("hex", 4)])
def test_premultiplied_operators_reproduce_direct_form(etype, p, scheme):
    """Appendix A: M6 C + (M4 - M6 M0) U equals the direct transformed
    gradient (eq. transqu) and M3 D + (M1 - M3 M2) F the direct divergence
    (eq. tdivflux), on random data, with the oracle's operator values."""
    if etype == "tri" and scheme != "dg":
        pytest.skip("SD and HU are built for tensor elements only")
    _lib()
    r = oref.ref_element(etype, p, scheme)
    D, Nu, Nf = r.ndims, r.nupts, r.nfpts
    rng = np.random.default_rng(p)
    m = 7
    U = rng.standard_normal((Nu, m))
    C = rng.standard_normal((Nf, m))
    Fd = rng.standard_normal((Nf, m))
    Ft = rng.standard_normal((D, Nu, m))
    M6 = P.reference_operator(etype, p, 3, scheme)
    M4p = P.reference_operator(etype, p, 2, scheme)
    M3 = P.reference_operator(etype, p, 1, scheme)
    M1p = P.reference_operator(etype, p, 4, scheme)
    lib_q = (M6 @ C + M4p @ U).reshape(D, Nu, m)
    uf = r.L_f @ U
    direct_q = np.einsum("irv,vm->irm", r.D_u, U) + np.einsum("rs,si,sm->irm", r.divg, r.fnorm, C - uf)
    assert np.allclose(lib_q, direct_q, atol=1e-11)
    lib_div = M3 @ Fd + M1p @ Ft.reshape(D * Nu, m)
    fperp = np.einsum("sr,si,irm->sm", r.L_f, r.fnorm, Ft)
    direct_div = np.einsum("irv,ivm->rm", r.D_u, Ft) + r.divg @ (Fd - fperp)
    assert np.allclose(lib_div, direct_div, atol=1e-11)


def test_unsupported_order():
    _lib()
    with pytest.raises(P.FRError) as e:
        P.reference_operator("hex", 5, 0)
    assert e.value.status == P.binding.FR_EUNSUPPORTED


def test_pairing_counts():
    _lib()
    w = configs.vortex_quads(5, 3)
    assert P.check_mesh(w.mesh) == 2 * 25 * 4
    w = configs.taylor_green_hexes(3, 2)
    assert P.check_mesh(w.mesh, "ns") == 3 * 27 * 9
    rng = np.random.default_rng(1)
    m = meshes.mixed_mesh(4, 4, order=2, split=rng.random(16) < 0.5, diag=rng.integers(0, 2, 16))
    ntri = m.blocks[1].nelem if len(m.blocks) > 1 else 0
    nq = m.blocks[0].nelem
    assert P.check_mesh(m) == (nq * 12 + ntri * 9) // 2


def test_inverted_element_is_a_mesh_error():
    _lib()
    w = configs.vortex_quads(4, 2)
    nodes = w.mesh.blocks[0].nodes.copy()
    nodes[0] = nodes[0][[1, 0, 3, 2]]
    w.mesh.blocks[0] = meshes.Block("quad", 2, 1, nodes)
    with pytest.raises(P.FRError) as e:
        P.check_mesh(w.mesh)
    assert e.value.status == P.binding.FR_EMESH


def test_mismatched_faces_are_a_mesh_error():
    _lib()
    w = configs.vortex_quads(4, 2)
    bad = w.mesh.pairs.copy()
    bad["shift"][0, 1] += 0.3
    with pytest.raises(P.FRError) as e:
        P.check_mesh(meshes.Mesh(2, w.mesh.blocks, bad, info=w.mesh.info))
    assert e.value.status == P.binding.FR_EMESH


def test_unpaired_flux_points_are_a_mesh_error():
    _lib()
    w = configs.vortex_quads(4, 2)
    with pytest.raises(P.FRError) as e:
        P.check_mesh(meshes.Mesh(2, w.mesh.blocks, w.mesh.pairs[:-1], info=w.mesh.info))
    assert e.value.status == P.binding.FR_EMESH


def test_solver_refuses_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(RuntimeError):
        P.Solver(configs.vortex_quads(3, 1).mesh)


@pytest.mark.parametrize("ndims,etype,nelem", [(3, "hex", 1 << 27), (2, "quad", 1 << 27),
                                               (3, "hex", 1 << 40)])
def test_block_too_large_is_rejected(ndims, etype, nelem):
    """The operator kernels address one row of a block (N_V ld values) with
    32-bit byte offsets: a block with N_V nelem >= 2^29 is refused up front,
    before its nodes are read (here they hold a single element)."""
    import ctypes
    L = _lib()
    nodes = np.zeros((1, 2 ** ndims, ndims))
    blk = P.binding.FrBlock(etype=P.binding.ETYPE[etype], order=1, geom_order=1, correction=0,
                            nelem=nelem, nodes=nodes.ctypes.data, problem=None)
    cfg = P.binding._config(ndims, "euler", "fp64", 1.4, 0.0, 0.72, 0.5, 0.1, 0, 1)
    n = ctypes.c_int64()
    st = L.fr_check_mesh(ctypes.byref(cfg), 1, ctypes.byref(blk), 0, None, ctypes.byref(n))
    assert st == P.binding.FR_EINVAL
    assert "too large" in L.fr_last_error(None).decode()


def _one_quad_block(nelem, etype="quad", ndims=2):
    nodes = np.zeros((max(nelem, 1), 2 ** ndims, ndims))
    return P.binding.FrBlock(etype=P.binding.ETYPE[etype], order=1, geom_order=1, correction=0,
                             nelem=nelem, nodes=nodes.ctypes.data, problem=None), nodes


@pytest.mark.parametrize("case", ["no blocks", "block without elements", "ndims 4",
                                  "hex in 2-D", "quad in 3-D"])
def test_degenerate_meshes_are_refused(case):
    """Empty and inconsistent meshes are refused by the host check with
    FR_EINVAL and a message, before anything is allocated."""
    import ctypes
    L = _lib()
    ndims = {"ndims 4": 4, "hex in 2-D": 2, "quad in 3-D": 3}.get(case, 2)
    etype = {"hex in 2-D": "hex", "quad in 3-D": "quad"}.get(case, "quad")
    blk, _nodes = _one_quad_block(0 if case == "block without elements" else 1, etype,
                                  3 if etype == "hex" else 2)
    cfg = P.binding._config(ndims, "euler", "fp64", 1.4, 0.0, 0.72, 0.5, 0.1, 0, 1)
    n = ctypes.c_int64()
    nblocks = 0 if case == "no blocks" else 1
    st = L.fr_check_mesh(ctypes.byref(cfg), nblocks, ctypes.byref(blk), 0, None, ctypes.byref(n))
    assert st == P.binding.FR_EINVAL, (case, st)
    assert L.fr_last_error(None).decode()
