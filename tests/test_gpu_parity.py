"""Parity of the HIP library (through the C ABI) with the FP64 oracle.

Tolerances: relative L2 over the whole SoA vector (every block and field),
and over each field on its own (so that a small field, such as momentum
beside the energy of a low-Mach flow, is held to the bar by itself).
u after RK4 steps: 1e-12 (FP64) and 1e-5 (FP32 operator path), the stated
bars.  du/dt: the stated bar, unless the case is ill-conditioned -- du/dt is
a small difference of flux derivatives much larger than itself (low-Mach
energy equation, a perturbed free stream) -- in which case the bar is four
times the case's measured FP64 rounding floor (the oracle's own distance
from a long-double evaluation of the same formula, whole-vector or per
field), times 2^29 for FP32 operands.  Errors are then measured against the
long-double evaluation.
"""
import numpy as np
import pytest

import frcases as C
from oracle import Discretisation
from workloads import configs

pytestmark = pytest.mark.gpu


def _both(w, prec="fp64", perturb=True):
    d = Discretisation(w)
    u = d.initial_state(w)
    if perturb:
        u = C.perturbed(d, u)
    s = C.solver_for(w, prec)
    return d, s, u


@pytest.mark.parametrize("name", sorted(C.SMALL))
def test_rhs_small(name):
    w = C.SMALL[name]()
    d, s, u = _both(w)
    ref = d.rhs(u)
    got = s.unpack(s.rhs(s.pack(u)))
    err = C.rel_l2(got, ref)
    print(f"{name}: rel L2 {err:.3e}")
    assert err < 1e-12
    _tol, ext, _floor = C.floor_tolerance(d, u, 1e-12)
    C.check_fields(name, got, ext, ext.field_tol)


@pytest.mark.parametrize("name", ["vortex7_p3", "mixed6_p3_euler", "tgv5_p3", "curved4_p4"])
def test_rhs_small_fp32(name):
    w = C.SMALL[name]()
    d, s, u = _both(w, "fp32")
    tol, ext, floor = C.floor_tolerance(d, u, 1e-5, C.FP32_OVER_FP64)
    got = s.unpack(s.rhs(s.pack(u)))
    err = C.rel_l2(got, ext)
    print(f"{name} fp32: rel L2 {err:.3e} (fp64 floor {floor:.2e}, tol {tol:.2e})")
    assert err < tol
    C.check_fields(f"{name} fp32", got, ext, ext.field_tol)


@pytest.mark.parametrize("name", ["vortex7_p3", "mixed6_p3_euler", "tgv5_p3", "curved4_p4"])
def test_rhs_small_bf16x3(name):
    """Split-precision bf16 operator products: du/dt within the error model
    (~2^-16 relative per product, amplified by the case's conditioning) and
    u after 5 RK4 steps within 1e-5."""
    w = C.SMALL[name]()
    d, s, u = _both(w, "bf16x3")
    tol, ext, floor = C.floor_tolerance(d, u, 1e-4, C.BF16X3_OVER_FP64)
    t = s.pack(u)
    got = s.unpack(s.rhs(t))
    err = C.rel_l2(got, ext)
    dt = 1e-4
    s.step(t, dt, 5)
    ref_u = d.rk4(u, dt, 5)
    eu = C.rel_l2(s.unpack(t), ref_u)
    print(f"{name} bf16x3: rhs rel L2 {err:.3e} (tol {tol:.2e}), u(5) {eu:.3e}")
    assert err < tol and eu < 1e-5
    C.check_fields(f"{name} bf16x3 rhs", got, ext, ext.field_tol)
    C.check_fields(f"{name} bf16x3 u(5)", s.unpack(t), ref_u,
                   C.state_bar(ref_u, u, 1e-5, ext.field_tol))


def _force_plans(s, w, variant):
    """Force one kernel family on every operator product of every block:
    'mfma' (matrix cores), 'sparse' (sparse-row, 4 rows per workgroup),
    'fused' (sparse-row, the gradient transform fused into step 3), the
    same two with every field of an element in one thread ('fields',
    'fused_fields'), the latter with the transformed flux of step 6 fused
    as well ('fused_flux'), and the LDS-staged kernel ('staged',
    'staged_fused').  Dense triangle operators have no sparse-row form and
    keep their plan."""
    import paper_1312_1638_amd as P
    steps = [1, 3, 5, 8] if w.system == "ns" else [1, 8]
    forced = 0
    for bi, b in enumerate(w.mesh.blocks):
        nu = s.blocks[bi]["nupts"]
        nf = P.reference_operator(b.etype, b.order, 6).shape[0]
        rows = {1: nf, 3: s.ndims * nu, 5: nf, 8: nu}
        for st in steps:
            if variant == "mfma":
                plan = (1, 1, -(-rows[st] // 16))
            elif variant == "sparse":
                plan = (0, 4, 0)
            elif variant == "fields":
                plan = (0, 5, 2)
            elif variant == "fused":
                plan = (0, 3, 1) if st == 3 else (0, 7, 0)
            elif variant == "staged":
                plan = (0, 64, 4)
            elif variant == "staged_fused":
                plan = (0, 64, 5) if st == 3 else (0, 64, 4)
            elif variant == "fused_flux":
                plan = (0, 2, 11) if st == 3 else (0, 3, 2)
            else:
                plan = (0, 2, 3) if st == 3 else (0, 3, 2)
            try:
                s.set_plan(bi, st, plan)
            except P.FRError:
                # dense triangle operators have no sparse form; the staged
                # kernel holds at most 160 rows (64 points when fused)
                assert variant != "mfma" and (b.etype == "tri" or variant.startswith("staged"))
                continue
            assert s.gemm_plan(bi, st) == plan
            forced += 1
    assert forced > 0


@pytest.mark.parametrize("name", ["tgv3_p4", "mixed5_p2_ns", "curved3_p2_ns", "vortex7_p3",
                                  "mixed6_p3_euler", "tgv5_p3", "vortex4_p6", "mixed5_p4_euler"])
@pytest.mark.parametrize("variant", ["mfma", "sparse", "fused", "fields", "fused_fields",
                                     "fused_flux", "staged", "staged_fused"])
def test_every_kernel_variant(name, variant):
    """du/dt and u after 3 RK4 steps (captured graph) with every operator
    product forced onto one kernel family.  The cases cover every ELL width
    the quad and hex operators use (2 to 21 entries per row)."""
    w = C.SMALL[name]()
    d, s, u = _both(w)
    _force_plans(s, w, variant)
    ref, ext, ref_u = _variant_refs(name, d, u)
    got = s.unpack(s.rhs(s.pack(u)))
    err = C.rel_l2(got, ref)
    t = s.pack(u)
    dt = 1e-4
    s.step(t, dt, 3)
    eu = C.rel_l2(s.unpack(t), ref_u)
    print(f"{name} {variant}: rhs rel L2 {err:.3e}, u(3) {eu:.3e}")
    assert err < 1e-12 and eu < 1e-12
    C.check_fields(f"{name} {variant} rhs", got, ext, ext.field_tol)
    C.check_fields(f"{name} {variant} u(3)", s.unpack(t), ref_u,
                   C.state_bar(ref_u, u, 1e-12, ext.field_tol))


_VARIANT_REFS = {}


def _variant_refs(name, d, u):
    """The oracle's du/dt, its long-double evaluation (with per-field bars at
    the stated 1e-12) and u after 3 RK4 steps of 1e-4, once per case."""
    if name not in _VARIANT_REFS:
        _tol, ext, _floor = C.floor_tolerance(d, u, 1e-12)
        _VARIANT_REFS[name] = (d.rhs(u), ext, d.rk4(u, 1e-4, 3))
    return _VARIANT_REFS[name]


@pytest.mark.parametrize("name", ["tgv3_p4", "mixed5_p2_ns", "curved3_p2_ns"])
def test_fused_flux_matches_the_separate_flux(name):
    """FP64: the transformed flux computed in step 3's epilogue is the same
    formula as step 6's kernel; only the compiler's multiply-add
    contraction may differ between the two kernels, so du/dt agrees to the
    case's rounding floor."""
    w = C.SMALL[name]()
    d, s, u = _both(w)
    t = s.pack(u)
    out = []
    for variant in ("fused_fields", "fused_flux"):
        _force_plans(s, w, variant)
        out.append(s.unpack(s.rhs(t)))
    _tol, _ext, floor = C.floor_tolerance(d, u, 1e-12)
    diff = C.rel_l2(out[1], out[0])
    print(f"{name}: fused vs separate flux rel L2 {diff:.2e} (floor {floor:.2e})")
    assert diff <= max(floor, 1e-15)


@pytest.mark.parametrize("variant", ["fused", "fused_fields", "fused_flux", "staged_fused"])
def test_fused_gradient_transform_fp32(variant):
    w = C.SMALL["tgv5_p3"]()
    d, s, u = _both(w, "fp32")
    _force_plans(s, w, variant)
    tol, ext, floor = C.floor_tolerance(d, u, 1e-5, C.FP32_OVER_FP64)
    got = s.unpack(s.rhs(s.pack(u)))
    err = C.rel_l2(got, ext)
    print(f"tgv5_p3 fp32 {variant}: rel L2 {err:.3e} (tol {tol:.2e})")
    assert err < tol
    C.check_fields(f"tgv5_p3 fp32 {variant}", got, ext, ext.field_tol)


@pytest.mark.parametrize("name", ["tgv3_p4", "curved4_p4", "mixed5_p4_euler"])
def test_staged_kernel_fp32(name):
    """FP32 with every sparse operator product forced onto the LDS-staged
    kernel: du/dt, and u after 3 RK4 steps (the staged kernel's RK4
    epilogue in the captured graph), against the oracle at the FP32 bars."""
    w = C.SMALL[name]()
    d, s, u = _both(w, "fp32")
    _force_plans(s, w, "staged")
    tol, ext, floor = C.floor_tolerance(d, u, 1e-5, C.FP32_OVER_FP64)
    got = s.unpack(s.rhs(s.pack(u)))
    err = C.rel_l2(got, ext)
    t = s.pack(u)
    s.step(t, 1e-4, 3)
    ref_u = d.rk4(u, 1e-4, 3)
    eu = C.rel_l2(s.unpack(t), ref_u)
    print(f"{name} fp32 staged: rhs rel L2 {err:.3e} (tol {tol:.2e}), u(3) {eu:.3e}")
    assert err < tol
    C.check_fields(f"{name} fp32 staged rhs", got, ext, ext.field_tol)
    C.check_fields(f"{name} fp32 staged u(3)", s.unpack(t), ref_u,
                   C.state_bar(ref_u, u, 1e-5, ext.field_tol))


@pytest.mark.parametrize("name", ["vortex1_p3", "tgv1_p3", "tgv1_p4_ns_fp32"])
def test_single_element_periodic_mesh(name):
    """The degenerate mesh: one element whose faces pair with its own
    opposite faces (15 padding columns of the 16-wide layout)."""
    if name == "vortex1_p3":
        w, prec = configs.vortex_quads(1, 3), "fp64"
    elif name == "tgv1_p3":
        w, prec = configs.taylor_green_hexes(1, 3), "fp64"
    else:
        w, prec = configs.taylor_green_hexes(1, 4), "fp32"
    d, s, u = _both(w, prec)
    stated = 1e-12 if prec == "fp64" else 1e-5
    tol, ext, floor = C.floor_tolerance(d, u, stated, 1.0 if prec == "fp64" else C.FP32_OVER_FP64)
    err = C.rel_l2(s.unpack(s.rhs(s.pack(u))), ext)
    t = s.pack(u)
    dt = 1e-4
    s.step(t, dt, 3)
    eu = C.rel_l2(s.unpack(t), d.rk4(u, dt, 3))
    print(f"{name}: rhs rel L2 {err:.2e} (tol {tol:.2e}), u(3) {eu:.2e}")
    assert err < tol and eu < (1e-12 if prec == "fp64" else 1e-5)


def test_rhs_alias_in_place():
    w = C.SMALL["mixed5_p2_ns"]()
    d, s, u = _both(w)
    t = s.pack(u)
    s.rhs(t, out=t)
    assert C.rel_l2(s.unpack(t), d.rhs(u)) < 1e-12


def test_padding_is_zero_and_inert():
    import torch
    w = configs.vortex_quads(7, 3)       # 49 elements -> ld 64
    d, s, u = _both(w)
    t = s.pack(u)
    blk = s.blocks[0]
    v = t.view(blk["nupts"], s.nvars, blk["ld"])
    v[:, :, blk["nelem"]:] = float("nan")
    out = s.rhs(t)
    o = out.view(blk["nupts"], s.nvars, blk["ld"])
    assert torch.all(o[:, :, blk["nelem"]:] == 0)
    assert C.rel_l2(s.unpack(out), d.rhs(u)) < 1e-12


def test_vortex20_p3_rhs_and_100_steps():
    """Vortex, 20x20 quads, p=3: du/dt and u after 100 RK4 steps, dt=1e-3."""
    w = configs.CONFIGS["vortex20_p3"]()
    d, s, u = _both(w, perturb=False)
    ref = d.rhs(u)
    t = s.pack(u)
    got = s.unpack(s.rhs(t))
    e_rhs = C.rel_l2(got, ref)
    s.step(t, w.dt, 40)
    s.step(t, w.dt, 60)           # two replays of the captured step graph
    ref_u = d.rk4(u, w.dt, 100)
    e_u = C.rel_l2(s.unpack(t), ref_u)
    print(f"vortex20_p3: rhs {e_rhs:.3e}  u(100) {e_u:.3e}")
    assert e_rhs < 1e-12 and e_u < 1e-12
    _tol, ext, _floor = C.floor_tolerance(d, u, 1e-12)
    C.check_fields("vortex20_p3 rhs", got, ext, ext.field_tol)
    C.check_fields("vortex20_p3 u(100)", s.unpack(t), ref_u, C.state_bar(ref_u, u, 1e-12, ext.field_tol))


def test_tgv16_p3_rhs_and_100_steps():
    """Taylor-Green, 16^3 hexes, p=3, Navier-Stokes: du/dt and u after the
    workload's 100 RK4 steps (dt 3e-4), in FP64 and on the FP32 operator
    path (FP64 state, update and reductions)."""
    w = configs.CONFIGS["tgv16_p3"]()
    assert w.nsteps == 100
    d, s, u = _both(w, perturb=False)
    tol64, ext, floor = C.floor_tolerance(d, u, 1e-12)
    ftol32 = np.maximum(1e-5, ext.field_floor * 4 * C.FP32_OVER_FP64)
    tol32 = max(1e-5, 4 * floor * C.FP32_OVER_FP64)
    t = s.pack(u)
    g64 = s.unpack(s.rhs(t))
    e_rhs = C.rel_l2(g64, ext)
    s.step(t, w.dt, w.nsteps)
    ref_u = u
    for k in range(0, w.nsteps, 20):          # the oracle, with a progress line per 20 steps
        ref_u = d.rk4(ref_u, w.dt, min(20, w.nsteps - k))
        print(f"tgv16_p3: oracle at step {min(k + 20, w.nsteps)}", flush=True)
    e_u = C.rel_l2(s.unpack(t), ref_u)
    s32 = C.solver_for(w, "fp32")
    t32 = s32.pack(u)
    g32 = s32.unpack(s32.rhs(t32))
    e32 = C.rel_l2(g32, ext)
    s32.step(t32, w.dt, w.nsteps)
    e32u = C.rel_l2(s32.unpack(t32), ref_u)
    print(f"tgv16_p3: fp64 floor {floor:.2e} | rhs {e_rhs:.3e} (tol {tol64:.1e}) u(100) {e_u:.3e} | "
          f"fp32 rhs {e32:.3e} (tol {tol32:.1e}) u(100) {e32u:.3e}")
    assert e_rhs < tol64 and e_u < 1e-12
    assert e32 < tol32 and e32u < 1e-5
    C.check_fields("tgv16_p3 fp64 rhs", g64, ext, ext.field_tol)
    C.check_fields("tgv16_p3 fp64 u(100)", s.unpack(t), ref_u,
                   C.state_bar(ref_u, u, 1e-12, ext.field_tol))
    C.check_fields("tgv16_p3 fp32 rhs", g32, ext, ftol32)
    C.check_fields("tgv16_p3 fp32 u(100)", s32.unpack(t32), ref_u, C.state_bar(ref_u, u, 1e-5, ftol32))


def test_rk_graph_replay_matches_single_steps():
    import torch
    w = configs.vortex_quads(6, 2)
    d, s, u = _both(w)
    a = s.pack(u)
    b = a.clone()
    s.step(a, w.dt, 5)
    for _ in range(5):
        s.step(b, w.dt, 1)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # a new dt value is picked up by the captured graph
    dt = torch.full((1,), 2e-3, dtype=torch.float64, device="cuda")
    c = s.pack(u)
    s.step(c, dt, 1)
    ref = d.rk4(u, 2e-3, 1)
    assert C.rel_l2(s.unpack(c), ref) < 1e-13


def test_integrals_and_conservation():
    w = C.SMALL["mixed5_p2_ns"]()
    d, s, u = _both(w)
    t = s.pack(u)
    got = s.integrate(t).cpu().numpy()[0]
    ref = sum(np.einsum("r,rn,ran->a", rf.W, g.detJ.T, ub) for rf, g, ub in zip(d.refs, d.geoms, u))
    assert np.allclose(got[:-1], ref, rtol=1e-13, atol=0)
    r = s.integrate(s.rhs(t)).cpu().numpy()[0]
    scale = sum(np.einsum("r,rn,ran->a", rf.W, g.detJ.T, np.abs(rb))
                for rf, g, rb in zip(d.refs, d.geoms, d.rhs(u)))
    assert np.all(np.abs(r[:-1]) < 1e-13 * scale)


def _ke(u, ndims):
    rho, m = u[:, 0], u[:, 1:1 + ndims]
    return 0.5 * np.sum(m * m, axis=1) / rho


@pytest.mark.parametrize("n", [6, 16])
def test_integrals_single_large_problem(n):
    """Integrals of a single-problem hex mesh, large enough that the library
    splits points into ranges and the element list into slices."""
    w = configs.taylor_green_hexes(n, 3)
    d, s, u = _both(w)
    got = s.integrate(s.pack(u)).cpu().numpy()[0]
    rf, g, ub = d.refs[0], d.geoms[0], u[0]
    ref = np.einsum("r,rn,ran->a", rf.W, g.detJ.T, ub)
    ke = np.einsum("r,rn,rn->", rf.W, g.detJ.T, _ke(ub, 3))
    print(f"n={n}: integrals rel err {np.abs(got[:-1] - ref).max() / np.abs(ref).max():.2e}, "
          f"kinetic energy rel err {abs(got[-1] - ke) / ke:.2e}")
    assert np.allclose(got[:-1], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    assert abs(got[-1] - ke) <= 1e-13 * ke


def test_check_finite():
    import paper_1312_1638_amd as P
    w = configs.vortex_quads(4, 2)
    d = Discretisation(w)
    u = d.initial_state(w)
    s = C.solver_for(w, check_finite=True)
    t = s.pack(u)
    s.step(t, w.dt, 1)
    u[0][0, 0, 3] = np.nan
    t = s.pack(u)
    with pytest.raises(P.FRError) as e:
        s.step(t, w.dt, 1)
    assert e.value.status == P.binding.FR_ENONFINITE


# LDS-staged BF16x3 plans (MBW, WM, column tile): the instantiated shapes
_BF16_LDS = [(1, 4, 64), (2, 4, 64), (3, 4, 64), (4, 4, 64), (6, 4, 64),
             (1, 2, 64), (2, 2, 64), (3, 2, 64), (4, 2, 64), (6, 2, 64), (8, 2, 64),
             (1, 1, 64), (2, 1, 64), (3, 1, 64), (4, 1, 64), (6, 1, 64), (8, 1, 64), (12, 1, 64),
             (1, 4, 128), (2, 4, 128), (1, 2, 128), (2, 2, 128), (3, 2, 128), (4, 2, 128),
             (1, 1, 128), (2, 1, 128), (4, 1, 128), (6, 1, 128), (8, 1, 128)]


def _force_bf16(s, w, wm, tw):
    """Every operator product on the direct BF16x3 kernel (tw = 0) or on
    the LDS-staged one with row split wm and column tile tw; returns False
    if some product has no staged shape for this split."""
    import paper_1312_1638_amd as P
    steps = [1, 3, 5, 8] if w.system == "ns" else [1, 8]
    for bi, b in enumerate(w.mesh.blocks):
        nu = s.blocks[bi]["nupts"]
        nf = P.reference_operator(b.etype, b.order, 6).shape[0]
        rows = {1: nf, 3: s.ndims * nu, 5: nf, 8: nu}
        for st in steps:
            mb = -(-rows[st] // 16)
            if tw == 0:
                plan = (1, 1, mb)
            else:
                fit = [m for m, k, t in _BF16_LDS if k == wm and t == tw and m * wm >= mb]
                if not fit:
                    return False
                plan = (min(fit), tw, wm)
            s.set_plan(bi, st, plan)
            assert s.gemm_plan(bi, st) == plan
    return True


@pytest.mark.parametrize("name", ["vortex7_p3", "mixed6_p3_euler", "tgv5_p3", "curved4_p4",
                                  "mixed5_p2_ns"])
def test_bf16x3_staged_kernel_matches_direct(name):
    """The LDS-staged BF16x3 kernel splits and accumulates exactly as the
    direct one (same hi/lo splits, same k order, same three products per
    k-step), so du/dt is bitwise the same for every row split and column
    tile; u after 3 RK4 steps stays within the stated 1e-5 of the oracle."""
    import torch
    w = C.SMALL[name]()
    d, s, u = _both(w, "bf16x3")
    t = s.pack(u)
    assert _force_bf16(s, w, 1, 0)
    ref = s.rhs(t).clone()
    ref_u = d.rk4(u, 1e-4, 3)
    ran = 0
    for wm in (1, 2, 4):
        for tw in (64, 128):
            if not _force_bf16(s, w, wm, tw):
                continue
            got = s.rhs(t)
            torch.cuda.synchronize()
            diff = (got - ref).abs().max().item()
            x = s.pack(u)
            s.step(x, 1e-4, 3)
            eu = C.rel_l2(s.unpack(x), ref_u)
            print(f"{name} staged wm={wm} tw={tw}: max |diff| vs direct {diff:.1e}, u(3) {eu:.2e}")
            assert diff == 0.0
            assert eu < 1e-5
            ran += 1
    assert ran >= 3
