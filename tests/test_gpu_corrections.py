"""SD and HU correction functions (the VCJH members of the super-accuracy
test) through the C ABI against the oracle: du/dt and RK4 steps on quads,
hexes (Euler and Navier-Stokes, straight and curved) and a walled Couette
channel, FP32 and split-bf16 operator products, every kernel family, and the
hand-written adjoint.  Tolerances as in the DG parity tests."""
import numpy as np
import pytest

import frcases as C
from oracle import Discretisation, jvp
from workloads import configs

pytestmark = pytest.mark.gpu

CASES = {
    "vortex7_p3_sd": lambda: configs.with_correction(configs.vortex_quads(7, 3), "sd"),
    "vortex7_p3_hu": lambda: configs.with_correction(configs.vortex_quads(7, 3), "hu"),
    "vortex4_p6_hu": lambda: configs.with_correction(configs.vortex_quads(4, 6), "hu"),
    "tgv3_p4_sd": lambda: configs.with_correction(configs.taylor_green_hexes(3, 4), "sd"),
    "tgv4_p3_hu": lambda: configs.with_correction(configs.taylor_green_hexes(4, 3), "hu"),
    "curved4_p4_sd": lambda: configs.with_correction(configs.curved_freestream_hexes(4, 4), "sd"),
    "couette_quad4_p3_hu": lambda: configs.with_correction(
        configs.couette(4, 3, "quad", start="constant"), "hu"),
    "couette_hex3_p2_sd": lambda: configs.with_correction(
        configs.couette(3, 2, "hex", start="constant"), "sd"),
}


def _both(name, prec="fp64"):
    w = CASES[name]()
    d = Discretisation(w)
    u = C.perturbed(d, d.initial_state(w))
    return w, d, u, C.solver_for(w, prec)


@pytest.mark.parametrize("name", sorted(CASES))
def test_corrections_rhs_and_steps(name):
    w, d, u, s = _both(name)
    tol, ext, floor = C.floor_tolerance(d, u, 1e-12)
    t = s.pack(u)
    err = C.rel_l2(s.unpack(s.rhs(t)), ext)
    dt = 0.2 * w.dt
    s.step(t, dt, 10)
    eu = C.rel_l2(s.unpack(t), d.rk4(u, dt, 10))
    print(f"{name}: rhs rel L2 {err:.2e} (floor {floor:.2e}, tol {tol:.2e}), u(10) {eu:.2e}")
    assert err < tol and eu < 1e-12


def test_corrections_differ_from_dg():
    """The scheme reaches the device: DG, SD and HU give different du/dt."""
    w = CASES["vortex7_p3_sd"]()
    d = Discretisation(w)
    u = C.perturbed(d, d.initial_state(w))
    out = {}
    for k in ("dg", "sd", "hu"):
        out[k] = C.solver_for(configs.with_correction(configs.vortex_quads(7, 3), k))
        out[k] = out[k].unpack(out[k].rhs(out[k].pack(u)))
    assert C.rel_l2(out["sd"], out["dg"]) > 1e-4
    assert C.rel_l2(out["hu"], out["dg"]) > 1e-4
    assert C.rel_l2(out["hu"], out["sd"]) > 1e-4


@pytest.mark.parametrize("name", ["vortex7_p3_hu", "tgv4_p3_hu", "curved4_p4_sd"])
def test_corrections_fp32(name):
    w, d, u, s = _both(name, "fp32")
    tol, ext, floor = C.floor_tolerance(d, u, 1e-5, C.FP32_OVER_FP64)
    err = C.rel_l2(s.unpack(s.rhs(s.pack(u))), ext)
    t = s.pack(u)
    dt = 0.2 * w.dt
    s.step(t, dt, 5)
    eu = C.rel_l2(s.unpack(t), d.rk4(u, dt, 5))
    print(f"{name} fp32: rel L2 {err:.2e} (tol {tol:.2e}), u(5) {eu:.2e}")
    assert err < tol and eu < 1e-5


@pytest.mark.parametrize("name", ["vortex7_p3_sd", "tgv4_p3_hu"])
def test_corrections_bf16x3(name):
    w, d, u, s = _both(name, "bf16x3")
    tol, ext, floor = C.floor_tolerance(d, u, 1e-4, C.BF16X3_OVER_FP64)
    err = C.rel_l2(s.unpack(s.rhs(s.pack(u))), ext)
    print(f"{name} bf16x3: rel L2 {err:.2e} (tol {tol:.2e})")
    assert err < tol


@pytest.mark.parametrize("variant", ["mfma", "sparse", "fused", "fields", "fused_fields",
                                     "fused_flux", "staged", "staged_fused"])
@pytest.mark.parametrize("name", ["tgv3_p4_sd", "vortex7_p3_hu"])
def test_corrections_every_kernel_variant(name, variant):
    from test_gpu_parity import _force_plans
    w, d, u, s = _both(name)
    _force_plans(s, w, variant)
    tol, ext, floor = C.floor_tolerance(d, u, 1e-12)
    err = C.rel_l2(s.unpack(s.rhs(s.pack(u))), ext)
    print(f"{name} {variant}: rel L2 {err:.2e} (tol {tol:.2e})")
    assert err < tol


@pytest.mark.parametrize("name", ["vortex7_p3_sd", "tgv4_p3_hu", "curved4_p4_sd"])
def test_corrections_adjoint_dot_product(name):
    from test_gpu_adjoint import _dot, _norm, _off_kink, _rand_like
    w = CASES[name]()
    d = Discretisation(w)
    u = _off_kink(d, d.initial_state(w))
    v = _rand_like(u, 1)
    lam = _rand_like(u, 2)
    Jv = jvp(d, u, v)
    s = C.solver_for(w)
    JTl = s.unpack(s.rhs_adjoint(s.pack(u), s.pack(lam)))
    lhs, rhs = _dot(Jv, lam), _dot(v, JTl)
    scale = _norm(Jv) * _norm(lam)
    print(f"{name}: <Jv,l> {lhs:.6e} <v,J^T l> {rhs:.6e} rel {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-13 * scale
