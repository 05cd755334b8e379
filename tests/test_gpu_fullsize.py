"""Parity at the full workload sizes, with the plans the library's tuner
picks for them and the captured RK4 graph (the configuration bench.py
times): du/dt on seeded samples of elements against the oracle run on a
patch around them (one ring of face neighbours for Euler, two for
Navier-Stokes; see test_patch_reproduces_full_mesh_rhs), and properties that
hold at any size: discrete conservation through RK4 steps, free-stream
preservation on the curved mesh, and the adjoint gradient against central
differences of the library's own forward map."""
import numpy as np
import pytest

import frcases as C
from oracle import Discretisation
from workloads import configs

pytestmark = pytest.mark.gpu


def _initial(s, w):
    return [np.ascontiguousarray(np.transpose(w.ic(b, s.solution_points(b)), (1, 2, 0)))
            for b in range(len(w.mesh.blocks))]


def _sample(nelem, nsample, seed):
    """Seeded random elements plus the places where an indexing slip at full
    size would show: element 0, the last element, one inside the last tile
    of 256 columns, and the two elements on either side of the first
    boundary between the sparse-row kernel's XCD tile groups (8 tiles of 256
    elements: elements 2047 and 2048)."""
    fixed = [0, nelem - 1, (nelem - 1) // 256 * 256 + min(97, (nelem - 1) % 256)]
    if nelem > 2048:
        fixed += [2047, 2048]
    rnd = np.random.default_rng(seed).choice(nelem, nsample, replace=False)
    return np.unique(np.concatenate([fixed, rnd]))


def _patch_reference(w, sample, rings, stated=1e-12, unit_ratio=1.0):
    """The oracle's long-double du/dt on the sampled elements, from a patch
    around them, with the whole-vector and per-field bars."""
    pw, loc = C.patch(w, sample, rings)
    d = Discretisation(pw, allow_unpaired=True)
    return C.sampled_floor_tolerance(d, d.initial_state(pw), loc, stated, unit_ratio)


def _sampled_rhs(w, s, t, rings, nsample=12, seed=33):
    r = s.unpack(s.rhs(t))[0]
    sample = _sample(w.mesh.blocks[0].nelem, nsample, seed)
    tol, ext, floor = _patch_reference(w, sample, rings)
    err = C.rel_l2([r[:, :, sample]], ext)
    C.check_fields(f"{w.name} sampled du/dt", [r[:, :, sample]], ext, ext.field_tol)
    return err, tol, floor, r


def _conserved(s, t, before, after_steps):
    i0 = before
    after_steps()
    i1 = s.integrate(t).cpu().numpy()[0]
    nv = len(i0) - 1
    return np.abs(i1[:nv] - i0[:nv]).max() / np.abs(i0[:nv]).max()


def _uniform_stream(w, shape):
    v = np.array([1.0, 0.5, 0.25]) / np.linalg.norm([1.0, 0.5, 0.25])
    rho, p = 1.0, 1.0 / (w.gamma * 0.25)
    cons = np.array([rho, *(rho * v), p / (w.gamma - 1) + 0.5 * rho])
    return np.broadcast_to(cons[None, :, None], shape).copy()


def test_curved48_p4():
    """48^3 curved Q2 hexes, p=4, Euler (6.9e7 DOF): sampled du/dt within
    the stated 1e-12 of the long-double evaluation (whole sample and each
    field), mass, momentum and energy through 10 RK4 steps, and a uniform
    stream."""
    w = configs.CONFIGS["curved48_p4"]()
    s = C.solver_for(w)
    u0 = _initial(s, w)
    t = s.pack(u0)
    err, tol, floor, r = _sampled_rhs(w, s, t, rings=1)
    print(f"curved48_p4 sampled du/dt rel L2 {err:.2e} (oracle's FP64 floor {floor:.2e}, bar 1e-12)")
    assert err < 1e-12
    drift = _conserved(s, t, s.integrate(t).cpu().numpy()[0], lambda: s.step(t, w.dt, w.nsteps))
    print(f"curved48_p4 integrals after {w.nsteps} steps: relative drift {drift:.2e}")
    assert drift < 1e-12
    # uniform stream: du/dt vanishes to round-off (free-stream preservation)
    ru = s.unpack(s.rhs(s.pack([_uniform_stream(w, u0[0].shape)])))[0]
    rel = np.abs(ru).max() / np.abs(r).max()
    print(f"curved48_p4 uniform stream: max|du/dt| / max|du/dt(perturbed)| = {rel:.2e}")
    assert rel < 1e-10


# Reduced-precision operator products on the same mesh.  du/dt: per field,
# the stated bar or 4 x the field's FP64 floor x the unit-roundoff ratio
# (2^29 for FP32, 2^37 for BF16x3).  Conservation: the state, update and
# integrals stay FP64, but the divergence product no longer telescopes
# exactly.  Its rounding (unit u: 2^-24, about 2^-16 for BF16x3) reaches
# the integrals through 40 stage increments of dt = 7.5e-5 times flux
# derivatives some 10^3 times the state, at most 40 x 7.5e-5 x 10^3 x u =
# 3 u: the bars are 1e-6 (FP32) and 1e-4 (BF16x3).  A uniform stream: the
# products of constant data round at u relative to the flux-derivative
# terms, which are some 10^4 times du/dt of the perturbed stream (the same
# amplification the FP64 floor of this case shows, 1.4e-11 / 2^-53): bars
# 2^15 u.
_REDUCED = {"fp32": (1e-5, C.FP32_OVER_FP64, 1e-6, 2.0 ** -9),
            "bf16x3": (1e-4, C.BF16X3_OVER_FP64, 1e-4, 2.0 ** -1)}


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_curved48_p4_reduced_precision(prec):
    stated, ratio, drift_bar, uni_bar = _REDUCED[prec]
    w = configs.CONFIGS["curved48_p4"]()
    s = C.solver_for(w, prec)
    u0 = _initial(s, w)
    t = s.pack(u0)
    r = s.unpack(s.rhs(t))[0]
    sample = _sample(w.mesh.blocks[0].nelem, 12, 33)
    tol, ext, floor = _patch_reference(w, sample, 1, stated, ratio)
    err = C.rel_l2([r[:, :, sample]], ext)
    print(f"curved48_p4 {prec} sampled du/dt rel L2 {err:.2e} (FP64 floor {floor:.2e}, bar {tol:.2e})")
    assert err < tol
    C.check_fields(f"curved48_p4 {prec} sampled du/dt", [r[:, :, sample]], ext, ext.field_tol)
    drift = _conserved(s, t, s.integrate(t).cpu().numpy()[0], lambda: s.step(t, w.dt, w.nsteps))
    print(f"curved48_p4 {prec} integrals after {w.nsteps} steps: relative drift {drift:.2e} "
          f"(bar {drift_bar:.0e})")
    assert drift < drift_bar
    ru = s.unpack(s.rhs(s.pack([_uniform_stream(w, u0[0].shape)])))[0]
    rel = np.abs(ru).max() / np.abs(r).max()
    print(f"curved48_p4 {prec} uniform stream: max|du/dt| / max|du/dt(perturbed)| = {rel:.2e} "
          f"(bar {uni_bar:.1e})")
    assert rel < uni_bar


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_curved12_p4_u_after_10_steps(prec):
    """The curved family of the 48^3 workload on 12^3 Q2 hexes, p=4: u after
    its 10 RK4 steps (dt 3e-4, captured step graph) against the oracle's at
    the stated bars (1e-12 FP64, 1e-5 FP32 and BF16x3 operator paths), over
    the whole state and per field (each field's bar widened, where its
    change over the steps is large, by that field's du/dt bar)."""
    w = configs.curved_freestream_hexes(12, 4)
    d = Discretisation(w)
    u = d.initial_state(w)
    s = C.solver_for(w, prec)
    t = s.pack(u)
    s.step(t, w.dt, w.nsteps)
    ref = _ORACLE_U10.get("curved12")
    if ref is None:
        ref = _ORACLE_U10["curved12"] = d.rk4(u, w.dt, w.nsteps)
    bar = 1e-12 if prec == "fp64" else 1e-5
    ratio = {"fp64": 1.0, "fp32": C.FP32_OVER_FP64, "bf16x3": C.BF16X3_OVER_FP64}[prec]
    _tol, ext, _floor = C.floor_tolerance(d, u, bar, ratio)
    err = C.rel_l2(s.unpack(t), ref)
    print(f"curved12 p4 {prec}: u({w.nsteps}) rel L2 {err:.2e}")
    assert err < bar
    C.check_fields(f"curved12 p4 {prec} u({w.nsteps})", s.unpack(t), ref,
                   C.state_bar(ref, u, bar, ext.field_tol))


_ORACLE_U10 = {}


def test_tgv24_p3_sampled_rhs_and_conservation():
    """24^3 hexes, p=3, Navier-Stokes: sampled du/dt (two-ring patches) and
    conservation through the 200 steps of the adjoint horizon."""
    w = configs.CONFIGS["tgv24_p3"]()
    s = C.solver_for(w)
    t = s.pack(_initial(s, w))
    err, tol, floor, _ = _sampled_rhs(w, s, t, rings=2, nsample=8)
    print(f"tgv24_p3 sampled du/dt rel L2 {err:.2e} (floor {floor:.2e}, tol {tol:.2e})")
    assert err < tol
    drift = _conserved(s, t, s.integrate(t).cpu().numpy()[0], lambda: s.step(t, w.dt, w.nsteps))
    print(f"tgv24_p3 integrals after {w.nsteps} steps: relative drift {drift:.2e}")
    assert drift < 1e-12


def test_tgv24_p3_gradient_against_central_differences_32_directions():
    """Gradient of E_k(u_200) with respect to u_0 (checkpoint every 20 steps)
    against central differences of the library's FP64 forward map along 32
    seeded directions, each scaled per field by that field's RMS."""
    import torch
    from paper_1312_1638_amd.autograd import KineticEnergy, integrate_steps
    w = configs.CONFIGS["tgv24_p3"]()
    s = C.solver_for(w)
    u0h = _initial(s, w)
    u0 = s.pack(u0h)
    ug = u0.clone().requires_grad_(True)
    J = KineticEnergy.apply(integrate_steps(s, ug, w.dt, w.nsteps, w.info["ckpt"]), s)
    (g,) = torch.autograd.grad(J, ug)
    rng = np.random.default_rng(5)
    rms = [np.sqrt(np.mean(x ** 2, axis=(0, 2), keepdims=True)) for x in u0h]

    def objective(x):
        x = x.contiguous()
        s.step(x, w.dt, w.nsteps)
        return float(s.integrate(x)[:, -1].sum())

    worst = 0.0
    eps = 1e-5
    for k in range(32):
        dirn = s.pack([rng.standard_normal(x.shape) * r for x, r in zip(u0h, rms)])
        fd = (objective(u0 + eps * dirn) - objective(u0 - eps * dirn)) / (2 * eps)
        ad = float(torch.sum(g * dirn))
        rel = abs(ad - fd) / abs(fd)
        worst = max(worst, rel)
        print(f"direction {k:2d}: adjoint {ad:+.10e} central FD {fd:+.10e} rel {rel:.1e}")
    print(f"worst relative difference over 32 directions: {worst:.2e}")
    assert worst <= 1e-6
