"""Many independent problems in one mesh (mixed quads/triangles, p = 2..4,
a step size per problem): parity of du/dt, RK4 steps and per-problem
integrals, on a small batch against the oracle run on the whole batch, and on
the full 512-problem batch against the oracle run problem by problem on a
seeded sample."""
import numpy as np
import pytest

import frcases as C
from oracle import Discretisation
from workloads import configs

pytestmark = pytest.mark.gpu


def _dt_blocks(w):
    return [w.dt_per_problem[b.problem] for b in w.mesh.blocks]


def _dt_dev(w):
    import torch
    return torch.tensor(w.dt_per_problem, dtype=torch.float64, device="cuda")


def test_small_batch_rhs_steps_integrals():
    w = configs.batched_vortices(12, seed=11, nmax=300)
    w.dt_per_problem = np.linspace(5e-4, 1.5e-3, 12)
    d = Discretisation(w)
    u = d.initial_state(w)
    s = C.solver_for(w)
    t = s.pack(u)
    tol_r, ext, floor = C.floor_tolerance(d, u, 1e-12)
    e_rhs = C.rel_l2(s.unpack(s.rhs(t)), ext)
    s.step(t, _dt_dev(w), 10)
    ref = d.rk4(u, _dt_blocks(w), 10)
    e_u = C.rel_l2(s.unpack(t), ref)
    got = s.integrate(t).cpu().numpy()
    want = np.zeros((12, 5))
    for b, (rf, g, x) in enumerate(zip(d.refs, d.geoms, ref)):
        prob = w.mesh.blocks[b].problem
        wj = rf.W[:, None] * g.detJ.T                         # (Nu, ne)
        for a in range(4):
            np.add.at(want[:, a], prob, np.sum(wj * x[:, a], 0))
        np.add.at(want[:, 4], prob, np.sum(wj * 0.5 * (x[:, 1] ** 2 + x[:, 2] ** 2) / x[:, 0], 0))
    e_int = np.abs(got - want).max() / np.abs(want).max()
    print(f"12 problems: rhs {e_rhs:.2e} u(10) {e_u:.2e} integrals {e_int:.2e}")
    assert e_rhs < tol_r and e_u < 1e-12 and e_int < 1e-13


def test_full_batch_sampled_problems():
    """512 problems (~5.7e5 elements, 6 element blocks), 20 RK4 steps in the
    captured graph; 4 seeded problems re-run alone through the oracle."""
    w = configs.CONFIGS["batched512"]()
    s = C.solver_for(w)
    u0 = [np.ascontiguousarray(np.transpose(w.ic(b, s.solution_points(b)), (1, 2, 0)))
          for b in range(len(w.mesh.blocks))]
    t = s.pack(u0)
    r = s.unpack(s.rhs(t))
    s.step(t, _dt_dev(w), w.nsteps)
    uN = s.unpack(t)
    rng = np.random.default_rng(2024)
    for j in sorted(rng.choice(w.mesh.nproblems, 4, replace=False)):
        pw, where = configs.single_problem(w, j)
        d = Discretisation(pw)
        u = d.initial_state(pw)
        tol_r, ref_r, floor = C.floor_tolerance(d, u, 1e-12)
        ref_u = d.rk4(u, pw.dt, w.nsteps)
        got_r = [r[b][:, :, o:o + n] for b, o, n in where]
        got_u = [uN[b][:, :, o:o + n] for b, o, n in where]
        # the two codes place the solution points independently: same inputs
        got_u0 = [u0[b][:, :, o:o + n] for b, o, n in where]
        assert C.rel_l2(got_u0, u) < 1e-14
        e_r, e_u = C.rel_l2(got_r, ref_r), C.rel_l2(got_u, ref_u)
        print(f"problem {j} (p={w.mesh.info['problems'][j]['p']}): rhs {e_r:.2e} "
              f"(fp64 floor {floor:.2e}, tol {tol_r:.2e}) u({w.nsteps}) {e_u:.2e}")
        assert e_r < tol_r and e_u < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_one_launch_per_kernel_family(prec):
    """Twelve problems in six element blocks (quads and triangles at p = 2, 3,
    4): steps 1 and 8 as one sparse-row launch over the quad blocks and one
    matrix-core launch over the triangle blocks, and the transformed flux
    as one launch, give du/dt and u after 3 RK4 steps (captured graph)
    bitwise equal to a launch per block -- every output sums the same
    entries in the same order -- and agree with the oracle."""
    import torch
    w = configs.batched_vortices(12, seed=11, nmax=300)
    w.dt_per_problem = np.linspace(5e-4, 1.5e-3, 12)
    d = Discretisation(w)
    u = C.perturbed(d, d.initial_state(w), seed=5)
    s = C.solver_for(w, prec)
    # the triangles on the matrix cores, the quads on the sparse-row kernel
    for bi, b in enumerate(w.mesh.blocks):
        for st in (1, 8):
            s.set_plan(bi, st, (1, 1, 1) if b.etype == "tri" else (0, 2, 0))
    out = {}
    # one state and one step-size tensor throughout: the step graph captured
    # in one mode must not be replayed after the launches change (setting
    # them releases the context's graphs)
    t = s.pack(u)
    dtd = _dt_dev(w)
    for mode in (0, 1, 2):
        state = [s.multi(st, mode) for st in (1, 8, 6)]
        if mode:
            assert state == [3, 3, 4], state
        else:
            assert state == [0, 0, 0], state
        r = s.rhs(s.pack(u))
        t.copy_(s.pack(u))
        s.step(t, dtd, 3)
        torch.cuda.synchronize()
        out[mode] = (r.cpu().numpy(), t.cpu().numpy())
    for mode in (1, 2):
        dr = np.abs(out[mode][0] - out[0][0]).max()
        du = np.abs(out[mode][1] - out[0][1]).max()
        print(f"{prec} mode {mode}: max |du/dt diff| {dr:.1e}, max |u(3) diff| {du:.1e}")
        assert dr == 0.0 and du == 0.0
    stated = 1e-12 if prec == "fp64" else 1e-5
    tol, ext, floor = C.floor_tolerance(d, u, stated, 1.0 if prec == "fp64" else C.FP32_OVER_FP64)
    s.multi(1, 1); s.multi(8, 1); s.multi(6, 1)
    got = s.unpack(s.rhs(s.pack(u)))
    err = C.rel_l2(got, ext)
    t = s.pack(u)
    s.step(t, _dt_dev(w), 3)
    eu = C.rel_l2(s.unpack(t), d.rk4(u, _dt_blocks(w), 3))
    print(f"{prec} one launch per family: rhs {err:.2e} (tol {tol:.1e}) u(3) {eu:.2e}")
    assert err < tol and eu < stated
    C.check_fields(f"{prec} one launch per family rhs", got, ext, ext.field_tol)
