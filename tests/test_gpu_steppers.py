"""Forward Euler and adaptive DOPRI5 through the C ABI against the oracle's
steppers.

DOPRI5 is compared attempt by attempt from the same inputs: before each
attempt the oracle takes the library's t and h, then both attempt once.
Decisions and counts must agree exactly, t bitwise, and the state to 1e-10
(FP64 operator path).  The new step size comes from the error norm, a small
difference of two solutions: relative perturbations of the slopes (the
right-hand side's parity, below 1e-12) reach it amplified by the attempt's
conditioning cond = ||h sum |E_j k_j| / sc|| / err, which the oracle logs,
and reach h at a fifth of that.  So h is held to max(1e-9, 1e-13 cond); a
wrong coefficient or controller rule moves it by O(1)."""
import numpy as np
import pytest

import frcases as C
from oracle import Discretisation
from oracle import steppers as S
from workloads import configs

pytestmark = pytest.mark.gpu


def _dev(x, dtype="float64"):
    import torch
    return torch.tensor(np.asarray(x), dtype=getattr(torch, dtype), device="cuda")


@pytest.mark.parametrize("name", ["vortex7_p3", "tgv3_p4", "mixed5_p2_ns"])
def test_euler_steps(name):
    w = C.SMALL[name]()
    d = Discretisation(w)
    u = C.perturbed(d, d.initial_state(w))
    s = C.solver_for(w)
    t = s.pack(u)
    dt = 0.1 * w.dt
    s.euler_step(t, dt, 10)
    err = C.rel_l2(s.unpack(t), S.euler(d, u, dt, 10))
    print(f"{name}: 10 Euler steps rel L2 {err:.2e}")
    assert err < 1e-12


def test_euler_per_problem_steps():
    wb = configs.batched_vortices(nproblems=6, seed=11, nmin=9, nmax=60, nsteps=1)
    d = Discretisation(wb)
    u = d.initial_state(wb)
    s = C.solver_for(wb)
    t = s.pack(u)
    dts = np.linspace(1e-4, 6e-4, 6)
    s.euler_step(t, _dev(dts), 5)
    prob = S.element_problems(d)
    ref = u
    for _ in range(5):
        r = d.rhs(ref)
        ref = [x + dts[p][None, None, :] * k for x, k, p in zip(ref, r, prob)]
    err = C.rel_l2(s.unpack(t), ref)
    print(f"batched Euler: rel L2 {err:.2e}")
    assert err < 1e-12


def _dopri_pair(w, h0, tend, atol, rtol, prec="fp64"):
    d = Discretisation(w)
    u = d.initial_state(w)
    s = C.solver_for(w, prec)
    nprob = s.nproblems
    h0 = np.broadcast_to(np.asarray(h0, float), (nprob,)).copy()
    tend = None if tend is None else np.broadcast_to(np.asarray(tend, float), (nprob,)).copy()
    dp = S.Dopri5(d, atol, rtol).start(u, np.zeros(nprob), h0, tend=tend)
    dev = dict(u=s.pack(u), t=_dev(np.zeros(nprob)), dt=_dev(h0),
               tend=None if tend is None else _dev(tend),
               counts=_dev(np.zeros((nprob, 2)), "int32"))
    return d, s, dp, dev


def _attempt_both(s, dp, dev, atol, rtol, n=1):
    """n attempts on both sides; the oracle starts each from the library's
    t and h (n = 1 compares every attempt from the same inputs)."""
    for i in range(n):
        if i == 0:
            dp.t = dev["t"].cpu().numpy().copy()
            dp.h = dev["dt"].cpu().numpy().copy()
            if dp.tend is not None:            # the cut every call begins with
                dp.h = np.minimum(dp.h, dp.tend - dp.t)
        dp.attempt()
    s.dopri5(dev["u"], dev["t"], dev["dt"], n, atol, rtol, tend=dev["tend"],
             counts=dev["counts"])


def _check_same(s, dp, dev, state_tol=1e-10, step_tol=1e-9, cond_factor=1e-13):
    t = dev["t"].cpu().numpy()
    h = dev["dt"].cpu().numpy()
    cnt = dev["counts"].cpu().numpy()
    acc = sum(e["accept"].astype(int) for e in dp.log)
    rej = sum(e["reject"].astype(int) for e in dp.log)
    assert np.array_equal(cnt[:, 0], acc) and np.array_equal(cnt[:, 1], rej), (cnt, acc, rej)
    cond = np.nan_to_num(dp.log[-1]["cond"], nan=0.0, posinf=0.0)
    htol = np.maximum(step_tol, cond_factor * cond)
    assert np.allclose(t, dp.t, rtol=step_tol, atol=0), (t, dp.t)
    assert np.all(np.abs(h - dp.h) <= htol * np.abs(dp.h)), (h, dp.h, htol)
    err = C.rel_l2(s.unpack(dev["u"]), dp.u)
    assert err < state_tol, err
    return err


@pytest.mark.parametrize("name,h0,tend,tol", [
    ("vortex7_p3", 1e-3, 0.3, 1e-9),
    ("tgv3_p4", 1e-4, 0.05, 1e-8),
    ("mixed5_p2_ns", 2e-3, 0.2, 1e-8),
    ("curved4_p4", 1e-4, 0.02, 1e-9),
])
def test_dopri5_attempt_by_attempt(name, h0, tend, tol):
    w = C.SMALL[name]()
    d, s, dp, dev = _dopri_pair(w, h0, tend, tol, tol)
    n = 0
    while dp.t[0] < tend:
        _attempt_both(s, dp, dev, tol, tol)
        err = _check_same(s, dp, dev)
        n += 1
        assert n < 200
    assert dev["t"].cpu().numpy()[0] == tend
    print(f"{name}: {n} attempts to t={tend}, final state rel L2 {err:.2e}")
    # at the end time the state stands still
    before = dev["u"].clone()
    _attempt_both(s, dp, dev, tol, tol, n=3)
    assert bool((dev["u"] == before).all())
    _check_same(s, dp, dev)


def test_dopri5_rejections():
    """A first step far too large: rejected attempts, shrinking, the capped
    growth after a rejection, then accepted steps -- the same decisions."""
    w = C.SMALL["vortex7_p3"]()
    d, s, dp, dev = _dopri_pair(w, 0.3, 0.6, 1e-10, 1e-10)
    for _ in range(10):
        _attempt_both(s, dp, dev, 1e-10, 1e-10)
        _check_same(s, dp, dev)
    dec = [bool(e["accept"][0]) for e in dp.log]
    print("decisions", "".join("A" if x else "R" for x in dec))
    assert not dec[0] and any(dec)


def test_dopri5_one_call_equals_single_attempts():
    """n attempts in one call (graph replays, first-same-as-last slope kept
    on the device) equal n calls of one attempt (slope recomputed), bitwise."""
    w = C.SMALL["mixed5_p2_ns"]()
    outs = []
    for chunk in (1, 7):
        d, s, dp, dev = _dopri_pair(w, 0.05, 0.3, 1e-7, 1e-7)
        for _ in range(7 // chunk):
            s.dopri5(dev["u"], dev["t"], dev["dt"], chunk, 1e-7, 1e-7, tend=dev["tend"],
                     counts=dev["counts"])
        outs.append((dev["u"].clone(), dev["t"].clone(), dev["dt"].clone(), dev["counts"].clone()))
    for a, b in zip(outs[0], outs[1]):
        assert bool((a == b).all())
    assert int(outs[0][3][0, 1]) > 0        # the sequence had a rejection


def test_dopri5_batched_problems():
    """Independent problems with their own first steps and end times."""
    wb = configs.batched_vortices(nproblems=8, seed=12, nmin=9, nmax=80, nsteps=1)
    rng = np.random.default_rng(3)
    h0 = rng.uniform(1e-3, 0.2, 8)
    tend = rng.uniform(0.02, 0.2, 8)
    d, s, dp, dev = _dopri_pair(wb, h0, tend, 1e-8, 1e-8)
    n = 0
    while np.any(dp.t < tend):
        _attempt_both(s, dp, dev, 1e-8, 1e-8)
        _check_same(s, dp, dev)
        n += 1
        assert n < 400
    assert np.array_equal(dev["t"].cpu().numpy(), tend)
    cnt = dev["counts"].cpu().numpy()
    print(f"batched: {n} attempts; accepted {cnt[:, 0]}, rejected {cnt[:, 1]}")
    assert len(set(cnt[:, 0])) > 1


def test_dopri5_problems_that_stand_still():
    """A batch where one problem starts with dt = 0 and one is already past
    its end time: both keep their state bitwise and count no attempt, while
    the third integrates as the oracle does."""
    wb = configs.batched_vortices(nproblems=3, seed=21, nmin=9, nmax=30, nsteps=1)
    h0 = np.array([0.01, 0.0, 0.01])
    tend = np.array([0.05, 0.05, -1.0])
    d, s, dp, dev = _dopri_pair(wb, h0, tend, 1e-8, 1e-8)
    before = [x.copy() for x in s.unpack(dev["u"])]
    for _ in range(10):
        _attempt_both(s, dp, dev, 1e-8, 1e-8)
        _check_same(s, dp, dev)
    after = s.unpack(dev["u"])
    cnt = dev["counts"].cpu().numpy()
    assert cnt[1].sum() == 0 and cnt[2].sum() == 0 and cnt[0, 0] > 0
    prob = S.element_problems(d)
    for b, (x0, x1, pb) in enumerate(zip(before, after, prob)):
        still = np.isin(pb, [1, 2])
        assert np.array_equal(x0[:, :, still], x1[:, :, still])
    assert dev["t"].cpu().numpy()[1] == 0.0 and dev["t"].cpu().numpy()[2] == 0.0


def test_dopri5_without_end_time():
    w = C.SMALL["vortex7_p3"]()
    d, s, dp, dev = _dopri_pair(w, 1e-3, None, 1e-9, 1e-9)
    for _ in range(12):
        _attempt_both(s, dp, dev, 1e-9, 1e-9)
        _check_same(s, dp, dev)


def test_dopri5_fp32_operators():
    """FP32 operator products: the slopes move by up to the case's FP32 du/dt
    bar (relative), which bounds the step sizes through the conditioning;
    the state is held to 1e-5.  (On low-Mach cases that bar is ~1e-3 and the
    error estimate is FP32 rounding; the vortex is well conditioned.)"""
    w = C.SMALL["vortex7_p3"]()
    d, s, dp, dev = _dopri_pair(w, 1e-3, 0.3, 1e-6, 1e-6, prec="fp32")
    bar, _ext, _floor = C.floor_tolerance(d, d.initial_state(w), 1e-5, C.FP32_OVER_FP64)
    for _ in range(8):
        _attempt_both(s, dp, dev, 1e-6, 1e-6)
        _check_same(s, dp, dev, state_tol=1e-5, step_tol=1e-9, cond_factor=bar)


def test_dopri5_argument_errors():
    import paper_1312_1638_amd as P
    w = C.SMALL["vortex7_p3"]()
    d, s, dp, dev = _dopri_pair(w, 1e-3, 0.1, 1e-9, 1e-9)
    for atol, rtol, n in ((0.0, 1e-9, 1), (1e-9, -1.0, 1), (float("nan"), 1e-9, 1),
                          (1e-9, 1e-9, -1)):
        with pytest.raises(P.FRError) as e:
            s.dopri5(dev["u"], dev["t"], dev["dt"], n, atol, rtol)
        assert e.value.status == P.binding.FR_EINVAL
    before = dev["u"].clone()
    s.dopri5(dev["u"], dev["t"], dev["dt"], 0, 1e-9, 1e-9)
    assert bool((dev["u"] == before).all())


@pytest.mark.parametrize("stepper", ["rk4", "euler"])
def test_grouped_step_graphs_equal_single_steps(stepper):
    """A call of 19 steps (two 8-step graphs, then three 1-step graphs) equals
    19 calls of one step bit for bit, also after the device step size
    changes between calls."""
    w = C.SMALL["mixed5_p2_ns"]()
    d = Discretisation(w)
    u = C.perturbed(d, d.initial_state(w))
    outs = []
    for grouped in (True, False):
        s = C.solver_for(w)
        t = s.pack(u)
        dt = _dev([0.05 * w.dt])
        go = s.step if stepper == "rk4" else s.euler_step
        for dtv in (0.05 * w.dt, 0.08 * w.dt):
            dt.fill_(dtv)
            if grouped:
                go(t, dt, 19)
            else:
                for _ in range(19):
                    go(t, dt, 1)
        outs.append(t.clone())
    assert bool((outs[0] == outs[1]).all())
    ref = u
    for dtv in (0.05 * w.dt, 0.08 * w.dt):
        ref = d.rk4(ref, dtv, 19) if stepper == "rk4" else S.euler(d, ref, dtv, 19)
    err = C.rel_l2(s.unpack(outs[0]), ref)
    print(f"{stepper}: 2 x 19 steps, grouped == single bitwise; rel L2 vs oracle {err:.2e}")
    assert err < 1e-12


def test_zero_steps_leave_the_state_and_negative_counts_are_refused():
    """RK4 and forward Euler with 0 steps leave the state bitwise as it was
    (no graph is captured or launched); a negative count is refused with
    FR_EINVAL before anything runs, and the state is still untouched."""
    import torch
    import paper_1312_1638_amd as P
    w = C.SMALL["vortex7_p3"]()
    d = Discretisation(w)
    s = C.solver_for(w)
    t = s.pack(C.perturbed(d, d.initial_state(w)))
    ref = t.clone()
    s.step(t, 1e-3, 0)
    s.euler_step(t, 1e-3, 0)
    torch.cuda.synchronize()
    assert torch.equal(t, ref)
    for call in (s.step, s.euler_step):
        with pytest.raises(P.FRError) as e:
            call(t, 1e-3, -1)
        assert e.value.status == P.binding.FR_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(t, ref)
