"""Pins of the oracle's time steppers (forward Euler, adaptive DOPRI5):
the Dormand-Prince tableau against the order conditions of Runge-Kutta
methods (exact rational arithmetic) and its published stability polynomial,
forward Euler's amplification factor, and whole adaptive integrations of
the FR right-hand side against scipy's independent Dormand-Prince
implementation (scipy.integrate.RK45, the same controller)."""
import math
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import Discretisation
from oracle import steppers as S
from workloads import configs

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _tableau():
    A = [[F(0)] * 7 for _ in range(7)]
    for i, row in enumerate(S.DP_A):
        for j, v in enumerate(row):
            A[i][j] = v
    return A


def _mv(A, v):
    return [sum(A[i][j] * v[j] for j in range(7)) for i in range(7)]


def _dot(b, v):
    return sum(x * y for x, y in zip(b, v))


def _order_conditions(A, c):
    """(elementary weight vector, 1/gamma) for the 17 rooted trees of order
    <= 5 (Butcher): sum_i b_i Phi_i(tree) = 1/gamma(tree)."""
    def el(f, g):
        return [x * y for x, y in zip(f, g)]
    one = [F(1)] * 7
    Ac, Ac2, Ac3 = _mv(A, c), _mv(A, el(c, c)), _mv(A, el(c, el(c, c)))
    AAc, AAc2 = _mv(A, Ac), _mv(A, Ac2)
    return [
        (1, one, F(1)),
        (2, c, F(1, 2)),
        (3, el(c, c), F(1, 3)), (3, Ac, F(1, 6)),
        (4, el(c, el(c, c)), F(1, 4)), (4, el(c, Ac), F(1, 8)), (4, Ac2, F(1, 12)),
        (4, AAc, F(1, 24)),
        (5, el(el(c, c), el(c, c)), F(1, 5)), (5, el(el(c, c), Ac), F(1, 10)),
        (5, el(c, Ac2), F(1, 15)), (5, el(c, AAc), F(1, 30)), (5, el(Ac, Ac), F(1, 20)),
        (5, Ac3, F(1, 20)), (5, _mv(A, el(c, Ac)), F(1, 40)), (5, AAc2, F(1, 60)),
        (5, _mv(A, AAc), F(1, 120)),
    ]


def test_dopri5_tableau_order_conditions():
    A = _tableau()
    c = S.DP_C
    # row sums are the nodes; the last stage is taken at the new state
    for i in range(7):
        assert sum(A[i]) == c[i]
    assert S.DP_A[6] + [F(0)] == S.DP_B
    conds = _order_conditions(A, c)
    assert len(conds) == 17
    for order, phi, inv_gamma in conds:
        assert _dot(S.DP_B, phi) == inv_gamma, (order, "b")
        if order <= 4:
            assert _dot(S.DP_BHAT, phi) == inv_gamma, (order, "bhat")
    # the embedded pair is of order exactly 4
    assert any(_dot(S.DP_BHAT, phi) != g for o, phi, g in conds if o == 5)


def test_dopri5_stability_polynomial():
    """R(z) = 1 + b^T (I - zA)^-1 1 z = sum_{k<=5} z^k/k! + z^6/600."""
    A = _tableau()
    v = [F(1)] * 7
    coef = []
    for _ in range(7):
        coef.append(_dot(S.DP_B, v))
        v = _mv(A, v)
    assert coef == [F(1, math.factorial(k + 1)) for k in range(5)] + [F(1, 600), F(0)]


def test_euler_linear_amplification():
    d = Discretisation(configs.vortex_quads(3, 1))
    lam = -0.7 + 2.3j
    d.rhs = lambda s: [lam * x for x in s]
    u = [np.ones((4, 4, 9), dtype=complex)]
    for dt in (0.1, 0.37):
        out = S.euler(d, u, dt, 3)[0]
        assert np.allclose(out, (1 + lam * dt) ** 3, rtol=0, atol=1e-15)


def _flat(state):
    return np.concatenate([x.ravel() for x in state])


def _unflat(v, like):
    out, off = [], 0
    for x in like:
        out.append(v[off:off + x.size].reshape(x.shape))
        off += x.size
    return out


@pytest.mark.parametrize("case", ["vortex_euler", "mixed_ns"])
def test_dopri5_matches_scipy_rk45(case):
    """The adaptive integration of du/dt = R(u) to t_end: the same accepted
    times, step sizes and states as scipy's RK45 from the same first step."""
    from scipy.integrate import RK45
    if case == "vortex_euler":
        w = configs.vortex_quads(3, 2)
        tend, h0, atol, rtol = 0.5, 1e-3, 1e-9, 1e-9
    else:
        import frcases
        w = frcases.mixed(3, 2, system="ns")
        tend, h0, atol, rtol = 0.2, 1e-3, 1e-8, 1e-8
    d = Discretisation(w)
    u0 = d.initial_state(w)
    dp = S.Dopri5(d, atol, rtol).start(u0, [0.0], [h0], tend=[tend])
    times, hs = [], []
    while dp.t[0] < tend:
        acc, _rej = dp.attempt()
        if acc[0]:
            times.append(dp.t[0])
            hs.append(dp.h[0])
        assert len(dp.log) < 500
    nrej = sum(int(e["reject"][0]) for e in dp.log)
    sp = RK45(lambda t, y: _flat(d.rhs(_unflat(y, u0))), 0.0, _flat(u0), tend,
              first_step=h0, atol=atol, rtol=rtol)
    st, sh = [], []
    while sp.status == "running":
        sp.step()
        st.append(sp.t)
        sh.append(sp.h_abs)
    print(f"{case}: {len(times)} accepted, {nrej} rejected; scipy {len(st)} steps")
    # The error estimate is the small difference of the two solutions: its
    # rounding (summation order) is amplified by about h |k| / (tol |u|),
    # some 1e-11 relative here, and moves each new h by a fifth of that; a
    # wrong coefficient or controller rule moves it by O(1).
    assert len(times) == len(st) and len(times) > 5
    assert np.allclose(times, st, rtol=1e-9, atol=0)
    # next step proposals; here they are already cut to the end time
    sh = np.minimum(sh, tend - np.array(st))
    assert np.allclose(hs[:-1], sh[:-1], rtol=1e-9, atol=0)
    assert times[-1] == tend
    scale = np.abs(sp.y).max()
    assert np.max(np.abs(_flat(dp.u) - sp.y)) < 1e-10 * scale


def test_dopri5_rejections_match_scipy():
    """A first step far too large: rejections, then the capped growth after
    a rejection; same sequence as scipy."""
    from scipy.integrate import RK45
    w = configs.vortex_quads(3, 2)
    d = Discretisation(w)
    u0 = d.initial_state(w)
    tend, h0, atol, rtol = 0.2, 0.2, 1e-8, 1e-8
    dp = S.Dopri5(d, atol, rtol).start(u0, [0.0], [h0], tend=[tend])
    for _ in range(12):
        dp.attempt()
    dec = [bool(e["accept"][0]) for e in dp.log]
    assert dec[0] is False and any(dec)
    sp = RK45(lambda t, y: _flat(d.rhs(_unflat(y, u0))), 0.0, _flat(u0), tend,
              first_step=h0, atol=atol, rtol=rtol)
    st = []
    while len(st) < sum(dec):
        sp.step()
        st.append(sp.t)
    got = [e for e in dp.log if e["accept"][0]]
    acc_t = np.cumsum([e["h"][0] for e in got])
    assert np.allclose(acc_t, st, rtol=1e-9)


def test_dopri5_problems_are_independent():
    """Two problems in one mesh: each follows the single-problem integration
    of its own mesh (own steps, rejections and end time)."""
    wb = configs.batched_vortices(nproblems=2, seed=5, nmin=9, nmax=16, nsteps=1)
    d = Discretisation(wb)
    u = d.initial_state(wb)
    h0, tend = np.array([0.05, 0.003]), np.array([0.06, 0.01])
    dp = S.Dopri5(d, 1e-7, 1e-7).start(u, [0.0, 0.0], h0, tend=tend)
    dp.run(25)
    assert np.all(dp.t == tend)
    for j in range(2):
        wj, _where = configs.single_problem(wb, j)
        dj = Discretisation(wj)
        sj = S.Dopri5(dj, 1e-7, 1e-7).start(dj.initial_state(wj), [0.0], [h0[j]], tend=[tend[j]])
        sj.run(25)
        hj = [e["h"][0] for e in sj.log if e["h"][0] > 0]
        hb = [e["h"][j] for e in dp.log if e["h"][j] > 0]
        assert np.allclose(hb, hj, rtol=1e-9)
        assert sj.t[0] == tend[j]
        ab = [bool(e["accept"][j]) for e in dp.log if e["h"][j] > 0]
        aj = [bool(e["accept"][0]) for e in sj.log if e["h"][0] > 0]
        assert ab == aj
