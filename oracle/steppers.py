"""Explicit time steppers of the paper's functionality table (Table 1 of the
implementation section: Euler, RK4 and DOPRI5) beyond the RK4 of ``rhs.py``.

TEST INFRASTRUCTURE ONLY: see the package docstring.

The paper names the steppers and nothing more.  Forward Euler is
u <- u + dt R(u).  DOPRI5 is the explicit Dormand-Prince 5(4) pair (Dormand
and Prince 1980), taken as follows (readings of a silent paper):
* the fifth-order solution advances the state; the embedded fourth-order one
  only estimates the error, e = h sum_j (b_j - bhat_j) k_j;
* the seventh stage is evaluated at the new state (a_7j = b_j), so its slope
  is the next step's first (first same as last);
* err = sqrt(mean over a problem's degrees of freedom of
  (e_i / (atol + rtol max(|u_i|, |u5_i|)))^2);
* the step is accepted when err < 1; the next h is h min(10, 0.9 err^-1/5)
  after an acceptance (10 when err = 0, at most h when the same step had a
  rejection) and h max(0.2, 0.9 err^-1/5) after a rejection -- the standard
  controller of Hairer, Norsett and Wanner (Solving ODEs I, II.4);
* h is cut so that t + h does not pass an optional end time, which is then
  reached exactly; a problem at its end time takes no further steps;
* independent problems in one mesh each carry their own t, h, error norm and
  decisions.
"""
from __future__ import annotations

from fractions import Fraction as F

import numpy as np

# Dormand-Prince 5(4): nodes c, stage matrix a (lower triangle), fifth-order
# weights b (= the last row of a) and fourth-order weights bhat.
DP_C = [F(0), F(1, 5), F(3, 10), F(4, 5), F(8, 9), F(1), F(1)]
DP_A = [
    [],
    [F(1, 5)],
    [F(3, 40), F(9, 40)],
    [F(44, 45), F(-56, 15), F(32, 9)],
    [F(19372, 6561), F(-25360, 2187), F(64448, 6561), F(-212, 729)],
    [F(9017, 3168), F(-355, 33), F(46732, 5247), F(49, 176), F(-5103, 18656)],
    [F(35, 384), F(0), F(500, 1113), F(125, 192), F(-2187, 6784), F(11, 84)],
]
DP_B = DP_A[6] + [F(0)]
DP_BHAT = [F(5179, 57600), F(0), F(7571, 16695), F(393, 640), F(-92097, 339200),
           F(187, 2100), F(1, 40)]

SAFETY, FAC_MIN, FAC_MAX = 0.9, 0.2, 10.0


def element_problems(disc):
    """Problem id of every element, per block ((ne,) int arrays)."""
    out = []
    for b in disc.mesh.blocks:
        p = getattr(b, "problem", None)
        out.append(np.zeros(b.nelem, dtype=np.int64) if p is None else np.asarray(p, np.int64))
    return out


def euler(disc, state, dt, nsteps):
    """nsteps forward Euler steps, u <- u + dt R(u) (dt scalar)."""
    for _ in range(nsteps):
        state = [u + dt * k for u, k in zip(state, disc.rhs(state))]
    return state


class Dopri5:
    """Adaptive DOPRI5 over the problems of one discretisation.

    t, h: (nproblems,) float arrays; ``tend``: (nproblems,) or None.  The
    attempts counted by ``attempt`` include rejected ones; ``log`` keeps, per
    attempt, the step sizes tried, the error norms and the decisions."""

    def __init__(self, disc, atol, rtol):
        self.d = disc
        self.atol, self.rtol = float(atol), float(rtol)
        self.prob = element_problems(disc)
        self.nprob = int(getattr(disc.mesh, "nproblems", 1))
        self.ndof = np.zeros(self.nprob)
        for b, pr in enumerate(self.prob):
            r = disc.refs[b]
            np.add.at(self.ndof, pr, r.nupts * disc.nvars)
        self.log = []

    def _per_elem(self, v, b):
        return v[self.prob[b]][None, None, :]

    def start(self, state, t, h, tend=None):
        """Begin (or resume) integrating: the first stage slope at u, and h cut
        to the end times."""
        self.t = np.array(t, dtype=np.float64)
        self.h = np.array(h, dtype=np.float64)
        self.tend = None if tend is None else np.array(tend, dtype=np.float64)
        if not hasattr(self, "rejected"):
            self.rejected = np.zeros(self.nprob, dtype=bool)
        if self.tend is not None:
            self.h = np.minimum(self.h, self.tend - self.t)
        self.u = [np.array(x) for x in state]
        self.k1 = self.d.rhs(self.u)
        return self

    def attempt(self):
        """One attempt on every problem (problems with h <= 0 stand still)."""
        u, h = self.u, self.h
        k = [self.k1]
        for i in range(1, 7):
            a = [float(x) for x in DP_A[i]]
            y = []
            for b, ub in enumerate(u):
                inc = sum(a[j] * k[j][b] for j in range(i))
                y.append(ub + self._per_elem(h, b) * inc)
            k.append(self.d.rhs(y))
        u5 = y                                     # stage 7 is taken at the new state
        e_w = [float(bb - bh) for bb, bh in zip(DP_B, DP_BHAT)]
        ssq = np.zeros(self.nprob)
        msq = np.zeros(self.nprob)          # diagnostics only: the same norm of sum |E_j k_j|
        for b, ub in enumerate(u):
            e = self._per_elem(h, b) * sum(e_w[j] * k[j][b] for j in range(7))
            sc = self.atol + self.rtol * np.maximum(np.abs(ub), np.abs(u5[b]))
            np.add.at(ssq, self.prob[b], np.sum((e / sc) ** 2, axis=(0, 1)))
            m = self._per_elem(h, b) * sum(abs(e_w[j]) * np.abs(k[j][b]) for j in range(7))
            np.add.at(msq, self.prob[b], np.sum((m / sc) ** 2, axis=(0, 1)))
        err = np.sqrt(ssq / self.ndof)
        # amplification of relative perturbations of the slopes into err
        with np.errstate(divide="ignore", invalid="ignore"):
            cond = np.sqrt(msq / self.ndof) / err
        active = h > 0
        accept = active & (err < 1.0)
        reject = active & ~accept
        with np.errstate(divide="ignore", invalid="ignore"):
            grow = np.where(err == 0.0, FAC_MAX,
                            np.minimum(FAC_MAX, SAFETY * err ** -0.2))
            shrink = np.maximum(FAC_MIN, SAFETY * err ** -0.2)
        shrink = np.where(np.isnan(err), FAC_MIN, shrink)
        grow = np.where(self.rejected, np.minimum(1.0, grow), grow)
        t_new = self.t + h
        if self.tend is not None:
            t_new = np.where(h >= self.tend - self.t, self.tend, t_new)
        self.log.append(dict(h=h.copy(), err=err, cond=cond, accept=accept.copy(),
                             reject=reject.copy()))
        self.t = np.where(accept, t_new, self.t)
        self.h = np.where(accept, h * grow, np.where(reject, h * shrink, h))
        self.rejected = np.where(accept, False, np.where(reject, True, self.rejected))
        if self.tend is not None:
            self.h = np.minimum(self.h, self.tend - self.t)
        self.u = [np.where(self._per_elem(accept.astype(float), b) > 0, u5[b], ub)
                  for b, ub in enumerate(u)]
        self.k1 = [np.where(self._per_elem(accept.astype(float), b) > 0, k[6][b], kb)
                   for b, kb in enumerate(self.k1)]
        return accept, reject

    def run(self, nattempts):
        for _ in range(nattempts):
            self.attempt()
        return self
