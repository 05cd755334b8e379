"""Pins of the oracle's interface fluxes that the invariants leave open.

Consistency, antisymmetry and rotation invariance hold for any wave speed s
that is symmetric in the two sides and rotation invariant, so they cannot
tell the Rusanov flux of App. B from a plausible variant of it (the larger
of the two sides' speeds, gamma dropped, the 1/2 on |n.v| dropped).  Here s
and the flux are checked against values worked out by hand from the printed
formula (tests/golden/rusanov.txt), and each variant, planted in the oracle,
is shown to fail that check.

The sign of the LDG penalty (paper section 4, LDG flux) is a reading: taken
literally, the printed flux subtracts tau (u_L - u_R), which adds energy for
tau > 0.  The eigenvalue diagnostic below linearises the oracle's right-hand
side about a fluid at rest and records both readings.
"""
import os

import numpy as np
import pytest

from oracle import Discretisation, jvp, physics
from workloads import meshes
from workloads.configs import Workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rusanov.txt")
GAMMA = 1.4


def _golden():
    cases = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, key, *vals = line.split()
            cases.setdefault(name, {})[key] = np.array([float(v) for v in vals])
    return cases


def _conserved(rho, v, p):
    """(NV, 1) conserved state from primitives (E = p/(g-1) + rho |v|^2/2)."""
    E = p / (GAMMA - 1) + 0.5 * rho * np.dot(v, v)
    return np.concatenate([rho, rho * v, E])[:, None]


def _states(c):
    uL = _conserved(c["rhoL"], c["vL"], c["pL"])
    uR = _conserved(c["rhoR"], c["vR"], c["pR"])
    return uL, uR, c["n"][:, None]


def _flux_errors():
    """Largest |oracle - golden| of s and F over the golden cases."""
    es = ef = 0.0
    for c in _golden().values():
        uL, uR, n = _states(c)
        s = physics.rusanov_wave_speed(uL, uR, n, GAMMA)
        F = physics.rusanov(uL, uR, n, GAMMA)
        es = max(es, float(np.abs(s[0] - c["s"][0])))
        ef = max(ef, float(np.abs(F[:, 0] - c["F"]).max()))
    return es, ef


def test_rusanov_golden_values():
    """s, the central part n.(fL + fR)/2 and F of three hand-worked cases
    (2-D and 3-D, one with a negative normal velocity)."""
    g = _golden()
    assert sorted(g) == ["A", "B", "C"]
    for name, c in g.items():
        uL, uR, n = _states(c)
        D = n.shape[0]
        s = physics.rusanov_wave_speed(uL, uR, n, GAMMA)
        assert abs(s[0] - c["s"][0]) < 1e-14, (name, s, c["s"])
        fL, fR = physics.inviscid_flux(uL, GAMMA), physics.inviscid_flux(uR, GAMMA)
        central = 0.5 * sum(n[j] * (fL[j] + fR[j]) for j in range(D))
        assert np.abs(central[:, 0] - c["central"]).max() < 1e-13, (name, central[:, 0])
        F = physics.rusanov(uL, uR, n, GAMMA)
        assert np.abs(F[:, 0] - c["F"]).max() < 1e-13, (name, F[:, 0], c["F"])
        # the dissipative part is exactly s (uL - uR) / 2, field by field
        diss = F[:, 0] - c["central"]
        assert np.abs(diss - 0.5 * c["s"][0] * (uL - uR)[:, 0]).max() < 1e-13


def _speed_max_of_sides(uL, uR, n, gamma):
    out = []
    for u in (uL, uR):
        rho, v, _, p = physics.primitives(u, gamma)
        vn = sum(n[j] * v[j] for j in range(n.shape[0]))
        out.append(np.sqrt(gamma * p / rho) + np.abs(vn))
    return np.maximum(*out)


def _speed_no_gamma(uL, uR, n, gamma):
    rL, vL, _, pL = physics.primitives(uL, gamma)
    rR, vR, _, pR = physics.primitives(uR, gamma)
    vn = sum(n[j] * (vL[j] + vR[j]) for j in range(n.shape[0]))
    return np.sqrt((pL + pR) / (rL + rR)) + 0.5 * np.abs(vn)


def _speed_no_half(uL, uR, n, gamma):
    rL, vL, _, pL = physics.primitives(uL, gamma)
    rR, vR, _, pR = physics.primitives(uR, gamma)
    vn = sum(n[j] * (vL[j] + vR[j]) for j in range(n.shape[0]))
    return np.sqrt(gamma * (pL + pR) / (rL + rR)) + np.abs(vn)


def _speed_signed(uL, uR, n, gamma):
    rL, vL, _, pL = physics.primitives(uL, gamma)
    rR, vR, _, pR = physics.primitives(uR, gamma)
    vn = sum(n[j] * (vL[j] + vR[j]) for j in range(n.shape[0]))
    return np.sqrt(gamma * (pL + pR) / (rL + rR)) + 0.5 * vn


def _speed_mean_of_sound_speeds(uL, uR, n, gamma):
    rL, vL, _, pL = physics.primitives(uL, gamma)
    rR, vR, _, pR = physics.primitives(uR, gamma)
    vn = sum(n[j] * (vL[j] + vR[j]) for j in range(n.shape[0]))
    return 0.5 * (np.sqrt(gamma * pL / rL) + np.sqrt(gamma * pR / rR)) + 0.5 * np.abs(vn)


@pytest.mark.parametrize("variant", [_speed_max_of_sides, _speed_no_gamma, _speed_no_half,
                                     _speed_signed, _speed_mean_of_sound_speeds])
def test_rusanov_golden_catches_planted_wave_speeds(monkeypatch, variant):
    """Each plausible misreading of s, planted in the oracle, moves F by far
    more than rounding in at least one golden case."""
    assert max(_flux_errors()) < 1e-13
    monkeypatch.setattr(physics, "rusanov_wave_speed", variant)
    es, ef = _flux_errors()
    assert es > 1e-3 and ef > 1e-3, (variant.__name__, es, ef)


def _rest_box(n, p, tau):
    """Navier-Stokes on a periodic n x n quad box at rest (rho 1, p 1)."""
    mesh = meshes.quad_mesh(n, n, (0.0, 0.0), (1.0, 1.0), order=p)

    def ic(b, x):
        u = np.zeros(x.shape[:-1] + (4,))
        u[..., 0] = 1.0
        u[..., 3] = 1.0 / (GAMMA - 1)
        return u
    return Workload("rest", mesh, "ns", mu=0.05, prandtl=0.72, ldg_beta=0.5, ldg_tau=tau, ic=ic)


def _max_real_eigenvalue(tau, n=3, p=2):
    """max Re(lambda) and max |lambda| of dR/du about the rest state, the
    Jacobian assembled column by column from complex-step JVPs."""
    w = _rest_box(n, p, tau)
    d = Discretisation(w)
    u = d.initial_state(w)
    shape = u[0].shape
    N = u[0].size
    J = np.empty((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        J[:, k] = jvp(d, u, [e.reshape(shape)])[0].ravel()
    lam = np.linalg.eigvals(J)
    return float(lam.real.max()), float(np.abs(lam).max())


def test_ldg_penalty_sign_eigenvalues(monkeypatch):
    """With the Rusanov dissipation switched off (s := 0, in this test only)
    and tau = 1, the linearised operator about a fluid at rest is
    non-expansive for the dissipative reading, +tau (u_L - u_R) in the total
    flux, and has eigenvalues with a clearly positive real part for the
    literal one, -tau (u_L - u_R).  The literal reading is the adopted
    formula with tau -> -tau."""
    monkeypatch.setattr(physics, "rusanov_wave_speed",
                        lambda uL, uR, n, gamma: 0.0 * uL[0])
    adopted, scale = _max_real_eigenvalue(+1.0)
    literal, scale_l = _max_real_eigenvalue(-1.0)
    print(f"max Re lambda: dissipative sign {adopted:.3e}, literal sign {literal:.3e}, "
          f"max |lambda| {scale:.3e} / {scale_l:.3e}")
    assert adopted <= 1e-10 * scale
    assert literal > 1e-2 * scale_l
