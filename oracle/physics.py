"""Euler / Navier-Stokes fluxes and interface fluxes (oracle side).

TEST INFRASTRUCTURE ONLY: see the package docstring.

Array convention: conserved variables u have shape (NV, ...) ordered
(rho, rho v_1..rho v_D, E); gradients q have shape (D, NV, ...) with
q[j, a] = d u_a / d x_j; fluxes have shape (D, NV, ...) with f[j, a] the
j-th Cartesian component of the flux of field a.

All functions are written to accept complex arrays so that complex-step
differentiation through them is exact; ``cabs`` is |x| extended
analytically as x * sign(Re x).
"""
from __future__ import annotations

import numpy as np


def cabs(x):
    return x * np.sign(np.real(x))


def primitives(u, gamma):
    D = u.shape[0] - 2
    rho = u[0]
    v = u[1:1 + D] / rho
    E = u[D + 1]
    p = (gamma - 1.0) * (E - 0.5 * np.sum(u[1:1 + D] * v, axis=0))
    return rho, v, E, p


def inviscid_flux(u, gamma):
    """Euler flux (eq. eulerflux) with the ideal gas law (eq. idealgas)."""
    D = u.shape[0] - 2
    rho, v, E, p = primitives(u, gamma)
    f = np.empty((D,) + u.shape, dtype=u.dtype)
    for j in range(D):
        f[j, 0] = u[1 + j]
        for i in range(D):
            f[j, 1 + i] = u[1 + i] * v[j] + (p if i == j else 0.0)
        f[j, D + 1] = (E + p) * v[j]
    return f


def viscous_flux(u, q, gamma, mu, prandtl):
    """Viscous flux (eq. visflux): stress tensor with Stokes' hypothesis and
    the heat flux Delta grad T, Delta = mu Cp / Pr, T = p / (rho Cv (g-1)).
    With gamma = Cp/Cv the heat term is mu gamma / (Pr (g-1)) grad(p/rho),
    so no gas constant is needed.  Primitive gradients by the quotient rule."""
    D = u.shape[0] - 2
    rho, v, E, p = primitives(u, gamma)
    # grad v_i, grad p, grad (p/rho)
    dv = np.empty((D, D) + rho.shape, dtype=u.dtype)             # dv[j, i] = d_j v_i
    for j in range(D):
        for i in range(D):
            dv[j, i] = (q[j, 1 + i] - v[i] * q[j, 0]) / rho
    divv = sum(dv[k, k] for k in range(D))
    f = np.zeros((D,) + u.shape, dtype=u.dtype)
    kappa = mu * gamma / (prandtl * (gamma - 1.0))
    for j in range(D):
        dp = (gamma - 1.0) * (q[j, D + 1]
                              - sum(v[i] * q[j, 1 + i] for i in range(D))
                              + 0.5 * sum(v[i] * v[i] for i in range(D)) * q[j, 0])
        dT = (dp - (p / rho) * q[j, 0]) / rho
        energy = kappa * dT
        for i in range(D):
            tau = mu * (dv[i, j] + dv[j, i]) - (2.0 / 3.0 * mu * divv if i == j else 0.0)
            f[j, 1 + i] = tau
            energy = energy + v[i] * tau
        f[j, D + 1] = energy
    return f


def flux(u, q, params):
    """f = f_inv - f_vis (f_vis only for Navier-Stokes)."""
    f = inviscid_flux(u, params["gamma"])
    if params["system"] == "ns":
        f = f - viscous_flux(u, q, params["gamma"], params["mu"], params["prandtl"])
    return f


def rusanov_wave_speed(uL, uR, n, gamma):
    """The wave-speed estimate s of the Rusanov flux (Appendix B): the
    sound speed of the summed pressures over the summed densities plus half
    the magnitude of the normal component of the summed velocities,
    s = sqrt(g (pL+pR)/(rhoL+rhoR)) + |n.(vL+vR)|/2."""
    rL, vL, _, pL = primitives(uL, gamma)
    rR, vR, _, pR = primitives(uR, gamma)
    D = n.shape[0]
    vn = sum(n[j] * (vL[j] + vR[j]) for j in range(D))
    return np.sqrt(gamma * (pL + pR) / (rL + rR)) + 0.5 * cabs(vn)


def rusanov(uL, uR, n, gamma):
    """Rusanov / local Lax-Friedrichs flux (Appendix B):
    F = n.(fL + fR)/2 + s (uL - uR)/2 with s from rusanov_wave_speed.
    n has shape (D, ...) and is the normal of the L side."""
    fL = inviscid_flux(uL, gamma)
    fR = inviscid_flux(uR, gamma)
    D = n.shape[0]
    s = rusanov_wave_speed(uL, uR, n, gamma)
    nf = sum(n[j] * (fL[j] + fR[j]) for j in range(D))
    return 0.5 * nf + 0.5 * s * (uL - uR)


def common_flux(uL, uR, qL, qR, n, params):
    """Common normal flux of eq. commpflux.  Euler: Rusanov.  Navier-Stokes:
    LDG, F = F_inv - n.((1/2+beta) fvis_L + (1/2-beta) fvis_R) + tau (uL-uR)
    (penalty taken with the dissipative sign)."""
    F = rusanov(uL, uR, n, params["gamma"])
    if params["system"] == "ns":
        g, mu, pr = params["gamma"], params["mu"], params["prandtl"]
        beta, tau = params["ldg_beta"], params["ldg_tau"]
        fvL = viscous_flux(uL, qL, g, mu, pr)
        fvR = viscous_flux(uR, qR, g, mu, pr)
        D = n.shape[0]
        fv = sum(n[j] * ((0.5 + beta) * fvL[j] + (0.5 - beta) * fvR[j]) for j in range(D))
        F = F - fv + tau * (uL - uR)
    return F


def common_solution(uL, uR, beta):
    """LDG common solution C(uL, uR) = (1/2 - beta) uL + (1/2 + beta) uR."""
    return (0.5 - beta) * uL + (0.5 + beta) * uR


# ---------------------------------------------------------------------------
# Boundary conditions (Appendix C): ghost states of the boundary element's
# solution at its flux points.  A boundary flux point is an interface of its
# own with the boundary element as the L side.
# ---------------------------------------------------------------------------
def boundary_ghosts(uL, qL, bc, gamma):
    """(B_inv u_L, B_ldg u_L, B_ldg q_L) for one boundary condition; uL is
    (NV, m), qL (D, NV, m) or None (Euler)."""
    D = uL.shape[0] - 2
    rho = uL[0]
    kind = bc["type"]
    if kind == "supersonic-inflow":
        rf, pf = bc["rho"], bc["p"]
        vf = np.asarray(bc["v"][:D], dtype=float)
        g = np.empty_like(uL)
        g[0] = rf
        g[1:1 + D] = rf * vf[:, None]
        g[D + 1] = pf / (gamma - 1) + 0.5 * rf * np.dot(vf, vf)
        return g, g, None if qL is None else np.zeros_like(qL)
    if kind == "subsonic-outflow":
        g = uL.copy()
        v = uL[1:1 + D] / rho
        g[D + 1] = bc["p"] / (gamma - 1) + 0.5 * rho * np.sum(v * v, axis=0)
        return g, g, None if qL is None else np.zeros_like(qL)
    if kind == "no-slip-isothermal-wall":
        vw = np.asarray(bc["vw"][:D], dtype=float)[:, None]
        w = 2 * vw - uL[1:1 + D] / rho
        e = bc["cp_tw"] / gamma
        ginv = np.concatenate([rho[None], rho * w, rho * (e + 0.5 * np.sum(w * w, axis=0))[None]])
        gldg = np.concatenate([rho[None], rho * vw * np.ones_like(rho),
                               rho[None] * (e + 0.5 * float(np.sum(vw * vw)))])
        return ginv, gldg, qL
    raise ValueError(kind)


def boundary_common_solution(uL, bc, params):
    """Common solution at boundary flux points: C(u_L, B_ldg u_L)."""
    _, gldg, _ = boundary_ghosts(uL, None, bc, params["gamma"])
    return common_solution(uL, gldg, params["ldg_beta"])


def boundary_common_flux(uL, qL, n, bc, params):
    """Common normal flux at boundary flux points: the Rusanov flux with the
    inviscid ghost and, for Navier-Stokes, the LDG viscous flux and penalty
    with the LDG ghost state and gradient."""
    ginv, gldg, gq = boundary_ghosts(uL, qL, bc, params["gamma"])
    F = rusanov(uL, ginv, n, params["gamma"])
    if params["system"] == "ns":
        g, mu, pr = params["gamma"], params["mu"], params["prandtl"]
        beta, tau = params["ldg_beta"], params["ldg_tau"]
        fvL = viscous_flux(uL, qL, g, mu, pr)
        fvR = viscous_flux(gldg, gq, g, mu, pr)
        D = n.shape[0]
        fv = sum(n[j] * ((0.5 + beta) * fvL[j] + (0.5 - beta) * fvR[j]) for j in range(D))
        F = F - fv + tau * (uL - gldg)
    return F
