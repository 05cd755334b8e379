"""Analytic flow fields evaluated at given physical coordinates.

Each function maps coordinates ``x`` of shape (..., ndims) to conserved
variables of shape (..., nvars) in the field order (rho, rho v_x, rho v_y
[, rho v_z], E) of the Euler equations.  Coordinates come from whichever side
(library or oracle) placed the solution points; these functions know nothing
about the discretisation.
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4


def primitive_to_conserved(rho, vel, p, gamma=GAMMA):
    """rho, vel (..., D), p -> (..., D+2) conserved; ideal gas E = p/(g-1) + rho|v|^2/2."""
    vel = np.asarray(vel)
    E = p / (gamma - 1.0) + 0.5 * rho * np.sum(vel * vel, axis=-1)
    return np.concatenate([rho[..., None], rho[..., None] * vel, E[..., None]], axis=-1)


def isentropic_vortex(x, S=5.0, R=1.0, M=None, gamma=GAMMA, centre=(0.0, 0.0),
                      shift=(0.0, 0.0)):
    """Isentropic vortex translating with free stream (1, 0).

    The paper's vortex (validation section) with its free stream rotated onto
    +x and its sense reflected; with M = gamma^-1/2 the far-field pressure is 1.
    ``shift`` evaluates the exact solution after translation by ``shift``.
    """
    if M is None:
        M = gamma ** -0.5
    X = x[..., 0] - centre[0] - shift[0]
    Y = x[..., 1] - centre[1] - shift[1]
    f = (1.0 - X * X - Y * Y) / (2.0 * R * R)
    ef = np.exp(f)
    rho = (1.0 - S * S * M * M * (gamma - 1.0) * ef * ef / (8.0 * np.pi ** 2)) ** (1.0 / (gamma - 1.0))
    u = 1.0 - S * Y * ef / (2.0 * np.pi * R)
    v = S * X * ef / (2.0 * np.pi * R)
    p = rho ** gamma / (gamma * M * M)
    return primitive_to_conserved(rho, np.stack([u, v], -1), p, gamma)


def taylor_green(x, Ma=0.1, gamma=GAMMA):
    """Taylor-Green vortex on [0, 2 pi]^3 with rho0 = V0 = L = 1 (isothermal rho = p/p0)."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    p0 = 1.0 / (gamma * Ma * Ma)
    u = np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(u)
    p = p0 + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
    rho = p / p0
    return primitive_to_conserved(rho, np.stack([u, v, w], -1), p, gamma)


def uniform(x, rho=1.0, vel=(1.0, 0.5, 0.25), p=1.0, gamma=GAMMA):
    D = x.shape[-1]
    shape = x.shape[:-1]
    v = np.broadcast_to(np.asarray(vel[:D], float), shape + (D,))
    return primitive_to_conserved(np.full(shape, rho), v, np.full(shape, p), gamma)


def freestream_modes(ndims, seed, nmodes=4, eps=0.05, kmax=2):
    """Draw the random smooth perturbation used on the curved periodic box.

    Fields (rho, v_1..v_D, p) in that order, then modes, then (k, a, phi):
    k uniform in {-kmax..kmax}^D minus 0, a ~ U[-1,1], phi ~ U[0, 2 pi).
    """
    rng = np.random.default_rng(seed)
    modes = []
    for _field in range(ndims + 2):
        fm = []
        for _m in range(nmodes):
            while True:
                k = rng.integers(-kmax, kmax + 1, size=ndims)
                if np.any(k != 0):
                    break
            a = rng.uniform(-1.0, 1.0)
            phi = rng.uniform(0.0, 2.0 * np.pi)
            fm.append((k.astype(float), a, phi))
        modes.append(fm)
    return dict(modes=modes, eps=eps)


def perturbed_freestream(x, modes, vel=(1.0, 0.5, 0.25), Ma=0.5, gamma=GAMMA,
                         period=1.0):
    D = x.shape[-1]
    v = np.asarray(vel[:D], float)
    v = v / np.linalg.norm(v)
    base = [1.0] + list(v) + [1.0 / (gamma * Ma * Ma)]
    prim = []
    for f, fm in enumerate(modes["modes"]):
        val = np.full(x.shape[:-1], base[f])
        for k, a, phi in fm:
            val = val + modes["eps"] * a * np.sin(2.0 * np.pi * (x @ k) / period + phi)
        prim.append(val)
    rho = prim[0]
    vel_ = np.stack(prim[1:1 + D], -1)
    p = prim[1 + D]
    return primitive_to_conserved(rho, vel_, p, gamma)


# Couette flow between isothermal plates (paper section 5): the bottom plate
# (y = 0) at rest, the top plate (y = H) moving with speed v_w in x.
COUETTE = dict(gamma=1.4, prandtl=0.72, mu=0.417, cp=1005.0, H=1.0, Tw=300.0, pc=1.0e5,
               vw=69.445)


def couette_density(phi, c=COUETTE):
    g = c["gamma"]
    return g / (g - 1) * 2 * c["pc"] / (2 * c["cp"] * c["Tw"] + c["prandtl"] * c["vw"] ** 2
                                        * phi * (1 - phi))


def couette(x, c=COUETTE):
    """The exact steady solution at points x (..., D), conserved variables."""
    phi = x[..., 1] / c["H"]
    rho = couette_density(phi, c)
    vel = np.stack([c["vw"] * phi] + [np.zeros_like(phi)] * (x.shape[-1] - 1), -1)
    return primitive_to_conserved(rho, vel, np.full_like(phi, c["pc"]), c["gamma"])


def couette_initial(x, c=COUETTE):
    """The paper's constant start: the mean density, v = v_w x, p = p_c."""
    t, w = np.polynomial.legendre.leggauss(64)
    rho_mean = 0.5 * np.sum(w * couette_density(0.5 * (t + 1), c))
    shape = x.shape[:-1]
    vel = np.stack([np.full(shape, c["vw"])] + [np.zeros(shape)] * (x.shape[-1] - 1), -1)
    return primitive_to_conserved(np.full(shape, rho_mean), vel, np.full(shape, c["pc"]),
                                  c["gamma"])
