"""The Euler-vortex super-accuracy test of the validation section at short
horizons, on the library: p = 3 on [-20, 20]^2 with h = 1/3, 2/7, 1/4, 2/9,
RK4 steps of 0.00125, DG, SD and HU corrections.  Every 40 time units the
vortex is back on the origin; there the L2 density error sigma over the box
[-2, 2]^2 (an 8 x 8 Gauss rule per element, of the numerical polynomial
against the initial field) gives, by a least-squares fit of log sigma against
log h over the four meshes, the observed order of each scheme.  The order
must be at least p + 1/2; the values are printed."""
import math

import numpy as np
import pytest

import frcases as C
from oracle import reference
from workloads import configs

pytestmark = pytest.mark.gpu

HORIZONS = (40.0, 80.0)


def _box_sigma(s, t, w, n):
    """sigma over the elements inside [-2, 2]^2 (straight quads of side h:
    J = h^2/4) with an 8 x 8 Gauss rule."""
    h = configs.VORTEX_E1["L"] / n
    xq, wq = reference.gauss_legendre(8)
    q = np.stack(np.meshgrid(xq, xq, indexing="xy"), -1).reshape(-1, 2)    # xi fastest
    wqq = np.outer(wq, wq).ravel()
    r = reference.ref_element("quad", w.mesh.blocks[0].order)
    B = r.basis(q)                                                          # (64, Nu)
    nodes = w.mesh.blocks[0].nodes                                          # (ne, 4, 2)
    lo = nodes.min(axis=1)
    centre = lo + 0.5 * h
    sel = np.nonzero(np.all(np.abs(centre) < 2.0, axis=1))[0]
    rho = s.unpack(t)[0][:, 0, sel]                                         # (Nu, ne_box)
    rho_q = B @ rho                                                         # (64, ne_box)
    xphys = lo[sel][None, :, :] + 0.5 * h * (q[:, None, :] + 1.0)           # (64, ne_box, 2)
    exact = w.ic(0, xphys)[..., 0]
    return math.sqrt(float(np.sum(wqq[:, None] * (h * h / 4) * (rho_q - exact) ** 2)))


@pytest.mark.parametrize("scheme", ["dg", "sd", "hu"])
def test_vortex_superaccuracy_short_horizon(scheme):
    ns = list(configs.VORTEX_E1_SPACINGS.values())
    dt = configs.VORTEX_E1["dt"]
    per = int(round(configs.VORTEX_E1["L"] / dt))
    sig = np.zeros((len(HORIZONS), len(ns)))
    sig0 = np.zeros(len(ns))
    for j, n in enumerate(ns):
        w = configs.vortex_superaccuracy(n, scheme)
        s = C.solver_for(w)
        x = s.solution_points(0)
        t = s.pack([np.ascontiguousarray(np.transpose(w.ic(0, x), (1, 2, 0)))])
        sig0[j] = _box_sigma(s, t, w, n)
        done = 0
        for k, tc in enumerate(HORIZONS):
            steps = int(round(tc / dt)) - done
            s.step(t, dt, steps)
            done += steps
            sig[k, j] = _box_sigma(s, t, w, n)
    hs = np.array([configs.VORTEX_E1["L"] / n for n in ns])
    orders = [float(np.polyfit(np.log(hs), np.log(sig[k]), 1)[0]) for k in range(len(HORIZONS))]
    print(f"{scheme} t=0 (projection): sigma " + " ".join(f"{v:.4e}" for v in sig0)
          + f"  order {float(np.polyfit(np.log(hs), np.log(sig0), 1)[0]):.2f}")
    for k, tc in enumerate(HORIZONS):
        print(f"{scheme} t={tc:.0f}: sigma " + " ".join(f"{v:.4e}" for v in sig[k])
              + f"  order {orders[k]:.2f}")
    assert per * dt == configs.VORTEX_E1["L"]
    assert np.all(np.isfinite(sig))
    assert min(orders) >= 3.5
