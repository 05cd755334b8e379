"""The FR semi-discrete right-hand side and classical RK4 (oracle side).

TEST INFRASTRUCTURE ONLY: see the package docstring.

The right-hand side follows paper section 2 in its direct index form, one
equation per step, with no pre-multiplied operators:

  1. u^f_sigma = sum_rho l_rho(x^f_sigma) u_rho                      (eq. ufpts)
  2. common solution at each flux-point pair, same value both sides (eq. commsoln)
  3. transformed gradient q~ = n~_sigma (div g_sigma)(C u - u^f)
     + sum_nu u_nu grad~ l_nu                                        (eq. transqu)
  4. q = J^-T q~ at solution points
  5. q^f = sum_rho l_rho(x^f_sigma) q_rho                            (eq. gradufpts)
  6. transformed flux f~ = J J^-1 f(u, q) at solution points
  7. f~perp_sigma = sum_rho l_rho(x^f_sigma) n~_sigma . f~_rho        (eq. tnormfluxf)
  8. common normal flux at each pair, scaled by J^(f) n^(f) per side,
     with opposite signs on the two sides                            (eq. commpflux)
  9. div~ f~ = (div g_sigma)(F f~perp - f~perp) + f~_nu . grad~ l_nu (eq. tdivflux)
 10. du/dt = -J^-1 div~ f~                                           (eq. negdivconf)

Steps 2-5 run only for Navier-Stokes.  State arrays follow the library's
public layout per block, u[rho, alpha, n].
"""
from __future__ import annotations

import numpy as np

from . import geometry, physics, reference


def _es(spec, *ops):
    """einsum with contraction-order optimisation (library primitive)."""
    return np.einsum(spec, *ops, optimize=True)


class Discretisation:
    """Set-up of one mesh: reference elements, geometry, flux-point pairs."""

    def __init__(self, workload, allow_unpaired=False):
        """allow_unpaired: the mesh is a patch cut out of a larger mesh; faces
        on its outer boundary have no partner and receive no common flux, so
        du/dt is right only on elements whose face neighbours (Euler), and
        their face neighbours (Navier-Stokes), are in the patch."""
        w = workload
        self.mesh = w.mesh
        self.ndims = w.mesh.ndims
        self.nvars = self.ndims + 2
        self.params = dict(system=w.system, gamma=w.gamma, mu=w.mu,
                           prandtl=w.prandtl, ldg_beta=w.ldg_beta,
                           ldg_tau=w.ldg_tau)
        self.refs = [reference.ref_element(b.etype, b.order, getattr(b, "correction", "dg"))
                     for b in w.mesh.blocks]
        self.geoms = [geometry.BlockGeometry(r, b) for r, b in zip(self.refs, w.mesh.blocks)]
        for g in self.geoms:
            if np.any(g.detJ <= 0) or np.any(g.detJf <= 0):
                raise ValueError("non-positive Jacobian")
        # flux points on boundary faces (Appendix C): (block, elem, sigma, bc)
        self.bcs = tuple(getattr(w.mesh, "bcs", ()))
        bcf = getattr(w.mesh, "bcfaces", None)
        bb, be, bs, bk = [], [], [], []
        if bcf is not None:
            for rec in bcf:
                b, e, f, k = int(rec["block"]), int(rec["elem"]), int(rec["face"]), int(rec["bc"])
                sig = np.nonzero(self.refs[b].fface == f)[0]
                bb += [b] * len(sig); be += [e] * len(sig); bs += list(sig); bk += [k] * len(sig)
        self.bnd = dict(b=np.array(bb, np.int64), e=np.array(be, np.int64),
                        s=np.array(bs, np.int64), bc=np.array(bk, np.int64))
        pr = geometry.pair_flux_points(w.mesh, self.refs, self.geoms,
                                       allow_unpaired=allow_unpaired,
                                       boundary=(self.bnd["b"], self.bnd["e"], self.bnd["s"]))
        self.pairs = pr
        # flat index of a flux point (block, sigma, n) into the concatenation
        # of every block's (Nf, ne) flux-point array
        self.fbase = np.cumsum([0] + [r.nfpts * g.nelem for r, g in zip(self.refs, self.geoms)])
        self.gl = self._flat(pr["lb"], pr["ls"], pr["le"])
        self.gr = self._flat(pr["rb"], pr["rs"], pr["re"])
        self.nL, self.magL, self.magR = self._pair_metrics(self.geoms)
        self.gb = self._flat(self.bnd["b"], self.bnd["s"], self.bnd["e"])
        self.nB, self.magB = self._boundary_metrics(self.geoms)
        self.dt_per_elem = None

    def _pair_metrics(self, geoms):
        """Unit normal of the L side (D, npairpts) and J^(f) n^(f) of both
        sides at every flux-point pair."""
        pr = self.pairs
        D = self.ndims
        dt = geoms[0].fmag.dtype
        nL = np.empty((len(self.gl), D), dtype=dt)
        magL = np.empty(len(self.gl), dtype=dt)
        magR = np.empty(len(self.gl), dtype=dt)
        for b, g in enumerate(geoms):
            s = pr["lb"] == b
            nL[s] = g.fnhat[pr["le"][s], pr["ls"][s]]
            magL[s] = g.fmag[pr["le"][s], pr["ls"][s]]
            s = pr["rb"] == b
            magR[s] = g.fmag[pr["re"][s], pr["rs"][s]]
        return nL.T.copy(), magL, magR

    def _boundary_metrics(self, geoms):
        """Outward unit normal (D, nbpts) and J^(f) n^(f) at boundary flux points."""
        bd = self.bnd
        dt = geoms[0].fmag.dtype
        nB = np.empty((len(bd["b"]), self.ndims), dtype=dt)
        magB = np.empty(len(bd["b"]), dtype=dt)
        for b, g in enumerate(geoms):
            s = bd["b"] == b
            nB[s] = g.fnhat[bd["e"][s], bd["s"][s]]
            magB[s] = g.fmag[bd["e"][s], bd["s"][s]]
        return nB.T.copy(), magB

    def extended(self):
        """A copy whose metric terms and normals are recomputed from the nodes
        in long double, so ``rhs`` on long-double states evaluates the same
        formula, geometry included, with 64-bit significands.  Used only to
        measure the FP64 rounding floor of a case (how far an FP64 evaluation
        of this formula can sit from the exact value of the same formula)."""
        import copy
        e = copy.copy(self)
        e.geoms = [geometry.BlockGeometry(r, b, np.longdouble)
                   for r, b in zip(self.refs, self.mesh.blocks)]
        e.nL, e.magL, e.magR = self._pair_metrics(e.geoms)
        e.nB, e.magB = self._boundary_metrics(e.geoms)
        return e

    def _flat(self, b, s, e):
        ne = np.array([g.nelem for g in self.geoms])
        return self.fbase[b] + s * ne[b] + e

    # -- layout helpers ------------------------------------------------------
    def solution_coords(self):
        """Physical solution-point coordinates per block, (ne, Nu, D)."""
        return [g.xu for g in self.geoms]

    def initial_state(self, workload):
        """Collocation projection of the analytic initial field: the field's
        values at the solution points, returned as u[rho, alpha, n]."""
        out = []
        for b, g in enumerate(self.geoms):
            u = workload.ic(b, g.xu)                                  # (ne, Nu, NV)
            out.append(np.ascontiguousarray(np.transpose(u, (1, 2, 0))))
        return out

    def _to_flat(self, arrs):
        """Per-block (..., Nf, NV, ne) -> (..., NV, total flux points)."""
        parts = []
        for a in arrs:
            a = np.swapaxes(a, -3, -2)                                # (..., NV, Nf, ne)
            parts.append(a.reshape(a.shape[:-2] + (-1,)))
        return np.concatenate(parts, axis=-1)

    def _from_flat(self, flat, b):
        """Inverse of _to_flat for block b: (..., NV, nfp) -> (..., Nf, NV, ne)."""
        r, g = self.refs[b], self.geoms[b]
        seg = flat[..., self.fbase[b]:self.fbase[b + 1]]
        seg = seg.reshape(seg.shape[:-1] + (r.nfpts, g.nelem))
        return np.swapaxes(seg, -3, -2)

    # -- right-hand side -------------------------------------------------------
    def rhs(self, state, record=None):
        """du/dt per block.  If ``record`` is a dict it receives the
        intermediate arrays of every step, per block: uf, cf, qt, q, qf, ft,
        df (flux-point arrays as [sigma, alpha, n], vectors as [i, row,
        alpha, n])."""
        P = self.params
        ns = P["system"] == "ns"
        D = self.ndims
        refs, geoms = self.refs, self.geoms
        nb = len(refs)
        # 1. solution at flux points
        uf = [_es("sr,ran->san", refs[b].L_f, state[b]) for b in range(nb)]
        UF = self._to_flat(uf)                                        # (NV, nfp)
        uL, uR = UF[:, self.gl], UF[:, self.gr]
        q = [None] * nb
        qf_flat = None
        if ns:
            # 2. common solution, assigned to both members of each pair
            c = physics.common_solution(uL, uR, P["ldg_beta"])
            CF = np.zeros_like(UF)        # zero at unpaired points of a patch
            CF[:, self.gl] = c
            CF[:, self.gr] = c
            # boundary flux points: common solution with the boundary's ghost
            for k, bc in enumerate(self.bcs):
                sel = self.gb[self.bnd["bc"] == k]
                CF[:, sel] = physics.boundary_common_solution(UF[:, sel], bc, P)
            qfs = []
            for b in range(nb):
                r, g = refs[b], geoms[b]
                jump = self._from_flat(CF, b) - uf[b]                 # (Nf, NV, ne)
                # 3. transformed gradient at solution points
                qt = (_es("irv,van->iran", r.D_u, state[b])
                      + _es("rs,si,san->iran", r.divg, r.fnorm, jump))
                if record is not None:
                    record.setdefault("cf", []).append(self._from_flat(CF, b))
                    record.setdefault("qt", []).append(qt)
                # 4. physical gradient q_j = (1/J) sum_i S_ij q~_i
                qb = _es("nrij,iran->jran", g.S, qt) / g.detJ.T[None, :, None, :]
                q[b] = qb
                if record is not None:
                    record.setdefault("q", []).append(qb)
                # 5. gradient at flux points
                qfs.append(_es("sr,jran->jsan", r.L_f, qb))
            qf_flat = self._to_flat(qfs)                              # (D, NV, nfp)
            if record is not None:
                record["qf"] = qfs
        # 6-7. transformed flux at solution points, its normal component at
        # flux points
        Ft, fperp = [], []
        for b in range(nb):
            r, g = refs[b], geoms[b]
            # physics works on (NV, ...) / (D, NV, ...) arrays
            ub = np.swapaxes(state[b], 0, 1)                          # (NV, Nu, ne)
            qb = np.swapaxes(q[b], 1, 2) if ns else None              # (D, NV, Nu, ne)
            f = np.swapaxes(physics.flux(ub, qb, P), 1, 2)            # (D, Nu, NV, ne)
            Ft_b = _es("nrij,jran->iran", g.S, f)
            Ft.append(Ft_b)
            fperp.append(_es("sr,si,iran->san", r.L_f, r.fnorm, Ft_b))
        # 8. common normal flux per pair, into reference space on each side
        qL = qf_flat[:, :, self.gl] if ns else None
        qR = qf_flat[:, :, self.gr] if ns else None
        F = physics.common_flux(uL, uR, qL, qR, self.nL, P)
        DF = np.zeros_like(UF)
        DF[:, self.gl] = self.magL * F
        DF[:, self.gr] = -self.magR * F
        # boundary flux points: common normal flux with the boundary's ghosts,
        # scaled like an L side
        for k, bc in enumerate(self.bcs):
            m = self.bnd["bc"] == k
            sel = self.gb[m]
            qB = qf_flat[:, :, sel] if ns else None
            FB = physics.boundary_common_flux(UF[:, sel], qB, self.nB[:, m], bc, P)
            DF[:, sel] = self.magB[m] * FB
        if record is not None:
            record["uf"] = uf
            record["ft"] = Ft
            record["df"] = [self._from_flat(DF, b) for b in range(nb)]
        out = []
        for b in range(nb):
            r, g = refs[b], geoms[b]
            # 9. divergence of the continuous transformed flux
            div = (_es("irv,ivan->ran", r.D_u, Ft[b])
                   + _es("rs,san->ran", r.divg, self._from_flat(DF, b) - fperp[b]))
            # 10. du/dt = -J^-1 div
            out.append(-div / g.detJ.T[:, None, :])
        return out

    # -- time stepping --------------------------------------------------------
    def rk4_step(self, state, dt):
        """Classical fourth-order Runge-Kutta step (dt scalar, or one value
        per element block given as a list of (ne,) arrays)."""
        def axpy(a, x, k):
            return [xb + _scale(a, b) * kb for b, (xb, kb) in enumerate(zip(x, k))]

        k1 = self.rhs(state)
        k2 = self.rhs(axpy(_half(dt), state, k1))
        k3 = self.rhs(axpy(_half(dt), state, k2))
        k4 = self.rhs(axpy(dt, state, k3))
        return [u + _scale(dt, b) / 6.0 * (a + 2.0 * b2 + 2.0 * c + d)
                for b, (u, a, b2, c, d) in enumerate(zip(state, k1, k2, k3, k4))]

    def rk4(self, state, dt, nsteps):
        for _ in range(nsteps):
            state = self.rk4_step(state, dt)
        return state


def _half(dt):
    return 0.5 * dt if np.isscalar(dt) else [0.5 * d for d in dt]


def _scale(dt, b):
    if np.isscalar(dt):
        return dt
    return dt[b][None, None, :]


def jvp(disc, state, direction, h=1e-30):
    """Directional derivative of the right-hand side, (dR/du)(u) v, by
    complex-step differentiation (Squire & Trapp): Im R(u + i h v) / h.  The
    right-hand side is real-analytic in u (|x| enters as x sign(Re x)), so
    the result is exact to rounding for any h far below the scale of u."""
    z = [u.astype(np.complex128) + 1j * h * v for u, v in zip(state, direction)]
    return [np.imag(r) / h for r in disc.rhs(z)]


def rk4_jvp(disc, state, direction, dt, h=1e-30):
    """Directional derivative of one classical RK4 step, by complex step."""
    z = [u.astype(np.complex128) + 1j * h * v for u, v in zip(state, direction)]
    return [np.imag(r) / h for r in disc.rk4_step(z, dt)]
