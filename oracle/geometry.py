"""Element mappings, metric terms and flux-point pairing (oracle side).

TEST INFRASTRUCTURE ONLY: see the package docstring.

Paper section 2: each element has a mapping x = M(xi) with Jacobian
J_ij = dx_i/dxi_j and J = det J.  The transformed flux is J J^-1 f, the
transformed gradient J^T q, and physical normals at flux points are
J^-T n~ = n^(f) n^.  Here the mapping is the Lagrange interpolant of the
element nodes (equispaced reference nodes of geometry order g), and the
scaled inverse S = adj J = J * J^-1 is formed from cross products of the
Jacobian's columns.
"""
from __future__ import annotations

import numpy as np

from .reference import lagrange_1d


def shape_functions(etype, g, xi, dtype=np.float64):
    """Values (m, nnodes) and reference gradients (m, nnodes, D) of the
    geometry shape functions at reference points xi (m, D)."""
    xi = np.asarray(xi, dtype=dtype)
    if etype in ("quad", "hex"):
        D = xi.shape[1]
        nodes = np.linspace(-1.0, 1.0, g + 1)
        vd = [lagrange_1d(nodes, xi[:, d]) for d in range(D)]
        vd = [(v.astype(dtype), dv.astype(dtype)) for v, dv in vd]
        n1 = g + 1

        def comb(parts):
            if D == 2:
                a, b = parts
                return (a[:, None, :] * b[:, :, None]).reshape(len(a), n1 ** 2)
            a, b, c = parts
            return (a[:, None, None, :] * b[:, None, :, None] *
                    c[:, :, None, None]).reshape(len(a), n1 ** 3)

        val = comb([v for v, _ in vd])
        grad = np.stack([comb([vd[d][1] if d == i else vd[d][0] for d in range(D)])
                         for i in range(D)], 2)
        return val, grad
    if etype == "tri":
        l0 = -(xi[:, 0] + xi[:, 1]) / 2
        l1 = (1 + xi[:, 0]) / 2
        l2 = (1 + xi[:, 1]) / 2
        dl = np.array([[-0.5, -0.5], [0.5, 0.0], [0.0, 0.5]], dtype=dtype)   # d lambda_k / d xi
        lam = [l0, l1, l2]
        if g == 1:
            val = np.stack(lam, 1)
            grad = np.broadcast_to(dl, (len(xi), 3, 2)).copy()
            return val, grad
        if g == 2:
            vals, grads = [], []
            for k in range(3):                                   # vertices
                vals.append(lam[k] * (2 * lam[k] - 1))
                grads.append((4 * lam[k] - 1)[:, None] * dl[k])
            for a, b in ((0, 1), (1, 2), (2, 0)):                # edge midpoints
                vals.append(4 * lam[a] * lam[b])
                grads.append(4 * (lam[b][:, None] * dl[a] + lam[a][:, None] * dl[b]))
            return np.stack(vals, 1), np.stack(grads, 1)
    raise ValueError((etype, g))


def adjugate(J):
    """S = adj J for J of shape (..., D, D) with J[..., i, j] = dx_i/dxi_j.
    Row i of S is the scaled contravariant vector det(J) * grad(xi_i)."""
    D = J.shape[-1]
    S = np.empty_like(J)
    if D == 2:
        S[..., 0, 0] = J[..., 1, 1]
        S[..., 0, 1] = -J[..., 0, 1]
        S[..., 1, 0] = -J[..., 1, 0]
        S[..., 1, 1] = J[..., 0, 0]
        return S
    a = [J[..., :, j] for j in range(3)]                       # columns dx/dxi_j
    S[..., 0, :] = np.cross(a[1], a[2])
    S[..., 1, :] = np.cross(a[2], a[0])
    S[..., 2, :] = np.cross(a[0], a[1])
    return S


def _det(J, S):
    """det J from the adjugate (J S = det(J) I): sum_j J[0, j] S[j, 0]."""
    return np.einsum("...j,...j->...", J[..., 0, :], S[..., :, 0])


class BlockGeometry:
    """Physical coordinates and metric terms of one element block (dtype
    long double: the same formulas with 64-bit significands, used only to
    measure rounding floors)."""

    def __init__(self, ref, block, dtype=np.float64):
        nodes = np.asarray(block.nodes).astype(dtype)           # (ne, nn, D)
        etype, g = block.etype, block.geom_order
        self.nelem = nodes.shape[0]
        # solution points
        N, dN = shape_functions(etype, g, ref.upts, dtype)
        self.xu = np.einsum("pk,ekd->epd", N, nodes)             # (ne, Nu, D)
        J = np.einsum("ekd,pkj->epdj", nodes, dN)               # (ne, Nu, D, D)
        self.S = adjugate(J)                                     # (ne, Nu, D, D)
        self.detJ = _det(J, self.S)                              # (ne, Nu)
        # flux points
        Nf, dNf = shape_functions(etype, g, ref.fpts, dtype)
        self.xf = np.einsum("pk,ekd->epd", Nf, nodes)            # (ne, Nf, D)
        Jf = np.einsum("ekd,pkj->epdj", nodes, dNf)
        Sf = adjugate(Jf)
        nu = np.einsum("epij,pi->epj", Sf, np.asarray(ref.fnorm).astype(dtype))   # S^T n~
        self.fmag = np.sqrt(np.sum(nu * nu, axis=-1))            # J^(f) n^(f)
        self.fnhat = nu / self.fmag[..., None]                   # unit physical normal
        self.detJf = _det(Jf, Sf)


def pair_flux_points(mesh, refs, geoms, tol_rel=1e-9, allow_unpaired=False, boundary=None):
    """Match the flux points of every face pair by physical coordinate.

    Returns a dict of int arrays (lb, le, ls, rb, re, rs), one entry per flux
    point pair, in face-pair order.  Raises ValueError if a pair does not
    match point for point, or if a flux point is paired more than once or
    (unless allow_unpaired: a patch cut out of a larger mesh) not at all.
    ``boundary`` (b, e, s) arrays: flux points of boundary faces, which count
    as their own interface.
    """
    pairs = mesh.pairs
    h = mesh.info.get("h", 1.0)
    tol = tol_rel * max(h, 1e-300) * 10.0
    out = {k: [] for k in ("lb", "le", "ls", "rb", "re", "rs")}
    keys = np.stack([pairs["lblock"], pairs["lface"], pairs["rblock"], pairs["rface"]], 1)
    ukeys = np.unique(keys, axis=0)
    order_chunks = []
    for lb, lf, rb, rf in ukeys:
        sel = np.nonzero((keys == (lb, lf, rb, rf)).all(1))[0]
        refL, refR = refs[lb], refs[rb]
        sigL = np.nonzero(refL.fface == lf)[0]
        sigR = np.nonzero(refR.fface == rf)[0]
        le = pairs["lelem"][sel]
        re = pairs["relem"][sel]
        D = mesh.ndims
        js = []
        for c0 in range(0, len(sel), 8192):
            c = slice(c0, c0 + 8192)
            xL = geoms[lb].xf[le[c]][:, sigL]                    # (m, nf, D)
            xR = geoms[rb].xf[re[c]][:, sigR] + pairs["shift"][sel[c], None, :D]
            d = np.linalg.norm(xL[:, :, None, :] - xR[:, None, :, :], axis=-1)
            jc = np.argmin(d, axis=2)                            # (m, nf)
            dmin = np.take_along_axis(d, jc[..., None], 2)[..., 0]
            if np.max(dmin) > tol:
                raise ValueError("flux points of a face pair do not coincide")
            js.append(jc)
        j = np.concatenate(js)
        if np.any(np.sort(j, axis=1) != np.arange(len(sigR))[None, :]):
            raise ValueError("flux point matching is not a bijection")
        m, nf = j.shape
        out["lb"].append(np.full(m * nf, lb))
        out["le"].append(np.repeat(le, nf))
        out["ls"].append(np.tile(sigL, m))
        out["rb"].append(np.full(m * nf, rb))
        out["re"].append(np.repeat(re, nf))
        out["rs"].append(sigR[j].ravel())
        order_chunks.append(np.repeat(sel, nf))
    res = {k: np.concatenate(v).astype(np.int64) for k, v in out.items()}
    # check every flux point of every block is used exactly once
    counts = [np.zeros((g.nelem, r.nfpts), np.int64) for g, r in zip(geoms, refs)]
    if boundary is not None:
        bb, be, bs = boundary
        for b in range(len(refs)):
            s = bb == b
            np.add.at(counts[b], (be[s], bs[s]), 1)
    for side in ("l", "r"):
        for b in range(len(refs)):
            s = res[side + "b"] == b
            np.add.at(counts[b], (res[side + "e"][s], res[side + "s"][s]), 1)
    if any(np.any(c > 1) or (not allow_unpaired and np.any(c != 1)) for c in counts):
        raise ValueError("flux points not paired exactly once")
    return res
