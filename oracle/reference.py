"""Reference elements, nodal bases and the FR operator values (oracle side).

TEST INFRASTRUCTURE ONLY: see the package docstring.

Everything is built in the most direct form the paper allows:
* solution points and the nodal basis (paper section 2, the generalised
  Vandermonde construction): tensor elements use products of 1-D Lagrange
  polynomials through Gauss-Legendre (GL) nodes, which is that construction
  evaluated in closed form; triangles use a monomial Vandermonde solved in
  extended precision;
* flux points with unit outward reference normals on every face (section 2);
* the DG correction functions (section 2, eq. corfn) through their defining
  property: the divergence of the correction field lies in the solution space
  and reproduces the face integral of the jump, i.e. mass-matrix lifting,
  with every integral done by explicit quadrature;
* the SD and HU correction functions of the vortex super-accuracy test
  (validation section), which the paper takes from the one-parameter
  energy-stable family of Vincent, Castonguay and Jameson (VCJH): on tensor
  elements the correction field of a flux point is the 1-D VCJH polynomial
  along the face normal times the face Lagrange polynomial of that point.
"""
from __future__ import annotations

import math

import numpy as np

LD = np.longdouble


# ---------------------------------------------------------------------------
# 1-D Gauss-Legendre nodes and weights
# ---------------------------------------------------------------------------
def legendre(n, x):
    """P_n(x) and P_n'(x) by the three-term recurrence (x in long double)."""
    x = np.asarray(x, dtype=LD)
    p0, p1 = np.ones_like(x), x.copy()
    if n == 0:
        return p0, np.zeros_like(x)
    for k in range(1, n):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
    dp = n * (x * p1 - p0) / (x * x - 1)
    return p1, dp


def gauss_legendre(n):
    """n-point GL rule on [-1,1]: Newton on P_n from Chebyshev-like guesses.
    Returns float64 nodes (ascending) and weights 2/((1-x^2) P_n'(x)^2)."""
    i = np.arange(n, dtype=LD)
    x = np.cos(np.pi * (i + LD(0.75)) / (n + LD(0.5)))
    for _ in range(100):
        p, dp = legendre(n, x)
        dx = p / dp
        x = x - dx
        if np.max(np.abs(dx)) < LD(1e-30):
            break
    p, dp = legendre(n, x)
    w = 2 / ((1 - x * x) * dp * dp)
    order = np.argsort(x)
    return x[order].astype(np.float64), w[order].astype(np.float64)


def gauss_lobatto_nodes(n):
    """n+1 Gauss-Lobatto-Legendre nodes: -1, roots of P_n', +1."""
    if n == 1:
        return np.array([-1.0, 1.0])
    inner = np.polynomial.legendre.Legendre.basis(n).deriv().roots()
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


def lagrange_1d(nodes, x):
    """Values and derivatives of the 1-D Lagrange polynomials through
    ``nodes`` at points ``x``: arrays (len(x), len(nodes))."""
    nodes = np.asarray(nodes, dtype=LD)
    x = np.asarray(x, dtype=LD)
    n = len(nodes)
    val = np.ones((len(x), n), dtype=LD)
    der = np.zeros((len(x), n), dtype=LD)
    for k in range(n):
        for m in range(n):
            if m != k:
                val[:, k] *= (x - nodes[m]) / (nodes[k] - nodes[m])
        for j in range(n):
            if j == k:
                continue
            term = np.full(len(x), 1 / (nodes[k] - nodes[j]), dtype=LD)
            for m in range(n):
                if m != k and m != j:
                    term *= (x - nodes[m]) / (nodes[k] - nodes[m])
            der[:, k] += term
    return val, der


# ---------------------------------------------------------------------------
# Triangle solution points: Warburton's warp-and-blend construction (alpha=0),
# Warburton, J. Eng. Math. 56 (2006); the steps follow the Warpfactor and
# Nodes2D routines of Hesthaven & Warburton, "Nodal Discontinuous Galerkin
# Methods" (2008), including its treatment of the edge points (warp kept
# unscaled where |r| = 1).
# ---------------------------------------------------------------------------
def _warp_factor(n, r):
    gll = gauss_lobatto_nodes(n)
    req = np.linspace(-1.0, 1.0, n + 1)
    lv, _ = lagrange_1d(req, r)
    warp = (lv.astype(np.float64)) @ (gll - req)
    inside = np.abs(r) < 1.0 - 1e-10
    sf = 1.0 - (inside * r) ** 2
    return warp / sf + warp * (inside - 1.0)


def triangle_points(n):
    """(n+1)(n+2)/2 warp-and-blend nodes (blend exponent alpha = 0) on the
    reference triangle (-1,-1),(1,-1),(-1,1).  Order: rows of constant
    barycentric L1 from the v0-v1 edge upward, left to right within a row."""
    pts = []
    for a in range(n + 1):
        for b in range(n + 1 - a):
            L1 = a / n
            L3 = b / n
            L2 = 1.0 - L1 - L3
            pts.append((L1, L2, L3))
    L = np.array(pts)
    L1, L2, L3 = L[:, 0], L[:, 1], L[:, 2]
    x = -L2 + L3
    y = (-L2 - L3 + 2 * L1) / math.sqrt(3.0)
    w1 = 4 * L2 * L3 * _warp_factor(n, L3 - L2)
    w2 = 4 * L1 * L3 * _warp_factor(n, L1 - L3)
    w3 = 4 * L1 * L2 * _warp_factor(n, L2 - L1)
    x = x + w1 + math.cos(2 * math.pi / 3) * w2 + math.cos(4 * math.pi / 3) * w3
    y = y + math.sin(2 * math.pi / 3) * w2 + math.sin(4 * math.pi / 3) * w3
    # equilateral -> reference right triangle
    l1 = (math.sqrt(3.0) * y + 1) / 3
    l2 = (-3 * x - math.sqrt(3.0) * y + 2) / 6
    l3 = (3 * x - math.sqrt(3.0) * y + 2) / 6
    r = -l2 + l3 - l1
    s = -l2 - l3 + l1
    return np.stack([r, s], 1)


# ---------------------------------------------------------------------------
# Faces of the reference elements
# ---------------------------------------------------------------------------
SQ2 = math.sqrt(2.0)


def face_table(etype):
    """List of (map(t) -> reference coords, unit outward normal, ds/dt scale).
    t has shape (m, ndims-1)."""
    if etype == "quad":
        return [
            (lambda t: np.stack([t[:, 0], -np.ones(len(t))], 1), (0.0, -1.0), 1.0),
            (lambda t: np.stack([np.ones(len(t)), t[:, 0]], 1), (1.0, 0.0), 1.0),
            (lambda t: np.stack([-t[:, 0], np.ones(len(t))], 1), (0.0, 1.0), 1.0),
            (lambda t: np.stack([-np.ones(len(t)), -t[:, 0]], 1), (-1.0, 0.0), 1.0),
        ]
    if etype == "tri":
        return [
            (lambda t: np.stack([t[:, 0], -np.ones(len(t))], 1), (0.0, -1.0), 1.0),
            (lambda t: np.stack([-t[:, 0], t[:, 0]], 1), (1 / SQ2, 1 / SQ2), SQ2),
            (lambda t: np.stack([-np.ones(len(t)), -t[:, 0]], 1), (-1.0, 0.0), 1.0),
        ]
    if etype == "hex":
        o = lambda t: np.ones(len(t))
        return [
            (lambda t: np.stack([t[:, 0], t[:, 1], -o(t)], 1), (0.0, 0.0, -1.0), 1.0),
            (lambda t: np.stack([t[:, 0], -o(t), t[:, 1]], 1), (0.0, -1.0, 0.0), 1.0),
            (lambda t: np.stack([o(t), t[:, 0], t[:, 1]], 1), (1.0, 0.0, 0.0), 1.0),
            (lambda t: np.stack([t[:, 0], o(t), t[:, 1]], 1), (0.0, 1.0, 0.0), 1.0),
            (lambda t: np.stack([-o(t), t[:, 0], t[:, 1]], 1), (-1.0, 0.0, 0.0), 1.0),
            (lambda t: np.stack([t[:, 0], t[:, 1], o(t)], 1), (0.0, 0.0, 1.0), 1.0),
        ]
    raise ValueError(etype)


def _tensor_nodes(x1, dim):
    """Tensor grid of 1-D nodes with the first coordinate fastest."""
    grids = np.meshgrid(*([x1] * dim), indexing="ij")
    return np.stack([g.T.ravel() if dim == 2 else np.transpose(g, (2, 1, 0)).ravel()
                     for g in grids], 1)


def _tensor_weights(w1, dim):
    ws = _tensor_nodes(w1, dim)
    return np.prod(ws, axis=1)


# ---------------------------------------------------------------------------
# VCJH correction functions in one dimension
# ---------------------------------------------------------------------------
CORRECTIONS = ("dg", "sd", "hu")


def legendre_leading(p):
    """Leading coefficient a_p = (2p)! / (2^p (p!)^2) of P_p."""
    return math.factorial(2 * p) / (2 ** p * math.factorial(p) ** 2)


def vcjh_c(scheme, p):
    """The family parameter c of the named scheme: 0 for DG; the SD and HU
    values of the VCJH family, with (a_p p!)^2 as their common scale."""
    k = (legendre_leading(p) * math.factorial(p)) ** 2
    if scheme == "dg":
        return 0.0
    if scheme == "sd":
        return 2.0 * p / ((2 * p + 1) * (p + 1) * k)
    if scheme == "hu":
        return 2.0 * (p + 1) / ((2 * p + 1) * p * k)
    raise ValueError(scheme)


def vcjh_left(p, c):
    """g_L of the VCJH family as a Legendre series: degree p + 1, g_L(-1) = 1,
    g_L(1) = 0, (-1)^p/2 [P_p - (eta P_{p-1} + P_{p+1}) / (1 + eta)] with
    eta = c (2p + 1) (a_p p!)^2 / 2.  The right function is g_L(-xi)."""
    eta = c * (2 * p + 1) * (legendre_leading(p) * math.factorial(p)) ** 2 / 2
    coef = np.zeros(p + 2)
    coef[p] = 1.0
    coef[p - 1] -= eta / (1 + eta)
    coef[p + 1] -= 1.0 / (1 + eta)
    return np.polynomial.legendre.Legendre(0.5 * (-1) ** p * coef)


class RefElement:
    """Points, basis and operator values of one (element type, order p,
    correction scheme)."""

    def __init__(self, etype: str, p: int, correction: str = "dg"):
        if correction not in CORRECTIONS:
            raise ValueError(correction)
        if correction != "dg" and etype == "tri":
            raise ValueError("SD and HU corrections are defined for tensor elements only")
        self.etype, self.p, self.correction = etype, p, correction
        self.ndims = 3 if etype == "hex" else 2
        D = self.ndims
        xg, wg = gauss_legendre(p + 1)
        self.gl_nodes, self.gl_weights = xg, wg
        # --- solution points -------------------------------------------------
        if etype == "tri":
            self.upts = triangle_points(p)
            self._init_tri_basis()
        else:
            self.upts = _tensor_nodes(xg, D)
        self.nupts = len(self.upts)
        # --- flux points: GL on every face ------------------------------------
        faces = face_table(etype)
        self.nfaces = len(faces)
        tf = xg[:, None] if D == 2 else _tensor_nodes(xg, 2)
        wf = wg if D == 2 else _tensor_weights(wg, 2)
        fp, fn, ff, fw = [], [], [], []
        for f, (fmap, nrm, scale) in enumerate(faces):
            fp.append(fmap(tf))
            fn.append(np.tile(nrm, (len(tf), 1)))
            ff.append(np.full(len(tf), f))
            fw.append(wf * scale)
        self.fpts = np.concatenate(fp)
        self.fnorm = np.concatenate(fn)
        self.fface = np.concatenate(ff)
        self.fweight = np.concatenate(fw)           # omega_sigma (reference)
        self.nfpts = len(self.fpts)
        self.nfpts_face = len(tf)
        self._face_param = tf
        self._faces = faces
        # --- operator values --------------------------------------------------
        self.L_f = self.basis(self.fpts)              # (Nf, Nu): l_rho(x^f_sigma)
        g = self.basis_grad(self.upts)               # (Nu, Nu, D): d_i l_nu(x_rho)
        self.D_u = np.transpose(g, (2, 0, 1))         # (D, Nu, Nu) [i, rho, nu]
        self._build_quadrature()
        self._build_lifting()
        if correction != "dg":
            self.divg = self.vcjh_divg(vcjh_c(correction, p))

    # -- basis -----------------------------------------------------------------
    def _init_tri_basis(self):
        p = self.p
        self._mono = [(a, b) for b in range(p + 1) for a in range(p + 1 - b)]
        V = self._mono_eval(self.upts)                # (Nu, Nmono)
        self._coef = _solve_ld(V, np.eye(len(V)))     # V c = I

    def _mono_eval(self, x, deriv=None):
        x = np.asarray(x, dtype=LD)
        cols = []
        for a, b in self._mono:
            if deriv is None:
                cols.append(x[:, 0] ** a * x[:, 1] ** b)
            elif deriv == 0:
                cols.append(a * x[:, 0] ** max(a - 1, 0) * x[:, 1] ** b if a else 0 * x[:, 0])
            else:
                cols.append(b * x[:, 0] ** a * x[:, 1] ** max(b - 1, 0) if b else 0 * x[:, 0])
        return np.stack(cols, 1)

    def basis(self, x):
        """l_rho(x) for every solution point rho: (len(x), Nu)."""
        if self.etype == "tri":
            return (self._mono_eval(x) @ self._coef).astype(np.float64)
        vals = [lagrange_1d(self.gl_nodes, x[:, d])[0] for d in range(self.ndims)]
        return self._tensor_combine(vals).astype(np.float64)

    def basis_grad(self, x):
        """d l_rho / d xi_i at x: (len(x), Nu, D)."""
        if self.etype == "tri":
            return np.stack([(self._mono_eval(x, d) @ self._coef).astype(np.float64)
                             for d in range(2)], 2)
        vd = [lagrange_1d(self.gl_nodes, x[:, d]) for d in range(self.ndims)]
        out = []
        for i in range(self.ndims):
            parts = [vd[d][1] if d == i else vd[d][0] for d in range(self.ndims)]
            out.append(self._tensor_combine(parts).astype(np.float64))
        return np.stack(out, 2)

    def _tensor_combine(self, parts):
        n1 = self.p + 1
        if self.ndims == 2:
            a, b = parts
            # rho = i + n1*j
            return (a[:, None, :] * b[:, :, None]).reshape(len(a), n1 * n1)
        a, b, c = parts
        return (a[:, None, None, :] * b[:, None, :, None] * c[:, :, None, None]
                ).reshape(len(a), n1 ** 3)

    # -- quadrature and DG lifting ----------------------------------------------
    def _build_quadrature(self):
        nq = self.p + 2
        xq, wq = gauss_legendre(nq)
        if self.etype == "tri":
            a = np.repeat(xq, nq)
            b = np.tile(xq, nq)
            wa = np.repeat(wq, nq)
            wb = np.tile(wq, nq)
            x = (1 + a) * (1 - b) / 2 - 1
            self.qpts = np.stack([x, b], 1)
            self.qwts = wa * wb * (1 - b) / 2
        else:
            self.qpts = _tensor_nodes(xq, self.ndims)
            self.qwts = _tensor_weights(wq, self.ndims)
        self._fq_t = xq[:, None] if self.ndims == 2 else _tensor_nodes(xq, 2)
        self._fq_w = wq if self.ndims == 2 else _tensor_weights(wq, 2)

    def _face_lagrange(self, t):
        """Face Lagrange polynomials through the face's flux points."""
        if self.ndims == 2:
            return lagrange_1d(self.gl_nodes, t[:, 0])[0].astype(np.float64)
        la = lagrange_1d(self.gl_nodes, t[:, 0])[0]
        lb = lagrange_1d(self.gl_nodes, t[:, 1])[0]
        n1 = self.p + 1
        return (la[:, None, :] * lb[:, :, None]).reshape(len(t), n1 * n1).astype(np.float64)

    def _build_lifting(self):
        Lq = self.basis(self.qpts)                               # (Nq, Nu)
        self.W = self.qwts @ Lq                                  # int l_rho
        self.mass = (Lq * self.qwts[:, None]).T @ Lq             # int l_rho l_nu
        lift = np.zeros((self.nupts, self.nfpts))
        omega = np.zeros(self.nfpts)
        nf = self.nfpts_face
        for f, (fmap, _nrm, scale) in enumerate(self._faces):
            xf = fmap(self._fq_t)
            lam = self._face_lagrange(self._fq_t)                # (Nq_f, nf)
            lr = self.basis(xf)                                  # (Nq_f, Nu)
            w = self._fq_w * scale
            lift[:, f * nf:(f + 1) * nf] = (lr * w[:, None]).T @ lam
            omega[f * nf:(f + 1) * nf] = w @ lam
        self.lift = lift
        self.omega_q = omega
        # (div g_sigma)(x_rho): solution-space field whose moments equal the
        # face moments of a unit jump at sigma
        self.divg = np.linalg.solve(self.mass, lift)             # (Nu, Nf)

    def vcjh_divg(self, c):
        """(div g_sigma)(x_rho) for the VCJH member c on a tensor element.

        A flux point sigma on the face with outward normal s e_i carries the
        field g_sigma = s e_i h(xi_i) prod_{j != i} ell_j(xi_j), h = g_L for
        s = -1 and g_L(-xi) for s = +1, ell_j the 1-D Lagrange polynomial
        through the GL nodes that is one at sigma's j-th coordinate; so
        n.g_sigma is one at sigma and zero at every other flux point, and
        div g_sigma = s h'(xi_i) prod ell_j."""
        gl = vcjh_left(self.p, c)
        dgl = gl.deriv()
        D = self.ndims
        out = np.zeros((self.nupts, self.nfpts))
        for sg in range(self.nfpts):
            n = self.fnorm[sg]
            i = int(np.argmax(np.abs(n)))
            s = float(np.sign(n[i]))
            xi = self.upts[:, i]
            dh = dgl(xi) if s < 0 else -dgl(-xi)        # h'(xi_i)
            val = s * dh
            tang = np.ones(self.nupts)
            for j in range(D):
                if j == i:
                    continue
                lj = lagrange_1d(self.gl_nodes, self.upts[:, j])[0].astype(np.float64)
                k = int(np.argmin(np.abs(self.gl_nodes - self.fpts[sg, j])))
                tang = tang * lj[:, k]
            out[:, sg] = val * tang
        return out


def _solve_ld(A, B):
    """Gaussian elimination with partial pivoting in long double."""
    A = np.array(A, dtype=LD)
    B = np.array(B, dtype=LD)
    n = len(A)
    for k in range(n):
        piv = k + int(np.argmax(np.abs(A[k:, k])))
        if piv != k:
            A[[k, piv]] = A[[piv, k]]
            B[[k, piv]] = B[[piv, k]]
        for i in range(k + 1, n):
            f = A[i, k] / A[k, k]
            A[i, k:] -= f * A[k, k:]
            B[i] -= f * B[k]
    X = np.zeros_like(B)
    for k in range(n - 1, -1, -1):
        X[k] = (B[k] - A[k, k + 1:] @ X[k + 1:]) / A[k, k]
    return X


_CACHE = {}


def ref_element(etype, p, correction="dg"):
    key = (etype, p, correction)
    if key not in _CACHE:
        _CACHE[key] = RefElement(etype, p, correction)
    return _CACHE[key]
