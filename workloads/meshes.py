"""Seeded synthetic meshes: element nodes and conforming face pairs.

This module produces *data only* (node coordinates, face-pair records and
per-element problem ids).  It contains none of the flux reconstruction
arithmetic: no solution or flux points, no basis functions, no metrics.  Both
the HIP library and the CPU oracle consume the arrays it returns.

Conventions (the paper leaves them open, so they are fixed here once):

* Reference quad [-1,1]^2 and hex [-1,1]^3; reference triangle with vertices
  v0=(-1,-1), v1=(1,-1), v2=(-1,1).
* Element nodes: Q1/Q2 quads and hexes are tensor-lexicographic on {-1,1} or
  {-1,0,1} with xi fastest.  P1 triangles list (v0, v1, v2); P2 triangles add
  the midpoints of v0v1, v1v2, v2v0.
* Faces: quad 0: eta=-1, 1: xi=+1, 2: eta=+1, 3: xi=-1.  Triangle 0: v0->v1,
  1: v1->v2, 2: v2->v0.  Hex 0: zeta=-1, 1: eta=-1, 2: xi=+1, 3: eta=+1,
  4: xi=-1, 5: zeta=+1.
* A face pair (L, R, shift) satisfies x_R + shift == x_L on the shared face.
  L is the element on the lower-coordinate side of the shared face, so the
  left/right roles are consistent across the whole (periodic) mesh.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

FACEPAIR_DTYPE = np.dtype([
    ("lblock", np.int32), ("lelem", np.int64), ("lface", np.int32),
    ("rblock", np.int32), ("relem", np.int64), ("rface", np.int32),
    ("shift", np.float64, (3,)),
])

# a face on the domain boundary and the boundary condition it carries
# (index into Mesh.bcs)
BCFACE_DTYPE = np.dtype([("block", np.int32), ("elem", np.int64), ("face", np.int32),
                         ("bc", np.int32)])

ETYPES = ("quad", "tri", "hex")
ETYPE_CODE = {"quad": 0, "tri": 1, "hex": 2}
ETYPE_NDIMS = {"quad": 2, "tri": 2, "hex": 3}


def nnodes(etype: str, geom_order: int) -> int:
    g = geom_order
    if etype == "quad":
        return (g + 1) ** 2
    if etype == "hex":
        return (g + 1) ** 3
    if etype == "tri":
        return (g + 1) * (g + 2) // 2
    raise ValueError(etype)


@dataclass
class Block:
    etype: str
    order: int
    geom_order: int
    nodes: np.ndarray                  # (nelem, nnodes, ndims) float64
    problem: np.ndarray | None = None  # (nelem,) int32 problem id, or None
    correction: str = "dg"             # correction-function scheme: "dg", "sd" or "hu"

    @property
    def nelem(self) -> int:
        return int(self.nodes.shape[0])


@dataclass
class Mesh:
    ndims: int
    blocks: list
    pairs: np.ndarray                  # FACEPAIR_DTYPE records
    nproblems: int = 1
    info: dict = field(default_factory=dict)
    bcfaces: np.ndarray | None = None  # BCFACE_DTYPE records (boundary faces)
    bcs: tuple = ()                    # boundary conditions: dicts with "type" and parameters


def _pairs(records):
    arr = np.zeros(len(records), dtype=FACEPAIR_DTYPE)
    for k, (lb, le, lf, rb, re, rf, sh) in enumerate(records):
        arr[k] = (lb, le, lf, rb, re, rf, tuple(list(sh) + [0.0] * (3 - len(sh))))
    return arr


def _pairs_vec(lb, le, lf, rb, re, rf, shift):
    n = len(le)
    arr = np.zeros(n, dtype=FACEPAIR_DTYPE)
    arr["lblock"], arr["lelem"], arr["lface"] = lb, le, lf
    arr["rblock"], arr["relem"], arr["rface"] = rb, re, rf
    sh = np.zeros((n, 3))
    sh[:, :shift.shape[1]] = shift
    arr["shift"] = sh
    return arr


def _lattice(ng):
    """Equispaced reference coordinates of a geometry order with ng=g+1 nodes."""
    return np.linspace(-1.0, 1.0, ng)


# ---------------------------------------------------------------------------
# Structured periodic quadrilateral meshes
# ---------------------------------------------------------------------------
def quad_mesh(nx, ny, lo=(-5.0, -5.0), hi=(5.0, 5.0), order=3, geom_order=1,
              mapping=None, walls_y=False, open_x=None):
    """nx*ny periodic quads; element n = i + nx*j.

    ``mapping`` (optional) maps lattice points (..., 2) to physical points; it
    must leave the domain boundary fixed so periodic faces still match.
    ``walls_y``: not periodic in y; the faces at y = lo carry boundary 0 and
    those at y = hi boundary 1 (Mesh.bcfaces; the caller sets Mesh.bcs).
    ``open_x`` = (left, right): not periodic in x; the faces at x = lo and
    x = hi carry those boundary indices.
    """
    g = geom_order
    xs = np.linspace(lo[0], hi[0], nx + 1)
    ys = np.linspace(lo[1], hi[1], ny + 1)
    hx, hy = xs[1] - xs[0], ys[1] - ys[0]
    t = (_lattice(g + 1) + 1.0) / 2.0
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    i, j = i.ravel(), j.ravel()          # element n = i + nx*j
    nodes = np.zeros((nx * ny, (g + 1) ** 2, 2))
    for b in range(g + 1):
        for a in range(g + 1):
            k = a + (g + 1) * b
            nodes[:, k, 0] = xs[i] + t[a] * hx
            nodes[:, k, 1] = ys[j] + t[b] * hy
    if mapping is not None:
        nodes = mapping(nodes)
    Lx, Ly = hi[0] - lo[0], hi[1] - lo[1]
    n = i + nx * j
    # xi=+1 face (1) of (i,j) <-> xi=-1 face (3) of (i+1,j)
    rx = (i + 1) % nx + nx * j
    shx = np.where(i == nx - 1, Lx, 0.0)
    px = _pairs_vec(0, n, 1, 0, rx, 3, np.stack([shx, 0 * shx], 1))
    if open_x is not None:
        px = px[i != nx - 1]
    ry = i + nx * ((j + 1) % ny)
    shy = np.where(j == ny - 1, Ly, 0.0)
    py = _pairs_vec(0, n, 2, 0, ry, 0, np.stack([0 * shy, shy], 1))
    bcf = None
    if walls_y:
        py = py[j != ny - 1]
        bot, top = n[j == 0], n[j == ny - 1]
        bcf = np.zeros(len(bot) + len(top), dtype=BCFACE_DTYPE)
        bcf["elem"] = np.concatenate([bot, top])
        bcf["face"] = np.concatenate([np.zeros(len(bot)), np.full(len(top), 2)])
        bcf["bc"] = np.concatenate([np.zeros(len(bot)), np.ones(len(top))])
    if open_x is not None:
        lft, rgt = n[i == 0], n[i == nx - 1]
        bx = np.zeros(len(lft) + len(rgt), dtype=BCFACE_DTYPE)
        bx["elem"] = np.concatenate([lft, rgt])
        bx["face"] = np.concatenate([np.full(len(lft), 3), np.ones(len(rgt))])
        bx["bc"] = np.concatenate([np.full(len(lft), open_x[0]), np.full(len(rgt), open_x[1])])
        bcf = bx if bcf is None else np.concatenate([bcf, bx])
    blk = Block("quad", order, g, nodes)
    return Mesh(2, [blk], np.concatenate([px, py]),
                info=dict(nx=nx, ny=ny, lo=lo, hi=hi, h=min(hx, hy)), bcfaces=bcf)


# ---------------------------------------------------------------------------
# Structured periodic hexahedral meshes
# ---------------------------------------------------------------------------
def hex_mesh(nx, ny, nz, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), order=3,
             geom_order=1, mapping=None, walls_y=False):
    """nx*ny*nz periodic hexes; element n = i + nx*(j + ny*k).  ``walls_y``:
    not periodic in y, faces at y = lo carry boundary 0 and at y = hi
    boundary 1."""
    g = geom_order
    xs = [np.linspace(lo[d], hi[d], m + 1) for d, m in enumerate((nx, ny, nz))]
    hs = [x[1] - x[0] for x in xs]
    t = (_lattice(g + 1) + 1.0) / 2.0
    k3, j3, i3 = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    i3, j3, k3 = i3.ravel(), j3.ravel(), k3.ravel()
    ne = nx * ny * nz
    nodes = np.zeros((ne, (g + 1) ** 3, 3))
    for c in range(g + 1):
        for b in range(g + 1):
            for a in range(g + 1):
                kk = a + (g + 1) * (b + (g + 1) * c)
                nodes[:, kk, 0] = xs[0][i3] + t[a] * hs[0]
                nodes[:, kk, 1] = xs[1][j3] + t[b] * hs[1]
                nodes[:, kk, 2] = xs[2][k3] + t[c] * hs[2]
    if mapping is not None:
        nodes = mapping(nodes)
    L = [hi[d] - lo[d] for d in range(3)]
    idx = lambda a, b, c: a + nx * (b + ny * c)
    n = idx(i3, j3, k3)
    z = np.zeros(ne)
    pieces = []
    # xi faces: 2 (xi=+1) <-> 4 (xi=-1)
    sh = np.stack([np.where(i3 == nx - 1, L[0], 0.0), z, z], 1)
    pieces.append(_pairs_vec(0, n, 2, 0, idx((i3 + 1) % nx, j3, k3), 4, sh))
    # eta faces: 3 (eta=+1) <-> 1 (eta=-1)
    sh = np.stack([z, np.where(j3 == ny - 1, L[1], 0.0), z], 1)
    py = _pairs_vec(0, n, 3, 0, idx(i3, (j3 + 1) % ny, k3), 1, sh)
    bcf = None
    if walls_y:
        py = py[j3 != ny - 1]
        bot, top = n[j3 == 0], n[j3 == ny - 1]
        bcf = np.zeros(len(bot) + len(top), dtype=BCFACE_DTYPE)
        bcf["elem"] = np.concatenate([bot, top])
        bcf["face"] = np.concatenate([np.ones(len(bot)), np.full(len(top), 3)])
        bcf["bc"] = np.concatenate([np.zeros(len(bot)), np.ones(len(top))])
    pieces.append(py)
    # zeta faces: 5 (zeta=+1) <-> 0 (zeta=-1)
    sh = np.stack([z, z, np.where(k3 == nz - 1, L[2], 0.0)], 1)
    pieces.append(_pairs_vec(0, n, 5, 0, idx(i3, j3, (k3 + 1) % nz), 0, sh))
    blk = Block("hex", order, g, nodes)
    return Mesh(3, [blk], np.concatenate(pieces),
                info=dict(n=(nx, ny, nz), lo=lo, hi=hi, h=min(hs)), bcfaces=bcf)


def sine_perturbation(amp=0.1, period=1.0):
    """x = X + amp * prod_d sin(2 pi X_d / period) * (1,...,1).

    Vanishes on every plane X_d = m*period, so a periodic box whose sides are
    multiples of the period keeps flat, matching boundary faces.
    """
    def f(X):
        s = np.ones(X.shape[:-1])
        for d in range(X.shape[-1]):
            s = s * np.sin(2.0 * np.pi * X[..., d] / period)
        return X + amp * s[..., None]
    return f


# ---------------------------------------------------------------------------
# Mixed quad/triangle meshes (quads split along a diagonal)
# ---------------------------------------------------------------------------
def mixed_quad_tri_mesh(nx, ny, lo=(-5.0, -5.0), hi=(5.0, 5.0), split=None,
                        diag=None, qblock=0, tblock=1, walls_y=False):
    """Periodic nx*ny grid; the cells flagged in ``split`` become two triangles.

    ``diag[c]`` = 0 splits cell c along B-C (from (x1,y0) to (x0,y1)), 1 along
    A-D.  Returns (quad_nodes, tri_nodes, pairs) as raw arrays so callers can
    assemble several problems into shared blocks; use :func:`mixed_mesh` for a
    ready Mesh.  ``walls_y``: not periodic in y; a fourth value, the boundary
    faces (bottom boundary 0, top boundary 1), is returned.
    """
    ncell = nx * ny
    if split is None:
        split = np.zeros(ncell, bool)
    if diag is None:
        diag = np.zeros(ncell, np.int32)
    xs = np.linspace(lo[0], hi[0], nx + 1)
    ys = np.linspace(lo[1], hi[1], ny + 1)
    Lx, Ly = hi[0] - lo[0], hi[1] - lo[1]
    quad_nodes, tri_nodes = [], []
    # side owner[c][s] = (block, elem, face), s: 0 bottom, 1 right, 2 top, 3 left
    owner = [[None] * 4 for _ in range(ncell)]
    internal = []
    for c in range(ncell):
        i, j = c % nx, c // nx
        A = (xs[i], ys[j]); B = (xs[i + 1], ys[j])
        C = (xs[i], ys[j + 1]); D = (xs[i + 1], ys[j + 1])
        if not split[c]:
            e = len(quad_nodes)
            quad_nodes.append([A, B, C, D])
            owner[c] = [(qblock, e, 0), (qblock, e, 1), (qblock, e, 2), (qblock, e, 3)]
        elif diag[c] == 0:
            e1 = len(tri_nodes); tri_nodes.append([A, B, C])   # faces: AB, BC, CA
            e2 = len(tri_nodes); tri_nodes.append([D, C, B])   # faces: DC, CB, BD
            owner[c] = [(tblock, e1, 0), (tblock, e2, 2), (tblock, e2, 0), (tblock, e1, 2)]
            internal.append((tblock, e1, 1, tblock, e2, 1, (0.0, 0.0)))
        else:
            e1 = len(tri_nodes); tri_nodes.append([B, D, A])   # faces: BD, DA, AB
            e2 = len(tri_nodes); tri_nodes.append([C, A, D])   # faces: CA, AD, DC
            owner[c] = [(tblock, e1, 2), (tblock, e1, 0), (tblock, e2, 2), (tblock, e2, 0)]
            internal.append((tblock, e1, 1, tblock, e2, 1, (0.0, 0.0)))
    recs = list(internal)
    for c in range(ncell):
        i, j = c % nx, c // nx
        cr = (i + 1) % nx + nx * j
        recs.append(owner[c][1] + owner[cr][3] + ((Lx if i == nx - 1 else 0.0, 0.0),))
        ct = i + nx * ((j + 1) % ny)
        if not (walls_y and j == ny - 1):
            recs.append(owner[c][2] + owner[ct][0] + ((0.0, Ly if j == ny - 1 else 0.0),))
    qn = np.array(quad_nodes, dtype=np.float64).reshape(-1, 4, 2)
    tn = np.array(tri_nodes, dtype=np.float64).reshape(-1, 3, 2)
    if not walls_y:
        return qn, tn, _pairs(recs)
    faces = [owner[c][0] + (0,) for c in range(nx)] + \
            [owner[c][2] + (1,) for c in range(nx * (ny - 1), nx * ny)]
    bcf = np.zeros(len(faces), dtype=BCFACE_DTYPE)
    for k, (b, e, f, bc) in enumerate(faces):
        bcf[k] = (b, e, f, bc)
    return qn, tn, _pairs(recs), bcf


def mixed_mesh(nx, ny, lo=(-5.0, -5.0), hi=(5.0, 5.0), order=3, split=None,
               diag=None, walls_y=False):
    out = mixed_quad_tri_mesh(nx, ny, lo, hi, split, diag, walls_y=walls_y)
    qn, tn, pairs = out[:3]
    bcf = out[3] if walls_y else None
    blocks = [Block("quad", order, 1, qn), Block("tri", order, 1, tn)]
    if len(tn) == 0:
        blocks = blocks[:1]
    if len(qn) == 0:
        # renumber tri block to 0
        pairs = pairs.copy()
        pairs["lblock"] = 0
        pairs["rblock"] = 0
        if bcf is not None:
            bcf["block"] = 0
        blocks = blocks[1:]
    return Mesh(2, blocks, pairs, bcfaces=bcf,
                info=dict(nx=nx, ny=ny, lo=lo, hi=hi,
                          h=min((hi[0] - lo[0]) / nx, (hi[1] - lo[1]) / ny)))
