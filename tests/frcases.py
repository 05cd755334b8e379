"""Shared helpers of the GPU parity tests: build the oracle and the library
on the same seeded workload, evaluate both, compare."""
import numpy as np

from oracle import Discretisation
from workloads import configs, fields, meshes
from workloads.configs import Workload


def solver_for(w, prec="fp64", check_finite=False):
    import paper_1312_1638_amd as P
    return P.Solver(w.mesh, system=w.system, gamma=w.gamma, mu=w.mu, prandtl=w.prandtl,
                    ldg_beta=w.ldg_beta, ldg_tau=w.ldg_tau, prec=prec,
                    check_finite=check_finite, nproblems=w.mesh.nproblems)


def rel_l2(a, b):
    """||a - b|| / ||b|| over every block and field (whole SoA vector)."""
    num = sum(float(np.sum((x - y) ** 2)) for x, y in zip(a, b))
    den = sum(float(np.sum(y ** 2)) for y in b)
    return np.sqrt(num / den)


def field_rel_l2(a, b):
    """Relative L2 error of each field alpha on its own, over every block:
    ||a_alpha - b_alpha|| / ||b_alpha|| (arrays u[rho, alpha, n]).  A field
    much smaller than the others (momentum beside the energy of a low-Mach
    flow) is then held to the bar by itself rather than hidden in the
    whole-vector norm."""
    nv = b[0].shape[1]
    num, den = np.zeros(nv), np.zeros(nv)
    for x, y in zip(a, b):
        num += np.sum((np.asarray(x, np.float64) - y) ** 2, axis=(0, 2))
        den += np.sum(np.asarray(y, np.float64) ** 2, axis=(0, 2))
    return np.sqrt(num / den)


def field_tolerance(ref64, ext, stated, unit_ratio=1.0, factor=4.0):
    """Per-field bar of du/dt: the stated bar, or `factor` times that field's
    FP64 rounding floor (the oracle's per-field distance from the long-double
    evaluation) times the unit-roundoff ratio.  Returns (tolerances, floors)."""
    floor = field_rel_l2(ref64, ext)
    return np.maximum(stated, factor * floor * unit_ratio), floor


def check_fields(label, got, ref, tol):
    """Assert every field's relative L2 error below its bar (a scalar bar
    applies to every field); prints the errors.  Returns them."""
    err = field_rel_l2(got, ref)
    tol = np.broadcast_to(np.asarray(tol, np.float64), err.shape)
    print(f"{label}: per-field rel L2 " + " ".join(f"{e:.1e}/{t:.0e}" for e, t in zip(err, tol)))
    assert np.all(err < tol), (label, err, tol)
    return err


def state_bar(ref_u, u0, stated, du_bar):
    """Per-field bar of u after RK4 steps: the stated bar, or -- for a field
    whose change over the steps is comparable to its size, such as a
    momentum component that starts at zero -- the du/dt bar of that field
    applied to the change: u(k) - u(0) is a weighted sum of right-hand
    sides, so its relative error is bounded by theirs.  du_bar: per-field
    du/dt bars (array) or one bar for every field."""
    nv = ref_u[0].shape[1]
    inc = np.zeros(nv)
    size = np.zeros(nv)
    for r, u in zip(ref_u, u0):
        inc += np.sum((r - u) ** 2, axis=(0, 2))
        size += np.sum(r ** 2, axis=(0, 2))
    ratio = np.sqrt(inc / size)
    return np.maximum(stated, np.broadcast_to(du_bar, ratio.shape) * ratio)


def floor_tolerance(d, u, stated, unit_ratio=1.0, factor=4.0):
    """Tolerance for du/dt of one case: the stated bar, or `factor` times
    the FP64 rounding floor of the oracle (its relative L2 distance from a
    long-double evaluation of the same formula) scaled by the ratio of unit
    roundoffs of the precision under test.  Returns (tolerance, exact
    reference, floor)."""
    ref64 = d.rhs(u)
    ext = d.extended().rhs([x.astype(np.longdouble) for x in u])
    ext = Reference(x.astype(np.float64) for x in ext)
    floor = rel_l2(ref64, ext)
    ext.field_tol, ext.field_floor = field_tolerance(ref64, ext, stated, unit_ratio, factor)
    return max(stated, factor * floor * unit_ratio), ext, floor


class Reference(list):
    """Per-block long-double du/dt (rounded to FP64) with the per-field bars
    and floors that floor_tolerance derived beside the whole-vector one."""
    field_tol = None
    field_floor = None


def patch(w, sample, rings):
    """The sampled elements of a single-block workload plus `rings` layers of
    face neighbours, as a workload of its own whose pairs are every face pair
    between two patch elements (the oracle's allow_unpaired mode).  Returns
    (workload, index of each sampled element in the patch)."""
    import dataclasses
    pr = w.mesh.pairs
    le, re = pr["lelem"].astype(np.int64), pr["relem"].astype(np.int64)
    b = w.mesh.blocks[0]
    inside = np.zeros(b.nelem, bool)
    inside[np.asarray(sample)] = True
    for _ in range(rings):
        touch = inside[le] | inside[re]
        inside[le[touch]] = True
        inside[re[touch]] = True
    elems = np.nonzero(inside)[0]
    local = -np.ones(b.nelem, np.int64)
    local[elems] = np.arange(len(elems))
    sel = inside[le] & inside[re]
    sub = pr[sel].copy()
    sub["lelem"] = local[le[sel]]
    sub["relem"] = local[re[sel]]
    blk = meshes.Block(b.etype, b.order, b.geom_order, b.nodes[elems])
    mesh = meshes.Mesh(w.mesh.ndims, [blk], sub, info=dict(w.mesh.info))
    return dataclasses.replace(w, mesh=mesh), local[np.asarray(sample)]


def sampled_floor_tolerance(d, u, loc, stated, unit_ratio=1.0, factor=4.0):
    """floor_tolerance restricted to the elements `loc` of a patch (the only
    ones whose du/dt is complete).  Returns (tolerance, exact reference on
    loc, floor); the reference is a Reference of one block."""
    ref64 = d.rhs(u)[0][:, :, loc]
    ext = d.extended().rhs([x.astype(np.longdouble) for x in u])[0][:, :, loc].astype(np.float64)
    floor = rel_l2([ref64], [ext])
    ext = Reference([ext])
    ext.field_tol, ext.field_floor = field_tolerance([ref64], ext, stated, unit_ratio, factor)
    return max(stated, factor * floor * unit_ratio), ext, floor


FP32_OVER_FP64 = 2.0 ** 29   # unit roundoff ratio 2^-24 / 2^-53
# BF16x3 products keep ~16 significant bits (hi + lo parts of both operands,
# the lo*lo term dropped): unit ratio 2^-16 / 2^-53
BF16X3_OVER_FP64 = 2.0 ** 37


def mixed(n=6, order=3, seed=0, system="euler", mu=0.02):
    rng = np.random.default_rng(seed)
    m = meshes.mixed_mesh(n, n, order=order, split=rng.random(n * n) < 0.5,
                          diag=rng.integers(0, 2, n * n))
    return Workload(f"mixed{n}_p{order}_{system}", m, system, mu=mu,
                    ic=lambda b, x: fields.isentropic_vortex(x))


def perturbed(d, u, seed=0, eps=1e-3):
    rng = np.random.default_rng(seed)
    return [x * (1 + eps * rng.standard_normal(x.shape)) for x in u]


SMALL = {
    "vortex7_p3": lambda: configs.vortex_quads(7, 3),
    "vortex5_p1": lambda: configs.vortex_quads(5, 1),
    "vortex4_p6": lambda: configs.vortex_quads(4, 6),
    "mixed6_p3_euler": lambda: mixed(6, 3),
    "mixed5_p4_euler": lambda: mixed(5, 4, seed=3),
    "mixed5_p2_ns": lambda: mixed(5, 2, system="ns"),
    "tgv5_p3": lambda: configs.taylor_green_hexes(5, 3),
    "tgv3_p4": lambda: configs.taylor_green_hexes(3, 4),
    "tgv4_p1": lambda: configs.taylor_green_hexes(4, 1),
    "curved4_p4": lambda: configs.curved_freestream_hexes(4, 4),
    "curved3_p2_ns": lambda: _curved_ns(),
}


def _curved_ns():
    w = configs.curved_freestream_hexes(4, 2)
    w.system = "ns"
    w.mu = 0.01
    w.prandtl = 0.71
    return w
