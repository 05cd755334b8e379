"""The five seeded workloads (and scaled-down variants for tests).

A workload is a mesh (from :mod:`workloads.meshes`), the physical parameters,
the RK4 time step and an initial-condition callback.  The callback receives a
block index and the physical coordinates of that block's solution points,
shape (nelem, nupts, ndims), and returns conserved variables of shape
(nelem, nupts, nvars).  Whoever places the solution points (library or
oracle) supplies the coordinates.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable

import numpy as np

from . import fields, meshes


@dataclass
class Workload:
    name: str
    mesh: meshes.Mesh
    system: str                      # "euler" | "ns"
    gamma: float = 1.4
    mu: float = 0.0
    prandtl: float = 0.72
    ldg_beta: float = 0.5
    ldg_tau: float = 0.1
    dt: float = 1e-3
    nsteps: int = 100
    ic: Callable = None              # (block, coords) -> (nelem, nupts, nvars)
    dt_per_problem: np.ndarray | None = None
    info: dict = field(default_factory=dict)

    @property
    def nvars(self):
        return self.mesh.ndims + 2


def vortex_quads(n=20, order=3, nsteps=100, dt=1e-3):
    """Isentropic vortex (strength 5, R=1, free stream (1,0)) on periodic
    n x n straight quads covering [-5,5]^2."""
    mesh = meshes.quad_mesh(n, n, (-5.0, -5.0), (5.0, 5.0), order=order)
    return Workload(f"vortex_quad{n}x{n}_p{order}", mesh, "euler", dt=dt,
                    nsteps=nsteps,
                    ic=lambda b, x: fields.isentropic_vortex(x))


def with_correction(w, scheme):
    """The same workload with every block on the named correction scheme
    ("dg", "sd" or "hu"); the name gets the scheme as a suffix."""
    for b in w.mesh.blocks:
        b.correction = scheme
    w.name = f"{w.name}_{scheme}"
    return w


# The vortex of the super-accuracy test (validation section): strength 13.5,
# Mach 0.4, radius 1.5 on [-20, 20]^2 with p = 3 and RK4 steps of 0.00125.
VORTEX_E1 = dict(S=13.5, M=0.4, R=1.5, L=40.0, order=3, dt=0.00125)
VORTEX_E1_SPACINGS = {"1/3": 120, "2/7": 140, "1/4": 160, "2/9": 180}


def vortex_superaccuracy(n=120, scheme="dg", order=3):
    """The super-accuracy vortex on n x n quads over [-20, 20]^2 (h = 40/n:
    n = 120, 140, 160, 180 give the spacings 1/3, 2/7, 1/4, 2/9), here with
    the free stream along +x: periodic in x, so the vortex is back on the
    origin every 40 time units, and the faces at y = +-20 held at the free
    stream through a fixed ghost state (boundaries 0 and 1)."""
    c = VORTEX_E1
    h = c["L"] / 2
    m = meshes.quad_mesh(n, n, (-h, -h), (h, h), order=order, walls_y=True)
    pinf = 1.0 / (fields.GAMMA * c["M"] ** 2)
    fixed = {"type": "supersonic-inflow", "rho": 1.0, "v": (1.0, 0.0, 0.0), "p": pinf}
    m.bcs = (fixed, fixed)
    for b in m.blocks:
        b.correction = scheme
    vortex = dict(S=c["S"], M=c["M"], R=c["R"])
    return Workload(f"vortex_e1_quad{n}_p{order}_{scheme}", m, "euler", dt=c["dt"],
                    ic=lambda b, x: fields.isentropic_vortex(x, **vortex),
                    info=dict(vortex=vortex, period=c["L"]))


def taylor_green_hexes(n=16, order=3, nsteps=100, dt=3e-4, Re=1600.0, Ma=0.1):
    """Navier-Stokes Taylor-Green vortex on periodic [0,2pi]^3, n^3 hexes."""
    L = 2.0 * np.pi
    mesh = meshes.hex_mesh(n, n, n, (0.0, 0.0, 0.0), (L, L, L), order=order)
    return Workload(f"tgv_hex{n}^3_p{order}", mesh, "ns", mu=1.0 / Re,
                    prandtl=0.71, ldg_beta=0.5, ldg_tau=0.1, dt=dt,
                    nsteps=nsteps, ic=lambda b, x: fields.taylor_green(x, Ma=Ma),
                    info=dict(Re=Re, Ma=Ma))


def curved_freestream_hexes(n=48, order=4, seed=3, nsteps=10, dt=None,
                            eps=0.05, amp=0.1):
    """Euler on [0,1]^3 with n^3 quadratic (Q2) hexes whose nodes are moved by
    amp*sin(2pi X)sin(2pi Y)sin(2pi Z)(1,1,1); uniform stream plus smooth
    random modes of amplitude eps drawn from ``seed``.

    dt defaults to 3.6e-3 / n: the spectral radius of the p=4 right-hand
    side's Jacobian, by power iteration on the mesh family, is about 540 n
    (5845 at n=12, 12451 at n=24, 25838 at n=48), and dt <= 2 / lambda_max
    keeps every mode inside RK4's stability region with margin (dt lambda
    about 1.95 at n=48).  A step of 2e-4 at n=48 (dt lambda 5.2) diverges
    within 20 steps."""
    if dt is None:
        dt = 3.6e-3 / n
    mesh = meshes.hex_mesh(n, n, n, order=order, geom_order=2,
                           mapping=meshes.sine_perturbation(amp, 1.0))
    modes = fields.freestream_modes(3, seed, eps=eps)
    return Workload(f"curved_hex{n}^3_q2_p{order}", mesh, "euler", dt=dt,
                    nsteps=nsteps,
                    ic=lambda b, x: fields.perturbed_freestream(x, modes),
                    info=dict(modes=modes))


def batched_vortices(nproblems=512, seed=4, nmin=50, nmax=5000, nsteps=20,
                     dt=1e-3):
    """Many independent periodic 2-D Euler problems in one mesh.

    Per problem, in draw order: target element count log-uniform in
    [nmin, nmax]; order p in {2,3,4}; split fraction f ~ U[0.25,0.75]; the
    grid side n = max(3, round(sqrt(N/(1+f)))); floor(f n^2) cells chosen by
    permutation, each split along a random diagonal; vortex centre ~ U[-2,2]^2
    and strength ~ U[2,5].  Elements are grouped into blocks by (type, p)
    with per-element problem ids.
    """
    rng = np.random.default_rng(seed)
    groups = {}          # (etype, p) -> list of node arrays / problem ids
    recs = []
    probs = []
    for prob in range(nproblems):
        N = np.exp(rng.uniform(np.log(nmin), np.log(nmax)))
        p = int(rng.integers(2, 5))
        f = rng.uniform(0.25, 0.75)
        n = max(3, int(round(np.sqrt(N / (1.0 + f)))))
        perm = rng.permutation(n * n)
        nsplit = int(np.floor(f * n * n))
        split = np.zeros(n * n, bool)
        split[perm[:nsplit]] = True
        diag = rng.integers(0, 2, size=n * n).astype(np.int32)
        centre = rng.uniform(-2.0, 2.0, size=2)
        S = rng.uniform(2.0, 5.0)
        qn, tn, pairs = meshes.mixed_quad_tri_mesh(n, n, split=split, diag=diag)
        probs.append(dict(p=p, n=n, centre=centre, S=S, quad_nodes=qn, tri_nodes=tn,
                          pairs=pairs))
        keys = {0: ("quad", p), 1: ("tri", p)}
        offs = {}
        for code, arr in ((0, qn), (1, tn)):
            g = groups.setdefault(keys[code], dict(nodes=[], prob=[], count=0))
            offs[code] = g["count"]
            if len(arr):
                g["nodes"].append(arr)
                g["prob"].append(np.full(len(arr), prob, np.int32))
                g["count"] += len(arr)
        recs.append((pairs, keys, offs))
        probs[-1]["offsets"] = dict(offs)
    order = sorted(groups.keys(), key=lambda k: (k[0] != "quad", k[1]))
    bidx = {k: i for i, k in enumerate(order)}
    blocks = []
    for k in order:
        g = groups[k]
        blocks.append(meshes.Block(k[0], k[1], 1, np.concatenate(g["nodes"]),
                                   np.concatenate(g["prob"])))
    allp = []
    for pairs, keys, offs in recs:
        q = pairs.copy()
        for side in ("l", "r"):
            code = pairs[side + "block"]
            q[side + "block"] = np.where(code == 0, bidx[keys[0]], bidx.get(keys[1], -1))
            q[side + "elem"] = pairs[side + "elem"] + np.where(code == 0, offs[0], offs[1])
        allp.append(q)
    mesh = meshes.Mesh(2, blocks, np.concatenate(allp), nproblems=nproblems,
                       info=dict(problems=probs, h=min(10.0 / pr["n"] for pr in probs)))

    def ic(b, x):
        blk = blocks[b]
        out = np.empty(x.shape[:-1] + (4,))
        for prob in np.unique(blk.problem):
            sel = blk.problem == prob
            pr = probs[prob]
            out[sel] = fields.isentropic_vortex(x[sel], S=pr["S"], centre=pr["centre"])
        return out

    for pr in probs:
        pr["blocks"] = (bidx[("quad", pr["p"])], bidx[("tri", pr["p"])])
    # step sizes differ per problem (smaller on finer grids)
    dts = np.array([dt * min(1.0, 10.0 / pr["n"] * 2.0) for pr in probs])
    return Workload(f"batched{nproblems}_vortex", mesh, "euler", dt=dt,
                    nsteps=nsteps, ic=ic, dt_per_problem=dts)


def single_problem(batched, j):
    """Problem j of a batched workload as a stand-alone workload, and the
    (block, first element) of its quads and triangles in the batched mesh."""
    pr = batched.mesh.info["problems"][j]
    qn, tn, pairs = pr["quad_nodes"], pr["tri_nodes"], pr["pairs"]
    m = meshes.Mesh(2, [meshes.Block("quad", pr["p"], 1, qn), meshes.Block("tri", pr["p"], 1, tn)],
                    pairs, info=dict(h=10.0 / pr["n"]))
    w = Workload(f"problem{j}", m, "euler", dt=float(batched.dt_per_problem[j]),
                 ic=lambda b, x: fields.isentropic_vortex(x, S=pr["S"], centre=pr["centre"]))
    where = [(pr["blocks"][0], pr["offsets"][0], len(qn)), (pr["blocks"][1], pr["offsets"][1], len(tn))]
    return w, where


def couette_walls(c=fields.COUETTE):
    """The two no-slip isothermal plates: boundary 0 at rest (y = 0), boundary
    1 moving with v_w in x (y = H)."""
    cptw = c["cp"] * c["Tw"]
    return ({"type": "no-slip-isothermal-wall", "cp_tw": cptw, "vw": (0.0, 0.0, 0.0)},
            {"type": "no-slip-isothermal-wall", "cp_tw": cptw, "vw": (c["vw"], 0.0, 0.0)})


def couette(n=8, order=2, etype="quad", seed=0, nsteps=1000, dt=None, start="exact"):
    """Couette flow (paper section 5) on [0, 1] x [0, H] (x [0, 1] in 3-D),
    periodic in x (and z), walls at y = 0 and y = H.  etype: "quad", "mixed"
    (random cells split into triangles, seed) or "hex".  start: "exact" (the
    analytic solution) or "constant" (the paper's constant start)."""
    c = fields.COUETTE
    if etype == "quad":
        m = meshes.quad_mesh(n, n, lo=(0.0, 0.0), hi=(1.0, c["H"]), order=order, walls_y=True)
    elif etype == "mixed":
        rng = np.random.default_rng(seed)
        m = meshes.mixed_mesh(n, n, lo=(0.0, 0.0), hi=(1.0, c["H"]), order=order,
                              split=rng.random(n * n) < 0.5, diag=rng.integers(0, 2, n * n),
                              walls_y=True)
    else:
        m = meshes.hex_mesh(n, n, n, lo=(0.0, 0.0, 0.0), hi=(1.0, c["H"], 1.0), order=order,
                            walls_y=True)
    m.bcs = couette_walls(c)
    h = c["H"] / n
    if dt is None:
        # acoustic bound of RK4 with margin: (|v| + c) (p + 1)^2 / h
        dt = 0.5 * h / (420.0 * (order + 1) ** 2)
    ic = fields.couette if start == "exact" else fields.couette_initial
    return Workload(f"couette_{etype}{n}_p{order}", m, "ns", gamma=c["gamma"], mu=c["mu"],
                    prandtl=c["prandtl"], dt=dt, nsteps=nsteps,
                    ic=lambda b, x: ic(x), info=dict(exact=fields.couette, couette=c))


def channel(n=6, order=3, system="euler", Ma=2.0, eps=0.0, seed=0, mu=0.01):
    """A stream along x through [0, 2] x [0, 1]: supersonic inflow of the
    stream at x = 0 (boundary 0), subsonic outflow at its pressure at x = 2
    (boundary 1), periodic in y.  eps > 0 adds smooth random modes to the
    initial state (the boundary data stay the unperturbed stream)."""
    rho, p = 1.0, 1.0 / (1.4 * Ma * Ma)
    m = meshes.quad_mesh(2 * n, n, lo=(0.0, 0.0), hi=(2.0, 1.0), order=order, open_x=(0, 1))
    m.bcs = ({"type": "supersonic-inflow", "rho": rho, "v": (1.0, 0.0, 0.0), "p": p},
             {"type": "subsonic-outflow", "p": p})
    modes = fields.freestream_modes(2, seed, eps=eps) if eps > 0 else None

    def ic(b, x):
        if modes is None:
            return fields.uniform(x, rho=rho, vel=(1.0, 0.0), p=p)
        return fields.perturbed_freestream(x, modes, vel=(1.0, 0.0), Ma=Ma)
    return Workload(f"channel{n}_p{order}_{system}", m, system, mu=mu if system == "ns" else 0.0,
                    dt=1e-3, ic=ic)


def adjoint_tgv(n=24, order=3, nsteps=200, dt=2e-4, ckpt=20):
    w = taylor_green_hexes(n=n, order=order, nsteps=nsteps, dt=dt)
    w.name = f"adjoint_tgv_hex{n}^3_p{order}"
    w.info["ckpt"] = ckpt
    return w


CONFIGS = {
    "vortex20_p3": lambda: vortex_quads(20, 3),
    "tgv16_p3": lambda: taylor_green_hexes(16, 3),
    "curved48_p4": lambda: curved_freestream_hexes(48, 4),
    "batched512": lambda: batched_vortices(512),
    "tgv24_p3": lambda: adjoint_tgv(24, 3),
}
