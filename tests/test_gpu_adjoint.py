"""The hand-written adjoint of the library against the oracle's exact
(complex-step) derivatives: the dot-product identity <J v, w> = <v, J^T w>
for the right-hand side and the RK4 step, a brute-force transpose on tiny
meshes, and central differences of a kinetic-energy objective through the
checkpointed autograd wrapper."""
import numpy as np
import pytest

import frcases as C
from oracle import Discretisation, jvp, rk4_jvp
from workloads import configs

pytestmark = pytest.mark.gpu


def _rand_like(u, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(x.shape) * np.abs(x).mean(axis=(0, 2), keepdims=True) for x in u]


def _off_kink(d, u, seed=9, eps=1e-3):
    """Additive perturbation of every field (scaled by the field's mean size):
    moves the state off the points where |n.v| in the Rusanov speed has a kink
    (e.g. a flux point on a symmetry line with v = 0 exactly), where the
    derivative is not defined and sign(0) := 0 is a convention."""
    rng = np.random.default_rng(seed)
    out = []
    for x in u:
        sc = np.abs(x).mean(axis=(0, 2))
        sc = np.maximum(sc, 0.1 * np.median(sc))       # fields that vanish (w = 0)
        out.append(x + eps * sc[None, :, None] * rng.standard_normal(x.shape))
    return out


def _dot(a, b):
    return sum(float(np.sum(x * y)) for x, y in zip(a, b))


def _norm(a):
    return np.sqrt(_dot(a, a))


@pytest.mark.parametrize("name", ["vortex7_p3", "mixed6_p3_euler", "mixed5_p2_ns", "tgv3_p4",
                                  "curved4_p4", "tgv4_p1", "curved3_p2_ns"])
def test_rhs_vjp_dot_product(name):
    w = C.SMALL[name]()
    d = Discretisation(w)
    u = _off_kink(d, d.initial_state(w))
    v = _rand_like(u, 1)
    lam = _rand_like(u, 2)
    Jv = jvp(d, u, v)
    s = C.solver_for(w)
    JTl = s.unpack(s.rhs_adjoint(s.pack(u), s.pack(lam)))
    lhs, rhs = _dot(Jv, lam), _dot(v, JTl)
    scale = _norm(Jv) * _norm(lam)
    print(f"{name}: <Jv,l> {lhs:.6e} <v,J^T l> {rhs:.6e} rel {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-13 * scale


@pytest.mark.parametrize("name", ["vortex3_p1", "tgv2_p1", "mixed3_p1_ns"])
def test_rhs_vjp_brute_force_transpose(name):
    if name == "vortex3_p1":
        w = configs.vortex_quads(3, 1)
    elif name == "tgv2_p1":
        w = configs.taylor_green_hexes(2, 1)
    else:
        w = C.mixed(3, 1, system="ns")
    d = Discretisation(w)
    u = C.perturbed(d, d.initial_state(w))
    shapes = [x.shape for x in u]
    sizes = [int(np.prod(sh)) for sh in shapes]
    n = sum(sizes)
    cols = []
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        parts, off = [], 0
        for sh, sz in zip(shapes, sizes):
            parts.append(e[off:off + sz].reshape(sh))
            off += sz
        cols.append(np.concatenate([x.ravel() for x in jvp(d, u, parts)]))
    J = np.stack(cols, 1)
    lam = _rand_like(u, 4)
    ref = J.T @ np.concatenate([x.ravel() for x in lam])
    s = C.solver_for(w)
    got = np.concatenate([x.ravel() for x in s.unpack(s.rhs_adjoint(s.pack(u), s.pack(lam)))])
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"{name}: {n} DOF, J^T lam rel L2 {err:.2e}")
    assert err < 1e-12


@pytest.mark.parametrize("name", ["vortex7_p3", "mixed5_p2_ns", "tgv3_p4"])
def test_rk_step_vjp_dot_product(name):
    w = C.SMALL[name]()
    d = Discretisation(w)
    u = _off_kink(d, d.initial_state(w))
    v = _rand_like(u, 5)
    lam = _rand_like(u, 6)
    dt = 2e-3 if w.system == "euler" else 1e-3
    Jv = rk4_jvp(d, u, v, dt)
    s = C.solver_for(w)
    lt = s.pack(lam)
    JTl = s.unpack(s.rk_step_adjoint(s.pack(u), dt, lt, out=lt))   # in place on lam
    lhs, rhs = _dot(Jv, lam), _dot(v, JTl)
    scale = _norm(Jv) * _norm(lam)
    print(f"{name}: rk step dot product rel {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-13 * scale


def test_kinetic_energy_gradient_against_central_differences():
    import torch
    from paper_1312_1638_amd.autograd import KineticEnergy, integrate_steps
    w = configs.taylor_green_hexes(3, 2, dt=1e-3)
    d = Discretisation(w)
    u = _off_kink(d, d.initial_state(w), eps=1e-2)
    s = C.solver_for(w)
    u0 = s.pack(u).requires_grad_(True)
    nsteps, ckpt = 10, 4
    J = KineticEnergy.apply(integrate_steps(s, u0, w.dt, nsteps, ckpt), s)
    (g,) = torch.autograd.grad(J, u0)
    g = g.detach()
    rng = np.random.default_rng(7)
    for k in range(3):
        dirn = _rand_like(u, 10 + k)
        dt_ = s.pack(dirn)

        def obj(eps):
            x = (u0.detach() + eps * dt_).contiguous()
            s.step(x, w.dt, nsteps)
            return float(s.integrate(x)[:, -1].sum())
        ep = 1e-5
        fd = (obj(ep) - obj(-ep)) / (2 * ep)
        ad = float(torch.sum(g * dt_))
        print(f"direction {k}: adjoint {ad:.10e} central FD {fd:.10e} rel {abs(ad - fd) / abs(fd):.2e}")
        assert abs(ad - fd) <= 1e-6 * abs(fd)


def test_gradient_through_steps_matches_oracle_complex_step():
    """d/deps E_k(u_N(u0 + eps d)) at eps = 0: the oracle by complex step
    through N RK4 steps (exact), the library by its checkpointed adjoint."""
    import torch
    from paper_1312_1638_amd.autograd import KineticEnergy, integrate_steps
    w = configs.taylor_green_hexes(4, 3, dt=2e-4)
    d = Discretisation(w)
    u = _off_kink(d, d.initial_state(w), eps=1e-2)
    nsteps, ckpt = 6, 4
    s = C.solver_for(w)
    u0 = s.pack(u).requires_grad_(True)
    J = KineticEnergy.apply(integrate_steps(s, u0, w.dt, nsteps, ckpt), s)
    (g,) = torch.autograd.grad(J, u0)
    gh = s.unpack(g)
    W, Jd = d.refs[0].W, d.geoms[0].detJ.T
    for k in range(2):
        dirn = _rand_like(u, 20 + k)
        z = [a.astype(np.complex128) + 1e-30j * b for a, b in zip(u, dirn)]
        z = d.rk4(z, w.dt, nsteps)[0]
        rho, m = z[:, 0], z[:, 1:4]
        ek = np.einsum("r,rn,rn->", W, Jd, 0.5 * np.sum(m * m, 1) / rho)
        ref = np.imag(ek) / 1e-30
        got = _dot(gh, dirn)
        print(f"direction {k}: adjoint {got:.12e} oracle complex step {ref:.12e} rel {abs(got - ref) / abs(ref):.2e}")
        assert abs(got - ref) <= 1e-10 * abs(ref)


@pytest.mark.parametrize("name", ["tgv3_p4", "mixed5_p2_ns", "curved4_p4", "vortex7_p3"])
def test_fused_flux_vjp_matches_separate_kernel(name):
    """The adjoint's (M1 - M3 M2)^T product with the flux VJP in its
    epilogue, against the product followed by the flux VJP kernel (and the
    dot-product identity for the fused form); blocks without a sparse form
    (dense triangles) keep their plan."""
    import paper_1312_1638_amd as P
    w = C.SMALL[name]()
    d = Discretisation(w)
    u = _off_kink(d, d.initial_state(w))
    lam = _rand_like(u, 2)
    s = C.solver_for(w)
    out = []
    for wm in (2, 18):
        forced = 0
        for bi in range(len(w.mesh.blocks)):
            try:
                s.set_plan(bi, 14, (0, 2, wm))
                forced += 1
            except P.FRError:
                assert w.mesh.blocks[bi].etype == "tri"
        assert forced > 0
        out.append(s.unpack(s.rhs_adjoint(s.pack(u), s.pack(lam))))
    diff = C.rel_l2(out[1], out[0])
    v = _rand_like(u, 1)
    Jv = jvp(d, u, v)
    lhs, rhs = _dot(Jv, lam), _dot(v, out[1])
    scale = _norm(Jv) * _norm(lam)
    print(f"{name}: fused vs separate flux VJP rel L2 {diff:.2e}; dot product rel "
          f"{abs(lhs - rhs) / scale:.2e}")
    assert diff < 1e-13
    assert abs(lhs - rhs) <= 1e-13 * scale


def test_stash_budget_leaves_the_gradient_unchanged():
    """Segments kept resident or replayed from checkpoints (budget 0, room
    for two segments with a short last one, everything resident) give the
    same gradient: the replay repeats the forward's arithmetic."""
    import torch
    from paper_1312_1638_amd.autograd import KineticEnergy, integrate_steps
    w = configs.taylor_green_hexes(3, 2, dt=1e-3)
    d = Discretisation(w)
    u = _off_kink(d, d.initial_state(w), eps=1e-2)
    s = C.solver_for(w)
    nsteps, ckpt = 10, 3
    two = 2 * ckpt * s.stash_len() * 8
    grads = []
    for budget in (0, two, None):
        u0 = s.pack(u).requires_grad_(True)
        J = KineticEnergy.apply(integrate_steps(s, u0, w.dt, nsteps, ckpt, budget), s)
        (g,) = torch.autograd.grad(J, u0)
        grads.append(g.detach().clone())
    for g in grads[1:]:
        err = float(torch.linalg.norm(g - grads[0]) / torch.linalg.norm(grads[0]))
        print(f"gradient rel difference {err:.2e}")
        # the same kernels in the same order, whether a segment is replayed
        # (as one captured graph) or kept resident
        assert torch.equal(g, grads[0])


@pytest.mark.parametrize("name", ["mixed5_p2_ns", "curved4_p4"])
def test_segment_adjoint_matches_step_adjoints(name):
    """fr_rk_segment_adjoint (replay with stashes, then the step adjoints,
    as one captured graph) against the eager per-step stash calls: bitwise
    on the first call and on replays of the captured graph with other work
    between them, out of place and in place; u_seg0 is left untouched."""
    import torch
    w = C.SMALL[name]()
    d = Discretisation(w)
    u = _off_kink(d, d.initial_state(w))
    s = C.solver_for(w)
    dt, n, L = 1e-3, 3, s.stash_len()
    u0 = s.pack(u)
    lam_end = s.pack(_rand_like(u, 5))
    work = u0.clone()
    st = torch.zeros(n * L, dtype=torch.float64, device="cuda")
    for i in range(n):
        s.step_stash(work, dt, st[i * L:(i + 1) * L])
    ref = lam_end.clone()
    for i in reversed(range(n)):
        s.rk_step_adjoint_stash(st[i * L:(i + 1) * L], dt, ref, out=ref)
    seg_stash = torch.zeros(n * L, dtype=torch.float64, device="cuda")
    out = s.empty()
    for rep in range(3):
        out.zero_()
        s.segment_adjoint(u0, dt, n, lam_end, seg_stash, out=out)
        torch.cuda.synchronize()
        print(f"{name}: replay {rep}: max |segment - steps| {float((out - ref).abs().max()):.2e}")
        assert torch.equal(out, ref)
        s.rhs(work)                           # other work between graph replays
        torch.cuda.synchronize()
    for rep in range(2):
        lam = lam_end.clone()
        s.segment_adjoint(u0, dt, n, lam, seg_stash, out=lam)
        torch.cuda.synchronize()
        assert torch.equal(lam, ref)
    assert torch.equal(u0, s.pack(u))
    assert torch.equal(seg_stash, st)
    copy = s.segment_adjoint(u0, dt, 0, lam_end, seg_stash)
    torch.cuda.synchronize()
    assert torch.equal(copy, lam_end)


@pytest.mark.parametrize("name", ["mixed5_p2_ns", "curved4_p4"])
def test_stash_path_matches_recompute_path(name):
    import torch
    w = C.SMALL[name]()
    d = Discretisation(w)
    u = _off_kink(d, d.initial_state(w))
    s = C.solver_for(w)
    a = s.pack(u)
    b = a.clone()
    stash = torch.empty(s.stash_len(), dtype=torch.float64, device="cuda")
    s.step(a, 1e-3, 1)
    s.step_stash(b, 1e-3, stash)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    lam = s.pack(_rand_like(u, 3))
    l1 = s.rk_step_adjoint(s.pack(u), 1e-3, lam)
    l2 = s.rk_step_adjoint_stash(stash, 1e-3, lam)
    err = float(torch.linalg.norm(l1 - l2) / torch.linalg.norm(l1))
    print(f"{name}: stash vs recompute step adjoint rel {err:.2e}")
    assert err < 1e-14


@pytest.mark.parametrize("name", ["mixed5_p2_ns", "tgv3_p4", "curved3_p2_ns"])
def test_adjoint_m0t_plans_agree(name):
    """The adjoint's M0^T product with the reverse gradient transform fused
    into its epilogue (sparse-row, one or all fields per thread) against the
    unfused paths (matrix cores, LDS-staged) followed by the separate
    transform kernel."""
    import paper_1312_1638_amd as P
    w = C.SMALL[name]()
    d = Discretisation(w)
    u = _off_kink(d, d.initial_state(w))
    lam = _rand_like(u, 2)
    s = C.solver_for(w)
    got = {}
    for tag in ("mfma", "sparse", "fields", "staged"):
        for bi in range(len(w.mesh.blocks)):
            nu = s.blocks[bi]["nupts"]
            plan = {"mfma": (1, 1, -(-nu // 16)), "sparse": (0, 4, 0), "fields": (0, 2, 2),
                    "staged": (0, 64, 4)}[tag]
            try:
                s.set_plan(bi, 13, plan)
            except P.FRError:
                assert tag == "staged"
        got[tag] = s.unpack(s.rhs_adjoint(s.pack(u), s.pack(lam)))
    for tag in ("sparse", "fields", "staged"):
        err = C.rel_l2(got[tag], got["mfma"])
        print(f"{name}: adjoint with M0^T plan {tag} vs matrix cores: rel L2 {err:.2e}")
        assert err < 1e-13
