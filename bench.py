#!/usr/bin/env python3
"""Throughput of the FR right-hand side on one MI355X.

One step = one classical RK4 step of the whole hot path: four right-hand-side
evaluations (interpolation to flux points, common solution, gradients,
transformed fluxes, common interface fluxes, correction-function divergence),
the fused FP64 register updates (one captured HIP graph), and the FP64
conservation / kinetic-energy integrals.  Metric: right-hand-side
DOF-updates per second, DOF = fields x solution points x elements (the
paper's unit), four evaluations per step.

Default workload: Euler on 48^3 curved quadratic (Q2) hexahedra over the
unit cube, p=4 (125 solution points each, 6.9e7 DOF), a uniform stream plus
seeded smooth perturbations, FP64 -- the largest single-GPU configuration,
far larger than the 256 MB Infinity Cache.  Synthetic, seeded inputs; the
state is resident in HBM when timing starts.

Prints one JSON line.  Extra keys: per-step kernel times, the FP32 and
BF16x3 operator paths, the relative L2 error of each precision against the
FP64 oracle on sampled elements, the roofline of the dominant kernel, the
CPU oracle baseline (all cores and one core), the cache-resident
Taylor-Green 16^3 workload, the other time steppers and the adjoint cost.
Progress lines go to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (constructor, description)
    "tgv16": ("taylor_green_hexes", dict(n=16, order=3), "ns"),
    "tgv48": ("taylor_green_hexes", dict(n=48, order=3), "ns"),
    "vortex20": ("vortex_quads", dict(n=20, order=3), "euler"),
    "curved48": ("curved_freestream_hexes", dict(n=48, order=4), "euler"),
    "curved24": ("curved_freestream_hexes", dict(n=24, order=4), "euler"),
    "tgv24": ("taylor_green_hexes", dict(n=24, order=3), "ns"),
    "batched512": ("batched_vortices", dict(nproblems=512), "euler"),
    # Couette channels between no-slip isothermal walls (boundary conditions)
    "couette_mixed64": ("couette", dict(n=64, order=3, etype="mixed", start="constant"), "ns"),
    "couette_hex32": ("couette", dict(n=32, order=3, etype="hex", start="constant"), "ns"),
    # the super-accuracy vortex on its finest mesh (h = 2/9, p = 3) with each
    # correction scheme: same kernels, different operator values
    "vortex_e1_dg": ("vortex_superaccuracy", dict(n=180, scheme="dg"), "euler"),
    "vortex_e1_sd": ("vortex_superaccuracy", dict(n=180, scheme="sd"), "euler"),
    "vortex_e1_hu": ("vortex_superaccuracy", dict(n=180, scheme="hu"), "euler"),
}

STEP_NAMES = {1: "interp_M0", 2: "common_solution", 3: "grad_M6_M4p", 4: "grad_transform",
              5: "grad_interp_M5", 6: "transformed_flux", 7: "common_flux", 8: "div_M3_M1p",
              9: "div_M3_M1p_rk4"}


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


PEAK_HBM = 8.0e12                                           # B/s
PEAK_MFMA = {"fp64": 78.6e12, "fp32": 157.3e12}             # dense FLOP/s
ROCPROF_TRAFFIC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "hbm_traffic.md")


def operator_nnz(P, etype, order, which, correction="dg"):
    """Structural non-zeros of a reference operator (entries above 1e-13 of
    their row's largest magnitude; the rest is rounding residue)."""
    import numpy as np
    A = P.reference_operator(etype, order, which, correction)
    mx = np.abs(A).max(axis=1, keepdims=True)
    return int((np.abs(A) > 1e-13 * mx).sum())


def step_model(s, step, ts):
    """Algorithmic (bytes, flops) of one launch of RHS step `step` over all
    blocks: each array read once and written once, operators cached; an
    operator product costs 2 flops per structural non-zero of the operator
    and state column (multiplications by structural zeros are not work)."""
    D, NV = s.ndims, s.nvars
    byts = flops = 0.0
    for bi, (blk, b) in enumerate(zip(s.blocks, s.mesh.blocks)):
        ne, nu = blk["nelem"], blk["nupts"]
        nf = s.nfpts[b.etype, b.order]
        nnz = s.nnz[b.etype, b.order]
        cols = NV * ne
        if step == 1:
            flops += 2.0 * nnz["M0"] * cols
            byts += cols * (nu * 8 + nf * ts)
        elif step == 3:
            flops += 2.0 * (nnz["M6"] + nnz["M4p"]) * cols
            byts += cols * (nf * ts + nu * 8 + D * nu * ts)
            if s.fused_gradt[bi]:        # step 4 in the epilogue: S = adj J and 1/J
                byts += (D * D + 1) * nu * ne * 8
            if s.fused_flux[bi]:         # step 6 too: F~ written (u is panel 2)
                byts += D * nu * cols * ts
        elif step == 4:
            if not s.fused_gradt[bi]:
                byts += 2.0 * D * nu * cols * ts + (D * D + 1) * nu * ne * 8
        elif step == 5:
            flops += 2.0 * D * nnz["M0"] * cols
            byts += D * cols * (nu + nf) * ts
        elif step == 6 and not s.fused_flux[bi]:
            byts += nu * ne * (NV * 8 + D * D * 8 + D * NV * ts)
            if s.system == "ns":
                byts += nu * ne * D * NV * ts
        elif step == 8:
            flops += 2.0 * (nnz["M3"] + nnz["M1p"]) * cols
            byts += cols * (nf + D * nu) * ts + nu * ne * 8 + nu * cols * 8
        elif step == 9:
            # step 8 with the RK4 update of a middle stage: u and the
            # accumulator read, the accumulator and the next stage written
            flops += 2.0 * (nnz["M3"] + nnz["M1p"]) * cols
            byts += cols * (nf + D * nu) * ts + nu * ne * 8 + 4 * nu * cols * 8
    npairs = s.npairs
    if step == 2:
        byts += npairs * (4 * NV * ts + 8)
    elif step == 7:
        byts += npairs * (4 * NV * ts + 8 + (D + 2) * 8)
        if s.system == "ns":
            byts += npairs * 2 * D * NV * ts
    return byts, flops


def make_solver(workload, prec, P, configs):
    import numpy as np
    w = getattr(configs, WORKLOADS[workload][0])(**WORKLOADS[workload][1])
    s = P.Solver(w.mesh, system=w.system, gamma=w.gamma, mu=w.mu, prandtl=w.prandtl,
                 ldg_beta=w.ldg_beta, ldg_tau=w.ldg_tau, prec=prec)
    s.system = w.system
    s.nfpts, s.nnz = {}, {}
    for b in w.mesh.blocks:
        s.nfpts[b.etype, b.order] = P.reference_operator(b.etype, b.order, 6).shape[0]
        s.nnz[b.etype, b.order] = {k: operator_nnz(P, b.etype, b.order, i, b.correction)
                                   for k, i in (("M0", 0), ("M3", 1), ("M4p", 2), ("M6", 3),
                                                ("M1p", 4))}
    # flux-point interfaces: face pairs, plus boundary faces (one side each)
    nfp_face = {b: P.reference_operator(blk.etype, blk.order, 6).shape[0] //
                {"quad": 4, "tri": 3, "hex": 6}[blk.etype] for b, blk in enumerate(w.mesh.blocks)}
    s.npairs = int(sum(nfp_face[int(b)] for b in w.mesh.pairs["lblock"]))
    bcf = getattr(w.mesh, "bcfaces", None)
    if bcf is not None:
        s.npairs += int(sum(nfp_face[int(b)] for b in bcf["block"]))
    # step 3 with the gradient transform (step 4) fused into its epilogue
    s.fused_gradt = [w.system == "ns" and s.gemm_plan(b, 3)[0] == 0 and s.gemm_plan(b, 3)[2] & 1
                     for b in range(len(w.mesh.blocks))]
    # ... and the transformed flux (step 6) as well
    s.fused_flux = [bool(f) and s.gemm_plan(b, 3)[2] & 15 == 11
                    for b, f in enumerate(s.fused_gradt)]
    u0 = [np.ascontiguousarray(np.transpose(w.ic(b, s.solution_points(b)), (1, 2, 0)))
          for b in range(len(w.mesh.blocks))]
    s.bench_dt = w.dt
    if w.dt_per_problem is not None:
        import torch
        s.bench_dt = torch.tensor(w.dt_per_problem, dtype=torch.float64, device="cuda")
    return w, s, u0


def time_steps(s, u, dt, steps, warmup, torch):
    for _ in range(warmup):
        s.step(u, dt, 1)
        s.integrate(u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.step(u, dt, 1)
        s.integrate(u)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def stepper_costs(s, u0, dt, steps, torch, atol=1e-8, rtol=1e-8):
    """The other time steppers on the same mesh: forward Euler (ms per
    step, one right-hand side) and adaptive DOPRI5 from dt (ms per attempt,
    six right-hand sides; one more per call), with the controller's accepted
    and rejected counts over `steps` attempts."""
    out = {}
    u = s.pack(u0)
    s.euler_step(u, dt, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.euler_step(u, dt, steps)
    torch.cuda.synchronize()
    out["euler_ms_per_step"] = (time.perf_counter() - t0) / steps * 1e3
    n = s.nproblems
    for rep in range(2):                       # the first call captures the graph
        u = s.pack(u0)
        t = torch.zeros(n, dtype=torch.float64, device="cuda")
        h = torch.full((n,), float(dt), dtype=torch.float64, device="cuda")
        cnt = torch.zeros((n, 2), dtype=torch.int32, device="cuda")
        k = 2 if rep == 0 else steps
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.dopri5(u, t, h, k, atol, rtol, counts=cnt)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    c = cnt.cpu().numpy()
    out["dopri5"] = dict(ms_per_attempt=el / steps * 1e3, rhs_per_attempt=6, atol=atol, rtol=rtol,
                         first_dt=float(dt), attempts=steps, accepted=int(c[:, 0].sum()),
                         rejected=int(c[:, 1].sum()), final_t=float(t.max().item()),
                         final_dt=float(h.max().item()))
    return out


def plan_name(plan, step=0):
    mbw, nc, wm = plan
    if mbw == 0 and wm & 4:
        return "sparse-row LDS-staged" + (" + fused J^-T (step 4)" if step == 3 and wm & 1 else "")
    if mbw == 0:
        return (f"sparse-row rpg={nc}" + (" all fields per thread" if wm & 2 else "")
                + (" + fused J^-T (step 4)" if step == 3 and wm & 1 else "")
                + (" + fused transformed flux (step 6)" if step == 3 and wm & 8 else ""))
    return f"mfma {mbw}x{nc} wm={wm}"


def time_kernels(s, u, torch, nrep=50):
    """Average launch duration of every RHS step, HIP events on the stream
    the kernels are launched on (torch's current stream, passed to the
    library)."""
    out = {}
    steps = [1, 6, 7, 8, 9] if s.system == "euler" else [1, 2, 3, 4, 5, 6, 7, 8, 9]
    stream = torch.cuda.current_stream()
    for st in steps:
        s.bench_step(u, st, 2)                           # warm
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        # the bench hook first re-runs the steps before `st` once; time that
        # alone and subtract it
        e0.record(stream)
        s.bench_step(u, st, 0)
        e1.record(stream)
        torch.cuda.synchronize()
        prep = e0.elapsed_time(e1)
        e0.record(stream)
        s.bench_step(u, st, nrep)
        e1.record(stream)
        torch.cuda.synchronize()
        out[st] = (e0.elapsed_time(e1) - prep) / nrep * 1e-3   # seconds per launch
    return out


def adjoint_ratio(P, configs, torch, n=24, nsteps=200, ckpt=20):
    """Wall time of the full gradient of E_k(u_N) with respect to u_0 (forward
    with checkpoints, segment replay, hand-written RK4 adjoint) over the wall
    time of the N forward steps: Taylor-Green, n^3 hexes, p=3, FP64.  value:
    the default stash budget (free device memory less a reserve: segments
    that fit keep their stash and are never replayed), a repeated gradient
    (the stash memory already mapped); value_first_call: the first gradient,
    which also maps that memory; value_replay_all: budget 0 (every segment
    but the last replayed from its checkpoint)."""
    import numpy as np
    from paper_1312_1638_amd.autograd import KineticEnergy, integrate_steps, stash_segments
    w = configs.adjoint_tgv(n=n, order=3, nsteps=nsteps, ckpt=ckpt)
    s = P.Solver(w.mesh, system=w.system, gamma=w.gamma, mu=w.mu, prandtl=w.prandtl,
                 ldg_beta=w.ldg_beta, ldg_tau=w.ldg_tau)
    u0h = [np.ascontiguousarray(np.transpose(w.ic(b, s.solution_points(b)), (1, 2, 0)))
           for b in range(len(w.mesh.blocks))]
    u0 = s.pack(u0h)
    x = u0.clone()
    s.step(x, w.dt, 2)                      # capture the step graph, warm
    x.copy_(u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(x, w.dt, nsteps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    u0g = u0.clone().requires_grad_(True)
    J = KineticEnergy.apply(integrate_steps(s, u0g, w.dt, 1, 1), s)   # warm the adjoint
    torch.autograd.grad(J, u0g)
    out = {}
    nseg = -(-nsteps // ckpt)
    for key, budget in (("replay_all", 0), ("default", None)):
        resident = min(nseg, max(1, int(stash_segments(s.stash_len(), ckpt, budget, u0.device))))
        times = []
        for _rep in range(2):               # the first call also maps the stash memory
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            J = KineticEnergy.apply(integrate_steps(s, u0g, w.dt, nsteps, ckpt, budget), s)
            (g,) = torch.autograd.grad(J, u0g)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            del J, g
        out[key] = (times, resident)
    seg_gb = s.stash_len() * ckpt * 8 / 1e9
    s.close()
    torch.cuda.empty_cache()
    (first, t_grad), resident = out["default"]
    return dict(value=t_grad / t_fwd, unit="gradient wall time / forward wall time",
                workload=w.name, steps=nsteps, checkpoint_every=ckpt,
                segments=nseg, segments_resident=resident, stash_GB_per_segment=seg_gb,
                value_replay_all=out["replay_all"][0][1] / t_fwd,
                value_first_call=first / t_fwd,
                forward_s=t_fwd, gradient_s=t_grad, gradient_first_call_s=first,
                gradient_replay_all_s=out["replay_all"][0][1],
                objective="kinetic energy at t_N")


def sample_elements(nelem, nsample, seed):
    """Seeded random elements plus element 0, the last element, one inside
    the last tile of 256 columns and the two elements either side of the
    first boundary between XCD tile groups (2047, 2048)."""
    import numpy as np
    fixed = [0, nelem - 1, (nelem - 1) // 256 * 256 + min(97, (nelem - 1) % 256)]
    if nelem > 2048:
        fixed += [2047, 2048]
    rnd = np.random.default_rng(seed).choice(nelem, min(nsample, nelem), replace=False)
    return np.unique(np.concatenate([fixed, rnd]))


def patch_workload(w, sample, rings):
    """The sampled elements of a single-block workload plus `rings` layers
    of face neighbours, as a workload of its own (faces on its outer
    boundary unpaired).  Returns (workload, index of each sample in it)."""
    import dataclasses
    import numpy as np
    from workloads import meshes
    pr = w.mesh.pairs
    le, re = pr["lelem"].astype(np.int64), pr["relem"].astype(np.int64)
    b = w.mesh.blocks[0]
    inside = np.zeros(b.nelem, bool)
    inside[sample] = True
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
    blk.correction = getattr(b, "correction", "dg")
    mesh = meshes.Mesh(w.mesh.ndims, [blk], sub, info=dict(w.mesh.info))
    return dataclasses.replace(w, mesh=mesh), local[sample]


def host_info():
    """nproc (CPUs this process may run on), the CPU model and the BLAS
    thread pool that numpy's contractions use."""
    info = dict(nproc=len(os.sched_getaffinity(0)), cpu_model=None, blas_threads=None)
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        info["blas_threads"] = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        pass
    return info


def cpu_baseline(w, nsample, seed=33, reps=5):
    """The FP64 oracle on the host, on a bounded sample of the workload.

    Single-block meshes (the curved and Taylor-Green hexes): a patch of the
    mesh -- `nsample` seeded elements (plus the fixed edge elements) and
    their face neighbours (two rings for Navier-Stokes) -- and the median of
    `reps` right-hand sides over the whole patch, with numpy's BLAS pool at
    its default size and again limited to one thread.  The oracle's du/dt
    on the sampled elements, which the patch computes completely, is
    returned as well: it is the reference of every precision's error.
    Other meshes: one RK4 step of the whole workload, timed."""
    import numpy as np
    from oracle import Discretisation
    hi = host_info()
    single_block = len(w.mesh.blocks) == 1 and getattr(w.mesh, "bcfaces", None) is None
    out = dict(unit="RHS DOF-updates/s", kind="oracle", nproc=hi["nproc"],
               cpu_model=hi["cpu_model"], cores=hi["blas_threads"] or 1,
               threads_note="plain numpy FP64 reference (not a tuned CPU solver): its "
                            "contractions run on numpy's BLAS pool (cores), the rest on one "
                            "thread")
    ref = None
    if single_block:
        sample = sample_elements(w.mesh.blocks[0].nelem, nsample, seed)
        pw, loc = patch_workload(w, sample, 2 if w.system == "ns" else 1)
        d = Discretisation(pw, allow_unpaired=True)
        u = d.initial_state(pw)
        dof = sum(r.nupts * g.nelem for r, g in zip(d.refs, d.geoms)) * d.nvars

        def timed(n):
            ts = []
            for _ in range(n):
                t0 = time.perf_counter()
                r = d.rhs(u)
                ts.append(time.perf_counter() - t0)
            return float(np.median(ts)), r

        t_all, r = timed(reps)
        ref = dict(sample=sample, rhs=r[0][:, :, loc])
        try:
            from threadpoolctl import threadpool_limits
            with threadpool_limits(1):
                t_one, _ = timed(max(3, reps // 2))
        except Exception:
            t_one = None
        out.update(value=dof / t_all, value_one_core=(dof / t_one) if t_one else None,
                   sample=f"median of {reps} right-hand sides on a patch of {d.geoms[0].nelem} "
                          f"elements of the same mesh ({len(sample)} seeded elements and their "
                          f"face neighbours; {dof} DOF per right-hand side), numpy FP64 oracle: "
                          f"{t_all:.2f} s per right-hand side on the BLAS pool, "
                          + (f"{t_one:.2f} s on one thread" if t_one else "one-thread run "
                             "unavailable"))
    else:
        d = Discretisation(w)
        u = d.initial_state(w)
        dof = sum(r.nupts * g.nelem for r, g in zip(d.refs, d.geoms)) * d.nvars
        t0 = time.perf_counter()
        d.rk4(u, w.dt, 1)
        el = time.perf_counter() - t0
        out.update(value=4.0 * dof / el, value_one_core=None,
                   sample=f"1 RK4 step (4 right-hand sides) of the whole workload, numpy FP64 "
                          f"oracle, {el:.1f} s")
    return out, ref


def sampled_error(s, u, ref):
    """Relative L2 error of the library's du/dt on the sampled elements
    against the FP64 oracle's, over the whole sample and per field."""
    import numpy as np
    r = s.unpack(s.rhs(s.pack(u)))[0][:, :, ref["sample"]]
    e = r - ref["rhs"]
    whole = float(np.sqrt(np.sum(e ** 2) / np.sum(ref["rhs"] ** 2)))
    per = np.sqrt(np.sum(e ** 2, axis=(0, 2)) / np.sum(ref["rhs"] ** 2, axis=(0, 2)))
    return dict(rel_l2=whole, rel_l2_per_field=[float(x) for x in per],
                sampled_elements=int(len(ref["sample"])),
                reference="FP64 oracle on a patch around the sampled elements")


def measure_workload(name, prec, args, P, configs, torch, with_kernels=True):
    """Solver set-up (with the plan tuner), timed RK4 steps and per-kernel
    launch times of one workload in one precision."""
    progress(f"{name} {prec}: set-up and plan tuning")
    w, s, u0 = make_solver(name, prec, P, configs)
    dof = sum(b["nupts"] * b["nelem"] for b in s.blocks) * s.nvars
    progress(f"{name} {prec}: {args.warmup} + {args.steps} RK4 steps")
    el = time_steps(s, s.pack(u0), s.bench_dt, args.steps, args.warmup, torch)
    kt = time_kernels(s, s.pack(u0), torch) if with_kernels else {}
    return w, s, u0, dof, el, kt


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="curved48", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-sample", type=int, default=256,
                    help="seeded elements of the oracle's patch for the CPU baseline and the "
                         "error of each precision (0: skip both)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-steppers", action="store_true",
                    help="skip the forward Euler and DOPRI5 timings")
    ap.add_argument("--no-extra-workload", action="store_true",
                    help="skip the cache-resident Taylor-Green 16^3 line")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="diagnostic: run only the adjoint cost measurement and print it")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(halo exchange across GPUs is designed, not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1312_1638_amd as P
    from workloads import configs
    assert torch.cuda.is_available(), "needs a HIP device"

    if args.adjoint_only:
        print(json.dumps(adjoint_ratio(P, configs, torch)))
        return

    w, s, u0, dof, el, kt = measure_workload(args.workload, "fp64", args, P, configs, torch)
    npts = dof // s.nvars
    ms = el / args.steps * 1e3
    value = 4.0 * dof * args.steps / el

    # the dominant kernel's roofline
    dom = max(kt, key=kt.get)
    byts, flops = step_model(s, dom, 8)
    ai = flops / byts if byts else 0.0
    ridge = PEAK_MFMA["fp64"] / PEAK_HBM
    if flops and ai > ridge:
        roof = dict(bound="mfma", achieved=flops / kt[dom] / 1e12, peak=PEAK_MFMA["fp64"] / 1e12,
                    unit="TFLOP/s")
    else:
        roof = dict(bound="hbm", achieved=byts / kt[dom] / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = STEP_NAMES[dom]
    roof["avg_launch_us"] = kt[dom] * 1e6
    roof["algorithmic_bytes"] = byts
    roof["algorithmic_flops"] = flops
    # HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    # table, null when it was taken on other library sources
    from paper_1312_1638_amd.profile_report import read_traffic_table
    roof["traffic"] = read_traffic_table(ROCPROF_TRAFFIC, args.workload, STEP_NAMES[dom])
    roof["measured_hbm_triad_GBps"] = round(P.binding.measure_ceiling(0), 1)
    roof["frac_of_measured_triad"] = (roof["achieved"] / roof["measured_hbm_triad_GBps"]
                                      if roof["unit"] == "GB/s" else None)
    kernels = {}
    for st, t in sorted(kt.items()):
        b_, f_ = step_model(s, st, 8)
        kernels[STEP_NAMES[st]] = dict(us=round(t * 1e6, 2), GBps=round(b_ / t / 1e9, 1),
                                       TFLOPs=round(f_ / t / 1e12, 2))
        if st in (1, 3, 5, 8, 9):
            kernels[STEP_NAMES[st]]["plan"] = plan_name(s.gemm_plan(0, min(st, 8)), st)
        if len(s.blocks) > 1 and st in (1, 5, 6, 8, 9):
            m = s.multi(min(st, 8))
            kernels[STEP_NAMES[st]]["launches"] = (
                "one launch over every block" if st == 6 and m else
                ", ".join(x for x, bit in (("one sparse-row launch over its blocks", 1),
                                            ("one matrix-core launch over its blocks", 2))
                          if m & bit) or "one launch per block")

    # the oracle on a bounded sample of the same mesh: CPU baseline, and the
    # reference of each precision's error on the sampled elements
    cpu, ref = None, None
    if args.cpu_sample > 0:
        progress(f"CPU oracle on a patch of {args.cpu_sample} sampled elements")
        cpu, ref = cpu_baseline(w, args.cpu_sample)
    errors = {}
    if ref is not None:
        errors["fp64"] = sampled_error(s, u0, ref)

    extra = {}
    if not args.no_steppers:
        progress("forward Euler and DOPRI5")
        extra["steppers"] = stepper_costs(s, u0, w.dt, args.steps, torch)
        extra["steppers"]["rk4_ms_per_step"] = ms
    s.close()
    torch.cuda.empty_cache()

    if not args.no_fp32:
        for prec in ("fp32", "bf16x3"):
            wr, sr, _, _, elr, ktr = measure_workload(args.workload, prec, args, P, configs, torch)
            extra[prec] = dict(value=4.0 * dof * args.steps / elr, ms_per_step=elr / args.steps * 1e3,
                               kernels_us={STEP_NAMES[k]: round(v * 1e6, 2) for k, v in ktr.items()},
                               plans={STEP_NAMES[k]: plan_name(sr.gemm_plan(0, k), k) for k in ktr
                                      if k in (1, 3, 5, 8)})
            if ref is not None:
                errors[prec] = sampled_error(sr, u0, ref)
                extra[prec]["error_vs_fp64_oracle"] = errors[prec]
            sr.close()
            torch.cuda.empty_cache()

    if not args.no_extra_workload and args.workload != "tgv16":
        wt, st_, _, doft, elt, ktt = measure_workload("tgv16", "fp64", args, P, configs, torch)
        extra["tgv16"] = dict(
            value=4.0 * doft * args.steps / elt, unit="DOF-updates/s", dtype="f64",
            ms_per_step=elt / args.steps * 1e3, workload=wt.name,
            note="every array fits in the 256 MB Infinity Cache: GB/s here are cache "
                 "bandwidth, not HBM",
            kernels_us={STEP_NAMES[k]: round(v * 1e6, 2) for k, v in ktt.items()})
        st_.close()
        torch.cuda.empty_cache()

    if not args.no_adjoint:
        progress("adjoint cost (Taylor-Green 24^3, 200 steps)")
        extra["adjoint"] = adjoint_ratio(P, configs, torch)

    line = {
        # the headline is the FP64 rate; the FP32 and BF16-split legs and the
        # adjoint/forward cost ratio are the "fp32", "bf16x3" and "adjoint" keys
        "metric": "RHS DOF-updates/s FP64 vs FP32/BF16-split; adjoint/forward cost ratio",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "system": w.system,
                   "elements": int(sum(b.nelem for b in w.mesh.blocks)),
                   "blocks": [f"{b.etype} p={b.order} x{b.nelem}" for b in w.mesh.blocks],
                   "problems": int(w.mesh.nproblems), "dof": int(dof), "solution_points": int(npts),
                   "rhs_per_step": 4, "dt": w.dt, "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "error_vs_fp64_oracle": errors.get("fp64"),
        "kernels": kernels,
        "points_per_s": value / s.nvars,
    }
    line.update(extra)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
