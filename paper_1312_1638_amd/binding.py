"""ctypes binding of libfr.so (argument marshalling only).

Every step of the right-hand side runs in the HIP library; this module only
converts meshes into the C structures of ``include/fr.h``, hands device
pointers and the current torch stream to the library, and raises
:class:`FRError` on a non-zero status.  Torch provides device memory and
streams.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libfr.so")

FR_OK, FR_EINVAL, FR_EMESH, FR_EUNSUPPORTED, FR_ENOMEM, FR_EDEVICE, FR_ENONFINITE = range(7)
ETYPE = {"quad": 0, "tri": 1, "hex": 2}
SYSTEM = {"euler": 0, "ns": 1}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}

EXPORTS = ("fr_setup_mesh", "fr_setup_mesh_bc", "fr_get_layout", "fr_get_solution_points", "fr_get_quadrature",
           "fr_rhs", "fr_rk_step", "fr_euler_step", "fr_dopri5_step", "fr_rhs_adjoint", "fr_rk_step_adjoint", "fr_integrate", "fr_integrate_noalloc",
           "fr_reference_operator", "fr_check_mesh", "fr_debug_stage", "fr_debug_scratch_len", "fr_bench_step",
           "fr_debug_gemm", "fr_measure_ceiling", "fr_bench_gemm", "fr_get_gemm_plan", "fr_integrate_grad", "fr_stash_len", "fr_rk_step_stash",
           "fr_rk_step_adjoint_stash", "fr_rk_segment_adjoint", "fr_debug_set_plan", "fr_debug_multi",
           "fr_last_error", "fr_destroy")


class FRError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fr status {status}: {msg}")
        self.status = status


class FrConfig(ctypes.Structure):
    _fields_ = [("ndims", ctypes.c_int32), ("system", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("check_finite", ctypes.c_int32), ("gamma", ctypes.c_double),
                ("mu", ctypes.c_double), ("prandtl", ctypes.c_double),
                ("ldg_beta", ctypes.c_double), ("ldg_tau", ctypes.c_double),
                ("nproblems", ctypes.c_int32), ("autotune", ctypes.c_int32)]


class FrBlock(ctypes.Structure):
    _fields_ = [("etype", ctypes.c_int32), ("order", ctypes.c_int32),
                ("geom_order", ctypes.c_int32), ("correction", ctypes.c_int32),
                ("nelem", ctypes.c_int64), ("nodes", ctypes.c_void_p),
                ("problem", ctypes.c_void_p)]


# numpy view of fr_facepair (natural C alignment, 56 bytes)
# fr_bc and fr_bcface (include/fr.h)
BC_C = np.dtype([("type", "<i4"), ("reserved", "<i4"), ("rho", "<f8"), ("v", "<f8", (3,)),
                 ("p", "<f8"), ("cp_tw", "<f8"), ("vw", "<f8", (3,))], align=True)
BCFACE_C = np.dtype([("block", "<i4"), ("face", "<i4"), ("elem", "<i8"), ("bc", "<i4"),
                     ("reserved", "<i4")], align=True)
BCTYPE = {"supersonic-inflow": 0, "subsonic-outflow": 1, "no-slip-isothermal-wall": 2}
CORRECTION = {"dg": 0, "sd": 1, "hu": 2}      # fr_correction

FACEPAIR_C = np.dtype([("lblock", "<i4"), ("lface", "<i4"), ("lelem", "<i8"),
                       ("rblock", "<i4"), ("rface", "<i4"), ("relem", "<i8"),
                       ("shift", "<f8", (3,))], align=True)

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfr.so; raises FileNotFoundError if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} not built: run paper_1312_1638_amd.build.build()")
    L = ctypes.CDLL(path)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    sig = {
        "fr_setup_mesh_bc": [ctypes.POINTER(FrConfig), i32, ctypes.POINTER(FrBlock), i64, vp, i32,
                             vp, i64, vp, vp, ctypes.POINTER(vp)],
        "fr_setup_mesh": [ctypes.POINTER(FrConfig), i32, ctypes.POINTER(FrBlock), i64, vp, vp,
                          ctypes.POINTER(vp)],
        "fr_get_layout": [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i64),
                          ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i64)],
        "fr_get_solution_points": [vp, i32, dp],
        "fr_get_quadrature": [vp, i32, dp],
        "fr_rhs": [vp, dp, dp, vp],
        "fr_rk_step": [vp, dp, dp, i32, vp],
        "fr_euler_step": [vp, dp, dp, i32, vp],
        "fr_dopri5_step": [vp, dp, dp, dp, dp, i32, ctypes.c_double, ctypes.c_double, vp, vp],
        "fr_rhs_adjoint": [vp, dp, dp, dp, vp],
        "fr_rk_step_adjoint": [vp, dp, dp, dp, dp, vp],
        "fr_integrate": [vp, dp, i32, dp, vp],
        "fr_integrate_noalloc": [vp, dp, i32, dp, vp],
        "fr_integrate_grad": [vp, dp, i32, dp, vp],
        "fr_stash_len": [vp, ctypes.POINTER(i64)],
        "fr_rk_step_stash": [vp, dp, dp, dp, vp],
        "fr_rk_step_adjoint_stash": [vp, dp, dp, dp, dp, vp],
        "fr_rk_segment_adjoint": [vp, dp, dp, i32, dp, dp, dp, vp],
        "fr_reference_operator": [i32, i32, i32, i32, dp, i64, ctypes.POINTER(i32),
                                  ctypes.POINTER(i32)],
        "fr_check_mesh": [ctypes.POINTER(FrConfig), i32, ctypes.POINTER(FrBlock), i64, vp,
                          ctypes.POINTER(i64)],
        "fr_debug_stage": [vp, dp, i32, dp, vp],
        "fr_debug_scratch_len": [vp, i32, ctypes.POINTER(i64)],
        "fr_bench_step": [vp, dp, i32, i32, vp],
        "fr_measure_ceiling": [i32, ctypes.POINTER(ctypes.c_double), vp],
        "fr_bench_gemm": [i32, i32, i32, i32, i64, i32, i32, i32, i32, i32,
                          ctypes.POINTER(ctypes.c_float), vp],
        "fr_get_gemm_plan": [vp, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                             ctypes.POINTER(i32)],
        "fr_debug_gemm": [i32, i32, i32, i32, dp, dp, dp, i64, dp, i64, i32, i32, i32, vp],
        "fr_debug_set_plan": [vp, i32, i32, i32, i32, i32, vp],
        "fr_debug_multi": [vp, i32, i32, ctypes.POINTER(i32), vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.fr_last_error.argtypes = [vp]
    L.fr_last_error.restype = ctypes.c_char_p
    L.fr_destroy.argtypes = [vp]
    L.fr_destroy.restype = None
    _lib = L
    return L


def _check(st, ctx=None):
    if st != FR_OK:
        msg = load_library().fr_last_error(ctx).decode()
        raise FRError(st, msg)


def reference_operator(etype: str, order: int, which: int, correction: str = "dg") -> np.ndarray:
    """Host-side reference operator of the library (no device needed)."""
    L = load_library()
    r, c = ctypes.c_int32(), ctypes.c_int32()
    k = CORRECTION[correction]
    _check(L.fr_reference_operator(ETYPE[etype], order, k, which, None, 0, ctypes.byref(r),
                                   ctypes.byref(c)))
    out = np.empty((r.value, c.value))
    _check(L.fr_reference_operator(ETYPE[etype], order, k, which, out.ctypes.data, out.size,
                                   ctypes.byref(r), ctypes.byref(c)))
    return out


def debug_gemm(A, B1, B2=None, prec="fp64", plan=(0, 0, 0)):
    """C = A [B1; B2] on the matrix cores (A host numpy, B device float64)."""
    import torch
    L = load_library()
    M = A.shape[0]
    K1 = B1.shape[0]
    K2 = 0 if B2 is None else B2.shape[0]
    N = B1.shape[1]
    A = np.ascontiguousarray(A, dtype=np.float64)
    C = torch.zeros((M, N), dtype=torch.float64 if prec == "fp64" else torch.float32,
                    device="cuda")
    _check(L.fr_debug_gemm(PREC[prec], M, K1, K2, A.ctypes.data, B1.data_ptr(),
                           None if B2 is None else B2.data_ptr(), B1.stride(0), C.data_ptr(),
                           N, plan[0], plan[1], plan[2], torch.cuda.current_stream().cuda_stream))
    return C


def measure_ceiling(kind):
    """0: HBM triad GB/s, 1: FP64 MFMA TFLOP/s, 2: FP32 MFMA TFLOP/s (measured)."""
    import torch
    v = ctypes.c_double()
    _check(load_library().fr_measure_ceiling(kind, ctypes.byref(v),
                                             torch.cuda.current_stream().cuda_stream))
    return v.value


def bench_gemm(prec, M, K1, K2, N, plan=(0, 0, 0), batch=1, nrep=20):
    """Milliseconds per launch of the operator GEMM kernel."""
    import torch
    ms = ctypes.c_float()
    _check(load_library().fr_bench_gemm(PREC[prec], M, K1, K2, N, plan[0], plan[1], plan[2],
                                        batch, nrep, ctypes.byref(ms),
                                        torch.cuda.current_stream().cuda_stream))
    return ms.value


def _config(ndims, system, prec, gamma, mu, prandtl, beta, tau, check_finite, nproblems,
            autotune=False):
    return FrConfig(ndims, SYSTEM[system], PREC[prec], int(check_finite), gamma, mu, prandtl,
                    beta, tau, nproblems, int(autotune))


def _marshal_mesh(mesh):
    """C arrays for the mesh; returns (blocks array, pairs array, keep-alive list)."""
    keep = []
    arr = (FrBlock * len(mesh.blocks))()
    for i, b in enumerate(mesh.blocks):
        nodes = np.ascontiguousarray(b.nodes, dtype=np.float64)
        keep.append(nodes)
        prob = None
        if b.problem is not None:
            prob = np.ascontiguousarray(b.problem, dtype=np.int32)
            keep.append(prob)
        corr = CORRECTION[getattr(b, "correction", "dg")]
        arr[i] = FrBlock(ETYPE[b.etype], b.order, b.geom_order, corr, b.nelem, nodes.ctypes.data,
                         prob.ctypes.data if prob is not None else None)
    src = mesh.pairs
    pairs = np.zeros(len(src), dtype=FACEPAIR_C)
    for f in FACEPAIR_C.names:
        pairs[f] = src[f]
    keep.append(pairs)
    return arr, pairs, keep


def _marshal_bcs(mesh):
    """mesh.bcs (dicts: type and parameters) and mesh.bcfaces (block, elem,
    face, bc records) -> fr_bc and fr_bcface arrays."""
    bcs = np.zeros(len(mesh.bcs), dtype=BC_C)
    for k, b in enumerate(mesh.bcs):
        bcs[k]["type"] = BCTYPE[b["type"]]
        bcs[k]["rho"] = b.get("rho", 0.0)
        bcs[k]["v"] = list(b.get("v", (0.0, 0.0, 0.0))) + [0.0] * (3 - len(b.get("v", (0.0, 0.0, 0.0))))
        bcs[k]["p"] = b.get("p", 0.0)
        bcs[k]["cp_tw"] = b.get("cp_tw", 0.0)
        vw = list(b.get("vw", (0.0, 0.0, 0.0)))
        bcs[k]["vw"] = vw + [0.0] * (3 - len(vw))
    f = mesh.bcfaces
    faces = np.zeros(len(f), dtype=BCFACE_C)
    for name in ("block", "face", "elem", "bc"):
        faces[name] = f[name]
    return bcs, faces


def check_mesh(mesh, system="euler") -> int:
    """Run the library's host set-up (metrics + pairing); returns the number of
    flux-point pairs or raises FRError."""
    L = load_library()
    arr, pairs, keep = _marshal_mesh(mesh)
    cfg = _config(mesh.ndims, system, "fp64", 1.4, 0.0, 0.72, 0.5, 0.1, 0, 1)
    n = ctypes.c_int64()
    _check(L.fr_check_mesh(ctypes.byref(cfg), len(mesh.blocks), arr, len(pairs),
                           pairs.ctypes.data, ctypes.byref(n)))
    return n.value


class Solver:
    """One FR discretisation on the GPU (a context of the library).

    The state is a float64 CUDA tensor of length ``total_len`` in the public
    layout; :meth:`pack` / :meth:`unpack` convert from/to per-block numpy
    arrays indexed [rho, alpha, n].
    """

    def __init__(self, mesh, system="euler", gamma=1.4, mu=0.0, prandtl=0.72,
                 ldg_beta=0.5, ldg_tau=0.1, prec="fp64", check_finite=False,
                 nproblems=None, autotune=True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the FR library needs a HIP device")
        self.torch = torch
        L = self.L = load_library()
        self.mesh = mesh
        self.ndims = mesh.ndims
        self.nvars = mesh.ndims + 2
        self.nproblems = nproblems or getattr(mesh, "nproblems", 1)
        self.prec = prec
        cfg = _config(mesh.ndims, system, prec, gamma, mu, prandtl, ldg_beta, ldg_tau,
                      check_finite, self.nproblems, autotune)
        arr, pairs, keep = _marshal_mesh(mesh)
        ctx = ctypes.c_void_p()
        stream = torch.cuda.current_stream().cuda_stream
        bcfaces = getattr(mesh, "bcfaces", None)
        if bcfaces is not None and len(bcfaces):
            bcs, faces = _marshal_bcs(mesh)
            _check(L.fr_setup_mesh_bc(ctypes.byref(cfg), len(mesh.blocks), arr, len(pairs),
                                      pairs.ctypes.data, len(bcs), bcs.ctypes.data, len(faces),
                                      faces.ctypes.data, stream, ctypes.byref(ctx)))
        else:
            _check(L.fr_setup_mesh(ctypes.byref(cfg), len(mesh.blocks), arr, len(pairs),
                                   pairs.ctypes.data, stream, ctypes.byref(ctx)))
        self.ctx = ctx
        self.blocks = []
        for b in range(len(mesh.blocks)):
            off, ld, total = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
            nu, nv = ctypes.c_int32(), ctypes.c_int32()
            _check(L.fr_get_layout(ctx, b, ctypes.byref(off), ctypes.byref(ld), ctypes.byref(nu),
                                   ctypes.byref(nv), ctypes.byref(total)), ctx)
            self.blocks.append(dict(offset=off.value, ld=ld.value, nupts=nu.value,
                                    nelem=mesh.blocks[b].nelem))
            self.total_len = total.value
        self._dt_cache = None

    # -- layout ---------------------------------------------------------------
    def solution_points(self, b):
        blk = self.blocks[b]
        out = np.empty((blk["nelem"], blk["nupts"], self.ndims))
        _check(self.L.fr_get_solution_points(self.ctx, b, out.ctypes.data), self.ctx)
        return out

    def quadrature(self, b):
        blk = self.blocks[b]
        out = np.empty((blk["nupts"], blk["nelem"]))
        _check(self.L.fr_get_quadrature(self.ctx, b, out.ctypes.data), self.ctx)
        return out

    def empty(self):
        return self.torch.zeros(self.total_len, dtype=self.torch.float64, device="cuda")

    def adjoint_state(self):
        """A second solver-owned state buffer at a fixed address (the
        cotangent of the checkpointed adjoint), like graph_state."""
        if getattr(self, "_adjoint_state", None) is None:
            self._adjoint_state = self.empty()
        return self._adjoint_state

    def graph_state(self):
        """A state buffer owned by the solver, at one address for its life: the
        library keeps the step graph captured for the state it last stepped,
        so stepping this buffer again reuses the graph."""
        if getattr(self, "_graph_state", None) is None:
            self._graph_state = self.empty()
        return self._graph_state

    def pack(self, arrays):
        """Per-block arrays [rho, alpha, n] -> device state tensor."""
        host = np.zeros(self.total_len)
        for blk, a in zip(self.blocks, arrays):
            nu, ld, ne = blk["nupts"], blk["ld"], blk["nelem"]
            view = host[blk["offset"]:blk["offset"] + nu * self.nvars * ld].reshape(nu, self.nvars, ld)
            view[:, :, :ne] = a
        return self.torch.from_numpy(host).to("cuda")

    def unpack(self, t):
        host = t.detach().to("cpu").numpy()
        out = []
        for blk in self.blocks:
            nu, ld, ne = blk["nupts"], blk["ld"], blk["nelem"]
            view = host[blk["offset"]:blk["offset"] + nu * self.nvars * ld].reshape(nu, self.nvars, ld)
            out.append(view[:, :, :ne].copy())
        return out

    # -- the hot path -----------------------------------------------------------
    def _stream(self):
        return self.torch.cuda.current_stream().cuda_stream

    def _ptr(self, t):
        assert t.dtype == self.torch.float64 and t.is_cuda and t.is_contiguous()
        assert t.numel() >= self.total_len
        return t.data_ptr()

    def rhs(self, u, out=None):
        if out is None:
            out = self.empty()
        _check(self.L.fr_rhs(self.ctx, self._ptr(u), self._ptr(out), self._stream()), self.ctx)
        return out

    def dt_tensor(self, dt):
        if isinstance(dt, (int, float)):
            if self._dt_cache is None or self._dt_cache[0] != dt:
                t = self.torch.full((self.nproblems,), float(dt), dtype=self.torch.float64,
                                    device="cuda")
                self._dt_cache = (dt, t)
            return self._dt_cache[1]
        return dt

    def step(self, u, dt, nsteps=1):
        """nsteps RK4 steps in place on u (dt: float or device tensor [nproblems])."""
        d = self.dt_tensor(dt)
        assert d.dtype == self.torch.float64 and d.is_cuda and d.numel() >= self.nproblems
        _check(self.L.fr_rk_step(self.ctx, self._ptr(u), d.data_ptr(), nsteps, self._stream()),
               self.ctx)
        return u

    def euler_step(self, u, dt, nsteps=1):
        """nsteps forward Euler steps in place on u (dt as for step)."""
        d = self.dt_tensor(dt)
        assert d.dtype == self.torch.float64 and d.is_cuda and d.numel() >= self.nproblems
        _check(self.L.fr_euler_step(self.ctx, self._ptr(u), d.data_ptr(), nsteps, self._stream()),
               self.ctx)
        return u

    def dopri5(self, u, t, dt, nattempts, atol, rtol, tend=None, counts=None):
        """nattempts adaptive DOPRI5 attempts in place on u.  t, dt (and tend):
        device float64 tensors [nproblems], updated in place; counts: device
        int32 [nproblems, 2] (accepted, rejected attempts added) or None."""
        T = self.torch
        for a in (t, dt) + ((tend,) if tend is not None else ()):
            assert a.dtype == T.float64 and a.is_cuda and a.is_contiguous()
            assert a.numel() >= self.nproblems
        if counts is not None:
            assert counts.dtype == T.int32 and counts.is_cuda and counts.is_contiguous()
            assert counts.numel() >= 2 * self.nproblems
        _check(self.L.fr_dopri5_step(self.ctx, self._ptr(u), t.data_ptr(), dt.data_ptr(),
                                     tend.data_ptr() if tend is not None else None, nattempts,
                                     float(atol), float(rtol),
                                     counts.data_ptr() if counts is not None else None,
                                     self._stream()), self.ctx)
        return u

    def rhs_adjoint(self, u, lam, out=None):
        if out is None:
            out = self.empty()
        _check(self.L.fr_rhs_adjoint(self.ctx, self._ptr(u), self._ptr(lam), self._ptr(out),
                                     self._stream()), self.ctx)
        return out

    def rk_step_adjoint(self, u, dt, lam, out=None):
        if out is None:
            out = self.empty()
        d = self.dt_tensor(dt)
        _check(self.L.fr_rk_step_adjoint(self.ctx, self._ptr(u), d.data_ptr(), self._ptr(lam),
                                         self._ptr(out), self._stream()), self.ctx)
        return out

    def debug_stage(self, u, stage):
        """Internal array after right-hand-side step `stage` (FP64 contexts)."""
        n = ctypes.c_int64()
        _check(self.L.fr_debug_scratch_len(self.ctx, stage, ctypes.byref(n)), self.ctx)
        out = self.torch.zeros(n.value, dtype=self.torch.float64, device="cuda")
        _check(self.L.fr_debug_stage(self.ctx, self._ptr(u), stage, out.data_ptr(),
                                     self._stream()), self.ctx)
        return out

    def bench_step(self, u, step, nrep):
        """Launch right-hand-side step `step` nrep times (after preparing its
        inputs) on the current stream; for kernel timing."""
        _check(self.L.fr_bench_step(self.ctx, self._ptr(u), step, nrep, self._stream()), self.ctx)

    def stash_len(self):
        n = ctypes.c_int64()
        _check(self.L.fr_stash_len(self.ctx, ctypes.byref(n)), self.ctx)
        return n.value

    def step_stash(self, u, dt, stash):
        """One RK4 step in place on u, keeping stage states and intermediates."""
        d = self.dt_tensor(dt)
        assert stash.dtype == self.torch.float64 and stash.numel() >= self.stash_len()
        _check(self.L.fr_rk_step_stash(self.ctx, self._ptr(u), d.data_ptr(), stash.data_ptr(),
                                       self._stream()), self.ctx)
        return u

    def rk_step_adjoint_stash(self, stash, dt, lam, out=None):
        if out is None:
            out = self.empty()
        d = self.dt_tensor(dt)
        _check(self.L.fr_rk_step_adjoint_stash(self.ctx, stash.data_ptr(), d.data_ptr(),
                                               self._ptr(lam), self._ptr(out), self._stream()),
               self.ctx)
        return out

    def segment_adjoint(self, u0, dt, nsteps, lam, stash, out=None):
        """(d u_{nsteps} / d u0)^T lam through a replay of nsteps steps from
        u0 stashed into `stash` (nsteps * stash_len float64), as one graph."""
        if out is None:
            out = self.empty()
        d = self.dt_tensor(dt)
        assert stash.dtype == self.torch.float64 and stash.numel() >= nsteps * self.stash_len()
        _check(self.L.fr_rk_segment_adjoint(self.ctx, self._ptr(u0), d.data_ptr(), nsteps,
                                            self._ptr(lam), self._ptr(out), stash.data_ptr(),
                                            self._stream()), self.ctx)
        return out

    def kinetic_energy_grad(self, u, out=None):
        """d(sum of kinetic energy integrals)/du, state layout."""
        if out is None:
            out = self.empty()
        _check(self.L.fr_integrate_grad(self.ctx, self._ptr(u), 1, self._ptr(out), self._stream()),
               self.ctx)
        return out

    def gemm_plan(self, block, step):
        m, n, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self.L.fr_get_gemm_plan(self.ctx, block, step, ctypes.byref(m), ctypes.byref(n),
                                       ctypes.byref(w)), self.ctx)
        return (m.value, n.value, w.value)

    def set_plan(self, block, step, plan):
        """Force the (mbw, nc, wm) plan of RHS step 1, 3, 5 or 8 of a block."""
        _check(self.L.fr_debug_set_plan(self.ctx, block, step, plan[0], plan[1], plan[2],
                                        self._stream()), self.ctx)

    def multi(self, step, mode=-1):
        """Multi-block launches of step 1, 5, 6 or 8: bit 0 sparse-row over
        several blocks, bit 1 matrix cores over several blocks, bit 2 (step
        6) the one-launch transformed flux.  mode >= 0 sets them first (0 a
        launch per block, 1 / 2 one launch per kernel family)."""
        st = ctypes.c_int32()
        _check(self.L.fr_debug_multi(self.ctx, step, mode, ctypes.byref(st), self._stream()),
               self.ctx)
        return st.value

    def integrate(self, u):
        """[nproblems, nvars + 1]: integral of every field, then kinetic energy.
        Every entry is written by the library (no zero fill needed)."""
        out = self.torch.empty((self.nproblems, self.nvars + 1), dtype=self.torch.float64,
                               device="cuda")
        _check(self.L.fr_integrate(self.ctx, self._ptr(u), 0, out.data_ptr(), self._stream()),
               self.ctx)
        return out

    def integrate_noalloc(self, u, out):
        """As integrate, into the caller's `out` [nproblems, nvars + 1], with
        the library's fixed scratch: the call allocates nothing."""
        assert out.dtype == self.torch.float64 and out.is_cuda
        assert out.numel() >= self.nproblems * (self.nvars + 1)
        _check(self.L.fr_integrate_noalloc(self.ctx, self._ptr(u), 0, out.data_ptr(),
                                           self._stream()), self.ctx)
        return out

    def close(self):
        if getattr(self, "ctx", None):
            self.L.fr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
