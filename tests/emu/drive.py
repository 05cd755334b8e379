"""The library's host code with its sparse-row, matrix-core and
transformed-flux kernels emulated on the CPU under AddressSanitizer, on a
12-problem batched mesh (six element blocks): set-up (autotuner and the
multi-block tuning), a right-hand side and RK4 steps, then the one-launch
test's sequence (forced plans; launches per block, then one launch per kernel
family with one and with all fields per thread).  Any out-of-bounds access of
an emulated kernel or of the host code aborts with AddressSanitizer's report.

    bash tests/emu/build.sh /tmp/fr_emu
    ASAN_OPTIONS=detect_leaks=0 LD_PRELOAD=$(gcc -print-file-name=libasan.so) \
        python3 tests/emu/drive.py /tmp/fr_emu/libfr_emu.so fp64   # or fp32

EMU_SEED picks the emulated event times, hence the tuner's plans."""
import ctypes, os, sys
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import numpy as np
from paper_1312_1638_amd import binding as B
from workloads import configs

L = ctypes.CDLL(sys.argv[1])
vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
L.fr_setup_mesh.argtypes = [ctypes.POINTER(B.FrConfig), i32, ctypes.POINTER(B.FrBlock), i64, vp, vp,
                            ctypes.POINTER(vp)]
L.fr_get_layout.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32),
                            ctypes.POINTER(i32), ctypes.POINTER(i64)]
L.fr_rhs.argtypes = [vp, dp, dp, vp]
L.fr_rk_step.argtypes = [vp, dp, dp, i32, vp]
L.fr_debug_multi.argtypes = [vp, i32, i32, ctypes.POINTER(i32), vp]
L.fr_last_error.argtypes = [vp]; L.fr_last_error.restype = ctypes.c_char_p
prec = sys.argv[2] if len(sys.argv) > 2 else "fp64"
nprob = int(sys.argv[3]) if len(sys.argv) > 3 else 12
w = configs.batched_vortices(nprob, seed=11, nmax=300)
arr, pairs, keep = B._marshal_mesh(w.mesh)
cfg = B._config(2, "euler", prec, w.gamma, 0.0, 0.72, 0.5, 0.1, 0, nprob, autotune=True)
ctx = vp()
st = L.fr_setup_mesh(ctypes.byref(cfg), len(w.mesh.blocks), arr, len(pairs), pairs.ctypes.data, None,
                     ctypes.byref(ctx))
print("setup", st, L.fr_last_error(ctx if st == 0 else None), flush=True)
assert st == 0
for step in (1, 8, 6):
    s = i32()
    L.fr_debug_multi(ctx, step, -1, ctypes.byref(s), None)
    print("multi state step", step, s.value, flush=True)
off, ld, nu, nv, total = i64(), i64(), i32(), i32(), i64()
L.fr_get_layout(ctx, 0, ctypes.byref(off), ctypes.byref(ld), ctypes.byref(nu), ctypes.byref(nv),
                ctypes.byref(total))
n = total.value
rng = np.random.default_rng(3)
u = np.empty(n); u[:] = 1.0
for b in range(len(w.mesh.blocks)):
    L.fr_get_layout(ctx, b, ctypes.byref(off), ctypes.byref(ld), ctypes.byref(nu), ctypes.byref(nv), ctypes.byref(total))
    ne = w.mesh.blocks[b].nelem
    v = u[off.value: off.value + nu.value * nv.value * ld.value].reshape(nu.value, nv.value, ld.value)
    v[:, 0, :ne] = 1.0 + 0.1 * rng.random((nu.value, ne))
    v[:, 1, :ne] = 0.1 * rng.random((nu.value, ne))
    v[:, 2, :ne] = 0.1 * rng.random((nu.value, ne))
    v[:, 3, :ne] = 2.5 + 0.1 * rng.random((nu.value, ne))
dudt = np.zeros(n)
st = L.fr_rhs(ctx, u.ctypes.data, dudt.ctypes.data, None)
print("rhs", st, L.fr_last_error(ctx), "finite", np.isfinite(dudt).all(), flush=True)
dt = np.full(nprob, 1e-4)
st = L.fr_rk_step(ctx, u.ctypes.data, dt.ctypes.data, 3, None)
print("rk", st, L.fr_last_error(ctx), flush=True)
print("done")
# the one-launch test's sequence: forced plans, then each multi mode with a
# right-hand side and RK4 steps
L.fr_debug_set_plan.argtypes = [vp, i32, i32, i32, i32, i32, vp]
for bi, b in enumerate(w.mesh.blocks):
    for stp in (1, 8):
        plan = (1, 1, 1) if b.etype == "tri" else (0, 2, 0)
        st = L.fr_debug_set_plan(ctx, bi, stp, plan[0], plan[1], plan[2], None)
        assert st == 0, L.fr_last_error(ctx)
for mode in (0, 1, 2):
    states = []
    for stp in (1, 8, 6):
        s_ = i32()
        st = L.fr_debug_multi(ctx, stp, mode, ctypes.byref(s_), None)
        assert st == 0, L.fr_last_error(ctx)
        states.append(s_.value)
    st = L.fr_rhs(ctx, u.ctypes.data, dudt.ctypes.data, None)
    st2 = L.fr_rk_step(ctx, u.ctypes.data, dt.ctypes.data, 3, None)
    print("mode", mode, states, "rhs", st, "rk", st2, L.fr_last_error(ctx), flush=True)
print("modes done")
