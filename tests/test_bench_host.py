"""Host-side checks of bench.py's contract that need no device: more than
one GPU is refused with a message, and the algorithmic byte model charges
each step's arrays once (against a hand count for the default workload)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_byte_model_of_the_fused_gradient_step():
    """Step 3 with steps 4 and 6 fused, TGV 16^3 p=3 FP64: C^f (96 flux points)
    and U (64 points) read per state column, S (9) and 1/J per point, Q and
    F~ (3 x 64 each) written per column."""
    sys.path.insert(0, ROOT)
    import bench

    class Blk:
        etype, order = "hex", 3

    class Mesh:
        blocks = [Blk()]

    class S:
        ndims, nvars, system = 3, 5, "ns"
        blocks = [dict(nelem=4096, nupts=64)]
        mesh = Mesh()
        nfpts = {("hex", 3): 96}
        nnz = {("hex", 3): dict(M0=384, M3=384, M4p=768, M6=384, M1p=1152)}
        fused_gradt = [True]
        fused_flux = [True]
        npairs = 0

    byts, _ = bench.step_model(S, 3, 8)
    cols, ne, nu = 5 * 4096, 4096, 64
    expect = cols * (96 + 64 + 3 * 64) * 8 + 10 * nu * ne * 8 + 3 * nu * cols * 8
    assert byts == expect
    assert abs(byts - 110100480) < 1          # the figure bench.py reports
    assert bench.step_model(S, 6, 8)[0] == 0   # step 6 costs nothing when fused


def test_byte_model_of_the_rk4_divergence_step():
    """The headline's dominant kernel, the divergence with the RK4 update of a
    middle stage (bench step 9), curved 48^3 p=4 FP64: D~ (150 flux points)
    and F~ (3 x 125 points) read per state column, 1/J per point, and four
    state arrays (u and the register read, the register and the next stage
    written): 4.645 GB per launch, the figure bench.py's roofline uses.
    Step 8 (-1/J only) writes du/dt instead of the four arrays."""
    sys.path.insert(0, ROOT)
    import bench

    class Blk:
        etype, order = "hex", 4

    class Mesh:
        blocks = [Blk()]

    class S:
        ndims, nvars, system = 3, 5, "euler"
        blocks = [dict(nelem=48 ** 3, nupts=125)]
        mesh = Mesh()
        nfpts = {("hex", 4): 150}
        nnz = {("hex", 4): dict(M0=750, M3=750, M4p=1875, M6=750, M1p=1875)}
        fused_gradt = [False]
        fused_flux = [False]
        npairs = 0

    ne, nu = 48 ** 3, 125
    cols = 5 * ne
    byts9, flops9 = bench.step_model(S, 9, 8)
    assert byts9 == cols * (150 + 3 * 125) * 8 + nu * ne * 8 + 4 * nu * cols * 8
    assert byts9 == 4644864000
    byts8, flops8 = bench.step_model(S, 8, 8)
    assert byts8 == byts9 - 3 * nu * cols * 8 and flops8 == flops9
    assert flops9 == 2.0 * (750 + 1875) * cols


def test_sample_holds_the_edge_elements():
    """The sampled elements always include element 0, the last element, one
    in the last 256-column tile and both sides of the first XCD tile-group
    boundary (2047, 2048), and are unique and in range."""
    sys.path.insert(0, ROOT)
    import numpy as np
    import bench
    for nelem in (110592, 4096, 300, 1):
        smp = bench.sample_elements(nelem, 12, 33)
        assert np.all(np.diff(smp) > 0) and smp[0] == 0 and smp[-1] == nelem - 1
        assert np.any(smp >= (nelem - 1) // 256 * 256)
        if nelem > 2048:
            assert 2047 in smp and 2048 in smp


def test_cpu_baseline_reference_is_the_oracle_on_the_sample():
    """On a small curved mesh the oracle's du/dt over the patch equals the
    full-mesh oracle's on the sampled elements, and the baseline reports the
    host it ran on."""
    sys.path.insert(0, ROOT)
    import numpy as np
    import bench
    from oracle import Discretisation
    from workloads import configs
    w = configs.curved_freestream_hexes(5, 2)
    cpu, ref = bench.cpu_baseline(w, 6, reps=1)
    d = Discretisation(w)
    full = d.rhs(d.initial_state(w))[0][:, :, ref["sample"]]
    assert np.abs(ref["rhs"] - full).max() <= 1e-13 * np.abs(full).max()
    assert cpu["value"] > 0 and cpu["nproc"] >= 1 and cpu["kind"] == "oracle"
    assert "patch" in cpu["sample"]
