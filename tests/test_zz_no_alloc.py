"""fr_integrate_noalloc (the integrals with the library's fixed scratch, for
callers that cannot allocate) against fr_integrate through the C ABI: two
calls in a row, the second on a smaller mesh, each bitwise equal to the
allocating entry point's result on the same state; and a mesh whose partials
exceed the fixed scratch is refused with an error."""
import ctypes

import numpy as np
import pytest

import frcases as C
from oracle import Discretisation
from workloads import configs

pytestmark = pytest.mark.gpu


def _state(w, s):
    d = Discretisation(w)
    return s.pack(C.perturbed(d, d.initial_state(w), seed=7))


def test_noalloc_integrals_match_twice_then_smaller():
    import torch
    import paper_1312_1638_amd as P
    cases = [configs.taylor_green_hexes(12, 3),     # 1728 elements, 27 slices of 64
             configs.vortex_quads(6, 3)]            # 36 elements, one slice
    for w in cases:
        s = C.solver_for(w)
        u = _state(w, s)
        ref = s.integrate(u)
        # a stale value in every output entry: the call must overwrite them all
        out = torch.full_like(ref, float("nan"))
        s.integrate_noalloc(u, out)
        torch.cuda.synchronize()
        print(f"{w.name}: {s.nproblems} problem(s), noalloc {out.cpu().numpy()[0]}")
        assert torch.equal(out, ref), (out, ref)
        # the same call again (the scratch holds the previous call's partials)
        out2 = torch.full_like(ref, float("nan"))
        s.integrate_noalloc(u, out2)
        torch.cuda.synchronize()
        assert torch.equal(out2, ref)
        s.close()


def test_noalloc_integrals_batched_problems():
    """Several problems of uneven size (per-problem element lists)."""
    import torch
    w = configs.batched_vortices(nproblems=6, nmin=50, nmax=400)
    s = C.solver_for(w)
    u = _state(w, s)
    ref = s.integrate(u)
    out = torch.full_like(ref, float("nan"))
    s.integrate_noalloc(u, out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    s.close()


def test_noalloc_refuses_a_mesh_beyond_the_fixed_scratch():
    """920 x 920 quads (p = 1): 846,400 elements x 5 partials exceed the
    4,194,304 doubles of the fixed scratch."""
    import paper_1312_1638_amd as P
    w = configs.vortex_quads(920, 1)
    s = P.Solver(w.mesh, system="euler", autotune=False)
    u = s.empty()
    import torch
    out = torch.empty((1, s.nvars + 1), dtype=torch.float64, device="cuda")
    with pytest.raises(P.FRError) as e:
        s.integrate_noalloc(u, out)
    assert "fixed scratch" in str(e.value)
    s.close()
