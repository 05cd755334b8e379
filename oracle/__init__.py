"""FP64 CPU oracle of the flux reconstruction right-hand side and RK4.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, direct restatement
of the paper's method (Witherden, Farrington & Vincent, "PyFR: an open source
framework for solving advection-diffusion type problems on streaming
architectures using the flux reconstruction approach", section 2 for the
scheme, section 4 and Appendices B for the physics).  It exists to check the
HIP library: only the test-suite, the smoke entry point and the CPU-baseline
leg of the benchmark may import it.  It shares no code, tables or constants
with the library; both only consume the seeded inputs of ``workloads``.

Every function here is written in the paper's order and notation, in FP64
(long double where a linear solve needs headroom), with numpy library
primitives (einsum contractions, a dense solve) as the only building blocks.
"""
from .rhs import Discretisation, jvp, rk4_jvp  # noqa: F401
