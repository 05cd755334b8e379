"""MI355X-native flux reconstruction right-hand side (HIP library + binding).

The compute path is ``_lib/libfr.so`` (built by :mod:`.build`); this package
only marshals arguments to it.  Importing the package does not need a GPU;
creating a :class:`Solver` does, and fails loudly if the library is missing.
"""
from .binding import (FRError, Solver, check_mesh, load_library,  # noqa: F401
                      reference_operator)
