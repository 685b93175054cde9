"""MI355X-native supernodal sparse Cholesky (the factorization hot path of
Lacoste et al., "Taking advantage of hybrid systems for sparse direct
solvers via task-based runtimes").

The work is done by the native library ``libspx.so`` (C ABI in
``include/spx.h``: HIP kernels for gfx950 and the C++ symbolic analysis);
this package only marshals arguments.  Build it with
``python -m paper_1405_2636_amd._build``.
"""
from .spx import (  # noqa: F401
    Solver,
    SpxError,
    NotPositiveDefinite,
    NotConverged,
    load_library,
    solve_autograd,
    SYMBOLIC_FIELDS,
)
