"""MI355X-native TILT solver: LADMAP with adaptive penalty and warm starts.

The solver is the HIP library ``libtilt.so`` (built from ``csrc/`` for
gfx950, interface in ``include/tilt.h``); this package is its thin ctypes
binding.  Importing it fails loudly when the library has not been built.
"""

from .tilt import (  # noqa: F401
    AFFINE,
    PROJECTIVE,
    Context,
    Params,
    Problem,
    Result,
    TiltError,
    default_params,
    make_problem,
    solve,
    status_string,
    tau_from_quad,
    version,
    workspace_bytes,
    EXPORTS,
    LIB_PATH,
)
