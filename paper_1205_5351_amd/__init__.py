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
    load_tuning,
    peak_probe,
    svt_layout,
    svt_layouts,
    svt_batch_noalloc,
    tune_clear,
    tune_set,
)

import os as _os

# Measured Jacobi layouts for this GPU (written by autotune.py); set
# TILT_NO_TUNING=1 to use the built-in cost model only.
TUNING_TABLE = _os.path.join(_os.path.dirname(_os.path.abspath(__file__)), "tuning", "mi355x_svt_layouts.json")
if _os.path.exists(TUNING_TABLE) and not _os.environ.get("TILT_NO_TUNING"):
    load_tuning(TUNING_TABLE)
