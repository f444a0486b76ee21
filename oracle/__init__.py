"""FP64 CPU oracle for TILT via LADMAP with warm starts (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s
``cpu_baseline`` leg may import this package.  See ``tilt_oracle`` for what
it computes and which passages of the paper each step follows.
"""

from .tilt_oracle import *  # noqa: F401,F403
from . import tilt_oracle  # noqa: F401
from . import pyramid  # noqa: F401
from . import svdws  # noqa: F401
from . import rasl  # noqa: F401
