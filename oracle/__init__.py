"""FP64 CPU oracle of the SHMM hot path (Lee & Engquist, seamless heterogeneous
multiscale method for passive advection-diffusion).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the HIP path is compared against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with ``paper_1510_00451_amd`` (neither imports
the other); both read their inputs from ``flowgen``, which holds none of the
method's arithmetic.

Every function cites the passage of the paper it follows, and every one is
pinned to something other than itself in tests/test_oracle_pins.py and
tests/test_oracle_surrogate.py (a function without such a pin would say
"parity unpinned" in its docstring; none does).
"""
from .core import *  # noqa: F401,F403
