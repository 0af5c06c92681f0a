"""FP64 CPU oracle of plain Levenberg-Marquardt and Stochastic Bundle Adjustment.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the GPU library never does, and
this package shares no code with it.
"""
from .stba_oracle import *  # noqa: F401,F403
from .stba_oracle import __all__  # noqa: F401
