"""FP64 CPU oracle for the Matsubara-time GW hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The HIP
library never calls it, shares no code with it and is never checked against
anything it did not compute itself.

Every function follows a passage of Chu et al., "All-electron self-consistent
GW in the Matsubara-time domain" (arXiv:1602.02313), cited in its docstring.
"""
from .gw import *  # noqa: F401,F403
from .continuation import *  # noqa: F401,F403
