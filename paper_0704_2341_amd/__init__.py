"""MI355X (gfx950) library for the coarse Dirac operator S_bb = D_bb - D_br D_rr^{-1} D_rb
of a one-step gauged renormalisation-group blocking of Wilson fermions
(arXiv:0704.2341).  The compute lives in libgrg.so (HIP); this package is
its ctypes binding (``binding``), which marshals arguments and does no
arithmetic; ``spectra`` computes eigenvalues of the small dense operators the
library assembles, and ``profiling`` summarises profiler output.
"""
from .binding import *  # noqa: F401,F403
from .binding import GrgError, load  # noqa: F401
