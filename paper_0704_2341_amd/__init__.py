"""MI355X (gfx950) library for the coarse Dirac operator S_bb = D_bb - D_br D_rr^{-1} D_rb
of a one-step gauged renormalisation-group blocking of Wilson fermions
(arXiv:0704.2341).  The compute lives in libgrg.so (HIP); this package is
its ctypes binding (``binding``) plus a small object wrapper (``api``).
"""
from .binding import *  # noqa: F401,F403
from .binding import GrgError, load  # noqa: F401
