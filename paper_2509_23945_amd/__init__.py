"""MI355X-native TNMCMC-1 slice proposal (arXiv 2509.23945).

The compute lives in ``libtnmc.so`` (hand-written HIP kernels for gfx950 behind
the C ABI of ``include/tnmc.h``); ``api`` is a thin ctypes binding with the same
names.  Importing the package does not load the library; the first call does,
and fails loudly if it has not been built.
"""
from . import api  # noqa: F401
from .api import *  # noqa: F401,F403
