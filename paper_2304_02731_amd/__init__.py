"""MI355X-native quasi-classical trajectory (QCT) hot path.

HIP kernels for gfx950 behind the C ABI of include/qcams.h (libqcams.so),
with a thin ctypes binding.  Koots & Perez-Rios, arXiv:2304.02731.
"""
from .qcams import *  # noqa: F401,F403
from .qcams import Context, QcamsError, lib  # noqa: F401
