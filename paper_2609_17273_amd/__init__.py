"""MI355X (gfx950) line-list cross sections: Q(T), S_i and sigma(nu; T, P).

The computation runs in libxsec.so (hand-written HIP kernels behind the C-ABI
of include/xsec.h); this package is its Python binding.  See ``xsec``.
"""
from .xsec import *  # noqa: F401,F403
from .xsec import Plan, DeviceStates, DeviceLines, ChunkStreamer, XsecFunction, XsecError, lib  # noqa: F401
