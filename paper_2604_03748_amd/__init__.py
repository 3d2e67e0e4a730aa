"""MI355X (gfx950) hot path of "Real-time Neural Six-way Lightmaps".

The work runs in liblnm.so (HIP kernels behind the C ABI of include/lnm.h);
``lnm`` is its ctypes binding.
"""
from . import lnm  # noqa: F401
