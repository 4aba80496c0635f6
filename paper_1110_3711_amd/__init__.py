"""MI355X (gfx950) WCSPH particle-interaction hot path.

``paper_1110_3711_amd.sph`` is the ctypes binding of ``libsph.so`` (the C ABI
declared in ``include/sph.h``) and a small double-buffered driver.  The
library must be built first (``python -m paper_1110_3711_amd.build``); nothing
here falls back to a CPU implementation.
"""

__all__ = ["sph", "build"]
