"""MI355X-native interaction phase of the Gadget3 method (arXiv 2003.10850).

SPH density with the smoothing-length solve, SPH hydro force and Barnes-Hut
gravity for the active particles, computed by hand-written HIP kernels for
gfx950 behind the C-ABI library ``libg3.so`` (declared in ``include/g3.h``).
``paper_2003_10850_amd.g3`` is the thin ctypes binding (same names as the
C entry points); ``paper_2003_10850_amd.ops`` wraps it for torch tensors.
The library is loaded on first use, so ``inputs`` imports without a GPU.
"""
