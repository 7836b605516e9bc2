"""MI355X (gfx950) BP-SF decoder: HIP kernels behind a C ABI (include/bpsf.h).

``paper_2507_00254_amd.bpsf`` is the Python binding; importing it loads
``libbpsf.so`` and fails loudly if the library has not been built.
"""
