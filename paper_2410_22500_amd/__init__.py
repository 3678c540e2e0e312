"""MI355X-native hot path of fast hyperspectral neutron tomography (arXiv 2410.22500).

The computation lives in libhsn.so (hand-written HIP for gfx950, C ABI in
include/hsn.h).  `paper_2410_22500_amd.hsn` is the thin ctypes binding; it
raises on import when the library has not been built.
"""
__all__ = ["hsn", "build"]
