"""MI355X-native QTB / QTB-PIMD integrator step (arXiv:1905.02521).

The hot path lives in ``libqtb.so`` (hand-written HIP for gfx950 behind a C
ABI declared in ``include/qtb.h``).  ``paper_1905_02521_amd.qtb`` is the thin
ctypes binding; importing this package does not load the library.
"""
__all__ = ["qtb", "workloads"]
