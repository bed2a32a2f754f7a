"""MI355X-native Gaussian-parameter hot path of GS-Scale-style 3DGS training.

The path (cull + ordered compaction, restoring gather, gradient scatter,
deferred Adam, flush) lives in the HIP library ``libgsdp.so`` behind the C ABI
declared in ``include/gsdp.h``; ``paper_2509_15645_amd.gsdp`` is its ctypes
binding.  Build with ``paper_2509_15645_amd.build.build()``.
"""
__all__ = ["build", "gsdp"]
