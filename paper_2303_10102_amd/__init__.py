"""MI355X-native hierarchical-matrix maximum likelihood for physics-based covariances.

The compute path is the HIP library libhmle.so (C ABI in include/hmle.h);
`hmle` is its ctypes binding.  Nothing here falls back to the CPU.
"""
__all__ = ["hmle", "build"]
