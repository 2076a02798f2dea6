"""MI355X-native Tensor Monte Carlo chain estimator (arXiv 1806.08593).

The estimator runs in libtmc.so (hand-written HIP kernels for gfx950 behind the C
ABI of include/tmc.h).  `tmc` is the ctypes binding, `autograd` the torch wrapper.
"""
__all__ = ["tmc", "autograd"]
