"""MI355X-native batched nested sampling (arXiv 2608.28514, BEST).

The sampler's hot path runs in hand-written HIP kernels behind the C ABI of
``include/ns.h`` (``libns.so``); ``paper_2608_28514_amd.native`` is the thin
ctypes binding with the same names.  Importing the package loads nothing.
"""
__all__ = ["native", "workloads", "mlp"]
