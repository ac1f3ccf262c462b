"""MI355X-native 3D Gaussian Splatting training hot path (HIP, gfx950).

The compute lives in ``libgs.so`` (hand-written HIP kernels behind the C ABI
of ``include/gs.h``); ``_lib`` is its ctypes binding and ``pipeline`` the
buffer management and training step.  Importing ``pipeline`` requires the
built library; there is no CPU fallback.
"""
__all__ = ["pipeline", "autograd", "schedule", "autotune"]
