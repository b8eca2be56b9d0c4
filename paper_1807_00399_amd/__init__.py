"""MI355X-native (gfx950) point-to-plane ICP hot path.

k-NN search, PCA normals and point-to-plane ICP run in hand-written HIP
kernels behind the C ABI of include/pcgpu.h; ``pcgpu`` is its ctypes
binding over torch device tensors.  Importing ``pcgpu`` fails loudly when
libpcgpu.so is not built.
"""
__all__ = ["pcgpu"]
