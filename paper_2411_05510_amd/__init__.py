"""MI355X-native SSI-COV identification with randomized SVD.

The compute path lives in libssicov.so (hand-written HIP kernels for gfx950,
C ABI in include/ssicov.h); `ssicov` is its thin ctypes binding and `synth`
draws seeded synthetic monitoring records.
"""
__all__ = ["ssicov", "synth"]
