"""Reduced HOSVD (canonical-to-Tucker rank reduction) for MI355X (gfx950).

The reduction runs in librhosvd.so (hand-written HIP kernels behind the C-ABI in
include/rhosvd.h); `rhosvd` is its ctypes binding and `inputs` builds seeded
synthetic canonical tensors.
"""
__version__ = "0.1.0"
