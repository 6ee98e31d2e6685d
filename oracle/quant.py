"""Storage rounding of control points -- oracle, test only.

Reduced-precision storage of the control points (FP32, BF16) with FP32
arithmetic is this implementation's precision study; the paper does not fix
a storage precision.  Canonical control points are FP64; FP32 storage is the
round-to-nearest-even (RNE) FP64 -> FP32 conversion, BF16 storage is that
FP32 value rounded RNE to its upper 16 bits.  ``dequant_*`` return the
stored value exactly, as FP64, so that an FP64 evaluation of the stored
model separates storage error from arithmetic error.
"""

import numpy as np


def dequant_f32(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """uint16 BF16 encodings (RNE from the FP32 value; finite inputs)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    b = b + np.uint64(0x7FFF) + lsb
    return ((b >> np.uint64(16)) & np.uint64(0xFFFF)).astype(np.uint16)


def dequant_bf16(x: np.ndarray) -> np.ndarray:
    bits = bf16_bits(x).astype(np.uint32) << np.uint32(16)
    return bits.view(np.float32).astype(np.float64).reshape(np.shape(x))
