"""Storage rounding of control points -- oracle, test only.

Reduced-precision storage of the control points (FP32, BF16, FP16) with
FP32 arithmetic is this implementation's precision study; the paper does
not fix a storage precision.  Canonical control points are FP64; FP32
storage is the round-to-nearest-even (RNE) FP64 -> FP32 conversion, BF16
storage is that FP32 value rounded RNE to its upper 16 bits, and FP16
storage is that FP32 value rounded RNE to IEEE binary16 (11-bit
significand, subnormals below 2^-14).  ``dequant_*`` return the
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


def f16_bits(x: np.ndarray) -> np.ndarray:
    """uint16 IEEE binary16 encodings, RNE from the FP32 value (finite inputs
    whose rounded magnitude is at most 65504), by integer arithmetic on the
    FP32 encoding."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32)).reshape(-1)
    u = f.view(np.uint32).astype(np.int64)
    sign = (u >> 16) & 0x8000
    e32 = (u >> 23) & 0xFF
    man = u & 0x7FFFFF
    out = np.empty(u.shape, dtype=np.int64)
    e = e32 - 127 + 15                      # binary16 biased exponent
    norm = e >= 1
    # normal: keep 10 fraction bits, round the 13 dropped bits to nearest even
    half = (e << 10) | (man >> 13)
    rem = man & 0x1FFF
    up = (rem > 0x1000) | ((rem == 0x1000) & ((half & 1) == 1))
    out[norm] = (half + up)[norm]           # a carry may raise the exponent
    # subnormal (e <= 0): significand with its leading one, shifted right
    sub = ~norm
    if sub.any():
        m = (man | 0x800000)[sub]
        shift = (14 - e[sub]).astype(np.int64)
        shift_c = np.minimum(shift, 40)
        q = m >> shift_c
        r = m & ((np.int64(1) << shift_c) - 1)
        halfway = np.int64(1) << (shift_c - 1)
        upq = (r > halfway) | ((r == halfway) & ((q & 1) == 1))
        val = q + upq
        val[e32[sub] == 0] = 0              # FP32 zero (and FP32 subnormals: far below 2^-25)
        out[sub] = val
    return (sign | out).astype(np.uint16).reshape(np.shape(x))


def dequant_f16(x: np.ndarray) -> np.ndarray:
    return f16_bits(x).view(np.float16).astype(np.float64).reshape(np.shape(x))
