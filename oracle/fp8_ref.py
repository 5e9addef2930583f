"""FP8 E4M3FN decoding and per-block dequantisation in float64.

TEST INFRASTRUCTURE ONLY: not imported by the library.

Format (OCP 8-bit floating point, E4M3 "FN" variant): 1 sign bit, 4 exponent bits
with bias 7, 3 mantissa bits; no infinities; the two codes with all exponent and
mantissa bits set (0x7F, 0xFF) are NaN; exponent field 0 encodes subnormals
(mantissa / 8) * 2^-6. The largest finite magnitude is 1.75 * 2^8 = 448.

Precision pattern of the spec path: weights are FP8 codes with one FP32
scale per b x b block, and the value a block element stands for is
decode(code) * scale. Both factors are exact in float64, and so is the product
(at most 4 significant bits times 24 significant bits).
"""
import numpy as np


def decode_e4m3fn(codes):
    """float64 values of E4M3FN codes (any integer array of values 0..255)."""
    codes = np.asarray(codes, dtype=np.int64)
    shape = codes.shape
    codes = codes.reshape(-1)
    sign = np.where((codes >> 7) & 1, -1.0, 1.0)
    e = (codes >> 3) & 0xF
    f = codes & 0x7
    out = np.empty(codes.shape, dtype=np.float64)
    sub = e == 0
    out[sub] = (f[sub] / 8.0) * 2.0 ** -6
    nrm = ~sub
    out[nrm] = (1.0 + f[nrm] / 8.0) * np.power(2.0, (e[nrm] - 7).astype(np.float64))
    out = sign * out
    out[(e == 0xF) & (f == 0x7)] = np.nan
    return out.reshape(shape)


def dequantize_blocks(codes, scales):
    """V[z] = decode(codes[z]) * scales[z] for codes [nnz, b, b] and scales [nnz]."""
    codes = np.asarray(codes)
    scales = np.asarray(scales, dtype=np.float32).astype(np.float64)
    return decode_e4m3fn(codes) * scales.reshape(-1, 1, 1)
