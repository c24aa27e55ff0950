"""Low-precision copies of X: BF16 and tile-scaled FP8-E4M3.

Test infrastructure (see ``oracle/__init__``).  Written from the number
formats' definitions (significand width, exponent range, round to nearest
with ties to even), with exact arithmetic in FP64 on the significand, so
that the result does not depend on any bit-manipulation trick.

The formats are not in the paper; they define the precision forms of the
filter product (X held in BF16, or in FP8 E4M3 with one FP32 scale per
128x128 tile).  Readings (not fixed by the paper):
  * BF16: round to nearest even, 8 significant bits, FP32 exponent range.
  * FP8: OCP E4M3FN (bias 7, max 448, no infinities), round to nearest
    even, saturating at +-448.  Per tile, scale = fp32(amax / 448) (1.0 for
    an all-zero tile) and code = e4m3(fp32(x / scale)) with IEEE FP32
    division, the same precision the device uses to take that decision.
"""
import numpy as np


def _round_sig(x, bits, min_normal_exp, sub_step_exp):
    """Round to nearest-even with ``bits`` significant bits; below
    2**min_normal_exp use the fixed subnormal step 2**sub_step_exp."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    finite = np.isfinite(x)
    out[~finite] = x[~finite]
    xf = x[finite]
    m, e = np.frexp(xf)                       # xf = m * 2**e, 0.5 <= |m| < 1
    normal = np.abs(xf) >= np.ldexp(1.0, min_normal_exp)
    r = np.empty_like(xf)
    # normal range: significand m*2**bits rounded half-to-even
    r[normal] = np.ldexp(np.round(np.ldexp(m[normal], bits)), e[normal] - bits)
    # subnormal range: multiples of 2**sub_step_exp
    r[~normal] = np.ldexp(np.round(np.ldexp(xf[~normal], -sub_step_exp)), sub_step_exp)
    out[finite] = r
    return out


BF16_MAX = float(np.ldexp(2.0 - 2.0 ** -7, 127))
E4M3_MAX = 448.0


def bf16_round(x):
    """Nearest BF16 value (ties to even), returned as float64.  Magnitudes
    that round above the largest finite BF16 become +-inf."""
    r = _round_sig(x, 8, -126, -133)
    big = np.isfinite(r) & (np.abs(r) > BF16_MAX)
    r[big] = np.copysign(np.inf, r[big])
    return r


def fp8_e4m3_round(x):
    """Nearest OCP E4M3FN value (ties to even), saturating to +-448."""
    r = _round_sig(x, 4, -6, -9)
    return np.clip(r, -E4M3_MAX, E4M3_MAX)


def fp8_tile_quantize(X, tile=128):
    """Per-tile FP8-E4M3 quantisation of an FP32 matrix.

    Returns (codes, scales): ``codes`` holds the E4M3 values (as float64,
    each exactly representable in E4M3) of fp32(x / scale) and ``scales``
    the FP32 per-tile scales, shape (ceil(m/tile), ceil(n/tile)).  Edge
    tiles cover the partial remainder.
    """
    X32 = np.asarray(X, dtype=np.float32)
    m, n = X32.shape
    tm, tn = -(-m // tile), -(-n // tile)
    scales = np.ones((tm, tn), dtype=np.float32)
    codes = np.zeros((m, n), dtype=np.float64)
    for I in range(tm):
        for J in range(tn):
            blk = X32[I * tile:(I + 1) * tile, J * tile:(J + 1) * tile]
            amax = np.float32(np.max(np.abs(blk))) if blk.size else np.float32(0)
            s = np.float32(amax / np.float32(448.0)) if amax > 0 else np.float32(1.0)
            scales[I, J] = s
            codes[I * tile:(I + 1) * tile, J * tile:(J + 1) * tile] = \
                fp8_e4m3_round((blk / s).astype(np.float32).astype(np.float64))
    return codes, scales


def fp8_tile_dequantize(codes, scales, tile=128):
    """Exact FP64 value code * scale of every element."""
    m, n = codes.shape
    S = np.repeat(np.repeat(scales.astype(np.float64), tile, axis=0), tile, axis=1)[:m, :n]
    return codes * S
