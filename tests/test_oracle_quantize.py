"""Pins of the oracle's BF16 / FP8-E4M3 quantisers (CPU).

References: brute-force nearest search over every E4M3 code decoded from
its bit pattern, torch's own float -> bfloat16 / float8_e4m3fn casts (an
independent implementation of round-to-nearest-even), and exact ties.
"""
import numpy as np
import pytest
import torch

import oracle


def e4m3_values():
    """All finite OCP E4M3FN values, decoded from the 8-bit patterns."""
    vals = []
    for code in range(256):
        s = -1.0 if code & 0x80 else 1.0
        E = (code >> 3) & 0xF
        M = code & 7
        if E == 0xF and M == 7:
            continue                                   # NaN encodings
        v = (M / 8.0) * 2.0 ** -6 if E == 0 else (1 + M / 8.0) * 2.0 ** (E - 7)
        vals.append(s * v)
    return np.unique(np.array(vals))


def test_e4m3_brute_force_nearest():
    grid = e4m3_values()
    assert grid.max() == 448.0 and np.min(grid[grid > 0]) == 2.0 ** -9
    x = np.concatenate([np.random.default_rng(0).uniform(-460, 460, 4000),
                        np.random.default_rng(1).uniform(-0.05, 0.05, 2000),
                        (grid[1:] + grid[:-1]) / 2])            # exact midpoints
    got = oracle.fp8_e4m3_round(x)
    for xi, gi in zip(x, got):
        dist = np.abs(grid - xi)
        cands = grid[dist == dist.min()]
        if len(cands) == 1:
            assert gi == cands[0]
        else:                                              # tie: even significand
            def even(v):
                if v == 0:
                    return True
                m, e = np.frexp(abs(v))
                if abs(v) < 2.0 ** -6:
                    return int(round(abs(v) / 2.0 ** -9)) % 2 == 0
                return int(round(m * 16)) % 2 == 0
            assert gi in cands and even(gi)


def test_e4m3_matches_torch_cast():
    x = np.random.default_rng(2).uniform(-448, 448, 20000).astype(np.float32)
    x = np.concatenate([x, np.float32([0.0, 2.0 ** -10, 3 * 2.0 ** -10, 448.0, -448.0, 1.0625, 1.1875])])
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.fp8_e4m3_round(x.astype(np.float64)), ref)


def test_e4m3_saturates():
    np.testing.assert_array_equal(oracle.fp8_e4m3_round(np.array([500.0, -1e6, 449.0])), [448.0, -448.0, 448.0])


def test_bf16_matches_torch_cast():
    g = np.random.default_rng(3)
    x = (g.standard_normal(50000) * np.exp(g.uniform(-60, 60, 50000))).astype(np.float32)
    bits = (g.integers(0, 2 ** 16, 1000, dtype=np.uint32) << 16) | np.uint32(0x8000)
    ties = bits.view(np.float32)                             # exactly halfway
    x = np.concatenate([x, ties[np.isfinite(ties)], np.float32([1e-40, -3e-39, 0.0])])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.bf16_round(x.astype(np.float64)), ref)


@pytest.mark.parametrize("shape", [(256, 256), (300, 200), (128, 129), (5, 7)])
def test_tile_quantize_properties(shape):
    g = np.random.default_rng(sum(shape))
    X = (g.standard_normal(shape) * np.exp(g.uniform(-4, 4, shape))).astype(np.float32)
    X[:min(128, shape[0]), :min(128, shape[1])][:3, :3] *= 1000.0
    if shape == (300, 200):
        X[256:, 128:] = 0.0                                 # an all-zero edge tile
    codes, scales = oracle.fp8_tile_quantize(X)
    assert scales.shape == (-(-shape[0] // 128), -(-shape[1] // 128))
    grid = set(e4m3_values().tolist())
    assert set(np.unique(codes).tolist()) <= grid
    for I in range(scales.shape[0]):
        for J in range(scales.shape[1]):
            blk = X[I * 128:(I + 1) * 128, J * 128:(J + 1) * 128]
            amax = np.abs(blk).max()
            exp = np.float32(amax / np.float32(448)) if amax > 0 else np.float32(1)
            assert scales[I, J] == exp
            cb = codes[I * 128:(I + 1) * 128, J * 128:(J + 1) * 128]
            assert np.abs(cb).max() <= 448.0
            if amax > 0:
                assert np.abs(cb).max() == 448.0
    D = oracle.fp8_tile_dequantize(codes, scales)
    S = np.repeat(np.repeat(scales.astype(np.float64), 128, 0), 128, 1)[:shape[0], :shape[1]]
    # half an E4M3 step: 2^-4 relative for normals, 2^-10 absolute (times scale) below
    err = np.abs(D - X.astype(np.float64))
    assert np.all(err <= np.maximum(np.abs(X) * 2.0 ** -4, 2.0 ** -10 * S) * (1 + 1e-6) + 1e-30)
