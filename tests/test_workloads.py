"""The seeded input generators (CPU only): the counter-based matrix stream of
the batched workload against the oracle's Philox4x64-10 (itself pinned to
the Random123 known-answer vectors), its value map, and the batched sizes."""
import numpy as np

import workloads as wl
from oracle.rng import philox4x64_10


def _value(word):
    s = sum((word >> (16 * i)) & 0xFFFF for i in range(4))
    return np.float32(s - 131070) * np.float32(float.fromhex("0x1.bb67aep-16"))


def test_philox_matrix_words_follow_the_counter():
    rows, cols, seed, stream = 7, 13, 3, 5
    x = wl.philox_matrix(rows, cols, seed, stream)
    for q in (0, 1, 2, 3, 4, 5, 17, 50, rows * cols - 1):
        block = philox4x64_10((q // 4, stream, 0, 3 << 32), (seed, 0))
        assert x.reshape(-1)[q] == _value(block[q % 4]), q


def test_philox_matrix_streams_and_scale():
    a = wl.philox_matrix(64, 64, 3, 0)
    b = wl.philox_matrix(64, 64, 3, 1)
    c = wl.philox_matrix(64, 64, 4, 0)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
    assert np.array_equal(wl.philox_matrix(64, 64, 3, 0, scale=0.5), a * np.float32(0.5))
    # a prefix of the stream does not depend on the matrix shape
    assert np.array_equal(wl.philox_matrix(8, 8, 3, 0).reshape(-1), a.reshape(-1)[:64])


def test_philox_matrix_moments():
    x = wl.philox_matrix(1000, 1000, 3, 9).astype(np.float64)
    assert abs(x.mean()) < 5e-3 and abs(x.var() - 1.0) < 5e-3
    # Irwin-Hall of four uniforms: excess kurtosis -1.2 / 4
    k = ((x - x.mean()) ** 4).mean() / x.var() ** 2 - 3.0
    assert abs(k + 0.3) < 0.02
    assert np.abs(x).max() <= 131070 * float.fromhex("0x1.bb67aep-16") + 1e-6


def test_batched_sizes_ranges():
    items = wl.batched_sizes(64, seed=11)
    for it in items:
        assert 256 <= it["m"] <= 2048 and 256 <= it["p"] <= 2048
        assert 4096 <= it["n"] <= 32768 and 16 <= it["c"] <= 256
        w = np.diff(it["off"])
        assert it["off"][0] == 0 and it["off"][-1] == it["n"]
        assert w.min() >= 8 and w.max() <= 128
