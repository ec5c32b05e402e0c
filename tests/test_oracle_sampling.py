"""Pins of the oracle's integer sampling machinery (CPU only).

Quantization, CDF search, Lemire's bounded integer and the draw-count
allocation are checked by hand-derived values, exhaustive enumeration and
invariants that any correct implementation must satisfy.
"""
import math

import numpy as np
import pytest

from oracle.sampling import (quantize_weights, inclusive_cdf, lemire_uniform,
                             search_cdf, draw_atoms, allocate_draws, ceil_log2,
                             wide_words)
from oracle.rng import philox4x64_10, TAG_SAMPLE


# --------------------------------------------------------------------------
# quantize_weights
# --------------------------------------------------------------------------

def test_quantize_hand_values():
    # A = 3 -> B = 63 - 2 = 61; max = 1.0 -> e = 0; scale 2^(B-1-e) = 2^60
    assert quantize_weights([1.0, 0.5, 0.25]) == [2**60, 2**59, 2**58]
    # 0.3 * 2^60 is not an integer: the ceiling is taken
    assert quantize_weights([1.0, 0.3, 0.0]) == [2**60, math.ceil(0.3 * 2**60), 0]
    # A = 1 -> B = 63; the single weight lands in [2^62, 2^63)
    assert quantize_weights([3.0]) == [3 * 2**61]
    # A = 4 -> B = 61; max 6 -> e = 2 -> scale 2^58
    assert quantize_weights([6.0, 1.0, 0.0, 2.0]) == [6 * 2**58, 2**58, 0, 2**59]


def test_quantize_takes_the_ceiling():
    # 2^-10 + 2^-62 scaled by 2^60 is 2^50 + 1/4: the ceiling is 2^50 + 1
    x = math.ldexp(1.0, -10) + math.ldexp(1.0, -62)
    assert quantize_weights([1.0, x, 0.5]) == [2**60, 2**50 + 1, 2**59]


def test_quantize_invariants():
    g = np.random.Generator(np.random.PCG64(5))
    for A in (1, 2, 3, 17, 1024, 5000):
        w = g.lognormal(0, 3, size=A)
        w[g.integers(0, A, size=A // 5)] = 0.0
        W = quantize_weights(w)
        B = 63 - ceil_log2(A)
        assert all(0 <= x <= 2**B for x in W)
        assert sum(W) <= 2**63
        assert all((x == 0) == (v == 0.0) for x, v in zip(W, w))
        imax = int(np.argmax(w))
        assert 2**(B - 1) <= W[imax] <= 2**B
        # ratios are kept to the resolution of the integer grid
        for x, v in zip(W, w):
            assert abs(x - v / w[imax] * W[imax]) <= 1.0 + 1e-9 * x


def test_quantize_power_of_two_invariance():
    w = [0.7, 1e-30, 3.25, 0.0, 12.5]
    for k in (-600, -3, 1, 40, 900):
        assert quantize_weights([math.ldexp(x, k) for x in w]) == quantize_weights(w)


def test_quantize_tiny_weights_get_one():
    W = quantize_weights([1.0, 1e-300])
    assert W[1] == 1


@pytest.mark.parametrize("bad", [[1.0, -1.0], [float("nan")], [1.0, float("inf")]])
def test_quantize_rejects_bad(bad):
    with pytest.raises(ValueError):
        quantize_weights(bad)


def test_quantize_all_zero():
    assert quantize_weights([0.0, 0.0]) == [0, 0]
    assert quantize_weights([]) == []


# --------------------------------------------------------------------------
# CDF search: brute force over every integer
# --------------------------------------------------------------------------

def test_search_brute_force():
    g = np.random.Generator(np.random.PCG64(8))
    for trial in range(40):
        A = int(g.integers(1, 9))
        W = [int(x) for x in g.integers(0, 6, size=A)]
        if sum(W) == 0:
            W[-1] = 1
        cdf = inclusive_cdf(W)
        T = cdf[-1]
        hits = [0] * A
        for r in range(T):
            a = search_cdf(cdf, r)
            lo = cdf[a - 1] if a else 0
            assert lo <= r < cdf[a]
            assert W[a] > 0
            hits[a] += 1
        assert hits == W
        with pytest.raises(ValueError):
            search_cdf(cdf, T)


# --------------------------------------------------------------------------
# Lemire: exhaustive at small word widths, definition at 64 bits
# --------------------------------------------------------------------------

@pytest.mark.parametrize("bits", [4, 8])
def test_lemire_exact_uniform_exhaustive(bits):
    mod = 1 << bits
    for T in range(1, mod + 1):
        counts = [0] * T
        rejected = 0
        for x in range(mod):
            try:
                r = lemire_uniform(iter([x]), T, word_bits=bits)
            except RuntimeError:
                rejected += 1
                continue
            counts[r] += 1
        assert counts == [mod // T] * T
        assert rejected == mod % T


def test_lemire_16bit_sample():
    mod = 1 << 16
    for T in (3, 1000, 40000, 65535):
        counts = np.zeros(T, dtype=np.int64)
        for x in range(mod):
            try:
                counts[lemire_uniform(iter([x]), T, word_bits=16)] += 1
            except RuntimeError:
                pass
        assert np.all(counts == mod // T)


def test_lemire_64bit_accepts_high_product():
    g = np.random.Generator(np.random.PCG64(3))
    for _ in range(2000):
        T = int(g.integers(1, 2**62)) * 2 + int(g.integers(0, 2))
        x = int(g.integers(0, 2**63)) * 2 + int(g.integers(0, 2))
        thr = (2**64 - T) % T
        if (x * T) % 2**64 >= thr:
            assert lemire_uniform(iter([x]), T) == (x * T) >> 64
        else:
            with pytest.raises(RuntimeError):
                lemire_uniform(iter([x]), T)


def test_lemire_rejection_consumes_next_word():
    # T = 3 at 8 bits: threshold = 256 mod 3 = 1 -> x = 0 is rejected
    assert lemire_uniform(iter([0, 255]), 3, word_bits=8) == (255 * 3) >> 8


# --------------------------------------------------------------------------
# draws: goodness of fit of the whole generator -> integer -> atom chain
# --------------------------------------------------------------------------

def test_draw_frequencies_chi_square():
    from scipy.stats import chisquare
    w = [0.5, 0.0, 2.0, 1.0, 0.25, 3.0]
    W = quantize_weights(w)
    cdf = inclusive_cdf(W)
    T = cdf[-1]
    n = 30000
    idx = draw_atoms(cdf, T, n, seed=77, trial=3, stratum=1)
    cnt = np.bincount(idx, minlength=len(w))
    assert cnt[1] == 0
    nz = [a for a in range(len(w)) if W[a] > 0]
    exp = np.array([W[a] / T * n for a in nz])
    stat, pval = chisquare(cnt[nz], exp)
    assert pval > 1e-4


def test_draw_uses_high_part_of_128_bit_product():
    # the first draw of (seed 5, trial 2, stratum 1, draw 0) takes the first
    # two Philox words of block 0 as one 128-bit word, high word first
    W = quantize_weights([1.0, 2.0, 3.0, 4.0, 0.5])
    cdf = inclusive_cdf(W)
    T = cdf[-1]
    w = philox4x64_10((0, 1, 2, (TAG_SAMPLE << 32) | 0), (5, 0))
    x = (w[0] << 64) | w[1]
    assert (x * T) % 2**128 >= (2**128 - T) % T      # accepted (p > 1 - 2^-64)
    r = (x * T) >> 128
    assert draw_atoms(cdf, T, 1, seed=5, trial=2, stratum=1) == [search_cdf(cdf, r)]
    assert list(wide_words([1, 2, 3, 4])) == [(1 << 64) | 2, (3 << 64) | 4]


def test_draw_stable_under_unit_change_of_total():
    # moving one weight by a unit (as last-bit noise in the norms does)
    # leaves the draws unchanged
    g = np.random.Generator(np.random.PCG64(4))
    W = [int(x) for x in g.integers(2**55, 2**56, size=64)]
    cdf = inclusive_cdf(W)
    W2 = list(W)
    W2[10] += 1
    cdf2 = inclusive_cdf(W2)
    a = draw_atoms(cdf, cdf[-1], 500, 1, 0, 0)
    b = draw_atoms(cdf2, cdf2[-1], 500, 1, 0, 0)
    assert a == b


def test_draws_reproducible_and_independent_of_count():
    W = quantize_weights([1.0, 2.0, 3.0, 4.0])
    cdf = inclusive_cdf(W)
    a = draw_atoms(cdf, cdf[-1], 50, 1, 2, 3)
    b = draw_atoms(cdf, cdf[-1], 20, 1, 2, 3)
    assert a[:20] == b          # draw j depends only on its own counter
    assert draw_atoms(cdf, cdf[-1], 50, 1, 2, 3) == a


# --------------------------------------------------------------------------
# allocation
# --------------------------------------------------------------------------

def test_allocate_hand_values():
    # 10 draws over three equal strata: quotas 3,3,3, remainders 1,1,1 -> the
    # extra draw goes to the lowest stratum
    assert allocate_draws(10, [1, 1, 1], [5, 5, 5]) == [4, 3, 3]
    # exact proportional split
    assert allocate_draws(12, [1, 2, 3], [1, 1, 1]) == [2, 4, 6]
    # remainders: 7*[5,3,2]/10 = [3.5, 2.1, 1.4] -> [3,2,1] + 1 to stratum 0
    assert allocate_draws(7, [5, 3, 2], [1, 1, 1]) == [4, 2, 1]
    # a zero-weight stratum that can be sampled still gets one draw, taken
    # from the stratum holding the most
    assert allocate_draws(5, [1, 0, 1], [1, 1, 1]) == [2, 1, 2]
    # a stratum with T = 0 gets nothing, even with positive G
    assert allocate_draws(4, [1, 9, 1], [1, 0, 1]) == [2, 0, 2]
    # all sampleable strata have G = 0: fall back to equal weights
    assert allocate_draws(6, [0, 0, 0], [2, 3, 4]) == [2, 2, 2]


def test_allocate_uniform_divisible():
    for K in (1, 2, 10, 50, 500):
        c = 100 * K
        assert allocate_draws(c, [1] * K, [1] * K) == [100] * K


def test_allocate_properties():
    g = np.random.Generator(np.random.PCG64(2))
    for _ in range(300):
        S = int(g.integers(1, 12))
        G = [int(x) for x in g.integers(0, 10**6, size=S)]
        T = [int(x) for x in g.integers(0, 3, size=S)]
        act = [s for s in range(S) if T[s] > 0]
        c = len(act) + int(g.integers(0, 40))
        if not act:
            assert allocate_draws(c, G, T) == [0] * S
            continue
        cs = allocate_draws(c, G, T)
        assert sum(cs) == c
        assert all(cs[s] >= 1 for s in act)
        assert all(cs[s] == 0 for s in range(S) if T[s] == 0)
        g_eff = [G[s] if T[s] > 0 else 0 for s in range(S)]
        if sum(g_eff) > 0 and all(c * g_eff[s] >= sum(g_eff) for s in act):
            # no stratum needed the minimum-one repair: largest remainders
            # keep every count within one of its real-valued share
            for s in range(S):
                assert abs(cs[s] - c * g_eff[s] / sum(g_eff)) < 1.0


def test_allocate_budget_too_small():
    with pytest.raises(ValueError):
        allocate_draws(2, [1, 1, 1], [1, 1, 1])
