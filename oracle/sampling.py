"""Integer sampling machinery of the oracle.

Test infrastructure only (see the package docstring).

The paper fixes the sampling law (Alg. 1: index ``s`` is drawn with
probability ``p_s``, independently, with replacement; Alg. 2: stratum ``k``
receives ``c_k`` such draws with its own probabilities) but says nothing
about how probabilities become draws, nor how the real-valued draw counts
(3.9), (4.2) and (4.7) become integers. This module holds the readings used
by the project, all in exact integer arithmetic so that the chosen indices do
not depend on any floating-point summation order:

* ``quantize_weights``  - non-negative float weights -> uint64 integers W
                          with a common power-of-two scale;
* ``inclusive_cdf``     - exact integer running sums of W (total T);
* ``lemire_uniform``    - Lemire's multiply-and-reject map from random words
                          to an exactly uniform integer in [0, T)
                          (D. Lemire, "Fast random integer generation in an
                          interval", ACM TOMACS 29(1), 2019), used with
                          128-bit words (two generator words) so that a
                          rejection has probability below 2^-64 for any
                          T < 2^64: the drawn index then depends only on the
                          high part of the product, which moves by at most
                          one unit when T moves by a unit, so last-bit
                          differences in the weights almost never change a
                          draw;
* ``search_cdf``        - the atom whose CDF interval holds that integer;
* ``allocate_draws``    - integer draw counts c_s with sum c and c_s >= 1 on
                          every stratum that can be sampled (Alg. 2 input
                          conditions).

The estimator then uses p_hat = W / T, the probability that is actually
sampled, in its rescaling, which keeps it exactly unbiased (Lemma 1).
"""

import bisect
import math

from .rng import draw_words, TAG_SAMPLE

UINT64_MAX = (1 << 64) - 1


def ceil_log2(a):
    """Smallest b >= 0 with 2**b >= a (a >= 1)."""
    if a < 1:
        raise ValueError("ceil_log2 needs a >= 1")
    return (a - 1).bit_length()


def quantize_weights(w):
    """Map non-negative finite float weights to uint64 integers.

    With A weights, e = floor(log2(max w)) and B = 63 - ceil(log2 A), weight
    x becomes W = ceil(x * 2**(B-1-e)); a positive weight that would become 0
    becomes 1, and 0 stays 0. Every W <= 2**B, so the total of all A weights
    is at most 2**63 and fits in 64 bits with room to spare. The scaling is by
    a power of two and the ceiling is exact, so W is a pure function of the
    float64 bit patterns of ``w``.

    Returns a list of Python ints (empty input -> empty list).
    """
    w = [float(x) for x in w]
    for x in w:
        if not math.isfinite(x) or x < 0.0:
            raise ValueError("weights must be finite and non-negative")
    if not w:
        return []
    wmax = max(w)
    if wmax == 0.0:
        return [0] * len(w)
    e = math.frexp(wmax)[1] - 1          # wmax in [2**e, 2**(e+1))
    b = 63 - ceil_log2(len(w))
    out = []
    for x in w:
        if x == 0.0:
            out.append(0)
            continue
        q = math.ceil(math.ldexp(x, b - 1 - e))
        out.append(max(int(q), 1))
    return out


def inclusive_cdf(W):
    """Exact running sums: cdf[a] = W[0] + ... + W[a]."""
    cdf, run = [], 0
    for x in W:
        run += int(x)
        cdf.append(run)
    if run > UINT64_MAX:
        raise OverflowError("CDF total exceeds 64 bits")
    return cdf


def lemire_uniform(words, T, word_bits=64):
    """Exactly uniform integer in [0, T) from a stream of random words.

    A word x (uniform on [0, 2**word_bits)) is multiplied by T; the high part
    of the product is the candidate and the low part decides acceptance: the
    word is rejected when low < (2**word_bits - T) mod T, which leaves exactly
    floor(2**word_bits / T) accepted words per outcome. ``word_bits`` is a
    parameter so that the tests can enumerate every word at a small width.
    """
    if T <= 0 or T > (1 << word_bits):
        raise ValueError("T out of range")
    mod = 1 << word_bits
    threshold = (mod - T) % T
    for x in words:
        prod = int(x) * T
        low = prod & (mod - 1)
        if low < threshold:
            continue
        return prod >> word_bits
    raise RuntimeError("word stream ended")


def search_cdf(cdf, r):
    """Index of the first CDF entry strictly greater than r (upper bound).

    Atom a owns the integers [cdf[a-1], cdf[a]); an atom with W = 0 owns none
    and is never returned.
    """
    a = bisect.bisect_right(cdf, r)
    if a >= len(cdf):
        raise ValueError("r is not below the CDF total")
    return a


WORD_BITS = 128


def wide_words(words):
    """Pairs of consecutive 64-bit words as 128-bit words, the first word of
    each pair being the high half."""
    it = iter(words)
    for hi in it:
        lo = next(it)
        yield (int(hi) << 64) | int(lo)


def draw_atoms(cdf, T, count, seed, trial, stratum, tag=TAG_SAMPLE):
    """``count`` independent draws from one stratum's integer CDF.

    Draw j reads its own Philox word stream (``rng.draw_words``), maps it to
    an exactly uniform integer r in [0, T) with 128-bit words, and returns
    the local atom index whose CDF interval holds r.
    """
    out = []
    for j in range(count):
        words = wide_words(draw_words(seed, trial, stratum, j, tag))
        r = lemire_uniform(words, T, word_bits=WORD_BITS)
        out.append(search_cdf(cdf, r))
    return out


def allocate_draws(c, G, T):
    """Integer draw counts c_s for the strata.

    ``G`` are non-negative integer allocation weights (quantized by
    ``quantize_weights``), ``T`` the CDF totals of the strata. A stratum with
    T_s = 0 holds only zero-weight atoms, its block product is zero and it
    gets no draws. Every other stratum gets at least one draw (Alg. 2 asks
    c_k >= 1), so c must be at least their number.

    Steps: if every sampleable stratum has G_s = 0, use G_s = 1 for them;
    give each the exact quota floor(c G_s / sum G); hand the remaining draws
    out one each in decreasing order of the remainders c G_s mod sum G, ties
    to the lower stratum; then, for ascending s, a sampleable stratum left at
    0 takes one draw from the stratum holding the most (ties to the lower s).
    """
    S = len(G)
    if len(T) != S:
        raise ValueError("G and T differ in length")
    active = [s for s in range(S) if T[s] > 0]
    if c < len(active):
        raise ValueError("budget c is below the number of sampleable strata")
    if not active:
        return [0] * S
    g = [int(G[s]) if T[s] > 0 else 0 for s in range(S)]
    if sum(g) == 0:
        g = [1 if T[s] > 0 else 0 for s in range(S)]
    tot = sum(g)
    cs = [c * g[s] // tot for s in range(S)]
    rem = [c * g[s] % tot for s in range(S)]
    left = c - sum(cs)
    order = sorted(active, key=lambda s: (-rem[s], s))
    for s in order[:left]:
        cs[s] += 1
    for s in active:
        if cs[s] == 0:
            donor = max(range(S), key=lambda q: (cs[q], -q))
            cs[donor] -= 1
            cs[s] += 1
    return cs
