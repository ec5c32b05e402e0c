"""Pins of the oracle's Philox4x64-10 (CPU only).

The generator is checked against published known-answer vectors and against
an independent implementation (numpy.random.Philox), so that a wrong constant,
a swapped output word or a wrong key schedule fails.
"""
import os

import numpy as np
import pytest

from oracle.rng import philox4x64_10, draw_words, TAG_SAMPLE, TAG_PILOT

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")
MASK = (1 << 64) - 1


def _kat_rows():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((tuple(v[0:4]), tuple(v[4:6]), tuple(v[6:10])))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat_rows())
def test_known_answer_vectors(ctr, key, out):
    assert philox4x64_10(ctr, key) == out


def _numpy_block(ctr, key):
    # numpy's Philox advances its 256-bit counter before each block, so the
    # block for counter X comes from a generator started at X - 1.
    c = sum(v << (64 * i) for i, v in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    start = [(c >> (64 * i)) & MASK for i in range(4)]
    bg = np.random.Philox(counter=np.array(start, dtype=np.uint64),
                          key=np.array(key, dtype=np.uint64))
    return tuple(int(x) for x in bg.random_raw(4))


def test_matches_numpy_philox_random_counters():
    g = np.random.Generator(np.random.PCG64(123))
    for _ in range(200):
        ctr = tuple(int(x) for x in g.integers(0, 2**64, size=4, dtype=np.uint64))
        key = tuple(int(x) for x in g.integers(0, 2**64, size=2, dtype=np.uint64))
        assert philox4x64_10(ctr, key) == _numpy_block(ctr, key)


def test_matches_numpy_philox_sampler_counters():
    # the counter shapes the sampler really uses
    for seed in (0, 1, 2**64 - 1):
        for s in (0, 3, 1023):
            for j in (0, 1, 255):
                for tag, blk in ((TAG_SAMPLE, 0), (TAG_SAMPLE, 7), (TAG_PILOT, 0)):
                    ctr = (j, s, 5, (tag << 32) | blk)
                    assert philox4x64_10(ctr, (seed, 0)) == _numpy_block(ctr, (seed, 0))


def test_draw_word_stream_order():
    it = draw_words(seed=9, trial=4, stratum=2, draw=17, tag=TAG_SAMPLE)
    words = [next(it) for _ in range(12)]
    for blk in range(3):
        ref = philox4x64_10((17, 2, 4, (TAG_SAMPLE << 32) | blk), (9, 0))
        assert tuple(words[4 * blk:4 * blk + 4]) == ref


def test_streams_differ_by_every_counter_field():
    base = next(draw_words(1, 0, 0, 0))
    assert next(draw_words(2, 0, 0, 0)) != base
    assert next(draw_words(1, 1, 0, 0)) != base
    assert next(draw_words(1, 0, 1, 0)) != base
    assert next(draw_words(1, 0, 0, 1)) != base
    assert next(draw_words(1, 0, 0, 0, TAG_PILOT)) != base
