"""Philox4x64-10 and the counter layout of the sampler (oracle side).

Test infrastructure only (see the package docstring).

The paper requires each index to be drawn independently and with replacement
(Alg. 1, step 1(a)) but names no generator. This oracle uses the
counter-based Philox4x64 generator with 10 rounds, written here from its
definition in Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3" (SC'11): the Philox S-box built from two 64x64->128 bit
multiplications per round, and the Weyl-sequence key schedule.

Counter layout (a reading of this project, not the paper's): the draw with
index ``j`` inside stratum ``s`` of trial ``trial`` reads the 64-bit words of

    counter = (j, s, trial, (tag << 32) | blk),   key = (seed, 0)

for ``blk = 0, 1, 2, ...`` in order, consuming the four output words of each
block from first to last. ``tag`` separates independent purposes.
"""

MASK64 = (1 << 64) - 1

# Round multipliers and key increments of Philox4x64 as published by Salmon
# et al.: the multipliers were chosen by the authors for avalanche, the
# increments are the golden ratio and sqrt(3)-1 in 0.64 fixed point.
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B

TAG_SAMPLE = 1   # the main with-replacement draws (Alg. 1 / Alg. 2)
TAG_PILOT = 2    # the pilot draws of the two-step algorithm (Alg. 3, step 1)


def philox4x64_10(counter, key):
    """One Philox4x64-10 block: four 64-bit counter words and two key words
    in, four 64-bit output words out.

    Each round multiplies counter words 0 and 2 by the two constants, keeps
    the high and low halves of the 128-bit products, and mixes them with the
    other two words and the round key; the key advances by the Weyl
    increments between rounds.
    """
    x0, x1, x2, x3 = (int(v) & MASK64 for v in counter)
    k0, k1 = (int(v) & MASK64 for v in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * x0
        p1 = PHILOX_M1 * x2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return (x0, x1, x2, x3)


def draw_words(seed, trial, stratum, draw, tag=TAG_SAMPLE):
    """Endless stream of 64-bit words owned by one draw (see module doc)."""
    if not (0 <= tag < (1 << 32)):
        raise ValueError("tag must fit in 32 bits")
    blk = 0
    while True:
        ctr = (draw, stratum, trial, ((tag << 32) | blk) & MASK64)
        for w in philox4x64_10(ctr, (seed, 0)):
            yield w
        blk += 1
        if blk >= (1 << 32):
            raise RuntimeError("draw exhausted 2^32 Philox blocks")
