"""Pins of the oracle's two-step algorithm (Alg. 3) against facts the
mathematics fixes (CPU only):

* a block whose outer products are positive multiples of one matrix is
  estimated exactly by a pilot under (3.8) whatever is drawn (each draw
  contributes (sum_j lambda_j) u v^T / r), and under uniform pilot
  probabilities when the multiples are equal; a wrong pilot scale, or a
  product taken across blocks, changes the value;
* a hand-computed pilot (forced draw) whose estimate exceeds s_k^2, where
  (4.7)'s absolute value and a clamp at zero differ;
* with the exact ||M^k N_k||_F^2 in place of the pilot, (4.7) equals (3.9),
  since s_k >= ||M^k N_k||_F (triangle inequality);
* the pilot's draw counts are the integer part of c0 / K per block that can
  be sampled, and c0 < K is rejected.
"""
import math

import numpy as np
import pytest

from oracle import method as om
from oracle.rng import TAG_PILOT, TAG_SAMPLE


def _gen(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _parallel_block_problem(equal, seed=1):
    """m=5, p=4, three blocks of widths 6, 7, 5; block 1 has outer products
    lambda_i * u v^T (lambda_i > 0; all equal when ``equal``), the others are
    Gaussian."""
    g = _gen(seed)
    off = [0, 6, 13, 18]
    M = g.standard_normal((5, 18))
    N = g.standard_normal((18, 4))
    u, v = g.standard_normal(5), g.standard_normal(4)
    lam = np.full(7, 1.7) if equal else g.uniform(0.2, 3.0, 7)
    # column i of M^1 = sqrt(lam_i) u * sign, row i of N_1 = sqrt(lam_i) v * sign
    sgn = np.where(g.standard_normal(7) > 0, 1.0, -1.0)
    M[:, 6:13] = np.outer(u, np.sqrt(lam) * sgn)
    N[6:13, :] = np.outer(np.sqrt(lam) * sgn, v)
    return M, N, off


@pytest.mark.parametrize("pilot_prob,equal", [("norm", False), ("norm", True), ("uniform", True)])
def test_pilot_exact_on_parallel_block(pilot_prob, equal):
    M, N, off = _parallel_block_problem(equal)
    exact = om.block_product_sq(M, N, off)
    for seed in range(5):
        pl = om.pilot(M, N, off, c0=9, pilot_prob=pilot_prob, seed=seed)
        assert pl.pilot_sq[1] == pytest.approx(exact[1], rel=1e-12)
    # the other blocks are random estimates, not the exact values
    assert not np.allclose(pl.pilot_sq[[0, 2]], exact[[0, 2]], rtol=1e-6)


def test_pilot_uniform_not_exact_on_unequal_multiples():
    # uniform pilot probabilities reproduce M^1 N_1 only when the outer
    # products are equal: with unequal multiples the estimate varies
    M, N, off = _parallel_block_problem(equal=False)
    exact = om.block_product_sq(M, N, off)[1]
    vals = {round(om.pilot(M, N, off, 9, "uniform", seed=s).pilot_sq[1] / exact, 9) for s in range(6)}
    assert len(vals) > 1


def test_two_step_allocation_abs_hand_computed():
    # one block of three unit atoms, m = 3, p = 1: X_i = M[:, i] (N rows are 1)
    # a_i b_i = 2, 1, 1, so s = 4 and s^2 = 16.  Uniform pilot, c0 = K = 1
    # (one draw, p = 1/3): drawing atom 0 gives C0 D0 = 3 X_0 = (6, 0, 0),
    # estimate 36 > 16, g = sqrt(|16 - 36|) = sqrt(20); drawing atom 1 gives
    # (0, 3, 0), estimate 9, g = sqrt(7).
    M = np.array([[2.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    N = np.ones((3, 1))
    off = [0, 3]
    for forced, est, g in (([0], 36.0, math.sqrt(20.0)), ([1], 9.0, math.sqrt(7.0))):
        pl = om.pilot(M, N, off, 1, "uniform", seed=0, forced=[forced])
        assert pl.pilot_sq[0] == pytest.approx(est, rel=1e-14)
        stats = om.block_stats(*om.column_row_sq(M, N), om.check_partition(off, 3))
        assert om.alloc_weights("two_step", stats, pilot_sq=pl.pilot_sq)[0] == pytest.approx(g, rel=1e-14)
    # a clamp at zero (the rule of (3.9)) would give 0 for the first case
    assert om.alloc_weights("opt", stats, blkprod_sq=np.array([36.0]))[0] == 0.0


def test_two_step_with_exact_estimates_is_opt():
    g = _gen(5)
    M = g.standard_normal((6, 40)) * np.exp(g.normal(0, 1.0, 40))
    N = g.standard_normal((40, 7))
    off = om.check_partition([0, 5, 17, 18, 30, 40], 40)
    stats = om.block_stats(*om.column_row_sq(M, N), off)
    exact = om.block_product_sq(M, N, off)
    assert np.all(stats.s ** 2 >= exact * (1 - 1e-12))
    two = om.alloc_weights("two_step", stats, pilot_sq=exact)
    opt = om.alloc_weights("opt", stats, blkprod_sq=exact)
    # where s_k^2 = ||M^k N_k||_F^2 (the one-column block) both vanish up to
    # the square root of a rounding residue, s_k * sqrt(eps)
    assert np.allclose(two, opt, rtol=1e-9, atol=1e-7 * stats.s.max())
    assert opt[2] == 0.0 and two[2] < 1e-7 * stats.s[2]


def test_pilot_counts_and_rejects():
    g = _gen(6)
    M = g.standard_normal((4, 50))
    N = g.standard_normal((50, 3))
    M[:, 10:20] = 0.0                        # block 1 cannot be sampled under (3.8)
    off = [0, 10, 20, 35, 50]
    pl = om.pilot(M, N, off, 27, "norm", seed=3)     # [27 / 4] = 6
    assert pl.design.cs == [6, 0, 6, 6]
    assert pl.pilot_sq[1] == 0.0
    assert np.array_equal(np.bincount(pl.draws.strat, minlength=4), [6, 0, 6, 6])
    pl_u = om.pilot(M, N, off, 27, "uniform", seed=3)
    assert pl_u.design.cs == [6, 6, 6, 6] and pl_u.pilot_sq[1] == 0.0
    with pytest.raises(ValueError):
        om.pilot(M, N, off, 3, "norm", seed=0)
    with pytest.raises(ValueError):
        om.pilot(M, N, off, 8, "exact", seed=0)


def test_pilot_uses_its_own_streams():
    # the pilot draws of stratum s, draw j, read the Philox counter with tag
    # TAG_PILOT; the same design sampled with TAG_SAMPLE differs
    g = _gen(7)
    M = g.standard_normal((4, 64))
    N = g.standard_normal((64, 3))
    off = [0, 32, 64]
    pl = om.pilot(M, N, off, 40, "norm", seed=11, trial=2)
    again = om.sample(pl.design, 11, 2, tag=TAG_PILOT)
    other = om.sample(pl.design, 11, 2, tag=TAG_SAMPLE)
    assert np.array_equal(pl.draws.atom, again.atom)
    assert not np.array_equal(pl.draws.atom, other.atom)


def test_two_step_run_is_stratified_norm_with_pilot_allocation():
    g = _gen(8)
    M = g.standard_normal((6, 120)) * np.exp(g.normal(0, 1.0, 120))
    N = g.standard_normal((120, 5))
    off = [0, 30, 50, 90, 120]
    res = om.run(M, N, off, 60, seed=4, trial=1, mode="stratified", prob="norm",
                 alloc="two_step", c0=20, pilot_prob="uniform")
    pl = om.pilot(M, N, off, 20, "uniform", seed=4, trial=1)
    assert sum(res.design.cs) == 60 and min(res.design.cs) >= 1
    g_k = om.alloc_weights("two_step", res.stats, pilot_sq=pl.pilot_sq)
    assert np.allclose(res.design.g, g_k)
    # counts follow g: the largest share goes to the largest weight
    assert res.design.cs[int(np.argmax(g_k))] == max(res.design.cs)
