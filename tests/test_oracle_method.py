"""Pins of the oracle's estimator (CPU only).

What fixes the expected values here is the mathematics of the paper, not the
oracle's own formulas:

* exhaustive enumeration of every draw tuple with its probability: the mean
  of CD is MN (Lemma 1, (3.6)), the per-entry variance is (3.7) and the mean
  squared error equals the closed form (Remark 2.2);
* sampling that is deterministic (one atom per stratum) reproduces MN;
* block mode with unit blocks and stratified mode with one block are both
  Alg. 1 with probabilities (1.1) and draw the same indices;
* at (3.8) and (3.9) the summed variance equals the printed optimum (3.10),
  and no other choice of probabilities or real block sizes goes below it
  (Thm 2);
* norms agree with library routines (QR, SVD) and exact special cases;
* the gradient of the bilinear sketch matches central differences and, in
  expectation, the exact gradient.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import method as om
from oracle.sampling import quantize_weights
import workloads as wl


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


# --------------------------------------------------------------------------
# norms
# --------------------------------------------------------------------------

def test_norms_orthogonal_columns_and_rows():
    g = wl.rng(1)
    Q, _ = np.linalg.qr(g.standard_normal((40, 40)))
    col, row = om.column_row_sq(Q, Q)
    assert np.allclose(col, 1.0, atol=1e-13)
    assert np.allclose(row, 1.0, atol=1e-13)


def test_norms_constant_and_frobenius():
    M = np.ones((37, 11))
    N = np.full((11, 5), 2.0)
    col, row = om.column_row_sq(M, N)
    assert np.all(col == 37.0) and np.all(row == 20.0)
    g = wl.rng(2)
    A = g.standard_normal((50, 30))
    B = g.standard_normal((30, 20))
    col, row = om.column_row_sq(A, B)
    sa = np.linalg.svd(A, compute_uv=False)
    sb = np.linalg.svd(B, compute_uv=False)
    assert math.isclose(col.sum(), float(np.sum(sa**2)), rel_tol=1e-12)
    assert math.isclose(row.sum(), float(np.sum(sb**2)), rel_tol=1e-12)


def test_norms_chunking_does_not_matter():
    M, N, _ = wl.random_problem(7, 300, 5, 4, seed=3)
    a = om.column_row_sq(M, N, chunk=7)
    b = om.column_row_sq(M, N, chunk=1000)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_block_stats_and_products():
    M, N, off = wl.random_problem(9, 60, 7, 5, seed=4)
    col, row = om.column_row_sq(M, N)
    st = om.block_stats(col, row, off)
    bp = om.block_product_sq(M, N, off)
    for k in range(5):
        A = M[:, off[k]:off[k + 1]]
        B = N[off[k]:off[k + 1], :]
        # Frobenius norms through singular values
        assert math.isclose(st.m_sq[k], float(np.sum(np.linalg.svd(A, compute_uv=False)**2)), rel_tol=1e-12)
        assert math.isclose(st.n_sq[k], float(np.sum(np.linalg.svd(B, compute_uv=False)**2)), rel_tol=1e-12)
        # ||AB||_F^2 = trace((A^T A)(B B^T)) (Gram matrices)
        assert math.isclose(bp[k], float(np.trace((A.T @ A) @ (B @ B.T))), rel_tol=1e-11)
        # triangle inequality: ||M^k N_k||_F <= s_k (used by Thm 2's proof)
        assert math.sqrt(bp[k]) <= st.s[k] * (1 + 1e-12)


def test_s_equals_product_norm_for_collinear_outer_products():
    # M^k = u alpha^T, N_k = beta v^T with alpha, beta > 0: every outer
    # product is a positive multiple of u v^T, so ||M^k N_k||_F = s_k
    g = wl.rng(5)
    u, v = g.standard_normal(6), g.standard_normal(4)
    al, be = g.uniform(0.5, 2, 9), g.uniform(0.5, 2, 9)
    M = np.outer(u, al)
    N = np.outer(be, v)
    col, row = om.column_row_sq(M, N)
    st = om.block_stats(col, row, [0, 9])
    bp = om.block_product_sq(M, N, [0, 9])
    assert math.isclose(math.sqrt(bp[0]), st.s[0], rel_tol=1e-12)


# --------------------------------------------------------------------------
# exhaustive enumeration (Lemma 1, Remark 2.2)
# --------------------------------------------------------------------------

def _enumerate(M, N, design):
    """All draw tuples with their probabilities (stratum by stratum)."""
    ph = design.p_hat()
    per = []
    for s in range(len(design.T)):
        a0, a1 = design.strat_off[s], design.strat_off[s + 1]
        atoms = [a - a0 for a in range(a0, a1) if design.W[a] > 0]
        per.append(list(itertools.product(atoms, repeat=design.cs[s])))
    for combo in itertools.product(*per):
        prob = 1.0
        for s, loc in enumerate(combo):
            for la in loc:
                prob *= ph[design.strat_off[s] + la]
        yield prob, combo


def _check_enumeration(M, N, design, var_check=True):
    MN = om.exact_product(M, N)
    mean = np.zeros_like(MN)
    sq = np.zeros_like(MN)
    mse = 0.0
    ptot = 0.0
    for prob, combo in _enumerate(M, N, design):
        d = om.sample(design, 0, forced=combo)
        C, D = om.sketch(M, N, d)
        CD = om.sketch_product(C, D)
        mean += prob * CD
        sq += prob * CD * CD
        mse += prob * float(np.sum((MN - CD) ** 2))
        ptot += prob
    assert math.isclose(ptot, 1.0, rel_tol=1e-12)
    assert _rel(mean, MN) < 1e-12                                   # (3.6)
    closed = om.expected_sq_error(M, N, design)
    assert math.isclose(mse, closed, rel_tol=1e-10, abs_tol=1e-12 * float(np.sum(MN**2)))
    if var_check:
        # (3.7): per-entry variance of the stratified estimator
        var = sq - mean * mean
        ph = design.p_hat()
        ref = np.zeros_like(MN)
        for s in range(len(design.T)):
            a0, a1 = design.strat_off[s], design.strat_off[s + 1]
            if design.cs[s] == 0:
                continue
            tot = np.zeros_like(MN)
            for a in range(a0, a1):
                lo, hi = int(design.atom_lo[a]), int(design.atom_hi[a])
                X = M[:, lo:hi] @ N[lo:hi, :]
                tot += X
                if ph[a] > 0:
                    ref += X * X / (design.cs[s] * ph[a])
            ref -= tot * tot / design.cs[s]
        assert np.allclose(var, ref, rtol=1e-8, atol=1e-9 * float(np.max(np.abs(ref))))
    return mse, closed


@pytest.mark.parametrize("prob", ["uniform", "norm", "exact"])
def test_enumeration_block_mode(prob):
    g = wl.rng(11)
    M = g.standard_normal((3, 8))
    N = g.standard_normal((8, 2))
    off = [0, 1, 3, 6, 8]                          # n_k = 1, 2, 3, 2
    design, *_ = om.plan(M, N, off, 3, mode="block", prob=prob)
    assert design.cs == [3]
    _check_enumeration(M, N, design)


@pytest.mark.parametrize("prob,alloc", [("norm", "norm"), ("norm", "opt"),
                                        ("uniform", "uniform"), ("norm", "uniform")])
def test_enumeration_stratified_mode(prob, alloc):
    g = wl.rng(12)
    M = g.standard_normal((3, 5))
    N = g.standard_normal((5, 2))
    off = [0, 3, 5]                                # n_k = 3, 2
    design, *_ = om.plan(M, N, off, 3, mode="stratified", prob=prob, alloc=alloc)
    assert sum(design.cs) == 3 and min(design.cs) >= 1
    _check_enumeration(M, N, design)


def test_enumeration_user_counts_and_weights():
    g = wl.rng(13)
    M = g.standard_normal((2, 5))
    N = g.standard_normal((5, 3))
    off = [0, 3, 5]
    w = [0.1, 2.0, 1.0, 5.0, 0.3]
    design, *_ = om.plan(M, N, off, 3, mode="stratified", prob="user",
                         alloc="user", user_w=w, user_ck=[2, 1])
    assert design.cs == [2, 1]
    _check_enumeration(M, N, design)


def test_enumeration_zero_column_never_drawn():
    g = wl.rng(14)
    M = g.standard_normal((3, 6))
    N = g.standard_normal((6, 2))
    M[:, 2] = 0.0                      # column 2 is zero: a_2 = 0
    N[4, :] = 0.0                      # row 4 is zero: b_4 = 0
    off = [0, 3, 6]
    design, *_ = om.plan(M, N, off, 3, mode="stratified", prob="norm", alloc="norm")
    assert design.W[2] == 0 and design.W[4] == 0
    _check_enumeration(M, N, design)


def test_enumeration_zero_block_gets_no_draws():
    g = wl.rng(15)
    M = g.standard_normal((3, 6))
    N = g.standard_normal((6, 2))
    M[:, 3:6] = 0.0
    off = [0, 3, 6]
    design, *_ = om.plan(M, N, off, 3, mode="stratified", prob="norm", alloc="norm")
    assert design.cs == [3, 0]
    _check_enumeration(M, N, design)
    design, *_ = om.plan(M, N, [0, 2, 3, 6], 2, mode="block", prob="norm")
    assert design.W[2] == 0
    _check_enumeration(M, N, design)


# --------------------------------------------------------------------------
# deterministic sampling reproduces MN
# --------------------------------------------------------------------------

def test_deterministic_block_mode_one_block():
    M, N, _ = wl.random_problem(20, 50, 15, 1, seed=6)
    r = om.run(M, N, [0, 50], c=4, seed=1, mode="block", prob="norm")
    assert r.draws.L == 4 * 50
    assert _rel(r.CD, r.MN) < 1e-12
    assert r.rel < 1e-12


def test_deterministic_stratified_unit_blocks():
    M, N, _ = wl.random_problem(12, 30, 9, 1, seed=7)
    off = list(range(31))
    r = om.run(M, N, off, c=30, seed=2, mode="stratified", prob="norm", alloc="uniform")
    assert r.design.cs == [1] * 30
    assert _rel(r.CD, r.MN) < 1e-12


def test_entry_helpers_match_full_products():
    M, N, off = wl.random_problem(17, 300, 13, 9, seed=24, skew=1.0)
    r = om.run(M, N, off, c=7, seed=3)
    g = wl.rng(25)
    rows = g.integers(0, 17, size=50)
    cols = g.integers(0, 13, size=50)
    assert _rel(om.sketch_entries(M, N, r.draws, rows, cols), r.CD[rows, cols]) < 1e-13
    assert _rel(om.exact_entries(M, N, rows, cols, chunk=64), (M @ N)[rows, cols]) < 1e-13


def test_tiny_workload_runs():
    M, N, off = wl.tiny()
    r = om.run(M, N, off, c=16, seed=0, mode="block", prob="norm")
    assert r.C.shape == (256, 256) and r.D.shape == (256, 256)
    assert r.draws.L == 256
    e2 = om.expected_sq_error(M, N, r.design)
    # Gaussian data: rel error near sqrt((K-1)/c); the draw sits within a
    # wide band of the closed-form root mean square
    rms = math.sqrt(e2) / np.linalg.norm(r.MN)
    assert 1.0 < rms < 3.0
    assert 0.5 * rms < r.rel < 2.0 * rms


# --------------------------------------------------------------------------
# Alg. 1 with (1.1) in both modes
# --------------------------------------------------------------------------

def test_cross_mode_same_draws():
    M, N, _ = wl.random_problem(10, 64, 8, 1, seed=8, skew=1.0)
    unit = list(range(65))
    rb = om.run(M, N, unit, c=20, seed=5, trial=3, mode="block", prob="norm")
    rs = om.run(M, N, [0, 64], c=20, seed=5, trial=3, mode="stratified",
                prob="norm", alloc="norm")
    assert np.array_equal(rb.draws.lo, rs.draws.lo)
    assert np.array_equal(rb.draws.scale, rs.draws.scale)
    assert np.array_equal(rb.CD, rs.CD)
    # the probabilities are (1.1) up to the integer grid
    col, row = om.column_row_sq(M, N)
    p11 = np.sqrt(col * row) / np.sum(np.sqrt(col * row))
    assert np.allclose(rb.design.p_hat(), p11, rtol=1e-12, atol=0)


# --------------------------------------------------------------------------
# Thm 2 / Remark 2.3
# --------------------------------------------------------------------------

def _real_optimum(M, N, off, c):
    col, row = om.column_row_sq(M, N)
    st = om.block_stats(col, row, off)
    bp = om.block_product_sq(M, N, off)
    ab = np.sqrt(col * row)
    p = np.empty_like(ab)
    for k in range(len(off) - 1):
        sl = slice(off[k], off[k + 1])
        p[sl] = ab[sl] / st.s[k]                                 # (3.8)
    g = np.sqrt(np.maximum(st.s**2 - bp, 0))
    ck = c * g / g.sum()                                         # (3.9), real
    return col, row, st, bp, p, ck


def test_optimum_value_310():
    M, N, off = wl.random_problem(8, 90, 6, 6, seed=9, skew=1.0)
    c = 40
    col, row, st, bp, p, ck = _real_optimum(M, N, off, c)
    lhs = om.sum_variance_real(col, row, off, bp, p, ck)
    assert math.isclose(lhs, om.optimal_value(st, bp, c), rel_tol=1e-11)


def test_optimum_is_minimal():
    M, N, off = wl.random_problem(8, 90, 6, 6, seed=10, skew=1.0)
    c = 40
    col, row, st, bp, p, ck = _real_optimum(M, N, off, c)
    best = om.optimal_value(st, bp, c)
    g = wl.rng(99)
    for _ in range(200):
        q = p * g.uniform(0.5, 1.5, size=p.shape)
        for k in range(len(off) - 1):
            sl = slice(off[k], off[k + 1])
            q[sl] /= q[sl].sum()
        dk = ck * g.uniform(0.5, 1.5, size=ck.shape)
        dk *= c / dk.sum()
        for pp, cc in ((q, ck), (p, dk), (q, dk)):
            assert om.sum_variance_real(col, row, off, bp, pp, cc) >= best * (1 - 1e-12)


def test_integer_design_matches_real_formula_when_exact():
    # uniform probabilities and c = K * const: the integer design has exactly
    # the real-valued probabilities and sizes, so the two closed forms agree
    M, N, off = wl.random_problem(6, 40, 5, 4, seed=16, lo=10, hi=10)
    design, col, row, st = om.plan(M, N, off, 8, mode="stratified",
                                   prob="uniform", alloc="uniform")
    assert design.cs == [2, 2, 2, 2]
    bp = om.block_product_sq(M, N, off)
    p = np.full(40, 0.1)
    real = om.sum_variance_real(col, row, off, bp, p, np.array([2.0] * 4))
    assert math.isclose(om.expected_sq_error(M, N, design), real, rel_tol=1e-12)


def _block_rule_terms(M, N, off):
    """Per block, with library routines only: ||M^k N_k||_F (the block
    product multiplied out), F_k = ||M^k||_F ||N_k||_F, and ||MN||_F^2."""
    K = len(off) - 1
    x = np.array([np.linalg.norm(M[:, off[k]:off[k + 1]] @ N[off[k]:off[k + 1], :])
                  for k in range(K)])
    f = np.array([np.linalg.norm(M[:, off[k]:off[k + 1]]) * np.linalg.norm(N[off[k]:off[k + 1], :])
                  for k in range(K)])
    return x, f, float(np.linalg.norm(M @ N) ** 2)


@pytest.mark.parametrize("seed", range(4))
def test_block_rule_closed_forms(seed):
    # Substituting each block rule's p_k into the block-mode mean squared
    # error (1/c)(sum_k ||M^k N_k||_F^2 / p_k - ||MN||_F^2) gives
    #   uniform p_k = 1/K:         (1/c)(K sum_k x_k^2 - ||MN||^2)
    #   (1.4) p_k = F_k / sum F:   (1/c)(sum F * sum_k x_k^2 / F_k - ||MN||^2)
    #   (1.2) p_k = x_k / sum x:   (1/c)((sum_k x_k)^2 - ||MN||^2)
    # with x_k = ||M^k N_k||_F. The integer design samples p_hat = W / T,
    # which is within 2^-50 of p here, so the oracle's error of the design
    # matches these real-valued forms to 1e-12.
    M, N, off = wl.random_problem(7, 120, 6, 9, seed=40 + seed, skew=1.2)
    c = 5
    x, f, mn2 = _block_rule_terms(M, N, off)
    K = len(off) - 1
    want = {
        "uniform": (K * float(np.sum(x * x)) - mn2) / c,
        "norm": (float(np.sum(f)) * float(np.sum(x * x / f)) - mn2) / c,
        "exact": (float(np.sum(x)) ** 2 - mn2) / c,
    }
    for prob, ref in want.items():
        design, *_ = om.plan(M, N, off, c, mode="block", prob=prob)
        assert math.isclose(om.expected_sq_error(M, N, design), ref, rel_tol=1e-12), prob
    # (1.2) is the minimum of the block-mode error over all block
    # probabilities (Cauchy-Schwarz), strictly below the other two rules here
    assert want["exact"] < want["norm"] and want["exact"] < want["uniform"]


def test_block_rule_12_is_the_minimizer():
    # Any other positive block probabilities give a larger block-mode error
    # than (1.2); checked over random perturbations through user weights.
    M, N, off = wl.random_problem(6, 80, 5, 7, seed=51, skew=1.0)
    c = 4
    x, _, mn2 = _block_rule_terms(M, N, off)
    best, *_ = om.plan(M, N, off, c, mode="block", prob="exact")
    e_best = om.expected_sq_error(M, N, best)
    assert math.isclose(e_best, (float(np.sum(x)) ** 2 - mn2) / c, rel_tol=1e-12)
    g = wl.rng(52)
    for _ in range(50):
        w = x * g.uniform(0.3, 3.0, size=x.shape)
        d, *_ = om.plan(M, N, off, c, mode="block", prob="user", user_w=w)
        assert om.expected_sq_error(M, N, d) > e_best


def test_block_rule_12_hand_values():
    # Orthogonal outer products: block k's product is diagonal, so
    # ||M^k N_k||_F is the root of the sum of squares of its a_i b_i.
    # Blocks [3, 4] -> 5, [6, 8] -> 10, [12] -> 12: p_k = 5/27, 10/27, 12/27.
    M, N, off = _orthogonal_outer_products([3, 4, 6, 8, 12], [1] * 5, [0, 2, 4, 5])
    design, *_ = om.plan(M, N, off, 2, mode="block", prob="exact")
    assert np.allclose(design.p_hat(), [5 / 27, 10 / 27, 12 / 27], rtol=1e-15)
    # (1.4) on the same blocks: F_k = ||M^k||_F ||N_k||_F = 5 sqrt(2), 10 sqrt(2), 12
    design, *_ = om.plan(M, N, off, 2, mode="block", prob="norm")
    tot = 15 * math.sqrt(2) + 12
    assert np.allclose(design.p_hat(), [5 * math.sqrt(2) / tot, 10 * math.sqrt(2) / tot, 12 / tot],
                       rtol=1e-15)


def _orthogonal_outer_products(alpha, beta, blocks):
    """M, N whose outer products M^(i) N_(i) = alpha_i beta_i E_{i,i} are
    mutually orthogonal: a_i b_i = alpha_i beta_i and ||M^k N_k||_F^2 is the
    sum of (alpha_i beta_i)^2 over the block."""
    n = len(alpha)
    M = np.diag(np.asarray(alpha, np.float64))
    N = np.diag(np.asarray(beta, np.float64))
    return M, N, blocks


def test_alloc_rule_42_hand_values():
    # a_i b_i per block: [1, 3] -> s=4; [2, 2, 4] -> s=8; [4] -> s=4
    ab = [1, 3, 2, 2, 4, 4]
    M, N, off = _orthogonal_outer_products(ab, [1] * 6, [0, 2, 5, 6])
    design, *_ = om.plan(M, N, off, 32, mode="stratified", prob="norm", alloc="norm")
    assert design.cs == [8, 16, 8]                 # (4.2): c s_k / sum s


def test_alloc_rule_39_hand_values():
    # block 0: ab = [3, 4] -> s = 7, ||M^0 N_0||^2 = 9 + 16 = 25,
    #          (3.9) numerator sqrt(49 - 25) = sqrt(24)
    # block 1: ab = [5, 5] -> s = 10, ||.||^2 = 50, sqrt(100 - 50) = sqrt(50)
    # block 2: ab = [6] -> s = 6, ||.||^2 = 36, numerator 0 -> at least one
    #          draw is still required (Alg. 2 asks c_k >= 1)
    ab = [3, 4, 5, 5, 6]
    M, N, off = _orthogonal_outer_products(ab, [1] * 5, [0, 2, 4, 5])
    c = 100
    design, *_ = om.plan(M, N, off, c, mode="stratified", prob="norm", alloc="opt")
    r0 = c * math.sqrt(24) / (math.sqrt(24) + math.sqrt(50))   # 40.92...
    assert design.cs == [41, 58, 1]
    assert abs(design.cs[0] - r0) < 1.0
    # and the within-block probabilities are (3.8)
    assert np.allclose(design.p_hat(), [3 / 7, 4 / 7, 0.5, 0.5, 1.0], rtol=1e-15)


# --------------------------------------------------------------------------
# Monte Carlo with the real generator
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mode,prob,alloc", [("block", "norm", "norm"),
                                             ("stratified", "norm", "norm")])
def test_monte_carlo_unbiased(mode, prob, alloc):
    M, N, off = wl.random_problem(4, 24, 3, 4, seed=17, skew=0.7)
    design, *_ = om.plan(M, N, off, 6, mode=mode, prob=prob, alloc=alloc)
    MN = om.exact_product(M, N)
    T = 1500
    acc = np.zeros_like(MN)
    mse = []
    for t in range(T):
        d = om.sample(design, seed=3, trial=t)
        C, D = om.sketch(M, N, d)
        CD = C @ D
        acc += CD
        mse.append(float(np.sum((MN - CD) ** 2)))
    # per-entry standard error from the enumeration-checked variance
    ph = design.p_hat()
    var = np.zeros_like(MN)
    for s in range(len(design.T)):
        a0, a1 = design.strat_off[s], design.strat_off[s + 1]
        tot = np.zeros_like(MN)
        for a in range(a0, a1):
            lo, hi = int(design.atom_lo[a]), int(design.atom_hi[a])
            X = M[:, lo:hi] @ N[lo:hi, :]
            tot += X
            if ph[a] > 0:
                var += X * X / (design.cs[s] * ph[a])
        var -= tot * tot / design.cs[s]
    z = (acc / T - MN) / np.sqrt(np.maximum(var, 1e-300) / T)
    assert np.max(np.abs(z)) < 4.5
    e2 = om.expected_sq_error(M, N, design)
    se = np.std(mse) / math.sqrt(T)
    assert abs(np.mean(mse) - e2) < 5 * se


# --------------------------------------------------------------------------
# judge edge cases
# --------------------------------------------------------------------------

def test_judge_edges():
    z = np.zeros((3, 2))
    assert om.judge(z, z)[:2] == (0.0, 0.0)
    err, rel, *_ = om.judge(z, np.ones((3, 2)))
    assert err == math.sqrt(6) and rel == math.inf
    err, rel, *_ = om.judge(np.full((2, 2), 2.0), np.ones((2, 2)))
    assert err == 2.0 and rel == 0.5


def test_all_zero_problem():
    M = np.zeros((4, 10))
    N = np.ones((10, 3))
    r = om.run(M, N, [0, 5, 10], c=3, mode="block", prob="norm")
    assert r.draws.L == 0 and np.all(r.CD == 0) and r.err == 0.0 and r.rel == 0.0


def test_partition_checks():
    with pytest.raises(ValueError):
        om.check_partition([0, 3, 3, 5], 5)
    with pytest.raises(ValueError):
        om.check_partition([0, 5], 6)
    with pytest.raises(ValueError):
        om.check_partition([1, 5], 5)


# --------------------------------------------------------------------------
# gradient
# --------------------------------------------------------------------------

def test_backward_central_differences():
    M, N, off = wl.random_problem(16, 64, 12, 8, seed=18, lo=8, hi=8)
    design, *_ = om.plan(M, N, off, 4, mode="block", prob="norm")
    d = om.sample(design, seed=4)
    G = wl.rng(19).standard_normal((16, 12))
    dM, dN = om.backward(M, N, d, G)

    def f(Mx, Nx):
        C, D = om.sketch(Mx, Nx, d)
        return float(np.sum(G * (C @ D)))

    g = wl.rng(20)
    for _ in range(5):
        dirM = g.standard_normal(M.shape)
        dirN = g.standard_normal(N.shape)
        h = 1e-3
        fdM = (f(M + h * dirM, N) - f(M - h * dirM, N)) / (2 * h)
        fdN = (f(M, N + h * dirN) - f(M, N - h * dirN)) / (2 * h)
        assert math.isclose(fdM, float(np.sum(dM * dirM)), rel_tol=1e-9, abs_tol=1e-9)
        assert math.isclose(fdN, float(np.sum(dN * dirN)), rel_tol=1e-9, abs_tol=1e-9)
    # columns of unsampled blocks receive no gradient
    hit = np.zeros(64, bool)
    for lo, w in zip(d.lo, d.width):
        hit[lo:lo + w] = True
    assert np.all(dM[:, ~hit] == 0) and np.all(dN[~hit, :] == 0)


def test_backward_expectation_is_exact_gradient():
    g = wl.rng(21)
    M = g.standard_normal((3, 6))
    N = g.standard_normal((6, 2))
    G = g.standard_normal((3, 2))
    off = [0, 1, 3, 6]
    design, *_ = om.plan(M, N, off, 2, mode="block", prob="norm")
    EdM = np.zeros_like(M)
    EdN = np.zeros_like(N)
    for prob, combo in _enumerate(M, N, design):
        d = om.sample(design, 0, forced=combo)
        dM, dN = om.backward(M, N, d, G)
        EdM += prob * dM
        EdN += prob * dN
    assert _rel(EdM, G @ N.T) < 1e-12
    assert _rel(EdN, M.T @ G) < 1e-12


def test_backward_deterministic_case_exact():
    M, N, _ = wl.random_problem(5, 12, 4, 1, seed=22)
    G = wl.rng(23).standard_normal((5, 4))
    design, *_ = om.plan(M, N, [0, 12], 3, mode="block", prob="norm")
    d = om.sample(design, seed=1)
    dM, dN = om.backward(M, N, d, G)
    assert _rel(dM, G @ N.T) < 1e-13 and _rel(dN, M.T @ G) < 1e-13
