"""Pins of the oracle's probability error bounds (Thm 3.3 (3.11)-(3.12),
Thm 4.2 (4.3)-(4.4), Thm 4.4 (4.8)-(4.9)) against what the mathematics fixes
(CPU only):

* with theta_1 = theta_2 = theta the bounds of Thm 3.3 and Thm 4.2 coincide
  for any beta (phi = phi^ = sqrt(1 - beta + beta theta), sqrt(theta) at
  beta = 1, as the paper remarks);
* the variance bound (3.11) is at least the exact minimum (3.10) of the summed
  variance, and (4.3) at least the summed variance of the block sizes (4.2),
  both computed from their own closed forms on random problems;
* Thm 4.4 with exact pilot estimates is Thm 3.3;
* the bound scales as 1 / c and grows as delta shrinks;
* beta, the largest constant with p_hat >= beta (3.8), by brute force on a
  design whose probabilities are known.
"""
import math

import numpy as np
import pytest

from oracle import method as om


def _gen(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _stats(M, N, off):
    col, row = om.column_row_sq(M, N)
    off = om.check_partition(off, M.shape[1])
    return col, row, off, om.block_stats(col, row, off), om.block_product_sq(M, N, off)


def test_equal_blocks_make_thm33_and_thm42_coincide():
    g = _gen(1)
    A = g.standard_normal((6, 9))
    B = g.standard_normal((9, 5))
    M = np.concatenate([A, 2.0 * A, 0.5 * A], axis=1)      # every block has the same v_k
    N = np.concatenate([B, B, 3.0 * B], axis=0)
    col, row, off, st, bp = _stats(M, N, [0, 9, 18, 27])
    # with theta_1 = theta_2 = theta both phi reduce to sqrt(1 - beta + beta theta)
    # for any beta (sqrt(theta) at beta = 1) and both eta to phi + sqrt((8/beta) log(1/delta))
    for beta in (1.0, 0.7):
        for delta in (0.5, 0.1, 0.01):
            a = om.error_bound("opt", st, 100, beta, delta, bp)
            b = om.error_bound("norm", st, 100, beta, delta, bp)
            th = a["theta1"]
            assert th == pytest.approx(a["theta2"], rel=1e-12)
            assert a["phi"] == pytest.approx(math.sqrt(1 - beta + beta * th), rel=1e-9)
            assert b["phi"] == pytest.approx(a["phi"], rel=1e-9)
            assert a["bound"] == pytest.approx(b["bound"], rel=1e-9)
            assert a["eta"] == pytest.approx(a["phi"] + math.sqrt(8 / beta * math.log(1 / delta)), rel=1e-9)


@pytest.mark.parametrize("seed", range(6))
def test_variance_bounds_dominate_the_closed_forms(seed):
    g = _gen(10 + seed)
    M = g.standard_normal((8, 90)) * np.exp(g.normal(0, 1.2, 90))
    N = g.standard_normal((90, 7)) * np.exp(g.normal(0, 1.2, 90))[:, None]
    off = [0, 10, 25, 31, 50, 72, 90]
    col, row, off, st, bp = _stats(M, N, off)
    c = 40
    # (3.10): the minimum over real block sizes with the probabilities (3.8)
    opt = om.optimal_value(st, bp, c)
    assert opt <= om.error_bound("opt", st, c, 1.0, 0.1, bp)["var_bound"] * (1 + 1e-12)
    # (4.2) block sizes, probabilities (3.8): the summed variance in closed form
    p = np.sqrt(col * row)
    for k in range(len(off) - 1):
        p[off[k]:off[k + 1]] /= st.s[k]
    ck = c * st.s / st.s.sum()
    onc = om.sum_variance_real(col, row, off, bp, p, ck)
    assert onc <= om.error_bound("norm", st, c, 1.0, 0.1, bp)["var_bound"] * (1 + 1e-12)
    assert opt <= onc * (1 + 1e-12)


def test_two_step_bound_with_exact_estimates_is_thm33():
    g = _gen(3)
    M = g.standard_normal((5, 60)) * np.exp(g.normal(0, 1.0, 60))
    N = g.standard_normal((60, 4))
    col, row, off, st, bp = _stats(M, N, [0, 12, 30, 41, 60])
    a = om.error_bound("opt", st, 30, 0.97, 0.05, bp)
    b = om.error_bound("two_step", st, 30, 0.97, 0.05, bp, pilot_sq=bp)
    assert b["phi"] == pytest.approx(a["phi"], rel=1e-12)
    assert b["bound"] == pytest.approx(a["bound"], rel=1e-12)


def test_bound_scaling():
    g = _gen(4)
    M = g.standard_normal((5, 40))
    N = g.standard_normal((40, 4))
    col, row, off, st, bp = _stats(M, N, [0, 10, 20, 40])
    for rule in ("opt", "norm"):
        b1 = om.error_bound(rule, st, 10, 1.0, 0.1, bp)["bound"]
        b2 = om.error_bound(rule, st, 20, 1.0, 0.1, bp)["bound"]
        assert b2 == pytest.approx(b1 / 2, rel=1e-12)
        assert om.error_bound(rule, st, 10, 1.0, 0.01, bp)["bound"] > b1


def test_sampled_beta_brute_force():
    # uniform within-block probabilities compared with (3.8): beta is the
    # smallest ratio (1 / n_k) / (a_i b_i / s_k) over the atoms
    g = _gen(5)
    M = g.standard_normal((4, 30))
    N = g.standard_normal((30, 3))
    off = [0, 7, 19, 30]
    col, row = om.column_row_sq(M, N)
    st = om.block_stats(col, row, om.check_partition(off, 30))
    w = om.atom_weights("stratified", "uniform", off, col, row, st)
    design = om.make_design("stratified", off, 12, w, g=np.ones(3))
    want = 1.0
    ab = np.sqrt(col * row)
    for k in range(3):
        sl = slice(off[k], off[k + 1])
        want = min(want, float(np.min((1.0 / (off[k + 1] - off[k])) / (ab[sl] / ab[sl].sum()))))
    assert om.sampled_beta(design, col, row) == pytest.approx(want, rel=1e-12)
    # the quantized (3.8) probabilities themselves give beta = 1 up to rounding
    w38 = om.atom_weights("stratified", "norm", off, col, row, st)
    d38 = om.make_design("stratified", off, 12, w38, g=np.ones(3))
    assert 1 - 1e-12 <= om.sampled_beta(d38, col, row) <= 1.0


def _hand_problem(second):
    """Two blocks of two atoms, 3 rows, 1 column, ||M||_F^2 = ||N||_F^2 = 4.

    Block 0: columns e1, u = (1/2, sqrt(3)/2, 0) of M against rows 1, 1 of N:
    s_0 = 2, ||M^0 N_0||_F^2 = ||e1 + u||^2 = 3, so 1 - v_0^2 = 1/4.
    second = "zero": columns e1, e1 against rows 1, -1: the block product is
    0 and s_1 = 2, so 1 - v_1^2 = 1.
    second = "orth": columns e1, e2 against rows 1, 1: ||e1 + e2||^2 = 2,
    s_1 = 2, so 1 - v_1^2 = 1/2.
    """
    u = np.array([0.5, math.sqrt(3.0) / 2.0, 0.0])
    e1 = np.array([1.0, 0.0, 0.0])
    e2 = np.array([0.0, 1.0, 0.0])
    if second == "zero":
        M = np.stack([e1, u, e1, e1], axis=1)
        N = np.array([[1.0], [1.0], [1.0], [-1.0]])
    else:
        M = np.stack([e1, u, e1, e2], axis=1)
        N = np.array([[1.0], [1.0], [1.0], [1.0]])
    return _stats(M, N, [0, 2, 4])


def test_bounds_hand_values_unequal_theta():
    # theta_1 = 1/4, theta_2 = 1, c = 8, ||M||^2 ||N||^2 = 16, and
    # delta = exp(-1/8) so that sqrt((8/beta) log(1/delta)) = sqrt(1/beta).
    col, row, off, st, bp = _hand_problem("zero")
    assert st.s == pytest.approx([2.0, 2.0], rel=1e-15)
    assert bp == pytest.approx([3.0, 0.0], abs=1e-15)
    delta = math.exp(-1.0 / 8.0)
    c = 8
    r2 = math.sqrt(2.0)
    # Thm 3.3: phi = sqrt(1 - beta/4 + beta/4) / (1/4)^(1/4) = sqrt(2) for any
    # beta; eta = phi + (theta_2/theta_1)^(1/2) sqrt(1/beta) = sqrt(2) + 2 sqrt(1/beta)
    for beta, eta, bound in ((1.0, r2 + 2.0, 12.0 + 8.0 * r2),
                             (0.5, 3.0 * r2, 72.0)):
        b = om.error_bound("opt", st, c, beta, delta, bp)
        assert b["theta1"] == pytest.approx(0.25, rel=1e-14)
        assert b["theta2"] == 1.0
        assert b["phi"] == pytest.approx(r2, rel=1e-13)
        assert b["eta"] == pytest.approx(eta, rel=1e-13)
        assert b["var_bound"] == pytest.approx(2.0 / (beta * c) * 16.0, rel=1e-13)
        assert b["bound"] == pytest.approx(bound, rel=1e-13)
    # Thm 4.2: phi^ = sqrt(1 - beta (1 - theta_2)) = 1; eta = 1 + sqrt(1/beta)
    for beta, bound in ((1.0, 8.0), (0.5, 12.0 + 8.0 * r2)):
        b = om.error_bound("norm", st, c, beta, delta, bp)
        assert b["phi"] == pytest.approx(1.0, rel=1e-14)
        assert b["bound"] == pytest.approx(bound, rel=1e-13)
    # Thm 4.4 with pilot estimates 3 and 20: |1 - v^_k^2| = 1/4 and
    # |1 - 20/4| = 4, so theta^_1 = 1/4, theta^_2 = 4 while the exact theta_2
    # stays 1: phi~ = sqrt(4 - beta/4 + 1 * beta/4) / (4 * 1/4)^(1/4) = 2 and
    # eta = 2 + (theta^_2/theta^_1)^(1/2) = 2 + 4 = 6 at beta = 1
    b = om.error_bound("two_step", st, c, 1.0, delta, bp, pilot_sq=[3.0, 20.0])
    assert b["theta1_hat"] == pytest.approx(0.25, rel=1e-14)
    assert b["theta2_hat"] == pytest.approx(4.0, rel=1e-14)
    assert b["phi"] == pytest.approx(2.0, rel=1e-13)
    assert b["eta"] == pytest.approx(6.0, rel=1e-13)
    assert b["var_bound"] == pytest.approx(8.0, rel=1e-13)
    assert b["bound"] == pytest.approx(72.0, rel=1e-13)


def test_bounds_hand_values_beta_terms():
    # theta_1 = 1/4, theta_2 = 1/2, beta = 1/2, c = 8:
    # Thm 3.3 phi^2 = (1/2 - 1/8 + 1/16) / (1/8)^(1/2) = 7 sqrt(2) / 8,
    #         variance bound phi^2 / (beta c) * 16 = 7 sqrt(2) / 2;
    # Thm 4.2 phi^2 = 1 - (1/2)(1/2) = 3/4, variance bound 3.
    col, row, off, st, bp = _hand_problem("orth")
    assert bp == pytest.approx([3.0, 2.0], rel=1e-15)
    a = om.error_bound("opt", st, 8, 0.5, 0.1, bp)
    assert a["theta1"] == pytest.approx(0.25, rel=1e-14)
    assert a["theta2"] == pytest.approx(0.5, rel=1e-14)
    assert a["phi"] ** 2 == pytest.approx(7.0 * math.sqrt(2.0) / 8.0, rel=1e-13)
    assert a["var_bound"] == pytest.approx(7.0 * math.sqrt(2.0) / 2.0, rel=1e-13)
    b = om.error_bound("norm", st, 8, 0.5, 0.1, bp)
    assert b["phi"] ** 2 == pytest.approx(0.75, rel=1e-14)
    assert b["var_bound"] == pytest.approx(3.0, rel=1e-13)
