"""The probability error bounds of Thm 3.3 (block sizes (3.9)), Thm 4.2
((4.2)) and Thm 4.4 ((4.7), the two-step algorithm) and the expected squared
error of the sampled design, evaluated by sbmm_bound on the GPU, against the
oracle on the same seeded inputs; then the bounds' claims checked
empirically over many trials of the GPU path: the mean squared error matches
the expected one, and the squared error exceeds the bound of delta in at most
a fraction delta of the trials."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import method as om

torch = pytest.importorskip("torch")
import paper_2105_04940_amd as pk  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
DELTAS = (0.5, 0.1, 0.01)
RTOL = 1e-10


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hd = pk.Handle(0)
    yield hd
    hd.close()


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host64(t):
    return t.detach().double().cpu().numpy()


def gpu_bound(h, prob, beta=0.0, deltas=DELTAS, blkprod=None):
    col, row, blk = h.norms(prob)
    _, bp, _ = h.exact(prob, store=False, blocknorm=True)
    if blkprod is not None:
        bp = blkprod(blk, bp)
    if prob.alloc == "two_step":
        prob.pilot_sq = h.pilot(prob, col, row, blk)
    if prob.alloc == "opt":
        prob.blkprod_sq = bp
    pl = h.plan(prob, col, row, blk)
    return h.bound(prob, col, row, blk, bp, pl, beta=beta, deltas=deltas), pl


def oracle_bound(M, N, off, c, prob, alloc, seed, trial, c0=None, pilot_prob=None, beta=0.0,
                 deltas=DELTAS, blkprod=None):
    col, row = om.column_row_sq(M, N)
    offc = om.check_partition(off, M.shape[1])
    st = om.block_stats(col, row, offc)
    bp = om.block_product_sq(M, N, offc)
    if blkprod is not None:
        bp = blkprod(st, bp)
    psq = None
    if alloc == "two_step":
        psq = om.pilot(M, N, off, c0, pilot_prob, seed, trial, (col, row)).pilot_sq
    design, _, _, _ = om.plan(M, N, off, c, "stratified", prob, alloc, blkprod_sq=bp,
                              col_row=(col, row), pilot_sq=psq)
    b = beta if beta > 0 else om.sampled_beta(design, col, row)
    rule = alloc
    res = [om.error_bound(rule, st, c, b, d, bp, psq) for d in deltas]
    exp = om.expected_sq_error(M, N, design) if blkprod is None else None
    return res, b, exp, design


def close(a, b, rtol=RTOL):
    if math.isinf(b):
        return math.isinf(a) and a > 0
    return abs(a - b) <= rtol * max(abs(b), 1e-300)


CASES = [
    ("norm", "opt", None, None),
    ("norm", "norm", None, None),
    ("norm", "two_step", 60, "uniform"),
    ("norm", "two_step", 60, "norm"),
    ("uniform", "norm", None, None),   # beta well below 1
    ("uniform", "opt", None, None),
]


@pytest.mark.parametrize("prob,alloc,c0,pilot", CASES)
def test_bound_matches_oracle(h, prob, alloc, c0, pilot):
    M, N, off = wl.random_problem(26, 6000, 28, 7, seed=31, skew=1.2)
    c, seed, trial = 900, 4, 2
    P = pk.Problem(to_dev(M), to_dev(N), off, c, mode="stratified", prob=prob, alloc=alloc,
                   c0=c0 or 0, pilot=pilot or "uniform", seed=seed, trial=trial)
    g, pl = gpu_bound(h, P)
    res, beta, exp, design = oracle_bound(M, N, off, c, prob, alloc, seed, trial, c0, pilot)
    assert pl.ck.cpu().tolist() == design.cs
    assert close(g["beta"], beta)
    if prob == "norm":
        assert 1 - 1e-12 <= g["beta"] <= 1.0
    else:
        assert g["beta"] < 0.5
    r0 = res[0]
    for f in ("theta1", "theta2", "phi"):
        assert close(g[f], r0[f]), f
    if alloc == "two_step":
        assert close(g["theta1_hat"], r0["theta1_hat"]) and close(g["theta2_hat"], r0["theta2_hat"])
    else:
        assert g["theta1_hat"] == 0.0 and g["theta2_hat"] == 0.0
    assert close(g["var_bound"], r0["var_bound"])
    assert close(g["mn"], math.fsum(np.sum(M * M, 0)) * math.fsum(np.sum(N * N, 1)))
    for j, r in enumerate(res):
        assert close(g["eta"][j], r["eta"]) and close(g["bound"][j], r["bound"])
    assert close(g["expected"], exp, 1e-9)
    # the expected error of the realized design lies below the variance bound
    assert g["expected"] <= g["var_bound"]


def test_bound_given_beta(h):
    M, N, off = wl.random_problem(10, 3000, 12, 5, seed=32, skew=0.8)
    P = pk.Problem(to_dev(M), to_dev(N), off, 300, mode="stratified", prob="norm", alloc="norm", seed=1)
    g, _ = gpu_bound(h, P, beta=0.6, deltas=(0.05,))
    res, _, _, _ = oracle_bound(M, N, off, 300, "norm", "norm", 1, 0, beta=0.6, deltas=(0.05,))
    assert g["beta"] == 0.6
    assert close(g["phi"], res[0]["phi"]) and close(g["bound"][0], res[0]["bound"])
    assert len(g["eta"]) == 1


def test_bound_opt_theta1_zero_is_infinite(h):
    # with ||M^0 N_0||_F = s_0 (v_0 = 1, theta_1 = 0), Thm 3.3 divides by
    # zero: phi, eta and the bounds are +inf on both sides
    M, N, off = wl.random_problem(12, 2000, 9, 4, seed=33, skew=0.5)

    def gpu_bp(blk, bp):
        K = bp.numel()
        bp = bp.clone()
        bp[0] = blk[2 * K] * blk[2 * K]
        return bp

    def ora_bp(st, bp):
        bp = bp.copy()
        bp[0] = st.s[0] * st.s[0]
        return bp

    P = pk.Problem(to_dev(M), to_dev(N), off, 200, mode="stratified", prob="norm", alloc="norm", seed=2)
    g, _ = gpu_bound(h, P, blkprod=gpu_bp)
    res, _, _, _ = oracle_bound(M, N, off, 200, "norm", "norm", 2, 0, blkprod=ora_bp)
    assert g["theta1"] == 0.0 and res[0]["theta1"] == 0.0
    P2 = pk.Problem(to_dev(M), to_dev(N), off, 200, mode="stratified", prob="norm", alloc="opt", seed=2)
    col, row, blk = h.norms(P2)
    _, bp, _ = h.exact(P2, store=False, blocknorm=True)
    P2.blkprod_sq = bp
    pl = h.plan(P2, col, row, blk)
    g2 = h.bound(P2, col, row, blk, gpu_bp(blk, bp), pl, deltas=(0.1,))
    r2 = om.error_bound("opt", om.block_stats(*om.column_row_sq(M, N), om.check_partition(off, 2000)),
                        200, g2["beta"], 0.1, ora_bp(om.block_stats(*om.column_row_sq(M, N),
                                                                    om.check_partition(off, 2000)),
                                                     om.block_product_sq(M, N, off)))
    assert math.isinf(r2["phi"]) and math.isinf(g2["phi"]) and math.isinf(g2["bound"][0])


def test_bound_zero_matrix(h):
    # M = 0: no block has s_k > 0, nothing is drawn, every bound is 0
    M = np.zeros((6, 500))
    N = np.random.Generator(np.random.PCG64(3)).standard_normal((500, 5))
    off = [0, 100, 350, 500]
    P = pk.Problem(to_dev(M), to_dev(N), off, 10, mode="stratified", prob="norm", alloc="norm")
    g, pl = gpu_bound(h, P)
    assert pl.ck.cpu().tolist() == [0, 0, 0]
    for f in ("theta1", "theta2", "phi", "var_bound", "expected"):
        assert g[f] == 0.0
    assert g["bound"] == [0.0, 0.0, 0.0] and g["mn"] == 0.0 and g["beta"] == 1.0


def test_bound_rejects(h):
    M, N, off = wl.random_problem(8, 400, 6, 4, seed=34)
    Md, Nd = to_dev(M), to_dev(N)
    P = pk.Problem(Md, Nd, off, 40, mode="stratified", prob="norm", alloc="norm")
    col, row, blk = h.norms(P)
    _, bp, _ = h.exact(P, store=False, blocknorm=True)
    pl = h.plan(P, col, row, blk)
    bad = [
        (P, dict(deltas=(1.0,))), (P, dict(deltas=(0.0,))), (P, dict(deltas=(0.1,) * 9)),
        (P, dict(beta=1.5)), (P, dict(beta=-0.1)),
        (pk.Problem(Md, Nd, off, 40, mode="stratified", prob="norm", alloc="uniform"), {}),
        (pk.Problem(Md, Nd, off, 40, mode="block", prob="norm"), {}),
        (pk.Problem(Md, Nd, off, 40, mode="stratified", prob="norm", alloc="two_step", c0=8), {}),
    ]
    for prob, kw in bad:
        with pytest.raises(pk.SbmmError) as ei:
            h.bound(prob, col, row, blk, bp, pl, **kw)
        assert ei.value.status == pk.SBMM_E_ARG
    with pytest.raises(pk.SbmmError):
        h.bound(P, col, row, blk, None, pl)


@pytest.mark.parametrize("alloc", ["opt", "norm", "two_step"])
def test_bound_empirical_coverage(h, alloc):
    # R independent trials of the GPU path: the mean of ||MN - CD||_F^2
    # matches E ||MN - CD||_F^2 of the design (within 5 standard errors; for
    # the two-step algorithm the design changes with the pilot, so the mean
    # of the per-trial expectations is the target), and the squared error
    # exceeds the bound of delta in at most a fraction delta (+ 3 binomial
    # standard deviations) of the trials
    M, N, off = wl.random_problem(26, 20000, 28, 5, seed=35, skew=1.0)
    R = 200 if alloc != "two_step" else 80
    Md, Nd = to_dev(M), to_dev(N)
    errs, exps, bounds = [], [], []
    for t in range(R):
        P = pk.Problem(Md, Nd, off, 1500, mode="stratified", prob="norm", alloc=alloc,
                       c0=100, pilot="norm", seed=9, trial=t)
        col, row, blk = h.norms(P)
        _, bp, _ = h.exact(P, store=False, blocknorm=True)
        if alloc == "opt":
            P.blkprod_sq = bp
        if alloc == "two_step":
            P.pilot_sq = h.pilot(P, col, row, blk)
        r = h.run(P, want_C=False, want_D=False)
        g = h.bound(P, col, row, blk, bp, r["plan"], deltas=DELTAS)
        errs.append(r["err"] ** 2)
        exps.append(g["expected"])
        bounds.append(g["bound"])
    errs = np.array(errs)
    target = float(np.mean(exps))
    se = float(np.std(errs, ddof=1)) / math.sqrt(R)
    assert abs(float(np.mean(errs)) - target) <= 5 * se
    for j, d in enumerate(DELTAS):
        frac = float(np.mean(errs > np.array([b[j] for b in bounds])))
        assert frac <= d + 3 * math.sqrt(d * (1 - d) / R)
