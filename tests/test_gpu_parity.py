"""Parity of the HIP path with the float64 oracle, element by element, on
seeded inputs that span several tiles and ragged tails.

Bars: indices, counts and offsets bit-exact; float64 outputs within a
relative Frobenius error of 1e-12, float32 outputs within 1e-5 (the
tolerances the method's accuracy targets state); bf16 inputs are compared on
their exactly promoted values.
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import method as om

torch = pytest.importorskip("torch")
import paper_2105_04940_amd as pk  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {torch.float64: 1e-12, torch.float32: 1e-5}


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hd = pk.Handle(0)
    yield hd
    hd.close()


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    d = np.linalg.norm(a - b)
    return d / nb if nb > 0 else d


def to_dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV).to(dtype)


def host64(t):
    return t.detach().to("cpu").to(torch.float64).numpy()


def oracle_run(Mh, Nh, off, c, **kw):
    return om.run(Mh, Nh, off, c, **kw)


# --------------------------------------------------------------------------
# norm pass
# --------------------------------------------------------------------------

NORM_SHAPES = [(1, 7, 1, [0, 3, 7]), (37, 129, 65, [0, 1, 50, 129]),
               (300, 1000, 200, None), (5, 3000, 3, None), (70, 513, 1030, None)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
@pytest.mark.parametrize("shape", NORM_SHAPES)
def test_norms(h, dtype, shape):
    m, n, p, off = shape
    M, N, off2 = wl.random_problem(m, n, p, max(1, n // 40), seed=m + n + p, skew=1.0)
    off = off or off2
    Md, Nd = to_dev(M, dtype), to_dev(N, dtype)
    prob = pk.Problem(Md, Nd, off, c=3)
    col, row, blk = h.norms(prob)
    torch.cuda.synchronize()
    Mh, Nh = host64(Md), host64(Nd)
    ocol, orow = om.column_row_sq(Mh, Nh)
    st = om.block_stats(ocol, orow, off)
    assert rel(host64(col), ocol) < 1e-13
    assert rel(host64(row), orow) < 1e-13
    K = len(off) - 1
    b = host64(blk)
    assert rel(b[:K], st.m_sq) < 1e-13
    assert rel(b[K:2 * K], st.n_sq) < 1e-13
    assert rel(b[2 * K:], st.s) < 1e-13


def test_norms_strided_rows(h):
    # leading dimensions larger than the row length, unaligned for 16-byte loads
    M, N, off = wl.random_problem(33, 301, 45, 7, seed=5)
    big_m = to_dev(np.pad(M, ((0, 0), (0, 3))), torch.float32)[:, :301]
    big_n = to_dev(np.pad(N, ((0, 0), (0, 5))), torch.float32)[:, :45]
    col, row, blk = h.norms(pk.Problem(big_m, big_n, off, c=2))
    torch.cuda.synchronize()
    ocol, orow = om.column_row_sq(M.astype(np.float32).astype(np.float64),
                                  N.astype(np.float32).astype(np.float64))
    assert rel(host64(col), ocol) < 1e-13 and rel(host64(row), orow) < 1e-13


@pytest.mark.parametrize("K", [1, 4, 10, 40])
def test_norms_wide_blocks(h, K):
    # blocks of 5e5 / K columns: the block statistics run in chunks of
    # columns per block and are combined in chunk order (K = 40: 12 500
    # columns, 7 chunks; K = 1: 245 chunks)
    g = np.random.Generator(np.random.PCG64(K))
    n = 500000
    M = g.standard_normal((6, n)) * np.exp(g.normal(0, 1.0, n))
    N = g.standard_normal((n, 5))
    off = wl.equal_blocks(n, K)
    prob = pk.Problem(to_dev(M, torch.float64), to_dev(N, torch.float64), off, c=3)
    col, row, blk = h.norms(prob)
    torch.cuda.synchronize()
    ocol, orow = om.column_row_sq(M, N)
    st = om.block_stats(ocol, orow, off)
    b = host64(blk)
    assert rel(host64(col), ocol) < 1e-13
    assert rel(b[:K], st.m_sq) < 1e-13 and rel(b[K:2 * K], st.n_sq) < 1e-13 and rel(b[2 * K:], st.s) < 1e-13


def test_partition_changes_between_calls(h):
    # one handle, the same inputs under partitions that alternate (same K,
    # then another K, then the first again): each call uses its own offsets
    M, N, _ = wl.random_problem(20, 3000, 15, 5, seed=77)
    Md, Nd = to_dev(M, torch.float64), to_dev(N, torch.float64)
    ocol, orow = om.column_row_sq(M, N)
    offs = [[0, 700, 1500, 3000], [0, 100, 2900, 3000], [0, 1000, 2000, 2500, 2999, 3000],
            [0, 700, 1500, 3000]]
    for off in offs + offs[::-1]:
        col, row, blk = h.norms(pk.Problem(Md, Nd, off, c=4))
        torch.cuda.synchronize()
        st = om.block_stats(ocol, orow, off)
        K = len(off) - 1
        assert rel(host64(blk)[2 * K:], st.s) < 1e-13, off
        assert rel(host64(blk)[:K], st.m_sq) < 1e-13, off


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_exact_error(h, dtype):
    # the exact product with the judge of a given CD in its epilogue, MN and
    # the per-block norms beside it, against the oracle and the run's error
    M, N, off = wl.random_problem(130, 3000, 70, 30, seed=41, skew=0.8)
    prob = pk.Problem(to_dev(M, dtype), to_dev(N, dtype), off, 100, prob="norm", seed=1)
    r = h.run(prob)
    out, MN, bp = h.exact_error(prob, r["CD"], store=True, blocknorm=True)
    torch.cuda.synchronize()
    Mh, Nh = host64(prob.M), host64(prob.N)
    MNo = om.exact_product(Mh, Nh)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    e2 = float(np.sum((host64(r["CD"]) - MNo) ** 2))
    assert abs(out[0].item() - e2) <= tol * e2
    assert abs(out[1].item() - float(np.sum(MNo ** 2))) <= tol * float(np.sum(MNo ** 2))
    # the run's own judge: the same sums in float64; with float32 products the
    # block-norm form of the product accumulates MN in another order
    assert abs(math.sqrt(out[0].item()) - r["err"]) <= tol * r["err"]
    assert rel(host64(MN), MNo) < tol
    assert rel(host64(bp), om.block_product_sq(Mh, Nh, off)) < tol
    with pytest.raises(pk.SbmmError):   # CD in another dtype than the product's
        h.exact_error(prob, r["CD"].to(torch.float32 if dtype == torch.float64 else torch.float64))


def test_reserved_workspace_needs_no_allocation():
    # after sbmm_reserve(sbmm_workspace_size(...)) the problem's calls on a
    # fresh handle allocate no device memory (torch's outputs are served from
    # its cache, warmed by the same calls on another handle)
    M, N, off = wl.random_problem(96, 20000, 80, 10, seed=43, skew=1.0)
    Md, Nd = to_dev(M, torch.float64), to_dev(N, torch.float64)

    def calls(hd):
        prob = pk.Problem(Md, Nd, off, 3000, mode="stratified", prob="norm", alloc="two_step", c0=500,
                          pilot="norm", seed=3)
        col, row, blk = hd.norms(prob)
        _, bp, _ = hd.exact(prob, store=False, blocknorm=True)
        prob.pilot_sq = hd.pilot(prob, col, row, blk)
        pl = hd.plan(prob, col, row, blk)
        g = hd.bound(prob, col, row, blk, bp, pl, deltas=(0.1,))
        r = hd.run(prob)
        out, _, _ = hd.exact_error(prob, r["CD"], blocknorm=True)
        torch.cuda.synchronize()
        return r["err"], g["bound"][0], out[0].item()

    h0 = pk.Handle(0)
    ref = calls(h0)
    calls(h0)
    h0.close()
    prob = pk.Problem(Md, Nd, off, 3000, mode="stratified", prob="norm", alloc="two_step", c0=500, pilot="norm")
    nbytes, _ = pk.sbmm_workspace_size(prob)
    h1 = pk.Handle(0)
    h1.reserve(nbytes)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    got = calls(h1)
    free1 = torch.cuda.mem_get_info()[0]
    h1.close()
    assert got == ref
    assert free1 == free0


@pytest.mark.parametrize("m,n,p", [(300, 2001, 259), (257, 4099, 513), (64, 130, 33)])
def test_f32_products_with_ragged_extents(h, m, n, p):
    # float32 rows padded to 16 bytes but n, p not multiples of 4: the
    # 256 x 256 product's per-dword zero fill of the last rows and its
    # clearing of the entries past the inner extent, on the exact product
    # and on the sketched one (D rows of p entries), against the oracle
    g = np.random.Generator(np.random.PCG64(m + n + p))
    Mb = torch.from_numpy(g.standard_normal((m, (n + 3) // 4 * 4)).astype(np.float32)).to(DEV)
    Nb = torch.from_numpy(g.standard_normal((n, (p + 3) // 4 * 4)).astype(np.float32)).to(DEV)
    # garbage in the padding must not reach the results
    Mb[:, n:] = float("nan")
    Nb[:, p:] = float("nan")
    M, N = Mb[:, :n], Nb[:, :p]
    off = wl.equal_blocks(n, 1) if n % 3 else wl.equal_blocks(n, 3)
    prob = pk.Problem(M, N, off, 40, prob="norm", seed=5)
    MN, _, mn_sq = h.exact(prob, store=True)
    torch.cuda.synchronize()
    Mh, Nh = host64(M), host64(N)
    MNo = om.exact_product(Mh, Nh)
    assert rel(host64(MN), MNo) < 1e-5
    assert abs(mn_sq.item() - float(np.sum(MNo ** 2))) <= 1e-5 * float(np.sum(MNo ** 2))
    r = h.run(prob)
    o = om.run(Mh, Nh, off, 40, seed=5, prob="norm")
    assert np.array_equal(r["plan"].idx.cpu().numpy(), o.draws.atom)
    assert rel(host64(r["CD"]), o.CD) < 1e-5


def test_norms_bitwise_reproducible(h):
    M, N, off = wl.random_problem(200, 4000, 150, 40, seed=9)
    prob = pk.Problem(to_dev(M, torch.float32), to_dev(N, torch.float32), off, c=4)
    a = [t.clone() for t in h.norms(prob)]
    b = h.norms(prob)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


# --------------------------------------------------------------------------
# design + sampling with the same weight vector: bit-exact
# --------------------------------------------------------------------------

def _user_weights(n_atoms, seed, zeros=0.2):
    g = wl.rng(seed)
    w = g.lognormal(0, 2, size=n_atoms)
    w[g.random(n_atoms) < zeros] = 0.0
    if not np.any(w > 0):
        w[0] = 1.0
    return w


@pytest.mark.parametrize("K,c,seed", [(64, 16, 0), (1024, 256, 1), (7, 300, 2), (1, 5, 3),
                                      (20000, 5000, 4)])   # design in chunks, offsets on many workgroups
def test_plan_block_user_weights_bit_exact(h, K, c, seed):
    n = K * 3
    off = wl.equal_blocks(n, K)
    M = np.zeros((2, n))
    N = np.zeros((n, 2))
    w = _user_weights(K, seed)
    prob = pk.Problem(to_dev(M, torch.float64), to_dev(N, torch.float64), off, c,
                      prob="user", user_w=to_dev(w, torch.float64), seed=seed * 77 + 1,
                      trial=seed)
    pl = h.plan(prob)
    design = om.make_design("block", off, c, w)
    draws = om.sample(design, seed * 77 + 1, seed)
    assert np.array_equal(pl.idx.cpu().numpy(), draws.atom)
    assert np.array_equal(pl.scale.cpu().numpy(), draws.scale)      # bitwise
    assert np.array_equal(pl.col_off.cpu().numpy(), draws.col_off)
    assert pl.L == draws.L
    assert pl.ck.cpu().tolist() == design.cs
    assert np.array_equal(pl.p_hat.cpu().numpy(), design.p_hat())
    cm = pl.colmap.cpu().numpy()
    cs = pl.colscale.cpu().numpy()
    exp = np.concatenate([np.arange(lo, lo + wd) for lo, wd in zip(draws.lo, draws.width)])
    assert np.array_equal(cm[:draws.L], exp)
    Lp = -(-draws.L // 32) * 32
    assert np.all(cm[draws.L:Lp] == -1) and np.all(cs[draws.L:Lp] == 0)


@pytest.mark.parametrize("alloc", ["uniform", "user"])
def test_plan_stratified_user_weights_bit_exact(h, alloc):
    off = [0, 5, 17, 18, 60, 100]
    n = 100
    w = _user_weights(n, 11, zeros=0.3)
    w[17] = 1.0   # block 2 (one atom) must be sampleable
    c = 40
    ck = None
    if alloc == "user":
        T = [np.any(w[off[k]:off[k + 1]] > 0) for k in range(5)]
        ck = [8 if t else 0 for t in T]
        ck[int(np.argmax(T))] += c - sum(ck)
    M = np.zeros((1, n))
    N = np.zeros((n, 1))
    prob = pk.Problem(to_dev(M, torch.float64), to_dev(N, torch.float64), off, c,
                      mode="stratified", prob="user", alloc=alloc,
                      user_w=to_dev(w, torch.float64), user_ck=ck, seed=5, trial=9)
    col, row, blk = h.norms(prob)
    pl = h.plan(prob, col, row, blk)
    g = np.ones(5) if alloc == "uniform" else None
    design = om.make_design("stratified", off, c, w, g=g, user_ck=ck)
    draws = om.sample(design, 5, 9)
    assert pl.ck.cpu().tolist() == design.cs
    assert np.array_equal(pl.idx.cpu().numpy(), draws.atom)
    assert np.array_equal(pl.scale.cpu().numpy(), draws.scale)
    assert np.array_equal(pl.col_off.cpu().numpy(), draws.col_off)


@pytest.mark.parametrize("alloc", ["uniform", "user"])
def test_plan_wide_strata_bit_exact(h, alloc):
    # strata of up to 20 000 atoms: the design runs in chunks of 2048 atoms per
    # stratum and the draw offsets on many workgroups; W, CDF, T, p_hat and the
    # draws are those of the oracle bit for bit
    off = [0, 20000, 31999, 32000, 50000]
    n = 50000
    w = _user_weights(n, 12, zeros=0.3)
    w[31999] = 2.5
    c = 3000
    ck = [1000, 700, 300, 1000] if alloc == "user" else None
    M = np.zeros((1, n))
    N = np.zeros((n, 1))
    prob = pk.Problem(to_dev(M, torch.float64), to_dev(N, torch.float64), off, c,
                      mode="stratified", prob="user", alloc=alloc,
                      user_w=to_dev(w, torch.float64), user_ck=ck, seed=6, trial=2)
    col, row, blk = h.norms(prob)
    pl = h.plan(prob, col, row, blk)
    g = np.ones(4) if alloc == "uniform" else None
    design = om.make_design("stratified", off, c, w, g=g, user_ck=ck)
    draws = om.sample(design, 6, 2)
    assert pl.ck.cpu().tolist() == design.cs
    assert np.array_equal(pl.p_hat.cpu().numpy(), design.p_hat())
    assert np.array_equal(pl.idx.cpu().numpy(), draws.atom)
    assert np.array_equal(pl.scale.cpu().numpy(), draws.scale)
    assert np.array_equal(pl.col_off.cpu().numpy(), draws.col_off)
    assert pl.L == draws.L == c


# --------------------------------------------------------------------------
# end to end
# --------------------------------------------------------------------------

def _check_run(h, M, N, off, c, dtype, **kw):
    Md, Nd = to_dev(M, dtype), to_dev(N, dtype)
    prob = pk.Problem(Md, Nd, off, c, **kw)
    r = h.run(prob)
    Mh, Nh = host64(Md), host64(Nd)
    okw = {k: v for k, v in kw.items() if k in ("seed", "trial", "mode", "prob", "alloc", "c0")}
    if "pilot" in kw:
        okw["pilot_prob"] = kw["pilot"]
    o = oracle_run(Mh, Nh, off, c, **okw)
    tol = TOL[dtype]
    idx = r["plan"].idx.cpu().numpy()
    if not np.array_equal(idx, o.draws.atom):
        # only a change of the integer weights (from last-bit differences of
        # the float64 norms) could explain this; report which case it is
        same_p = np.array_equal(r["plan"].p_hat.cpu().numpy(), o.design.p_hat())
        pytest.fail(f"indices differ (sampled probabilities identical: {same_p})")
    assert r["L"] == o.draws.L
    L = o.draws.L
    Lp = -(-L // 32) * 32
    C, D = host64(r["C"]), host64(r["D"])
    # the scales agree to the last bit when the weights do; the norms (summed
    # in another order) may move a weight by an ulp
    ctol = 1e-15 if dtype == torch.float64 else 1e-7
    assert rel(C[:, :L], o.C) <= ctol
    assert rel(D[:L], o.D) <= ctol
    assert np.all(C[:, L:Lp] == 0) and np.all(D[L:Lp] == 0)
    assert rel(host64(r["CD"]), o.CD) < tol
    assert rel(host64(r["MN"]), o.MN) < tol
    if o.err > 0:
        assert abs(r["err"] - o.err) <= tol * max(o.err, 1e-300) + tol * np.linalg.norm(o.MN)
        assert abs(r["rel"] - o.rel) <= tol * max(o.rel, 1.0)
    return r, o


def test_tiny_workload_f64(h):
    M, N, off = wl.tiny(0)
    r, o = _check_run(h, M, N, off, 16, torch.float64, seed=0)
    assert r["L"] == 256
    assert abs(r["rel"] - o.rel) < 1e-12 * o.rel


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", [(300, 2000, 260, 50, 37), (129, 777, 65, 13, 5),
                                   (1, 64, 1, 4, 3), (513, 4100, 7, 80, 64)])
def test_block_norm_ragged(h, dtype, shape):
    m, n, p, K, c = shape
    M, N, off = wl.random_problem(m, n, p, K, seed=m * 7 + p, skew=1.2)
    _check_run(h, M, N, off, c, dtype, seed=3, trial=1)


@pytest.mark.parametrize("prob", ["uniform", "exact"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_block_other_rules(h, prob, dtype):
    M, N, off = wl.random_problem(200, 1500, 170, 30, seed=12, skew=1.0)
    _check_run(h, M, N, off, 20, dtype, prob=prob, seed=4)


@pytest.mark.parametrize("prob,alloc", [("uniform", "uniform"), ("norm", "norm"),
                                        ("norm", "opt"), ("norm", "uniform")])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_stratified_rules(h, prob, alloc, dtype):
    M, N, off = wl.random_problem(26, 3000, 28, 6, seed=21, skew=1.5)
    r, o = _check_run(h, M, N, off, 600, dtype, mode="stratified", prob=prob, alloc=alloc,
                      seed=8, trial=2)
    assert r["plan"].ck.cpu().tolist() == o.design.cs


def test_block_product_norms(h):
    for dtype in (torch.float64, torch.float32):
        M, N, off = wl.random_problem(150, 1300, 140, 17, seed=31, skew=0.8)
        prob = pk.Problem(to_dev(M, dtype), to_dev(N, dtype), off, c=3)
        MN, bp, mn_sq = h.exact(prob, store=True, blocknorm=True)
        torch.cuda.synchronize()
        Mh, Nh = host64(prob.M), host64(prob.N)
        ref = om.block_product_sq(Mh, Nh, off)
        assert rel(host64(bp), ref) < TOL[dtype]
        MNo = om.exact_product(Mh, Nh)
        assert rel(host64(MN), MNo) < TOL[dtype]
        assert abs(mn_sq.item() - float(np.sum(MNo**2))) < TOL[dtype] * float(np.sum(MNo**2))


def test_block_gram_tile_counts(h):
    # per block, against the oracle: widths giving every count of 16-wide
    # index tiles (1..8), on and off the tile edges, row and column extents
    # that leave ragged contraction steps
    widths = [1, 15, 16, 17, 31, 32, 33, 48, 63, 64, 65, 80, 97, 100, 112, 113, 127, 128, 2, 7, 50]
    off = [0]
    for wdt in widths:
        off.append(off[-1] + wdt)
    M, N, _ = wl.random_problem(150, off[-1], 70, 1, seed=41, skew=0.8)
    prob = pk.Problem(to_dev(M, torch.float32), to_dev(N, torch.float32), off, c=3)
    _, bp, _ = h.exact(prob, store=False, blocknorm=True)
    torch.cuda.synchronize()
    ref = om.block_product_sq(host64(prob.M), host64(prob.N), off)
    got = host64(bp)
    assert np.all(np.abs(got - ref) <= TOL[torch.float32] * ref), np.max(np.abs(got - ref) / ref)


@pytest.mark.parametrize("ld_m,ld_n", [((1 << 22) - 8, (1 << 22) - 8), ((1 << 22) + 8, 8), (8, (1 << 22) + 8)])
def test_block_gram_large_strides(h, ld_m, ld_n):
    # row strides just below 2^22 floats take the Gram kernel at its largest
    # 32-bit buffer offsets; at 2^22 or more they take the block-by-block
    # product path; the same result either way
    M, N, off = wl.random_problem(3, 300, 5, 6, seed=42, skew=0.5)
    off = [0, 16, 50, 128, 131, 200, 300]
    bigM = torch.zeros((3, max(ld_m, 300)), dtype=torch.float32, device=DEV)
    bigM[:, :300] = to_dev(M, torch.float32)
    bigN = torch.zeros((300, max(ld_n, 5)), dtype=torch.float32, device=DEV)
    bigN[:, :5] = to_dev(N, torch.float32)
    Mv, Nv = bigM[:, :300], bigN[:, :5]
    ref = om.block_product_sq(host64(Mv), host64(Nv), off)
    _, bp, _ = h.exact(pk.Problem(Mv, Nv, off, c=3), store=False, blocknorm=True)
    torch.cuda.synchronize()
    assert np.all(np.abs(host64(bp) - ref) <= TOL[torch.float32] * ref)
    del bigM, bigN


def test_block_product_norms_wide_blocks(h):
    # blocks wider than the Gram tile take the block-by-block product path
    M, N, _ = wl.random_problem(140, 700, 90, 1, seed=33, skew=0.5)
    off = [0, 200, 201, 500, 700]
    for dtype in (torch.float64, torch.float32):
        prob = pk.Problem(to_dev(M, dtype), to_dev(N, dtype), off, c=3)
        _, bp, _ = h.exact(prob, store=False, blocknorm=True)
        torch.cuda.synchronize()
        ref = om.block_product_sq(host64(prob.M), host64(prob.N), off)
        assert rel(host64(bp), ref) < TOL[dtype]


def test_deterministic_single_block(h):
    M, N, _ = wl.random_problem(90, 300, 70, 1, seed=2)
    r, o = _check_run(h, M, N, [0, 300], 3, torch.float64, seed=1)
    assert rel(host64(r["CD"]), host64(r["MN"])) < 1e-12
    assert r["rel"] < 1e-12


def test_unit_strata_deterministic(h):
    M, N, _ = wl.random_problem(20, 64, 10, 1, seed=3)
    off = list(range(65))
    r, o = _check_run(h, M, N, off, 64, torch.float64, mode="stratified", prob="norm",
                      alloc="uniform")
    assert r["plan"].ck.cpu().tolist() == [1] * 64
    assert r["rel"] < 1e-12


def test_run_bitwise_reproducible(h):
    M, N, off = wl.random_problem(260, 3000, 300, 40, seed=4, skew=1.0)
    prob = pk.Problem(to_dev(M, torch.float32), to_dev(N, torch.float32), off, 32, seed=6)
    a = h.run(prob)
    b = h.run(prob)
    assert torch.equal(a["CD"], b["CD"]) and torch.equal(a["MN"], b["MN"])
    assert a["err"] == b["err"]
    prob.trial = 1
    c = h.run(prob)
    assert not torch.equal(a["plan"].idx, c["plan"].idx)


def test_all_zero_problem(h):
    M = np.zeros((40, 100))
    N = np.ones((100, 30))
    prob = pk.Problem(to_dev(M, torch.float64), to_dev(N, torch.float64), [0, 50, 100], 5)
    r = h.run(prob)
    assert r["L"] == 0 and r["err"] == 0.0 and r["rel"] == 0.0
    assert torch.count_nonzero(r["CD"]).item() == 0


def test_empty_outer_dims(h):
    for m, p in ((0, 5), (5, 0)):
        M = torch.zeros((m, 40), dtype=torch.float32, device=DEV)
        N = torch.ones((40, p), dtype=torch.float32, device=DEV)
        r = h.run(pk.Problem(M, N, [0, 20, 40], 3, prob="uniform"))
        assert r["err"] == 0.0


def test_sketch_gemm_error_epilogue_matches_error_kernel(h):
    M, N, off = wl.random_problem(300, 2500, 200, 30, seed=7, skew=1.0)
    prob = pk.Problem(to_dev(M, torch.float32), to_dev(N, torch.float32), off, 24, seed=2)
    col, row, blk = h.norms(prob)
    pl = h.plan(prob, col, row, blk)
    C, D = h.sketch(prob, pl)
    MN, _, mn_sq = h.exact(prob)
    CD, err = h.sketch_gemm(C, D, pl, MN=MN)
    e2 = h.error(CD, MN)
    torch.cuda.synchronize()
    assert abs(err.item() - e2[0].item()) <= 1e-12 * e2[0].item()
    assert abs(mn_sq.item() - e2[1].item()) <= 1e-12 * e2[1].item()


# --------------------------------------------------------------------------
# errors reported through the status word
# --------------------------------------------------------------------------

def test_nonfinite_input(h):
    M, N, off = wl.random_problem(50, 200, 40, 5, seed=8)
    M[3, 17] = np.nan
    prob = pk.Problem(to_dev(M, torch.float64), to_dev(N, torch.float64), off, 4)
    with pytest.raises(pk.SbmmError) as ei:
        h.run(prob)
    assert ei.value.status == pk.SBMM_E_NONFINITE
    # the handle recovers
    M[3, 17] = 0.0
    h.run(pk.Problem(to_dev(M, torch.float64), to_dev(N, torch.float64), off, 4))


def test_budget_below_sampleable_strata(h):
    M, N, _ = wl.random_problem(10, 60, 8, 1, seed=9)
    off = [0, 10, 20, 30, 40, 50, 60]
    M[:, 50:60] = 0.0               # one stratum has zero weight
    prob = pk.Problem(to_dev(M, torch.float64), to_dev(N, torch.float64), off, 5,
                      mode="stratified", prob="norm", alloc="norm")
    r = h.run(prob)                  # 5 draws for 5 sampleable strata: fine
    assert r["plan"].ck.cpu().tolist() == [1, 1, 1, 1, 1, 0]
    prob.c = 4
    with pytest.raises(pk.SbmmError) as ei:
        h.run(prob)
    assert ei.value.status == pk.SBMM_E_BUDGET


# --------------------------------------------------------------------------
# bf16 sketch (float32 accumulation)
# --------------------------------------------------------------------------

def _bf16_round(x):
    """float64 -> float32 -> bf16 (round to nearest even each time), back to
    float64: the rounding the gather applies to the scaled sketch."""
    return torch.from_numpy(np.asarray(x, np.float64)).to(torch.float32).to(
        torch.bfloat16).to(torch.float64).numpy()


@pytest.mark.parametrize("in_dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("shape", [(300, 2000, 260, 50, 37), (513, 4100, 129, 80, 64)])
def test_bf16_sketch(h, in_dtype, shape):
    m, n, p, K, c = shape
    M, N, off = wl.random_problem(m, n, p, K, seed=m + 3 * p, skew=1.0)
    Md, Nd = to_dev(M, in_dtype), to_dev(N, in_dtype)
    r = h.run(pk.Problem(Md, Nd, off, c, seed=2), compute=torch.bfloat16)
    Mh, Nh = host64(Md), host64(Nd)
    o = om.run(Mh, Nh, off, c, seed=2)
    assert np.array_equal(r["plan"].idx.cpu().numpy(), o.draws.atom)
    L = o.draws.L
    Cq, Dq = _bf16_round(o.C), _bf16_round(o.D)
    C, D = host64(r["C"]), host64(r["D"])
    assert np.array_equal(C[:, :L], Cq) and np.array_equal(D[:L], Dq)
    # float32 accumulation of the bf16 operands
    assert rel(host64(r["CD"]), Cq @ Dq) < 1e-5
    assert rel(host64(r["MN"]), o.MN) < 1e-5
    # the operand rounding itself: reported, bounded by a few bf16 units
    arith = rel(host64(r["CD"]), o.CD)
    print(f"bf16 sketch vs float64 sketch: {arith:.2e}")
    assert arith < 2e-2


# p a multiple of 8: D's rows are 16-byte aligned and the product reads D as
# gathered (K x p rows, transposing LDS reads of B); ragged row and column
# tiles (m, p not multiples of 256) and, with equal blocks of 50 and c = 45,
# an inner extent L_pad = 2272 that ends half way through a 64-wide k-step
@pytest.mark.parametrize("m,p,n,K,c", [(300, 264, 3000, 60, 45), (257, 520, 5000, 100, 64), (64, 8, 800, 16, 9)])
def test_bf16_sketch_product_reads_d_rows(h, m, p, n, K, c):
    M, N, _ = wl.random_problem(m, n, p, K, seed=m + p, skew=1.0)
    off = np.arange(0, n + 1, n // K, dtype=np.int64)
    Md, Nd = to_dev(M, torch.float32), to_dev(N, torch.float32)
    prob = pk.Problem(Md, Nd, off, c, prob="uniform", seed=4)
    col, row, blk = h.norms(prob)
    pl = h.plan(prob, col, row, blk)
    C, D = h.sketch(prob, pl, out_dtype=torch.bfloat16)
    o = om.run(host64(Md), host64(Nd), off, c, prob="uniform", seed=4)
    assert np.array_equal(pl.idx.cpu().numpy(), o.draws.atom)
    L = o.draws.L
    Cq, Dq = _bf16_round(o.C), _bf16_round(o.D)
    assert np.array_equal(host64(C)[:, :L], Cq) and np.array_equal(host64(D)[:L], Dq)
    MN = torch.from_numpy(o.MN.astype(np.float32)).to(Md.device)
    CD, err = h.sketch_gemm(C, D, pl, MN=MN)
    ref = Cq @ Dq
    assert rel(host64(CD), ref) < 1e-5
    e_ref = float(np.sum((o.MN.astype(np.float32).astype(np.float64) - ref) ** 2))
    assert abs(err.item() - e_ref) <= 1e-4 * e_ref


class _Extent:
    """Stands in for a plan where a product reads only the sketch width."""

    def __init__(self, L):
        self.L_dev = torch.tensor([L], dtype=torch.int64, device="cuda:0")


# the k-row bf16 product over inner extents of one to eight 64-wide k-steps
# (its A tiles come two steps ahead through a ring of three stages, B one
# step ahead through two, so the first steps and the ring's turns are the edge
# cases), some ending half way through a step; ragged 300 x 264 tiles; NaN past
# the extent must not reach the product
@pytest.mark.parametrize("L", [17, 64, 96, 160, 192, 250, 320, 352, 416, 480])
def test_bf16_kn_product_short_extents(h, L):
    m, p, Lp = 300, 264, 512
    K = (L + 31) // 32 * 32
    g = np.random.default_rng(L)
    C = torch.from_numpy(g.standard_normal((m, Lp)).astype(np.float32)).to(torch.bfloat16)
    D = torch.from_numpy(g.standard_normal((Lp, p)).astype(np.float32)).to(torch.bfloat16)
    C[:, L:K] = 0
    D[L:K] = 0
    C[:, K:] = float("nan")
    D[K:] = float("nan")
    Cd, Dd = C.to("cuda:0"), D.to("cuda:0")
    MN = torch.from_numpy(g.standard_normal((m, p)).astype(np.float32)).to("cuda:0")
    CD, err = h.sketch_gemm(Cd, Dd, _Extent(L), MN=MN)
    ref = C[:, :L].double().numpy() @ D[:L].double().numpy()
    assert rel(host64(CD), ref) < 1e-5
    e_ref = float(np.sum((host64(MN) - ref) ** 2))
    assert abs(err.item() - e_ref) <= 1e-4 * e_ref


# the exact product of bf16 inputs with row-major N read as it is (aligned rows)
@pytest.mark.parametrize("m,n,p", [(300, 1000, 264), (257, 4104, 520)])
def test_bf16_exact_product_reads_n_rows(h, m, n, p):
    M, N, off = wl.random_problem(m, n, p, 20, seed=n + p, skew=1.0)
    Md, Nd = to_dev(M, torch.bfloat16), to_dev(N, torch.bfloat16)
    MN, _, mn_sq = h.exact(pk.Problem(Md, Nd, off, 4), store=True)
    omn = host64(Md) @ host64(Nd)
    assert rel(host64(MN), omn) < 1e-5
    assert abs(mn_sq.item() - np.sum(omn * omn)) <= 1e-5 * np.sum(omn * omn)


def test_plan_rejects_missing_block_norms(h):
    M, N, off = wl.random_problem(10, 60, 8, 3, seed=40)
    for kw in (dict(prob="exact"), dict(mode="stratified", alloc="opt")):
        prob = pk.Problem(to_dev(M, torch.float64), to_dev(N, torch.float64), off, 4, **kw)
        col, row, blk = h.norms(prob)
        with pytest.raises(pk.SbmmError) as ei:
            h.plan(prob, col, row, blk)
        assert ei.value.status == pk.SBMM_E_ARG


# --------------------------------------------------------------------------
# backward (draws and p held fixed)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mode,off", [("block", None), ("stratified", None)])
def test_backward_f64_matches_oracle(h, mode, off):
    # the finite-difference case: 64 x 256 x 64, 8 blocks of 32, c = 4
    M, N, _ = wl.random_problem(64, 256, 64, 8, seed=41)
    off = wl.equal_blocks(256, 8)
    c = 4 if mode == "block" else 16
    Md = to_dev(M, torch.float64).requires_grad_(True)
    Nd = to_dev(N, torch.float64).requires_grad_(True)
    G = wl.rng(42).standard_normal((64, 64))
    kw = dict(mode=mode, prob="norm", alloc="norm", seed=3)
    prob = pk.Problem(Md.detach(), Nd.detach(), off, c, **kw)
    col, row, blk = h.norms(prob)
    pl = h.plan(prob, col, row, blk)
    C, D = h.sketch(prob, pl)
    CD, _ = h.sketch_gemm(C, D, pl)
    dM, dN = h.backward(prob, pl, C, D, to_dev(G, torch.float64))
    o = om.run(M, N, off, c, **kw)
    assert np.array_equal(pl.idx.cpu().numpy(), o.draws.atom)
    odM, odN = om.backward(M, N, o.draws, G)
    assert rel(host64(dM), odM) < 1e-12 and rel(host64(dN), odN) < 1e-12
    # columns of M / rows of N outside the drawn atoms get exactly zero
    hit = np.zeros(256, bool)
    for lo, w in zip(o.draws.lo, o.draws.width):
        hit[lo:lo + w] = True
    assert np.all(host64(dM)[:, ~hit] == 0) and np.all(host64(dN)[~hit] == 0)


def test_backward_finite_differences_autograd(h):
    # fixed user weights keep the draws and p fixed, so <G, CD> is bilinear
    # in (M, N) and central differences are exact up to rounding
    M, N, _ = wl.random_problem(64, 256, 64, 8, seed=43)
    off = wl.equal_blocks(256, 8)
    w = to_dev(wl.rng(44).uniform(0.5, 2.0, size=8), torch.float64)
    G = to_dev(wl.rng(45).standard_normal((64, 64)), torch.float64)
    SM = pk.SampledMatmul
    X = to_dev(M, torch.float64).requires_grad_(True)
    W = to_dev(N, torch.float64).requires_grad_(True)
    Y = SM.apply(X, W, off, 4, 7, 0, "user", None, w)
    (Y * G).sum().backward()
    g = wl.rng(46)
    for _ in range(3):
        dx = to_dev(g.standard_normal(M.shape), torch.float64)
        dw = to_dev(g.standard_normal(N.shape), torch.float64)
        eps = 1e-3
        with torch.no_grad():
            fp = (SM.apply(X + eps * dx, W + eps * dw, off, 4, 7, 0, "user", None, w) * G).sum()
            fm = (SM.apply(X - eps * dx, W - eps * dw, off, 4, 7, 0, "user", None, w) * G).sum()
        fd = ((fp - fm) / (2 * eps)).item()
        an = ((X.grad * dx).sum() + (W.grad * dw).sum()).item()
        assert abs(fd - an) <= 1e-8 * max(1.0, abs(an))


def test_backward_bf16_linear_layer(h):
    # the differentiable linear layer at a reduced size: X 1024 x 4096,
    # W 4096 x 2048 (bf16), 128 blocks of 32, c = 32
    X, W, G = wl.linear_layer(1024, 4096, 2048, seed=47)
    off = wl.equal_blocks(4096, 128)
    Xd = to_dev(X, torch.bfloat16).requires_grad_(True)
    Wd = to_dev(W, torch.bfloat16).requires_grad_(True)
    Gd = to_dev(G, torch.float32)
    Y = pk.SampledMatmul.apply(Xd, Wd, off, 32, 5, 0, "norm", None, None)
    Y.backward(Gd)
    Xh, Wh = host64(Xd), host64(Wd)
    o = om.run(Xh, Wh, off, 32, seed=5, prob="norm")
    assert np.array_equal(Y.grad_fn.plan.idx.cpu().numpy(), o.draws.atom)
    # the gradient of the estimator over the bf16 operands the kernels
    # multiply (X, W as stored, G rounded to bf16), draws merged per block
    dX, dW = om.backward(Xh, Wh, o.draws, _bf16_round(G))
    # bf16 outputs: within the bf16 rounding of the float64 reference
    assert rel(host64(Xd.grad), dX) < 4e-3 and rel(host64(Wd.grad), dW) < 4e-3
    # and an unbiased estimate of the exact gradient G W^T (reported)
    exact = G.astype(np.float64) @ Wh.T
    print("bf16 sampled dX vs exact-product gradient:", rel(host64(Xd.grad), exact))


# bf16 block norms ||M^k N_k||_F^2: the Gram path (blocks up to 128 wide,
# ragged widths, a block of 1) and the float32 product over promoted copies
# (a block wider than 128)
BF16_BLOCKNORM = [
    dict(m=300, n=2000, p=260, off=None, K=30),
    dict(m=77, n=500, p=45, off=[0, 1, 129, 200, 328, 400, 500], K=None),
    dict(m=64, n=1000, p=96, off=[0, 100, 400, 1000], K=None),
]


@pytest.mark.parametrize("d", BF16_BLOCKNORM)
def test_bf16_block_norms_match_oracle(h, d):
    M, N, off = wl.random_problem(d["m"], d["n"], d["p"], d["K"] or 3, seed=50, skew=1.0)
    if d["off"] is not None:
        off = d["off"]
    Md, Nd = to_dev(M, torch.bfloat16), to_dev(N, torch.bfloat16)
    Mq, Nq = host64(Md), host64(Nd)
    MN, bp, mn_sq = h.exact(pk.Problem(Md, Nd, off, 4), store=True, blocknorm=True)
    ref = om.block_product_sq(Mq, Nq, off)
    got = bp.cpu().numpy()
    # float32 accumulation of exact products of bf16 values
    assert np.all(np.abs(got - ref) <= 2e-5 * ref + 1e-30), float(np.max(np.abs(got - ref) / ref))
    omn = Mq @ Nq
    assert rel(host64(MN), omn) < 1e-5
    assert abs(mn_sq.item() - np.sum(omn * omn)) <= 1e-5 * np.sum(omn * omn)


def test_sampled_matmul_exact_rule_bf16(h):
    # rule (1.2) on the linear layer's dtype: the forward's draws equal the
    # oracle's for the same block norms
    X, W, G = wl.linear_layer(512, 2048, 384, seed=51)
    off = wl.equal_blocks(2048, 64)
    Xd = to_dev(X, torch.bfloat16).requires_grad_(True)
    Wd = to_dev(W, torch.bfloat16).requires_grad_(True)
    Y = pk.SampledMatmul.apply(Xd, Wd, off, 24, 3, 0, "exact", None, None)
    bp = Y.grad_fn.problem.blkprod_sq.cpu().numpy()
    Xh, Wh = host64(Xd), host64(Wd)
    ref = om.block_product_sq(Xh, Wh, off)
    assert np.all(np.abs(bp - ref) <= 2e-5 * ref)
    o = om.run(Xh, Wh, off, 24, seed=3, prob="exact", blkprod_sq=bp)
    assert np.array_equal(Y.grad_fn.plan.idx.cpu().numpy(), o.draws.atom)
    # the bf16 sketched product: float32 accumulation of the bf16-rounded sketch
    Cq, Dq = _bf16_round(o.C), _bf16_round(o.D)
    assert rel(host64(Y), Cq @ Dq) < 1e-5
    Y.backward(to_dev(G, torch.float32))
    dX, dW = om.backward(Xh, Wh, o.draws, _bf16_round(G))
    assert rel(host64(Xd.grad), dX) < 4e-3 and rel(host64(Wd.grad), dW) < 4e-3


# ragged extents (m, p not multiples of 8, uneven blocks), many duplicate
# draws (c above K), stratified mode, float32 and bf16 inputs
BF16_BACKWARD = [
    dict(m=203, n=517, p=139, K=9, c=40, mode="block", dtype=torch.bfloat16),
    dict(m=203, n=517, p=139, K=9, c=40, mode="block", dtype=torch.float32),
    dict(m=300, n=700, p=260, K=7, c=300, mode="stratified", dtype=torch.bfloat16),
    dict(m=64, n=2000, p=520, K=40, c=300, mode="block", dtype=torch.float32),
]


@pytest.mark.parametrize("d", BF16_BACKWARD)
def test_backward_bf16_merged_matches_oracle(h, d):
    M, N, off = wl.random_problem(d["m"], d["n"], d["p"], d["K"], seed=48, skew=1.0)
    dt = d["dtype"]
    Md, Nd = to_dev(M, dt), to_dev(N, dt)
    Mq, Nq = host64(Md), host64(Nd)          # the values the GPU holds
    kw = dict(mode=d["mode"], prob="norm", alloc="norm", seed=9)
    prob = pk.Problem(Md, Nd, off, d["c"], **kw)
    col, row, blk = h.norms(prob)
    pl = h.plan(prob, col, row, blk)
    G = wl.rng(49).standard_normal((d["m"], d["p"]))
    dM, dN = h.backward(prob, pl, None, None, to_dev(G, torch.float32), compute=torch.bfloat16)
    o = om.run(Mq, Nq, off, d["c"], **kw)
    assert np.array_equal(pl.idx.cpu().numpy(), o.draws.atom)
    # products of the bf16 values of M, N and G: float32 outputs carry only
    # float32 accumulation, bf16 outputs their own rounding
    odM, odN = om.backward(_bf16_round(Mq), _bf16_round(Nq), o.draws, _bf16_round(G))
    tol = 1e-5 if dt == torch.float32 else 4e-3
    assert rel(host64(dM), odM) < tol and rel(host64(dN), odN) < tol
    hit = np.zeros(d["n"], bool)
    for lo, w in zip(o.draws.lo, o.draws.width):
        hit[lo:lo + w] = True
    assert np.all(host64(dM)[:, ~hit] == 0) and np.all(host64(dN)[~hit] == 0)


@pytest.mark.parametrize("kw", [dict(prob="exact", dtype=torch.float32),
                                dict(mode="stratified", alloc="opt", dtype=torch.float64),
                                dict(mode="stratified", alloc="opt", dtype=torch.float32),
                                dict(mode="stratified", alloc="two_step", c0=60, pilot="norm",
                                     dtype=torch.float64)])
def test_run_on_fresh_handle_sizes_its_workspace(kw):
    # the whole-path call sizes its workspace before the rules' optional
    # buffers (block norms, pilot estimates) exist; a fresh handle has no
    # slack from earlier calls, so an undersized workspace would show here
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kw = dict(kw)
    dtype = kw.pop("dtype")
    M, N, off = wl.random_problem(200, 3000, 170, 30, seed=12, skew=1.0)
    c = 20 if kw.get("mode", "block") == "block" else 600
    hd = pk.Handle(0)
    try:
        _check_run(hd, M, N, off, c, dtype, seed=4, **kw)
    finally:
        hd.close()
