"""Products with small outputs and long inner extents (m, p <= 128, inner
extent >= 2048) take the split-K path: exact MN with its norm and per-block
norms ||M^k N_k||_F^2, the sketched product with its error, against the
oracle in float64 and float32, over ragged tile grids, tiny outputs, many
blocks, blocks shorter and longer than a segment."""
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


def to_dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV).to(dtype)


def host64(t):
    return t.detach().double().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


SHAPES = [
    (26, 60000, 28, [0, 12580, 22078, 31783, 39096, 50858, 60000]),   # Sec. 4-like, one tile
    (100, 9000, 70, None),                                             # 4 x 3 tiles, ragged edges
    (1, 5000, 1, [0, 1, 2, 4999, 5000]),                               # one element, blocks of width 1
    (128, 4096, 128, None),                                            # 16 tiles, the largest output taken
]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", SHAPES)
def test_exact_and_block_norms(h, dtype, shape):
    m, n, p, off = shape
    M, N, off2 = wl.random_problem(m, n, p, 37, seed=m + p, skew=1.0)
    off = off if off is not None else off2
    prob = pk.Problem(to_dev(M, dtype), to_dev(N, dtype), off, c=3)
    MN, bp, mn_sq = h.exact(prob, store=True, blocknorm=True)
    torch.cuda.synchronize()
    Mh, Nh = host64(prob.M), host64(prob.N)
    MNo = om.exact_product(Mh, Nh)
    assert rel(host64(MN), MNo) < TOL[dtype]
    assert rel(host64(bp), om.block_product_sq(Mh, Nh, off)) < TOL[dtype]
    assert abs(mn_sq.item() - np.sum(MNo ** 2)) <= TOL[dtype] * np.sum(MNo ** 2)


def test_many_blocks(h):
    # 3000 blocks of 1..4 columns: more segments than blocks per tile
    g = np.random.Generator(np.random.PCG64(9))
    widths = g.integers(1, 5, 3000)
    off = np.concatenate([[0], np.cumsum(widths)]).tolist()
    n = off[-1]
    M = g.standard_normal((20, n))
    N = g.standard_normal((n, 9))
    prob = pk.Problem(to_dev(M, torch.float64), to_dev(N, torch.float64), off, c=3)
    _, bp, _ = h.exact(prob, store=False, blocknorm=True)
    torch.cuda.synchronize()
    assert rel(host64(bp), om.block_product_sq(M, N, off)) < 1e-12


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_sketched_product_and_error(h, dtype):
    # stratified sampling at c = 20000 over 26 x 28: the sketch product and
    # its error take the split-K path
    M, N, off = wl.random_problem(26, 40000, 28, 8, seed=44, skew=1.5)
    Md, Nd = to_dev(M, dtype), to_dev(N, dtype)
    prob = pk.Problem(Md, Nd, off, 20000, mode="stratified", prob="norm", alloc="norm", seed=2)
    r = h.run(prob)
    o = om.run(host64(Md), host64(Nd), off, 20000, seed=2, mode="stratified", prob="norm", alloc="norm")
    assert np.array_equal(r["plan"].idx.cpu().numpy(), o.draws.atom)
    assert rel(host64(r["CD"]), o.CD) < TOL[dtype]
    assert abs(r["rel"] - o.rel) <= TOL[dtype] * max(o.rel, 1.0)
    # the same product through the step entry points, with the fused error
    col, row, blk = h.norms(prob)
    pl = h.plan(prob, col, row, blk)
    C, D = h.sketch(prob, pl)
    CD, err = h.sketch_gemm(C, D, pl, MN=r["MN"])
    torch.cuda.synchronize()
    assert rel(host64(CD), o.CD) < TOL[dtype]
    e2 = float(np.sum((host64(CD) - host64(r["MN"])) ** 2))
    assert abs(err.item() - e2) <= 1e-9 * e2
