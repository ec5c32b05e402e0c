"""Parity at the full paper-scale block workload (M 4096 x 65536, N 65536 x
4096 float32, 1024 uneven blocks of 16..112, lognormal(0, 1.5) column / row
factors), in the launch configuration the benchmark times.

The oracle computes the norms, design and draws at full size, CD and MN on a
seeded sample of entries (one by one, from their definitions), and CD and MN
in full (float64 products of its own sketch, and of M and N; about 3 TFLOP on
the host); the norms are compared in full. Indices must be identical; float32
outputs must be within 1e-5 (relative Frobenius over the sampled entries and
over all entries), and every entry within 1e-5 of the largest in magnitude.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import method as om

torch = pytest.importorskip("torch")
import paper_2105_04940_amd as pk  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def paper_inputs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    M, N, off = wl.paper_scale()
    col, row = om.column_row_sq(M, N)
    Md = torch.from_numpy(M).to(DEV)
    Nd = torch.from_numpy(N).to(DEV)
    return M, N, off, Md, Nd, col, row


@pytest.fixture(scope="module")
def h():
    hd = pk.Handle(0)
    yield hd
    hd.close()


def test_paper_scale_norms(h, paper_inputs):
    M, N, off, Md, Nd, col, row = paper_inputs
    gcol, grow, gblk = h.norms(pk.Problem(Md, Nd, off, 256))
    torch.cuda.synchronize()
    assert rel(gcol.cpu().numpy(), col) < 1e-13
    assert rel(grow.cpu().numpy(), row) < 1e-13
    st = om.block_stats(col, row, off)
    b = gblk.cpu().numpy()
    K = len(off) - 1
    assert rel(b[:K], st.m_sq) < 1e-13 and rel(b[2 * K:], st.s) < 1e-13


@pytest.fixture(scope="module")
def paper_mn(paper_inputs):
    M, N, *_ = paper_inputs
    return om.exact_product(M, N)


@pytest.fixture(scope="module")
def paper_blkprod(paper_inputs):
    M, N, off, *_ = paper_inputs
    return om.block_product_sq(M, N, off)


@pytest.mark.parametrize("c,prob", [(256, "norm"), (64, "uniform"), (128, "exact")])
def test_paper_scale_run(h, paper_inputs, paper_blkprod, paper_mn, c, prob):
    M, N, off, Md, Nd, col, row = paper_inputs
    bp = None
    if prob == "exact":
        _, bpd, _ = h.exact(pk.Problem(Md, Nd, off, c), store=False, blocknorm=True)
        torch.cuda.synchronize()
        assert rel(bpd.cpu().numpy(), paper_blkprod) < 1e-5
        # and block by block (1024 blocks of 16..112 columns, every tile count 1..7)
        got = bpd.cpu().numpy()
        assert np.all(np.abs(got - paper_blkprod) <= 1e-5 * paper_blkprod), \
            float(np.max(np.abs(got - paper_blkprod) / paper_blkprod))
        # the draws are a function of the weight vector: the oracle plans with
        # the GPU's (float32-accumulated) block norms, checked above
        bp = got
    r = h.run(pk.Problem(Md, Nd, off, c, prob=prob, seed=0, trial=0))
    design, *_ = om.plan(M, N, off, c, prob=prob, col_row=(col, row), blkprod_sq=bp)
    draws = om.sample(design, 0, 0)
    idx = r["plan"].idx.cpu().numpy()
    assert np.array_equal(idx, draws.atom)
    assert r["L"] == draws.L
    g = wl.rng(1234)
    S = 1500
    rows = g.integers(0, M.shape[0], size=S)
    cols = g.integers(0, N.shape[1], size=S)
    cd_o = om.sketch_entries(M, N, draws, rows, cols)
    mn_o = om.exact_entries(M, N, rows, cols)
    CD = r["CD"].cpu().numpy()
    MN = r["MN"].cpu().numpy()
    assert rel(CD[rows, cols], cd_o) < 1e-5
    assert rel(MN[rows, cols], mn_o) < 1e-5
    # every entry: the oracle's float64 MN, and CD from its own sketch
    C_o, D_o = om.sketch(M, N, draws)
    CD_o = om.sketch_product(C_o, D_o)
    del C_o, D_o
    for got, ref in ((CD, CD_o), (MN, paper_mn)):
        assert rel(got, ref) < 1e-5
        assert float(np.max(np.abs(got - ref))) <= 1e-5 * float(np.max(np.abs(ref)))
    # the fused error equals the standalone error kernel on the same outputs
    e2 = h.error(r["CD"], r["MN"]).cpu().numpy()
    assert abs(r["err"] ** 2 - e2[0]) <= 1e-12 * e2[0]
    assert abs(r["rel"] - np.sqrt(e2[0] / e2[1])) <= 1e-12 * r["rel"]


def _bf16_round(x):
    """float64 -> float32 -> bf16 (nearest even each time) -> float64: the
    rounding the gather applies to the scaled sketch."""
    return torch.from_numpy(np.asarray(x, np.float64)).to(torch.float32).to(torch.bfloat16).to(
        torch.float64).numpy()


def test_paper_scale_bf16_sketch(h, paper_inputs):
    # the bf16 sketch the benchmark times (D's rows read as gathered): C and D
    # bit-exact against the oracle's sketch rounded the gather's way, CD in
    # every entry against the float64 product of those values
    M, N, off, Md, Nd, col, row = paper_inputs
    prob = pk.Problem(Md, Nd, off, 256, prob="norm", seed=0, trial=0)
    gcol, grow, gblk = h.norms(prob)
    pl = h.plan(prob, gcol, grow, gblk)
    C, D = h.sketch(prob, pl, out_dtype=torch.bfloat16)
    CD, _ = h.sketch_gemm(C, D, pl)
    torch.cuda.synchronize()
    design, *_ = om.plan(M, N, off, 256, prob="norm", col_row=(col, row))
    draws = om.sample(design, 0, 0)
    assert np.array_equal(pl.idx.cpu().numpy(), draws.atom)
    L = draws.L
    C_o, D_o = om.sketch(M, N, draws)
    Cq, Dq = _bf16_round(C_o), _bf16_round(D_o)
    del C_o, D_o
    assert np.array_equal(C[:, :L].double().cpu().numpy(), Cq)
    assert np.array_equal(D[:L].double().cpu().numpy(), Dq)
    ref = Cq @ Dq
    got = CD.double().cpu().numpy()
    assert rel(got, ref) < 1e-5
    assert float(np.max(np.abs(got - ref))) <= 1e-5 * float(np.max(np.abs(ref)))
