"""The sketch in OCP MX E4M3 (8-bit floats with a power-of-two scale per 32
sketch columns) and its product on the block-scaled matrix instruction,
against the oracle: the draws come from the float64 oracle, the sketch is the
oracle's float32-rounded C and D quantized by the oracle's MX definition
(oracle/lowp.py); the GPU's codes and scale bytes must equal it bit for bit,
and CD must equal the float64 product of the quantized values within the
error bound of the block-scaled matrix instruction (below)."""
import numpy as np
import pytest

import workloads as wl
from oracle import lowp
from oracle import method as om

torch = pytest.importorskip("torch")
import paper_2105_04940_amd as pk  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


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
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


_TABLE = lowp.e4m3_values()


def decode(codes, scales, L_pad):
    """Values of MX E4M3 rows: codes (r x >= L_pad uint8), scale bytes."""
    c = codes[:, :L_pad].astype(np.int64)
    mag = _TABLE[np.minimum(c & 0x7F, 126)]
    assert not np.any((c & 0x7F) == 0x7F), "NaN code"
    v = np.where(c & 0x80, -mag, mag)
    e = scales[:, :L_pad // 32].astype(np.int64) - 127
    return np.ldexp(v, np.repeat(e, 32, axis=1)), e


def oracle_mx(Mh, Nh, off, c, prob, seed):
    design, *_ = om.plan(Mh, Nh, off, c, prob=prob)
    draws = om.sample(design, seed, 0)
    C, D = om.sketch(Mh, Nh, draws)
    L = draws.L
    Lp = (L + 31) // 32 * 32
    Cf = np.zeros((Mh.shape[0], Lp))
    Cf[:, :L] = lowp.f32(C)
    Dtf = np.zeros((Nh.shape[1], Lp))
    Dtf[:, :L] = lowp.f32(D).T
    Cq, Ec = lowp.mx_quantize(Cf)
    Dq, Ed = lowp.mx_quantize(Dtf)
    return draws, Lp, Cq, Ec, Dq, Ed


def _binade(v):
    """Exponent of each E4M3 value's binade (subnormals and zero at -6)."""
    a = np.abs(v)
    _, e = np.frexp(np.where(a > 0, a, 1.0))
    return np.maximum(e - 1, -6)


def instruction_bound(Cq, Ec, Dq, Ed, Lp, kept_bits=12):
    """Elementwise bound on |CD - Cq Dq^T| for the block-scaled E4M3 product.

    Measured behaviour of the instruction (one-wave probes, E4M3 x E4M3): in
    each run of 8 consecutive inner indices it aligns the 8 products to the
    largest exponent sum e = (code exponents + block scales) of the run and
    drops each product's bits below 2^(e-13), toward zero; the runs, the two
    scale blocks and the accumulator input are then added exactly and rounded
    once to float32 per instruction (64 inner indices). The bound allows one
    bit more than measured (2^(e-12) per nonzero product) plus a float32
    rounding of the running sum per inner index, which covers any
    instruction count."""
    m, p = Cq.shape[0], Dq.shape[0]
    Xc = np.repeat(Ec, 32, axis=1)
    Xd = np.repeat(Ed, 32, axis=1)
    ec = _binade(Cq / 2.0 ** Xc) + Xc
    ed = _binade(Dq / 2.0 ** Xd) + Xd
    nzc, nzd = Cq != 0, Dq != 0
    trunc = np.zeros((m, p))
    for g in range(0, Lp, 8):
        emax = np.full((m, p), -1000.0)
        cnt = np.zeros((m, p))
        for k in range(g, g + 8):
            live = nzc[:, k, None] & nzd[None, :, k]
            emax = np.where(live, np.maximum(emax, ec[:, k, None] + ed[None, :, k]), emax)
            cnt += live
        trunc += cnt * np.exp2(emax - kept_bits)
    return trunc + 2.0 * Lp * 2.0 ** -24 * (np.abs(Cq) @ np.abs(Dq).T)


CASES = [
    dict(m=300, n=2000, p=260, K=50, c=40, prob="norm", skew=1.5),     # ragged tiles, partial k-step
    dict(m=512, n=4096, p=512, K=64, c=64, prob="uniform", skew=0.0),  # whole tiles, several k-steps
    dict(m=7, n=300, p=5, K=10, c=3, prob="norm", skew=3.0),           # tiny, strongly skewed scales
]


@pytest.mark.parametrize("case", CASES)
def test_mx_sketch_and_product(h, case):
    M, N, off = wl.random_problem(case["m"], case["n"], case["p"], case["K"], seed=31, dtype=np.float32,
                                  skew=case["skew"])
    Md = torch.from_numpy(np.ascontiguousarray(M)).to(DEV)
    Nd = torch.from_numpy(np.ascontiguousarray(N)).to(DEV)
    prob = pk.Problem(Md, Nd, off, case["c"], prob=case["prob"], seed=2)
    col, row, blk = h.norms(prob)
    plan = h.plan(prob, col, row, blk, sync=True)
    C8, Cs, Dt8, Ds = h.sketch_mx(prob, plan)
    MN = Md @ Nd
    CD, err = h.sketch_gemm_mx(C8, Cs, Dt8, Ds, plan, MN=MN)
    torch.cuda.synchronize()
    Mh, Nh = M.astype(np.float64), N.astype(np.float64)
    draws, Lp, Cq, Ec, Dq, Ed = oracle_mx(Mh, Nh, off, case["c"], case["prob"], 2)
    assert np.array_equal(plan.idx.cpu().numpy(), draws.atom)
    assert plan.L == draws.L
    Cg, Ecg = decode(C8.cpu().numpy(), Cs.cpu().numpy(), Lp)
    Dg, Edg = decode(Dt8.cpu().numpy(), Ds.cpu().numpy(), Lp)
    assert np.array_equal(Ecg, Ec) and np.array_equal(Edg, Ed)
    assert np.array_equal(Cg, Cq) and np.array_equal(Dg, Dq)
    # the scale bytes after the last block, up to a multiple of 4 blocks, are 1
    nb = Lp // 32
    pad = (nb + 3) // 4 * 4
    assert np.all(Cs.cpu().numpy()[:, nb:pad] == 127) and np.all(Ds.cpu().numpy()[:, nb:pad] == 127)
    ref = Cq @ Dq.T
    gpu = CD.double().cpu().numpy()
    bound = instruction_bound(Cq, Ec, Dq, Ed, Lp)
    assert np.all(np.abs(gpu - ref) <= bound)
    print("MX E4M3 product vs float64 product of the same values:", rel(gpu, ref),
          "largest error / bound:", float(np.max(np.abs(gpu - ref) / np.maximum(bound, 1e-300))))
    mn = MN.double().cpu().numpy()
    e2 = float(((CD.double().cpu().numpy() - mn) ** 2).sum())
    assert abs(err.item() - e2) <= 1e-9 * e2
    # the quantization error itself, relative to the float32 sketch product
    f32_ref = lowp.f32(om.sketch(Mh, Nh, draws)[0]) @ lowp.f32(om.sketch(Mh, Nh, draws)[1])
    print("MX E4M3 sketch product vs float32 sketch product:", rel(CD.cpu().numpy(), f32_ref))


def test_mx_zero_problem(h):
    Md = torch.zeros((40, 100), dtype=torch.float32, device=DEV)
    Nd = torch.zeros((100, 30), dtype=torch.float32, device=DEV)
    prob = pk.Problem(Md, Nd, list(range(0, 101, 10)), 5)
    col, row, blk = h.norms(prob)
    plan = h.plan(prob, col, row, blk, sync=True)
    C8, Cs, Dt8, Ds = h.sketch_mx(prob, plan)
    CD, _ = h.sketch_gemm_mx(C8, Cs, Dt8, Ds, plan)
    torch.cuda.synchronize()
    assert plan.L == 0 and torch.count_nonzero(CD).item() == 0


def test_mx_paper_scale(h):
    # the paper-scale block workload at c = 256, rule (1.4): every code and
    # scale byte of C and D^T against the oracle's quantization of its own
    # sketch, and the product on a 128 x 128 block of sampled entries within
    # the instruction bound (the full bound would take hours on the host)
    M, N, off = wl.paper_scale()
    Md = torch.from_numpy(M).to(DEV)
    Nd = torch.from_numpy(N).to(DEV)
    prob = pk.Problem(Md, Nd, off, 256, prob="norm", seed=0)
    col, row, blk = h.norms(prob)
    plan = h.plan(prob, col, row, blk, sync=True)
    C8, Cs, Dt8, Ds = h.sketch_mx(prob, plan)
    CD, _ = h.sketch_gemm_mx(C8, Cs, Dt8, Ds, plan)
    torch.cuda.synchronize()
    draws, Lp, Cq, Ec, Dq, Ed = oracle_mx(M.astype(np.float64), N.astype(np.float64), off, 256, "norm", 0)
    assert np.array_equal(plan.idx.cpu().numpy(), draws.atom)
    assert plan.L == draws.L
    Cg, Ecg = decode(C8.cpu().numpy(), Cs.cpu().numpy(), Lp)
    assert np.array_equal(Ecg, Ec) and np.array_equal(Cg, Cq)
    del Cg
    Dg, Edg = decode(Dt8.cpu().numpy(), Ds.cpu().numpy(), Lp)
    assert np.array_equal(Edg, Ed) and np.array_equal(Dg, Dq)
    del Dg
    g = wl.rng(77)
    rows = np.sort(g.choice(M.shape[0], size=128, replace=False))
    cols = np.sort(g.choice(N.shape[1], size=128, replace=False))
    ref = Cq[rows] @ Dq[cols].T
    bound = instruction_bound(Cq[rows], Ec[rows], Dq[cols], Ed[cols], Lp)
    gpu = CD.double().cpu().numpy()[np.ix_(rows, cols)]
    assert np.all(np.abs(gpu - ref) <= bound), float(np.max(np.abs(gpu - ref) / np.maximum(bound, 1e-300)))
