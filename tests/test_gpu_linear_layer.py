"""The differentiable linear layer at full size: X 8192 x 16384 and W 16384 x
8192 in bf16 (X ~ N(0,1), W ~ N(0, 0.01^2)), 512 blocks of 32, c = 128,
upstream gradient G 8192 x 8192 ~ N(0,1), through SampledMatmul.

The oracle draws from its own norms. The forward output is checked in full
against the float64 product of the oracle's sketch rounded as the gather
rounds it (to float32, then bf16); the gradients in every drawn column of dX
and row of dW (and, separately, on a seeded sample of them) against float64
products of the bf16 operands (X, W and G rounded to bf16) with each block's
draws merged (the sum of scale^2); every untouched column / row must be
exactly zero."""
import numpy as np
import pytest

import workloads as wl
from oracle import method as om

torch = pytest.importorskip("torch")
import paper_2105_04940_amd as pk  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def bf16_round(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).to(torch.float32).to(
        torch.bfloat16).to(torch.float64).numpy()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def test_linear_layer_full_size():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    X, W, G = wl.linear_layer()
    off = wl.equal_blocks(X.shape[1], 512)
    Xd = torch.from_numpy(X).to(DEV).to(torch.bfloat16).requires_grad_(True)
    Wd = torch.from_numpy(W).to(DEV).to(torch.bfloat16).requires_grad_(True)
    Gd = torch.from_numpy(G).to(DEV)
    Y = pk.SampledMatmul.apply(Xd, Wd, off, 128, 11, 0, "norm", None, None)
    gpu_idx = Y.grad_fn.plan.idx.cpu().numpy()
    Yh = Y.detach().float().cpu().numpy().astype(np.float64)
    Y.backward(Gd)
    torch.cuda.synchronize()
    Xh = Xd.detach().float().cpu().numpy().astype(np.float64)
    Wh = Wd.detach().float().cpu().numpy().astype(np.float64)
    design, col, row, st = om.plan(Xh, Wh, off, 128, prob="norm")
    draws = om.sample(design, 11, 0)
    assert draws.L == 4096
    assert np.array_equal(gpu_idx, draws.atom)
    dX = Xd.grad.float().cpu().numpy()
    dW = Wd.grad.float().cpu().numpy()
    hit = np.zeros(X.shape[1], bool)
    for lo, w in zip(draws.lo, draws.width):
        hit[lo:lo + w] = True
    assert np.all(dX[:, ~hit] == 0) and np.all(dW[~hit] == 0)
    Gq = bf16_round(G)
    g = wl.rng(5)
    cols = g.choice(np.nonzero(hit)[0], size=12, replace=False)
    # the gradient of the estimator: each sampled inner index gets the sum of
    # scale^2 over the draws of its block times G W[i, :]^T (dX) and
    # X[:, i]^T G (dW), over the bf16 values the kernels multiply
    ref_x, ref_w, got_x, got_w = [], [], [], []
    for i in cols:
        f = sum(draws.scale[t] ** 2 for t in range(len(draws.atom))
                if draws.lo[t] <= i < draws.lo[t] + draws.width[t])
        ref_x.append(f * (Gq @ Wh[i, :]))
        ref_w.append(f * (Xh[:, i] @ Gq))
        got_x.append(dX[:, i])
        got_w.append(dW[i, :])
    # bf16 outputs: within the bf16 rounding of the float64 reference
    assert rel(np.array(got_x), np.array(ref_x)) < 4e-3
    assert rel(np.array(got_w), np.array(ref_w)) < 4e-3
    # every drawn column of dX and row of dW
    fac = np.zeros(X.shape[1])
    for t in range(len(draws.atom)):
        fac[draws.lo[t]:draws.lo[t] + draws.width[t]] += draws.scale[t] ** 2
    hi = np.nonzero(hit)[0]
    ref_dx = (Gq @ Wh[hi, :].T) * fac[hi][None, :]
    assert rel(dX[:, hi], ref_dx) < 4e-3
    del ref_dx
    ref_dw = (Xh[:, hi].T @ Gq) * fac[hi][:, None]
    assert rel(dW[hi], ref_dw) < 4e-3
    del ref_dw
    # the forward output in full: the sketch rounded to float32 then bf16, the
    # product of those values (float32 accumulation on the device)
    C_o, D_o = om.sketch(Xh, Wh, draws)
    y_ref = bf16_round(C_o) @ bf16_round(D_o)
    del C_o, D_o
    tol = 1e-5 if Y.dtype == torch.float32 else 4e-3
    assert rel(Yh, y_ref) < tol, (rel(Yh, y_ref), Y.dtype)
