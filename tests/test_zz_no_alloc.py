"""sbmm_plan_noalloc, the plan entry point whose scratch is the library's
fixed per-GPU array: its outputs are those of sbmm_plan bit for bit (same
kernels on the same inputs), on two calls in a row where the second problem
is smaller than the first (the array keeps the first call's contents); it
allocates no device memory; and a problem whose plan does not fit the array
is rejected before anything is enqueued."""
import numpy as np
import pytest

import workloads as wl

torch = pytest.importorskip("torch")
import paper_2105_04940_amd as pk  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
FIELDS = ("idx", "scale", "col_off", "ck", "p_hat", "colmap", "colscale")


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hd = pk.Handle(0)
    yield hd
    hd.close()


def _problem(M, N, off, c, **kw):
    return pk.Problem(torch.from_numpy(M).to(DEV), torch.from_numpy(N).to(DEV), off, c, **kw)


def _wide_stratified():
    # 10 strata of 6000 single-column atoms (wider than one design chunk of
    # 2048) and 6000 draws (more than one offsets workgroup of 256)
    M, N, _ = wl.random_problem(6, 60000, 5, 10, seed=3, skew=1.0)
    off = wl.equal_blocks(60000, 10)
    return _problem(M, N, off, 6000, mode="stratified", prob="norm", alloc="norm", seed=5, trial=2)


def _small_block():
    M, N, off = wl.tiny(0)
    return _problem(M, N, off, 16, prob="norm", seed=0)


def _same(a, b):
    L = a.L
    assert L == b.L
    for f in FIELDS:
        x = getattr(a, f).cpu()
        y = getattr(b, f).cpu()
        if f in ("colmap", "colscale"):
            pad = -(-L // pk.SKETCH_PAD) * pk.SKETCH_PAD
            x, y = x[:pad], y[:pad]
        assert torch.equal(x, y), f


def test_noalloc_plan_equals_plan_on_two_calls(h):
    big, small = _wide_stratified(), _small_block()
    norms = [h.norms(pr) for pr in (big, small)]
    got = [h.plan_noalloc(pr, *nm) for pr, nm in zip((big, small), norms)]
    ref = [h.plan(pr, *nm) for pr, nm in zip((big, small), norms)]
    for g, r in zip(got, ref):
        _same(g, r)
    # and once more after sbmm_plan has run: the array's old contents matter not
    again = h.plan_noalloc(small, *norms[1])
    _same(again, ref[1])


def test_noalloc_plan_allocates_nothing():
    hd = pk.Handle(0)   # fresh handle: its workspace has never grown
    try:
        pr = _wide_stratified()
        nm = hd.norms(pr)
        out = pk.Plan(pr, pk.sbmm_query_sizes(pr), DEV)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        hd.plan_noalloc(pr, *nm, out=out)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        ref = hd.plan(pr, *nm)
        _same(out, ref)
    finally:
        hd.close()


def test_noalloc_plan_rejects_oversize(h):
    n = 1_200_000   # 16 bytes per atom alone exceed the 16 MiB array
    M = torch.ones((1, n), dtype=torch.float32, device=DEV)
    N = torch.ones((n, 1), dtype=torch.float32, device=DEV)
    pr = pk.Problem(M, N, [0, n // 2, n], 4, mode="stratified", prob="uniform", alloc="uniform")
    with pytest.raises(pk.SbmmError) as e:
        h.plan_noalloc(pr)
    assert e.value.status == pk.SBMM_E_ARG
    assert "scratch" in str(e.value)
    # the same problem runs through sbmm_plan (its workspace grows)
    pl = h.plan(pr)
    assert pl.L == 4
