"""Host-only size queries of the C ABI (no GPU needed): sbmm_query_sizes and
sbmm_workspace_size on problems whose device pointers are never read."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
import paper_2105_04940_amd as pk  # noqa: E402


def _problem(m, n, p, off, c, dtype=torch.float32, **kw):
    M = torch.zeros((m, n), dtype=dtype)
    N = torch.zeros((n, p), dtype=dtype)
    return pk.Problem(M, N, off, c, **kw)


def test_workspace_size_grows_with_c_and_matches_L_max():
    off = [0, 16, 50, 112, 200]
    sizes = []
    for c in (8, 64, 256):
        b, L = pk.sbmm_workspace_size(_problem(300, 200, 100, off, c))
        assert L == c * 88
        assert L == pk.sbmm_query_sizes(_problem(300, 200, 100, off, c))["L_max"]
        sizes.append(b)
    assert 0 < sizes[0] < sizes[1] < sizes[2]


def test_workspace_size_covers_pilot_and_bf16():
    off = list(range(0, 50001, 5000))
    base = _problem(26, 50000, 28, off, 5000, dtype=torch.float64, mode="stratified", alloc="norm")
    two = _problem(26, 50000, 28, off, 5000, dtype=torch.float64, mode="stratified", alloc="two_step",
                   c0=5000, pilot="norm")
    b0, _ = pk.sbmm_workspace_size(base)
    b1, _ = pk.sbmm_workspace_size(two)
    assert b1 > b0       # the pilot sketch and its estimates
    f32 = _problem(64, 4096, 64, [0, 1024, 4096], 16)
    b32, _ = pk.sbmm_workspace_size(f32, torch.float32)
    b16, _ = pk.sbmm_workspace_size(f32, torch.bfloat16)
    assert b32 > 0 and b16 > 0


def test_workspace_size_rejects():
    with pytest.raises(pk.SbmmError):
        pk.sbmm_workspace_size(_problem(4, 10, 4, [0, 10], 2, dtype=torch.float64), torch.float32)
    with pytest.raises(pk.SbmmError):
        pk.sbmm_workspace_size(_problem(4, 10, 4, [0, 5, 12], 2))       # offsets do not end at n
    with pytest.raises(pk.SbmmError):
        pk.sbmm_workspace_size(_problem(4, 10, 4, [0, 10], 0))           # c < 1
