"""Failure paths of the C ABI on the device: an allocation the GPU cannot
satisfy reports SBMM_E_NOMEM with its text in sbmm_last_error and leaves the
handle usable; argument errors of device entry points are reported before
anything is enqueued."""
import ctypes

import numpy as np
import pytest

import workloads as wl
from oracle import method as om

torch = pytest.importorskip("torch")
import paper_2105_04940_amd as pk  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture()
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hd = pk.Handle(0)
    yield hd
    hd.close()


def test_reserve_beyond_device_memory_is_nomem(h):
    with pytest.raises(pk.SbmmError) as e:
        h.reserve(1 << 50)          # 1 PiB
    assert e.value.status == pk.SBMM_E_NOMEM
    assert b"workspace" in pk.lib().sbmm_last_error(h.h)
    # the handle keeps working: the tiny workload against the oracle
    M, N, off = wl.tiny(0)
    r = h.run(pk.Problem(torch.from_numpy(M).to(DEV), torch.from_numpy(N).to(DEV), off, 16, seed=0))
    o = om.run(M, N, off, 16, seed=0, prob="norm")
    assert np.array_equal(r["plan"].idx.cpu().numpy(), o.draws.atom)
    assert np.linalg.norm(r["CD"].cpu().numpy() - o.CD) <= 1e-12 * np.linalg.norm(o.CD)


def test_device_entry_points_reject_bad_arguments(h):
    M, N, off = wl.tiny(0)
    Md, Nd = torch.from_numpy(M).to(DEV), torch.from_numpy(N).to(DEV)
    prob = pk.Problem(Md, Nd, off, 16, seed=0)
    s = prob.struct()
    lib = pk.lib()
    col = torch.empty(1024, dtype=torch.float64, device=DEV)
    # missing outputs, misaligned M, unknown dtype of a product
    assert lib.sbmm_norms(h.h, ctypes.byref(s), None, None, None, None) == pk.SBMM_E_ARG
    s2 = prob.struct()
    s2.M = s2.M + 4                 # a float64 matrix four bytes off
    assert lib.sbmm_norms(h.h, ctypes.byref(s2), col.data_ptr(), col.data_ptr(), col.data_ptr(),
                          None) == pk.SBMM_E_ARG
    L = torch.zeros(1, dtype=torch.int64, device=DEV)
    assert lib.sbmm_sketch_gemm(h.h, 4, 4, 32, L.data_ptr(), 11, None, 32, None, 4, None, 4, None, 4,
                                None, None) == pk.SBMM_E_UNSUPPORTED
    assert lib.sbmm_error(h.h, 4, 4, 9, None, 4, None, 4, col.data_ptr(), None) == pk.SBMM_E_ARG
    torch.cuda.synchronize()


def test_peak_probe_rates_are_ordered(h):
    # the measured matrix-core rates: positive, below the specification's
    # 2.4 GHz peaks (157.3 / 2500 / 5000 TFLOP/s, a little margin for the
    # clock), and in the order of the instructions' widths
    f32, bf16, f8 = h.peak_probe("f32"), h.peak_probe("bf16"), h.peak_probe("f8e4m3")
    print(f"measured matrix-core TFLOP/s: f32 {f32:.1f}, bf16 {bf16:.1f}, f8e4m3 {f8:.1f}")
    assert 0.3 * 157.3 < f32 < 1.05 * 157.3
    assert 0.3 * 2500.0 < bf16 < 1.05 * 2500.0
    assert 0.3 * 5000.0 < f8 < 1.05 * 5000.0
    assert f32 < bf16 < f8
    out = ctypes.c_double()
    assert pk.lib().sbmm_peak_probe(h.h, pk.SBMM_F64, ctypes.byref(out)) == pk.SBMM_E_UNSUPPORTED
    assert pk.lib().sbmm_peak_probe(h.h, 17, ctypes.byref(out)) == pk.SBMM_E_UNSUPPORTED
    assert pk.lib().sbmm_peak_probe(h.h, pk.SBMM_F32, None) == pk.SBMM_E_ARG
