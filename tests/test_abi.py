"""The C-ABI library loads and exports every symbol include/sbmm.h declares
(CPU only: no compute call is made), and the host-side validation of a
problem (sbmm_query_sizes, which launches nothing) returns the documented
status for every class of bad argument."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2105_04940_amd as pk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sbmm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sbmm_[a-z_]+)\s*\(", text)))


def test_header_matches_binding_list():
    assert declared_functions() == sorted(pk.EXPORTS)


def test_library_exports_every_symbol():
    lib = ctypes.CDLL(pk.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings():
    lib = pk.lib()
    for st in range(8):
        assert lib.sbmm_status_string(st)
    assert lib.sbmm_status_string(99) == b"unknown status"


class FakeTensor:
    """Host stand-in with the attributes Problem.struct reads (no device)."""

    def __init__(self, rows, cols, dtype, ptr=0x1000):
        self.shape = (rows, cols)
        self.dtype = dtype
        self._ptr = ptr

    def dim(self):
        return 2

    def stride(self, i):
        return (self.shape[1], 1)[i]

    def data_ptr(self):
        return self._ptr

    def numel(self):
        return self.shape[0] * self.shape[1]


def _problem(m=8, n=10, p=6, off=(0, 4, 10), c=3, **kw):
    import torch
    M = FakeTensor(m, n, torch.float32)
    N = FakeTensor(n, p, torch.float32, ptr=0x2000)
    return pk.Problem(M, N, list(off), c, **kw)


def _status(problem):
    s = problem.struct()
    out = pk.Sizes_t()
    return pk.lib().sbmm_query_sizes(ctypes.byref(s), ctypes.byref(out)), out


def test_sizes_block_and_stratified():
    st, out = _status(_problem(off=(0, 4, 10), c=3))
    assert st == pk.SBMM_OK
    assert (out.atoms, out.strata, out.max_width, out.L_max, out.L_pad_max) == (2, 1, 6, 18, 32)
    st, out = _status(_problem(off=(0, 4, 10), c=3, mode="stratified"))
    assert st == pk.SBMM_OK
    assert (out.atoms, out.strata, out.max_width, out.L_max, out.L_pad_max) == (10, 2, 1, 3, 32)


@pytest.mark.parametrize("kw", [
    dict(off=(0, 4, 4, 10)),                 # empty block
    dict(off=(0, 4, 9)),                     # does not end at n
    dict(off=(1, 4, 10)),                    # does not start at 0
    dict(off=(0, 6, 4, 10)),                 # decreasing
    dict(c=0),                               # no draws
    dict(c=2**31),                           # too many draws
    dict(prob="user"),                       # user weights missing
    dict(mode="stratified", alloc="user"),   # counts missing
    dict(mode="stratified", alloc="user", user_ck=[1, 1]),      # sum != c
    dict(mode="stratified", alloc="user", user_ck=[4, -1]),     # negative
])
def test_validation_rejects(kw):
    st, _ = _status(_problem(**kw))
    assert st == pk.SBMM_E_ARG


def test_validation_shape_and_pointer_errors():
    import torch
    M = FakeTensor(8, 10, torch.float32, ptr=0)      # NULL M with m > 0
    N = FakeTensor(10, 6, torch.float32)
    st, _ = _status(pk.Problem(M, N, [0, 10], 2))
    assert st == pk.SBMM_E_ARG
    # empty outer dimensions are valid (nothing to compute)
    M = FakeTensor(0, 10, torch.float32, ptr=0)
    N = FakeTensor(10, 0, torch.float32, ptr=0)
    st, _ = _status(pk.Problem(M, N, [0, 10], 2))
    assert st == pk.SBMM_OK


def test_validation_bad_enum():
    p = _problem()
    s = p.struct()
    s.mode = 7
    out = pk.Sizes_t()
    assert pk.lib().sbmm_query_sizes(ctypes.byref(s), ctypes.byref(out)) == pk.SBMM_E_ARG
    s = p.struct()
    s.in_dtype = pk.SBMM_F8E4M3
    assert pk.lib().sbmm_query_sizes(ctypes.byref(s), ctypes.byref(out)) == pk.SBMM_E_ARG


def test_null_handle_is_state_error():
    lib = pk.lib()
    assert lib.sbmm_destroy(None) == pk.SBMM_E_STATE
    assert lib.sbmm_sync(None, None) == pk.SBMM_E_STATE
    assert lib.sbmm_reserve(None, 16) == pk.SBMM_E_STATE
    out = ctypes.c_double()
    assert lib.sbmm_peak_probe(None, pk.SBMM_F32, ctypes.byref(out)) == pk.SBMM_E_STATE


def _struct_status(s):
    out = pk.Sizes_t()
    return pk.lib().sbmm_query_sizes(ctypes.byref(s), ctypes.byref(out))


def test_misaligned_and_short_leading_dimensions():
    import torch
    # a float32 M one byte off its element boundary, a float64 N four bytes off
    M = FakeTensor(8, 10, torch.float32, ptr=0x1001)
    N = FakeTensor(10, 6, torch.float32)
    assert _status(pk.Problem(M, N, [0, 10], 2))[0] == pk.SBMM_E_ARG
    M = FakeTensor(8, 10, torch.float64)
    N = FakeTensor(10, 6, torch.float64, ptr=0x2004)
    assert _status(pk.Problem(M, N, [0, 10], 2))[0] == pk.SBMM_E_ARG
    # bf16 needs two-byte alignment only; float32 at a 4-byte (not 16-byte) boundary is valid
    M = FakeTensor(8, 10, torch.bfloat16, ptr=0x1002)
    N = FakeTensor(10, 6, torch.bfloat16, ptr=0x2006)
    assert _status(pk.Problem(M, N, [0, 10], 2))[0] == pk.SBMM_OK
    M = FakeTensor(8, 10, torch.float32, ptr=0x1004)
    assert _status(pk.Problem(M, FakeTensor(10, 6, torch.float32), [0, 10], 2))[0] == pk.SBMM_OK
    # leading dimensions below the row length
    s = _problem().struct()
    s.ldm = s.n - 1
    assert _struct_status(s) == pk.SBMM_E_ARG
    s = _problem().struct()
    s.ldn = s.p - 1
    assert _struct_status(s) == pk.SBMM_E_ARG


@pytest.mark.parametrize("field,value,extra", [
    ("prob", 99, {}), ("prob", -1, {}), ("in_dtype", 4, {}), ("in_dtype", -7, {}),
    ("mode", 2, {}), ("alloc", 99, dict(mode="stratified")),
    ("pilot_prob", 2, dict(mode="stratified", alloc="two_step", c0=4)),
    ("pilot_prob", 99, dict(mode="stratified", alloc="two_step", c0=4)),
])
def test_enum_values_outside_their_range(field, value, extra):
    s = _problem(**extra).struct()
    setattr(s, field, value)
    if field == "pilot_prob":
        s.pilot_sq = 0x3000     # present, so the pilot's own checks run
        st = pk.lib().sbmm_workspace_size(ctypes.byref(s), pk.SBMM_F32, ctypes.byref(ctypes.c_size_t()), None)
    else:
        st = _struct_status(s)
    assert st == pk.SBMM_E_ARG


def test_workspace_size_rejects_unknown_compute_dtype():
    s = _problem().struct()
    n = ctypes.c_size_t()
    for bad in (pk.SBMM_F8E4M3, 17, -1):
        assert pk.lib().sbmm_workspace_size(ctypes.byref(s), bad, ctypes.byref(n), None) == pk.SBMM_E_ARG
    assert pk.lib().sbmm_workspace_size(ctypes.byref(s), pk.SBMM_F32, ctypes.byref(n), None) == pk.SBMM_OK


def test_status_string_of_any_int():
    lib = pk.lib()
    for v in (-1, 8, 99, 2**31 - 1):
        assert lib.sbmm_status_string(v) == b"unknown status"
