"""Python binding of libsbmm, the MI355X (gfx950) sampled block matrix product.

Argument marshalling only: every step of the path runs in the library's HIP
kernels. PyTorch tensors provide device memory and the current stream. The
C entry points are re-exported under the same names (``sbmm_norms``,
``sbmm_plan``, ...); ``Handle`` bundles them with tensor allocation.

The library must be built (``python -m paper_2105_04940_amd.build``); there is
no fallback: importing the binding without ``libsbmm.so`` raises.
"""
import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SBMM_LIB names another build of the same library (the host-sanitized one
# of the CPU tests); the default is the in-tree libsbmm.so
LIB_PATH = os.environ.get("SBMM_LIB") or os.path.join(_HERE, "libsbmm.so")

SBMM_OK, SBMM_E_ARG, SBMM_E_BUDGET, SBMM_E_NONFINITE, SBMM_E_UNSUPPORTED, \
    SBMM_E_NOMEM, SBMM_E_HIP, SBMM_E_STATE = range(8)
SBMM_F64, SBMM_F32, SBMM_BF16, SBMM_F8E4M3 = range(4)
MODES = {"block": 0, "stratified": 1}
PROBS = {"uniform": 0, "norm": 1, "exact": 2, "user": 3}
ALLOCS = {"uniform": 0, "norm": 1, "opt": 2, "user": 3, "two_step": 4}
SKETCH_PAD = 32

# Names of every function the C header declares (checked by the ABI test).
EXPORTS = (
    "sbmm_create", "sbmm_destroy", "sbmm_status_string", "sbmm_last_error",
    "sbmm_reserve", "sbmm_sync", "sbmm_query_sizes", "sbmm_norms",
    "sbmm_exact", "sbmm_plan", "sbmm_sketch", "sbmm_sketch_gemm",
    "sbmm_error", "sbmm_run", "sbmm_backward",
    "sbmm_batch_create", "sbmm_batch_destroy", "sbmm_batch_run", "sbmm_batch_capture",
    "sbmm_batch_replay", "sbmm_batch_tune", "sbmm_batch_set_tuning",
    "sbmm_sketch_mx", "sbmm_sketch_gemm_mx", "sbmm_pilot", "sbmm_bound",
    "sbmm_workspace_size", "sbmm_exact_error", "sbmm_plan_noalloc", "sbmm_peak_probe",
)
NOALLOC_SCRATCH_BYTES = 16 << 20   # SBMM_NOALLOC_SCRATCH_BYTES
# Layout of sbmm_bound's output (SBMM_BOUND_* in the header), then eta_j and
# the bound of every delta_j.
BOUND_FIELDS = ("theta1", "theta2", "theta1_hat", "theta2_hat", "beta", "mn", "phi",
                "var_bound", "expected")
BOUND_MAX_DELTA = 8
BATCH_TILES = ((128, 128), (64, 128), (128, 64), (64, 64), (256, 256), (128, 128))


class SbmmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"sbmm status {status}: {msg}")
        self.status = status


class Problem_t(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("p", ctypes.c_int64),
        ("in_dtype", ctypes.c_int),
        ("M", ctypes.c_void_p), ("ldm", ctypes.c_int64),
        ("N", ctypes.c_void_p), ("ldn", ctypes.c_int64),
        ("K", ctypes.c_int32), ("block_off", ctypes.c_void_p),
        ("c", ctypes.c_int64),
        ("mode", ctypes.c_int), ("prob", ctypes.c_int), ("alloc", ctypes.c_int),
        ("user_w", ctypes.c_void_p), ("user_ck", ctypes.c_void_p),
        ("blkprod_sq", ctypes.c_void_p),
        ("seed", ctypes.c_uint64), ("trial", ctypes.c_uint64),
        ("c0", ctypes.c_int64), ("pilot_prob", ctypes.c_int), ("pilot_sq", ctypes.c_void_p),
    ]


class Sizes_t(ctypes.Structure):
    _fields_ = [("atoms", ctypes.c_int64), ("strata", ctypes.c_int64),
                ("max_width", ctypes.c_int64), ("L_max", ctypes.c_int64),
                ("L_pad_max", ctypes.c_int64)]


class PlanOut_t(ctypes.Structure):
    _fields_ = [("idx", ctypes.c_void_p), ("scale", ctypes.c_void_p),
                ("col_off", ctypes.c_void_p), ("ck", ctypes.c_void_p),
                ("p_hat", ctypes.c_void_p), ("colmap", ctypes.c_void_p),
                ("colscale", ctypes.c_void_p)]


class BatchItem_t(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("p", ctypes.c_int64),
        ("M", ctypes.c_void_p), ("ldm", ctypes.c_int64),
        ("N", ctypes.c_void_p), ("ldn", ctypes.c_int64),
        ("K", ctypes.c_int32), ("block_off", ctypes.c_void_p),
        ("c", ctypes.c_int64), ("prob", ctypes.c_int),
        ("seed", ctypes.c_uint64), ("trial", ctypes.c_uint64),
        ("CD", ctypes.c_void_p), ("ldcd", ctypes.c_int64),
        ("MN", ctypes.c_void_p), ("ldmn", ctypes.c_int64),
    ]


class BatchOutputs_t(ctypes.Structure):
    _fields_ = [("err2_mn2", ctypes.c_void_p), ("L", ctypes.c_void_p), ("idx", ctypes.c_void_p)]


BATCH_TUNING_SLOTS = 24   # SBMM_BATCH_TUNING_SLOTS


class BatchTuning_t(ctypes.Structure):
    _fields_ = [("cfg", ctypes.c_int32 * 2), ("lpt", ctypes.c_int32 * 2),
                ("ms", (ctypes.c_float * BATCH_TUNING_SLOTS) * 2)]


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -m paper_2105_04940_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64, i32, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "sbmm_create": (st, [P(vp), ctypes.c_int]),
        "sbmm_destroy": (st, [vp]),
        "sbmm_status_string": (ctypes.c_char_p, [st]),
        "sbmm_last_error": (ctypes.c_char_p, [vp]),
        "sbmm_reserve": (st, [vp, ctypes.c_size_t]),
        "sbmm_sync": (st, [vp, vp]),
        "sbmm_query_sizes": (st, [P(Problem_t), P(Sizes_t)]),
        "sbmm_norms": (st, [vp, P(Problem_t), vp, vp, vp, vp]),
        "sbmm_exact": (st, [vp, P(Problem_t), vp, i64, vp, vp, vp]),
        "sbmm_plan": (st, [vp, P(Problem_t), vp, vp, vp, P(PlanOut_t), P(i64), vp]),
        "sbmm_plan_noalloc": (st, [vp, P(Problem_t), vp, vp, vp, P(PlanOut_t), P(i64), vp]),
        "sbmm_pilot": (st, [vp, P(Problem_t), vp, vp, vp, P(PlanOut_t), vp, vp]),
        "sbmm_bound": (st, [vp, P(Problem_t), vp, vp, vp, vp, P(PlanOut_t), ctypes.c_double, i32,
                            P(ctypes.c_double), P(ctypes.c_double), vp]),
        "sbmm_workspace_size": (st, [P(Problem_t), st, P(ctypes.c_size_t), P(i64)]),
        "sbmm_exact_error": (st, [vp, P(Problem_t), vp, i64, st, vp, i64, vp, vp, vp]),
        "sbmm_sketch": (st, [vp, P(Problem_t), P(PlanOut_t), st, vp, i64, vp, i64, vp]),
        "sbmm_sketch_gemm": (st, [vp, i64, i64, i64, vp, st, vp, i64, vp, i64, vp, i64,
                                  vp, i64, vp, vp]),
        "sbmm_error": (st, [vp, i64, i64, st, vp, i64, vp, i64, vp, vp]),
        "sbmm_peak_probe": (st, [vp, st, P(ctypes.c_double)]),
        "sbmm_run": (st, [vp, P(Problem_t), st, vp, i64, vp, i64, vp, i64, vp, i64,
                          P(PlanOut_t), P(ctypes.c_double), P(ctypes.c_double), P(i64), vp]),
        "sbmm_backward": (st, [vp, P(Problem_t), P(PlanOut_t), i64, st, vp, i64, vp, i64, vp, i64,
                               vp, i64, vp, i64, vp]),
        "sbmm_batch_create": (st, [vp, i32, P(BatchItem_t), P(BatchOutputs_t), P(vp)]),
        "sbmm_batch_destroy": (st, [vp]),
        "sbmm_batch_run": (st, [vp, vp, vp]),
        "sbmm_batch_capture": (st, [vp, vp]),
        "sbmm_batch_replay": (st, [vp, vp, vp]),
        "sbmm_batch_tune": (st, [vp, vp, i32, P(BatchTuning_t), vp]),
        "sbmm_batch_set_tuning": (st, [vp, vp, P(BatchTuning_t)]),
        "sbmm_sketch_mx": (st, [vp, P(Problem_t), P(PlanOut_t), vp, i64, vp, i64, vp, i64, vp, i64, vp]),
        "sbmm_sketch_gemm_mx": (st, [vp, i64, i64, i64, vp, vp, i64, vp, i64, vp, i64, vp, i64, vp, i64,
                                     vp, i64, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _torch():
    import torch
    return torch


def dtype_code(t):
    torch = _torch()
    if t == torch.float64:
        return SBMM_F64
    if t == torch.float32:
        return SBMM_F32
    if t == torch.bfloat16:
        return SBMM_BF16
    raise ValueError(f"unsupported dtype {t}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class Problem:
    """One sampling problem (M, N on the device, block offsets on the host)."""
    M: object
    N: object
    off: object
    c: int
    mode: str = "block"
    prob: str = "norm"
    alloc: str = "norm"
    seed: int = 0
    trial: int = 0
    user_w: object = None       # device float64 tensor
    user_ck: object = None      # host int64 sequence
    blkprod_sq: object = None   # device float64 tensor
    c0: int = 0                 # two-step algorithm: pilot draws (alloc "two_step")
    pilot: str = "uniform"      # pilot probabilities: "uniform" (ONU) or "norm" (ONMCNR)
    pilot_sq: object = None     # device float64 tensor of K pilot estimates

    def struct(self):
        M, N = self.M, self.N
        if M.dim() != 2 or N.dim() != 2 or M.shape[1] != N.shape[0]:
            raise ValueError("M must be m x n and N n x p")
        if M.stride(1) != 1 or N.stride(1) != 1:
            raise ValueError("M and N must be row-major (unit column stride)")
        if M.dtype != N.dtype:
            raise ValueError("M and N must share a dtype")
        off = np.ascontiguousarray(np.asarray(self.off, dtype=np.int64))
        ck = (None if self.user_ck is None
              else np.ascontiguousarray(np.asarray(self.user_ck, dtype=np.int64)))
        s = Problem_t()
        s._keep = (off, ck)          # the host arrays live as long as the struct
        s.m, s.n = M.shape
        s.p = N.shape[1]
        s.in_dtype = dtype_code(M.dtype)
        s.M = M.data_ptr() if M.numel() else None
        s.ldm = max(M.stride(0), M.shape[1]) if M.shape[0] > 1 else M.shape[1]
        s.N = N.data_ptr() if N.numel() else None
        s.ldn = max(N.stride(0), N.shape[1]) if N.shape[0] > 1 else N.shape[1]
        s.K = len(off) - 1
        s.block_off = off.ctypes.data
        s.c = int(self.c)
        s.mode = MODES[self.mode]
        s.prob = PROBS[self.prob]
        s.alloc = ALLOCS[self.alloc]
        s.user_w = None if self.user_w is None else self.user_w.data_ptr()
        s.user_ck = None if ck is None else ck.ctypes.data
        s.blkprod_sq = None if self.blkprod_sq is None else self.blkprod_sq.data_ptr()
        s.seed = int(self.seed) & (2**64 - 1)
        s.trial = int(self.trial) & (2**64 - 1)
        s.c0 = int(self.c0)
        s.pilot_prob = PROBS[self.pilot]
        s.pilot_sq = None if self.pilot_sq is None else self.pilot_sq.data_ptr()
        return s


def sbmm_workspace_size(problem, compute=None):
    """Device workspace bytes the problem's calls need (see the header) and
    L_max; host only."""
    s = problem.struct()
    cd = dtype_code(compute or problem.M.dtype)
    b = ctypes.c_size_t()
    L = ctypes.c_int64()
    st = lib().sbmm_workspace_size(ctypes.byref(s), cd, ctypes.byref(b), ctypes.byref(L))
    if st != SBMM_OK:
        raise SbmmError(st, "sbmm_workspace_size: invalid problem or compute dtype")
    return b.value, L.value


def sbmm_query_sizes(problem):
    s = problem.struct()
    out = Sizes_t()
    st = lib().sbmm_query_sizes(ctypes.byref(s), ctypes.byref(out))
    if st != SBMM_OK:
        raise SbmmError(st, lib().sbmm_status_string(st).decode())
    return dict(atoms=out.atoms, strata=out.strata, max_width=out.max_width,
                L_max=out.L_max, L_pad_max=out.L_pad_max)


class Plan:
    """Device buffers of the planning step."""

    def __init__(self, problem, sizes, device, c=None):
        torch = _torch()
        c = int(problem.c if c is None else c)
        kw = dict(device=device)
        self.idx = torch.empty(c, dtype=torch.int32, **kw)
        self.scale = torch.empty(c, dtype=torch.float64, **kw)
        self.col_off = torch.empty(c + 1, dtype=torch.int64, **kw)
        self.ck = torch.empty(sizes["strata"], dtype=torch.int64, **kw)
        self.p_hat = torch.empty(sizes["atoms"], dtype=torch.float64, **kw)
        self.colmap = torch.empty(sizes["L_pad_max"], dtype=torch.int32, **kw)
        self.colscale = torch.empty(sizes["L_pad_max"], dtype=torch.float64, **kw)

    def struct(self):
        s = PlanOut_t()
        s.idx, s.scale, s.col_off, s.ck = (self.idx.data_ptr(), self.scale.data_ptr(),
                                           self.col_off.data_ptr(), self.ck.data_ptr())
        s.p_hat = self.p_hat.data_ptr()
        s.colmap, s.colscale = self.colmap.data_ptr(), self.colscale.data_ptr()
        self._s = s
        return s

    @property
    def L_dev(self):
        return self.col_off[-1:]


class Handle:
    """A libsbmm handle on one device, with tensor-level helpers."""

    def __init__(self, device=0):
        self._lib = lib()
        h = ctypes.c_void_p()
        st = self._lib.sbmm_create(ctypes.byref(h), int(device))
        if st != SBMM_OK:
            raise SbmmError(st, "sbmm_create failed")
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            self._lib.sbmm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != SBMM_OK:
            msg = self._lib.sbmm_last_error(self.h).decode(errors="replace")
            raise SbmmError(st, f"{self._lib.sbmm_status_string(st).decode()}: {msg}")

    # -- steps --------------------------------------------------------------
    def norms(self, problem):
        torch = _torch()
        s = problem.struct()
        n, K = s.n, s.K
        dev = problem.M.device
        col_sq = torch.empty(n, dtype=torch.float64, device=dev)
        row_sq = torch.empty(n, dtype=torch.float64, device=dev)
        blk = torch.empty(3 * K, dtype=torch.float64, device=dev)
        self._check(self._lib.sbmm_norms(self.h, ctypes.byref(s), _ptr(col_sq), _ptr(row_sq),
                                         _ptr(blk), _stream()))
        return col_sq, row_sq, blk

    def exact(self, problem, store=True, blocknorm=False):
        torch = _torch()
        s = problem.struct()
        dev = problem.M.device
        pd = torch.float64 if problem.M.dtype == torch.float64 else torch.float32
        MN = torch.empty((s.m, s.p), dtype=pd, device=dev) if store else None
        bp = torch.empty(s.K, dtype=torch.float64, device=dev) if blocknorm else None
        mn_sq = torch.empty(1, dtype=torch.float64, device=dev)
        self._check(self._lib.sbmm_exact(self.h, ctypes.byref(s), _ptr(MN), s.p if store else 0,
                                         _ptr(bp), _ptr(mn_sq), _stream()))
        return MN, bp, mn_sq

    def reserve(self, nbytes):
        self._check(self._lib.sbmm_reserve(self.h, int(nbytes)))

    def exact_error(self, problem, CD, store=False, blocknorm=False):
        """The exact product with ||MN - CD||_F^2 and ||MN||_F^2 from its
        epilogue (device float64 tensor of 2); MN and the per-block norms
        optional."""
        torch = _torch()
        s = problem.struct()
        dev = problem.M.device
        pd = torch.float64 if problem.M.dtype == torch.float64 else torch.float32
        MN = torch.empty((s.m, s.p), dtype=pd, device=dev) if store else None
        bp = torch.empty(s.K, dtype=torch.float64, device=dev) if blocknorm else None
        out = torch.empty(2, dtype=torch.float64, device=dev)
        self._check(self._lib.sbmm_exact_error(self.h, ctypes.byref(s), _ptr(CD), CD.stride(0), dtype_code(CD.dtype),
                                               _ptr(MN), s.p if store else 0, _ptr(bp), _ptr(out), _stream()))
        return out, MN, bp

    def plan(self, problem, col_sq=None, row_sq=None, blk=None, sync=True, out=None):
        return self._plan(self._lib.sbmm_plan, problem, col_sq, row_sq, blk, sync, out)

    def plan_noalloc(self, problem, col_sq=None, row_sq=None, blk=None, sync=True, out=None):
        """sbmm_plan_noalloc: the plan with its scratch in the library's fixed
        per-GPU array (the caller's output Plan may be passed as `out`)."""
        return self._plan(self._lib.sbmm_plan_noalloc, problem, col_sq, row_sq, blk, sync, out)

    def _plan(self, fn, problem, col_sq, row_sq, blk, sync, out):
        s = problem.struct()
        sizes = sbmm_query_sizes(problem)
        pl = out if out is not None else Plan(problem, sizes, problem.M.device)
        ps = pl.struct()
        L = ctypes.c_int64(-1)
        self._check(fn(self.h, ctypes.byref(s), _ptr(col_sq), _ptr(row_sq), _ptr(blk), ctypes.byref(ps),
                       ctypes.byref(L) if sync else None, _stream()))
        pl.L = L.value if sync else None
        pl.sizes = sizes
        return pl

    def pilot(self, problem, col_sq=None, row_sq=None, blk=None, keep_plan=False):
        """Step 1 of the two-step algorithm: the K pilot estimates
        ||C^{0k} D_{0k}||_F^2 (float64 tensor) and, with keep_plan, the pilot
        draws (a Plan sized for c0 draws; entries past the drawn total have
        idx -1)."""
        torch = _torch()
        s = problem.struct()
        dev = problem.M.device
        out = torch.empty(s.K, dtype=torch.float64, device=dev)
        pl = None
        if keep_plan:
            Lp = -(-int(problem.c0) // SKETCH_PAD) * SKETCH_PAD
            sizes = dict(atoms=s.n, strata=s.K, max_width=1, L_max=int(problem.c0), L_pad_max=Lp)
            pl = Plan(problem, sizes, dev, c=problem.c0)
            pl.sizes = sizes
            pl.L = None
        ps = pl.struct() if pl is not None else None
        self._check(self._lib.sbmm_pilot(self.h, ctypes.byref(s), _ptr(col_sq), _ptr(row_sq), _ptr(blk),
                                         ctypes.byref(ps) if ps is not None else None, _ptr(out), _stream()))
        return (out, pl) if keep_plan else out

    def bound(self, problem, col_sq, row_sq, blk, blkprod_sq, plan, beta=0.0, deltas=()):
        """Probability error bounds of the problem's block-size rule (OPT:
        Thm 3.3, NORM: Thm 4.2, TWO_STEP: Thm 4.4 with problem.pilot_sq) and
        the expected squared error of the sampled design (synchronizing).
        Returns a dict with the BOUND_FIELDS and lists ``eta`` and ``bound``,
        one entry per delta."""
        s = problem.struct()
        deltas = [float(d) for d in deltas]
        nd = len(deltas)
        out = (ctypes.c_double * (len(BOUND_FIELDS) + 2 * nd))()
        dl = (ctypes.c_double * max(nd, 1))(*deltas)
        ps = plan.struct()
        self._check(self._lib.sbmm_bound(self.h, ctypes.byref(s), _ptr(col_sq), _ptr(row_sq), _ptr(blk),
                                         _ptr(blkprod_sq), ctypes.byref(ps), float(beta), nd, dl, out,
                                         _stream()))
        r = {f: out[i] for i, f in enumerate(BOUND_FIELDS)}
        base = len(BOUND_FIELDS)
        r["eta"] = [out[base + 2 * j] for j in range(nd)]
        r["bound"] = [out[base + 2 * j + 1] for j in range(nd)]
        return r

    def sketch(self, problem, plan, out_dtype=None, want_C=True, want_D=True):
        torch = _torch()
        s = problem.struct()
        od = out_dtype or problem.M.dtype
        Lp = plan.sizes["L_pad_max"]
        dev = problem.M.device
        C = torch.empty((s.m, Lp), dtype=od, device=dev) if want_C else None
        D = torch.empty((Lp, s.p), dtype=od, device=dev) if want_D else None
        ps = plan.struct()
        self._check(self._lib.sbmm_sketch(self.h, ctypes.byref(s), ctypes.byref(ps),
                                          dtype_code(od), _ptr(C), Lp, _ptr(D), s.p, _stream()))
        return C, D

    def sketch_gemm(self, C, D, plan, MN=None, store=True):
        torch = _torch()
        m, Lp = C.shape
        p = D.shape[1]
        od = torch.float64 if C.dtype == torch.float64 else torch.float32
        CD = torch.empty((m, p), dtype=od, device=C.device) if store else None
        err = torch.empty(1, dtype=torch.float64, device=C.device) if MN is not None else None
        self._check(self._lib.sbmm_sketch_gemm(
            self.h, m, p, Lp, _ptr(plan.L_dev), dtype_code(C.dtype), _ptr(C), C.stride(0),
            _ptr(D), D.stride(0), _ptr(CD), p, _ptr(MN), p if MN is not None else 0,
            _ptr(err), _stream()))
        return CD, err

    def sketch_mx(self, problem, plan):
        """The sketch in MX E4M3: (C, Cs, Dt, Ds) uint8 tensors: C m x L_pad_max
        codes, Cs m x nsc scale bytes, Dt (D transposed) p x L_pad_max codes,
        Ds p x nsc scale bytes, nsc = round_up(L_pad_max / 32, 4)."""
        torch = _torch()
        s = problem.struct()
        Lp = plan.sizes["L_pad_max"]
        nsc = (Lp // 32 + 3) // 4 * 4
        dev = problem.M.device
        C = torch.empty((s.m, Lp), dtype=torch.uint8, device=dev)
        Cs = torch.empty((s.m, nsc), dtype=torch.uint8, device=dev)
        Dt = torch.empty((s.p, Lp), dtype=torch.uint8, device=dev)
        Ds = torch.empty((s.p, nsc), dtype=torch.uint8, device=dev)
        ps = plan.struct()
        self._check(self._lib.sbmm_sketch_mx(self.h, ctypes.byref(s), ctypes.byref(ps), _ptr(C), Lp, _ptr(Cs),
                                             nsc, _ptr(Dt), Lp, _ptr(Ds), nsc, _stream()))
        return C, Cs, Dt, Ds

    def sketch_gemm_mx(self, C, Cs, Dt, Ds, plan, MN=None, store=True):
        torch = _torch()
        m, Lp = C.shape
        p = Dt.shape[0]
        CD = torch.empty((m, p), dtype=torch.float32, device=C.device) if store else None
        err = torch.empty(1, dtype=torch.float64, device=C.device) if MN is not None else None
        self._check(self._lib.sbmm_sketch_gemm_mx(
            self.h, m, p, Lp, _ptr(plan.L_dev), _ptr(C), C.stride(0), _ptr(Cs), Cs.stride(0), _ptr(Dt),
            Dt.stride(0), _ptr(Ds), Ds.stride(0), _ptr(CD), p, _ptr(MN), p if MN is not None else 0,
            _ptr(err), _stream()))
        return CD, err

    def peak_probe(self, dtype):
        """sbmm_peak_probe: the device's measured matrix-core TFLOP/s for
        "f32", "bf16" or "f8e4m3" (register operands, no memory traffic)."""
        codes = {"f32": SBMM_F32, "bf16": SBMM_BF16, "f8e4m3": SBMM_F8E4M3}
        out = ctypes.c_double()
        self._check(self._lib.sbmm_peak_probe(self.h, codes[dtype], ctypes.byref(out)))
        return out.value

    def error(self, X, Y):
        torch = _torch()
        out = torch.empty(2, dtype=torch.float64, device=X.device)
        self._check(self._lib.sbmm_error(self.h, X.shape[0], X.shape[1], dtype_code(X.dtype),
                                         _ptr(X), X.stride(0), _ptr(Y), Y.stride(0), _ptr(out),
                                         _stream()))
        return out

    def backward(self, problem, plan, C, D, G, L=None, compute=None):
        """dM, dN of <G, CD> with the draws of `plan` held fixed (C, D from
        the forward in the compute dtype; bf16 compute reads M and N instead
        and takes C = D = None with compute=torch.bfloat16; G float64 for
        float64 compute, else float32). Returns tensors in the dtype of M
        and N."""
        torch = _torch()
        s = problem.struct()
        ps = plan.struct()
        if L is None:
            L = plan.L if plan.L is not None else plan.sizes["L_pad_max"]
        cdt = compute if compute is not None else C.dtype
        want = torch.float64 if cdt == torch.float64 else torch.float32
        if G.dtype != want or G.stride(1) != 1:
            raise ValueError(f"G must be a row-major {want} tensor")
        dM = torch.empty((s.m, s.n), dtype=problem.M.dtype, device=problem.M.device)
        dN = torch.empty((s.n, s.p), dtype=problem.N.dtype, device=problem.N.device)
        self._check(self._lib.sbmm_backward(
            self.h, ctypes.byref(s), ctypes.byref(ps), int(L), dtype_code(cdt),
            _ptr(C), C.stride(0) if C is not None else 0, _ptr(D), D.stride(0) if D is not None else 0,
            _ptr(G), G.stride(0), _ptr(dM), s.n, _ptr(dN), s.p, _stream()))
        return dM, dN

    def sync(self):
        self._check(self._lib.sbmm_sync(self.h, _stream()))

    def run(self, problem, compute=None, want_C=True, want_D=True, want_MN=True):
        """The whole forward path (synchronizing). Returns a dict with C, D
        (padded to L_pad_max columns / rows), CD, MN, the plan, L, err, rel."""
        torch = _torch()
        s = problem.struct()
        sizes = sbmm_query_sizes(problem)
        dev = problem.M.device
        cd = compute or problem.M.dtype
        pd = torch.float64 if cd == torch.float64 else torch.float32
        Lp = sizes["L_pad_max"]
        C = torch.empty((s.m, Lp), dtype=cd, device=dev) if want_C else None
        D = torch.empty((Lp, s.p), dtype=cd, device=dev) if want_D else None
        CD = torch.empty((s.m, s.p), dtype=pd, device=dev)
        MN = torch.empty((s.m, s.p), dtype=pd, device=dev) if want_MN else None
        pl = Plan(problem, sizes, dev)
        ps = pl.struct()
        err = ctypes.c_double()
        rel = ctypes.c_double()
        L = ctypes.c_int64()
        self._check(self._lib.sbmm_run(
            self.h, ctypes.byref(s), dtype_code(cd), _ptr(C), Lp, _ptr(D), s.p, _ptr(CD), s.p,
            _ptr(MN), s.p, ctypes.byref(ps), ctypes.byref(err), ctypes.byref(rel),
            ctypes.byref(L), _stream()))
        pl.L = L.value
        pl.sizes = sizes
        return dict(C=C, D=D, CD=CD, MN=MN, plan=pl, L=L.value, err=err.value, rel=rel.value)


class Batch:
    """Many independent block-mode problems run as one pass (sbmm_batch_*).

    ``problems`` is a list of dicts with keys M, N (float32 device tensors,
    row-major, any leading dimension), off (block offsets), c, and optional
    prob ("norm" / "uniform"), seed, trial. The batch allocates CD and MN per
    problem, the per-problem (err^2, ||MN||^2) pairs, the sketch widths and
    the draws, and keeps every pointer: run(), capture() / replay() and tune()
    take no arguments beyond the stream (torch's current one)."""

    def __init__(self, handle, problems):
        torch = _torch()
        self.handle = handle
        self._lib = handle._lib
        self.problems = problems
        T = len(problems)
        dev = problems[0]["M"].device
        self.CD, self.MN, self._offs = [], [], []
        items = (BatchItem_t * T)()
        for t, pr in enumerate(problems):
            M, N = pr["M"], pr["N"]
            if M.dtype != torch.float32 or N.dtype != torch.float32:
                raise ValueError("batches take float32 M and N")
            if M.stride(1) != 1 or N.stride(1) != 1:
                raise ValueError("M and N must be row-major")
            m, n = M.shape
            p = N.shape[1]
            off = np.ascontiguousarray(np.asarray(pr["off"], dtype=np.int64))
            self._offs.append(off)
            CD = torch.empty((m, p), dtype=torch.float32, device=dev)
            MN = torch.empty((m, p), dtype=torch.float32, device=dev)
            self.CD.append(CD)
            self.MN.append(MN)
            it = items[t]
            it.m, it.n, it.p = m, n, p
            it.M, it.ldm = M.data_ptr(), M.stride(0)
            it.N, it.ldn = N.data_ptr(), N.stride(0)
            it.K = len(off) - 1
            it.block_off = off.ctypes.data
            it.c = int(pr["c"])
            it.prob = PROBS[pr.get("prob", "norm")]
            it.seed = int(pr.get("seed", 0))
            it.trial = int(pr.get("trial", 0))
            it.CD, it.ldcd = CD.data_ptr(), p
            it.MN, it.ldmn = MN.data_ptr(), p
        self.cs = [int(pr["c"]) for pr in problems]
        self.err2_mn2 = torch.zeros(2 * T, dtype=torch.float64, device=dev)
        self.L = torch.zeros(T, dtype=torch.int64, device=dev)
        self.idx = torch.zeros(sum(self.cs), dtype=torch.int32, device=dev)
        outs = BatchOutputs_t(self.err2_mn2.data_ptr(), self.L.data_ptr(), self.idx.data_ptr())
        b = ctypes.c_void_p()
        handle._check(self._lib.sbmm_batch_create(handle.h, T, items, ctypes.byref(outs),
                                                  ctypes.byref(b)))
        self.b = b

    def run(self):
        self.handle._check(self._lib.sbmm_batch_run(self.handle.h, self.b, _stream()))

    def capture(self):
        self.handle._check(self._lib.sbmm_batch_capture(self.handle.h, self.b))

    def replay(self):
        self.handle._check(self._lib.sbmm_batch_replay(self.handle.h, self.b, _stream()))

    def tune(self, reps=3):
        """Time every tile configuration and work order of the two grouped
        products and keep the fastest; returns the tuning record as a dict."""
        t = BatchTuning_t()
        self.handle._check(self._lib.sbmm_batch_tune(self.handle.h, self.b, reps, ctypes.byref(t),
                                                     _stream()))
        return self._tuning_dict(t)

    def set_tuning(self, d):
        t = BatchTuning_t()
        for g in range(2):
            t.cfg[g] = d["cfg"][g]
            t.lpt[g] = d["lpt"][g]
            for i in range(BATCH_TUNING_SLOTS):
                t.ms[g][i] = d.get("ms", [[-1.0] * BATCH_TUNING_SLOTS] * 2)[g][i]
        self.handle._check(self._lib.sbmm_batch_set_tuning(self.handle.h, self.b, ctypes.byref(t)))

    @staticmethod
    def _tuning_dict(t):
        n = len(BATCH_TILES)
        return {"cfg": [t.cfg[0], t.cfg[1]], "lpt": [t.lpt[0], t.lpt[1]],
                "tiles": [list(BATCH_TILES[t.cfg[0] % n]), list(BATCH_TILES[t.cfg[1] % n])],
                "sketch_materialized": t.cfg[1] >= n,
                "ms": [[t.ms[g][i] for i in range(BATCH_TUNING_SLOTS)] for g in range(2)]}

    def draws(self, t):
        """The drawn blocks of problem t (device tensor view)."""
        a = sum(self.cs[:t])
        return self.idx[a:a + self.cs[t]]

    def close(self):
        if getattr(self, "b", None):
            self._lib.sbmm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_handles = {}


def default_handle(device):
    """One library handle per device index, created on first use."""
    import torch
    idx = torch.device(device).index or 0
    if idx not in _handles:
        _handles[idx] = Handle(idx)
    return _handles[idx]


def _sampled_matmul_class():
    import torch

    class SampledMatmul(torch.autograd.Function):
        """Y ~ X W by sampling blocks of the inner dimension (block mode):
        forward = norm pass, design and draws, gather of C and D, sketched
        product CD; backward = sbmm_backward with the forward's draws (p is
        held fixed). Arguments: X (m x n), W (n x p), block offsets, c, seed,
        trial, probability rule ("norm", "uniform", "exact" or "user" with
        user weights), compute dtype of the sketch (None = input dtype)."""

        @staticmethod
        def forward(ctx, X, W, off, c, seed=0, trial=0, prob="norm", compute=None, user_w=None):
            h = default_handle(X.device)
            problem = Problem(X.detach(), W.detach(), off, c, prob=prob, seed=seed, trial=trial,
                              user_w=user_w)
            if prob == "exact":
                _, problem.blkprod_sq, _ = h.exact(problem, store=False, blocknorm=True)
            col, row, blk = h.norms(problem)
            plan = h.plan(problem, col, row, blk, sync=True)
            C, D = h.sketch(problem, plan, out_dtype=compute or X.dtype)
            CD, _ = h.sketch_gemm(C, D, plan)
            ctx.compute = C.dtype
            if C.dtype == torch.bfloat16:
                ctx.save_for_backward()       # the bf16 gradient reads X and W, not the sketch
            else:
                ctx.save_for_backward(C, D)
            ctx.problem, ctx.plan, ctx.h = problem, plan, h
            return CD

        @staticmethod
        def backward(ctx, G):
            C, D = ctx.saved_tensors if ctx.compute != torch.bfloat16 else (None, None)
            dM, dN = ctx.h.backward(ctx.problem, ctx.plan, C, D, G.contiguous(), compute=ctx.compute)
            return dM, dN, None, None, None, None, None, None, None

    return SampledMatmul


def __getattr__(name):
    if name == "SampledMatmul":
        cls = _sampled_matmul_class()
        globals()["SampledMatmul"] = cls
        return cls
    # module-level access to the raw C entry points, e.g. sbmm_norms
    if name in EXPORTS:
        return getattr(lib(), name)
    raise AttributeError(name)
