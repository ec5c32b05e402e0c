"""Seeded synthetic inputs for the sampled block matrix product.

This module only makes inputs: matrices, block partitions and problem sizes.
It holds none of the method's arithmetic (no norms, probabilities, draws or
products), so that both the HIP library's tests and the CPU oracle can take
their inputs from it without sharing any computation.

All generators are NumPy ``Generator(PCG64(seed))`` streams.

Workloads (shapes and distributions from the paper's experiments, Sec. 4,
and the block-sampling settings this project measures):

* ``tiny``        M 256x1024, N 1024x256 float64 N(0,1), 64 blocks of 16.
* ``paper_scale`` M 4096x65536, N 65536x4096 float32, M = G1 diag(f),
                  N = diag(g) G2 with G N(0,1) and f, g independent
                  lognormal(0, 1.5) factors, 1024 uneven blocks of 16..112.
* ``case1/case2`` the paper's Case I / Case II data (Sec. 4): columns of M
                  i.i.d. N(0, S1) or multivariate t_1 located at the all-ones
                  vector with scale S1, rows of N likewise with S2, where
                  S1 = (0.7^|i-j|) (m x m) and S2 = (2 * 0.7^|i-j|) (p x p).
* ``batched``     per-trial sizes of the 512-problem batched workload; its
                  matrices come from a counter-based stream (``philox_matrix``
                  on the host, ``device_fill`` on the GPU, bit-identical) so
                  that 87 GB of inputs can be written in place on the device
                  and any trial regenerated on the host.
* ``linear``      the activations / weights / upstream gradient of the
                  differentiable linear layer.
"""

import numpy as np

__all__ = [
    "rng", "gaussian", "uneven_blocks", "equal_blocks", "tiny",
    "paper_scale", "paper_scale_factors", "case_data", "batched_sizes",
    "linear_layer", "random_problem", "philox_matrix", "device_fill",
    "INPUT_SEED", "batched_item_streams", "batched_device_inputs",
]

INPUT_SEED = 3          # key word 0 of the batched workload's input streams
_TAG_INPUT = 3
_UNIT_SCALE = np.float32(float.fromhex("0x1.bb67aep-16"))   # float32(1/sqrt((2^32-1)/3))


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def gaussian(shape, seed, dtype=np.float64, scale=1.0, gen=None):
    g = gen if gen is not None else rng(seed)
    if dtype in (np.float32, np.float64):
        x = g.standard_normal(shape, dtype=dtype)
    else:
        x = g.standard_normal(shape, dtype=np.float32)
    if scale != 1.0:
        x *= np.asarray(scale, dtype=x.dtype)
    return x


def equal_blocks(n, K):
    """Offsets of K blocks of n/K (K must divide n)."""
    if n % K:
        raise ValueError("K must divide n")
    return [k * (n // K) for k in range(K + 1)]


def uneven_blocks(n, K, lo, hi, seed):
    """K block sizes drawn uniformly in [lo, hi] and then repaired, one
    seeded +-1 step at a time inside the bounds, until they sum to n.
    Returns the K+1 offsets."""
    if not (K * lo <= n <= K * hi):
        raise ValueError("n is not reachable with K blocks in [lo, hi]")
    g = rng(seed)
    sz = g.integers(lo, hi + 1, size=K).astype(np.int64)
    diff = n - int(sz.sum())
    while diff != 0:
        step = 1 if diff > 0 else -1
        movable = np.nonzero(sz < hi if step > 0 else sz > lo)[0]
        take = movable[g.integers(0, len(movable), size=min(abs(diff), len(movable)))]
        take = np.unique(take)
        sz[take] += step
        diff -= step * len(take)
    return [0] + np.cumsum(sz).tolist()


def tiny(seed=0):
    """M 256x1024, N 1024x256 float64 N(0,1) from one stream (M then N),
    64 equal blocks of 16 columns / rows."""
    g = rng(seed)
    M = g.standard_normal((256, 1024))
    N = g.standard_normal((1024, 256))
    return M, N, equal_blocks(1024, 64)


def paper_scale_factors(n, seed=2, sigma=1.5):
    """Independent lognormal(0, sigma) factors f (columns of M) and g (rows
    of N)."""
    g = rng(seed)
    f = g.lognormal(0.0, sigma, size=n)
    h = g.lognormal(0.0, sigma, size=n)
    return f, h


def paper_scale(m=4096, n=65536, p=4096, K=1024, dtype=np.float32,
                seeds=(1, 2, 3)):
    """M = G1 diag(f), N = diag(g) G2: Gaussian matrices whose column j of M
    and row j of N are scaled by lognormal(0, 1.5) factors, so that the
    block norms are skewed; 1024 uneven blocks of 16..112 summing to n."""
    g = rng(seeds[0])
    M = g.standard_normal((m, n), dtype=np.float32)
    N = g.standard_normal((n, p), dtype=np.float32)
    f, h = paper_scale_factors(n, seeds[1])
    M *= f.astype(np.float32)[None, :]
    N *= h.astype(np.float32)[:, None]
    lo, hi = (16, 112) if n >= 16 * K else (1, max(1, 2 * n // K - 1))
    off = uneven_blocks(n, K, lo, hi, seeds[2])
    if dtype != np.float32:
        M = M.astype(dtype)
        N = N.astype(dtype)
    return M, N, off


def _toeplitz(dim, base, rho=0.7):
    idx = np.arange(dim)
    return base * rho ** np.abs(idx[:, None] - idx[None, :])


def case_data(case, m=26, n=500000, p=28, seed=7):
    """The paper's Sec. 4 data. Case I: columns of M ~ N(0, S1), rows of N ~
    N(0, S2). Case II: columns of M ~ t_1 with location the all-ones vector
    and scale S1 (x = 1 + z / sqrt(w), z ~ N(0, S1), w ~ chi^2_1), rows of N
    likewise with S2. S1 = (0.7^|i-j|), S2 = (2 * 0.7^|i-j|)."""
    g = rng(seed)
    L1 = np.linalg.cholesky(_toeplitz(m, 1.0))
    L2 = np.linalg.cholesky(_toeplitz(p, 2.0))
    Z1 = g.standard_normal((n, m)) @ L1.T    # row j = column j of M
    Z2 = g.standard_normal((n, p)) @ L2.T    # row j = row j of N
    if case == 1:
        return np.ascontiguousarray(Z1.T), Z2
    if case == 2:
        w1 = g.chisquare(1.0, size=n)
        w2 = g.chisquare(1.0, size=n)
        M = 1.0 + Z1 / np.sqrt(w1)[:, None]
        N = 1.0 + Z2 / np.sqrt(w2)[:, None]
        return np.ascontiguousarray(M.T), N
    raise ValueError("case must be 1 or 2")


def batched_sizes(T=512, seed=11):
    """Per-trial sizes of the batched workload: m, p uniform in [256, 2048],
    n uniform in [4096, 32768], blocks of 8..128, c uniform in [16, 256].
    Returns a list of dicts (m, n, p, off, c)."""
    g = rng(seed)
    out = []
    for t in range(T):
        m = int(g.integers(256, 2049))
        p = int(g.integers(256, 2049))
        n = int(g.integers(4096, 32769))
        K = max(1, round(n / 68))            # mean of U{8..128} is 68
        off = uneven_blocks(n, K, 8, 128, int(g.integers(0, 2**31)))
        c = int(g.integers(16, 257))
        out.append(dict(m=m, n=n, p=p, off=off, c=c))
    return out


def linear_layer(batch=8192, d_in=16384, d_out=8192, seed=21):
    """Activations X ~ N(0,1), weights W ~ N(0, 0.01^2), upstream gradient
    G ~ N(0,1), all float32 (the caller casts to bf16)."""
    g = rng(seed)
    X = g.standard_normal((batch, d_in), dtype=np.float32)
    W = g.standard_normal((d_in, d_out), dtype=np.float32) * np.float32(0.01)
    G = g.standard_normal((batch, d_out), dtype=np.float32)
    return X, W, G


def random_problem(m, n, p, K, seed, dtype=np.float64, lo=None, hi=None,
                   skew=0.0):
    """Small random problem for tests: Gaussian M, N (optionally with
    lognormal(0, skew) column / row factors) and K uneven blocks."""
    g = rng(seed)
    M = g.standard_normal((m, n))
    N = g.standard_normal((n, p))
    if skew > 0:
        M *= g.lognormal(0.0, skew, size=n)[None, :]
        N *= g.lognormal(0.0, skew, size=n)[:, None]
    avg = n // K
    lo = max(1, avg // 2) if lo is None else lo
    hi = max(lo, 2 * avg - lo) if hi is None else hi
    if K * lo > n or K * hi < n:
        lo, hi = 1, n
    off = uneven_blocks(n, K, lo, hi, seed + 1000003)
    return M.astype(dtype), N.astype(dtype), off


def batched_item_streams(t):
    """Stream ids of trial t's M and N in the batched workload."""
    return 2 * t, 2 * t + 1


def philox_matrix(rows, cols, seed, stream, scale=1.0):
    """rows x cols float32: element q = r * cols + c from 64-bit word q % 4
    of the Philox4x64-10 block with key (seed, 0) and counter
    (q // 4, stream, 0, 3 * 2^32) (NumPy's Philox, which advances its
    counter before each block, so it starts one below); the four 16-bit
    pieces of the word are summed, centred and scaled to unit variance
    (Irwin-Hall of four uniforms), then multiplied by ``scale`` in float32
    (skipped for 1). The same bits as workloads/gen.hip on the device."""
    total = rows * cols
    nblk = (total + 3) // 4
    ctr = (0 | (stream << 64) | (0 << 128) | ((_TAG_INPUT << 32) << 192)) - 1
    ctr %= 1 << 256
    start = np.array([(ctr >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(counter=start, key=np.array([seed, 0], dtype=np.uint64))
    w = bg.random_raw(4 * nblk)[:total]
    m16 = np.uint64(0xffff)
    s = (w & m16) + ((w >> np.uint64(16)) & m16) + ((w >> np.uint64(32)) & m16) + (w >> np.uint64(48))
    x = (s.astype(np.int64) - 131070).astype(np.float32) * _UNIT_SCALE
    if scale != 1.0:
        x = x * np.float32(scale)
    return x.reshape(rows, cols)


_wl_lib = None


def device_fill(x, seed, stream, scale=1.0):
    """Fill the float32 device tensor x (2-D, row-major, any leading
    dimension; memory between rows is not touched) with the stream
    ``philox_matrix`` describes, on torch's current stream."""
    import ctypes
    import os
    import torch
    global _wl_lib
    if _wl_lib is None:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsbmm_workload.so")
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: run paper_2105_04940_amd.build.build_workload()")
        lib = ctypes.CDLL(path)
        lib.sbmm_workload_fill.restype = ctypes.c_int
        lib.sbmm_workload_fill.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_uint64, ctypes.c_uint64, ctypes.c_float, ctypes.c_void_p]
        _wl_lib = lib
    if x.dtype != torch.float32 or x.dim() != 2 or x.stride(1) != 1:
        raise ValueError("device_fill takes a row-major 2-D float32 tensor")
    rows, cols = x.shape
    ld = x.stride(0)
    err = _wl_lib.sbmm_workload_fill(ctypes.c_void_p(x.data_ptr()), rows, cols, ld, seed, stream,
                                     float(scale), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if err != 0:
        raise RuntimeError(f"sbmm_workload_fill failed with hipError {err}")


def batched_device_inputs(T=512, seed=11, device="cuda:0"):
    """The batched workload on the device: per trial t (sizes from
    ``batched_sizes``) M_t and N_t written in place by ``device_fill`` from
    streams ``batched_item_streams(t)`` of INPUT_SEED, each with its leading
    dimension rounded up to a multiple of 4 floats (16-byte rows). Returns
    the size dicts and a list of (M_t, N_t) tensor views."""
    import torch
    items = batched_sizes(T, seed=seed)
    mats = []
    for t, it in enumerate(items):
        sm, sn = batched_item_streams(t)
        Mb = torch.empty((it["m"], (it["n"] + 3) // 4 * 4), dtype=torch.float32, device=device)
        Nb = torch.empty((it["n"], (it["p"] + 3) // 4 * 4), dtype=torch.float32, device=device)
        M = Mb[:, :it["n"]]
        N = Nb[:, :it["p"]]
        device_fill(M, INPUT_SEED, sm)
        device_fill(N, INPUT_SEED, sn)
        mats.append((M, N))
    return items, mats
