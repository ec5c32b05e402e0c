// Split-K products for small outputs with long inner extents.
//
// The paper's own experiments (Sec. 4) multiply 26 x 5e5 by 5e5 x 28: the
// exact product, the per-block norms ||M^k N_k||_F that (3.9) needs, the
// pilot estimates ||C^{0k} D_{0k}||_F of Alg. 3 and the sketched product CD
// (26 x 5e4 by 5e4 x 28) all have a single output tile, so a tiled kernel
// would run on one workgroup while 255 compute units idle. Here the inner
// dimension is cut into segments that never cross a block boundary; every
// (tile, segment) pair is one workgroup writing its partial tile, and a
// reduction adds the segments of each block in a fixed order, squares the
// block sums for the per-block norms, adds the blocks into the product and
// runs the usual epilogue (store, error against a reference, squared norm).
// These products move (m + p) K elements for 2 m p K flops (m, p <= 128), so
// they are bound by memory and latency, not by the matrix cores: the partial
// kernel is a plain LDS-tiled FMA loop (32 x 32 output tile, 32-wide inner
// chunks, four outputs per thread).
//
// The segment table is built on the device (block offsets may be device
// values, e.g. the strata of a pilot sketch), sized on the host by the bound
// sum_k ceil(n_k / len) <= K_blocks + extent / len.
#include "common.h"

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 32;

struct Seg { int64_t k0, k1; };

template <typename T>
struct SkinnyArgs {
  const T* A; int64_t lda;          // m x extent
  const T* B; int64_t ldb;          // extent x p
  int64_t m, p;
  int64_t K_host; const int64_t* K_dev;
  int32_t nblk; const int64_t* off;  // per-block sums when nblk > 0
  int64_t seg_len, max_segs;
  Seg* segs; int64_t* seg_first; int64_t* nseg;
  double* part;                     // [max_segs][m * p]
  T* C; int64_t ldc;
  const T* Y; int64_t ldy;
  int64_t nred;                     // workgroups of the reduction
  double* e2n2;                     // [2][nred]
  double* blk;                      // [nblk][nred]
};

__device__ double wg_sum(double v, double* sm) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = warp_sum_f64(v);
  __syncthreads();
  if (lane == 0) sm[wave] = v;
  __syncthreads();
  return ((sm[0] + sm[1]) + sm[2]) + sm[3];
}

// Segment table (one workgroup): blocks split into runs of at most seg_len.
template <typename T>
__global__ __launch_bounds__(kThreads) void skinny_segments_kernel(SkinnyArgs<T> a) {
  __shared__ int64_t sm[kThreads];
  const int64_t extent = a.K_dev ? (*a.K_dev + SBMM_SKETCH_PAD - 1) / SBMM_SKETCH_PAD * SBMM_SKETCH_PAD : a.K_host;
  const int64_t nb = a.nblk > 0 ? a.nblk : 1;
  auto range = [&](int64_t k, int64_t* lo, int64_t* hi) {
    *lo = a.nblk > 0 ? min(a.off[k], extent) : 0;
    *hi = a.nblk > 0 ? min(a.off[k + 1], extent) : extent;
  };
  const int64_t per = (nb + kThreads - 1) / kThreads;
  const int64_t b0 = min(nb, (int64_t)threadIdx.x * per), b1 = min(nb, b0 + per);
  int64_t local = 0;
  for (int64_t k = b0; k < b1; ++k) {
    int64_t lo, hi;
    range(k, &lo, &hi);
    local += hi > lo ? (hi - lo + a.seg_len - 1) / a.seg_len : 0;
  }
  sm[threadIdx.x] = local;
  __syncthreads();
  for (int o = 1; o < kThreads; o <<= 1) {
    const int64_t add = (int)threadIdx.x >= o ? sm[threadIdx.x - o] : 0;
    __syncthreads();
    sm[threadIdx.x] += add;
    __syncthreads();
  }
  int64_t run = sm[threadIdx.x] - local;
  const int64_t total = sm[kThreads - 1];
  for (int64_t k = b0; k < b1; ++k) {
    int64_t lo, hi;
    range(k, &lo, &hi);
    a.seg_first[k] = min(run, a.max_segs);
    for (int64_t s = lo; s < hi; s += a.seg_len, ++run)
      if (run < a.max_segs) a.segs[run] = Seg{s, min(hi, s + a.seg_len)};
  }
  if (threadIdx.x == 0) {
    a.seg_first[nb] = min(total, a.max_segs);
    *a.nseg = min(total, a.max_segs);
  }
}

// Partial product of one 32 x 32 output tile over one segment.
template <typename T>
__global__ __launch_bounds__(kThreads) void skinny_partial_kernel(SkinnyArgs<T> a) {
  __shared__ T As[kTile][kTile + 1];   // [row][k]
  __shared__ T Bs[kTile][kTile + 1];   // [k][col]
  const int64_t seg = blockIdx.y;
  if (seg >= *a.nseg) return;
  const Seg sg = a.segs[seg];
  const int64_t tiles_n = (a.p + kTile - 1) / kTile;
  const int64_t m0 = (int64_t)(blockIdx.x / tiles_n) * kTile, n0 = (int64_t)(blockIdx.x % tiles_n) * kTile;
  const int tid = threadIdx.x, c = tid & 31, r0 = tid >> 5;
  T acc[4] = {T(0), T(0), T(0), T(0)};
  for (int64_t kb = sg.k0; kb < sg.k1; kb += kTile) {
#pragma unroll
    for (int q = 0; q < kTile * kTile / kThreads; ++q) {
      const int e = tid + kThreads * q;
      const int hi = e >> 5, lo = e & 31;
      const int64_t ka = kb + lo, row = m0 + hi;
      As[hi][lo] = (row < a.m && ka < sg.k1) ? a.A[row * a.lda + ka] : T(0);
      const int64_t kr = kb + hi, col = n0 + lo;
      Bs[hi][lo] = (kr < sg.k1 && col < a.p) ? a.B[kr * a.ldb + col] : T(0);
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < kTile; ++kk) {
      const T b = Bs[kk][c];
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] = fma(As[r0 + 8 * i][kk], b, acc[i]);
    }
    __syncthreads();
  }
  double* out = a.part + seg * (a.m * a.p);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = m0 + r0 + 8 * i, col = n0 + c;
    if (row < a.m && col < a.p) out[row * a.p + col] = (double)acc[i];
  }
}

// One thread per output element: per block, the fixed-order sum of its
// segments (squared and reduced over the workgroup for the block norms);
// the blocks add up to the product, then store, error and norm.
template <typename T>
__global__ __launch_bounds__(kThreads) void skinny_reduce_kernel(SkinnyArgs<T> a) {
  __shared__ double sm[4];
  const int64_t mp = a.m * a.p;
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool valid = e < mp;
  const int64_t nb = a.nblk > 0 ? a.nblk : 1;
  double total = 0.0;
  for (int64_t k = 0; k < nb; ++k) {
    const int64_t s0 = a.seg_first[k], s1 = a.seg_first[k + 1];
    double z = 0.0;
    if (valid) {
#pragma unroll 8
      for (int64_t s = s0; s < s1; ++s) z += a.part[s * mp + e];
    }
    total += z;
    if (a.nblk > 0) {
      const double sq = wg_sum(valid ? z * z : 0.0, sm);
      if (threadIdx.x == 0) a.blk[k * a.nred + blockIdx.x] = sq;
    }
  }
  double e2 = 0.0, n2 = 0.0;
  if (valid) {
    const int64_t row = e / a.p, col = e % a.p;
    const T val = (T)total;
    if (a.C) a.C[row * a.ldc + col] = val;
    const double dv = (double)val;
    if (a.Y) {
      const double d = dv - (double)a.Y[row * a.ldy + col];
      e2 = d * d;
    }
    n2 = dv * dv;
  }
  e2 = wg_sum(e2, sm);
  n2 = wg_sum(n2, sm);
  if (threadIdx.x == 0) {
    a.e2n2[blockIdx.x] = e2;
    a.e2n2[a.nred + blockIdx.x] = n2;
  }
}

// Row r of src ([rows][cols]) summed in a fixed order into column 0 of row r
// of dst ([rows][dcols]); the other columns of dst are zeroed, so the
// callers' own reduction over dcols columns yields the sum.
__global__ __launch_bounds__(kThreads) void skinny_place_kernel(const double* __restrict__ src, int64_t cols,
                                                                double* __restrict__ dst, int64_t dcols) {
  __shared__ double sm[4];
  const int64_t r = blockIdx.x;
  double s = 0.0;
  for (int64_t c = threadIdx.x; c < cols; c += kThreads) s += src[r * cols + c];
  s = wg_sum(s, sm);
  for (int64_t c = threadIdx.x; c < dcols; c += kThreads) dst[r * dcols + c] = c == 0 ? s : 0.0;
}

struct Plan {
  int64_t tiles, seg_len, max_segs, nred, nb;
};

Plan skinny_plan(int64_t m, int64_t p, int64_t K_max, int32_t nblk) {
  Plan q{};
  q.tiles = ceil_div(m, kTile) * ceil_div(p, kTile);
  // about 1024 workgroups over the tiles, partials capped near 32 MiB
  int64_t target = std::max<int64_t>(1, 1024 / q.tiles);
  target = std::min<int64_t>(target, std::max<int64_t>(16, ((int64_t)1 << 22) / (m * p)));
  q.seg_len = std::min<int64_t>(4096, std::max<int64_t>(128, round_up(ceil_div(K_max, target), kTile)));
  q.nb = nblk > 0 ? nblk : 1;
  q.max_segs = q.nb + ceil_div(K_max, q.seg_len);
  q.nred = ceil_div(m * p, kThreads);
  return q;
}

size_t take(size_t& off, size_t bytes) {
  off = (off + 255) & ~size_t(255);
  const size_t at = off;
  off += bytes ? bytes : 1;
  return at;
}

struct Layout {
  size_t segs, seg_first, nseg, part, e2n2, blk, total;
};

Layout skinny_layout(const Plan& q, int64_t m, int64_t p, int32_t nblk) {
  Layout l{};
  size_t off = 0;
  l.segs = take(off, sizeof(Seg) * q.max_segs);
  l.seg_first = take(off, sizeof(int64_t) * (q.nb + 1));
  l.nseg = take(off, sizeof(int64_t));
  l.part = take(off, sizeof(double) * q.max_segs * m * p);
  l.e2n2 = take(off, sizeof(double) * 2 * q.nred);
  l.blk = take(off, sizeof(double) * (nblk > 0 ? nblk : 1) * q.nred);
  l.total = off;
  return l;
}

template <typename T>
hipError_t run_skinny(const GemmLaunch& L, int64_t tiles_out, int64_t blk_cols, hipStream_t s) {
  const bool bn = L.blk_part != nullptr;
  const int32_t nblk = bn ? L.K_blocks : 0;
  const int64_t K_max = L.skinny_K_max;
  const Plan q = skinny_plan(L.m, L.p, K_max, nblk);
  const Layout l = skinny_layout(q, L.m, L.p, nblk);
  char* ws = reinterpret_cast<char*>(L.skinny_ws);
  SkinnyArgs<T> a{};
  a.A = reinterpret_cast<const T*>(L.A); a.lda = L.lda;
  a.B = reinterpret_cast<const T*>(L.B); a.ldb = L.ldb;
  a.m = L.m; a.p = L.p; a.K_host = L.K_host; a.K_dev = L.K_dev;
  a.nblk = nblk; a.off = L.off_dev;
  a.seg_len = q.seg_len; a.max_segs = q.max_segs;
  a.segs = reinterpret_cast<Seg*>(ws + l.segs);
  a.seg_first = reinterpret_cast<int64_t*>(ws + l.seg_first);
  a.nseg = reinterpret_cast<int64_t*>(ws + l.nseg);
  a.part = reinterpret_cast<double*>(ws + l.part);
  a.C = reinterpret_cast<T*>(L.Cout); a.ldc = L.ldc;
  a.Y = reinterpret_cast<const T*>(L.Y); a.ldy = L.ldy;
  a.nred = q.nred;
  a.e2n2 = reinterpret_cast<double*>(ws + l.e2n2);
  a.blk = reinterpret_cast<double*>(ws + l.blk);
  hipLaunchKernelGGL(skinny_segments_kernel<T>, dim3(1), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(skinny_partial_kernel<T>, dim3((unsigned)q.tiles, (unsigned)q.max_segs), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(skinny_reduce_kernel<T>, dim3((unsigned)q.nred), dim3(kThreads), 0, s, a);
  if (L.tile_part)
    hipLaunchKernelGGL(skinny_place_kernel, dim3(2), dim3(kThreads), 0, s, a.e2n2, q.nred, L.tile_part, tiles_out);
  if (bn && nblk > 0)
    hipLaunchKernelGGL(skinny_place_kernel, dim3((unsigned)nblk), dim3(kThreads), 0, s, a.blk, q.nred, L.blk_part,
                       blk_cols);
  return hipGetLastError();
}

}  // namespace

size_t gemm_skinny_ws_bytes(sbmm_dtype dt, int64_t m, int64_t p, int64_t K_max, int32_t nblk) {
  if (dt != SBMM_F32 && dt != SBMM_F64) return 0;
  if (m < 1 || p < 1 || K_max < 2048) return 0;
  if (m > 128 || p > 128) return 0;
  const Plan q = skinny_plan(m, p, K_max, nblk);
  if (q.max_segs > 65535) return 0;   // grid.y limit: very many blocks take the tiled kernels
  return skinny_layout(q, m, p, nblk).total;
}

hipError_t launch_gemm_skinny(const GemmLaunch& L, int64_t tiles_out, int64_t blk_cols, hipStream_t s) {
  if (L.dt == SBMM_F64) return run_skinny<double>(L, tiles_out, blk_cols, s);
  if (L.dt == SBMM_F32) return run_skinny<float>(L, tiles_out, blk_cols, s);
  return hipErrorInvalidValue;
}
