// Norm pass: squared column norms of M, squared row norms of N and the
// per-block statistics ||M^k||_F^2, ||N_k||_F^2 and s_k = sum_i a_i b_i that
// the probability rules (1.1), (1.4), (3.8) and the block sizes (4.2) are
// built from.
//
// Both inputs are row-major and streamed once from HBM with 16-byte loads:
//  * M (m x n): a wave covers 64 * E consecutive columns of one row (E
//    elements per 16 bytes), the four waves of a workgroup take rows
//    round-robin, and the row range is split R ways; each workgroup leaves a
//    float64 partial per column, summed in split order by the finalize
//    kernel.
//  * N (n x p): a group of G lanes (G = 64 for wide rows, fewer for short
//    rows) reduces one row with cross-lane shuffles.
// Sums are float64 in a fixed order, so the result is bitwise reproducible.
#include <algorithm>
#include <cstring>

#include "common.h"

namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 8;

template <typename T> __device__ __forceinline__ void vec_to_double(const uint4& v, double* out);
template <> __device__ __forceinline__ void vec_to_double<double>(const uint4& v, double* out) {
  out[0] = __hiloint2double(v.y, v.x);
  out[1] = __hiloint2double(v.w, v.z);
}
template <> __device__ __forceinline__ void vec_to_double<float>(const uint4& v, double* out) {
  out[0] = (double)__uint_as_float(v.x); out[1] = (double)__uint_as_float(v.y);
  out[2] = (double)__uint_as_float(v.z); out[3] = (double)__uint_as_float(v.w);
}
template <> __device__ __forceinline__ void vec_to_double<uint16_t>(const uint4& v, double* out) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    out[2 * i] = (double)__uint_as_float(w[i] << 16);
    out[2 * i + 1] = (double)__uint_as_float(w[i] & 0xffff0000u);
  }
}

struct NormArgs {
  const void* M; int64_t ldm;
  const void* N; int64_t ldn;
  int64_t m, n, p;
  int rsplit; int64_t rows_per_split;
  int64_t mtiles;            // column tiles of M
  int64_t nblocks_m;         // workgroups on the M part
  int n_group;               // lanes per row of N
  int64_t rows_per_wg_n;     // rows of N per workgroup
  int vec_m, vec_n;          // 16-byte loads allowed (alignment of base and leading dim)
  double* partial;
  double* row_sq;
};

template <typename T>
__device__ void colsq_part(const NormArgs& a, int64_t bid, double* sm) {
  constexpr int E = 16 / sizeof(T);
  constexpr int TC = 64 * E;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t tile = bid % a.mtiles;
  const int64_t split = bid / a.mtiles;
  const int64_t j0 = tile * TC + (int64_t)lane * E;
  const int64_t r0 = split * a.rows_per_split;
  const int64_t r1 = min(a.m, r0 + a.rows_per_split);
  const T* M = reinterpret_cast<const T*>(a.M);

  double acc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) acc[e] = 0.0;

  const bool full = a.vec_m && (j0 + E <= a.n);
  if (full) {
    int64_t r = r0 + wave;
    for (; r + 4 * (kUnroll - 1) < r1; r += 4 * kUnroll) {
      uint4 v[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
        v[u] = *reinterpret_cast<const uint4*>(M + (r + 4 * u) * a.ldm + j0);
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        double x[E];
        vec_to_double<T>(v[u], x);
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] = fma(x[e], x[e], acc[e]);
      }
    }
    for (; r < r1; r += 4) {
      uint4 v = *reinterpret_cast<const uint4*>(M + r * a.ldm + j0);
      double x[E];
      vec_to_double<T>(v, x);
#pragma unroll
      for (int e = 0; e < E; ++e) acc[e] = fma(x[e], x[e], acc[e]);
    }
  } else if (j0 < a.n) {
    for (int64_t r = r0 + wave; r < r1; r += 4) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (j0 + e < a.n) {
          double x = Elem<T>::to_double(M[r * a.ldm + j0 + e]);
          acc[e] = fma(x, x, acc[e]);
        }
      }
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) sm[wave * TC + lane * E + e] = acc[e];
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int c = lane * E + e;
      double s = sm[c];
      s += sm[TC + c];
      s += sm[2 * TC + c];
      s += sm[3 * TC + c];
      if (j0 + e < a.n) a.partial[split * a.n + j0 + e] = s;
    }
  }
}

template <typename T>
__device__ void rowsq_part(const NormArgs& a, int64_t bid) {
  constexpr int E = 16 / sizeof(T);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int G = a.n_group;
  const int per_wave = 64 / G;
  const int grp = lane / G;
  const int li = lane % G;
  const T* N = reinterpret_cast<const T*>(a.N);
  const int64_t row_begin = bid * a.rows_per_wg_n;
  const int64_t row_end = min(a.n, row_begin + a.rows_per_wg_n);
  const int64_t nvec = (a.p + E - 1) / E;
  for (int64_t rb = row_begin + (int64_t)wave * per_wave; rb < row_end; rb += 4 * per_wave) {
    const int64_t i = rb + grp;
    double acc = 0.0;
    if (i < row_end) {
      const T* row = N + i * a.ldn;
      int64_t v = li;
      if (a.vec_n) {
        for (; v + (int64_t)G * 3 < nvec; v += 4 * (int64_t)G) {
          uint4 q[4];
          bool ok[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int64_t c = (v + (int64_t)u * G) * E;
            ok[u] = c + E <= a.p;
            if (ok[u]) q[u] = *reinterpret_cast<const uint4*>(row + c);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int64_t c = (v + (int64_t)u * G) * E;
            if (ok[u]) {
              double x[E];
              vec_to_double<T>(q[u], x);
#pragma unroll
              for (int e = 0; e < E; ++e) acc = fma(x[e], x[e], acc);
            } else {
              for (int e = 0; e < E; ++e)
                if (c + e < a.p) {
                  double x = Elem<T>::to_double(row[c + e]);
                  acc = fma(x, x, acc);
                }
            }
          }
        }
      }
      for (; v < nvec; v += G) {
        const int64_t c = v * E;
        if (a.vec_n && c + E <= a.p) {
          double x[E];
          vec_to_double<T>(*reinterpret_cast<const uint4*>(row + c), x);
#pragma unroll
          for (int e = 0; e < E; ++e) acc = fma(x[e], x[e], acc);
        } else {
          for (int e = 0; e < E; ++e)
            if (c + e < a.p) {
              double x = Elem<T>::to_double(row[c + e]);
              acc = fma(x, x, acc);
            }
        }
      }
    }
    for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (li == 0 && i < row_end) a.row_sq[i] = acc;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void norms_kernel(NormArgs a) {
  __shared__ double sm[4 * 64 * (16 / sizeof(T))];
  const int64_t bid = blockIdx.x;
  if (bid < a.nblocks_m)
    colsq_part<T>(a, bid, sm);
  else
    rowsq_part<T>(a, bid - a.nblocks_m);
}

struct StatsArgs {
  const double* partial; int rsplit; int64_t n;
  const int64_t* off; int32_t K;
  double* col_sq; const double* row_sq; double* blk;
  int32_t* status;
  int32_t chunks;            // workgroups per block (1: whole block, writes blk)
  double* stats_part;        // chunks > 1: [3][K][chunks]
};

// Columns of a statistics chunk (blocks wider than one workgroup's share).
constexpr int64_t kStatsChunk = (int64_t)kThreads * 8;

// Workgroup (block k, chunk c): finish the column sums over the row splits
// for its columns and form the three block statistics over them (the whole
// block when chunks == 1, then written to blk; else to the chunk partials).
__device__ void block_stats_body(const StatsArgs& s, int k, int c) {
  const double* __restrict__ partial = s.partial;
  const int rsplit = s.rsplit;
  const int64_t n = s.n;
  const int64_t* __restrict__ off = s.off;
  const int32_t K = s.K;
  double* __restrict__ col_sq = s.col_sq;
  const double* __restrict__ row_sq = s.row_sq;
  double* __restrict__ blk = s.blk;
  int32_t* status = s.status;
  __shared__ double sm[3][kThreads];
  int64_t lo = off[k], hi = off[k + 1];
  if (s.chunks > 1) {
    lo += c * kStatsChunk;
    hi = min(hi, lo + kStatsChunk);
  }
  double am = 0.0, an = 0.0, as = 0.0;
  bool bad = false;
#pragma unroll 8
  for (int64_t j = lo + threadIdx.x; j < hi; j += kThreads) {
    double cs = 0.0;
    for (int r = 0; r < rsplit; ++r) cs += partial[(int64_t)r * n + j];
    col_sq[j] = cs;
    const double rs = row_sq[j];
    bad |= !isfinite(cs) || !isfinite(rs);
    am += cs;
    an += rs;
    as += sqrt(cs * rs);
  }
  if (bad) *status = SBMM_DEV_NONFINITE;
  sm[0][threadIdx.x] = am;
  sm[1][threadIdx.x] = an;
  sm[2][threadIdx.x] = as;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sm[0][threadIdx.x] += sm[0][threadIdx.x + h];
      sm[1][threadIdx.x] += sm[1][threadIdx.x + h];
      sm[2][threadIdx.x] += sm[2][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (s.chunks == 1) {
      blk[k] = sm[0][0];
      blk[K + k] = sm[1][0];
      blk[2 * K + k] = sm[2][0];
    } else {
      const int64_t q = (int64_t)k * s.chunks + c, stride = (int64_t)K * s.chunks;
      s.stats_part[q] = sm[0][0];
      s.stats_part[stride + q] = sm[1][0];
      s.stats_part[2 * stride + q] = sm[2][0];
    }
  }
}

// chunks > 1: per block, the chunk partials summed in chunk order (chunks
// past the block's end hold zeros)
__global__ __launch_bounds__(kThreads) void block_stats_combine_kernel(StatsArgs s) {
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k >= s.K) return;
  const int64_t stride = (int64_t)s.K * s.chunks;
  for (int f = 0; f < 3; ++f) {
    double v = 0.0;
    for (int c = 0; c < s.chunks; ++c) v += s.stats_part[f * stride + k * s.chunks + c];
    s.blk[f * s.K + k] = v;
  }
}

__global__ __launch_bounds__(kThreads) void block_stats_kernel(StatsArgs s) {
  block_stats_body(s, blockIdx.x / s.chunks, blockIdx.x % s.chunks);
}

// Last t with off[t] <= x (off ascending, off[0] = 0 <= x).
__device__ __forceinline__ int32_t find_problem(const int64_t* __restrict__ off, int32_t T, int64_t x) {
  int32_t lo = 0, hi = T;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// Norm pass of many problems in one launch: workgroup b belongs to the
// problem t with wg_off[t] <= b < wg_off[t+1] and runs that problem's
// workgroup b - wg_off[t].
template <typename T>
__global__ __launch_bounds__(kThreads) void batch_norms_kernel(const NormArgs* __restrict__ args,
                                                               const int64_t* __restrict__ wg_off, int32_t count) {
  __shared__ double sm[4 * 64 * (16 / sizeof(T))];
  const int64_t bid = blockIdx.x;
  const int32_t t = find_problem(wg_off, count, bid);
  const NormArgs a = args[t];   // a copy: read once, not reloaded behind the kernel's stores
  const int64_t local = bid - wg_off[t];
  if (local < a.nblocks_m)
    colsq_part<T>(a, local, sm);
  else
    rowsq_part<T>(a, local - a.nblocks_m);
}

__global__ __launch_bounds__(kThreads) void batch_stats_kernel(const StatsArgs* __restrict__ args,
                                                               const int64_t* __restrict__ blk_off, int32_t count) {
  const int64_t bid = blockIdx.x;
  const int32_t t = find_problem(blk_off, count, bid);
  const StatsArgs a = args[t];
  block_stats_body(a, (int)(bid - blk_off[t]), 0);
}

int elems_per_vec(sbmm_dtype dt) { return 16 / (int)dtype_size(dt); }

// Argument block of one problem's norm pass; returns its workgroup count.
int64_t make_norm_args(const NormLaunch& L, NormArgs* out) {
  NormArgs a{};
  a.M = L.M; a.ldm = L.ldm; a.N = L.N; a.ldn = L.ldn;
  a.m = L.m; a.n = L.n; a.p = L.p;
  a.partial = L.partial; a.row_sq = L.row_sq;
  const int E = elems_per_vec(L.dt);
  const size_t es = dtype_size(L.dt);
  a.rsplit = L.rsplit;
  a.rows_per_split = ceil_div(L.m > 0 ? L.m : 1, L.rsplit);
  a.mtiles = ceil_div(L.n, 64 * E);
  a.nblocks_m = L.m > 0 ? a.mtiles * L.rsplit : 0;
  a.vec_m = ((uintptr_t)L.M % 16 == 0) && ((L.ldm * (int64_t)es) % 16 == 0);
  a.vec_n = ((uintptr_t)L.N % 16 == 0) && ((L.ldn * (int64_t)es) % 16 == 0);
  const int64_t nvec = ceil_div(L.p, E);
  int G = 1;
  while (G < 64 && G < nvec) G <<= 1;
  a.n_group = G;
  const int64_t rows_per_step = 4 * (64 / G);
  const int64_t steps = L.p > 0 ? std::max<int64_t>(1, ceil_div(L.n, rows_per_step * 8192)) : 0;
  a.rows_per_wg_n = rows_per_step * std::max<int64_t>(steps, 1);
  const int64_t nblocks_n = L.p > 0 ? ceil_div(L.n, a.rows_per_wg_n) : 0;
  *out = a;
  return a.nblocks_m + nblocks_n;
}

StatsArgs make_stats_args(const NormLaunch& L) {
  return StatsArgs{L.partial, L.m > 0 ? L.rsplit : 1, L.n, L.off_dev, L.K, L.col_sq, L.row_sq, L.blk, L.status,
                   L.stats_part ? std::max<int32_t>(L.stats_chunks, 1) : 1, L.stats_part};
}

}  // namespace

// Row splits of M: about 1024 workgroups on M (four per CU, each streaming
// a long run of rows: on a 4096 x 65536 float32 M this reads at 6.2 TB/s,
// against 5.9 TB/s with 4096 shorter ones), but at least 32 rows per split.
// The N part adds about 8192 workgroups of its own (8 rows of 16 KB each at
// that shape).
size_t norms_partial_elems(sbmm_dtype dt, int64_t m, int64_t n, int* rsplit_out) {
  const int64_t tiles = ceil_div(n, 64 * elems_per_vec(dt));
  int64_t want = ceil_div(1024, tiles > 0 ? tiles : 1);
  int64_t maxr = m / 32 > 1 ? m / 32 : 1;
  int64_t R = want < 1 ? 1 : (want > maxr ? maxr : want);
  if (R > 64) R = 64;
  *rsplit_out = (int)R;
  return (size_t)R * (size_t)n;
}

hipError_t launch_norms(const NormLaunch& L, hipStream_t s) {
  NormArgs a;
  const int64_t total = make_norm_args(L, &a);
  hipError_t e = hipSuccess;
  if (L.m == 0 && (e = launch_fill_f64(L.partial, L.rsplit * L.n, 0.0, s)) != hipSuccess) return e;
  if (L.p == 0 && (e = launch_fill_f64(L.row_sq, L.n, 0.0, s)) != hipSuccess) return e;
  if (total > 0) {
    dim3 grid((unsigned)total), block(kThreads);
    switch (L.dt) {
      case SBMM_F64: hipLaunchKernelGGL(norms_kernel<double>, grid, block, 0, s, a); break;
      case SBMM_F32: hipLaunchKernelGGL(norms_kernel<float>, grid, block, 0, s, a); break;
      case SBMM_BF16: hipLaunchKernelGGL(norms_kernel<uint16_t>, grid, block, 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  const StatsArgs st = make_stats_args(L);
  hipLaunchKernelGGL(block_stats_kernel, dim3((unsigned)((int64_t)L.K * st.chunks)), dim3(kThreads), 0, s, st);
  if (st.chunks > 1)
    hipLaunchKernelGGL(block_stats_combine_kernel, dim3((unsigned)ceil_div(L.K, kThreads)), dim3(kThreads), 0, s, st);
  return hipGetLastError();
}

// Blocks wider than two chunks are split when that keeps the grid dense
// (at most twice the workgroups a perfect split would need).
int32_t norms_stats_chunks(int64_t n, int32_t K, int64_t max_width) {
  const int64_t c = ceil_div(max_width, kStatsChunk);
  if (c <= 2) return 1;
  const int64_t dense = ceil_div(n, kStatsChunk) + K;
  return (int64_t)K * c <= 2 * dense ? (int32_t)c : 1;
}

// ----------------------------------------------------------------------------
// Batched form: host-built argument blocks, uploaded once by the caller.
// ----------------------------------------------------------------------------
size_t batch_norm_args_bytes() { return sizeof(NormArgs); }
size_t batch_stats_args_bytes() { return sizeof(StatsArgs); }

int64_t build_batch_norm_args(const NormLaunch& L, void* norm_out, void* stats_out) {
  NormArgs a;
  const int64_t wg = make_norm_args(L, &a);
  std::memcpy(norm_out, &a, sizeof(a));
  const StatsArgs st = make_stats_args(L);
  std::memcpy(stats_out, &st, sizeof(st));
  return wg;
}

hipError_t launch_batch_norms(sbmm_dtype dt, const void* norm_args, const int64_t* wg_off, int64_t total_wg,
                              const void* stats_args, const int64_t* blk_off, int64_t total_blk,
                              int32_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const NormArgs* na = reinterpret_cast<const NormArgs*>(norm_args);
  if (total_wg > 0) {
    dim3 grid((unsigned)total_wg), block(kThreads);
    switch (dt) {
      case SBMM_F64: hipLaunchKernelGGL(batch_norms_kernel<double>, grid, block, 0, s, na, wg_off, count); break;
      case SBMM_F32: hipLaunchKernelGGL(batch_norms_kernel<float>, grid, block, 0, s, na, wg_off, count); break;
      case SBMM_BF16: hipLaunchKernelGGL(batch_norms_kernel<uint16_t>, grid, block, 0, s, na, wg_off, count); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (total_blk > 0)
    hipLaunchKernelGGL(batch_stats_kernel, dim3((unsigned)total_blk), dim3(kThreads), 0, s,
                       reinterpret_cast<const StatsArgs*>(stats_args), blk_off, count);
  return hipGetLastError();
}
