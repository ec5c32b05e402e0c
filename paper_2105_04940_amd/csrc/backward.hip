// Gradient of the sketched product with the draws held fixed.
//
// CD = C D with C[:, l] = scale_l M[:, colmap[l]] and D[l, :] = scale_l
// N[colmap[l], :] (eq. 3.3), so for an upstream gradient G = dL/d(CD):
//     dC = G D^T,   dD = C^T G,
//     dM[:, i] = sum over sketch columns l with colmap[l] = i of scale_l dC[:, l],
//     dN[i, :] = sum over the same l of scale_l dD[l, :],
// and every column of M (row of N) that no draw touched gets zero. The two
// products run on the matrix-core kernels; the sums run here, per inner
// index, over the draws of its atom in draw order (no atomics, bitwise
// reproducible).
//
// The per-atom draw lists are a counting sort of the draws by atom that keeps
// draw order within an atom.
#include <algorithm>

#include "common.h"

namespace {

constexpr int kThreads = 256;

// One workgroup: per-atom counts and offsets, and the draws of each atom in
// ascending draw order. The ranks come from one thread walking the draws in
// order (chunks of the draw list staged in LDS), or for at most kParRank
// draws from every thread counting the equal draws before its own; with up
// to kLdsAtoms atoms the counts live in LDS.
constexpr int kLdsAtoms = 8192, kIdxChunk = 2048, kParRank = 512;

__global__ __launch_bounds__(kThreads) void draw_lists_kernel(const int32_t* __restrict__ idx, int64_t c,
                                                              int64_t A, int32_t* __restrict__ cnt,
                                                              int32_t* __restrict__ rank,
                                                              int64_t* __restrict__ aoff,
                                                              int32_t* __restrict__ list) {
  __shared__ int64_t sm[kThreads];
  __shared__ int32_t scnt[kLdsAtoms];
  __shared__ int32_t sidx[kIdxChunk];
  const bool lds = A <= kLdsAtoms;
  int32_t* cn = lds ? scnt : cnt;
  for (int64_t a = threadIdx.x; a < A; a += kThreads) cn[a] = 0;
  for (int64_t c0 = 0; c0 < c; c0 += kIdxChunk) {
    const int64_t nc = min((int64_t)kIdxChunk, c - c0);
    __syncthreads();
    for (int64_t t = threadIdx.x; t < nc; t += kThreads) sidx[t] = idx[c0 + t];
    __syncthreads();
    if (c <= kParRank) {
      // few draws: each thread ranks its draws by counting the equal earlier
      // ones (broadcast LDS reads), and the counts come from LDS atomics
      for (int64_t t = threadIdx.x; t < nc; t += kThreads) {
        const int32_t a = sidx[t];
        int32_t r = 0;
        for (int64_t u = 0; u < t; ++u) r += sidx[u] == a;
        rank[t] = a >= 0 ? r : -1;
        if (a >= 0) atomicAdd(&cn[a], 1);
      }
    } else if (threadIdx.x == 0) {
      for (int64_t t = 0; t < nc; ++t) {
        const int32_t a = sidx[t];
        rank[c0 + t] = a >= 0 ? cn[a]++ : -1;
      }
    }
  }
  __syncthreads();
  // exclusive scan of the counts (each thread owns a contiguous run)
  const int64_t per = (A + kThreads - 1) / kThreads;
  const int64_t b0 = (int64_t)threadIdx.x * per, b1 = min(A, b0 + per);
  int64_t local = 0;
  for (int64_t a = b0; a < b1; ++a) local += cn[a];
  sm[threadIdx.x] = local;
  __syncthreads();
  for (int o = 1; o < kThreads; o <<= 1) {
    const int64_t add = (int)threadIdx.x >= o ? sm[threadIdx.x - o] : 0;
    __syncthreads();
    sm[threadIdx.x] += add;
    __syncthreads();
  }
  int64_t run = sm[threadIdx.x] - local;
  for (int64_t a = b0; a < b1; ++a) {
    aoff[a] = run;
    run += cn[a];
    if (lds) cnt[a] = cn[a];
  }
  if (threadIdx.x == kThreads - 1) aoff[A] = sm[kThreads - 1];
  __syncthreads();
  for (int64_t t = threadIdx.x; t < c; t += kThreads)
    if (rank[t] >= 0) list[aoff[idx[t]] + rank[t]] = (int32_t)t;
}

struct ScatterArgs {
  int mode;
  const int64_t* off;      // block offsets (block mode: atom -> columns)
  int32_t K;
  const int64_t* aoff; const int32_t* list;
  const double* scale; const int64_t* col_off;
  int64_t m, n, p;
  int64_t L;               // columns of dC / rows of dD
  int32_t* status;
};

__device__ __forceinline__ void atom_of(const ScatterArgs& a, int64_t i, int64_t& atom, int64_t& j) {
  if (a.mode == SBMM_MODE_BLOCK) {
    int64_t lo = 0, hi = a.K;            // last block with off[k] <= i
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (a.off[mid] <= i) lo = mid; else hi = mid;
    }
    atom = lo;
    j = i - a.off[lo];
  } else {
    atom = i;
    j = 0;
  }
}

template <typename T> __device__ __forceinline__ void put(T* p, int64_t i, double v);
template <> __device__ __forceinline__ void put<double>(double* p, int64_t i, double v) { p[i] = v; }
template <> __device__ __forceinline__ void put<float>(float* p, int64_t i, double v) { p[i] = (float)v; }
template <> __device__ __forceinline__ void put<uint16_t>(uint16_t* p, int64_t i, double v) {
  p[i] = float_to_bf16_bits((float)v);
}

// dM[h, i] for a 256-column x 16-row block; dC is m x ldc (float or double)
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kThreads) void scatter_cols_kernel(ScatterArgs a, const Tin* __restrict__ dC,
                                                                int64_t lddc, Tout* __restrict__ dM,
                                                                int64_t lddm, int64_t ctiles) {
  const int64_t i = (blockIdx.x % ctiles) * kThreads + threadIdx.x;
  const int64_t h0 = (blockIdx.x / ctiles) * 16;
  if (i >= a.n) return;
  int64_t atom, j;
  atom_of(a, i, atom, j);
  const int64_t q0 = a.aoff[atom], q1 = a.aoff[atom + 1];
  const int64_t h1 = min(a.m, h0 + 16);
  for (int64_t h = h0; h < h1; ++h) {
    double s = 0.0;
    for (int64_t q = q0; q < q1; ++q) {
      const int32_t t = a.list[q];
      const int64_t l = a.col_off[t] + j;
      if (l >= a.L) { *a.status = SBMM_DEV_USER_CK; continue; }   // L below the sketch width
      s += a.scale[t] * (double)dC[h * lddc + l];
    }
    put<Tout>(dM, h * lddm + i, s);
  }
}

// dN[i, f]: one wave per inner index, lanes across f; dD is L x lddd
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kThreads) void scatter_rows_kernel(ScatterArgs a, const Tin* __restrict__ dD,
                                                                int64_t lddd, Tout* __restrict__ dN,
                                                                int64_t lddn) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= a.n) return;
  int64_t atom, j;
  atom_of(a, i, atom, j);
  const int64_t q0 = a.aoff[atom], q1 = a.aoff[atom + 1];
  for (int64_t f = lane; f < a.p; f += 64) {
    double s = 0.0;
    for (int64_t q = q0; q < q1; ++q) {
      const int32_t t = a.list[q];
      const int64_t l = a.col_off[t] + j;
      if (l >= a.L) { *a.status = SBMM_DEV_USER_CK; continue; }
      s += a.scale[t] * (double)dD[l * lddd + f];
    }
    put<Tout>(dN, i * lddn + f, s);
  }
}

// C[i][j] = sum_k A(i, k) B(k, j) with arbitrary element strides, 16 x 16
// output tile per workgroup, float64 accumulation (small problems).
template <typename T>
__global__ __launch_bounds__(kThreads) void gemm_strided_kernel(const T* __restrict__ A, int64_t ars, int64_t aks,
                                                                const T* __restrict__ B, int64_t bks, int64_t bjs,
                                                                T* __restrict__ C, int64_t ldc, int64_t M,
                                                                int64_t Nc, int64_t K, int64_t tiles_m) {
  __shared__ T As[16][17], Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t i = (blockIdx.x % tiles_m) * 16 + ty;
  const int64_t j = (blockIdx.x / tiles_m) * 16 + tx;
  double acc = 0.0;
  for (int64_t k0 = 0; k0 < K; k0 += 16) {
    As[ty][tx] = (i < M && k0 + tx < K) ? A[i * ars + (k0 + tx) * aks] : T(0);
    Bs[ty][tx] = (k0 + ty < K && j < Nc) ? B[(k0 + ty) * bks + j * bjs] : T(0);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) acc += (double)As[ty][kk] * (double)Bs[kk][tx];
    __syncthreads();
  }
  if (i < M && j < Nc) C[i * ldc + j] = (T)acc;
}

__global__ void bf16_to_f32_kernel(const uint16_t* __restrict__ x, int64_t rows, int64_t cols, int64_t ldx,
                                   float* __restrict__ y, int64_t ldy) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / cols, c = e % cols;
    y[r * ldy + c] = __uint_as_float((uint32_t)x[r * ldx + c] << 16);
  }
}

__global__ void to_bf16_kernel(const float* __restrict__ x, int64_t rows, int64_t cols, int64_t ldx,
                               uint16_t* __restrict__ y) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / cols, c = e % cols;
    y[e] = float_to_bf16_bits(x[r * ldx + c]);
  }
}

// y (cols x rows, leading dimension ldy) = bf16 of x^T (x rows x cols,
// float32 or bf16, leading dimension ldx), through 64 x 64 LDS tiles: reads
// and writes are both along contiguous rows. With rows_dev, only the first
// round_up(*rows_dev, 32) rows of x are transposed (the rest of the grid
// exits).
template <typename Tin>
__global__ __launch_bounds__(256) void transpose_bf16_kernel(const Tin* __restrict__ x, int64_t rows, int64_t cols,
                                                             int64_t ldx, const int64_t* __restrict__ rows_dev,
                                                             uint16_t* __restrict__ y, int64_t ldy) {
  __shared__ uint16_t t[64][66];
  const int64_t tiles_c = (cols + 63) / 64;
  const int64_t r0 = (int64_t)(blockIdx.x / tiles_c) * 64, c0 = (int64_t)(blockIdx.x % tiles_c) * 64;
  int64_t nrows = rows;
  if (rows_dev) nrows = min(rows, (*rows_dev + SBMM_SKETCH_PAD - 1) / SBMM_SKETCH_PAD * SBMM_SKETCH_PAD);
  if (r0 >= nrows) return;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int64_t r = r0 + i, c = c0 + tx;
    uint16_t v = 0;
    if (r < nrows && c < cols) {
      if constexpr (sizeof(Tin) == 4) v = float_to_bf16_bits(x[r * ldx + c]);
      else v = x[r * ldx + c];
    }
    t[i][tx] = v;
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < cols && r < nrows) y[c * ldy + r] = t[tx][i];
  }
}

// ---------------------------------------------------------------------------
// bf16 backward with the draws merged per atom. Every draw t of atom a feeds
// the same columns of M and rows of N, so the gradient of the estimator
// sum_t scale_t^2 M^{a_t} N_{a_t} is w_a G N_a^T for the columns of atom a
// and w_a M^{aT} G for its rows, w_a = sum of scale_t^2 over a's draws: the
// drawn atoms are compacted once (each drawn inner index is one column of the
// compact operands), the two products run over the compact width L_U <= L,
// and their epilogues write w_a times the product straight into dM / dN.
// ---------------------------------------------------------------------------

// One workgroup: per atom the compact offset (-1 if undrawn) and w_a summed
// over its draws in draw order; the compact width, at most cap, goes to *lu.
__global__ __launch_bounds__(1024) void dedup_atoms_kernel(int mode, const int64_t* __restrict__ off, int64_t A,
                                                           const int32_t* __restrict__ cnt,
                                                           const int64_t* __restrict__ aoff,
                                                           const int32_t* __restrict__ list,
                                                           const double* __restrict__ scale,
                                                           int64_t* __restrict__ uoff, double* __restrict__ wsum,
                                                           int64_t cap, int64_t* __restrict__ lu,
                                                           int32_t* __restrict__ status) {
  __shared__ int64_t sm[1024];
  const int nt = blockDim.x;
  const int64_t per = (A + nt - 1) / nt;
  const int64_t b0 = (int64_t)threadIdx.x * per, b1 = min(A, b0 + per);
  auto width = [&](int64_t a) { return mode == SBMM_MODE_BLOCK ? off[a + 1] - off[a] : (int64_t)1; };
  int64_t local = 0;
  for (int64_t a = b0; a < b1; ++a)
    if (cnt[a] > 0) local += width(a);
  sm[threadIdx.x] = local;
  __syncthreads();
  for (int o = 1; o < nt; o <<= 1) {
    const int64_t add = (int)threadIdx.x >= o ? sm[threadIdx.x - o] : 0;
    __syncthreads();
    sm[threadIdx.x] += add;
    __syncthreads();
  }
  int64_t run = sm[threadIdx.x] - local;
  for (int64_t a = b0; a < b1; ++a) {
    if (cnt[a] > 0) {
      double w = 0.0;
      for (int64_t q = aoff[a]; q < aoff[a + 1]; ++q) {
        const double sc = scale[list[q]];
        w += sc * sc;
      }
      uoff[a] = run;
      wsum[a] = w;
      run += width(a);
    } else {
      uoff[a] = -1;
      wsum[a] = 0.0;
    }
  }
  if (threadIdx.x == nt - 1) {
    // the compact width cannot pass the sketch width the caller sized for;
    // a smaller L than the plan's is an argument error
    *lu = min(sm[nt - 1], cap);
    if (sm[nt - 1] > cap) *status = SBMM_DEV_USER_CK;
  }
}

// One thread per inner index: its compact column (map and weight) if its
// atom was drawn, and the drawn flag every index gets.
__global__ __launch_bounds__(kThreads) void dedup_cols_kernel(int mode, const int64_t* __restrict__ off, int32_t K,
                                                              int64_t n, const int64_t* __restrict__ uoff,
                                                              const double* __restrict__ wsum,
                                                              int32_t* __restrict__ ucol, double* __restrict__ uw,
                                                              uint8_t* __restrict__ drawn, int64_t cap) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  int64_t atom = i, lo = i;
  if (mode == SBMM_MODE_BLOCK) {
    int64_t a = 0, b = K;            // last block with off[k] <= i
    while (b - a > 1) {
      const int64_t mid = (a + b) >> 1;
      if (off[mid] <= i) a = mid; else b = mid;
    }
    atom = a;
    lo = off[a];
  }
  const int64_t u = uoff[atom];
  drawn[i] = u >= 0;
  if (u >= 0 && u + (i - lo) < cap) {
    ucol[u + (i - lo)] = (int32_t)i;
    uw[u + (i - lo)] = wsum[atom];
  }
}

template <typename T> __device__ __forceinline__ uint16_t to_bf16(T x);
template <> __device__ __forceinline__ uint16_t to_bf16<uint16_t>(uint16_t x) { return x; }
template <> __device__ __forceinline__ uint16_t to_bf16<float>(float x) { return float_to_bf16_bits(x); }

// NU[j, :] = bf16(N[ucol[j], :]) for the live compact rows j < *lu, zero in
// the columns p .. ld - 1: one wave per row, 8 elements per lane and step
// (16-byte loads and stores where the source row allows: vec).
template <typename T>
__device__ __forceinline__ uint4 load8_bf16(const T* src, int64_t f, int64_t p, bool vec) {
  uint16_t e[8];
  if (vec && f + 8 <= p) {
    if constexpr (sizeof(T) == 2) return *reinterpret_cast<const uint4*>(src + f);
    const float4 x0 = *reinterpret_cast<const float4*>(src + f);
    const float4 x1 = *reinterpret_cast<const float4*>(src + f + 4);
    e[0] = to_bf16<float>(x0.x); e[1] = to_bf16<float>(x0.y); e[2] = to_bf16<float>(x0.z); e[3] = to_bf16<float>(x0.w);
    e[4] = to_bf16<float>(x1.x); e[5] = to_bf16<float>(x1.y); e[6] = to_bf16<float>(x1.z); e[7] = to_bf16<float>(x1.w);
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) e[q] = f + q < p ? to_bf16<T>(src[f + q]) : (uint16_t)0;
  }
  return make_uint4(e[0] | (uint32_t)e[1] << 16, e[2] | (uint32_t)e[3] << 16, e[4] | (uint32_t)e[5] << 16,
                    e[6] | (uint32_t)e[7] << 16);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void gather_rows_bf16_kernel(const T* __restrict__ N, int64_t ldn, int64_t p,
                                                                    const int32_t* __restrict__ ucol,
                                                                    const int64_t* __restrict__ lu, int64_t L_max,
                                                                    uint16_t* __restrict__ out, int64_t ld, int vec) {
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= min(*lu, L_max)) return;
  const T* src = N + (int64_t)ucol[j] * ldn;
  uint16_t* dst = out + j * ld;
  for (int64_t f = 8 * (int64_t)lane; f < ld; f += 512)
    *reinterpret_cast<uint4*>(dst + f) = load8_bf16<T>(src, f, p, vec != 0);
}

// MUt[j, h] = bf16(M[h, ucol[j]]) for j < *lu, zero for m <= h < ld:
// 64 x 64 tiles through LDS. A thread reads 8 consecutive compact columns of
// a row (one 16-byte load when they are 8 consecutive, aligned columns of M:
// runs inside an atom) and writes 8 consecutive h of an output row.
template <typename T>
__global__ __launch_bounds__(kThreads) void gather_cols_t_bf16_kernel(const T* __restrict__ M, int64_t ldm, int64_t m,
                                                                      const int32_t* __restrict__ ucol,
                                                                      const int64_t* __restrict__ lu, int64_t L_max,
                                                                      int64_t h_tiles, uint16_t* __restrict__ out,
                                                                      int64_t ld, int vec) {
  __shared__ uint16_t t[64][72];
  const int64_t j0 = (int64_t)(blockIdx.x / h_tiles) * 64, h0 = (int64_t)(blockIdx.x % h_tiles) * 64;
  const int64_t L = min(*lu, L_max);
  if (j0 >= L) return;
  const int tid = threadIdx.x;
  const int jg = 8 * (tid & 7);
  int64_t col[8];
  bool run = vec != 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    col[q] = j0 + jg + q < L ? (int64_t)ucol[j0 + jg + q] : -1;
    run = run && col[q] == col[0] + q;
  }
  run = run && col[0] >= 0 && col[0] % 8 == 0;
  for (int pass = 0; pass < 2; ++pass) {
    const int i = (tid >> 3) + 32 * pass;
    const int64_t h = h0 + i;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (h < m) {
      const T* row = M + h * ldm;
      if (run) {
        v = load8_bf16<T>(row, col[0], col[0] + 8, true);
      } else {
        uint16_t e[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) e[q] = col[q] >= 0 ? to_bf16<T>(row[col[q]]) : (uint16_t)0;
        v = make_uint4(e[0] | (uint32_t)e[1] << 16, e[2] | (uint32_t)e[3] << 16, e[4] | (uint32_t)e[5] << 16,
                       e[6] | (uint32_t)e[7] << 16);
      }
    }
    *reinterpret_cast<uint4*>(&t[i][jg]) = v;
  }
  __syncthreads();
  const int hg = 8 * (tid & 7);
  for (int pass = 0; pass < 2; ++pass) {
    const int jj = (tid >> 3) + 32 * pass;
    const int64_t j = j0 + jj, h = h0 + hg;
    if (j >= L || h >= ld) continue;
    uint16_t e[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) e[q] = t[hg + q][jj];
    *reinterpret_cast<uint4*>(out + j * ld + h) =
        make_uint4(e[0] | (uint32_t)e[1] << 16, e[2] | (uint32_t)e[3] << 16, e[4] | (uint32_t)e[5] << 16,
                   e[6] | (uint32_t)e[7] << 16);
  }
}

// G16 (m x ldp, bf16 of G, zero in columns p .. ldp - 1) and G16t (p x ldm,
// bf16 of G^T, zero in columns m .. ldm - 1) from one read of G (m x p
// float32), 64 x 64 tiles through LDS; a thread converts 8 consecutive
// elements of a row (two 16-byte loads where aligned: vec) and writes 8
// consecutive elements of a G16t row.
__global__ __launch_bounds__(kThreads) void g_prep_kernel(const float* __restrict__ G, int64_t ldg, int64_t m,
                                                          int64_t p, int64_t c_tiles, uint16_t* __restrict__ G16,
                                                          int64_t ldp, uint16_t* __restrict__ G16t, int64_t ldm,
                                                          int vec) {
  __shared__ uint16_t t[64][72];
  const int64_t r0 = (int64_t)(blockIdx.x / c_tiles) * 64, c0 = (int64_t)(blockIdx.x % c_tiles) * 64;
  const int tid = threadIdx.x;
  const int cg = 8 * (tid & 7);
  for (int pass = 0; pass < 2; ++pass) {
    const int i = (tid >> 3) + 32 * pass;
    const int64_t r = r0 + i, c = c0 + cg;
    const uint4 v = r < m ? load8_bf16<float>(G + r * ldg, c, p, vec != 0) : make_uint4(0, 0, 0, 0);
    *reinterpret_cast<uint4*>(&t[i][cg]) = v;
    if (r < m && c < ldp) *reinterpret_cast<uint4*>(G16 + r * ldp + c) = v;
  }
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    const int cc = (tid >> 3) + 32 * pass;
    const int64_t c = c0 + cc, r = r0 + cg;
    if (c >= p || r >= ldm) continue;
    uint16_t e[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) e[q] = t[cg + q][cc];
    *reinterpret_cast<uint4*>(G16t + c * ldm + r) =
        make_uint4(e[0] | (uint32_t)e[1] << 16, e[2] | (uint32_t)e[3] << 16, e[4] | (uint32_t)e[5] << 16,
                   e[6] | (uint32_t)e[7] << 16);
  }
}

// Zero the columns of dM (m x n, ld) whose inner index was not drawn: one
// thread per 8-column chunk and rows h0 .. h0 + R - 1; whole undrawn chunks
// as 16-byte stores when rows are 16-byte aligned (vec).
template <typename T>
__global__ __launch_bounds__(kThreads) void zero_undrawn_cols_kernel(T* __restrict__ dM, int64_t ld, int64_t m,
                                                                     int64_t n, const uint8_t* __restrict__ drawn,
                                                                     int64_t chunk_blocks, int rows_per, int vec) {
  const int64_t e = (int64_t)(blockIdx.x % chunk_blocks) * kThreads + threadIdx.x;
  const int64_t h0 = (int64_t)(blockIdx.x / chunk_blocks) * rows_per;
  const int64_t c0 = 8 * e;
  if (c0 >= n) return;
  uint32_t mask = 0;   // bit q: column c0 + q must be zeroed
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (c0 + q < n && !drawn[c0 + q]) mask |= 1u << q;
  if (!mask) return;
  const int64_t h1 = min(m, h0 + rows_per);
  const bool whole = vec && mask == 0xffu;
  for (int64_t h = h0; h < h1; ++h) {
    T* row = dM + h * ld + c0;
    if (whole) {
      uint4* v = reinterpret_cast<uint4*>(row);
#pragma unroll
      for (int q = 0; q < (int)(8 * sizeof(T) / 16); ++q) v[q] = make_uint4(0, 0, 0, 0);
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (mask >> q & 1u) row[q] = T(0);
    }
  }
}

// Zero the rows of dN (n x p, ld) whose inner index was not drawn: one wave
// per row, 16-byte stores when rows are 16-byte aligned (vec).
template <typename T>
__global__ __launch_bounds__(kThreads) void zero_undrawn_rows_kernel(T* __restrict__ dN, int64_t ld, int64_t n,
                                                                     int64_t p, const uint8_t* __restrict__ drawn,
                                                                     int vec) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n || drawn[i]) return;
  T* row = dN + i * ld;
  constexpr int E = 16 / sizeof(T);   // elements per 16-byte store
  int64_t f = 0;
  if (vec) {
    for (f = (int64_t)E * lane; f + E <= p; f += (int64_t)E * 64)
      *reinterpret_cast<uint4*>(row + f) = make_uint4(0, 0, 0, 0);
    f = p / E * E;
  }
  for (int64_t q = f + lane; q < p; q += 64) row[q] = T(0);
}

}  // namespace

hipError_t launch_transpose_bf16(sbmm_dtype src_dt, const void* x, int64_t rows, int64_t cols, int64_t ldx,
                                 const int64_t* rows_dev, uint16_t* y, int64_t ldy, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const dim3 grid((unsigned)(ceil_div(rows, 64) * ceil_div(cols, 64)));
  if (src_dt == SBMM_F32)
    hipLaunchKernelGGL(transpose_bf16_kernel<float>, grid, dim3(256), 0, s, reinterpret_cast<const float*>(x), rows,
                       cols, ldx, rows_dev, y, ldy);
  else if (src_dt == SBMM_BF16)
    hipLaunchKernelGGL(transpose_bf16_kernel<uint16_t>, grid, dim3(256), 0, s, reinterpret_cast<const uint16_t*>(x),
                       rows, cols, ldx, rows_dev, y, ldy);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float* x, int64_t rows, int64_t cols, int64_t ldx, uint16_t* y,
                          hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const int64_t nb = std::min<int64_t>(ceil_div(rows * cols, 256), 8192);
  hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)nb), dim3(256), 0, s, x, rows, cols, ldx, y);
  return hipGetLastError();
}

hipError_t launch_bf16_to_f32(const uint16_t* x, int64_t rows, int64_t cols, int64_t ldx, float* y, int64_t ldy,
                              hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const int64_t nb = std::min<int64_t>(ceil_div(rows * cols, 256), 16384);
  hipLaunchKernelGGL(bf16_to_f32_kernel, dim3((unsigned)nb), dim3(256), 0, s, x, rows, cols, ldx, y, ldy);
  return hipGetLastError();
}

hipError_t launch_draw_lists(const int32_t* idx, int64_t c, int64_t A, int32_t* cnt, int32_t* rank,
                             int64_t* aoff, int32_t* list, hipStream_t s) {
  hipLaunchKernelGGL(draw_lists_kernel, dim3(1), dim3(kThreads), 0, s, idx, c, A, cnt, rank, aoff, list);
  return hipGetLastError();
}

hipError_t launch_scatter(const BackwardScatter& b, hipStream_t s) {
  ScatterArgs a{};
  a.mode = b.mode; a.off = b.off_dev; a.K = b.K; a.aoff = b.aoff; a.list = b.list;
  a.scale = b.scale; a.col_off = b.col_off; a.m = b.m; a.n = b.n; a.p = b.p;
  a.L = b.L; a.status = b.status;
  const int64_t ctiles = ceil_div(b.n, kThreads);
  const dim3 gc((unsigned)(ctiles * ceil_div(std::max<int64_t>(b.m, 1), 16)));
  const dim3 gr((unsigned)ceil_div(b.n, 4));
  if (b.m > 0 && b.dM) {
    if (b.grad_dt == SBMM_F64) {
      hipLaunchKernelGGL((scatter_cols_kernel<double, double>), gc, dim3(kThreads), 0, s, a,
                         (const double*)b.dC, b.lddc, (double*)b.dM, b.lddm, ctiles);
    } else if (b.out_dt == SBMM_F32) {
      hipLaunchKernelGGL((scatter_cols_kernel<float, float>), gc, dim3(kThreads), 0, s, a,
                         (const float*)b.dC, b.lddc, (float*)b.dM, b.lddm, ctiles);
    } else {
      hipLaunchKernelGGL((scatter_cols_kernel<float, uint16_t>), gc, dim3(kThreads), 0, s, a,
                         (const float*)b.dC, b.lddc, (uint16_t*)b.dM, b.lddm, ctiles);
    }
  }
  if (b.p > 0 && b.dN) {
    if (b.grad_dt == SBMM_F64) {
      hipLaunchKernelGGL((scatter_rows_kernel<double, double>), gr, dim3(kThreads), 0, s, a,
                         (const double*)b.dD, b.lddd, (double*)b.dN, b.lddn);
    } else if (b.out_dt == SBMM_F32) {
      hipLaunchKernelGGL((scatter_rows_kernel<float, float>), gr, dim3(kThreads), 0, s, a,
                         (const float*)b.dD, b.lddd, (float*)b.dN, b.lddn);
    } else {
      hipLaunchKernelGGL((scatter_rows_kernel<float, uint16_t>), gr, dim3(kThreads), 0, s, a,
                         (const float*)b.dD, b.lddd, (uint16_t*)b.dN, b.lddn);
    }
  }
  return hipGetLastError();
}

hipError_t launch_gemm_strided(sbmm_dtype dt, const void* A, int64_t ars, int64_t aks, const void* B,
                               int64_t bks, int64_t bjs, void* C, int64_t ldc, int64_t M, int64_t Nc,
                               int64_t K, hipStream_t s) {
  if (M <= 0 || Nc <= 0) return hipSuccess;
  const int64_t tm = ceil_div(M, 16), tn = ceil_div(Nc, 16);
  const dim3 grid((unsigned)(tm * tn));
  if (dt == SBMM_F64)
    hipLaunchKernelGGL(gemm_strided_kernel<double>, grid, dim3(kThreads), 0, s, (const double*)A, ars, aks,
                       (const double*)B, bks, bjs, (double*)C, ldc, M, Nc, K, tm);
  else if (dt == SBMM_F32)
    hipLaunchKernelGGL(gemm_strided_kernel<float>, grid, dim3(kThreads), 0, s, (const float*)A, ars, aks,
                       (const float*)B, bks, bjs, (float*)C, ldc, M, Nc, K, tm);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_dedup(const BackwardDedup& d, hipStream_t s) {
  hipLaunchKernelGGL(dedup_atoms_kernel, dim3(1), dim3(1024), 0, s, d.mode, d.off_dev, d.A, d.cnt, d.aoff, d.list,
                     d.scale, d.uoff, d.wsum, d.cap, d.lu, d.status);
  hipLaunchKernelGGL(dedup_cols_kernel, dim3((unsigned)ceil_div(d.n, kThreads)), dim3(kThreads), 0, s, d.mode,
                     d.off_dev, d.K, d.n, d.uoff, d.wsum, d.ucol, d.uw, d.drawn, d.cap);
  return hipGetLastError();
}

hipError_t launch_gather_compact(sbmm_dtype in_dt, const void* N, int64_t ldn, int64_t p, const void* M, int64_t ldm,
                                 int64_t m, const int32_t* ucol, const int64_t* lu, int64_t L_max, uint16_t* NU,
                                 int64_t ldnu, uint16_t* MUt, int64_t ldmu, hipStream_t s) {
  if (L_max <= 0) return hipSuccess;
  const dim3 gr((unsigned)ceil_div(L_max, 4));
  const int64_t ht = ceil_div(ldmu, 64);
  const dim3 gc((unsigned)(ceil_div(L_max, 64) * ht));
  const int64_t es = in_dt == SBMM_BF16 ? 2 : 4;
  // 16-byte loads of 8 elements: rows of N / M start on 16-byte boundaries
  const int vn = (uintptr_t)N % 16 == 0 && (ldn * es) % 16 == 0;
  const int vm = (uintptr_t)M % 16 == 0 && (ldm * es) % 16 == 0;
  if (in_dt == SBMM_BF16) {
    hipLaunchKernelGGL(gather_rows_bf16_kernel<uint16_t>, gr, dim3(kThreads), 0, s, (const uint16_t*)N, ldn, p, ucol,
                       lu, L_max, NU, ldnu, vn);
    hipLaunchKernelGGL(gather_cols_t_bf16_kernel<uint16_t>, gc, dim3(kThreads), 0, s, (const uint16_t*)M, ldm, m,
                       ucol, lu, L_max, ht, MUt, ldmu, vm);
  } else if (in_dt == SBMM_F32) {
    hipLaunchKernelGGL(gather_rows_bf16_kernel<float>, gr, dim3(kThreads), 0, s, (const float*)N, ldn, p, ucol, lu,
                       L_max, NU, ldnu, vn);
    hipLaunchKernelGGL(gather_cols_t_bf16_kernel<float>, gc, dim3(kThreads), 0, s, (const float*)M, ldm, m, ucol,
                       lu, L_max, ht, MUt, ldmu, vm);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_g_prep(const float* G, int64_t ldg, int64_t m, int64_t p, uint16_t* G16, int64_t ldp,
                         uint16_t* G16t, int64_t ldm, hipStream_t s) {
  if (m <= 0 || p <= 0) return hipSuccess;
  // tiles cover the padded extents, so every padding element is written
  const int64_t ct = ceil_div(std::max(p, ldp), 64), rt = ceil_div(std::max(m, ldm), 64);
  const int vec = (uintptr_t)G % 16 == 0 && (ldg * 4) % 16 == 0;
  hipLaunchKernelGGL(g_prep_kernel, dim3((unsigned)(rt * ct)), dim3(kThreads), 0, s, G, ldg, m, p, ct, G16, ldp, G16t,
                     ldm, vec);
  return hipGetLastError();
}

hipError_t launch_zero_undrawn(sbmm_dtype out_dt, void* dM, int64_t lddm, int64_t m, void* dN, int64_t lddn,
                               int64_t p, int64_t n, const uint8_t* drawn, hipStream_t s) {
  const int64_t es = out_dt == SBMM_BF16 ? 2 : 4;
  if (m > 0 && dM) {
    const int vec = (uintptr_t)dM % 16 == 0 && (lddm * es) % 16 == 0;
    const int64_t cb = ceil_div(ceil_div(n, 8), kThreads);
    const int rows_per = 16;
    const dim3 g((unsigned)(cb * ceil_div(m, rows_per)));
    if (out_dt == SBMM_BF16)
      hipLaunchKernelGGL(zero_undrawn_cols_kernel<uint16_t>, g, dim3(kThreads), 0, s, (uint16_t*)dM, lddm, m, n,
                         drawn, cb, rows_per, vec);
    else
      hipLaunchKernelGGL(zero_undrawn_cols_kernel<float>, g, dim3(kThreads), 0, s, (float*)dM, lddm, m, n, drawn, cb,
                         rows_per, vec);
  }
  if (p > 0 && dN) {
    const int vec = (uintptr_t)dN % 16 == 0 && (lddn * es) % 16 == 0;
    const dim3 g((unsigned)ceil_div(n, 4));
    if (out_dt == SBMM_BF16)
      hipLaunchKernelGGL(zero_undrawn_rows_kernel<uint16_t>, g, dim3(kThreads), 0, s, (uint16_t*)dN, lddn, n, p, drawn,
                         vec);
    else
      hipLaunchKernelGGL(zero_undrawn_rows_kernel<float>, g, dim3(kThreads), 0, s, (float*)dN, lddn, n, p, drawn, vec);
  }
  return hipGetLastError();
}
