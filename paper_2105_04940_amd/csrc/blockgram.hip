// Per-block product norms ||M^k N_k||_F^2 without forming M^k N_k.
//
// The rules (1.2) and (3.9) need ||M^k N_k||_F, which the paper computes
// from the m x p block product (2 m n_k p flops per block). The same number
// is the Frobenius inner product of the two n_k x n_k Gram matrices,
//     ||M^k N_k||_F^2 = trace(N_k^T M^k^T M^k N_k) = < M^k^T M^k , N_k N_k^T >_F,
// which costs 2 n_k^2 (m + p) flops and reads M^k and N_k once. For blocks
// much narrower than m and p (the block-sampling workloads) this is far
// cheaper, so the exact product can run without per-block bookkeeping.
//
// One workgroup per block (n_k <= 128). Both Gram matrices are accumulated
// on matrix cores (v_mfma_f32_32x32x2_f32) into a 128 x 128 tile split in
// 64 x 64 quadrants over the four waves; since both are symmetric only the
// quadrants (0,0), (0,1), (1,1) are formed and (0,1) counts twice. The
// contraction runs over the rows of M^k (stored as loaded: step k = row h,
// index i = column) and over the columns of N_k (stored transposed), so both
// operands of every step come from the same LDS tile layout [k][i]. The
// inner product and its reduction are float64 in a fixed order.
#include "common.h"

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;
constexpr int kT = 128;         // Gram tile (max block width)
constexpr int kBK = 32;         // contraction step
constexpr int kS = kT + 4;      // LDS row stride

struct GramArgs {
  const float* M; int64_t ldm;
  const float* N; int64_t ldn;
  int64_t m, p;
  const int64_t* off;
  double* out;     // [K]
};

__global__ __launch_bounds__(kThreads) void block_gram_kernel(GramArgs a) {
  __shared__ float Xs[2][kBK][kS];
  __shared__ double red[4];
  const int k = blockIdx.x;
  const int64_t lo = a.off[k];
  const int nk = (int)(a.off[k + 1] - lo);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 31, lh = lane >> 5;
  const int wave_m0 = (wave & 1) * 64, wave_n0 = (wave >> 1) * 64;
  // quadrant (1,0) mirrors (0,1); quadrants outside the block are all zero
  const bool active = wave != 1 && wave_m0 < nk && wave_n0 < nk;

  f32x16 acc[2][2], gm[2][2];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c) { acc[b][c] = f32x16{}; gm[b][c] = f32x16{}; }

  // phase 0: rows of M^k (step = row h, index i = column lo + i)
  // phase 1: columns of N_k (step = column f, index i = row lo + i)
  float r[kBK * kT / kThreads];
  for (int phase = 0; phase < 2; ++phase) {
    const int64_t ext = phase == 0 ? a.m : a.p;
    const int64_t nsteps = (ext + kBK - 1) / kBK;
    auto load = [&](int64_t st) {
      const int64_t s0 = st * kBK;
      if (phase == 0) {
        // 2 rows per pass, 128 consecutive columns per row
#pragma unroll
        for (int q = 0; q < kBK * kT / kThreads; ++q) {
          const int row = q * 2 + (tid >> 7), i = tid & 127;
          const int64_t h = s0 + row;
          r[q] = (h < a.m && i < nk) ? a.M[h * a.ldm + lo + i] : 0.0f;
        }
      } else {
        // 8 rows of N_k per pass, 32 consecutive columns per row
#pragma unroll
        for (int q = 0; q < kBK * kT / kThreads; ++q) {
          const int i = q * 8 + (tid >> 5), f = tid & 31;
          const int64_t col = s0 + f;
          r[q] = (col < a.p && i < nk) ? a.N[(lo + i) * a.ldn + col] : 0.0f;
        }
      }
    };
    auto store = [&](int buf) {
      if (phase == 0) {
#pragma unroll
        for (int q = 0; q < kBK * kT / kThreads; ++q) Xs[buf][q * 2 + (tid >> 7)][tid & 127] = r[q];
      } else {
#pragma unroll
        for (int q = 0; q < kBK * kT / kThreads; ++q) Xs[buf][tid & 31][q * 8 + (tid >> 5)] = r[q];
      }
    };
    __syncthreads();
    if (nsteps > 0) {
      load(0);
      store(0);
    }
    __syncthreads();
    for (int64_t st = 0; st < nsteps; ++st) {
      const int cur = (int)(st & 1);
      if (st + 1 < nsteps) load(st + 1);
      if (active) {
#pragma unroll
        for (int s = 0; s < kBK / 2; ++s) {
          const int kk = 2 * s + lh;
          const f32x2 av = *reinterpret_cast<const f32x2*>(&Xs[cur][kk][wave_m0 + 2 * lr]);
          const f32x2 bv = *reinterpret_cast<const f32x2*>(&Xs[cur][kk][wave_n0 + 2 * lr]);
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c)
              acc[b][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[b], bv[c], acc[b][c], 0, 0, 0);
        }
      }
      if (st + 1 < nsteps) store(cur ^ 1);
      __syncthreads();
    }
    if (phase == 0) {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) { gm[b][c] = acc[b][c]; acc[b][c] = f32x16{}; }
    }
  }
  // < G_M, G_N > over this wave's quadrant (same lane layout for both)
  double dot = 0.0;
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 16; ++v) dot = fma((double)gm[b][c][v], (double)acc[b][c][v], dot);
  if (wave == 2) dot *= 2.0;
  if (!active) dot = 0.0;
  dot = warp_sum_f64(dot);
  if (lane == 0) red[wave] = dot;
  __syncthreads();
  if (tid == 0) a.out[k] = ((red[0] + red[1]) + red[2]) + red[3];
}

}  // namespace

hipError_t launch_block_gram(const float* M, int64_t ldm, const float* N, int64_t ldn, int64_t m, int64_t p,
                             const int64_t* off_dev, int32_t K, double* out, hipStream_t s) {
  GramArgs a{M, ldm, N, ldn, m, p, off_dev, out};
  hipLaunchKernelGGL(block_gram_kernel, dim3((unsigned)K), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

int64_t block_gram_max_width() { return kT; }
