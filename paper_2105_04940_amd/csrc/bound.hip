// Probability error bounds of the stratified sampler, evaluated on the device
// from the data and the realized design: Thm 3.3 ((3.11)-(3.12), block sizes
// (3.9)), Thm 4.2 ((4.3)-(4.4), block sizes (4.2)) and Thm 4.4 ((4.8)-(4.9),
// block sizes (4.7) from the pilot), plus the exact expected squared error
// E ||MN - CD||_F^2 of the design that was actually sampled.
//
// Two launches. The atom pass splits every block into chunks of
// kChunk atoms (one workgroup each) and writes per chunk the sum of
// a_i^2 b_i^2 / p_hat_i and the smallest ratio p_hat_i / p_i of the sampled
// probabilities to (3.8) (the largest beta the theorems can use). The final
// pass (one workgroup) sums the chunks of every block in order, forms the
// per-block quantities v_k^2 = ||M^k N_k||_F^2 / s_k^2 (and the pilot's
// v^_k^2), reduces them to theta_1, theta_2 (theta^_1, theta^_2), and
// evaluates the bounds. Every sum runs in a fixed order, so the results are
// reproducible bit for bit.
#include <cmath>

#include "common.h"

namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 8;
constexpr int64_t kChunk = (int64_t)kThreads * kPerThread;

__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// op 0: sum, 1: min, 2: max over the workgroup (wave trees, then the four
// wave results in order); the result is returned to every thread.
template <int Op>
__device__ double block_reduce(double v, double* sm) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = Op == 0 ? warp_sum_f64(v) : (Op == 1 ? wave_min(v) : wave_max(v));
  __syncthreads();
  if (lane == 0) sm[wave] = v;
  __syncthreads();
  double r = sm[0];
  for (int w = 1; w < kThreads / 64; ++w)
    r = Op == 0 ? r + sm[w] : (Op == 1 ? fmin(r, sm[w]) : fmax(r, sm[w]));
  return r;
}

// the block holding chunk b: the largest k with chunk_off[k] <= b
__device__ int32_t chunk_block(const int64_t* chunk_off, int32_t K, int64_t b) {
  int32_t lo = 0, hi = K - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (chunk_off[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(kThreads) bound_atoms_kernel(BoundLaunch a) {
  __shared__ double sm[kThreads / 64];
  const int64_t b = blockIdx.x;
  const int32_t k = chunk_block(a.chunk_off, a.K, b);
  const int64_t lo = a.off[k] + (b - a.chunk_off[k]) * kChunk;
  const int64_t hi = min(lo + kChunk, a.off[k + 1]);
  const double s = a.blk[2 * a.K + k];
  double acc = 0.0, rmin = 1.0;
#pragma unroll 8
  for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
    const double x = a.col_sq[i] * a.row_sq[i];
    if (x > 0.0) {
      const double ph = a.p_hat[i];
      // a positive product drawn with probability 0 leaves the estimator
      // biased: its expected error is unbounded and no beta > 0 holds
      acc += ph > 0.0 ? x / ph : __builtin_inf();
      rmin = fmin(rmin, ph * s / sqrt(x));
    }
  }
  acc = block_reduce<0>(acc, sm);
  rmin = block_reduce<1>(rmin, sm);
  if (threadIdx.x == 0) {
    a.part[b] = acc;
    a.part[a.chunks + b] = rmin;
  }
}

__global__ void __launch_bounds__(kThreads) bound_final_kernel(BoundLaunch a) {
  __shared__ double sm[kThreads / 64];
  const int32_t K = a.K;
  double e = 0.0, bmin = 1.0, ms = 0.0, ns = 0.0;
  double t1 = __builtin_inf(), t2 = -__builtin_inf(), h1 = __builtin_inf(), h2 = -__builtin_inf();
  double live = 0.0;
  for (int32_t k = threadIdx.x; k < K; k += kThreads) {
    double sum = 0.0;
    for (int64_t b = a.chunk_off[k]; b < a.chunk_off[k + 1]; ++b) {
      sum += a.part[b];
      bmin = fmin(bmin, a.part[a.chunks + b]);
    }
    const double bp = a.blkprod_sq[k];
    const int64_t ck = a.ck[k];
    if (ck > 0) e += (sum - bp) / (double)ck;
    ms += a.blk[k];
    ns += a.blk[K + k];
    const double s = a.blk[2 * K + k];
    if (s > 0.0) {
      const double s2 = s * s;
      const double t = 1.0 - bp / s2;
      t1 = fmin(t1, t);
      t2 = fmax(t2, t);
      if (a.pilot_sq) {
        const double h = fabs(1.0 - a.pilot_sq[k] / s2);
        h1 = fmin(h1, h);
        h2 = fmax(h2, h);
      }
      live = 1.0;
    }
  }
  e = block_reduce<0>(e, sm);
  ms = block_reduce<0>(ms, sm);
  ns = block_reduce<0>(ns, sm);
  bmin = block_reduce<1>(bmin, sm);
  t1 = block_reduce<1>(t1, sm);
  t2 = block_reduce<2>(t2, sm);
  h1 = block_reduce<1>(h1, sm);
  h2 = block_reduce<2>(h2, sm);
  live = block_reduce<2>(live, sm);
  if (threadIdx.x != 0) return;
  double* o = a.out;
  const double beta = a.beta > 0.0 ? a.beta : bmin;
  const double mn = ms * ns;
  const double inf = __builtin_inf();
  if (live == 0.0) {
    // no block with s_k > 0: MN = 0, nothing is drawn and every bound is 0
    for (int j = 0; j < SBMM_BOUND_FIXED + 2 * a.n_delta; ++j) o[j] = 0.0;
    o[SBMM_BOUND_BETA] = beta;
    o[SBMM_BOUND_MN] = mn;
    return;
  }
  double phi, ratio;   // ratio: the factor (theta_2 / theta_1)^(1/2) of the tail term
  if (a.rule == SBMM_ALLOC_OPT) {
    phi = t1 > 0.0 ? sqrt(t2 - t1 * beta + t2 * t1 * beta) / sqrt(sqrt(t2 * t1)) : inf;
    ratio = t1 > 0.0 ? sqrt(t2 / t1) : inf;
  } else if (a.rule == SBMM_ALLOC_NORM) {
    phi = sqrt(1.0 - beta * (1.0 - t2));
    ratio = 1.0;
  } else {
    phi = h1 > 0.0 ? sqrt(h2 - h1 * beta + t2 * h1 * beta) / sqrt(sqrt(h2 * h1)) : inf;
    ratio = h1 > 0.0 ? sqrt(h2 / h1) : inf;
  }
  const double scale = mn / (beta * (double)a.c);
  o[SBMM_BOUND_THETA1] = t1;
  o[SBMM_BOUND_THETA2] = t2;
  o[SBMM_BOUND_THETA1_HAT] = a.pilot_sq ? h1 : 0.0;
  o[SBMM_BOUND_THETA2_HAT] = a.pilot_sq ? h2 : 0.0;
  o[SBMM_BOUND_BETA] = beta;
  o[SBMM_BOUND_MN] = mn;
  o[SBMM_BOUND_PHI] = phi;
  o[SBMM_BOUND_VAR] = phi * phi * scale;
  o[SBMM_BOUND_EXPECTED] = e;
  for (int j = 0; j < a.n_delta; ++j) {
    const double eta = phi + ratio * sqrt((8.0 / beta) * log(1.0 / a.delta[j]));
    o[SBMM_BOUND_FIXED + 2 * j] = eta;
    o[SBMM_BOUND_FIXED + 2 * j + 1] = eta * eta * scale;
  }
}

}  // namespace

int64_t bound_chunks(int64_t width) { return ceil_div(width, kChunk); }

hipError_t launch_bound(const BoundLaunch& a, hipStream_t s) {
  if (a.chunks > 0) {
    hipLaunchKernelGGL(bound_atoms_kernel, dim3((unsigned)a.chunks), dim3(kThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(bound_final_kernel, dim3(1), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}
