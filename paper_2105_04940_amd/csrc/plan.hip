// Design and sampling: the probabilities of the chosen rule, their integer
// quantization and per-stratum CDF, the draw counts of the strata, the
// with-replacement draws (Alg. 1 step 1(a)), their 1/sqrt(c_s p) scales
// (Alg. 1 step 1(b)) and the column map of the sketch.
//
// Rules (atom weights w, proportional to the probabilities):
//   block mode       uniform 1; norm ||M^k||_F ||N_k||_F (1.4);
//                    exact ||M^k N_k||_F (1.2); user
//   stratified mode  uniform 1 (p = 1/n_k); norm ||M^(i)||_2 ||N_(i)||_2
//                    (3.8); user
// Block sizes (stratified mode, weights g per block):
//   uniform 1 (c/K); norm s_k (4.2); opt sqrt(max(0, s_k^2 - ||M^k N_k||_F^2))
//   (3.9); two-step |s_k^2 - ||C^{0k} D_{0k}||_F^2|^(1/2) (4.7), from the
//   pilot estimates; user counts
// The pilot of the two-step algorithm (Alg. 3 step 1) is a stratified plan
// with [c0/K] draws in every block that can be sampled, on its own Philox
// streams (counter word 3 carries tag 2 instead of 1).
//
// Every step after the float64 weights is exact integer arithmetic:
// W = ceil(w 2^(B-1-e)) with e = floor(log2 max w) and B = 63 -
// ceil(log2 A_s) per stratum, CDF = running sum, the allocation is a
// largest-remainder split of c with 128-bit products, and a draw is Lemire's
// exactly uniform integer in [0, T) from 128-bit words of a Philox4x64-10
// stream (rejection probability below 2^-64, so a unit change of T almost
// never changes a draw) followed by an upper-bound search of the CDF.
#include "common.h"

namespace {

constexpr int kThreads = 256;

// ----------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64->128-bit multiplications, the Weyl key schedule between rounds.
// ----------------------------------------------------------------------------
struct U64x4 { uint64_t v[4]; };

__device__ __forceinline__ U64x4 philox4x64_10(U64x4 x, uint64_t k0, uint64_t k1) {
  constexpr uint64_t kMul0 = 0xD2E7470EE14C6C93ull;
  constexpr uint64_t kMul1 = 0xCA5A826395121157ull;
  constexpr uint64_t kInc0 = 0x9E3779B97F4A7C15ull;
  constexpr uint64_t kInc1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += kInc0; k1 += kInc1; }
    const uint64_t lo0 = kMul0 * x.v[0], hi0 = __umul64hi(kMul0, x.v[0]);
    const uint64_t lo1 = kMul1 * x.v[2], hi1 = __umul64hi(kMul1, x.v[2]);
    U64x4 y;
    y.v[0] = hi1 ^ x.v[1] ^ k0;
    y.v[1] = lo1;
    y.v[2] = hi0 ^ x.v[3] ^ k1;
    y.v[3] = lo0;
    x = y;
  }
  return x;
}

constexpr uint64_t kTagSample = 1;   // the draws of Alg. 1 / Alg. 2
constexpr uint64_t kTagPilot = 2;    // the pilot draws of Alg. 3 step 1

// (hi * 2^64) mod T for hi < T, by shift-and-subtract long division.
__device__ uint64_t mod_shifted(uint64_t hi, uint64_t T) {
  uint64_t r = 0;
  for (int i = 127; i >= 0; --i) {
    const uint64_t bit = i >= 64 ? (hi >> (i - 64)) & 1ull : 0ull;
    const bool over = (r >> 63) != 0;
    r = (r << 1) | bit;
    if (over || r >= T) r -= T;
  }
  return r;
}

// Lemire's bounded integer with one 128-bit word x = xh 2^64 + xl: the
// candidate is floor(x T / 2^128); the word is rejected when the low 128
// bits of x T fall below 2^128 mod T (probability < T / 2^128). Returns
// whether the word was accepted.
__device__ __forceinline__ bool lemire128(uint64_t xh, uint64_t xl, uint64_t T, uint64_t* r) {
  const uint64_t l1 = xl * T, h1 = __umul64hi(xl, T);
  const uint64_t l0 = xh * T, h0 = __umul64hi(xh, T);
  const uint64_t mid = l0 + h1;
  const uint64_t carry = mid < l0 ? 1ull : 0ull;
  *r = h0 + carry;
  if (mid != 0 || l1 >= T) return true;          // low part >= T > threshold
  const uint64_t a = (0ull - T) % T;              // 2^64 mod T
  const uint64_t thr = mod_shifted(a, T);          // 2^128 mod T
  return l1 >= thr;
}

__device__ __forceinline__ int ceil_log2_u64(uint64_t a) {
  return a <= 1 ? 0 : 64 - __clzll(a - 1);
}

// Quantize one non-negative weight with the stratum's shift (B - 1 - e).
__device__ __forceinline__ uint64_t quantize(double w, int shift) {
  if (!(w > 0.0)) return 0;
  const double q = ceil(ldexp(w, shift));
  const uint64_t W = (uint64_t)q;
  return W == 0 ? 1 : W;
}

__device__ __forceinline__ double atom_weight(const PlanLaunch& a, int64_t atom) {
  if (a.prob == SBMM_P_USER) return a.user_w[atom];
  if (a.prob == SBMM_P_UNIFORM) return 1.0;
  if (a.mode == SBMM_MODE_BLOCK) {
    if (a.prob == SBMM_P_NORM) return sqrt(a.blk[atom] * a.blk[a.K + atom]);
    return sqrt(a.blkprod_sq[atom]);   // EXACT
  }
  return sqrt(a.col_sq[atom] * a.row_sq[atom]);   // stratified NORM
}

__device__ __forceinline__ int64_t strat_begin(const PlanLaunch& a, int64_t s) {
  return a.mode == SBMM_MODE_BLOCK ? (s == 0 ? 0 : a.K) : a.off_dev[s];
}

// Block-wide reductions / scans over kThreads values in a fixed order.
__device__ double block_max(double v, double* sm) {
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = sm[0];
  __syncthreads();
  return r;
}

// Exclusive scan of one uint64 per thread; returns the thread's prefix and
// writes the total to *total.
__device__ uint64_t block_excl_scan(uint64_t v, uint64_t* sm, uint64_t* total) {
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < kThreads; o <<= 1) {
    const uint64_t add = (int)threadIdx.x >= o ? sm[threadIdx.x - o] : 0;
    __syncthreads();
    sm[threadIdx.x] += add;
    __syncthreads();
  }
  const uint64_t incl = sm[threadIdx.x];
  *total = sm[kThreads - 1];
  __syncthreads();
  return incl - v;
}

// One workgroup per stratum: weights, maximum, quantization, CDF.
__device__ void design_body(const PlanLaunch& a, int64_t s) {
  __shared__ double smd[kThreads];
  __shared__ uint64_t smu[kThreads];
  const int64_t a0 = strat_begin(a, s), a1 = strat_begin(a, s + 1);
  const int64_t As = a1 - a0;
  double mx = 0.0;
  bool bad = false;
  #pragma unroll 8
  for (int64_t i = a0 + threadIdx.x; i < a1; i += kThreads) {
    const double w = atom_weight(a, i);
    bad |= !isfinite(w) || w < 0.0;
    mx = fmax(mx, w);
  }
  if (bad) *a.status = SBMM_DEV_NONFINITE;
  mx = block_max(mx, smd);
  const int shift = (mx > 0.0) ? (63 - ceil_log2_u64((uint64_t)As)) - 1 - ilogb(mx) : 0;
  // each thread owns a contiguous run of atoms
  const int64_t per = (As + kThreads - 1) / kThreads;
  const int64_t b0 = a0 + (int64_t)threadIdx.x * per;
  const int64_t b1 = min(a1, b0 + per);
  uint64_t local = 0;
  #pragma unroll 8
  for (int64_t i = b0; i < b1; ++i) {
    const uint64_t W = (mx > 0.0) ? quantize(atom_weight(a, i), shift) : 0;
    a.W[i] = W;
    local += W;
  }
  uint64_t total;
  uint64_t run = block_excl_scan(local, smu, &total);
  #pragma unroll 8
  for (int64_t i = b0; i < b1; ++i) {
    run += a.W[i];
    a.cdf[i] = run;
  }
  if (threadIdx.x == 0) a.T[s] = total;
  if (a.p_hat) {
    __syncthreads();
    #pragma unroll 8
    for (int64_t i = a0 + threadIdx.x; i < a1; i += kThreads)
      a.p_hat[i] = total > 0 ? (double)a.W[i] / (double)total : 0.0;
  }
}

__global__ __launch_bounds__(kThreads) void design_kernel(PlanLaunch a) { design_body(a, blockIdx.x); }

// ----------------------------------------------------------------------------
// The same design for wide strata, in chunks of kDesignChunk atoms (one
// workgroup each, dchunks per stratum): the chunk maxima; then the stratum
// maximum, the quantization and the chunk sums; then the CDF from the sums of
// the chunks before (exact integers, so W, CDF, T and p_hat are the bits of
// the one-workgroup form).
// ----------------------------------------------------------------------------
constexpr int kDesignPer = 8;
constexpr int64_t kDesignChunk = (int64_t)kThreads * kDesignPer;

__device__ __forceinline__ void chunk_range(const PlanLaunch& a, int64_t* s, int64_t* a0, int64_t* a1) {
  const int64_t b = blockIdx.x;
  *s = b / a.dchunks;
  const int64_t c = b % a.dchunks;
  *a0 = strat_begin(a, *s) + c * kDesignChunk;
  *a1 = min(strat_begin(a, *s + 1), *a0 + kDesignChunk);
}

__global__ __launch_bounds__(kThreads) void design_max_kernel(PlanLaunch a) {
  __shared__ double smd[kThreads];
  int64_t s, a0, a1;
  chunk_range(a, &s, &a0, &a1);
  double mx = 0.0;
  bool bad = false;
#pragma unroll
  for (int u = 0; u < kDesignPer; ++u) {
    const int64_t i = a0 + threadIdx.x + (int64_t)u * kThreads;
    if (i < a1) {
      const double w = atom_weight(a, i);
      bad |= !isfinite(w) || w < 0.0;
      mx = fmax(mx, w);
    }
  }
  if (bad) *a.status = SBMM_DEV_NONFINITE;
  mx = block_max(mx, smd);
  if (threadIdx.x == 0) a.dpart_max[blockIdx.x] = mx;
}

__global__ __launch_bounds__(kThreads) void design_quant_kernel(PlanLaunch a) {
  __shared__ double smd[kThreads];
  __shared__ uint64_t smu[kThreads];
  int64_t s, a0, a1;
  chunk_range(a, &s, &a0, &a1);
  double mx = 0.0;
  for (int64_t c = threadIdx.x; c < a.dchunks; c += kThreads) mx = fmax(mx, a.dpart_max[s * a.dchunks + c]);
  mx = block_max(mx, smd);
  const int64_t As = strat_begin(a, s + 1) - strat_begin(a, s);
  const int shift = (mx > 0.0) ? (63 - ceil_log2_u64((uint64_t)As)) - 1 - ilogb(mx) : 0;
  uint64_t local = 0;
#pragma unroll
  for (int u = 0; u < kDesignPer; ++u) {
    const int64_t i = a0 + threadIdx.x + (int64_t)u * kThreads;
    if (i < a1) {
      const uint64_t W = (mx > 0.0) ? quantize(atom_weight(a, i), shift) : 0;
      a.W[i] = W;
      local += W;
    }
  }
  uint64_t total;
  block_excl_scan(local, smu, &total);
  if (threadIdx.x == 0) a.dpart_sum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void design_scan_kernel(PlanLaunch a) {
  __shared__ uint64_t tile[kDesignChunk];
  __shared__ uint64_t smu[kThreads];
  __shared__ uint64_t sm_base[2];
  int64_t s, a0, a1;
  chunk_range(a, &s, &a0, &a1);
  const int64_t c = blockIdx.x % a.dchunks;
  if (threadIdx.x == 0) {
    uint64_t before = 0, total = 0;
    for (int64_t q = 0; q < a.dchunks; ++q) {
      const uint64_t v = a.dpart_sum[s * a.dchunks + q];
      if (q < c) before += v;
      total += v;
    }
    sm_base[0] = before;
    sm_base[1] = total;
  }
  uint64_t w[kDesignPer];
#pragma unroll
  for (int u = 0; u < kDesignPer; ++u) {
    const int64_t i = a0 + threadIdx.x + (int64_t)u * kThreads;
    w[u] = i < a1 ? a.W[i] : 0;
    tile[threadIdx.x + u * kThreads] = w[u];
  }
  __syncthreads();
  // each thread scans its run of kDesignPer consecutive atoms of the chunk
  uint64_t local = 0;
#pragma unroll
  for (int u = 0; u < kDesignPer; ++u) local += tile[threadIdx.x * kDesignPer + u];
  uint64_t tot;
  uint64_t run = block_excl_scan(local, smu, &tot) + sm_base[0];
#pragma unroll
  for (int u = 0; u < kDesignPer; ++u) {
    run += tile[threadIdx.x * kDesignPer + u];
    tile[threadIdx.x * kDesignPer + u] = run;
  }
  __syncthreads();
  const uint64_t T = sm_base[1];
#pragma unroll
  for (int u = 0; u < kDesignPer; ++u) {
    const int64_t i = a0 + threadIdx.x + (int64_t)u * kThreads;
    if (i < a1) {
      a.cdf[i] = tile[threadIdx.x + u * kThreads];
      if (a.p_hat) a.p_hat[i] = T > 0 ? (double)w[u] / (double)T : 0.0;
    }
  }
  if (c == 0 && threadIdx.x == 0) a.T[s] = T;
}

// 128-bit helpers for the apportionment.
struct U128 { uint64_t hi, lo; };
__device__ __forceinline__ U128 mul64(uint64_t x, uint64_t y) { return {__umul64hi(x, y), x * y}; }
__device__ __forceinline__ bool le128(U128 a, U128 b) { return a.hi < b.hi || (a.hi == b.hi && a.lo <= b.lo); }

// floor(c * G / tot) and (c * G) mod tot for c < 2^31, G, tot <= 2^63, tot > 0.
__device__ void quota_rem(uint64_t c, uint64_t G, uint64_t tot, int64_t* q_out, uint64_t* r_out) {
  const U128 num = mul64(c, G);
  double est = (double)c * ((double)G / (double)tot);
  uint64_t q = (uint64_t)est;
  if (q > c) q = c;
  // correct the estimate to the exact floor (a few steps at most)
  for (int it = 0; it < 8 && !le128(mul64(q, tot), num); ++it) --q;
  for (int it = 0; it < 8 && le128(mul64(q + 1, tot), num); ++it) ++q;
  const U128 qt = mul64(q, tot);
  *q_out = (int64_t)q;
  *r_out = num.lo - qt.lo;   // < tot, so the low word is exact
}

// Allocation weight g_s of stratum s (stratified mode).
__device__ __forceinline__ double alloc_weight(const PlanLaunch& a, int64_t s) {
  if (a.alloc == SBMM_ALLOC_NORM) return a.blk[2 * a.K + s];
  if (a.alloc == SBMM_ALLOC_OPT) {
    const double sk = a.blk[2 * a.K + s];
    return sqrt(fmax(sk * sk - a.blkprod_sq[s], 0.0));
  }
  if (a.alloc == SBMM_ALLOC_TWO_STEP) {
    const double sk = a.blk[2 * a.K + s];
    return sqrt(fabs(sk * sk - a.pilot_sq[s]));
  }
  return 1.0;
}

// Stratified mode: draw counts of the K strata (single workgroup).
__global__ __launch_bounds__(kThreads) void alloc_kernel(PlanLaunch a) {
  __shared__ double smd[kThreads];
  __shared__ uint64_t smu[kThreads];
  __shared__ int64_t sm_left;
  __shared__ int sm_donor;
  const int64_t S = a.S;
  const uint64_t c = (uint64_t)a.c;
  if (a.pilot_r > 0) {
    for (int64_t s = threadIdx.x; s < S; s += kThreads) a.ck[s] = a.T[s] > 0 ? a.pilot_r : 0;
  } else if (a.alloc == SBMM_ALLOC_USER) {
    bool bad = false;
    for (int64_t s = threadIdx.x; s < S; s += kThreads) {
      const int64_t v = a.user_ck_dev[s];
      bad |= (a.T[s] > 0) != (v > 0);
      a.ck[s] = v;
    }
    if (bad) *a.status = SBMM_DEV_USER_CK;
  } else {
    // allocation weights g and their quantization over the strata
    double mx = 0.0;
    int64_t act = 0;
    for (int64_t s = threadIdx.x; s < S; s += kThreads) {
      double g = alloc_weight(a, s);
      if (!isfinite(g) || g < 0.0) { *a.status = SBMM_DEV_NONFINITE; g = 0.0; }
      mx = fmax(mx, g);
      a.rem[s] = 0;
      act += a.T[s] > 0 ? 1 : 0;
    }
    mx = block_max(mx, smd);
    uint64_t nact;
    block_excl_scan((uint64_t)act, smu, &nact);
    if (nact > c) *a.status = SBMM_DEV_BUDGET;
    const int shift = (mx > 0.0) ? (63 - ceil_log2_u64((uint64_t)S)) - 1 - ilogb(mx) : 0;
    uint64_t gsum_local = 0;
    for (int64_t s = threadIdx.x; s < S; s += kThreads) {
      double g = alloc_weight(a, s);
      if (!isfinite(g) || g < 0.0) g = 0.0;
      const uint64_t G = (a.T[s] > 0 && mx > 0.0) ? quantize(g, shift) : 0;
      a.G[s] = G;
      gsum_local += G;
    }
    uint64_t gsum;
    block_excl_scan(gsum_local, smu, &gsum);
    if (gsum == 0) {   // every sampleable stratum has zero weight: equal weights
      for (int64_t s = threadIdx.x; s < S; s += kThreads) a.G[s] = a.T[s] > 0 ? 1 : 0;
      gsum = nact;
    }
    __syncthreads();
    int64_t qsum_local = 0;
    for (int64_t s = threadIdx.x; s < S; s += kThreads) {
      int64_t q = 0;
      uint64_t r = 0;
      if (gsum > 0 && nact <= c) quota_rem(c, a.G[s], gsum, &q, &r);
      a.quota[s] = q;
      a.rem[s] = r;
      qsum_local += q;
    }
    uint64_t qsum;
    block_excl_scan((uint64_t)qsum_local, smu, &qsum);
    if (threadIdx.x == 0) sm_left = (gsum > 0 && nact <= c) ? (int64_t)(c - qsum) : 0;
    __syncthreads();
    const int64_t left = sm_left;
    // largest remainders first, ties to the lower stratum
    for (int64_t s = threadIdx.x; s < S; s += kThreads) {
      int64_t cnt = a.quota[s];
      if (a.T[s] > 0) {
        const uint64_t rs = a.rem[s];
        int64_t rank = 0;
        for (int64_t t = 0; t < S && rank < left; ++t) {
          if (a.T[t] == 0) continue;
          const uint64_t rt = a.rem[t];
          rank += (rt > rs || (rt == rs && t < s)) ? 1 : 0;
        }
        if (rank < left) ++cnt;
      }
      a.ck[s] = cnt;
    }
    __syncthreads();
    // a sampleable stratum left at zero takes one draw from the stratum
    // holding the most (ties to the lower index), in ascending order
    if (nact <= c) {
      for (int64_t s = 0; s < S; ++s) {
        if (!(a.T[s] > 0 && a.ck[s] == 0)) continue;   // uniform across the block
        int64_t best = -1, bi = 0;
        for (int64_t t = threadIdx.x; t < S; t += kThreads) {
          const int64_t v = a.ck[t];
          if (v > best) { best = v; bi = t; }
        }
        // block argmax with ties to the lower index
        smu[threadIdx.x] = ((uint64_t)(best + 1) << 32) | (uint64_t)(0xffffffffu - (uint32_t)bi);
        __syncthreads();
        for (int o = kThreads / 2; o > 0; o >>= 1) {
          if ((int)threadIdx.x < o) smu[threadIdx.x] = max(smu[threadIdx.x], smu[threadIdx.x + o]);
          __syncthreads();
        }
        if (threadIdx.x == 0) {
          sm_donor = (int)(0xffffffffu - (uint32_t)(smu[0] & 0xffffffffu));
          a.ck[sm_donor] -= 1;
          a.ck[s] += 1;
        }
        __syncthreads();
      }
    } else {
      for (int64_t s = threadIdx.x; s < S; s += kThreads) a.ck[s] = 0;
    }
  }
  __syncthreads();
  // draw offsets of the strata
  const int64_t per = (S + kThreads - 1) / kThreads;
  const int64_t b0 = (int64_t)threadIdx.x * per, b1 = min(S, b0 + per);
  uint64_t local = 0;
  for (int64_t s = b0; s < b1; ++s) local += (uint64_t)a.ck[s];
  uint64_t tot;
  uint64_t run = block_excl_scan(local, smu, &tot);
  for (int64_t s = b0; s < b1; ++s) {
    a.draw_off[s] = (int64_t)run;
    run += (uint64_t)a.ck[s];
  }
  if (threadIdx.x == 0) a.draw_off[S] = (int64_t)tot;
}

// Block mode: the single stratum gets all c draws (none if every weight is 0).
__device__ __forceinline__ void alloc_block_body(const PlanLaunch& a) {
  if (threadIdx.x == 0) {
    const int64_t cnt = a.T[0] > 0 ? a.c : 0;
    a.ck[0] = cnt;
    a.draw_off[0] = 0;
    a.draw_off[1] = cnt;
  }
}

__global__ void alloc_block_kernel(PlanLaunch a) { alloc_block_body(a); }

// Draw t (t < c).
__device__ void sample_one(const PlanLaunch& a, int64_t t) {
  const int64_t total = a.draw_off[a.S];
  if (t >= total) {   // no draws (budget error or all-zero weights)
    a.idx[t] = -1; a.scale[t] = 0.0; a.width[t] = 0;
    return;
  }
  // stratum of draw t: last s with draw_off[s] <= t
  int64_t lo = 0, hi = a.S;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (a.draw_off[mid] <= t) lo = mid; else hi = mid;
  }
  const int64_t s = lo;
  const uint64_t j = (uint64_t)(t - a.draw_off[s]);
  const uint64_t T = a.T[s];
  if (T == 0) {   // draws on a zero-weight stratum (inconsistent user counts)
    *a.status = SBMM_DEV_USER_CK;
    a.idx[t] = -1; a.scale[t] = 0.0; a.width[t] = 0;
    return;
  }
  uint64_t r = 0;
  bool done = false;
  for (uint64_t blk = 0; blk < 1024 && !done; ++blk) {
    U64x4 ctr;
    ctr.v[0] = j; ctr.v[1] = (uint64_t)s; ctr.v[2] = a.trial; ctr.v[3] = ((a.pilot_r > 0 ? kTagPilot : kTagSample) << 32) | blk;
    const U64x4 w = philox4x64_10(ctr, a.seed, 0);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (!done) {
        uint64_t cand;
        if (lemire128(w.v[2 * q], w.v[2 * q + 1], T, &cand)) { r = cand; done = true; }
      }
    }
  }
  if (!done) *a.status = SBMM_DEV_RNG;
  // first atom of the stratum whose CDF exceeds r
  const int64_t a0 = strat_begin(a, s);
  int64_t l = a0, h = strat_begin(a, s + 1);
  while (l < h) {
    const int64_t mid = (l + h) >> 1;
    if (a.cdf[mid] > r) h = mid; else l = mid + 1;
  }
  const int64_t atom = l;
  const double q = (double)a.W[atom] / (double)T;
  a.idx[t] = (int32_t)atom;
  a.scale[t] = 1.0 / sqrt((double)a.ck[s] * q);
  a.width[t] = a.mode == SBMM_MODE_BLOCK ? a.off_dev[atom + 1] - a.off_dev[atom] : 1;
}

// One thread per draw; with wpart, the workgroup also leaves the sum of its
// draws' widths for the many-workgroup offsets pass.
__global__ __launch_bounds__(kThreads) void sample_kernel(PlanLaunch a) {
  __shared__ uint64_t smu[kThreads];
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t < a.c) sample_one(a, t);
  if (a.wpart) {
    uint64_t tot;
    block_excl_scan(t < a.c ? (uint64_t)a.width[t] : 0, smu, &tot);
    if (threadIdx.x == 0) a.wpart[blockIdx.x] = tot;
  }
}

// Draw offsets on many workgroups: workgroup b scans the widths of its 256
// draws on top of the width sums of the workgroups before it.
__global__ __launch_bounds__(kThreads) void offsets_wide_kernel(PlanLaunch a) {
  __shared__ uint64_t smu[kThreads];
  const int64_t b = blockIdx.x;
  uint64_t before = 0;
  for (int64_t q = threadIdx.x; q < b; q += kThreads) before += a.wpart[q];
  uint64_t base;
  block_excl_scan(before, smu, &base);
  const int64_t t = b * kThreads + threadIdx.x;
  const uint64_t w = t < a.c ? (uint64_t)a.width[t] : 0;
  uint64_t tot;
  const uint64_t ex = block_excl_scan(w, smu, &tot);
  if (t < a.c) a.col_off[t] = (int64_t)(base + ex);
  if (b == gridDim.x - 1 && threadIdx.x == 0) a.col_off[a.c] = (int64_t)(base + tot);
}

// Exclusive scan of the draw widths into col_off (single workgroup).
__device__ void offsets_body(const PlanLaunch& a) {
  __shared__ uint64_t smu[kThreads];
  const int64_t c = a.c;
  const int64_t per = (c + kThreads - 1) / kThreads;
  const int64_t b0 = (int64_t)threadIdx.x * per, b1 = min(c, b0 + per);
  uint64_t local = 0;
  #pragma unroll 8
  for (int64_t t = b0; t < b1; ++t) local += (uint64_t)a.width[t];
  uint64_t tot;
  uint64_t run = block_excl_scan(local, smu, &tot);
  #pragma unroll 8
  for (int64_t t = b0; t < b1; ++t) {
    a.col_off[t] = (int64_t)run;
    run += (uint64_t)a.width[t];
  }
  if (threadIdx.x == 0) a.col_off[c] = (int64_t)tot;
}

__global__ __launch_bounds__(kThreads) void offsets_kernel(PlanLaunch a) { offsets_body(a); }

// Columns of the sketch fed by draw t.
__device__ __forceinline__ void colmap_one(const PlanLaunch& a, int64_t t) {
  {
    const int64_t w = a.width[t];
    const int64_t c0 = a.col_off[t];
    if (w > 0) {
      const int64_t atom = a.idx[t];
      const int64_t lo = a.mode == SBMM_MODE_BLOCK ? a.off_dev[atom] : atom;
      const double sc = a.scale[t];
      for (int64_t j = 0; j < w; ++j) {
        a.colmap[c0 + j] = (int32_t)(lo + j);
        a.colscale[c0 + j] = sc;
      }
    }
  }
}

// Zero padding of the column map up to the next multiple of 32.
__device__ __forceinline__ void colmap_pad(const PlanLaunch& a) {
  if (threadIdx.x < SBMM_SKETCH_PAD) {
    const int64_t L = a.col_off[a.c];
    const int64_t Lp = (L + SBMM_SKETCH_PAD - 1) / SBMM_SKETCH_PAD * SBMM_SKETCH_PAD;
    const int64_t l = L + threadIdx.x;
    if (l < Lp && l < a.L_pad_max) {
      a.colmap[l] = -1;
      a.colscale[l] = 0.0;
    }
  }
}

// Column map of the sketch: one thread per draw fills its columns; the
// first workgroup also writes the padding.
__global__ __launch_bounds__(kThreads) void colmap_kernel(PlanLaunch a) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t < a.c) colmap_one(a, t);
  if (blockIdx.x == 0) colmap_pad(a);
}

// Many independent block-mode problems: one workgroup runs the whole plan of
// problem blockIdx.x (design, allocation, draws, offsets, column map), with
// workgroup barriers between the steps.
__global__ __launch_bounds__(kThreads) void batch_plan_kernel(const PlanLaunch* __restrict__ plans) {
  const PlanLaunch a = plans[blockIdx.x];   // a copy: read once, not reloaded behind the kernel's stores
  design_body(a, 0);
  __syncthreads();
  alloc_block_body(a);
  __syncthreads();
  for (int64_t t = threadIdx.x; t < a.c; t += kThreads) sample_one(a, t);
  __syncthreads();
  offsets_body(a);
  __syncthreads();
  for (int64_t t = threadIdx.x; t < a.c; t += kThreads) colmap_one(a, t);
  colmap_pad(a);
}

}  // namespace

hipError_t launch_batch_plan(const PlanLaunch* plans_dev, int32_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_plan_kernel, dim3((unsigned)count), dim3(kThreads), 0, s, plans_dev);
  return hipGetLastError();
}

// Strata wider than two chunks are cut into chunks when that keeps the grid
// dense (at most twice the workgroups a perfect split would need).
int32_t plan_design_chunks(int64_t max_atoms, int64_t A, int64_t S) {
  const int64_t c = ceil_div(max_atoms, kDesignChunk);
  if (c <= 2) return 1;
  return S * c <= 2 * (ceil_div(A, kDesignChunk) + S) ? (int32_t)c : 1;
}

// Many-workgroup offsets for more than one workgroup of draws, up to 2^20
// draws (each workgroup sums the width sums before it).
bool plan_wide_offsets(int64_t c) { return c > kThreads && c <= (int64_t(1) << 20); }

hipError_t launch_plan(const PlanLaunch& a, hipStream_t s) {
  if (a.dchunks > 1) {
    const dim3 grid((unsigned)(a.S * a.dchunks));
    hipLaunchKernelGGL(design_max_kernel, grid, dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(design_quant_kernel, grid, dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(design_scan_kernel, grid, dim3(kThreads), 0, s, a);
  } else {
    hipLaunchKernelGGL(design_kernel, dim3((unsigned)a.S), dim3(kThreads), 0, s, a);
  }
  if (a.mode == SBMM_MODE_BLOCK)
    hipLaunchKernelGGL(alloc_block_kernel, dim3(1), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(alloc_kernel, dim3(1), dim3(kThreads), 0, s, a);
  const unsigned nb = (unsigned)ceil_div(a.c, kThreads);
  hipLaunchKernelGGL(sample_kernel, dim3(nb), dim3(kThreads), 0, s, a);
  if (a.wpart)
    hipLaunchKernelGGL(offsets_wide_kernel, dim3(nb), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(offsets_kernel, dim3(1), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(colmap_kernel, dim3(nb), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}
