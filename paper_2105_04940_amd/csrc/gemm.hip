// Matrix-core products for the sampled block product:
//  * the sketched product CD = C D (Alg. 2 step 4, eq. 3.3) over the padded
//    sketch width, and
//  * the exact product MN that the estimate is judged against, optionally
//    with ||M^k N_k||_F^2 per block (the quantity (1.2) and (3.9) need).
// Both operands are row-major with the inner dimension along A's rows and
// down B's columns (the bf16 kernel also takes either operand transposed,
// for the backward products). Each workgroup (4 waves, 2 x 2) owns one
// output tile and walks the inner dimension through double-buffered LDS,
// prefetching the next step into registers while the matrix cores work on
// the current one.
//
// float32 accumulation is two-level. The plain float32 product (sgemm)
// folds its matrix-core accumulators into a float32 staging slot per lane in
// global memory every 4096 inner indices, so the inner loop keeps a single
// accumulator set; the product with per-block norms (gemm_f32) folds into a
// second register set every 256 inner indices and at block boundaries. The
// rounding error then grows like u (sqrt(F) + sqrt(K/F)) for fold period F
// instead of u sqrt(K).
//
// The epilogue optionally stores the tile and adds float64 partial sums of
// (C - Y)^2 and C^2 for the error ||MN - CD||_F; partials are reduced in a
// fixed order by a second kernel, so every result is bitwise reproducible.
#include "common.h"

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;

struct GemmArgs {
  const void* A; int64_t lda;
  const void* B; int64_t ldb;
  int64_t m, p;
  int64_t K_host; const int64_t* K_dev;
  void* C; int64_t ldc;
  const void* Y; int64_t ldy;
  double* tile_part;            // [2][tiles]
  int32_t nblk; const int64_t* off; double* blk_part;   // [nblk][tiles*4]
  int64_t tiles_m, tiles_n;
  int vec_a, vec_b;
  float* stage; int64_t ldstage;   // float32 partial sums of long inner extents
};

__device__ __forceinline__ int64_t inner_extent(const GemmArgs& g) {
  if (g.K_dev) {
    const int64_t L = *g.K_dev;
    return (L + SBMM_SKETCH_PAD - 1) / SBMM_SKETCH_PAD * SBMM_SKETCH_PAD;
  }
  return g.K_host;
}

// Map a workgroup to its output tile. Workgroups are dealt round-robin to
// the 8 XCDs (each with its own L2), so the launch index is first permuted
// XCD-major (XCD x gets a contiguous range of logical tiles), and logical
// tiles are ordered in groups of 8 tile rows walked column by column: the
// workgroups resident on one XCD at a time then share a few A and B panels.
constexpr int64_t kXcds = 8, kGroupM = 8;
__device__ __forceinline__ void tile_coords(const GemmArgs& g, int64_t& tm, int64_t& tn) {
  const int64_t bid = blockIdx.x;
  const int64_t tiles = g.tiles_m * g.tiles_n;
  const int64_t per = tiles / kXcds;
  const int64_t lg = bid < per * kXcds ? (bid % kXcds) * per + bid / kXcds : bid;
  const int64_t span = kGroupM * g.tiles_n;
  const int64_t first = (lg / span) * kGroupM;
  const int64_t gm = min(g.tiles_m - first, kGroupM);
  const int64_t r = lg % span;
  tm = first + r % gm;
  tn = r / gm;
}

// Reduce the epilogue partial sums of the workgroup in a fixed order.
__device__ void write_tile_partials(const GemmArgs& g, double e2, double n2, double* sm) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  e2 = warp_sum_f64(e2);
  n2 = warp_sum_f64(n2);
  if (lane == 0) { sm[wave] = e2; sm[4 + wave] = n2; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t tiles = g.tiles_m * g.tiles_n;
    const int64_t t = blockIdx.x;
    g.tile_part[t] = ((sm[0] + sm[1]) + sm[2]) + sm[3];
    g.tile_part[tiles + t] = ((sm[4] + sm[5]) + sm[6]) + sm[7];
  }
}

// ============================================================================
// float32: v_mfma_f32_32x32x2_f32. A wave owns (32 WMB) x (32 WNB); lane
// (r = lane % 32, h = lane / 32) feeds A row 32-block b, row r with inner
// index 2s + h. The wave's rows are interleaved so that one LDS vector read
// gives the lane its WMB A values (row WMB r + b), likewise for B columns.
// ============================================================================
template <int WMB, int WNB, bool BLOCKNORM>
__global__ __launch_bounds__(kThreads, 1) void gemm_f32_kernel(GemmArgs g) {
  constexpr int BM = 64 * WMB, BN = 64 * WNB, BK = 32;
  constexpr int SA = BM + 4, SB = BN + 4;
  constexpr int NA = BM * BK / 4 / kThreads;   // float4 loads of A per thread
  constexpr int NB = BK * BN / 4 / kThreads;   // float4 loads of B per thread
  constexpr int FOLD_TILES = 8;                // fold every 256 inner indices
  __shared__ float As[2][BK][SA];
  __shared__ float Bs[2][BK][SB];
  __shared__ double sm_red[8];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 31, lh = lane >> 5;
  const int wave_m0 = (wave & 1) * 32 * WMB;
  const int wave_n0 = (wave >> 1) * 32 * WNB;
  int64_t tm, tn;
  tile_coords(g, tm, tn);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int64_t K = inner_extent(g);
  const int64_t nkt = (K + BK - 1) / BK;
  const float* __restrict__ A = reinterpret_cast<const float*>(g.A);
  const float* __restrict__ B = reinterpret_cast<const float*>(g.B);

  f32x16 acc[WMB][WNB], tot[WMB][WNB];
  f32x16 bacc[BLOCKNORM ? WMB : 1][BLOCKNORM ? WNB : 1];
#pragma unroll
  for (int b = 0; b < WMB; ++b)
#pragma unroll
    for (int c = 0; c < WNB; ++c) {
      acc[b][c] = f32x16{};
      tot[b][c] = f32x16{};
      if constexpr (BLOCKNORM) bacc[b][c] = f32x16{};
    }

  f32x4 ra[NA], rb[NB];
  // Tiles that lie wholly inside both operands (every tile of large aligned
  // products) load with unpredicated 16-byte loads from per-thread pointers
  // advanced by one step each time; edge tiles take the predicated path.
  const bool interior = g.vec_a && g.vec_b && m0 + BM <= g.m && n0 + BN <= g.p;
  const float* pa = A + (m0 + (tid >> 3)) * g.lda + 4 * (tid & 7);
  const float* pb = B + (int64_t)(tid / (BN / 4)) * g.ldb + n0 + 4 * (tid % (BN / 4));
  const int64_t a_q_stride = (int64_t)(kThreads >> 3) * g.lda;          // rows per q step of A
  const int64_t b_q_stride = (int64_t)(kThreads / (BN / 4)) * g.ldb;    // rows per q step of B
  auto load_tile = [&](int64_t kt) {
    const int64_t k0 = kt * BK;
    if (interior && k0 + BK <= K) {
      const float* a0 = pa + k0;
      const float* b0 = pb + k0 * g.ldb;
#pragma unroll
      for (int q = 0; q < NA; ++q) ra[q] = *reinterpret_cast<const f32x4*>(a0 + q * a_q_stride);
#pragma unroll
      for (int q = 0; q < NB; ++q) rb[q] = *reinterpret_cast<const f32x4*>(b0 + q * b_q_stride);
      return;
    }
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int f = tid + kThreads * q;
      const int r = f >> 3, c4 = f & 7;
      const int64_t row = m0 + r, col = k0 + 4 * c4;
      if (g.vec_a && row < g.m && col + 4 <= K) {
        ra[q] = *reinterpret_cast<const f32x4*>(A + row * g.lda + col);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          ra[q][e] = (row < g.m && col + e < K) ? A[row * g.lda + col + e] : 0.0f;
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int f = tid + kThreads * q;
      const int kr = f / (BN / 4), c4 = f % (BN / 4);
      const int64_t krow = k0 + kr, col = n0 + 4 * c4;
      if (g.vec_b && krow < K && col + 4 <= g.p) {
        rb[q] = *reinterpret_cast<const f32x4*>(B + krow * g.ldb + col);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          rb[q][e] = (krow < K && col + e < g.p) ? B[krow * g.ldb + col + e] : 0.0f;
      }
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int f = tid + kThreads * q;
      const int r = f >> 3, c4 = f & 7;
#pragma unroll
      for (int e = 0; e < 4; ++e) As[buf][4 * c4 + e][r] = ra[q][e];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int f = tid + kThreads * q;
      const int kr = f / (BN / 4), c4 = f % (BN / 4);
      *reinterpret_cast<f32x4*>(&Bs[buf][kr][4 * c4]) = rb[q];
    }
  };

  // block boundaries (absolute inner index of the next block end)
  int32_t blk = 0;
  int64_t next_b = BLOCKNORM ? g.off[1] : INT64_MAX;
  const int64_t tiles4 = g.tiles_m * g.tiles_n * 4;

  auto close_block = [&]() {
    if constexpr (BLOCKNORM) {
      double nrm = 0.0;
#pragma unroll
      for (int b = 0; b < WMB; ++b)
#pragma unroll
        for (int c = 0; c < WNB; ++c) {
          bacc[b][c] += acc[b][c];
          acc[b][c] = f32x16{};
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const double x = (double)bacc[b][c][v];
            nrm = fma(x, x, nrm);
          }
          tot[b][c] += bacc[b][c];
          bacc[b][c] = f32x16{};
        }
      nrm = warp_sum_f64(nrm);
      if (lane == 0) g.blk_part[(int64_t)blk * tiles4 + (int64_t)blockIdx.x * 4 + wave] = nrm;
      ++blk;
      next_b = blk < g.nblk ? g.off[blk + 1] : INT64_MAX;
    }
  };

  auto mfma_step = [&](int buf, int s, int64_t klo, int64_t khi, int64_t ks) {
    const int k = 2 * s + lh;
    float av[WMB], bv[WNB];
    if constexpr (WMB == 4) {
      const f32x4 t = *reinterpret_cast<const f32x4*>(&As[buf][k][wave_m0 + 4 * lr]);
      av[0] = t[0]; av[1] = t[1]; av[2] = t[2]; av[3] = t[3];
    } else {
      const f32x2 t = *reinterpret_cast<const f32x2*>(&As[buf][k][wave_m0 + 2 * lr]);
      av[0] = t[0]; av[1] = t[1];
    }
    if constexpr (WNB == 2) {
      const f32x2 t = *reinterpret_cast<const f32x2*>(&Bs[buf][k][wave_n0 + 2 * lr]);
      bv[0] = t[0]; bv[1] = t[1];
    } else {
      const f32x4 t = *reinterpret_cast<const f32x4*>(&Bs[buf][k][wave_n0 + 4 * lr]);
      bv[0] = t[0]; bv[1] = t[1]; bv[2] = t[2]; bv[3] = t[3];
    }
    if constexpr (BLOCKNORM) {
      const int64_t kabs = ks + lh;
      if (kabs < klo || kabs >= khi) {
#pragma unroll
        for (int b = 0; b < WMB; ++b) av[b] = 0.0f;
      }
    }
#pragma unroll
    for (int b = 0; b < WMB; ++b)
#pragma unroll
      for (int c = 0; c < WNB; ++c)
        acc[b][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[b], bv[c], acc[b][c], 0, 0, 0);
  };

  auto compute = [&](int buf, int64_t kt) {
#pragma unroll
    for (int s = 0; s < BK / 2; ++s) {
      const int64_t ks = kt * BK + 2 * s;
      if constexpr (BLOCKNORM) {
        int64_t lo = ks;
        while (next_b < ks + 2) {          // a block ends inside this step
          mfma_step(buf, s, lo, next_b, ks);
          lo = next_b;
          close_block();
        }
        mfma_step(buf, s, lo, ks + 2, ks);
        if (next_b == ks + 2) close_block();
      } else {
        mfma_step(buf, s, ks, ks + 2, ks);
      }
    }
  };

  if (nkt > 0) {
    load_tile(0);
    store_tile(0);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nkt; ++kt) {
    const int cur = (int)(kt & 1);
    if (kt + 1 < nkt) load_tile(kt + 1);
    compute(cur, kt);
    if (kt + 1 < nkt) store_tile(cur ^ 1);
    __syncthreads();
    if ((kt + 1) % FOLD_TILES == 0) {
#pragma unroll
      for (int b = 0; b < WMB; ++b)
#pragma unroll
        for (int c = 0; c < WNB; ++c) {
          if constexpr (BLOCKNORM) bacc[b][c] += acc[b][c];
          else tot[b][c] += acc[b][c];
          acc[b][c] = f32x16{};
        }
    }
  }
  // blocks that end at or past the padded extent
  if constexpr (BLOCKNORM) {
    while (blk < g.nblk) close_block();
  } else {
#pragma unroll
    for (int b = 0; b < WMB; ++b)
#pragma unroll
      for (int c = 0; c < WNB; ++c) tot[b][c] += acc[b][c];
  }

  // epilogue
  float* __restrict__ Cout = reinterpret_cast<float*>(g.C);
  const float* __restrict__ Y = reinterpret_cast<const float*>(g.Y);
  double e2 = 0.0, n2 = 0.0;
#pragma unroll
  for (int b = 0; b < WMB; ++b)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int i = 8 * (v >> 2) + 4 * lh + (v & 3);
      const int64_t row = m0 + wave_m0 + WMB * i + b;
      if (row >= g.m) continue;
#pragma unroll
      for (int c = 0; c < WNB; ++c) {
        const int64_t col = n0 + wave_n0 + WNB * lr + c;
        if (col >= g.p) continue;
        const float val = tot[b][c][v];
        if (Cout) Cout[row * g.ldc + col] = val;
        const double dv = (double)val;
        if (Y) {
          const double d = dv - (double)Y[row * g.ldy + col];
          e2 = fma(d, d, e2);
        }
        n2 = fma(dv, dv, n2);
      }
    }
  if (g.tile_part) write_tile_partials(g, e2, n2, sm_red);
}

// ============================================================================
// float32, fast path: one accumulator set per wave; every FOLD_K = 4096
// inner indices the accumulators are added into a float32 staging slot in
// global memory private to the workgroup, which keeps the rounding error near
// u (sqrt(FOLD_K) + sqrt(K / FOLD_K)) while leaving the registers to the
// matrix-core accumulators. Same lane layout as above. Interior tiles run a
// loop with unpredicated 16-byte loads (the inner-dimension tail, if any, is
// one predicated step after it); edge tiles run a separate fully predicated
// loop, so neither loop carries the other's registers.
// ============================================================================
template <int WMB, int WNB, int BK>
struct SgemmTile {
  static constexpr int BM = 64 * WMB, BN = 64 * WNB;
  static constexpr int SA = BM + 4, SB = BN + 4;
  static constexpr int KC = BK / 4;                   // float4 chunks per A row
  static constexpr int NA = BM * BK / 4 / kThreads;   // float4 loads of A per thread
  static constexpr int NB = BK * BN / 4 / kThreads;   // float4 loads of B per thread
  static constexpr int FOLD_TILES = 4096 / BK;
  static constexpr int NACC = WMB * WNB * 16;
  float As[2][BK][SA];
  float Bs[2][BK][SB];
  double red[8];
};

template <int WMB, int WNB, int BK, bool EDGE>
__device__ __forceinline__ void sgemm_body(const GemmArgs& g, SgemmTile<WMB, WNB, BK>& sh,
                                           int64_t m0, int64_t n0, int64_t K) {
  using T = SgemmTile<WMB, WNB, BK>;
  constexpr int BN = T::BN, KC = T::KC, NA = T::NA, NB = T::NB, NACC = T::NACC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 31, lh = lane >> 5;
  const int wave_m0 = (wave & 1) * 32 * WMB;
  const int wave_n0 = (wave >> 1) * 32 * WNB;
  const float* __restrict__ A = reinterpret_cast<const float*>(g.A);
  const float* __restrict__ B = reinterpret_cast<const float*>(g.B);

  f32x16 acc[WMB][WNB];
#pragma unroll
  for (int b = 0; b < WMB; ++b)
#pragma unroll
    for (int c = 0; c < WNB; ++c) acc[b][c] = f32x16{};

  f32x4 ra[NA], rb[NB];
  // unpredicated loads of a whole step (interior tiles)
  const float* pa = A + (m0 + tid / KC) * g.lda + 4 * (tid % KC);
  const float* pb = B + (int64_t)(tid / (BN / 4)) * g.ldb + n0 + 4 * (tid % (BN / 4));
  const int64_t a_q_stride = (int64_t)(kThreads / KC) * g.lda;
  const int64_t b_q_stride = (int64_t)(kThreads / (BN / 4)) * g.ldb;
  auto load_fast = [&](int64_t kt) {
    const float* a0 = pa + kt * BK;
    const float* b0 = pb + kt * BK * g.ldb;
#pragma unroll
    for (int q = 0; q < NA; ++q) ra[q] = *reinterpret_cast<const f32x4*>(a0 + q * a_q_stride);
#pragma unroll
    for (int q = 0; q < NB; ++q) rb[q] = *reinterpret_cast<const f32x4*>(b0 + q * b_q_stride);
  };
  // predicated element loads (edge tiles and the inner-dimension tail)
  auto load_pred = [&](int64_t kt) {
    const int64_t k0 = kt * BK;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int f = tid + kThreads * q;
      const int r = f / KC, c4 = f % KC;
      const int64_t row = m0 + r, col = k0 + 4 * c4;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        ra[q][e] = (row < g.m && col + e < K) ? A[row * g.lda + col + e] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int f = tid + kThreads * q;
      const int kr = f / (BN / 4), c4 = f % (BN / 4);
      const int64_t krow = k0 + kr, col = n0 + 4 * c4;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        rb[q][e] = (krow < K && col + e < g.p) ? B[krow * g.ldb + col + e] : 0.0f;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int f = tid + kThreads * q;
      const int r = f / KC, c4 = f % KC;
#pragma unroll
      for (int e = 0; e < 4; ++e) sh.As[buf][4 * c4 + e][r] = ra[q][e];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int f = tid + kThreads * q;
      const int kr = f / (BN / 4), c4 = f % (BN / 4);
      *reinterpret_cast<f32x4*>(&sh.Bs[buf][kr][4 * c4]) = rb[q];
    }
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int s = 0; s < BK / 2; ++s) {
      const int k = 2 * s + lh;
      float av[WMB], bv[WNB];
      if constexpr (WMB == 4) {
        const f32x4 t = *reinterpret_cast<const f32x4*>(&sh.As[buf][k][wave_m0 + 4 * lr]);
        av[0] = t[0]; av[1] = t[1]; av[2] = t[2]; av[3] = t[3];
      } else {
        const f32x2 t = *reinterpret_cast<const f32x2*>(&sh.As[buf][k][wave_m0 + 2 * lr]);
        av[0] = t[0]; av[1] = t[1];
      }
      if constexpr (WNB == 2) {
        const f32x2 t = *reinterpret_cast<const f32x2*>(&sh.Bs[buf][k][wave_n0 + 2 * lr]);
        bv[0] = t[0]; bv[1] = t[1];
      } else {
        const f32x4 t = *reinterpret_cast<const f32x4*>(&sh.Bs[buf][k][wave_n0 + 4 * lr]);
        bv[0] = t[0]; bv[1] = t[1]; bv[2] = t[2]; bv[3] = t[3];
      }
#pragma unroll
      for (int b = 0; b < WMB; ++b)
#pragma unroll
        for (int c = 0; c < WNB; ++c)
          acc[b][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[b], bv[c], acc[b][c], 0, 0, 0);
    }
  };
  // staging slot in lane-major order: [workgroup][wave][accumulator][lane]
  float* const stg = g.stage + ((int64_t)blockIdx.x * 4 + wave) * (NACC * 64) + lane;
  int folds = 0;
  auto fold = [&]() {
#pragma unroll
    for (int b = 0; b < WMB; ++b)
#pragma unroll
      for (int c = 0; c < WNB; ++c) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          float* q = stg + ((b * WNB + c) * 16 + v) * 64;
          *q = folds ? *q + acc[b][c][v] : acc[b][c][v];
        }
        acc[b][c] = f32x16{};
        __builtin_amdgcn_sched_barrier(0);
      }
    ++folds;
  };

  // main loop: whole steps (interior) or every step (edge tiles)
  const int64_t nkt = EDGE ? (K + BK - 1) / BK : K / BK;
  if (nkt > 0) {
    if constexpr (EDGE) load_pred(0); else load_fast(0);
    store_tile(0);
  }
  __syncthreads();
  // the inner loop holds only loads, LDS traffic and matrix-core steps; the
  // fold sits between chunks of FOLD_TILES steps
  int64_t kt = 0;
  while (true) {
    const int64_t kend = min(nkt, kt + (int64_t)T::FOLD_TILES);
    for (; kt < kend; ++kt) {
      const int cur = (int)(kt & 1);
      if (kt + 1 < nkt) {
        if constexpr (EDGE) load_pred(kt + 1); else load_fast(kt + 1);
      }
      compute(cur);
      if (kt + 1 < nkt) store_tile(cur ^ 1);
      __syncthreads();
    }
    if (kt >= nkt || kt * BK >= K) break;
    fold();
  }
  if constexpr (!EDGE) {
    if (nkt * BK < K) {   // inner-dimension tail of an interior tile
      load_pred(nkt);
      store_tile(0);
      __syncthreads();
      compute(0);
    }
  }

  float* __restrict__ Cout = reinterpret_cast<float*>(g.C);
  const float* __restrict__ Y = reinterpret_cast<const float*>(g.Y);
  double e2 = 0.0, n2 = 0.0;
#pragma unroll
  for (int b = 0; b < WMB; ++b)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t row = m0 + wave_m0 + WMB * (8 * (v >> 2) + 4 * lh + (v & 3)) + b;
      if (EDGE && row >= g.m) continue;
#pragma unroll
      for (int c = 0; c < WNB; ++c) {
        const int64_t col = n0 + wave_n0 + WNB * lr + c;
        if (EDGE && col >= g.p) continue;
        float val = acc[b][c][v];
        if (folds) val += stg[((b * WNB + c) * 16 + v) * 64];
        if (Cout) Cout[row * g.ldc + col] = val;
        const double dv = (double)val;
        if (Y) {
          const double d = dv - (double)Y[row * g.ldy + col];
          e2 = fma(d, d, e2);
        }
        n2 = fma(dv, dv, n2);
      }
      if ((v & 3) == 3) __builtin_amdgcn_sched_barrier(0);   // bound the loads in flight
    }
  if (g.tile_part) write_tile_partials(g, e2, n2, sh.red);
}

template <int WMB, int WNB, int BK, int WG_PER_CU>
__global__ __launch_bounds__(kThreads, WG_PER_CU) void sgemm_kernel(GemmArgs g) {
  using T = SgemmTile<WMB, WNB, BK>;
  __shared__ T sh;
  int64_t tm, tn;
  tile_coords(g, tm, tn);
  const int64_t m0 = tm * T::BM, n0 = tn * T::BN;
  const int64_t K = inner_extent(g);
  const bool interior = g.vec_a && g.vec_b && m0 + T::BM <= g.m && n0 + T::BN <= g.p;
  if (interior)
    sgemm_body<WMB, WNB, BK, false>(g, sh, m0, n0, K);
  else
    sgemm_body<WMB, WNB, BK, true>(g, sh, m0, n0, K);
}

// ============================================================================
// bf16 operands, float32 accumulation: v_mfma_f32_32x32x16_bf16. Lane
// (r = lane % 32, h = lane / 32) holds 8 consecutive inner indices 8h..8h+7
// of A row r and B column r, so both operands sit in LDS with the inner index
// contiguous: the C tile as loaded ([row][k]) and the D tile transposed
// ([col][k], two inner indices per 32-bit LDS write). Rows and columns are
// interleaved across a wave's 32-blocks as in the float32 kernel, and the
// output layout is the same. bf16 products are exact in float32 and the
// operand rounding (2^-9) dominates the error, so there is no fold.
// ============================================================================
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int WMB, int WNB, int BK>
struct HgemmTile {
  static constexpr int BM = 64 * WMB, BN = 64 * WNB;
  static constexpr int SA = BK + 8, SB = BK + 8;        // bf16 elements per LDS row
  static constexpr int KC = BK / 8;                     // 16-byte chunks per A row
  static constexpr int NA = BM * KC / kThreads;         // 16-byte loads of A per thread
  static constexpr int NBP = (BK / 2) * (BN / 8) / kThreads;  // row-pair chunks of B per thread
  static constexpr int NAP = (BK / 2) * (BM / 8) / kThreads;  // row-pair chunks of A (transposed A)
  static constexpr int NBK = BN * KC / kThreads;               // 16-byte runs of B (transposed B)
  uint16_t As[2][BM][SA];
  uint16_t Bs[2][BN][SB];
  double red[8];
};

// AT: A is given as K x M (A[i][k] at A + k lda + i); BT: B is given as
// N x K (B[k][j] at B + j ldb + k). The LDS layouts stay [row][k] / [col][k].
template <int WMB, int WNB, int BK, bool EDGE, bool AT, bool BT>
__device__ __forceinline__ void hgemm_body(const GemmArgs& g, HgemmTile<WMB, WNB, BK>& sh,
                                           int64_t m0, int64_t n0, int64_t K) {
  using T = HgemmTile<WMB, WNB, BK>;
  constexpr int BN = T::BN, KC = T::KC, NA = T::NA, NBP = T::NBP;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 31, lh = lane >> 5;
  const int wave_m0 = (wave & 1) * 32 * WMB;
  const int wave_n0 = (wave >> 1) * 32 * WNB;
  const uint16_t* __restrict__ A = reinterpret_cast<const uint16_t*>(g.A);
  const uint16_t* __restrict__ B = reinterpret_cast<const uint16_t*>(g.B);

  f32x16 acc[WMB][WNB];
#pragma unroll
  for (int b = 0; b < WMB; ++b)
#pragma unroll
    for (int c = 0; c < WNB; ++c) acc[b][c] = f32x16{};

  // Each operand tile is gathered either as 16-byte runs along k (stored
  // directly) or as pairs of k-rows of 8 consecutive rows/columns (stored
  // transposed, two k per 32-bit write).
  constexpr int RA = NA > T::NAP ? NA : T::NAP;       // registers for either A layout
  constexpr int RB = NBP > T::NBK ? NBP : T::NBK;     // registers for either B layout
  uint4 ra0[RA], ra1[RA], rb0[RB], rb1[RB];
  auto pack8 = [](const uint16_t* t) {
    return make_uint4(t[0] | (uint32_t)t[1] << 16, t[2] | (uint32_t)t[3] << 16,
                      t[4] | (uint32_t)t[5] << 16, t[6] | (uint32_t)t[7] << 16);
  };
  // 16-byte run along k of row r (k contiguous, leading dimension ld)
  auto run_k = [&](const uint16_t* X, int64_t ld, int64_t r, int64_t rmax, int64_t k, bool vec) {
    if (!EDGE || (r < rmax && k + 8 <= K && vec)) return *reinterpret_cast<const uint4*>(X + r * ld + k);
    uint16_t t[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) t[e] = (r < rmax && k + e < K) ? X[r * ld + k + e] : 0;
    return pack8(t);
  };
  // 8 consecutive rows/columns c..c+7 of k-row kr (index contiguous)
  auto run_i = [&](const uint16_t* X, int64_t ld, int64_t kr, int64_t c, int64_t cmax, bool vec) {
    if (!EDGE || (kr < K && c + 8 <= cmax && vec)) return *reinterpret_cast<const uint4*>(X + kr * ld + c);
    uint16_t t[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) t[e] = (kr < K && c + e < cmax) ? X[kr * ld + c + e] : 0;
    return pack8(t);
  };
  auto load = [&](int64_t kt) {
    const int64_t k0 = kt * BK;
    if constexpr (!AT) {
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int f = tid + kThreads * q;
        ra0[q] = run_k(A, g.lda, m0 + f / KC, g.m, k0 + 8 * (f % KC), g.vec_a);
      }
    } else {
#pragma unroll
      for (int q = 0; q < T::NAP; ++q) {
        const int f = tid + kThreads * q;
        const int pr = f / (T::BM / 8), c8 = f % (T::BM / 8);
        ra0[q] = run_i(A, g.lda, k0 + 2 * pr, m0 + 8 * c8, g.m, g.vec_a);
        ra1[q] = run_i(A, g.lda, k0 + 2 * pr + 1, m0 + 8 * c8, g.m, g.vec_a);
      }
    }
    if constexpr (BT) {
#pragma unroll
      for (int q = 0; q < T::NBK; ++q) {
        const int f = tid + kThreads * q;
        rb0[q] = run_k(B, g.ldb, n0 + f / KC, g.p, k0 + 8 * (f % KC), g.vec_b);
      }
    } else {
#pragma unroll
      for (int q = 0; q < NBP; ++q) {
        const int f = tid + kThreads * q;
        const int pr = f / (BN / 8), c8 = f % (BN / 8);
        rb0[q] = run_i(B, g.ldb, k0 + 2 * pr, n0 + 8 * c8, g.p, g.vec_b);
        rb1[q] = run_i(B, g.ldb, k0 + 2 * pr + 1, n0 + 8 * c8, g.p, g.vec_b);
      }
    }
  };
  // write 8 rows/columns x 2 k of a transposed pair into an LDS [row][k] tile
  auto store_pair = [](uint16_t (*X)[T::SA], int c0, int k, const uint4& a0, const uint4& a1) {
    const uint32_t w0[4] = {a0.x, a0.y, a0.z, a0.w};
    const uint32_t w1[4] = {a1.x, a1.y, a1.z, a1.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint32_t lo = (w0[e >> 1] >> (16 * (e & 1))) & 0xffffu;
      const uint32_t hi = (w1[e >> 1] >> (16 * (e & 1))) & 0xffffu;
      *reinterpret_cast<uint32_t*>(&X[c0 + e][k]) = lo | (hi << 16);
    }
  };
  auto store = [&](int buf) {
    if constexpr (!AT) {
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int f = tid + kThreads * q;
        *reinterpret_cast<uint4*>(&sh.As[buf][f / KC][8 * (f % KC)]) = ra0[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < T::NAP; ++q) {
        const int f = tid + kThreads * q;
        store_pair(sh.As[buf], 8 * (f % (T::BM / 8)), 2 * (f / (T::BM / 8)), ra0[q], ra1[q]);
      }
    }
    if constexpr (BT) {
#pragma unroll
      for (int q = 0; q < T::NBK; ++q) {
        const int f = tid + kThreads * q;
        *reinterpret_cast<uint4*>(&sh.Bs[buf][f / KC][8 * (f % KC)]) = rb0[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < NBP; ++q) {
        const int f = tid + kThreads * q;
        store_pair(sh.Bs[buf], 8 * (f % (BN / 8)), 2 * (f / (BN / 8)), rb0[q], rb1[q]);
      }
    }
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int s = 0; s < BK / 16; ++s) {
      bf16x8 av[WMB], bv[WNB];
#pragma unroll
      for (int b = 0; b < WMB; ++b)
        av[b] = *reinterpret_cast<const bf16x8*>(&sh.As[buf][wave_m0 + WMB * lr + b][16 * s + 8 * lh]);
#pragma unroll
      for (int c = 0; c < WNB; ++c)
        bv[c] = *reinterpret_cast<const bf16x8*>(&sh.Bs[buf][wave_n0 + WNB * lr + c][16 * s + 8 * lh]);
#pragma unroll
      for (int b = 0; b < WMB; ++b)
#pragma unroll
        for (int c = 0; c < WNB; ++c)
          acc[b][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[b], bv[c], acc[b][c], 0, 0, 0);
    }
  };

  // interior tiles of products whose inner extent is a multiple of BK run
  // unpredicated; anything else takes the predicated loads
  const int64_t nkt = (K + BK - 1) / BK;
  if (nkt > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nkt; ++kt) {
    const int cur = (int)(kt & 1);
    if (kt + 1 < nkt) load(kt + 1);
    compute(cur);
    if (kt + 1 < nkt) store(cur ^ 1);
    __syncthreads();
  }
  float* __restrict__ Cout = reinterpret_cast<float*>(g.C);
  const float* __restrict__ Y = reinterpret_cast<const float*>(g.Y);
  double e2 = 0.0, n2 = 0.0;
#pragma unroll
  for (int b = 0; b < WMB; ++b)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t row = m0 + wave_m0 + WMB * (8 * (v >> 2) + 4 * lh + (v & 3)) + b;
      if (EDGE && row >= g.m) continue;
#pragma unroll
      for (int c = 0; c < WNB; ++c) {
        const int64_t col = n0 + wave_n0 + WNB * lr + c;
        if (EDGE && col >= g.p) continue;
        const float val = acc[b][c][v];
        if (Cout) Cout[row * g.ldc + col] = val;
        const double dv = (double)val;
        if (Y) {
          const double d = dv - (double)Y[row * g.ldy + col];
          e2 = fma(d, d, e2);
        }
        n2 = fma(dv, dv, n2);
      }
      if ((v & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
  if (g.tile_part) write_tile_partials(g, e2, n2, sh.red);
}

template <int WMB, int WNB, int BK, int WG_PER_CU, bool AT = false, bool BT = false>
__global__ __launch_bounds__(kThreads, WG_PER_CU) void hgemm_kernel(GemmArgs g) {
  using T = HgemmTile<WMB, WNB, BK>;
  __shared__ T sh;
  int64_t tm, tn;
  tile_coords(g, tm, tn);
  const int64_t m0 = tm * T::BM, n0 = tn * T::BN;
  const int64_t K = inner_extent(g);
  const bool interior = g.vec_a && g.vec_b && m0 + T::BM <= g.m && n0 + T::BN <= g.p && K % BK == 0;
  if (interior)
    hgemm_body<WMB, WNB, BK, false, AT, BT>(g, sh, m0, n0, K);
  else
    hgemm_body<WMB, WNB, BK, true, AT, BT>(g, sh, m0, n0, K);
}

// ============================================================================
// float64: v_mfma_f64_16x16x4_f64. A wave owns (16 WMB) x (16 WNB); lane
// (r = lane % 16, q = lane / 16) feeds row r with inner index 4s + q.
// ============================================================================
template <int WMB, int WNB, bool BLOCKNORM>
__global__ __launch_bounds__(kThreads) void gemm_f64_kernel(GemmArgs g) {
  constexpr int BM = 32 * WMB, BN = 32 * WNB, BK = 16;
  constexpr int SA = BM + 2, SB = BN + 2;
  constexpr int NA = BM * BK / 2 / kThreads;
  constexpr int NB = BK * BN / 2 / kThreads;
  __shared__ double As[2][BK][SA];
  __shared__ double Bs[2][BK][SB];
  __shared__ double sm_red[8];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int wave_m0 = (wave & 1) * 16 * WMB;
  const int wave_n0 = (wave >> 1) * 16 * WNB;
  int64_t tm, tn;
  tile_coords(g, tm, tn);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int64_t K = inner_extent(g);
  const int64_t nkt = (K + BK - 1) / BK;
  const double* __restrict__ A = reinterpret_cast<const double*>(g.A);
  const double* __restrict__ B = reinterpret_cast<const double*>(g.B);

  f64x4 acc[WMB][WNB], tot[WMB][WNB];
#pragma unroll
  for (int b = 0; b < WMB; ++b)
#pragma unroll
    for (int c = 0; c < WNB; ++c) { acc[b][c] = f64x4{}; tot[b][c] = f64x4{}; }

  f64x2 ra[NA], rb[NB];
  auto load_tile = [&](int64_t kt) {
    const int64_t k0 = kt * BK;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int f = tid + kThreads * q;
      const int r = f / (BK / 2), c2 = f % (BK / 2);
      const int64_t row = m0 + r, col = k0 + 2 * c2;
      if (g.vec_a && row < g.m && col + 2 <= K) {
        ra[q] = *reinterpret_cast<const f64x2*>(A + row * g.lda + col);
      } else {
#pragma unroll
        for (int e = 0; e < 2; ++e)
          ra[q][e] = (row < g.m && col + e < K) ? A[row * g.lda + col + e] : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int f = tid + kThreads * q;
      const int kr = f / (BN / 2), c2 = f % (BN / 2);
      const int64_t krow = k0 + kr, col = n0 + 2 * c2;
      if (g.vec_b && krow < K && col + 2 <= g.p) {
        rb[q] = *reinterpret_cast<const f64x2*>(B + krow * g.ldb + col);
      } else {
#pragma unroll
        for (int e = 0; e < 2; ++e)
          rb[q][e] = (krow < K && col + e < g.p) ? B[krow * g.ldb + col + e] : 0.0;
      }
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int f = tid + kThreads * q;
      const int r = f / (BK / 2), c2 = f % (BK / 2);
      As[buf][2 * c2][r] = ra[q][0];
      As[buf][2 * c2 + 1][r] = ra[q][1];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int f = tid + kThreads * q;
      const int kr = f / (BN / 2), c2 = f % (BN / 2);
      *reinterpret_cast<f64x2*>(&Bs[buf][kr][2 * c2]) = rb[q];
    }
  };

  int32_t blk = 0;
  int64_t next_b = BLOCKNORM ? g.off[1] : INT64_MAX;
  const int64_t tiles4 = g.tiles_m * g.tiles_n * 4;
  auto close_block = [&]() {
    if constexpr (BLOCKNORM) {
      double nrm = 0.0;
#pragma unroll
      for (int b = 0; b < WMB; ++b)
#pragma unroll
        for (int c = 0; c < WNB; ++c) {
#pragma unroll
          for (int v = 0; v < 4; ++v) nrm = fma(acc[b][c][v], acc[b][c][v], nrm);
          tot[b][c] += acc[b][c];
          acc[b][c] = f64x4{};
        }
      nrm = warp_sum_f64(nrm);
      if (lane == 0) g.blk_part[(int64_t)blk * tiles4 + (int64_t)blockIdx.x * 4 + wave] = nrm;
      ++blk;
      next_b = blk < g.nblk ? g.off[blk + 1] : INT64_MAX;
    }
  };
  auto mfma_step = [&](int buf, int s, int64_t klo, int64_t khi, int64_t ks) {
    const int k = 4 * s + lq;
    double av[WMB], bv[WNB];
#pragma unroll
    for (int b = 0; b < WMB; b += 2) {
      const f64x2 t = *reinterpret_cast<const f64x2*>(&As[buf][k][wave_m0 + WMB * lr + b]);
      av[b] = t[0]; av[b + 1] = t[1];
    }
#pragma unroll
    for (int c = 0; c < WNB; c += 2) {
      const f64x2 t = *reinterpret_cast<const f64x2*>(&Bs[buf][k][wave_n0 + WNB * lr + c]);
      bv[c] = t[0]; bv[c + 1] = t[1];
    }
    if constexpr (BLOCKNORM) {
      const int64_t kabs = ks + lq;
      if (kabs < klo || kabs >= khi) {
#pragma unroll
        for (int b = 0; b < WMB; ++b) av[b] = 0.0;
      }
    }
#pragma unroll
    for (int b = 0; b < WMB; ++b)
#pragma unroll
      for (int c = 0; c < WNB; ++c)
        acc[b][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[b], bv[c], acc[b][c], 0, 0, 0);
  };
  auto compute = [&](int buf, int64_t kt) {
#pragma unroll
    for (int s = 0; s < BK / 4; ++s) {
      const int64_t ks = kt * BK + 4 * s;
      if constexpr (BLOCKNORM) {
        int64_t lo = ks;
        while (next_b < ks + 4) {
          mfma_step(buf, s, lo, next_b, ks);
          lo = next_b;
          close_block();
        }
        mfma_step(buf, s, lo, ks + 4, ks);
        if (next_b == ks + 4) close_block();
      } else {
        mfma_step(buf, s, ks, ks + 4, ks);
      }
    }
  };

  if (nkt > 0) {
    load_tile(0);
    store_tile(0);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nkt; ++kt) {
    const int cur = (int)(kt & 1);
    if (kt + 1 < nkt) load_tile(kt + 1);
    compute(cur, kt);
    if (kt + 1 < nkt) store_tile(cur ^ 1);
    __syncthreads();
  }
  if constexpr (BLOCKNORM) {
    while (blk < g.nblk) close_block();
  } else {
#pragma unroll
    for (int b = 0; b < WMB; ++b)
#pragma unroll
      for (int c = 0; c < WNB; ++c) tot[b][c] += acc[b][c];
  }

  double* __restrict__ Cout = reinterpret_cast<double*>(g.C);
  const double* __restrict__ Y = reinterpret_cast<const double*>(g.Y);
  double e2 = 0.0, n2 = 0.0;
#pragma unroll
  for (int b = 0; b < WMB; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = lq + 4 * v;   // row held by (lane group lq, register v)
      const int64_t row = m0 + wave_m0 + WMB * i + b;
      if (row >= g.m) continue;
#pragma unroll
      for (int c = 0; c < WNB; ++c) {
        const int64_t col = n0 + wave_n0 + WNB * lr + c;
        if (col >= g.p) continue;
        const double val = tot[b][c][v];
        if (Cout) Cout[row * g.ldc + col] = val;
        if (Y) {
          const double d = val - Y[row * g.ldy + col];
          e2 = fma(d, d, e2);
        }
        n2 = fma(val, val, n2);
      }
    }
  if (g.tile_part) write_tile_partials(g, e2, n2, sm_red);
}

// out[r] = sum over c of part[r * cols + c], one workgroup per row, fixed order.
__global__ __launch_bounds__(kThreads) void reduce_rows_kernel(const double* __restrict__ part,
                                                               int64_t cols, double* __restrict__ out) {
  __shared__ double sm[kThreads];
  const int64_t r = blockIdx.x;
  double s = 0.0;
  for (int64_t c = threadIdx.x; c < cols; c += kThreads) s += part[r * cols + c];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[r] = sm[0];
}

// Partial sums of (X - Y)^2 and Y^2 over a grid-stride walk of the m x p
// matrices; part[0][b], part[1][b] for workgroup b.
template <typename T>
__global__ __launch_bounds__(kThreads) void error_kernel(const T* __restrict__ X, int64_t ldx,
                                                         const T* __restrict__ Y, int64_t ldy,
                                                         int64_t m, int64_t p, double* part,
                                                         int64_t nparts) {
  __shared__ double sm[8];
  double e2 = 0.0, n2 = 0.0;
  const int64_t total = m * p;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kThreads) {
    const int64_t r = i / p, c = i % p;
    const double y = (double)Y[r * ldy + c];
    const double d = (double)X[r * ldx + c] - y;
    e2 = fma(d, d, e2);
    n2 = fma(y, y, n2);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  e2 = warp_sum_f64(e2);
  n2 = warp_sum_f64(n2);
  if (lane == 0) { sm[wave] = e2; sm[4 + wave] = n2; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[blockIdx.x] = ((sm[0] + sm[1]) + sm[2]) + sm[3];
    part[nparts + blockIdx.x] = ((sm[4] + sm[5]) + sm[6]) + sm[7];
  }
}

__global__ void fill_f64_kernel(double* p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Tile shapes
constexpr int F32_WMB = 2, F32_WNB = 2, F32_BK = 16, F32_WGS = 2;   // 128 x 128, 2 per CU
constexpr int F32B_WMB = 2, F32B_WNB = 2;    // 128 x 128 with block norms
constexpr int F64_WMB = 2, F64_WNB = 2;      // 64 x 64
constexpr int BF16_WMB = 2, BF16_WNB = 2, BF16_BK = 64, BF16_WGS = 2;   // 128 x 128

void tile_shape(sbmm_dtype dt, bool blocknorm, int64_t* bm, int64_t* bn) {
  if (dt == SBMM_F64) { *bm = 32 * F64_WMB; *bn = 32 * F64_WNB; return; }
  if (dt == SBMM_BF16) { *bm = 64 * BF16_WMB; *bn = 64 * BF16_WNB; return; }
  if (blocknorm) { *bm = 64 * F32B_WMB; *bn = 64 * F32B_WNB; return; }
  *bm = 64 * F32_WMB; *bn = 64 * F32_WNB;
}

}  // namespace

int64_t gemm_tiles(sbmm_dtype dt, int64_t m, int64_t p, bool blocknorm) {
  int64_t bm, bn;
  tile_shape(dt, blocknorm, &bm, &bn);
  return ceil_div(m, bm) * ceil_div(p, bn);
}

hipError_t launch_gemm(const GemmLaunch& L, hipStream_t s) {
  const bool blocknorm = L.blk_part != nullptr;
  int64_t bm, bn;
  tile_shape(L.dt, blocknorm, &bm, &bn);
  GemmArgs g{};
  g.A = L.A; g.lda = L.lda; g.B = L.B; g.ldb = L.ldb;
  g.m = L.m; g.p = L.p; g.K_host = L.K_host; g.K_dev = L.K_dev;
  g.C = L.Cout; g.ldc = L.ldc; g.Y = L.Y; g.ldy = L.ldy;
  g.tile_part = L.tile_part;
  g.nblk = L.K_blocks; g.off = L.off_dev; g.blk_part = L.blk_part;
  g.tiles_m = ceil_div(L.m, bm);
  g.tiles_n = ceil_div(L.p, bn);
  g.stage = L.stage;
  g.ldstage = 0;
  const size_t es = dtype_size(L.dt);
  const size_t vb = 16;
  g.vec_a = ((uintptr_t)L.A % vb == 0) && ((L.lda * (int64_t)es) % (int64_t)vb == 0);
  g.vec_b = ((uintptr_t)L.B % vb == 0) && ((L.ldb * (int64_t)es) % (int64_t)vb == 0);
  const int64_t tiles = g.tiles_m * g.tiles_n;
  if (tiles == 0) return hipSuccess;
  // the float32 product folds partial sums into its staging slots once the
  // inner extent passes 4096; it must always have them
  if (L.dt == SBMM_F32 && !blocknorm && L.stage == nullptr) return hipErrorInvalidValue;
  dim3 grid((unsigned)tiles), block(kThreads);
  if (L.dt == SBMM_F64) {
    if (blocknorm) hipLaunchKernelGGL((gemm_f64_kernel<F64_WMB, F64_WNB, true>), grid, block, 0, s, g);
    else hipLaunchKernelGGL((gemm_f64_kernel<F64_WMB, F64_WNB, false>), grid, block, 0, s, g);
  } else if (L.dt == SBMM_F32) {
    if (blocknorm) hipLaunchKernelGGL((gemm_f32_kernel<F32B_WMB, F32B_WNB, true>), grid, block, 0, s, g);
    else hipLaunchKernelGGL((sgemm_kernel<F32_WMB, F32_WNB, F32_BK, F32_WGS>), grid, block, 0, s, g);
  } else if (L.dt == SBMM_BF16) {
    if (L.a_trans && L.b_trans)
      hipLaunchKernelGGL((hgemm_kernel<BF16_WMB, BF16_WNB, BF16_BK, BF16_WGS, true, true>), grid, block, 0, s, g);
    else if (L.a_trans)
      hipLaunchKernelGGL((hgemm_kernel<BF16_WMB, BF16_WNB, BF16_BK, BF16_WGS, true, false>), grid, block, 0, s, g);
    else if (L.b_trans)
      hipLaunchKernelGGL((hgemm_kernel<BF16_WMB, BF16_WNB, BF16_BK, BF16_WGS, false, true>), grid, block, 0, s, g);
    else
      hipLaunchKernelGGL((hgemm_kernel<BF16_WMB, BF16_WNB, BF16_BK, BF16_WGS>), grid, block, 0, s, g);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t gemm_stage_bytes(sbmm_dtype dt, int64_t m, int64_t p) {
  if (dt != SBMM_F32) return 0;
  int64_t bm, bn;
  tile_shape(dt, false, &bm, &bn);
  return sizeof(float) * (size_t)(ceil_div(m, bm) * ceil_div(p, bn) * bm * bn);
}

hipError_t launch_reduce_cols(const double* part, int64_t rows, int64_t cols, double* out, hipStream_t s) {
  // rows of `part` are the outputs; each is summed over its `cols` entries
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_rows_kernel, dim3((unsigned)rows), dim3(kThreads), 0, s, part, cols, out);
  return hipGetLastError();
}

int64_t error_parts(int64_t m, int64_t p) {
  const int64_t want = ceil_div(m * p, kThreads * 16);
  return want < 1 ? 1 : (want > 2048 ? 2048 : want);
}

hipError_t launch_error(sbmm_dtype dt, int64_t m, int64_t p, const void* X, int64_t ldx,
                        const void* Y, int64_t ldy, double* part, int64_t nparts, hipStream_t s) {
  dim3 grid((unsigned)nparts), block(kThreads);
  if (dt == SBMM_F64)
    hipLaunchKernelGGL(error_kernel<double>, grid, block, 0, s, (const double*)X, ldx, (const double*)Y, ldy, m, p, part, nparts);
  else if (dt == SBMM_F32)
    hipLaunchKernelGGL(error_kernel<float>, grid, block, 0, s, (const float*)X, ldx, (const float*)Y, ldy, m, p, part, nparts);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t nb = ceil_div(count, 256) < 1024 ? ceil_div(count, 256) : 1024;
  hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)nb), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t nb = ceil_div(count, 256) < 1024 ? ceil_div(count, 256) : 1024;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)nb), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}
