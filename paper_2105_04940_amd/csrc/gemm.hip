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

#include <cstring>

#include "gemm_common.h"

namespace {

using namespace gemm_detail;

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

template <int WMB, int WNB, int BK, bool EDGE, bool GATHER = false>
__device__ __forceinline__ void sgemm_body(const GemmArgs& g, SgemmTile<WMB, WNB, BK>& sh,
                                           int64_t m0, int64_t n0, int64_t K, int64_t slot,
                                           int64_t part, int64_t nparts) {
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
  // gathered loads (sketch read in place): the A tile is loaded in the same
  // layout as the plain one (a lane reads 4 consecutive sketch columns of a
  // row), from columns colmap[k..k+3] of M: one 16-byte load when they are 4
  // consecutive columns with one scale (the common case inside a drawn
  // block), else 4 element loads; B rows are rows colmap[k] of N. Each value
  // is (float)(x * scale) with the product in float64, as the gather writes
  // it. The column map and scales of step kt + 1 are fetched while step kt's
  // matrix loads are in flight, so a step never waits on the map and then
  // on the data.
  int4 ja = {-1, -1, -1, -1};
  double sa[4] = {0.0, 0.0, 0.0, 0.0};
  int32_t jb[NB];
  double sb[NB];
  const int ca = tid % KC;   // A chunk of this lane (the same for every q since kThreads % KC == 0)
  const int64_t nsteps = EDGE ? (K + BK - 1) / BK : K / BK;
  auto load_meta = [&](int64_t kt) {
    const int64_t k0 = kt * BK;
    const int64_t ka = k0 + 4 * ca;
    if (!EDGE || ka < K) {
      ja = *reinterpret_cast<const int4*>(g.colmap + ka);
      const f64x2 s01 = *reinterpret_cast<const f64x2*>(g.colscale + ka);
      const f64x2 s23 = *reinterpret_cast<const f64x2*>(g.colscale + ka + 2);
      sa[0] = s01[0]; sa[1] = s01[1]; sa[2] = s23[0]; sa[3] = s23[1];
    } else {
      ja = int4{-1, -1, -1, -1};
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int64_t krow = k0 + (tid + kThreads * q) / (BN / 4);
      jb[q] = (!EDGE || krow < K) ? g.colmap[krow] : -1;
      sb[q] = jb[q] >= 0 ? g.colscale[krow] : 0.0;
    }
  };
  auto load_gather = [&](int64_t kt) {
    const bool run = ja.x >= 0 && ja.y == ja.x + 1 && ja.z == ja.x + 2 && ja.w == ja.x + 3 &&
                     sa[1] == sa[0] && sa[2] == sa[0] && sa[3] == sa[0];
    const int jj[4] = {ja.x, ja.y, ja.z, ja.w};
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int64_t row = m0 + (tid + kThreads * q) / KC;
      const bool row_ok = !EDGE || row < g.m;
      if (run && row_ok) {
        f32x4 x;
        __builtin_memcpy(&x, A + row * g.lda + ja.x, sizeof(x));   // 4-byte aligned 16-byte load
#pragma unroll
        for (int e = 0; e < 4; ++e) ra[q][e] = (float)((double)x[e] * sa[0]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          ra[q][e] = (jj[e] >= 0 && row_ok) ? (float)((double)A[row * g.lda + jj[e]] * sa[e]) : 0.0f;
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int f = tid + kThreads * q;
      const int64_t col = n0 + 4 * (f % (BN / 4));
      if (jb[q] < 0) {
        rb[q] = f32x4{};
        continue;
      }
      const float* src = B + (int64_t)jb[q] * g.ldb + col;
      if (!EDGE) {
        const f32x4 x = *reinterpret_cast<const f32x4*>(src);
#pragma unroll
        for (int e = 0; e < 4; ++e) rb[q][e] = (float)((double)x[e] * sb[q]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) rb[q][e] = col + e < g.p ? (float)((double)src[e] * sb[q]) : 0.0f;
      }
    }
    if (kt + 1 < nsteps) load_meta(kt + 1);
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
      } else if constexpr (WMB == 2) {
        const f32x2 t = *reinterpret_cast<const f32x2*>(&sh.As[buf][k][wave_m0 + 2 * lr]);
        av[0] = t[0]; av[1] = t[1];
      } else {
        av[0] = sh.As[buf][k][wave_m0 + lr];
      }
      if constexpr (WNB == 2) {
        const f32x2 t = *reinterpret_cast<const f32x2*>(&sh.Bs[buf][k][wave_n0 + 2 * lr]);
        bv[0] = t[0]; bv[1] = t[1];
      } else if constexpr (WNB == 4) {
        const f32x4 t = *reinterpret_cast<const f32x4*>(&sh.Bs[buf][k][wave_n0 + 4 * lr]);
        bv[0] = t[0]; bv[1] = t[1]; bv[2] = t[2]; bv[3] = t[3];
      } else {
        bv[0] = sh.Bs[buf][k][wave_n0 + lr];
      }
#pragma unroll
      for (int b = 0; b < WMB; ++b)
#pragma unroll
        for (int c = 0; c < WNB; ++c)
          acc[b][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[b], bv[c], acc[b][c], 0, 0, 0);
    }
  };
  // staging slot in lane-major order: [workgroup][wave][accumulator][lane]
  float* const stg = g.stage + (slot * 4 + wave) * (NACC * 64) + lane;
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
  auto load = [&](int64_t kt) {
    if constexpr (GATHER) load_gather(kt);
    else if constexpr (EDGE) load_pred(kt);
    else load_fast(kt);
  };
  if (nkt > 0) {
    if constexpr (GATHER) load_meta(0);
    load(0);
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
      if (kt + 1 < nkt) load(kt + 1);
      compute(cur);
      if (kt + 1 < nkt) store_tile(cur ^ 1);
      __syncthreads();
    }
    if (kt >= nkt || kt * BK >= K) break;
    fold();
  }
  if constexpr (!EDGE && !GATHER) {
    if (nkt * BK < K) {   // inner-dimension tail of an interior tile
      load_pred(nkt);
      store_tile(0);
      __syncthreads();
      compute(0);
    }
  }

  double e2 = 0.0, n2 = 0.0;
  // one group ahead: these register-staged tiles have less room
  store_block_with_error<WMB, WNB, 1>(
      acc, [=](int b, int v) { return m0 + wave_m0 + WMB * (8 * (v >> 2) + 4 * lh + (v & 3)) + b; },
      [=](int c) { return n0 + wave_n0 + WNB * lr + c; }, reinterpret_cast<float*>(g.C), g.ldc,
      reinterpret_cast<const float*>(g.Y), g.ldy, g.m, g.p, e2, n2, folds > 0,
      [&](int b, int c, int v) { return stg[((b * WNB + c) * 16 + v) * 64]; });
  if (g.tile_part) write_tile_partials_at(g, e2, n2, sh.red, part, nparts);
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
  const int64_t tiles = g.tiles_m * g.tiles_n;
  if (interior)
    sgemm_body<WMB, WNB, BK, false>(g, sh, m0, n0, K, blockIdx.x, blockIdx.x, tiles);
  else
    sgemm_body<WMB, WNB, BK, true>(g, sh, m0, n0, K, blockIdx.x, blockIdx.x, tiles);
}

// ============================================================================
// Float32 products on 256 x 256 tiles with LDS-direct loads: one workgroup of
// eight waves per CU (two per SIMD), each wave a 128 x 64 part of the tile as
// 4 x 2 blocks of v_mfma_f32_32x32x2_f32 (128 accumulators). A (m x K) rows
// are streamed into LDS as 16-byte chunks of 4 consecutive k, XOR-swizzled per
// row; B (K x p, row-major) rows are streamed as they are (rows padded by 8
// floats so the two half-waves of a column read hit different banks). A step
// covers 32 k: a lane reads one chunk of its A row (4 k) and the matching 4
// rows of its B columns, and feeds 4 MFMAs whose k are the chunk's 4 entries
// in the lane's half-wave (half h takes k = 8u + 4h + q in MFMA q of
// super-step u): every k of the step meets its partner exactly once. Two
// stages in LDS, the next step's loads in flight while the current one
// computes.
//
// The output is accounted for in the 128 x 128 tiling of the other float32
// kernels: the two waves of a 128 x 128 quarter share its staging slot (the
// fold every 4096 k, one half each) and its error partials (combined in LDS,
// written once), so callers size and reduce both as before.
// ============================================================================

struct SgemmLdsTile {
  static constexpr int BM = 256, BN = 256, BK = 32, KC = 8, STAGES = 2;
  static constexpr int SBN = BN + 8;           // padded B row (floats)
  static constexpr int FOLD_STEPS = 4096 / BK;
  uint4 As[STAGES][BM * KC];
  float Bs[STAGES][BK][SBN];
  double red[2][8];
};

// waves per workgroup of the kernel below: two per SIMD, 128 x 64 each (one
// per SIMD with 128 x 128 each spills its registers)
constexpr int kLdsWaves = 8;

__device__ __forceinline__ int lds_a_slot(int row, int chunk) { return row * 8 + (chunk ^ ((row >> 1) & 7)); }

// Buffer resource over `bytes` bytes from `base` (fields made wave-uniform).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t f32_rsrc(const float* base, int64_t bytes) {
  const uint64_t u = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  const int nb = __builtin_amdgcn_readfirstlane((int)(bytes > 0 ? bytes : 0));
  void* p = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, nb, 0x00020000);
}

// Tile (tm, tn) of a product. GROUPED: one work item of a grouped launch,
// whose staging slot is the item (a 256 x 256 slot, one eighth per wave) and
// whose error partials go to slot `part` of [2][nparts] (the eight waves'
// sums added in wave order). Otherwise the 128 x 128 accounting above.
template <int NW, bool GROUPED>
__device__ __forceinline__ void sgemm_lds_body(const GemmArgs& g, SgemmLdsTile& sh, int64_t tm, int64_t tn,
                                               int64_t item, int64_t part, int64_t nparts) {
  using T = SgemmLdsTile;
  constexpr int KC = T::KC, BK = T::BK;
  constexpr int CB = 16 / NW;                    // 32-column blocks per wave (2 or 4)
  constexpr int AINSTS = T::BM * KC / 64 / NW;   // A: instructions per wave per stage (4)
  constexpr int BINSTS = BK / NW;                // B: rows per wave per stage (4)
  const int64_t m0 = tm * T::BM, n0 = tn * T::BN;
  const int64_t K = inner_extent(g);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 31, lh = lane >> 5;
  const int qm = wave & 1, qn = wave >> 1;       // 128-row half, column part of 32 CB
  const int wm0 = qm * 128, wn0 = qn * 32 * CB;
  const float* A = reinterpret_cast<const float*>(g.A) + m0 * g.lda;
  const float* B = reinterpret_cast<const float*>(g.B);
  // A records end at the last row's K-th entry: the range check is per
  // dword (and counts the scalar offset), so a chunk straddling K in the
  // last row reads zeros past K; in the other rows it reads the row's next
  // entries, which the last step clears in LDS (below)
  const int64_t arows = min((int64_t)T::BM, g.m - m0);
  const i32x4 ra = buffer_words(A, arows > 0 ? (int)(((arows - 1) * g.lda + K) * 4) : 0);
  constexpr unsigned kOut = 0x80000000u;   // past any record count

  f32x16 acc[4][CB];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[b][c] = f32x16{};

  // the parts of B's per-step record count, made scalar once: computed next
  // to the loads from the vector copies the compiler keeps for the lane
  // offsets, they came back through a readfirstlane right before a load
  // (whose resource then needs five wait states)
  const int ldb_bytes = __builtin_amdgcn_readfirstlane((int)(g.ldb * 4));
  const int btail_bytes = __builtin_amdgcn_readfirstlane((int)((g.p - n0) * 4));
  auto issue = [&](int64_t kt, int buf) {
    const int64_t k0 = kt * BK;
    const unsigned sk = (unsigned)(k0 * 4);
#pragma unroll
    for (int j = 0; j < AINSTS; ++j) {
      const int row = (AINSTS * wave + j) * (64 / KC) + lane / KC;
      const int chunk = (lane % KC) ^ ((row >> 1) & 7);
      const bool live = k0 + 4 * chunk < K;
      const unsigned oa = live ? (unsigned)(row * g.lda * 4 + chunk * 16) : kOut;
      lds_dma16(ra, lds_offset(&sh.As[buf][(AINSTS * wave + j) * 64]), oa, sk);
    }
    // B: rows k0 .. k0 + 31 of columns n0 .. n0 + 255; a row past K, or an
    // entry past p in the stage's last row, lies past the record count and
    // reads 0 (the check is per dword); entries past p in the other rows
    // only feed output columns that are not stored
    const int brows = (int)min((int64_t)BK, K - k0);
    const i32x4 rb = buffer_words(B + k0 * g.ldb + n0, brows > 0 ? (brows - 1) * ldb_bytes + btail_bytes : 0);
#pragma unroll
    for (int j = 0; j < BINSTS; ++j) {
      const int r = BINSTS * wave + j;
      const unsigned ob = (unsigned)(r * g.ldb * 4 + lane * 16);
      lds_dma16(rb, lds_offset(&sh.Bs[buf][r][0]), ob, 0u);
    }
  };
  // the fragments of super-step u + 1 are read from LDS while the MFMAs of
  // super-step u run (two register sets; four super-steps a step, so
  // super-step 0 of every step uses set 0)
  constexpr int NU = BK / 8;
  static_assert(NU % 2 == 0, "super-step 0 of every step in register set 0");
  f32x4 av[2][4];
  float bv[2][CB][4];
  auto frag = [&](int buf, int u, int r) {
#pragma unroll
    for (int b = 0; b < 4; ++b)
      av[r][b] = __builtin_bit_cast(f32x4, sh.As[buf][lds_a_slot(wm0 + 32 * b + lr, 2 * u + lh)]);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < CB; ++c) bv[r][c][q] = sh.Bs[buf][8 * u + 4 * lh + q][wn0 + 32 * c + lr];
  };
  auto mfmas = [&](int r) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < CB; ++c)
          acc[b][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[r][b][q], bv[r][c][q], acc[b][c], 0, 0, 0);
  };

  // the 128 x 128 tile of the 128 x 128 tiling this wave's part lies in
  // (staging slot and error partials), if it lies inside the output
  const int64_t tn128 = (g.p + 127) / 128, tiles128 = ((g.m + 127) / 128) * tn128;
  constexpr int PER = 4 / CB;                    // waves sharing a 128 x 128 tile (2 or 1)
  const int64_t srow = 2 * tm + qm, scol = 2 * tn + qn / PER;
  const bool inside = GROUPED || (srow * 128 < g.m && scol * 128 < g.p);
  const int64_t slot = GROUPED ? 0 : (inside ? srow * tn128 + scol : 0);
  // this wave's part of the slot, [accumulator][lane], through a buffer
  // resource so that each accumulator's offset is a scalar (no per-lane
  // address registers); a wave outside the output gets no records
  float* const sbase = GROUPED ? g.stage + item * (256 * 256) + wave * (128 * 32 * CB)
                               : g.stage + slot * (128 * 128) + (qn % PER) * (128 * 32 * CB);
  const __amdgpu_buffer_rsrc_t rs = f32_rsrc(sbase, inside ? 128 * 32 * CB * 4 : 0);
  const int vo = lane * 4;
  int folds = 0;
  // slot += acc (acc first), one accumulator block at a time; the slot
  // values of the next block are requested before the current one is added
  auto fold = [&]() {
    float nx[2][16];
    auto ld = [&](int q) {
#pragma unroll
      for (int v = 0; v < 16; ++v)
        nx[q & 1][v] = folds ? __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, vo, (q * 16 + v) * 256, 0))
                             : 0.0f;
    };
    ld(0);
#pragma unroll
    for (int q = 0; q < 4 * CB; ++q) {   // accumulator block q = b CB + c
      if (q + 1 < 4 * CB) ld(q + 1);
      const int b = q / CB, c = q % CB;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        float x = acc[b][c][v];
        if (folds) x += nx[q & 1][v];
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), rs, vo, (q * 16 + v) * 256, 0);
      }
      acc[b][c] = f32x16{};
      __builtin_amdgcn_sched_barrier(0);
    }
    ++folds;
  };

  // The inner extent ends inside a chunk of the last step kt: clear the A
  // entries past K of that chunk in every row (B rows past K already read
  // zero), once the step's tile has landed and before any wave reads it.
  auto clear_tail = [&](int64_t kt) {
    if (K & 3) {
      const int kz = (int)(K - kt * BK), cs = kz >> 2, e0 = kz & 3;
      if (tid < T::BM) {
        float* q = reinterpret_cast<float*>(&sh.As[kt & 1][lds_a_slot(tid, cs)]);
        for (int e = e0; e < 4; ++e) q[e] = 0.0f;
      }
      __syncthreads();
    }
  };
  // Step kt's tile was issued one step ahead into stage kt & 1. A step runs
  // super-steps 0 .. NU - 2; then every wave waits for its own LDS reads and
  // for step kt + 1's tile, and barriers: step kt + 1's stage is complete and
  // no wave reads stage kt & 1 any more, so step kt + 2's tile goes there.
  // The last super-step's matrix instructions then run after the first
  // fragments of step kt + 1 are requested, so the barrier, the loads' issue
  // and that first read no longer stand between two steps' matrix work.
  const int64_t nkt = (K + BK - 1) / BK;
  auto body = [&](int64_t kt, int buf) {
#pragma unroll
    for (int u = 0; u + 1 < NU; ++u) {
      frag(buf, u + 1, (u + 1) & 1);
      __builtin_amdgcn_sched_barrier(0);
      mfmas(u & 1);
      __builtin_amdgcn_sched_barrier(0);
    }
    // (after the last step the barrier is uniform and the reads of the
    // other stage, in bounds, go unused: one path for every step)
    wait_loads_reads_barrier<0>();
    if (kt + 2 < nkt) issue(kt + 2, buf);
    if (kt + 2 == nkt) clear_tail(kt + 1);
    frag(buf ^ 1, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
    mfmas((NU - 1) & 1);
    __builtin_amdgcn_sched_barrier(0);
    if ((kt + 1) % T::FOLD_STEPS == 0 && kt + 1 < nkt) fold();
  };
  if (nkt > 0) {
    issue(0, 0);
    wait_loads_barrier<0>();
    if (nkt > 1) issue(1, 1);
    else clear_tail(0);
    frag(0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
  for (int64_t kt = 0; kt < nkt; kt += 2) {
    body(kt, 0);
    if (kt + 1 < nkt) body(kt + 1, 1);
  }

  double e2 = 0.0, n2 = 0.0;
  store_tile_with_error<CB>(
      acc, reinterpret_cast<float*>(g.C), g.ldc, reinterpret_cast<const float*>(g.Y), g.ldy, g.m, g.p,
      m0 + wm0 + 4 * lh, n0 + wn0 + lr, e2, n2, folds > 0, [&](int b, int c, int v) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, vo, ((b * CB + c) * 16 + v) * 256, 0));
      });
  if (g.tile_part && GROUPED) {
    e2 = warp_sum_f64(e2);
    n2 = warp_sum_f64(n2);
    if (lane == 0) {
      sh.red[0][wave] = e2;
      sh.red[1][wave] = n2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = 0.0, b = 0.0;
      for (int w = 0; w < NW; ++w) {
        a += sh.red[0][w];
        b += sh.red[1][w];
      }
      g.tile_part[part] = a;
      g.tile_part[nparts + part] = b;
    }
  } else if (g.tile_part) {
    // the two waves of a 128 x 128 tile (qn = 2s, 2s + 1): the first adds
    // the second's sums after its own, in that order
    e2 = warp_sum_f64(e2);
    n2 = warp_sum_f64(n2);
    if constexpr (PER == 1) {
      if (inside && lane == 0) {
        g.tile_part[slot] = e2;
        g.tile_part[tiles128 + slot] = n2;
      }
    } else {
      if (lane == 0) {
        sh.red[0][wave] = e2;
        sh.red[1][wave] = n2;
      }
      __syncthreads();
      if (inside && lane == 0 && (qn & 1) == 0) {
        g.tile_part[slot] = sh.red[0][wave] + sh.red[0][wave + 2];
        g.tile_part[tiles128 + slot] = sh.red[1][wave] + sh.red[1][wave + 2];
      }
    }
  }
}

template <int NW>
__global__ __launch_bounds__(NW * 64, 1) void sgemm_lds_kernel(GemmArgs g) {
  __shared__ SgemmLdsTile sh;
  int64_t tm, tn;
  tile_coords(g, tm, tn);
  sgemm_lds_body<NW, false>(g, sh, tm, tn, 0, 0, 0);
}

// ============================================================================
// Many independent float32 products in one launch. The host lists the work
// items (problem, tile) in the order they should start (longest inner extent
// first) and workgroup i takes item i; the hardware dispatches workgroups in
// index order as compute units free up, so short products fill in behind
// long ones. A workgroup runs exactly one tile: there is no loop over items
// around the barriers of the tile body (with thread-0-only blocks on such a
// loop's back edge, the compiler can split the loop so that the other lanes
// re-enter the next item before thread 0 has fetched it). The float32
// staging slot and the error partials are indexed by the item.
// ============================================================================
struct GroupedArgs {
  const GemmArgs* probs;       // per problem
  const int32_t* item_prob;    // per work item: problem
  const int32_t* item_tile;    // per work item: tile of the problem (row-major over its tiles)
  const int64_t* part_base;    // per problem: first partial slot
  int64_t items;
  int64_t nparts;
};

template <int WMB, int WNB, int BK, int WG_PER_CU, bool GATHER>
__global__ __launch_bounds__(kThreads, WG_PER_CU) void sgemm_grouped_kernel(GroupedArgs ga) {
  using T = SgemmTile<WMB, WNB, BK>;
  __shared__ T sh;
  const int64_t it = blockIdx.x;
  const int32_t pi = __builtin_amdgcn_readfirstlane(ga.item_prob[it]);
  const int64_t local = __builtin_amdgcn_readfirstlane(ga.item_tile[it]);
  // a copy of the problem's arguments: read once into scalar registers (through
  // a reference the compiler reloads them inside the k loop, since the
  // kernel's stores might alias them)
  const GemmArgs g = ga.probs[pi];
  const int64_t m0 = (local / g.tiles_n) * T::BM, n0 = (local % g.tiles_n) * T::BN;
  const int64_t K = inner_extent(g);
  const bool interior = (GATHER || g.vec_a) && g.vec_b && m0 + T::BM <= g.m && n0 + T::BN <= g.p;
  const int64_t part = ga.part_base[pi] + local;
  if (interior)
    sgemm_body<WMB, WNB, BK, false, GATHER>(g, sh, m0, n0, K, it, part, ga.nparts);
  else
    sgemm_body<WMB, WNB, BK, true, GATHER>(g, sh, m0, n0, K, it, part, ga.nparts);
}

// The 256 x 256 LDS-direct tiles as a grouped launch (sketch materialized or
// exact product; no fused gather).
template <int NW>
__global__ __launch_bounds__(NW * 64, 1) void sgemm_grouped_lds_kernel(GroupedArgs ga) {
  __shared__ SgemmLdsTile sh;
  const int64_t it = blockIdx.x;
  const int32_t pi = __builtin_amdgcn_readfirstlane(ga.item_prob[it]);
  const int64_t local = __builtin_amdgcn_readfirstlane(ga.item_tile[it]);
  const GemmArgs g = ga.probs[pi];   // by value, as in the kernel above
  sgemm_lds_body<NW, true>(g, sh, local / g.tiles_n, local % g.tiles_n, it, ga.part_base[pi] + local, ga.nparts);
}

// ============================================================================
// Grouped float32 products on 128 x 128 tiles with LDS-direct loads, two
// workgroups per CU, four waves of 64 x 64 (2 x 2 blocks of
// v_mfma_f32_32x32x2_f32). For the many small products of a batch, where
// 256 x 256 tiles waste their ragged edges and the register-staged 128 x 128
// kernel spends its issue slots on staging. A step covers 32 k as in the
// 256 x 256 kernel (A rows as XOR-swizzled 16-byte chunks of 4 k, B rows as
// loaded); a B load instruction fills two 128-float rows (one per half-wave),
// so B rows are stored in pairs padded by 16 floats, which puts rows four
// apart (the two half-waves of a fragment read) 32 banks apart. The two
// stages are separate LDS objects over a two-step loop, so the loads into
// one never look like they alias the reads of the other. Staging slot (fold
// every 4096 k) and error partials per work item, as the other grouped
// kernels keep them.
// ============================================================================
constexpr int kL128Pair = 2 * 128 + 16;   // floats per stored pair of B rows

struct Lds128Stage {
  uint4 A[128 * 8];
  float B[16 * kL128Pair];
};

__global__ __launch_bounds__(256, 2) void sgemm_grouped_lds128_kernel(GroupedArgs ga) {
  __shared__ Lds128Stage st0, st1;
  __shared__ double red[2][4];
  constexpr int BK = 32, FOLD_STEPS = 4096 / BK;
  const int64_t it = blockIdx.x;
  const int32_t pi = __builtin_amdgcn_readfirstlane(ga.item_prob[it]);
  const int64_t local = __builtin_amdgcn_readfirstlane(ga.item_tile[it]);
  const GemmArgs g = ga.probs[pi];   // by value, as in the kernels above
  const int64_t m0 = (local / g.tiles_n) * 128, n0 = (local % g.tiles_n) * 128;
  const int64_t K = inner_extent(g);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 31, lh = lane >> 5;
  const int wm0 = (wave & 1) * 64, wn0 = (wave >> 1) * 64;
  const float* A = reinterpret_cast<const float*>(g.A) + m0 * g.lda;
  const float* B = reinterpret_cast<const float*>(g.B);
  // A records end at the last row's K-th entry (the range check is per
  // dword): a chunk straddling K reads zeros past K in the last row and the
  // row's next entries elsewhere, which the last step clears in LDS
  const int64_t arows = min((int64_t)128, g.m - m0);
  const __amdgpu_buffer_rsrc_t ra = f32_rsrc(A, arows > 0 ? ((arows - 1) * g.lda + K) * 4 : 0);
  constexpr unsigned kOut = 0x80000000u;

  f32x16 acc[2][2];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[b][c] = f32x16{};

  auto issue = [&](int64_t kt, Lds128Stage& dst) {
    const int64_t k0 = kt * BK;
    const unsigned sk = (unsigned)(k0 * 4);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = (4 * wave + j) * 8 + (lane >> 3);
      const int chunk = (lane & 7) ^ ((row >> 1) & 7);
      const bool live = k0 + 4 * chunk < K;
      const unsigned oa = live ? (unsigned)(row * g.lda * 4 + chunk * 16) : kOut;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          ra, (__attribute__((address_space(3))) void*)&dst.A[(4 * wave + j) * 64], 16, oa, sk, 0, 0);
    }
    // B rows k0 .. k0 + 31 of columns n0 .. n0 + 127: a row past K, or an
    // entry past p in the step's last row, lies past the record count and
    // reads 0; entries past p in other rows only feed columns not stored
    const int64_t brows = min((int64_t)BK, K - k0);
    const int64_t bbytes = brows > 0 ? ((brows - 1) * g.ldb + (g.p - n0)) * 4 : 0;
    const __amdgpu_buffer_rsrc_t rb = f32_rsrc(B + k0 * g.ldb + n0, bbytes);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = 4 * wave + j;                 // rows 2q (lanes 0..31) and 2q + 1 (32..63)
      const unsigned ob = (unsigned)((2 * q + lh) * g.ldb * 4 + lr * 16);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (__attribute__((address_space(3))) void*)&dst.B[q * kL128Pair],
                                               16, ob, 0, 0, 0);
    }
  };
  auto brow = [](const Lds128Stage& st, int r, int col) { return st.B[(r >> 1) * kL128Pair + (r & 1) * 128 + col]; };
  // half-wave h takes k = 8u + 4h + q in MFMA q of super-step u; the next
  // super-step's fragments are read while the current MFMAs run
  auto compute = [&](const Lds128Stage& src) {
    f32x4 av[2][2];
    float bv[2][2][4];
    auto frag = [&](int u, int r) {
#pragma unroll
      for (int b = 0; b < 2; ++b)
        av[r][b] = __builtin_bit_cast(f32x4, src.A[lds_a_slot(wm0 + 32 * b + lr, 2 * u + lh)]);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 2; ++c) bv[r][c][q] = brow(src, 8 * u + 4 * lh + q, wn0 + 32 * c + lr);
    };
    frag(0, 0);
#pragma unroll
    for (int u = 0; u < BK / 8; ++u) {
      if (u + 1 < BK / 8) frag(u + 1, (u + 1) & 1);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int c = 0; c < 2; ++c)
            acc[b][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[u & 1][b][q], bv[u & 1][c][q], acc[b][c], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  };
  // this wave's quarter of the item's staging slot, [accumulator][lane]
  const __amdgpu_buffer_rsrc_t rs = f32_rsrc(g.stage + it * (128 * 128) + wave * (64 * 64), 64 * 64 * 4);
  const int vo = lane * 4;
  int folds = 0;
  // slot += acc (acc first) one accumulator block at a time, the next
  // block's slot values requested before the current one is added
  auto fold = [&]() {
    float nx[2][16];
    auto ld = [&](int q) {
#pragma unroll
      for (int v = 0; v < 16; ++v)
        nx[q & 1][v] = folds ? __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, vo, (q * 16 + v) * 256, 0))
                             : 0.0f;
    };
    ld(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {   // accumulator block q = 2 b + c
      if (q + 1 < 4) ld(q + 1);
      const int b = q / 2, c = q % 2;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        float x = acc[b][c][v];
        if (folds) x += nx[q & 1][v];
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), rs, vo, (q * 16 + v) * 256, 0);
      }
      acc[b][c] = f32x16{};
      __builtin_amdgcn_sched_barrier(0);
    }
    ++folds;
  };

  const int64_t nkt = (K + BK - 1) / BK;
  auto step = [&](int64_t kt, Lds128Stage& cur, Lds128Stage& nxt) {
    if (kt + 1 < nkt) {
      issue(kt + 1, nxt);
    } else if (K & 3) {
      // the inner extent ends inside a chunk: clear the A entries past K of
      // that chunk in every row (B rows past K already read zero)
      const int kz = (int)(K - kt * BK), cs = kz >> 2, e0 = kz & 3;
      if (tid < 128) {
        float* q = reinterpret_cast<float*>(&cur.A[lds_a_slot(tid, cs)]);
        for (int e = e0; e < 4; ++e) q[e] = 0.0f;
      }
      __syncthreads();
    }
    compute(cur);
    if ((kt + 1) % FOLD_STEPS == 0 && kt + 1 < nkt) fold();
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };
  if (nkt > 0) issue(0, st0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  for (int64_t kt = 0; kt < nkt; kt += 2) {
    step(kt, st0, st1);
    if (kt + 1 < nkt) step(kt + 1, st1, st0);
  }

  double e2 = 0.0, n2 = 0.0;
  store_block_with_error<2, 2>(
      acc, [=](int b, int v) { return m0 + wm0 + 4 * lh + 32 * b + 8 * (v >> 2) + (v & 3); },
      [=](int c) { return n0 + wn0 + lr + 32 * c; }, reinterpret_cast<float*>(g.C), g.ldc,
      reinterpret_cast<const float*>(g.Y), g.ldy, g.m, g.p, e2, n2, folds > 0, [&](int b, int c, int v) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, vo, ((b * 2 + c) * 16 + v) * 256, 0));
      });
  if (g.tile_part) {
    // the four waves' sums added in wave order
    e2 = warp_sum_f64(e2);
    n2 = warp_sum_f64(n2);
    if (lane == 0) {
      red[0][wave] = e2;
      red[1][wave] = n2;
    }
    __syncthreads();
    if (tid == 0) {
      const int64_t part = ga.part_base[pi] + local;
      g.tile_part[part] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
      g.tile_part[ga.nparts + part] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    }
  }
}

// Per problem t: out[2t] = sum of the error partials of its sketched tiles,
// out[2t+1] = sum of the squared-norm partials of its exact tiles (one
// workgroup per problem, fixed order); L[t] = *col_end[t].
__global__ __launch_bounds__(kThreads) void grouped_reduce_kernel(
    const double* __restrict__ sk_part, int64_t sk_nparts, const int64_t* __restrict__ sk_base,
    const double* __restrict__ ex_part, int64_t ex_nparts, const int64_t* __restrict__ ex_base,
    const int64_t* const* __restrict__ col_end, double* __restrict__ out, int64_t* __restrict__ L) {
  __shared__ double sm[2][kThreads];
  const int t = blockIdx.x;
  double e2 = 0.0, n2 = 0.0;
  for (int64_t i = sk_base[t] + threadIdx.x; i < sk_base[t + 1]; i += kThreads) e2 += sk_part[i];
  for (int64_t i = ex_base[t] + threadIdx.x; i < ex_base[t + 1]; i += kThreads) n2 += ex_part[ex_nparts + i];
  sm[0][threadIdx.x] = e2;
  sm[1][threadIdx.x] = n2;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sm[0][threadIdx.x] += sm[0][threadIdx.x + o];
      sm[1][threadIdx.x] += sm[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * t] = sm[0][0];
    out[2 * t + 1] = sm[1][0];
    if (L) L[t] = *col_end[t];
  }
  (void)sk_nparts;
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

void tile_shape(sbmm_dtype dt, bool blocknorm, int64_t* bm, int64_t* bn) {
  if (dt == SBMM_F64) { *bm = 32 * F64_WMB; *bn = 32 * F64_WNB; return; }
  if (dt == SBMM_BF16) { hgemm_tile_shape(bm, bn); return; }
  if (blocknorm) { *bm = 64 * F32B_WMB; *bn = 64 * F32B_WNB; return; }
  *bm = 64 * F32_WMB; *bn = 64 * F32_WNB;
}

}  // namespace

namespace {
// The LDS-direct float32 kernel needs 16-byte aligned rows (A and B aligned
// with leading dimensions of whole 16-byte chunks; any p and inner extent)
// and 32-bit panel offsets.
bool sgemm_lds_ok(const GemmLaunch& L, const GemmArgs& g) {
  if (!g.vec_a || !g.vec_b || L.stage == nullptr) return false;
  const int64_t kmax = L.K_dev ? L.lda : L.K_host;
  const int64_t lim = (int64_t)1 << 31;
  return 257 * L.lda * 4 + kmax * 4 < lim && 33 * L.ldb * 4 < lim;
}
}  // namespace

int64_t gemm_tiles(sbmm_dtype dt, int64_t m, int64_t p, bool blocknorm) {
  int64_t bm, bn;
  tile_shape(dt, blocknorm, &bm, &bn);
  return ceil_div(m, bm) * ceil_div(p, bn);
}

hipError_t launch_gemm(const GemmLaunch& L, hipStream_t s) {
  if (L.dt == SBMM_BF16) return launch_hgemm(L, s);
  const bool blocknorm = L.blk_part != nullptr;
  int64_t bm, bn;
  tile_shape(L.dt, blocknorm, &bm, &bn);
  const GemmArgs g = make_gemm_args(L, bm, bn);
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
    if (blocknorm) {
      hipLaunchKernelGGL((gemm_f32_kernel<F32B_WMB, F32B_WNB, true>), grid, block, 0, s, g);
    } else if (sgemm_lds_ok(L, g)) {
      // 256 x 256 tiles over the same 128 x 128 accounting
      const GemmArgs g2 = make_gemm_args(L, SgemmLdsTile::BM, SgemmLdsTile::BN);
      hipLaunchKernelGGL(sgemm_lds_kernel<kLdsWaves>, dim3((unsigned)(g2.tiles_m * g2.tiles_n)), dim3(kLdsWaves * 64), 0,
                         s, g2);
    } else {
      hipLaunchKernelGGL((sgemm_kernel<F32_WMB, F32_WNB, F32_BK, F32_WGS>), grid, block, 0, s, g);
    }
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Grouped float32 products: tile configurations the tuner chooses from.
// ----------------------------------------------------------------------------
namespace {
struct GroupedCfg { int bm, bn, wg_per_cu; };
// 0..3: the register-staged kernel; 4: 256 x 256 and 5: 128 x 128 tiles with
// LDS-direct loads (no fused gather, 16-byte aligned rows)
constexpr GroupedCfg kGroupedCfgs[] = {{128, 128, 2}, {64, 128, 2}, {128, 64, 2}, {64, 64, 4}, {256, 256, 1},
                                       {128, 128, 2}};
constexpr int kGroupedCfgCount = sizeof(kGroupedCfgs) / sizeof(kGroupedCfgs[0]);

template <bool GATHER>
void launch_grouped_cfg(int cfg, dim3 grid, const GroupedArgs& ga, hipStream_t s) {
  const dim3 block(kThreads);
  switch (cfg) {
    case 0: hipLaunchKernelGGL((sgemm_grouped_kernel<2, 2, F32_BK, 2, GATHER>), grid, block, 0, s, ga); break;
    case 1: hipLaunchKernelGGL((sgemm_grouped_kernel<1, 2, F32_BK, 2, GATHER>), grid, block, 0, s, ga); break;
    case 2: hipLaunchKernelGGL((sgemm_grouped_kernel<2, 1, F32_BK, 2, GATHER>), grid, block, 0, s, ga); break;
    case 3: hipLaunchKernelGGL((sgemm_grouped_kernel<1, 1, F32_BK, 4, GATHER>), grid, block, 0, s, ga); break;
    case 4:
      if constexpr (!GATHER)
        hipLaunchKernelGGL(sgemm_grouped_lds_kernel<kLdsWaves>, grid, dim3(kLdsWaves * 64), 0, s, ga);
      break;
    default:
      if constexpr (!GATHER) hipLaunchKernelGGL(sgemm_grouped_lds128_kernel, grid, dim3(256), 0, s, ga);
      break;
  }
}
}  // namespace

int grouped_cfg_count() { return kGroupedCfgCount; }

void grouped_cfg_shape(int cfg, int64_t* bm, int64_t* bn, int* wg_per_cu) {
  const GroupedCfg& c = kGroupedCfgs[cfg < 0 || cfg >= kGroupedCfgCount ? 0 : cfg];
  *bm = c.bm; *bn = c.bn; *wg_per_cu = c.wg_per_cu;
}

size_t grouped_gemm_args_bytes() { return sizeof(GemmArgs); }

void build_grouped_gemm_args(const GemmLaunch& L, int cfg, void* out) {
  int64_t bm, bn;
  int w;
  grouped_cfg_shape(cfg, &bm, &bn, &w);
  const GemmArgs g = make_gemm_args(L, bm, bn);
  std::memcpy(out, &g, sizeof(g));
}

bool grouped_lds_ok(const GemmLaunch& L) {
  const GemmArgs g = make_gemm_args(L, SgemmLdsTile::BM, SgemmLdsTile::BN);
  GemmLaunch S = L;
  S.stage = reinterpret_cast<float*>(256);   // presence only
  return sgemm_lds_ok(S, g);
}

hipError_t launch_grouped_gemm(const GroupedLaunch& L, hipStream_t s) {
  if (L.items <= 0) return hipSuccess;
  if (L.stage == nullptr) return hipErrorInvalidValue;
  if (L.gather && L.cfg >= 4) return hipErrorInvalidValue;   // no fused gather on the LDS-direct tiles
  GroupedArgs ga{reinterpret_cast<const GemmArgs*>(L.probs), L.item_prob, L.item_tile, L.part_base,
                 L.items, L.nparts};
  const dim3 grid((unsigned)L.items);
  if (L.gather) launch_grouped_cfg<true>(L.cfg, grid, ga, s);
  else launch_grouped_cfg<false>(L.cfg, grid, ga, s);
  return hipGetLastError();
}

hipError_t launch_grouped_reduce(const double* sk_part, int64_t sk_nparts, const int64_t* sk_base,
                                 const double* ex_part, int64_t ex_nparts, const int64_t* ex_base,
                                 const int64_t* const* col_end, int32_t count, double* out, int64_t* L,
                                 hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(grouped_reduce_kernel, dim3((unsigned)count), dim3(kThreads), 0, s, sk_part, sk_nparts,
                     sk_base, ex_part, ex_nparts, ex_base, col_end, out, L);
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
