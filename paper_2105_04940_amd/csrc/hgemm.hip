// bf16 matrix-core product (sketched product of a bf16 sketch, and the two
// products of the backward, which take one operand transposed). The tile
// order, argument block and error epilogue are those of the float32 product.
#include "gemm_common.h"

namespace {

using namespace gemm_detail;

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
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef short i16x8 __attribute__((ext_vector_type(8)));

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
// "TN" form: A is M x K and B is N x K, both row-major with the inner index
// contiguous (every bf16 product of the path is brought to this form). A
// workgroup owns a 256 x 256 tile; each of its four waves a 128 x 128 quarter
// as 4 x 4 blocks of v_mfma_f32_32x32x16_bf16, so every 16-byte fragment read
// from LDS feeds four matrix instructions. One k-step is 64 wide: 32 KB of A
// and 32 KB of B, double-buffered (128 KB of LDS, one workgroup per CU),
// loaded as 16-byte chunks (8 consecutive k) whose position within their
// 128-byte LDS row is XOR-swizzled by the row index (chunk c of row r at
// c ^ (r & 7)): the 8 lanes of each read phase then hit 8 different chunk
// positions, and rows need no padding.
// ============================================================================
struct TnTile {
  static constexpr int BM = 256, BN = 256, BK = 64, KC = BK / 8;
  static constexpr int NL = BM * KC / kThreads;     // 16-byte chunks of A (and of B) per thread
  uint4 As[2][BM * KC];
  uint4 Bs[2][BN * KC];
  double red[8];
};

__device__ __forceinline__ int tn_slot(int row, int chunk) { return row * TnTile::KC + (chunk ^ (row & 7)); }

template <bool EDGE>
__device__ __forceinline__ void hgemm_tn_body(const GemmArgs& g, TnTile& sh, int64_t m0, int64_t n0, int64_t K) {
  constexpr int BK = TnTile::BK, KC = TnTile::KC, NL = TnTile::NL;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 31, lh = lane >> 5;
  const int wm0 = (wave & 1) * 128, wn0 = (wave >> 1) * 128;
  const uint16_t* __restrict__ A = reinterpret_cast<const uint16_t*>(g.A);
  const uint16_t* __restrict__ B = reinterpret_cast<const uint16_t*>(g.B);

  f32x16 acc[4][4];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[b][c] = f32x16{};

  // chunk f = tid + 256 q of a tile: row f / 8, k-chunk f % 8
  uint4 ra[NL], rb[NL];
  // interior tiles: whole 16-byte chunks, zero past K (K is a multiple of 8)
  auto load_one = [&](const uint16_t* X, int64_t ld, int64_t r, int64_t rmax, int64_t k, bool vec) -> uint4 {
    if (!EDGE) return k < K ? *reinterpret_cast<const uint4*>(X + r * ld + k) : make_uint4(0, 0, 0, 0);
    if (r < rmax && k + 8 <= K && vec) return *reinterpret_cast<const uint4*>(X + r * ld + k);
    uint16_t t[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) t[e] = (r < rmax && k + e < K) ? X[r * ld + k + e] : 0;
    return make_uint4(t[0] | (uint32_t)t[1] << 16, t[2] | (uint32_t)t[3] << 16, t[4] | (uint32_t)t[5] << 16,
                      t[6] | (uint32_t)t[7] << 16);
  };
  auto load = [&](int64_t kt) {
    const int64_t k0 = kt * BK;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int f = tid + kThreads * q;
      ra[q] = load_one(A, g.lda, m0 + f / KC, g.m, k0 + 8 * (f % KC), g.vec_a);
      rb[q] = load_one(B, g.ldb, n0 + f / KC, g.p, k0 + 8 * (f % KC), g.vec_b);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int f = tid + kThreads * q;
      sh.As[buf][tn_slot(f / KC, f % KC)] = ra[q];
      sh.Bs[buf][tn_slot(f / KC, f % KC)] = rb[q];
    }
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int s = 0; s < BK / 16; ++s) {
      bf16x8 av[4], bv[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint4 v = sh.As[buf][tn_slot(wm0 + 32 * b + lr, 2 * s + lh)];
        av[b] = __builtin_bit_cast(bf16x8, v);
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint4 v = sh.Bs[buf][tn_slot(wn0 + 32 * c + lr, 2 * s + lh)];
        bv[c] = __builtin_bit_cast(bf16x8, v);
      }
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[b][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[b], bv[c], acc[b][c], 0, 0, 0);
    }
  };

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
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t row = m0 + wm0 + 32 * b + 8 * (v >> 2) + 4 * lh + (v & 3);
      if (EDGE && row >= g.m) continue;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t col = n0 + wn0 + 32 * c + lr;
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

__global__ __launch_bounds__(kThreads, 1) void hgemm_tn_kernel(GemmArgs g) {
  __shared__ TnTile sh;
  int64_t tm, tn;
  tile_coords(g, tm, tn);
  const int64_t m0 = tm * TnTile::BM, n0 = tn * TnTile::BN;
  const int64_t K = inner_extent(g);
  const bool interior = g.vec_a && g.vec_b && m0 + TnTile::BM <= g.m && n0 + TnTile::BN <= g.p && K % 8 == 0;
  if (interior)
    hgemm_tn_body<false>(g, sh, m0, n0, K);
  else
    hgemm_tn_body<true>(g, sh, m0, n0, K);
}


// ============================================================================
// The same 256 x 256 product with the operand tiles fetched straight into LDS
// (buffer_load_dwordx4 ... lds): no staging registers and no LDS store phase,
// so the 256 accumulator registers of a wave leave room for the fragments
// without spilling. A wave instruction fills 64 consecutive 16-byte LDS
// slots, lane l at slot base + l; slot P of a tile is (row P / 8, swizzled
// chunk P % 8), so lane l fetches chunk (l & 7) ^ (l >> 3) of row
// 64 w + 8 j + l / 8 for instruction j of wave w. Row offsets live in one
// register per operand (the instruction's row step added per load, so the
// hardware range check, which covers the vector offset, sees every row) and
// the k-step in the scalar offset. Rows past the operand's end fall outside
// the buffer's record count and chunks past the inner extent get an
// out-of-range offset: both read as zero, so edge tiles need no separate
// path, and a live chunk of a valid row never reads past that row's first K
// elements. The k-step loop (below, at the kernel's main loop) overlaps the
// loads of later steps, the step barrier and the fragment reads with the
// matrix instructions.
// ============================================================================
template <int BK_, int SA_, int SB_>
struct TnLdsTile {
  static constexpr int BM = 256, BN = 256, BK = BK_, KC = BK / 8, SA = SA_, SB = SB_;
  uint4 As[SA][BM * KC];   // after the main loop, the first stage holds the error partials
  uint4 Bs[SB][BN * KC];
};

// LDS slot of 16-byte chunk `chunk` of tile row `row`: a row holds KC chunks
// and the chunk index is XORed with a row-dependent value chosen so that the
// 16 consecutive rows a 16-lane group of ds_read_b128 reads (same chunk) fall
// in 16 different 16-byte bank groups.
template <int KC>
__device__ __forceinline__ int tn_lds_slot(int row, int chunk) {
  if constexpr (KC == 8) return row * 8 + (chunk ^ ((row >> 1) & 7));
  else return row * 4 + (chunk ^ ((row >> 2) & 3));
}

// NW waves per workgroup: 4 (one per SIMD, 128 x 128 each) or 8 (two per
// SIMD, 128 x 64 each). EPI: SC_NONE stores the float32 product (and the
// error partials); SC_COLS / SC_ROWS scatter the weighted product into the
// columns / rows of another matrix (the backward's dM, dN).
//
// BKN: B is given as K x p rows (the sketch's D as gathered) instead of p x K.
// A k-step's B tile is then its 64 k-rows of 256 columns (512 bytes each, two
// rows per wave instruction: lane l fills slot 32 (l >> 5) + (l & 31) of the
// instruction's pair of rows), chunk c of row r at slot c ^ 4 (r & 3). The
// matrix instruction wants, in lane l, the 8 k-values of column l & 31 at k
// 8 (l >> 5) .. + 7: two transposing LDS reads (ds_read_b64_tr_b16) give
// them. In such a read lane i of each 16-lane group names 8 bytes (4 columns)
// of one row and receives the element of its own column from the 4 rows the
// group named (a one-wave probe of the instruction: element e of lane i
// comes from the 8 bytes lane 4 e + (i >> 2) named, position i & 3), so the
// group names rows k0 + (i >> 2), columns n0 + 4 (i & 3). The four rows of a
// group differ in r & 3, so the swizzle spreads their 32-byte pieces over
// distinct banks.
template <int BK, int STAGES, int NW, int EPI, bool BKN = false>
__global__ __launch_bounds__(NW * 64, 1) void hgemm_tn_lds_kernel(GemmArgs g) {
  static_assert(STAGES == 2, "a ring of two stages");
  static_assert(!BKN || (BK == 64 && NW == 8), "the k-row B form: k-step 64, 8 waves");
  // the k-row B form keeps A in a ring of three stages (A tiles two steps
  // ahead) beside B in a ring of two: 96 + 64 KB, all of LDS
  constexpr int SA = BKN ? 3 : 2, SB = 2;
  using Tile = TnLdsTile<BK, SA, SB>;
  constexpr int KC = Tile::KC;
  constexpr int CB = 16 / NW;                          // 32-column blocks per wave
  constexpr int ROWS_PER_INST = 64 / KC;               // tile rows one wave instruction fills
  constexpr int INSTS = Tile::BM / ROWS_PER_INST / NW; // instructions per wave per operand and stage
  __shared__ Tile sh;
  int64_t tm, tn;
  tile_coords(g, tm, tn);
  const int64_t m0 = tm * Tile::BM, n0 = tn * Tile::BN;
  // output extents: the grid covers m x p, the live part may be smaller
  // (read on the device); a tile past it leaves before any barrier
  if (g.m_dev) g.m = min(g.m, *g.m_dev);
  if (g.p_dev) g.p = min(g.p, *g.p_dev);
  if (m0 >= g.m || n0 >= g.p) return;
  const int64_t K = inner_extent(g);
  const int tid = threadIdx.x, lane = tid & 63;
  // uniform across the wave: the LDS destination of a load is a scalar
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 31, lh = lane >> 5;
  const int wm0 = (wave & 1) * 128, wn0 = (wave >> 1) * 32 * CB;
  const uint16_t* A = reinterpret_cast<const uint16_t*>(g.A) + m0 * g.lda;
  // BKN: B's columns from n0 on, to the end of its K rows (rows at or past K
  // read as zero, as do chunks at or past column p)
  const uint16_t* B = reinterpret_cast<const uint16_t*>(g.B) + (BKN ? n0 : n0 * g.ldb);
  const i32x4 ra = buffer_words(A, (int)(min((int64_t)Tile::BM, g.m - m0) * g.lda * 2));
  const i32x4 rb = buffer_words(B, BKN ? (int)((K * g.ldb - n0) * 2)
                                       : (int)(min((int64_t)Tile::BN, g.p - n0) * g.ldb * 2));
  constexpr unsigned kOut = 0x80000000u;   // past any record count

  f32x16 acc[4][CB];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[b][c] = f32x16{};

  // instruction j of wave w fills slots [(INSTS w + j) 64, +64): lane l holds
  // slot P = (INSTS w + j) 64 + l, i.e. tile row P / KC and the chunk whose
  // swizzled slot is P % KC
  // A's tile of step kt into A stage buf (and, in the p x K form, B's into B
  // stage buf: the same rows and chunks)
  auto issue_a = [&](int64_t kt, int buf) {
    const int64_t k0 = kt * BK;
    const unsigned sk = (unsigned)(k0 * 2);
#pragma unroll
    for (int j = 0; j < INSTS; ++j) {
      const int row = (INSTS * wave + j) * ROWS_PER_INST + lane / KC;
      const int slot = lane % KC;
      const int chunk = KC == 8 ? (slot ^ ((row >> 1) & 7)) : (slot ^ ((row >> 2) & 3));
      const bool live = k0 + 8 * chunk < K;   // the inner tail reads zero
      const unsigned oa = live ? (unsigned)(row * g.lda * 2 + chunk * 16) : kOut;
      const unsigned ob = live ? (unsigned)(row * g.ldb * 2 + chunk * 16) : kOut;
      lds_dma16(ra, lds_offset(&sh.As[buf][(INSTS * wave + j) * 64]), oa, sk);
      if constexpr (!BKN) lds_dma16(rb, lds_offset(&sh.Bs[buf][(INSTS * wave + j) * 64]), ob, sk);
    }
  };
  // BKN: B's tile of step kt (its 64 k-rows) into B stage buf. The byte
  // stride of a k-step is made scalar here, once: computed next to the loads
  // from the vector copy of ldb the compiler keeps for the lane offsets, it
  // came back through a readfirstlane right before a load (the load's
  // soffset then needs five wait states)
  const unsigned kstep_b = __builtin_amdgcn_readfirstlane((unsigned)(BK * g.ldb * 2));
  auto issue_b = [&](int64_t kt, int buf) {
    if constexpr (BKN) {
      constexpr int BINSTS = BK / 2 / NW;   // two k-rows per instruction
      const unsigned skb = (unsigned)kt * kstep_b;
#pragma unroll
      for (int j = 0; j < BINSTS; ++j) {
        const int r = 2 * (BINSTS * wave + j) + (lane >> 5);
        const int c = (lane & 31) ^ (4 * (r & 3));
        const unsigned ob = n0 + 8 * c < g.p ? (unsigned)(r * g.ldb * 2 + c * 16) : kOut;
        lds_dma16(rb, lds_offset(&sh.Bs[buf][(BINSTS * wave + j) * 64]), ob, skb);
      }
    }
  };
  // BKN: byte offset in a B stage of this lane's first transposing read for
  // column block c (k-row 8 (l >> 5) + ((l & 15) >> 2), column wn0 + 32 c +
  // 16 ((l >> 4) & 1) + 4 (l & 3)); other sub-steps (16 rows on) and the
  // second read (4 rows on) keep r & 3, so they add constants
  int bkn_off[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    const int i = lane & 15, G = lane >> 4;
    const int r = 8 * (G >> 1) + (i >> 2);
    const int n = wn0 + 32 * c + 16 * (G & 1) + 4 * (i & 3);
    bkn_off[c] = r * 512 + (((n >> 3) ^ (4 * (r & 3))) << 4) + ((n >> 2) & 1) * 8;
  }
  auto b_frag = [&](int buf, int s, int c) -> bf16x8 {
    if constexpr (BKN) {
      const char* base = reinterpret_cast<const char*>(&sh.Bs[buf][0]) + bkn_off[c] + 16 * s * 512;
      const i16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
          (__attribute__((address_space(3))) i16x4*)(base));
      const i16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
          (__attribute__((address_space(3))) i16x4*)(base + 4 * 512));
      const i16x8 v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
      return __builtin_bit_cast(bf16x8, v);
    } else {
      return __builtin_bit_cast(bf16x8, sh.Bs[buf][tn_lds_slot<KC>(wn0 + 32 * c + lr, 2 * s + lh)]);
    }
  };
  auto frags = [&](int sa, int sb, int s, bf16x8 (&av)[4], bf16x8 (&bv)[CB]) {
#pragma unroll
    for (int b = 0; b < 4; ++b)
      av[b] = __builtin_bit_cast(bf16x8, sh.As[sa][tn_lds_slot<KC>(wm0 + 32 * b + lr, 2 * s + lh)]);
#pragma unroll
    for (int c = 0; c < CB; ++c) bv[c] = b_frag(sb, s, c);
  };
  // The fragments of sub-step s + 1 are read while the matrix instructions
  // of sub-step s run (one LDS read between two matrix instructions, an
  // order the scheduling-group barriers impose: left alone, the compiler
  // issues each sub-step's reads just before their use and waits on them).
  // Fragment sets alternate by sub-step; four sub-steps a step, so sub-step 0
  // of every step uses set 0.
  constexpr int READS = 4 + (BKN ? 2 : 1) * CB;   // LDS read instructions per sub-step
  constexpr int NS = BK / 16;
  static_assert(NS % 2 == 0, "sub-step 0 of every step in fragment set 0");
  bf16x8 av[2][4], bv[2][CB];
  auto mfmas = [&](int set) {
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int c = 0; c < CB; ++c)
        acc[b][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[set][b], bv[set][c], acc[b][c], 0, 0, 0);
  };
  auto interleave = [&]() {
#pragma unroll
    for (int i = 0; i < 4 * CB; ++i) {
      if (i < READS) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
  };

  // Step kt reads A stage kt % SA and B stage kt % 2. A step runs sub-steps
  // 0 .. NS - 2, each reading the next sub-step's fragments; then every wave
  // waits for its own LDS reads and for step kt + 1's tiles, and barriers:
  // step kt + 1's stages are complete and no wave reads step kt's any more,
  // so the tiles of the steps that take them over are issued there. The
  // last sub-step's matrix instructions then run while the first fragments
  // of step kt + 1 are read, so the barrier and that first read overlap
  // matrix work instead of following it. Two A stages: step kt + 2's tiles,
  // one step ahead. Three A stages: B of step kt + 2, then A of step kt + 3,
  // two steps ahead (in the 8 x 4 tile block of an XCD every A panel is
  // shared by 4 tiles and every B panel by 8, so A misses the L2 twice as
  // often; timing-only copies of the kernel ran 9 % faster with A's loads
  // all hitting L2, 3 % with B's). Loads complete in issue order, so at the
  // barrier of step kt the newest A tile (step kt + 2) may still be in
  // flight while everything older has landed.
  const int64_t nkt = (K + BK - 1) / BK;
  constexpr int AINSTS = INSTS;   // load instructions per wave in one A tile
  static_assert(!BKN || BK / 2 / NW == INSTS, "A and B tiles take the same number of loads");
  auto body = [&](int64_t kt, int sa, int sb) {
#pragma unroll
    for (int s = 0; s + 1 < NS; ++s) {
      frags(sa, sb, s + 1, av[(s + 1) & 1], bv[(s + 1) & 1]);
      mfmas(s & 1);
      interleave();
    }
    // (after the last step the barrier is uniform and the reads of the
    // next stages, in bounds, go unused: one path for every step)
    if constexpr (SA == 3) {
      if (kt + 2 < nkt) wait_loads_reads_barrier<AINSTS>();
      else wait_loads_reads_barrier<0>();
      if (kt + 2 < nkt) issue_b(kt + 2, sb);
      if (kt + 3 < nkt) issue_a(kt + 3, sa);
    } else {
      wait_loads_reads_barrier<0>();
      if (kt + 2 < nkt) {
        issue_a(kt + 2, sa);
        issue_b(kt + 2, sb);
      }
    }
    frags(sa + 1 < SA ? sa + 1 : 0, sb ^ 1, 0, av[0], bv[0]);
    mfmas(1);
    interleave();
  };
  if (nkt > 0) {
    issue_a(0, 0);
    issue_b(0, 0);
    if (nkt > 1) {
      issue_a(1, 1);
      issue_b(1, 1);
    }
    if constexpr (SA == 3) {
      if (nkt > 2) issue_a(2, 2);
      // step 0's tiles landed; those issued after them may still be in flight
      if (nkt > 2) wait_loads_barrier<3 * AINSTS>();
      else if (nkt > 1) wait_loads_barrier<2 * AINSTS>();
      else wait_loads_barrier<0>();
    } else {
      if (nkt > 1) wait_loads_barrier<2 * AINSTS>();
      else wait_loads_barrier<0>();
    }
    frags(0, 0, 0, av[0], bv[0]);
    __builtin_amdgcn_sched_barrier(0);
  }
  if constexpr (SA == 3) {
    for (int64_t kt = 0; kt < nkt; kt += 6) {
      body(kt, 0, 0);
      if (kt + 1 < nkt) body(kt + 1, 1, 1);
      if (kt + 2 < nkt) body(kt + 2, 2, 0);
      if (kt + 3 < nkt) body(kt + 3, 0, 1);
      if (kt + 4 < nkt) body(kt + 4, 1, 0);
      if (kt + 5 < nkt) body(kt + 5, 2, 1);
    }
  } else {
    for (int64_t kt = 0; kt < nkt; kt += 2) {
      body(kt, 0, 0);
      if (kt + 1 < nkt) body(kt + 1, 1, 1);
    }
  }

  if constexpr (EPI != SC_NONE) {
    // weighted scatter: consecutive lanes hold consecutive columns, so a
    // store instruction writes 32-element runs wherever the map is contiguous
    uint16_t* __restrict__ o16 = reinterpret_cast<uint16_t*>(g.sc_out);
    float* __restrict__ o32 = reinterpret_cast<float*>(g.sc_out);
    int64_t cdst[CB];
    double cw[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int64_t col = n0 + wn0 + 32 * c + lr;
      const bool ok = col < g.p;
      cdst[c] = EPI == SC_COLS ? (ok ? (int64_t)g.sc_map[col] : -1) : col;
      cw[c] = (EPI == SC_COLS && ok) ? g.sc_w[col] : 0.0;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = m0 + wm0 + 32 * b + 8 * (v >> 2) + 4 * lh + (v & 3);
        if (row >= g.m) continue;
        int64_t rdst = row;
        double rw = 1.0;
        if constexpr (EPI == SC_ROWS) {
          rdst = g.sc_map[row];
          rw = g.sc_w[row];
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          const int64_t col = n0 + wn0 + 32 * c + lr;
          if (col >= g.p) continue;
          const double w = EPI == SC_COLS ? cw[c] : rw;
          const float val = (float)(w * (double)acc[b][c][v]);
          const int64_t e = rdst * g.sc_ld + cdst[c];
          if (g.sc_f32) o32[e] = val;
          else o16[e] = float_to_bf16_bits(val);
        }
        if ((v & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    return;
  }
  double e2 = 0.0, n2 = 0.0;
  store_tile_with_error<CB>(acc, reinterpret_cast<float*>(g.C), g.ldc, reinterpret_cast<const float*>(g.Y), g.ldy,
                            g.m, g.p, m0 + wm0 + 4 * lh, n0 + wn0 + lr, e2, n2);
  if (g.tile_part) {
    // NW waves' sums added in wave order, through the first A stage once
    // every wave is past its last LDS read (no tile load is in flight: the
    // last step's barrier waited for all of them)
    double* red = reinterpret_cast<double*>(&sh.As[0][0]);
    e2 = warp_sum_f64(e2);
    n2 = warp_sum_f64(n2);
    __syncthreads();
    if (lane == 0) {
      red[wave] = e2;
      red[NW + wave] = n2;
    }
    __syncthreads();
    if (tid == 0) {
      double a = 0.0, b = 0.0;
      for (int w = 0; w < NW; ++w) {
        a += red[w];
        b += red[NW + w];
      }
      g.tile_part[blockIdx.x] = a;
      g.tile_part[g.tiles_m * g.tiles_n + blockIdx.x] = b;
    }
  }
}

constexpr int TN_BK = 64, TN_STAGES = 2, TN_WAVES = 8;

constexpr int BF16_WMB = 2, BF16_WNB = 2, BF16_BK = 64, BF16_WGS = 2;   // 128 x 128

}  // namespace

void hgemm_tile_shape(int64_t* bm, int64_t* bn) { *bm = 64 * BF16_WMB; *bn = 64 * BF16_WNB; }

void hgemm_tn_tile_shape(int64_t* bm, int64_t* bn) { *bm = TnTile::BM; *bn = TnTile::BN; }

int64_t gemm_tiles_tn(int64_t m, int64_t p) { return ceil_div(m, TnTile::BM) * ceil_div(p, TnTile::BN); }

bool hgemm_kn_ok(const GemmLaunch& L);

int64_t hgemm_tiles(const GemmLaunch& L) {
  int64_t bm, bn;
  if (hgemm_kn_ok(L) || (L.b_trans && !L.a_trans)) hgemm_tn_tile_shape(&bm, &bn);
  else hgemm_tile_shape(&bm, &bn);
  return ceil_div(L.m, bm) * ceil_div(L.p, bn);
}

bool hgemm_kn_ok(const GemmLaunch& L) {
  const int64_t K_max = L.K_dev ? L.K_max : L.K_host;
  const bool rows16 = (uintptr_t)L.A % 16 == 0 && (L.lda * 2) % 16 == 0 && (uintptr_t)L.B % 16 == 0 &&
                      (L.ldb * 2) % 16 == 0;
  // whole 8-element chunks of A along k (a device extent is a multiple of
  // 32), 32-bit offsets over A's 256-row panels and all of B's rows
  const bool chunks = L.K_dev != nullptr || L.K_host % 8 == 0;
  const bool fits = 257 * L.lda * 2 < ((int64_t)1 << 31) && (K_max + 1) * L.ldb * 2 < ((int64_t)1 << 31);
  return L.dt == SBMM_BF16 && !L.a_trans && !L.b_trans && L.sc_mode == SC_NONE && !L.m_dev && !L.p_dev &&
         K_max > 0 && rows16 && chunks && fits;
}

hipError_t launch_hgemm(const GemmLaunch& L, hipStream_t s) {
  int64_t bm, bn;
  if (hgemm_kn_ok(L)) {
    // B as K x p rows: the 256 x 256 kernel with transposing reads of B
    hgemm_tn_tile_shape(&bm, &bn);
    const GemmArgs g = make_gemm_args(L, bm, bn);
    const int64_t tiles = g.tiles_m * g.tiles_n;
    if (tiles == 0) return hipSuccess;
    hipLaunchKernelGGL((hgemm_tn_lds_kernel<TN_BK, TN_STAGES, TN_WAVES, SC_NONE, true>), dim3((unsigned)tiles),
                       dim3(TN_WAVES * 64), 0, s, g);
    return hipGetLastError();
  }
  if (L.b_trans && !L.a_trans) {
    // both operands inner-index contiguous: the 256 x 256 kernels
    hgemm_tn_tile_shape(&bm, &bn);
    const GemmArgs g = make_gemm_args(L, bm, bn);
    const int64_t tiles = g.tiles_m * g.tiles_n;
    if (tiles == 0) return hipSuccess;
    // LDS-direct loads need whole aligned 16-byte chunks (an inner extent
    // read on the device is a multiple of 32) and 32-bit panel offsets
    const int64_t ld = std::max(L.lda, L.ldb);
    const bool fits = 257 * ld * 2 < ((int64_t)1 << 31);
    const bool chunks = L.K_dev != nullptr || L.K_host % 8 == 0;
    const bool lds = g.vec_a && g.vec_b && fits && chunks;
    if (L.sc_mode != SC_NONE || L.m_dev || L.p_dev) {
      // the scatter epilogue and device extents exist on the LDS-direct kernel only
      if (!lds) return hipErrorInvalidValue;
      if (L.sc_mode == SC_COLS)
        hipLaunchKernelGGL((hgemm_tn_lds_kernel<TN_BK, TN_STAGES, TN_WAVES, SC_COLS>), dim3((unsigned)tiles),
                           dim3(TN_WAVES * 64), 0, s, g);
      else if (L.sc_mode == SC_ROWS)
        hipLaunchKernelGGL((hgemm_tn_lds_kernel<TN_BK, TN_STAGES, TN_WAVES, SC_ROWS>), dim3((unsigned)tiles),
                           dim3(TN_WAVES * 64), 0, s, g);
      else
        hipLaunchKernelGGL((hgemm_tn_lds_kernel<TN_BK, TN_STAGES, TN_WAVES, SC_NONE>), dim3((unsigned)tiles),
                           dim3(TN_WAVES * 64), 0, s, g);
      return hipGetLastError();
    }
    if (lds)
      hipLaunchKernelGGL((hgemm_tn_lds_kernel<TN_BK, TN_STAGES, TN_WAVES, SC_NONE>), dim3((unsigned)tiles),
                         dim3(TN_WAVES * 64), 0, s, g);
    else
      hipLaunchKernelGGL(hgemm_tn_kernel, dim3((unsigned)tiles), dim3(kThreads), 0, s, g);
    return hipGetLastError();
  }
  hgemm_tile_shape(&bm, &bn);
  const GemmArgs g = make_gemm_args(L, bm, bn);
  const int64_t tiles = g.tiles_m * g.tiles_n;
  if (tiles == 0) return hipSuccess;
  dim3 grid((unsigned)tiles), block(kThreads);
  if (L.a_trans && L.b_trans)
    hipLaunchKernelGGL((hgemm_kernel<BF16_WMB, BF16_WNB, BF16_BK, BF16_WGS, true, true>), grid, block, 0, s, g);
  else if (L.a_trans)
    hipLaunchKernelGGL((hgemm_kernel<BF16_WMB, BF16_WNB, BF16_BK, BF16_WGS, true, false>), grid, block, 0, s, g);
  else if (L.b_trans)
    hipLaunchKernelGGL((hgemm_kernel<BF16_WMB, BF16_WNB, BF16_BK, BF16_WGS, false, true>), grid, block, 0, s, g);
  else
    hipLaunchKernelGGL((hgemm_kernel<BF16_WMB, BF16_WNB, BF16_BK, BF16_WGS>), grid, block, 0, s, g);
  return hipGetLastError();
}
