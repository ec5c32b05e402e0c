// The sketch in 8-bit floating point with block scales (OCP MX E4M3) and
// its product on the block-scaled matrix instruction
// v_mfma_scale_f32_32x32x64_f8f6f4.
//
// Quantization (per row of C and per column of D, blocks of 32 consecutive
// sketch columns): the sketch value x = (float)(colscale[l] * M[i, colmap[l]])
// is formed as the float32 gather forms it; the block's shared exponent is
// X = floor(log2(amax)) - 8 (8 = largest E4M3 exponent; 0 for an all-zero
// block), stored as the E8M0 byte X + 127; each element is x / 2^X (exact),
// clamped to +-448 and rounded to nearest-even E4M3. D is written transposed
// (p x L_pad, sketch index contiguous), so both operands of the product have
// the inner index contiguous.
//
// Product: 256 x 256 tiles, four waves of 128 x 128 as 4 x 4 blocks of the
// 32x32x64 instruction; a k-step is 128 sketch columns (128 bytes per row,
// double-buffered in LDS with the XOR chunk swizzle of the bf16 kernel).
// Lane (r = lane % 32, h = lane / 32) of an instruction holds, for row r,
// two 16-byte pieces: inner indices 16h..16h+15 (bytes 0-15) and
// 32+16h..32+16h+15 (bytes 16-31), and the E8M0 scale of the 32-block
// 32h..32h+31 (so the scale of lane half h covers the first pieces of both
// halves, then the second pieces); this placement was measured with single-
// lane scale changes. Products of E4M3 values are exact in float32 and
// accumulate in float32.
#include "gemm_common.h"

namespace {

using namespace gemm_detail;

typedef int i32x8 __attribute__((ext_vector_type(8)));

constexpr int kBlk = 32;   // MX block

// E8M0 exponent byte and the scale-down factor of one block
__device__ __forceinline__ void mx_block_scale(float amax, uint8_t* ebyte, float* down) {
  int X = 0;
  if (amax > 0.0f) X = max(ilogbf(amax) - 8, -127);   // E8M0 holds 2^-127 .. 2^127
  *ebyte = (uint8_t)(X + 127);
  *down = ldexpf(1.0f, -X);
}

__device__ __forceinline__ uint32_t pack4_e4m3(float a, float b, float c, float d) {
  auto cl = [](float v) { return fminf(fmaxf(v, -448.0f), 448.0f); };
  uint32_t w = __builtin_amdgcn_cvt_pk_fp8_f32(cl(a), cl(b), 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(cl(c), cl(d), w, true);
  return w;
}

struct MxGatherArgs {
  const float* M; int64_t ldm;
  const float* N; int64_t ldn;
  int64_t m, p;
  const int64_t* L_dev;
  int64_t nblk_max;                 // L_pad_max / 32
  const int32_t* colmap; const double* colscale;
  uint8_t* C; int64_t ldc; uint8_t* Cs; int64_t ldcs;     // m x L_pad, m x L_pad/32
  uint8_t* Dt; int64_t lddt; uint8_t* Ds; int64_t ldds;   // p x L_pad, p x L_pad/32
  int64_t cchunks;                  // workgroups per row of C (64 blocks each)
  int64_t cgroups;                  // workgroups on the C part
};

constexpr int kMxCBlocksPerWave = 16;   // C part: blocks of one row per wave

// C part: workgroup (row i, chunk of 64 blocks), 16 blocks per wave, two at
// a time: lane l holds sketch column 32 kb + (l & 31) of block kb = base + 2t
// + (l >> 5), so a wave reads 64 consecutive sketch columns of the row (runs
// of M's row inside drawn blocks), a block's absolute maximum comes from a
// reduction over its 32 lanes, and every fourth lane packs its own and the
// next three lanes' codes into one word.
// Dt part: workgroup (256 columns j, block kb), one column per thread (the
// reads of one sketch row are coalesced across the threads).
__global__ __launch_bounds__(256) void mx_gather_kernel(MxGatherArgs a) {
  const int64_t L = *a.L_dev;
  const int64_t nblk = (L + kBlk - 1) / kBlk;
  const int64_t bid = blockIdx.x;
  float x[kBlk];
  if (bid < a.cgroups) {
    const int64_t i = bid / a.cchunks;
    const int lane = threadIdx.x & 63, e = lane & 31;
    const int64_t kb0 = ((bid % a.cchunks) * 4 + (threadIdx.x >> 6)) * kMxCBlocksPerWave + (lane >> 5);
    constexpr int T = kMxCBlocksPerWave / 2;
    // every load first (a block past the sketch reads entry 0, a padding
    // column column 0; their values are not used)
    int32_t jj[T];
    double scl[T];
    float raw[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int64_t kb = kb0 + 2 * t;
      const int64_t l = kb < nblk ? kb * kBlk + e : 0;
      jj[t] = a.colmap[l];
      scl[t] = a.colscale[l];
    }
#pragma unroll
    for (int t = 0; t < T; ++t) raw[t] = a.M[i * a.ldm + (jj[t] >= 0 ? jj[t] : 0)];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int64_t kb = kb0 + 2 * t;
      const float x = jj[t] >= 0 ? (float)((double)raw[t] * scl[t]) : 0.0f;
      float amax = fabsf(x);
#pragma unroll
      for (int o = 16; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
      uint8_t eb;
      float down;
      mx_block_scale(amax, &eb, &down);
      const float y = x * down;
      const float y1 = __shfl_down(y, 1, 64), y2 = __shfl_down(y, 2, 64), y3 = __shfl_down(y, 3, 64);
      if (kb < nblk) {
        if ((e & 3) == 0)
          *reinterpret_cast<uint32_t*>(a.C + i * a.ldc + kb * kBlk + e) = pack4_e4m3(y, y1, y2, y3);
        if (e == 0) a.Cs[i * a.ldcs + kb] = eb;
      } else if (e == 0 && kb < (nblk + 3) / 4 * 4) {
        // the product reads scales in words of 4 blocks: the rest of the
        // last word is 1 (127), its data is never read
        a.Cs[i * a.ldcs + kb] = 127;
      }
    }
  } else {
    const int64_t b = bid - a.cgroups;
    const int64_t jgroups = (a.p + 255) / 256;
    const int64_t kb = b / jgroups;
    const int64_t j = (b % jgroups) * 256 + threadIdx.x;
    if (j >= a.p) return;
    if (kb >= nblk) {
      if (kb < (nblk + 3) / 4 * 4) a.Ds[j * a.ldds + kb] = 127;
      return;
    }
    // as above: the 32 loads first, a padding row reads row 0
    int32_t rr[kBlk];
    float raw[kBlk];
#pragma unroll
    for (int e = 0; e < kBlk; ++e) rr[e] = a.colmap[kb * kBlk + e];
#pragma unroll
    for (int e = 0; e < kBlk; ++e) raw[e] = a.N[(int64_t)(rr[e] >= 0 ? rr[e] : 0) * a.ldn + j];
    float amax = 0.0f;
#pragma unroll
    for (int e = 0; e < kBlk; ++e) {
      x[e] = rr[e] >= 0 ? (float)((double)raw[e] * a.colscale[kb * kBlk + e]) : 0.0f;
      amax = fmaxf(amax, fabsf(x[e]));
    }
    uint8_t eb;
    float down;
    mx_block_scale(amax, &eb, &down);
    uint32_t w[kBlk / 4];
#pragma unroll
    for (int q = 0; q < kBlk / 4; ++q)
      w[q] = pack4_e4m3(x[4 * q] * down, x[4 * q + 1] * down, x[4 * q + 2] * down, x[4 * q + 3] * down);
    uint4* dst = reinterpret_cast<uint4*>(a.Dt + j * a.lddt + kb * kBlk);
    dst[0] = make_uint4(w[0], w[1], w[2], w[3]);
    dst[1] = make_uint4(w[4], w[5], w[6], w[7]);
    a.Ds[j * a.ldds + kb] = eb;
  }
}

// ---------------------------------------------------------------------------
// Product
// ---------------------------------------------------------------------------
struct MxArgs {
  const uint8_t* A; int64_t lda; const uint8_t* As; int64_t ldas;   // M x K bytes, M x K/32 scales
  const uint8_t* B; int64_t ldb; const uint8_t* Bs; int64_t ldbs;   // N x K bytes, N x K/32 scales
  int64_t m, p;
  const int64_t* K_dev;             // inner extent = round_up(*K_dev, 32)
  float* C; int64_t ldc;
  const float* Y; int64_t ldy;
  double* tile_part;
  int64_t tiles_m, tiles_n;
};

struct MxTile {
  static constexpr int BM = 256, BN = 256, BK = 128, KC = BK / 16;   // 16-byte chunks per row
  static constexpr int NL = BM * KC / kThreads;
  uint4 As[2][BM * KC];
  uint4 Bs[2][BN * KC];
  double red[16];
};

__device__ __forceinline__ int mx_slot(int row, int chunk) { return row * MxTile::KC + (chunk ^ (row & 7)); }

__device__ __forceinline__ void mx_tile_coords(const MxArgs& g, int64_t& tm, int64_t& tn) {
  // the XCD-aware order of the other products
  constexpr int64_t kXcd = 8, kGroup = 8;
  const int64_t bid = blockIdx.x;
  const int64_t tiles = g.tiles_m * g.tiles_n;
  const int64_t per = tiles / kXcd;
  const int64_t lg = bid < per * kXcd ? (bid % kXcd) * per + bid / kXcd : bid;
  const int64_t span = kGroup * g.tiles_n;
  const int64_t first = (lg / span) * kGroup;
  const int64_t gm = min(g.tiles_m - first, kGroup);
  const int64_t r = lg % span;
  tm = first + r % gm;
  tn = r / gm;
}

template <bool EDGE>
__device__ __forceinline__ void mx_body(const MxArgs& g, MxTile& sh, int64_t m0, int64_t n0, int64_t K) {
  constexpr int BK = MxTile::BK, KC = MxTile::KC, NL = MxTile::NL;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 31, lh = lane >> 5;
  const int wm0 = (wave & 1) * 128, wn0 = (wave >> 1) * 128;

  f32x16 acc[4][4];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[b][c] = f32x16{};

  uint4 ra[NL], rb[NL];
  // K is a multiple of 32; chunks past K or outside the matrix are zero
  auto load_one = [&](const uint8_t* X, int64_t ld, int64_t r, int64_t rmax, int64_t k) -> uint4 {
    if ((!EDGE || r < rmax) && k < K) return *reinterpret_cast<const uint4*>(X + r * ld + k);
    return make_uint4(0, 0, 0, 0);
  };
  auto load = [&](int64_t kt) {
    const int64_t k0 = kt * BK;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int f = tid + kThreads * q;
      ra[q] = load_one(g.A, g.lda, m0 + f / KC, g.m, k0 + 16 * (f % KC));
      rb[q] = load_one(g.B, g.ldb, n0 + f / KC, g.p, k0 + 16 * (f % KC));
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int f = tid + kThreads * q;
      sh.As[buf][mx_slot(f / KC, f % KC)] = ra[q];
      sh.Bs[buf][mx_slot(f / KC, f % KC)] = rb[q];
    }
  };
  // the four E8M0 scales of this k-step for the rows / columns of a lane
  // (one 32-bit word per block of the wave; 127 = 1 outside the matrix)
  auto scales = [&](const uint8_t* S, int64_t lds, int64_t r, int64_t rmax, int64_t kt) -> uint32_t {
    if (EDGE && r >= rmax) return 0x7f7f7f7fu;
    return *reinterpret_cast<const uint32_t*>(S + r * lds + 4 * kt);
  };
  auto compute = [&](int buf, int64_t kt) {
    uint32_t sa[4], sb[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) sa[b] = scales(g.As, g.ldas, m0 + wm0 + 32 * b + lr, g.m, kt);
#pragma unroll
    for (int c = 0; c < 4; ++c) sb[c] = scales(g.Bs, g.ldbs, n0 + wn0 + 32 * c + lr, g.p, kt);
#pragma unroll
    for (int s = 0; s < BK / 64; ++s) {
      i32x8 av[4], bv[4];
      const int c0 = 4 * s + lh;   // this lane's 16-byte chunks: c0 and c0 + 2 (indices 64s + 16h, 64s + 32 + 16h)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int row = wm0 + 32 * b + lr;
        const uint4 u0 = sh.As[buf][mx_slot(row, c0)], u1 = sh.As[buf][mx_slot(row, c0 + 2)];
        av[b] = i32x8{(int)u0.x, (int)u0.y, (int)u0.z, (int)u0.w, (int)u1.x, (int)u1.y, (int)u1.z, (int)u1.w};
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int row = wn0 + 32 * c + lr;
        const uint4 u0 = sh.Bs[buf][mx_slot(row, c0)], u1 = sh.Bs[buf][mx_slot(row, c0 + 2)];
        bv[c] = i32x8{(int)u0.x, (int)u0.y, (int)u0.z, (int)u0.w, (int)u1.x, (int)u1.y, (int)u1.z, (int)u1.w};
      }
      const int sh_bits = 8 * (2 * s + lh);
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[b][c] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
              av[b], bv[c], acc[b][c], 0, 0, 0, (int)((sa[b] >> sh_bits) & 0xffu), 0,
              (int)((sb[c] >> sh_bits) & 0xffu));
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
    compute(cur, kt);
    if (kt + 1 < nkt) store(cur ^ 1);
    __syncthreads();
  }

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
        if (g.C) g.C[row * g.ldc + col] = val;
        const double dv = (double)val;
        if (g.Y) {
          const double d = dv - (double)g.Y[row * g.ldy + col];
          e2 = fma(d, d, e2);
        }
        n2 = fma(dv, dv, n2);
      }
      if ((v & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
  if (g.tile_part) {
    e2 = warp_sum_f64(e2);
    n2 = warp_sum_f64(n2);
    if (lane == 0) { sh.red[wave] = e2; sh.red[4 + wave] = n2; }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int64_t tiles = g.tiles_m * g.tiles_n;
      g.tile_part[blockIdx.x] = ((sh.red[0] + sh.red[1]) + sh.red[2]) + sh.red[3];
      g.tile_part[tiles + blockIdx.x] = ((sh.red[4] + sh.red[5]) + sh.red[6]) + sh.red[7];
    }
  }
}

__global__ __launch_bounds__(kThreads, 1) void mx_gemm_kernel(MxArgs g) {
  __shared__ MxTile sh;
  int64_t tm, tn;
  mx_tile_coords(g, tm, tn);
  const int64_t m0 = tm * MxTile::BM, n0 = tn * MxTile::BN;
  const int64_t K = (*g.K_dev + kBlk - 1) / kBlk * kBlk;
  if (m0 + MxTile::BM <= g.m && n0 + MxTile::BN <= g.p)
    mx_body<false>(g, sh, m0, n0, K);
  else
    mx_body<true>(g, sh, m0, n0, K);
}

// ============================================================================
// The same product with the code tiles fetched straight into LDS
// (buffer_load_dwordx4 ... lds), as the bf16 inner-index-contiguous kernel
// does: a wave instruction fills 64 consecutive 16-byte slots (lane l at
// slot base + l), slot P of a tile being row P / 8 and the chunk whose
// swizzled position (chunk ^ ((row >> 1) & 7)) is P % 8, so the 16-lane
// groups of ds_read_b128 (16 consecutive rows, one chunk) hit 16 bank
// groups. Rows past the end lie outside the buffer's record count and
// chunks past the inner extent get an out-of-range offset; both read zero.
// The scale words of step k + 1 are loaded into registers before that
// step's tile loads are issued, so the in-order wait for the tile also
// covers them and nothing inside the compute phase waits on memory.
// ============================================================================
__device__ __forceinline__ int mx_lds_slot(int row, int chunk) { return row * 8 + (chunk ^ ((row >> 1) & 7)); }

__device__ __forceinline__ __amdgpu_buffer_rsrc_t mx_panel_rsrc(const uint8_t* base, int64_t rows, int64_t ld) {
  const uint64_t u = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  const int bytes = __builtin_amdgcn_readfirstlane((int)(rows > 0 ? rows * ld : 0));
  void* p = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, bytes, 0x00020000);
}

// eight waves (two per SIMD), each 128 x 64 of the tile
constexpr int kMxWaves = 8;

// The two tile stages and the two scale stages are separate LDS objects: the
// loads into one and the reads of the other are then provably disjoint, so
// the compiler's wait for the loads stays at the step boundary instead of
// before every fragment read.
struct MxStage {
  uint4 A[MxTile::BM * MxTile::KC];
  uint4 B[MxTile::BN * MxTile::KC];
};
// E8M0 scale words of four k-steps for the 256 rows of A and the 256 columns
// of B: [row][k-step % 4], rows of B after those of A. 16-byte aligned, so a
// row's four words are one ds_read_b128 (with 4-byte alignment the compiler
// splits it into dword pairs, which at a 16-byte lane stride put rows r and
// r + 16 in one bank)
struct alignas(16) MxScales {
  uint32_t w[2 * MxTile::BM * 4];
};

__global__ __launch_bounds__(kMxWaves * 64, 1) void mx_gemm_lds_kernel(MxArgs g) {
  __shared__ MxStage st0, st1;
  __shared__ MxScales sc0, sc1;
  __shared__ double red[16];
  constexpr int BK = MxTile::BK, NW = kMxWaves, CB = 16 / NW;
  constexpr int INSTS = MxTile::BM / 8 / NW;   // load instructions per wave per operand and step
  static_assert(2 * MxTile::BM == 64 * NW, "one scale row per lane of the workgroup");
  int64_t tm, tn;
  mx_tile_coords(g, tm, tn);
  const int64_t m0 = tm * MxTile::BM, n0 = tn * MxTile::BN;
  const int64_t K = (*g.K_dev + kBlk - 1) / kBlk * kBlk;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 31, lh = lane >> 5;
  const int wm0 = (wave & 1) * 128, wn0 = (wave >> 1) * 32 * CB;
  const __amdgpu_buffer_rsrc_t ra = mx_panel_rsrc(g.A + m0 * g.lda, min((int64_t)MxTile::BM, g.m - m0), g.lda);
  const __amdgpu_buffer_rsrc_t rb = mx_panel_rsrc(g.B + n0 * g.ldb, min((int64_t)MxTile::BN, g.p - n0), g.ldb);
  constexpr unsigned kOut = 0x80000000u;

  f32x16 acc[4][CB];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[b][c] = f32x16{};

  auto issue = [&](int64_t kt, MxStage& dst) {
    const int64_t k0 = kt * BK;
    const unsigned sk = (unsigned)k0;
#pragma unroll
    for (int j = 0; j < INSTS; ++j) {
      const int row = (INSTS * wave + j) * 8 + (lane >> 3);
      const int chunk = (lane & 7) ^ ((row >> 1) & 7);
      const bool live = k0 + 16 * chunk < K;
      const unsigned oa = live ? (unsigned)(row * g.lda + chunk * 16) : kOut;
      const unsigned ob = live ? (unsigned)(row * g.ldb + chunk * 16) : kOut;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          ra, (__attribute__((address_space(3))) void*)&dst.A[(INSTS * wave + j) * 64], 16, oa, sk, 0, 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rb, (__attribute__((address_space(3))) void*)&dst.B[(INSTS * wave + j) * 64], 16, ob, sk, 0, 0);
    }
  };
  // The scale words of k-steps 4q .. 4q + 3 (16 bytes of a scale row) for
  // every row of the tile, one row per lane of the workgroup, straight into
  // LDS: one instruction per wave every four k-steps, instead of one 4-byte
  // load per row, block and k-step. Rows past the matrix lie outside the
  // buffer's range and read 0 (scale 2^-127 on zero codes); words past a
  // row's scale blocks belong to k-steps that are never computed.
  const int srow = 64 * wave + lane;           // 0 .. 511: A rows, then B rows
  const bool sis_a = srow < MxTile::BM;
  const __amdgpu_buffer_rsrc_t rsa = mx_panel_rsrc(g.As, g.m, g.ldas);
  const __amdgpu_buffer_rsrc_t rsb = mx_panel_rsrc(g.Bs, g.p, g.ldbs);
  const unsigned svo = sis_a ? (unsigned)((m0 + srow) * g.ldas) : (unsigned)((n0 + srow - MxTile::BM) * g.ldbs);
  auto issue_scales = [&](int64_t q, MxScales& dst) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(sis_a ? rsa : rsb,
        (__attribute__((address_space(3))) void*)&dst.w[64 * wave * 4], 16, svo, (unsigned)(16 * q), 0, 0);
  };
  auto compute = [&](const MxStage& src, const uint32_t* sa, const uint32_t* sb) {
#pragma unroll 1
    for (int s = 0; s < BK / 64; ++s) {
      i32x8 av[4], bv[CB];
      const int c0 = 4 * s + lh;   // this lane's 16-byte chunks: c0 and c0 + 2
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int row = wm0 + 32 * b + lr;
        const uint4 u0 = src.A[mx_lds_slot(row, c0)], u1 = src.A[mx_lds_slot(row, c0 + 2)];
        av[b] = i32x8{(int)u0.x, (int)u0.y, (int)u0.z, (int)u0.w, (int)u1.x, (int)u1.y, (int)u1.z, (int)u1.w};
      }
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const int row = wn0 + 32 * c + lr;
        const uint4 u0 = src.B[mx_lds_slot(row, c0)], u1 = src.B[mx_lds_slot(row, c0 + 2)];
        bv[c] = i32x8{(int)u0.x, (int)u0.y, (int)u0.z, (int)u0.w, (int)u1.x, (int)u1.y, (int)u1.z, (int)u1.w};
      }
      const int sh_bits = 8 * (2 * s + lh);
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < CB; ++c)
          acc[b][c] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
              av[b], bv[c], acc[b][c], 0, 0, 0, (int)((sa[b] >> sh_bits) & 0xffu), 0,
              (int)((sb[c] >> sh_bits) & 0xffu));
    }
  };
  // One k-step: the next step's tile (and, before a group of four, the next
  // group's scales) is issued into the other stage, this step's tile is
  // consumed, then everything lands.
  const int64_t nkt = (K + BK - 1) / BK;
  // the scale words of the current group of four steps for this lane's four
  // rows of A and two columns of B, read from LDS once per group (16 bytes a
  // row: conflict-free, where one word per step at a 16-byte stride is not)
  uint4 sa4[4], sb4[CB];
  auto step = [&](int64_t kt, int kq, const MxStage& cur, MxStage& nxt, const MxScales& scur, MxScales& snxt) {
    if (kq == 0) {
#pragma unroll
      for (int b = 0; b < 4; ++b) sa4[b] = *reinterpret_cast<const uint4*>(&scur.w[(wm0 + 32 * b + lr) * 4]);
#pragma unroll
      for (int c = 0; c < CB; ++c)
        sb4[c] = *reinterpret_cast<const uint4*>(&scur.w[(MxTile::BM + wn0 + 32 * c + lr) * 4]);
    }
    if (kt + 1 < nkt) {
      if (kq == 3) issue_scales((kt + 1) >> 2, snxt);
      issue(kt + 1, nxt);
    }
    auto word = [kq](const uint4& v) { return kq == 0 ? v.x : kq == 1 ? v.y : kq == 2 ? v.z : v.w; };
    uint32_t sa[4], sb[CB];
#pragma unroll
    for (int b = 0; b < 4; ++b) sa[b] = word(sa4[b]);
#pragma unroll
    for (int c = 0; c < CB; ++c) sb[c] = word(sb4[c]);
    compute(cur, sa, sb);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  };
  if (nkt > 0) {
    issue_scales(0, sc0);
    issue(0, st0);
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  // eight steps per trip: the tile stages alternate every step, the scale
  // stages every four, each at a fixed LDS object (kt is a multiple of 8, so
  // each call's step within its group of four is a constant)
  for (int64_t kt = 0; kt < nkt; kt += 8) {
    step(kt, 0, st0, st1, sc0, sc1);
    if (kt + 1 < nkt) step(kt + 1, 1, st1, st0, sc0, sc1);
    if (kt + 2 < nkt) step(kt + 2, 2, st0, st1, sc0, sc1);
    if (kt + 3 < nkt) step(kt + 3, 3, st1, st0, sc0, sc1);
    if (kt + 4 < nkt) step(kt + 4, 0, st0, st1, sc1, sc0);
    if (kt + 5 < nkt) step(kt + 5, 1, st1, st0, sc1, sc0);
    if (kt + 6 < nkt) step(kt + 6, 2, st0, st1, sc1, sc0);
    if (kt + 7 < nkt) step(kt + 7, 3, st1, st0, sc1, sc0);
  }

  double e2 = 0.0, n2 = 0.0;
  store_tile_with_error<CB>(acc, g.C, g.ldc, g.Y, g.ldy, g.m, g.p, m0 + wm0 + 4 * lh, n0 + wn0 + lr, e2, n2);
  if (g.tile_part) {
    e2 = warp_sum_f64(e2);
    n2 = warp_sum_f64(n2);
    if (lane == 0) { red[wave] = e2; red[NW + wave] = n2; }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int64_t tiles = g.tiles_m * g.tiles_n;
      double a = 0.0, b = 0.0;
      for (int w = 0; w < NW; ++w) {
        a += red[w];
        b += red[NW + w];
      }
      g.tile_part[blockIdx.x] = a;
      g.tile_part[tiles + blockIdx.x] = b;
    }
  }
}

}  // namespace

hipError_t launch_mx_gather(const MxGatherLaunch& L, hipStream_t s) {
  MxGatherArgs a{};
  a.M = L.M; a.ldm = L.ldm; a.N = L.N; a.ldn = L.ldn; a.m = L.m; a.p = L.p; a.L_dev = L.L_dev;
  a.nblk_max = L.L_pad_max / kBlk;
  a.colmap = L.colmap; a.colscale = L.colscale;
  a.C = L.C; a.ldc = L.ldc; a.Cs = L.Cs; a.ldcs = L.ldcs;
  a.Dt = L.Dt; a.lddt = L.lddt; a.Ds = L.Ds; a.ldds = L.ldds;
  // blocks up to the next multiple of 4 (their scales are written as 1)
  const int64_t nblk_w = round_up(a.nblk_max, 4);
  a.nblk_max = nblk_w;
  a.cchunks = ceil_div(nblk_w, 4 * kMxCBlocksPerWave);
  a.cgroups = (L.C && L.m > 0) ? L.m * a.cchunks : 0;
  const int64_t dgroups = (L.Dt && L.p > 0) ? nblk_w * ceil_div(L.p, 256) : 0;
  const int64_t total = a.cgroups + dgroups;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(mx_gather_kernel, dim3((unsigned)total), dim3(256), 0, s, a);
  return hipGetLastError();
}

int64_t mx_gemm_tiles(int64_t m, int64_t p) { return ceil_div(m, MxTile::BM) * ceil_div(p, MxTile::BN); }

hipError_t launch_mx_gemm(const MxGemmLaunch& L, hipStream_t s) {
  MxArgs g{};
  g.A = L.A; g.lda = L.lda; g.As = L.As; g.ldas = L.ldas;
  g.B = L.B; g.ldb = L.ldb; g.Bs = L.Bs; g.ldbs = L.ldbs;
  g.m = L.m; g.p = L.p; g.K_dev = L.K_dev; g.C = L.Cout; g.ldc = L.ldc; g.Y = L.Y; g.ldy = L.ldy;
  g.tile_part = L.tile_part;
  g.tiles_m = ceil_div(L.m, MxTile::BM);
  g.tiles_n = ceil_div(L.p, MxTile::BN);
  const int64_t tiles = g.tiles_m * g.tiles_n;
  if (tiles == 0) return hipSuccess;
  // LDS-direct loads: 32-bit offsets within a 256-row panel (the API
  // already requires 16-byte aligned codes and leading dimensions)
  const int64_t ld = std::max(L.lda, L.ldb);
  if (257 * ld < ((int64_t)1 << 31))
    hipLaunchKernelGGL(mx_gemm_lds_kernel, dim3((unsigned)tiles), dim3(kMxWaves * 64), 0, s, g);
  else
    hipLaunchKernelGGL(mx_gemm_kernel, dim3((unsigned)tiles), dim3(kThreads), 0, s, g);
  return hipGetLastError();
}
