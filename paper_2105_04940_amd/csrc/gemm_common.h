// Shared pieces of the matrix-core product kernels: the argument block, the
// XCD-aware tile order and the fixed-order reduction of the error partials.
#pragma once
#include "common.h"

namespace gemm_detail {

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
  // sketch read in place (gather fused into the product): A column k is
  // colscale[k] * M[:, colmap[k]] and B row k is colscale[k] * N[colmap[k], :]
  // (colmap < 0: zero), with A = M and B = N
  const int32_t* colmap; const double* colscale;
  // device output extents and scatter epilogue (GemmLaunch)
  const int64_t* m_dev; const int64_t* p_dev;
  int sc_mode; void* sc_out; int64_t sc_ld; int sc_f32; const int32_t* sc_map; const double* sc_w;
};

// Words of a raw buffer resource (base address, range in bytes, the flags of
// an untyped buffer), each made wave-uniform so the quad sits in scalar
// registers. Offsets at or past `bytes` read as zero.
typedef int i32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ i32x4 buffer_words(const void* base, int bytes) {
  const uint64_t u = reinterpret_cast<uint64_t>(base);
  i32x4 r;
  r.x = (int)__builtin_amdgcn_readfirstlane((uint32_t)u);
  r.y = (int)__builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  r.z = __builtin_amdgcn_readfirstlane(bytes);
  r.w = 0x00020000;
  return r;
}

// LDS address of a __shared__ object.
__device__ __forceinline__ uint32_t lds_offset(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

// One LDS-DMA load of 16 bytes a lane: lane l's bytes at voff + soff of the
// buffer land at LDS address lds + 16 l (lds wave-uniform). Written as inline
// asm rather than the load-to-LDS builtin on purpose: with the builtin the
// compiler may sink the loads to the end of the matrix-instruction sequence
// that follows (leaving them a fraction of a k-step to land; a timing probe
// showed it) and adds its own conservative waits before reads of the other
// stage. Here the load issues where it is written, nothing else waits for
// it, and the "memory" clobber keeps LDS reads from moving across it. The
// caller waits with wait_loads_barrier before any wave reads the
// destination.
//
// The compiler's hazard checks do not look inside inline asm, so the wait
// states the load needs after its operands are written are in the asm: one
// after m0 is written (always, the compiler sets m0 just before), and
// WAIT + 1 in all. A vector instruction that writes an SGPR the load reads
// (a readfirstlane below, when an operand lives in vector registers) needs
// five, WAIT = 4; operands computed from scalars need none of those, and
// the build's tests check the compiled kernels for that pattern.
template <int WAIT = 0>
__device__ __forceinline__ void lds_dma16(i32x4 rs, uint32_t lds, uint32_t voff, uint32_t soff) {
  // the scalar operands are uniform by contract; readfirstlane makes that
  // visible where the compiler cannot prove it (free where it can)
  rs.x = __builtin_amdgcn_readfirstlane(rs.x); rs.y = __builtin_amdgcn_readfirstlane(rs.y);
  rs.z = __builtin_amdgcn_readfirstlane(rs.z); rs.w = __builtin_amdgcn_readfirstlane(rs.w);
  lds = __builtin_amdgcn_readfirstlane(lds); soff = __builtin_amdgcn_readfirstlane(soff);
  // m0 (the LDS base of the load) is an input operand, so the compiler sets
  // it and knows its value; nothing is clobbered behind its back
  asm volatile("s_nop %4\n\tbuffer_load_dwordx4 %0, %1, %2 offen lds"
               :: "v"(voff), "s"(rs), "s"(soff), "{m0}"(lds), "n"(WAIT) : "memory");
}

// Wait until at most N of this wave's vector-memory loads are outstanding
// (they complete in order), then barrier: every wave's loads older than its
// newest N have landed in LDS. One statement, so no LDS read moves above it;
// a bare barrier, since __syncthreads() adds a fence that waits for all loads.
template <int N>
__device__ __forceinline__ void wait_loads_barrier() {
  asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" :: "n"(N) : "memory");
}

// As wait_loads_barrier, and this wave's LDS reads have returned too: for a
// barrier after which other waves overwrite what those reads fetched, while
// the values read are still to be used.
template <int N>
__device__ __forceinline__ void wait_loads_reads_barrier() {
  asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" :: "n"(N) : "memory");
}

__device__ inline __attribute__((always_inline)) int64_t inner_extent(const GemmArgs& g) {
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
__device__ inline __attribute__((always_inline)) void tile_coords(const GemmArgs& g, int64_t& tm, int64_t& tn) {
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

// Epilogue of a wave's RB x CB blocks of 32x32 matrix-instruction
// accumulators: acc[b][c][v] is output element (rowf(b, v), colf(c)). The
// value is acc, plus extra(b, c, v) when has_extra (a float32 add, acc
// first: the staged partial sums of a long inner extent); it goes to C (if
// given), and the float64 squared difference to Y (if given) and the squared
// value are added into e2 / n2, in the order b, v, c. The elements go in
// groups of 4 v; the Y and extra values of group g + AHEAD are requested
// before group g is consumed, so several groups' loads overlap. The loads
// are unconditional (an element outside the output reads Y[0], and extra
// must be safe to call for any (b, c, v)) and their values are only looked
// at later: a load under a per-element condition becomes a branch that waits
// for it on the spot, one full memory latency per element.
struct NoExtra {
  __device__ float operator()(int, int, int) const { return 0.0f; }
};
template <int RB, int CB, int AHEAD, bool HAS_Y, bool HAS_X, typename RowF, typename ColF, typename Extra>
__device__ __forceinline__ void store_block_impl(const f32x16 (&acc)[RB][CB], RowF& rowf, ColF& colf,
                                                 float* __restrict__ C, int64_t ldc, const float* __restrict__ Y,
                                                 int64_t ldy, int64_t m, int64_t p, double& e2, double& n2,
                                                 Extra& extra) {
  constexpr int NG = 4 * RB;
  float y[AHEAD + 1][4][CB], x[AHEAD + 1][4][CB];
  auto load = [&](int gi) {
#pragma unroll
    for (int vv = 0; vv < 4; ++vv)
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const int b = gi >> 2, v = 4 * (gi & 3) + vv;
        const int64_t row = rowf(b, v), col = colf(c);
        if constexpr (HAS_Y) y[gi % (AHEAD + 1)][vv][c] = Y[row < m && col < p ? row * ldy + col : 0];
        if constexpr (HAS_X) x[gi % (AHEAD + 1)][vv][c] = extra(b, c, v);
      }
  };
#pragma unroll
  for (int gi = 0; gi < AHEAD && gi < NG; ++gi) load(gi);
#pragma unroll
  for (int gi = 0; gi < NG; ++gi) {
    if (gi + AHEAD < NG) load(gi + AHEAD);
#pragma unroll
    for (int vv = 0; vv < 4; ++vv) {
      const int b = gi >> 2, v = 4 * (gi & 3) + vv;
      const int64_t row = rowf(b, v);
      if (row >= m) continue;
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        const int64_t col = colf(c);
        if (col >= p) continue;
        float val = acc[b][c][v];
        if constexpr (HAS_X) val += x[gi % (AHEAD + 1)][vv][c];
        if (C) C[row * ldc + col] = val;
        const double dv = (double)val;
        if constexpr (HAS_Y) {
          const double d = dv - (double)y[gi % (AHEAD + 1)][vv][c];
          e2 = fma(d, d, e2);
        }
        n2 = fma(dv, dv, n2);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}
template <int RB, int CB, int AHEAD = 2, typename RowF, typename ColF, typename Extra = NoExtra>
__device__ __forceinline__ void store_block_with_error(const f32x16 (&acc)[RB][CB], RowF rowf, ColF colf,
                                                       float* __restrict__ C, int64_t ldc,
                                                       const float* __restrict__ Y, int64_t ldy, int64_t m,
                                                       int64_t p, double& e2, double& n2, bool has_extra = false,
                                                       Extra extra = Extra()) {
  // both conditions are uniform over the workgroup
  if (Y) {
    if (has_extra) store_block_impl<RB, CB, AHEAD, true, true>(acc, rowf, colf, C, ldc, Y, ldy, m, p, e2, n2, extra);
    else store_block_impl<RB, CB, AHEAD, true, false>(acc, rowf, colf, C, ldc, Y, ldy, m, p, e2, n2, extra);
  } else {
    if (has_extra) store_block_impl<RB, CB, AHEAD, false, true>(acc, rowf, colf, C, ldc, Y, ldy, m, p, e2, n2, extra);
    else store_block_impl<RB, CB, AHEAD, false, false>(acc, rowf, colf, C, ldc, Y, ldy, m, p, e2, n2, extra);
  }
}
// The 128 x 32 CB block of a wave in the 256 x 256 tile kernels: row
// r0 + 32 b + 8 (v >> 2) + (v & 3), column c0 + 32 c.
template <int CB, typename Extra = NoExtra>
__device__ __forceinline__ void store_tile_with_error(const f32x16 (&acc)[4][CB], float* __restrict__ C,
                                                      int64_t ldc, const float* __restrict__ Y, int64_t ldy,
                                                      int64_t m, int64_t p, int64_t r0, int64_t c0, double& e2,
                                                      double& n2, bool has_extra = false, Extra extra = Extra()) {
  store_block_with_error<4, CB>(
      acc, [=](int b, int v) { return r0 + 32 * b + 8 * (v >> 2) + (v & 3); }, [=](int c) { return c0 + 32 * c; },
      C, ldc, Y, ldy, m, p, e2, n2, has_extra, extra);
}

// Reduce the epilogue partial sums of the workgroup in a fixed order into
// slot `part` of the [2][nparts] partials.
__device__ inline void write_tile_partials_at(const GemmArgs& g, double e2, double n2, double* sm,
                                              int64_t part, int64_t nparts) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  e2 = warp_sum_f64(e2);
  n2 = warp_sum_f64(n2);
  if (lane == 0) { sm[wave] = e2; sm[4 + wave] = n2; }
  __syncthreads();
  if (threadIdx.x == 0) {
    g.tile_part[part] = ((sm[0] + sm[1]) + sm[2]) + sm[3];
    g.tile_part[nparts + part] = ((sm[4] + sm[5]) + sm[6]) + sm[7];
  }
}

// One launch per product: the partial slot is the workgroup index.
__device__ inline void write_tile_partials(const GemmArgs& g, double e2, double n2, double* sm) {
  write_tile_partials_at(g, e2, n2, sm, blockIdx.x, g.tiles_m * g.tiles_n);
}


// Argument block of one launch with tiles of bm x bn.
inline GemmArgs make_gemm_args(const GemmLaunch& L, int64_t bm, int64_t bn) {
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
  g.colmap = L.colmap;
  g.colscale = L.colscale;
  g.m_dev = L.m_dev; g.p_dev = L.p_dev;
  g.sc_mode = L.sc_mode; g.sc_out = L.sc_out; g.sc_ld = L.sc_ld; g.sc_f32 = L.sc_f32;
  g.sc_map = L.sc_map; g.sc_w = L.sc_w;
  const int64_t es = (int64_t)dtype_size(L.dt);
  const int64_t vb = 16;
  g.vec_a = ((uintptr_t)L.A % vb == 0) && ((L.lda * es) % vb == 0);
  g.vec_b = ((uintptr_t)L.B % vb == 0) && ((L.ldb * es) % vb == 0);
  return g;
}

}  // namespace gemm_detail
