// Internal declarations shared by the libsbmm HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "sbmm.h"

// Device status word bits (set by kernels with plain vector stores; read
// and cleared by the synchronizing calls).
enum : int32_t {
  SBMM_DEV_NONFINITE = 1,   // NaN/Inf in a norm or weight
  SBMM_DEV_BUDGET = 2,      // c below the number of strata that can be sampled
  SBMM_DEV_USER_CK = 4,     // user draw counts inconsistent with the weights
  SBMM_DEV_RNG = 8          // a draw ran out of generator blocks (never expected)
};

// Sketch columns are padded (with zero columns) to a multiple of this, so
// the sketched product needs no tail handling along its inner dimension.
constexpr int64_t SBMM_SKETCH_PAD = 32;

inline int64_t round_up(int64_t x, int64_t q) { return (x + q - 1) / q * q; }
inline int64_t ceil_div(int64_t x, int64_t q) { return (x + q - 1) / q; }

inline size_t dtype_size(sbmm_dtype t) {
  switch (t) {
    case SBMM_F64: return 8;
    case SBMM_F32: return 4;
    case SBMM_BF16: return 2;
    case SBMM_F8E4M3: return 1;
  }
  return 0;
}

// ----------------------------------------------------------------------------
// Device helpers
// ----------------------------------------------------------------------------

__device__ __forceinline__ float bf16_bits_to_float(uint16_t b) {
  return __uint_as_float(((uint32_t)b) << 16);
}

// Round-to-nearest-even float -> bf16 bits (NaN kept quiet).
__device__ __forceinline__ uint16_t float_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

template <typename T> struct Elem;
template <> struct Elem<double> {
  __device__ static double to_double(double x) { return x; }
};
template <> struct Elem<float> {
  __device__ static double to_double(float x) { return (double)x; }
};
template <> struct Elem<uint16_t> {  // bf16 stored as raw bits
  __device__ static double to_double(uint16_t x) { return (double)bf16_bits_to_float(x); }
};

__device__ __forceinline__ double warp_sum_f64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ----------------------------------------------------------------------------
// Host-side launch helpers (defined in the .hip files)
// ----------------------------------------------------------------------------

struct NormLaunch {
  sbmm_dtype dt;
  const void* M; int64_t ldm;
  const void* N; int64_t ldn;
  int64_t m, n, p;
  int32_t K;
  const int64_t* off_dev;   // K+1
  double* partial;          // [R][n]
  int rsplit;               // R
  double* col_sq; double* row_sq; double* blk;
  int32_t* status;
  // blocks wider than one statistics chunk: chunks per block (1: one
  // workgroup per block writes blk directly) and the [3][K][chunks] partials
  int32_t stats_chunks = 1;
  double* stats_part = nullptr;
};
size_t norms_partial_elems(sbmm_dtype dt, int64_t m, int64_t n, int* rsplit_out);
// statistics chunks per block for a partition whose widest block is max_width
// (1 when a workgroup per block suffices)
int32_t norms_stats_chunks(int64_t n, int32_t K, int64_t max_width);
hipError_t launch_norms(const NormLaunch& a, hipStream_t s);
// Batched norm pass: per problem, build_batch_norm_args writes the argument
// blocks (batch_norm_args_bytes / batch_stats_args_bytes bytes) of a
// NormLaunch (m, n, p >= 1) and returns its workgroup count; the caller
// uploads them with the prefix sums of workgroups (wg_off) and of blocks
// (blk_off), count + 1 entries each.
size_t batch_norm_args_bytes();
size_t batch_stats_args_bytes();
int64_t build_batch_norm_args(const NormLaunch& L, void* norm_out, void* stats_out);
hipError_t launch_batch_norms(sbmm_dtype dt, const void* norm_args, const int64_t* wg_off, int64_t total_wg,
                              const void* stats_args, const int64_t* blk_off, int64_t total_blk,
                              int32_t count, hipStream_t s);

struct PlanLaunch {
  int mode;                 // sbmm_mode
  int prob;                 // sbmm_prob
  int alloc;                // sbmm_alloc
  int64_t n; int32_t K; int64_t c;
  int64_t A, S;
  const int64_t* off_dev;   // K+1
  const double* col_sq; const double* row_sq; const double* blk;
  const double* user_w; const int64_t* user_ck_dev; const double* blkprod_sq;
  const double* pilot_sq;   // K pilot estimates, alloc == TWO_STEP (4.7)
  uint64_t seed, trial;
  // > 0: the pilot of the two-step algorithm (Alg. 3 step 1): pilot_r draws
  // in every stratum that can be sampled, from the Philox streams of tag 2
  int64_t pilot_r;
  // workspace
  uint64_t* W; uint64_t* cdf; uint64_t* T; int64_t* draw_off; int64_t* width;
  uint64_t* G; int64_t* quota; uint64_t* rem; int64_t* left;
  // outputs
  int32_t* idx; double* scale; int64_t* col_off; int64_t* ck; double* p_hat;
  int32_t* colmap; double* colscale; int64_t L_pad_max;
  int32_t* status;
  // strata wider than two design chunks: chunks per stratum (1: one
  // workgroup per stratum) and the per-chunk maxima and integer sums
  int32_t dchunks = 1;
  double* dpart_max = nullptr;
  uint64_t* dpart_sum = nullptr;
  // non-null: the draw offsets run on many workgroups, from the width sum
  // of every 256 draws that the sampler leaves here
  uint64_t* wpart = nullptr;
};
// design chunks per stratum for strata of at most max_atoms atoms (A atoms,
// S strata in all); 1 when a workgroup per stratum suffices
int32_t plan_design_chunks(int64_t max_atoms, int64_t A, int64_t S);
// whether the draw offsets of c draws take the many-workgroup form
bool plan_wide_offsets(int64_t c);
hipError_t launch_plan(const PlanLaunch& a, hipStream_t s);
// block-mode plans of many problems, one workgroup each (plans in device memory)
hipError_t launch_batch_plan(const PlanLaunch* plans_dev, int32_t count, hipStream_t s);

struct GatherLaunch {
  sbmm_dtype in_dt, out_dt;
  const void* M; int64_t ldm;
  const void* N; int64_t ldn;
  int64_t m, p;
  const int64_t* L_dev;
  int64_t L_pad_max;
  const int32_t* colmap; const double* colscale;
  void* C; int64_t ldc;
  void* D; int64_t ldd;
};
hipError_t launch_gather(const GatherLaunch& a, hipStream_t s);
// float32 gathers of many problems in one launch: args holds one
// build_batch_gather_args record per problem (which returns that problem's
// workgroup count), wg_off the count + 1 running workgroup offsets.
size_t batch_gather_args_bytes();
int64_t build_batch_gather_args(const GatherLaunch& g, void* out);
hipError_t launch_batch_gather(const void* args, const int64_t* wg_off, int32_t count, int64_t total_wg,
                               hipStream_t s);

struct GemmLaunch {
  sbmm_dtype dt;            // F64 or F32 operands
  const void* A; int64_t lda;   // m x K row-major
  const void* B; int64_t ldb;   // K x p row-major
  int64_t m, p;
  int64_t K_host;           // inner extent if K_dev == nullptr
  const int64_t* K_dev;     // device inner extent (rounded up to 32 by the kernel)
  void* Cout; int64_t ldc;  // optional output (F64 for F64, else F32)
  const void* Y; int64_t ldy;   // optional reference for the error epilogue
  double* tile_part;        // [tiles][2]: sum (C - Y)^2, sum C^2
  // block-product norms (optional)
  int32_t K_blocks; const int64_t* off_dev; double* blk_part;  // [K][tiles*4]
  // float32 staging of the partial sums of inner extents above 4096 (one
  // tile-sized slot per workgroup, private to it)
  float* stage;
  // bf16 only: A given as K x M (a_trans) / B given as N x K (b_trans)
  bool a_trans, b_trans;
  // grouped float32 only: read the sketch in place from A = M, B = N
  const int32_t* colmap; const double* colscale;
  // split-K path for small outputs (launch_gemm_skinny): its workspace of
  // gemm_skinny_ws_bytes(dt, m, p, skinny_K_max, blocks) bytes
  void* skinny_ws; int64_t skinny_K_max;
  // bf16 256 x 256 product only: output extents read on the device (at most
  // m / p, which size the grid; tiles past them exit), and the scatter
  // epilogue: instead of Cout, output element (r, j) goes, times sc_w[j], to
  // sc_out[r][sc_map[j]] (SC_COLS), or times sc_w[r] to sc_out[sc_map[r]][j]
  // (SC_ROWS), as bf16 or (sc_f32) float32, leading dimension sc_ld
  const int64_t* m_dev; const int64_t* p_dev;
  int sc_mode; void* sc_out; int64_t sc_ld; int sc_f32; const int32_t* sc_map; const double* sc_w;
  // upper bound of the device inner extent (0: unknown); the bf16 product
  // with B as K x p rows needs it to bound its 32-bit offsets
  int64_t K_max;
};
enum { SC_NONE = 0, SC_COLS = 1, SC_ROWS = 2 };
// Workspace of the split-K path for an m x p product with inner extent up to
// K_max (nblk > 0: per-block norms of that many blocks); 0 when the product
// should take the tiled kernels (large outputs, short inner extents).
size_t gemm_skinny_ws_bytes(sbmm_dtype dt, int64_t m, int64_t p, int64_t K_max, int32_t nblk);
// The same product as launch_gemm (F32 / F64), writing its epilogue sums into
// column 0 of tile_part ([2][tiles_out]) and the block norms into column 0 of
// blk_part ([K][blk_cols]), zeros elsewhere.
hipError_t launch_gemm_skinny(const GemmLaunch& L, int64_t tiles_out, int64_t blk_cols, hipStream_t s);
// bytes of the float32 staging buffer launch_gemm needs
size_t gemm_stage_bytes(sbmm_dtype dt, int64_t m, int64_t p);
int64_t gemm_tiles(sbmm_dtype dt, int64_t m, int64_t p, bool blocknorm);
// tiles of a bf16 product in the inner-index-contiguous form (B given as N x K)
int64_t gemm_tiles_tn(int64_t m, int64_t p);
hipError_t launch_gemm(const GemmLaunch& a, hipStream_t s);
// Many float32 products in one launch, one workgroup per (problem, tile)
// item (see gemm.hip). The per problem argument blocks (grouped_gemm_args_bytes
// each, built on the host by build_grouped_gemm_args for tile configuration
// cfg) and the work list live in device memory; `stage` holds items * bm * bn
// floats (one staging slot per item).
struct GroupedLaunch {
  const void* probs;
  const int32_t* item_prob; const int32_t* item_tile; const int64_t* part_base;
  int64_t items, nparts;
  float* stage;
  int cfg;
  bool gather;
};
int grouped_cfg_count();
// whether a product can take grouped configuration 4 (256 x 256 tiles with
// LDS-direct loads: 16-byte aligned rows, 32-bit panel offsets)
bool grouped_lds_ok(const GemmLaunch& L);
void grouped_cfg_shape(int cfg, int64_t* bm, int64_t* bn, int* wg_per_cu);
size_t grouped_gemm_args_bytes();
void build_grouped_gemm_args(const GemmLaunch& L, int cfg, void* out);
hipError_t launch_grouped_gemm(const GroupedLaunch& L, hipStream_t s);
// Per problem t: out[2t] = its sketched tiles' error partials summed,
// out[2t+1] = its exact tiles' squared-norm partials summed (fixed order);
// L[t] = *col_end[t] when L is not null.
hipError_t launch_grouped_reduce(const double* sk_part, int64_t sk_nparts, const int64_t* sk_base,
                                 const double* ex_part, int64_t ex_nparts, const int64_t* ex_base,
                                 const int64_t* const* col_end, int32_t count, double* out, int64_t* L,
                                 hipStream_t s);
// bf16 products (launch_gemm forwards SBMM_BF16 here) and their tile shape
hipError_t launch_hgemm(const GemmLaunch& a, hipStream_t s);
// Measured matrix-core throughput (peak.hip): `grid` workgroups of four
// waves, each wave running independent chains of the dtype's 32x32
// instruction `iters` times; *instructions receives their total count. out
// holds one float per thread (grid x 256).
hipError_t launch_mfma_peak(sbmm_dtype dt, int grid, int64_t iters, float* out, int64_t* instructions,
                            hipStream_t s);
int64_t mfma_peak_flops_per_instruction(sbmm_dtype dt);
// The bf16 product takes A (m x K) and B (K x p) as they are, both row-major
// (no transposed copy of B): 16-byte aligned rows and 32-bit offsets over the
// K_max (or K_host) rows of B.
bool hgemm_kn_ok(const GemmLaunch& a);
// Workgroup tiles (error-partial slots) of the bf16 product launch_gemm runs
// for these operands (256 x 256 tiles for the forms above, else 128 x 128).
int64_t hgemm_tiles(const GemmLaunch& a);
void hgemm_tile_shape(int64_t* bm, int64_t* bn);

// ||M^k N_k||_F^2 per block through the Gram matrices (float32 or bf16
// inputs, promoted exactly; blocks at most block_gram_max_width() wide), one
// workgroup per block and operand.
// workspace of launch_block_gram: the two Gram matrices of every block, in
// tiles of 16 up to the widest block
size_t block_gram_ws_bytes(int32_t K, int64_t max_width);
hipError_t launch_block_gram(sbmm_dtype dt, const void* M, int64_t ldm, const void* N, int64_t ldn, int64_t m,
                             int64_t p, const int64_t* off_dev, int32_t K, int64_t max_width, double* out, void* ws,
                             hipStream_t s);
// y (rows x cols, leading dimension ldy) = float32 of the bf16 x (ldx)
hipError_t launch_bf16_to_f32(const uint16_t* x, int64_t rows, int64_t cols, int64_t ldx, float* y, int64_t ldy,
                              hipStream_t s);
int64_t block_gram_max_width();
// the row strides (elements) the Gram kernel's 32-bit buffer offsets cover
bool block_gram_strides_ok(int64_t ldm, int64_t ldn);

// Backward of the sketch: per-atom draw lists and the scatter of dC / dD
// into dM / dN.
hipError_t launch_draw_lists(const int32_t* idx, int64_t c, int64_t A, int32_t* cnt, int32_t* rank,
                             int64_t* aoff, int32_t* list, hipStream_t s);
struct BackwardScatter {
  int mode; const int64_t* off_dev; int32_t K;
  const int64_t* aoff; const int32_t* list; const double* scale; const int64_t* col_off;
  int64_t m, n, p;
  sbmm_dtype grad_dt;   // dtype of dC / dD (F64 or F32)
  sbmm_dtype out_dt;    // dtype of dM / dN
  const void* dC; int64_t lddc; const void* dD; int64_t lddd;
  void* dM; int64_t lddm; void* dN; int64_t lddn;
  int64_t L; int32_t* status;
};
hipError_t launch_scatter(const BackwardScatter& b, hipStream_t s);
// bf16 backward over the drawn atoms merged: per atom the compact offset
// uoff (-1 undrawn) and w = sum of scale^2 over its draws; per compact column
// its inner index ucol and weight uw; per inner index the drawn flag; the
// compact width in *lu.
struct BackwardDedup {
  int mode; const int64_t* off_dev; int32_t K; int64_t A, n;
  const int32_t* cnt; const int64_t* aoff; const int32_t* list; const double* scale;
  int64_t* uoff; double* wsum; int32_t* ucol; double* uw; uint8_t* drawn; int64_t* lu;
  int64_t cap;        // room in ucol / uw (the compact width is clamped to it)
  int32_t* status;    // device status word (a compact width above cap)
};
hipError_t launch_dedup(const BackwardDedup& d, hipStream_t s);
// NU (L_max x ldnu) = bf16 rows ucol of N, MUt (L_max x ldmu) = bf16 of the
// columns ucol of M transposed; rows past *lu untouched, padding zero.
hipError_t launch_gather_compact(sbmm_dtype in_dt, const void* N, int64_t ldn, int64_t p, const void* M, int64_t ldm,
                                 int64_t m, const int32_t* ucol, const int64_t* lu, int64_t L_max, uint16_t* NU,
                                 int64_t ldnu, uint16_t* MUt, int64_t ldmu, hipStream_t s);
// G16 = bf16(G) (m x ldp), G16t = bf16(G^T) (p x ldm), padding zero.
hipError_t launch_g_prep(const float* G, int64_t ldg, int64_t m, int64_t p, uint16_t* G16, int64_t ldp,
                         uint16_t* G16t, int64_t ldm, hipStream_t s);
// Zero the columns of dM and rows of dN whose inner index was not drawn.
hipError_t launch_zero_undrawn(sbmm_dtype out_dt, void* dM, int64_t lddm, int64_t m, void* dN, int64_t lddn,
                               int64_t p, int64_t n, const uint8_t* drawn, hipStream_t s);
hipError_t launch_gemm_strided(sbmm_dtype dt, const void* A, int64_t ars, int64_t aks, const void* B,
                               int64_t bks, int64_t bjs, void* C, int64_t ldc, int64_t M, int64_t Nc,
                               int64_t K, hipStream_t s);
hipError_t launch_to_bf16(const float* x, int64_t rows, int64_t cols, int64_t ldx, uint16_t* y,
                          hipStream_t s);
// y (cols x rows, ldy) = bf16(x^T) for x rows x cols (ldx) in F32 or BF16;
// with rows_dev only the first round_up(*rows_dev, 32) rows are transposed.
hipError_t launch_transpose_bf16(sbmm_dtype src_dt, const void* x, int64_t rows, int64_t cols, int64_t ldx,
                                 const int64_t* rows_dev, uint16_t* y, int64_t ldy, hipStream_t s);

// MX E4M3 sketch (blocks of 32 sketch columns, E8M0 scales) and its
// product on the block-scaled matrix instruction. C: m x L_pad bytes (ldc a
// multiple of 16), Cs: m x L_pad/32 scales; Dt: D transposed, p x L_pad
// bytes, Ds: p x L_pad/32 scales; scale leading dimensions at least
// round_up(L_pad_max / 32, 4) and multiples of 4.
struct MxGatherLaunch {
  const float* M; int64_t ldm;
  const float* N; int64_t ldn;
  int64_t m, p;
  const int64_t* L_dev; int64_t L_pad_max;
  const int32_t* colmap; const double* colscale;
  uint8_t* C; int64_t ldc; uint8_t* Cs; int64_t ldcs;
  uint8_t* Dt; int64_t lddt; uint8_t* Ds; int64_t ldds;
};
hipError_t launch_mx_gather(const MxGatherLaunch& a, hipStream_t s);
struct MxGemmLaunch {
  const uint8_t* A; int64_t lda; const uint8_t* As; int64_t ldas;
  const uint8_t* B; int64_t ldb; const uint8_t* Bs; int64_t ldbs;
  int64_t m, p;
  const int64_t* K_dev;
  float* Cout; int64_t ldc;
  const float* Y; int64_t ldy;
  double* tile_part;
};
int64_t mx_gemm_tiles(int64_t m, int64_t p);
hipError_t launch_mx_gemm(const MxGemmLaunch& a, hipStream_t s);

// Probability error bounds (Thm 3.3, 4.2, 4.4) and the expected squared
// error of a stratified design; every block is split into chunks of
// bound_chunks(n_k) workgroups.
struct BoundLaunch {
  int32_t K;
  const int64_t* off;         // [K+1] block offsets
  const int64_t* chunk_off;   // [K+1] first chunk of every block
  int64_t chunks;             // chunk_off[K]
  const double* col_sq; const double* row_sq; const double* blk;
  const double* blkprod_sq; const double* pilot_sq;   // pilot_sq: TWO_STEP only, else null
  const double* p_hat; const int64_t* ck;
  double* part;               // [2 * chunks]
  int32_t rule;               // SBMM_ALLOC_OPT / NORM / TWO_STEP
  int64_t c;
  double beta;                // > 0: given; 0: the sampled one
  int32_t n_delta;
  double delta[SBMM_BOUND_MAX_DELTA];
  double* out;                // device [SBMM_BOUND_FIXED + 2 n_delta]
};
int64_t bound_chunks(int64_t width);
hipError_t launch_bound(const BoundLaunch& a, hipStream_t s);

// Fill kernels (used instead of memset so that captured graphs hold only
// kernel nodes).
hipError_t launch_fill_f64(double* p, int64_t count, double v, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s);

// Sum `rows` x `cols` float64 partials (row-major) over rows in a fixed order
// into out[cols].
hipError_t launch_reduce_cols(const double* part, int64_t rows, int64_t cols,
                              double* out, hipStream_t s);

hipError_t launch_error(sbmm_dtype dt, int64_t m, int64_t p, const void* X,
                        int64_t ldx, const void* Y, int64_t ldy,
                        double* part, int64_t nparts, hipStream_t s);
int64_t error_parts(int64_t m, int64_t p);
