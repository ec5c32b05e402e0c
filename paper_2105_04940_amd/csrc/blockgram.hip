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
// One workgroup per (block, operand) (n_k <= 128) forms the upper triangle
// of one Gram matrix on matrix cores (v_mfma_f32_16x16x4_f32) in 16 x 16
// tiles: with T = ceil(n_k / 16) index tiles, only the T (T + 1) / 2 tiles
// (ti <= tj) the block needs are formed, the off-diagonal ones counting twice
// in the inner product. Tile rows are dealt out in pairs (r, T - 1 - r), one
// pair per wave (T + 1 tiles; a middle row alone when T is odd), and the
// wave that takes pair 0 turns with the block index, so the four SIMDs of a
// compute unit carry the same work on average. The contraction runs over the
// rows of M^k (stored as loaded: step k = row h, index i = column) and over
// the columns of N_k (stored transposed), so both operands of every step come
// from the same LDS layout [k][i], and the two Gram matrices of a block land
// in the same lane layout. They are written to a workspace in that layout and
// a second kernel forms the inner product in float64 in a fixed order.
// Splitting the two operands over workgroups halves the accumulators a
// workgroup holds and doubles the workgroups streaming the inputs.
#include <algorithm>

#include "common.h"

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kT = 128;          // Gram tile (max block width)
constexpr int kTiles = kT / 16;  // index tiles of 16

struct GramArgs {
  const void* M; int64_t ldm;   // float32 or bf16 (raw bits), the kernels' template type
  const void* N; int64_t ldn;
  int64_t m, p;
  const int64_t* off;
  double* out;     // [K]
};

// The Gram tiles of every block: [K][2][tiles][tiles][4 values][64 lanes],
// tiles = ceil(widest block / 16) <= kTiles, tiles ti <= tj written.
struct GramWs {
  float* g;
  int tiles;
};

constexpr int64_t kTileVals = 4 * 64;
__device__ __forceinline__ int64_t gram_per_operand(int tiles) { return (int64_t)tiles * tiles * kTileVals; }

// element loads through a buffer resource, promoted exactly to float32
template <typename T> __device__ __forceinline__ float gram_load(__amdgpu_buffer_rsrc_t rs, uint32_t vo, int so);
template <> __device__ __forceinline__ float gram_load<float>(__amdgpu_buffer_rsrc_t rs, uint32_t vo, int so) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, 0));
}
template <> __device__ __forceinline__ float gram_load<uint16_t>(__amdgpu_buffer_rsrc_t rs, uint32_t vo, int so) {
  return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(rs, vo, so, 0) << 16);
}

// A stage holds kStage floats: R = kStage / W contraction rows of W block
// columns, W = 32, 64 or 128 the smallest multiple of 32 (a power of two)
// that covers the block, so a narrow block streams more rows per step with
// the same registers and LDS.
constexpr int kStage = 4096;
__host__ __device__ constexpr int stage_width(int T) { return T <= 2 ? 32 : (T <= 4 ? 64 : 128); }

// Position of element (contraction row kk, block column i) in a stage of
// width W: i XOR ((kk & 1) << 4 | (kk >> 1) & 15). The transposed store of
// N_k (32 lanes writing 32 consecutive rows of one column) and the
// matrix-core reads (16 lanes on each of rows kk, kk + 1) both fall on
// distinct banks, W being a multiple of 32.
__device__ __forceinline__ int lds_pos(int W, int kk, int i) {
  return kk * W + (i ^ (((kk & 1) << 4) | ((kk >> 1) & 15)));
}

// Buffer resource over `bytes` bytes from `base` (fields made wave-uniform).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t gram_rsrc(const void* base, int64_t bytes) {
  const uint64_t u = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  const int nb = __builtin_amdgcn_readfirstlane((int)(bytes > 0 ? bytes : 0));
  void* p = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, nb, 0x00020000);
}

// Accumulator slots of a wave: tile (A, A + j) in slot j < T - A, tile
// (B, B + j') in slot T - A + j'; at most T + 1 <= kTiles + 1 of them.
constexpr int kSlots = kTiles + 1;

// One stage of the tile rows A and B = T - 1 - A (B >= A; B == A holds one
// row). Sub-step s of group g covers rows 32 g + 4 s .. + 3; lane l reads row
// kk = 32 g + 4 s + (l >> 4) at column (16 t + (l & 15)) XOR the row's
// swizzle, i.e. 16 (t XOR hb) + ((l & 15) XOR (2 s + (l >> 5))) with
// hb = (l >> 4) & 1: pe (even t) and po (odd t) hold the lane's row and the
// +-16 hb shift, so the tile offset 16 t and the row offset of s are
// immediates.
template <int T, int A>
__device__ __forceinline__ void gram_step(const float* xs, int lane, f32x4 (&acc)[kSlots]) {
  constexpr int B = T - 1 - A;
  constexpr int W = stage_width(T), R = kStage / W;
  const int hb = (lane >> 4) & 1;
  const int x0 = (lane & 15) ^ (lane >> 5);
  // the swizzle repeats every 8 sub-steps (32 rows): groups of 8 unrolled
#pragma unroll 1
  for (int g = 0; g < R / 32; ++g) {
    const float* pe = xs + (32 * g + (lane >> 4)) * W + 16 * hb;
    const float* po = xs + (32 * g + (lane >> 4)) * W - 16 * hb;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int xo = x0 ^ (2 * s);
      const float* re = pe + xo + s * 4 * W;
      const float* ro = po + xo + s * 4 * W;
      float fr[T];
#pragma unroll
      for (int t = 0; t < T; ++t) fr[t] = (t & 1 ? ro : re)[16 * t];
#pragma unroll
      for (int t = A; t < T; ++t)
        acc[t - A] = __builtin_amdgcn_mfma_f32_16x16x4f32(fr[A], fr[t], acc[t - A], 0, 0, 0);
      if constexpr (B > A) {
#pragma unroll
        for (int t = B; t < T; ++t)
          acc[T - A + t - B] = __builtin_amdgcn_mfma_f32_16x16x4f32(fr[B], fr[t], acc[T - A + t - B], 0, 0, 0);
      }
    }
  }
}

// (T, A) pairs with A <= T - 1 - A
#define SBMM_GRAM_CASES(X) \
  X(1, 0) X(2, 0) X(3, 0) X(3, 1) X(4, 0) X(4, 1) X(5, 0) X(5, 1) X(5, 2) X(6, 0) X(6, 1) X(6, 2) \
  X(7, 0) X(7, 1) X(7, 2) X(7, 3) X(8, 0) X(8, 1) X(8, 2) X(8, 3)

// The stage loop of one workgroup for stage width W (uniform over the
// block): loads of the next stage into registers, the matrix-core work of
// the current one, stores into the other LDS buffer, one barrier per stage.
template <typename ET, int W>
__device__ __forceinline__ void gram_loop(const GramArgs& a, float (*Xs)[kStage], int phase, int64_t lo, int nk,
                                          int code, f32x4 (&acc)[kSlots]) {
  constexpr int ES = sizeof(ET);
  const ET* Mp = reinterpret_cast<const ET*>(a.M);
  const ET* Np = reinterpret_cast<const ET*>(a.N);
  constexpr int R = kStage / W;                   // contraction rows per stage
  constexpr int kPasses = kStage / kThreads;
  constexpr int PR0 = kThreads / W, PR1 = kThreads / R;   // rows per pass (phase 0: of M, 1: of N_k)
  const int tid = threadIdx.x, lane = tid & 63;
  // Buffer loads: per step a resource whose base is the step's first element
  // and whose range ends after the last valid one, a 32-bit lane offset and a
  // scalar offset per pass. Lanes past the block or the extent take offset
  // 2^31, beyond every range (the strides are bounded on the host so that
  // 2^31 plus the largest scalar offset stays below 2^32); the range check
  // returns zero for them. Phase 0: lane -> (row tid / W, column tid % W);
  // phase 1: lane -> (row of N_k tid / R, column tid % R); both read runs of
  // consecutive elements.
  float r[kPasses];
  const int64_t ext = phase == 0 ? a.m : a.p;
  const int64_t nsteps = (ext + R - 1) / R;
  constexpr uint32_t kOut = 0x80000000u;
  const int p_lo = phase == 0 ? tid / W : tid / R;
  const int p_in = phase == 0 ? tid % W : tid % R;
  auto load = [&](int64_t st) {
    const int64_t s0 = st * R;
    const int64_t live = min((int64_t)R, ext - s0);   // valid contraction rows of the step
    if (phase == 0) {
      const int64_t bytes = ((live - 1) * a.ldm + nk) * ES;
      const __amdgpu_buffer_rsrc_t rs = gram_rsrc(Mp + s0 * a.ldm + lo, bytes);
      const uint32_t vo = p_in < nk ? (uint32_t)((p_lo * a.ldm + p_in) * ES) : kOut;
      const int pass = (int)(PR0 * a.ldm * ES);
#pragma unroll
      for (int q = 0; q < kPasses; ++q) r[q] = gram_load<ET>(rs, vo, q * pass);
    } else {
      const int64_t bytes = nk > 0 ? ((nk - 1) * a.ldn + live) * ES : 0;
      const __amdgpu_buffer_rsrc_t rs = gram_rsrc(Np + lo * a.ldn + s0, bytes);
      const uint32_t vo = p_in < live ? (uint32_t)((p_lo * a.ldn + p_in) * ES) : kOut;
      const int pass = (int)(PR1 * a.ldn * ES);
#pragma unroll
      for (int q = 0; q < kPasses; ++q) r[q] = gram_load<ET>(rs, vo, q * pass);
    }
  };
  auto store = [&](int buf) {
    if (phase == 0) {
#pragma unroll
      for (int q = 0; q < kPasses; ++q) Xs[buf][lds_pos(W, p_lo + q * PR0, p_in)] = r[q];
    } else {
#pragma unroll
      for (int q = 0; q < kPasses; ++q) Xs[buf][lds_pos(W, p_in, p_lo + q * PR1)] = r[q];
    }
  };
  if (nsteps > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int64_t st = 0; st < nsteps; ++st) {
    const int cur = (int)(st & 1);
    if (st + 1 < nsteps) load(st + 1);
    switch (code) {
#define SBMM_GRAM_STEP(TT, AA)                                                    \
      case TT * 4 + AA:                                                           \
        if constexpr (stage_width(TT) == W) gram_step<TT, AA>(&Xs[cur][0], lane, acc); \
        break;
      SBMM_GRAM_CASES(SBMM_GRAM_STEP)
#undef SBMM_GRAM_STEP
      default: break;
    }
    if (st + 1 < nsteps) store(cur ^ 1);
    __syncthreads();
  }
}

template <typename ET>
__global__ __launch_bounds__(kThreads, 4) void block_gram_half_kernel(GramArgs a, GramWs w) {
  __shared__ float Xs[2][kStage];
  const int k = blockIdx.x;
  const int phase = blockIdx.y;   // 0: rows of M^k; 1: columns of N_k
  const int64_t lo = a.off[k];
  const int nk = (int)(a.off[k + 1] - lo);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int T = (nk + 15) >> 4;
  const int ra = (wave + k) & 3, rb = T - 1 - ra;
  const bool active = ra <= rb;
  const int code = active ? T * 4 + ra : -1;

  f32x4 acc[kSlots];
#pragma unroll
  for (int j = 0; j < kSlots; ++j) acc[j] = f32x4{};
  const int W = stage_width(T);
  if (W == 32) gram_loop<ET, 32>(a, Xs, phase, lo, nk, code, acc);
  else if (W == 64) gram_loop<ET, 64>(a, Xs, phase, lo, nk, code, acc);
  else gram_loop<ET, 128>(a, Xs, phase, lo, nk, code, acc);
  if (!active) return;
  float* out = w.g + ((int64_t)k * 2 + phase) * gram_per_operand(w.tiles) + lane;
  const int na = T - ra, nb = rb > ra ? T - rb : 0;
#pragma unroll
  for (int j = 0; j < kSlots; ++j) {
    int tile = -1;
    if (j < na) tile = ra * w.tiles + ra + j;
    else if (j < na + nb) tile = rb * w.tiles + rb + (j - na);
    if (tile >= 0) {
      float* o = out + tile * kTileVals;
#pragma unroll
      for (int v = 0; v < 4; ++v) o[v * 64] = acc[j][v];
    }
  }
}

// < G_M, G_N > per block: the tiles ti <= tj in row order are dealt to the
// waves in turn; each lane multiplies the values it holds in both matrices
// (same layout) in float64, an off-diagonal tile counting twice; fixed-order
// reduction over lanes and waves.
__global__ __launch_bounds__(kThreads) void block_gram_dot_kernel(GramArgs a, GramWs w) {
  __shared__ double red[4];
  const int k = blockIdx.x;
  const int nk = (int)(a.off[k + 1] - a.off[k]);
  const int T = (nk + 15) >> 4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const float* gm = w.g + (int64_t)k * 2 * gram_per_operand(w.tiles) + lane;
  const float* gn = gm + gram_per_operand(w.tiles);
  double dot = 0.0;
  int e = 0;
  for (int ti = 0; ti < T; ++ti) {
    for (int tj = ti; tj < T; ++tj, ++e) {
      if ((e & 3) != wave) continue;
      const int64_t base = (ti * w.tiles + tj) * kTileVals;
      double ts = 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) ts = fma((double)gm[base + v * 64], (double)gn[base + v * 64], ts);
      dot += ti < tj ? 2.0 * ts : ts;
    }
  }
  dot = warp_sum_f64(dot);
  if (lane == 0) red[wave] = dot;
  __syncthreads();
  if (tid == 0) a.out[k] = ((red[0] + red[1]) + red[2]) + red[3];
}

}  // namespace

namespace {
int gram_tiles(int64_t max_width) { return (int)std::max<int64_t>(1, (max_width + 15) / 16); }
}  // namespace

size_t block_gram_ws_bytes(int32_t K, int64_t max_width) {
  const size_t t = (size_t)gram_tiles(max_width);
  return sizeof(float) * (size_t)K * 2 * t * t * kTileVals;
}

hipError_t launch_block_gram(sbmm_dtype dt, const void* M, int64_t ldm, const void* N, int64_t ldn, int64_t m,
                             int64_t p, const int64_t* off_dev, int32_t K, int64_t max_width, double* out, void* ws,
                             hipStream_t s) {
  if (K <= 0) return hipSuccess;
  if (max_width > kT) return hipErrorInvalidValue;
  GramArgs a{M, ldm, N, ldn, m, p, off_dev, out};
  GramWs w{reinterpret_cast<float*>(ws), gram_tiles(max_width)};
  if (dt == SBMM_F32)
    hipLaunchKernelGGL(block_gram_half_kernel<float>, dim3((unsigned)K, 2), dim3(kThreads), 0, s, a, w);
  else if (dt == SBMM_BF16)
    hipLaunchKernelGGL(block_gram_half_kernel<uint16_t>, dim3((unsigned)K, 2), dim3(kThreads), 0, s, a, w);
  else
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(block_gram_dot_kernel, dim3((unsigned)K), dim3(kThreads), 0, s, a, w);
  return hipGetLastError();
}

int64_t block_gram_max_width() { return kT; }

// The 32-bit buffer offsets of the Gram kernel: a stage spans at most 128
// rows of M or N, so every range stays below 2^31 and 2^31 plus the largest
// scalar offset (120 rows) below 2^32.
bool block_gram_strides_ok(int64_t ldm, int64_t ldn) { return ldm < (int64_t(1) << 22) && ldn < (int64_t(1) << 22); }
