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
// One workgroup per (block, operand) (n_k <= 128) forms one Gram matrix on
// matrix cores (v_mfma_f32_32x32x2_f32) in a 128 x 128 tile split in 64 x 64
// quadrants over the four waves; since both are symmetric only the quadrants
// (0,0), (0,1), (1,1) are formed and (0,1) counts twice. The contraction runs
// over the rows of M^k (stored as loaded: step k = row h, index i = column)
// and over the columns of N_k (stored transposed), so both operands of every
// step come from the same LDS tile layout [k][i], and the two Gram matrices
// of a block land in the same lane layout. They are written to a workspace
// in that layout and a second kernel forms the inner product in float64 in a
// fixed order. Splitting the two operands over workgroups halves the
// accumulators a workgroup holds, which lets two workgroups share a compute
// unit and doubles the workgroups streaming the inputs.
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

struct GramWs {
  float* g;        // [K][2][4 waves][2][2][16][64 lanes]
};

constexpr int kGramVals = 2 * 2 * 16;                   // accumulator values per lane
constexpr int64_t kGramPerOperand = 4 * kGramVals * 64;  // floats per (block, operand)

__device__ __forceinline__ bool gram_wave_active(int wave, int nk) {
  // quadrant (1,0) mirrors (0,1); quadrants outside the block are all zero
  const int wave_m0 = (wave & 1) * 64, wave_n0 = (wave >> 1) * 64;
  return wave != 1 && wave_m0 < nk && wave_n0 < nk;
}

__global__ __launch_bounds__(kThreads, 2) void block_gram_half_kernel(GramArgs a, GramWs w) {
  __shared__ float Xs[2][kBK][kS];
  const int k = blockIdx.x;
  const int phase = blockIdx.y;   // 0: rows of M^k; 1: columns of N_k
  const int64_t lo = a.off[k];
  const int nk = (int)(a.off[k + 1] - lo);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 31, lh = lane >> 5;
  const int wave_m0 = (wave & 1) * 64, wave_n0 = (wave >> 1) * 64;
  const bool active = gram_wave_active(wave, nk);

  f32x16 acc[2][2];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[b][c] = f32x16{};

  float r[kBK * kT / kThreads];
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
  if (!active) return;
  float* out = w.g + ((int64_t)k * 2 + phase) * kGramPerOperand + (int64_t)wave * kGramVals * 64;
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 16; ++v) out[((b * 2 + c) * 16 + v) * 64 + lane] = acc[b][c][v];
}

// < G_M, G_N > per block: each lane multiplies the values it holds in both
// matrices (same layout) in float64, in the order (b, c, v); the quadrant
// (0,1) counts twice; fixed-order reduction over lanes and waves.
__global__ __launch_bounds__(kThreads) void block_gram_dot_kernel(GramArgs a, GramWs w) {
  __shared__ double red[4];
  const int k = blockIdx.x;
  const int nk = (int)(a.off[k + 1] - a.off[k]);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double dot = 0.0;
  if (gram_wave_active(wave, nk)) {
    const float* gm = w.g + (int64_t)k * 2 * kGramPerOperand + (int64_t)wave * kGramVals * 64;
    const float* gn = gm + kGramPerOperand;
#pragma unroll
    for (int e = 0; e < kGramVals; ++e) dot = fma((double)gm[e * 64 + lane], (double)gn[e * 64 + lane], dot);
    if (wave == 2) dot *= 2.0;
  }
  dot = warp_sum_f64(dot);
  if (lane == 0) red[wave] = dot;
  __syncthreads();
  if (tid == 0) a.out[k] = ((red[0] + red[1]) + red[2]) + red[3];
}

}  // namespace

size_t block_gram_ws_bytes(int32_t K) { return sizeof(float) * (size_t)K * 2 * kGramPerOperand; }

hipError_t launch_block_gram(const float* M, int64_t ldm, const float* N, int64_t ldn, int64_t m, int64_t p,
                             const int64_t* off_dev, int32_t K, double* out, void* ws, hipStream_t s) {
  if (K <= 0) return hipSuccess;
  GramArgs a{M, ldm, N, ldn, m, p, off_dev, out};
  GramWs w{reinterpret_cast<float*>(ws)};
  hipLaunchKernelGGL(block_gram_half_kernel, dim3((unsigned)K, 2), dim3(kThreads), 0, s, a, w);
  hipLaunchKernelGGL(block_gram_dot_kernel, dim3((unsigned)K), dim3(kThreads), 0, s, a, w);
  return hipGetLastError();
}

int64_t block_gram_max_width() { return kT; }
