// Matrix-core throughput of the device, measured: the reference beside the
// specification's peaks that the products' fractions are also given against
// (those peaks assume a 2.4 GHz clock that the power limit holds lower under
// matrix work). Not part of the method.
//
// Every workgroup of four waves runs kChains independent accumulator chains
// of one dtype's 32x32 matrix instruction per wave on operands held in
// registers (no memory traffic inside the loop); four workgroups per compute
// unit, so each SIMD has four waves to issue from. Operands are hashed from
// the lane index (mixed bit patterns rather than constants, which draw less
// power), without NaN or infinity.
#include "common.h"
#include "gemm_common.h"

namespace {

using gemm_detail::f32x16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
constexpr int kChains = 8;

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
  return x;
}
__device__ __forceinline__ float unit(uint32_t x) { return (float)(x & 0xffffu) * (1.0f / 65536.0f) - 0.5f; }

template <int DT>
__global__ __launch_bounds__(256) void mfma_peak_kernel(int64_t iters, float* __restrict__ out) {
  const uint32_t h0 = mix32(blockIdx.x * 256u + threadIdx.x), h1 = mix32(h0 + 1u);
  f32x16 acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc[c] = f32x16{};
  if constexpr (DT == SBMM_F32) {
    const float a = unit(h0), b = unit(h1);
    for (int64_t it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[c], 0, 0, 0);
  } else if constexpr (DT == SBMM_BF16) {
    bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = (__bf16)unit(mix32(h0 + e));
      b[e] = (__bf16)unit(mix32(h1 + e));
    }
    for (int64_t it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
  } else {
    // E4M3 codes with every byte's top exponent bit or lowest mantissa bit
    // clear (mask 0x77): at most 448, never NaN; scales 2^0
    i32x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[e] = (int)(mix32(h0 + e) & 0x77777777u);
      b[e] = (int)(mix32(h1 + e) & 0x77777777u);
    }
    for (int64_t it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < kChains; ++c)
        acc[c] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc[c], 0, 0, 0, 127, 0, 127);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c)
#pragma unroll
    for (int v = 0; v < 16; ++v) s += acc[c][v];
  out[blockIdx.x * 256 + threadIdx.x] = s;   // keeps the chains live
}

}  // namespace

int64_t mfma_peak_flops_per_instruction(sbmm_dtype dt) {
  switch (dt) {
    case SBMM_F32: return 2LL * 32 * 32 * 2;
    case SBMM_BF16: return 2LL * 32 * 32 * 16;
    case SBMM_F8E4M3: return 2LL * 32 * 32 * 64;
    default: return 0;
  }
}

hipError_t launch_mfma_peak(sbmm_dtype dt, int grid, int64_t iters, float* out, int64_t* instructions,
                            hipStream_t s) {
  *instructions = (int64_t)grid * 4 * iters * kChains;
  switch (dt) {
    case SBMM_F32:
      hipLaunchKernelGGL(mfma_peak_kernel<SBMM_F32>, dim3((unsigned)grid), dim3(256), 0, s, iters, out);
      break;
    case SBMM_BF16:
      hipLaunchKernelGGL(mfma_peak_kernel<SBMM_BF16>, dim3((unsigned)grid), dim3(256), 0, s, iters, out);
      break;
    case SBMM_F8E4M3:
      hipLaunchKernelGGL(mfma_peak_kernel<SBMM_F8E4M3>, dim3((unsigned)grid), dim3(256), 0, s, iters, out);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
