// Seeded synthetic matrices written directly on the device (input generation
// only; nothing of the sampled product is computed here).
//
// Element q of a rows x cols matrix (q = row * cols + col) takes 64-bit word
// q % 4 of the Philox4x64-10 block (Salmon, Moraes, Dror, Shaw, SC'11) with
// key (seed, 0) and counter (q / 4, stream, 0, 3 * 2^32). The word's four
// 16-bit pieces are summed, centred and scaled to unit variance:
//     x = float(h0 + h1 + h2 + h3 - 131070) * float32(1 / sqrt((2^32 - 1) / 3)),
// an integer exact in float32 times a float32 constant, rounded once, so any
// IEEE implementation (the NumPy one in workloads/__init__.py) gives the same
// bits. The distribution is the Irwin-Hall sum of four uniforms: mean 0,
// variance 1, close to Gaussian. Columns [cols, ld) are not touched.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

struct Block { uint64_t v[4]; };

__device__ __forceinline__ Block philox4x64_10(Block x, uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B97F4A7C15ull;
      k1 += 0xBB67AE8584CAA73Bull;
    }
    const uint64_t a = 0xD2E7470EE14C6C93ull * x.v[0], ah = __umul64hi(0xD2E7470EE14C6C93ull, x.v[0]);
    const uint64_t b = 0xCA5A826395121157ull * x.v[2], bh = __umul64hi(0xCA5A826395121157ull, x.v[2]);
    x = Block{{bh ^ x.v[1] ^ k0, b, ah ^ x.v[3] ^ k1, a}};
  }
  return x;
}

constexpr uint64_t kTagInput = 3;
constexpr float kUnitScale = 0x1.bb67aep-16f;   // float32(1 / sqrt((2^32 - 1) / 3))

__device__ __forceinline__ float word_to_value(uint64_t w) {
  const int s = (int)(w & 0xffff) + (int)((w >> 16) & 0xffff) + (int)((w >> 32) & 0xffff) + (int)(w >> 48);
  return (float)(s - 131070) * kUnitScale;
}

__global__ __launch_bounds__(256) void fill_kernel(float* __restrict__ x, int64_t rows, int64_t cols, int64_t ld,
                                                   uint64_t seed, uint64_t stream, float scale) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;   // Philox block = 4 elements
  const int64_t total = rows * cols;
  const int64_t q0 = 4 * j;
  if (q0 >= total) return;
  const Block w = philox4x64_10(Block{{(uint64_t)j, stream, 0, kTagInput << 32}}, seed, 0);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t q = q0 + e;
    if (q < total) {
      const int64_t r = q / cols, c = q % cols;
      const float v = word_to_value(w.v[e]);
      x[r * ld + c] = scale == 1.0f ? v : v * scale;
    }
  }
}

}  // namespace

extern "C" {

// Fill the rows x cols float32 matrix x (device, row-major, leading
// dimension ld >= cols) with stream `stream` of `seed`, each value times
// `scale` (one float32 multiplication, skipped for 1). Returns a hipError_t.
int sbmm_workload_fill(float* x, int64_t rows, int64_t cols, int64_t ld, uint64_t seed, uint64_t stream,
                       float scale, void* hip_stream) {
  if (rows < 0 || cols < 0 || ld < cols || (rows * cols > 0 && !x)) return (int)hipErrorInvalidValue;
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t blocks = (rows * cols + 3) / 4;
  if (blocks > 0)
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((blocks + 255) / 256)), dim3(256), 0, s, x, rows, cols, ld,
                       seed, stream, scale);
  return (int)hipGetLastError();
}

}  // extern "C"
