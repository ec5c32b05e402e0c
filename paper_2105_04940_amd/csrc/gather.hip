// Gather and rescale (Alg. 1 step 1(b); Alg. 2 step 3): the drawn columns of
// M and rows of N, each multiplied by its draw's 1/sqrt(c_s p), side by side
// in draw order. Column l of the sketch reads inner index colmap[l] with
// factor colscale[l]; the padding columns (colmap = -1) up to the next
// multiple of 32 are written as zeros, so the sketched product can run over
// whole 32-wide steps.
//
// The sketch width L is read on the device; the grid covers the upper bound
// L_pad_max and workgroups past round_up(L, 32) exit at once.
#include <cstring>

#include "common.h"

namespace {

constexpr int kThreads = 256;
constexpr int kRowsC = 16;   // rows of C per workgroup
constexpr int kRowsD = 4;    // rows of D per workgroup (one per wave)

template <typename T> __device__ __forceinline__ double load_d(const void* p, int64_t i) {
  return Elem<T>::to_double(reinterpret_cast<const T*>(p)[i]);
}

template <typename T> __device__ __forceinline__ void store_d(void* p, int64_t i, double v);
template <> __device__ __forceinline__ void store_d<double>(void* p, int64_t i, double v) {
  reinterpret_cast<double*>(p)[i] = v;
}
template <> __device__ __forceinline__ void store_d<float>(void* p, int64_t i, double v) {
  reinterpret_cast<float*>(p)[i] = (float)v;
}
template <> __device__ __forceinline__ void store_d<uint16_t>(void* p, int64_t i, double v) {
  reinterpret_cast<uint16_t*>(p)[i] = float_to_bf16_bits((float)v);
}

struct GatherArgs {
  const void* M; int64_t ldm;
  const void* N; int64_t ldn;
  int64_t m, p;
  const int64_t* L_dev;
  int64_t ctiles, cblocks;   // column tiles of C, workgroups on C
  const int32_t* colmap; const double* colscale;
  void* C; int64_t ldc;
  void* D; int64_t ldd;
};

// Workgroup `bid` of one problem's gather: the first cblocks workgroups
// write C (256 sketch columns x 16 rows each), the rest D (one row per wave).
template <typename Tin, typename Tout>
__device__ __forceinline__ void gather_body(const GatherArgs& a, int64_t bid) {
  const int64_t L = *a.L_dev;
  const int64_t Lp = (L + SBMM_SKETCH_PAD - 1) / SBMM_SKETCH_PAD * SBMM_SKETCH_PAD;
  if (bid < a.cblocks) {
    if (!a.C) return;
    const int64_t lt = bid % a.ctiles;
    const int64_t hb = bid / a.ctiles;
    const int64_t l = lt * kThreads + threadIdx.x;
    if (l >= Lp) return;
    const int32_t j = a.colmap[l];
    const double sc = a.colscale[l];
    const int64_t h1 = min(a.m, (hb + 1) * kRowsC);
    for (int64_t h = hb * kRowsC; h < h1; ++h) {
      const double v = j >= 0 ? load_d<Tin>(a.M, h * a.ldm + j) * sc : 0.0;
      store_d<Tout>(a.C, h * a.ldc + l, v);
    }
  } else {
    if (!a.D) return;
    const int64_t l = (bid - a.cblocks) * kRowsD + (threadIdx.x >> 6);
    if (l >= Lp) return;
    const int lane = threadIdx.x & 63;
    const int32_t j = a.colmap[l];
    const double sc = a.colscale[l];
    for (int64_t f = lane; f < a.p; f += 64) {
      const double v = j >= 0 ? load_d<Tin>(a.N, (int64_t)j * a.ldn + f) * sc : 0.0;
      store_d<Tout>(a.D, l * a.ldd + f, v);
    }
  }
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kThreads) void gather_kernel(GatherArgs a) {
  gather_body<Tin, Tout>(a, blockIdx.x);
}

// the problem t with wg_off[t] <= x < wg_off[t + 1]
__device__ __forceinline__ int32_t find_item(const int64_t* __restrict__ off, int32_t count, int64_t x) {
  int32_t lo = 0, hi = count - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The float32 gathers of many problems in one launch: workgroup b runs
// workgroup b - wg_off[t] of problem t.
__global__ __launch_bounds__(kThreads) void batch_gather_kernel(const GatherArgs* __restrict__ args,
                                                                const int64_t* __restrict__ wg_off,
                                                                int32_t count) {
  const int64_t bid = blockIdx.x;
  const int32_t t = find_item(wg_off, count, bid);
  gather_body<float, float>(args[t], bid - wg_off[t]);
}

template <typename Tin>
hipError_t dispatch_out(const GatherArgs& a, sbmm_dtype out, dim3 grid, hipStream_t s) {
  switch (out) {
    case SBMM_F64: hipLaunchKernelGGL((gather_kernel<Tin, double>), grid, dim3(kThreads), 0, s, a); break;
    case SBMM_F32: hipLaunchKernelGGL((gather_kernel<Tin, float>), grid, dim3(kThreads), 0, s, a); break;
    case SBMM_BF16: hipLaunchKernelGGL((gather_kernel<Tin, uint16_t>), grid, dim3(kThreads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

GatherArgs make_gather_args(const GatherLaunch& g, int64_t* total) {
  GatherArgs a{};
  a.M = g.M; a.ldm = g.ldm; a.N = g.N; a.ldn = g.ldn;
  a.m = g.m; a.p = g.p; a.L_dev = g.L_dev;
  a.colmap = g.colmap; a.colscale = g.colscale;
  a.C = g.C; a.ldc = g.ldc; a.D = g.D; a.ldd = g.ldd;
  a.ctiles = ceil_div(g.L_pad_max, kThreads);
  a.cblocks = (g.C && g.m > 0) ? a.ctiles * ceil_div(g.m, kRowsC) : 0;
  const int64_t dblocks = (g.D && g.p > 0) ? ceil_div(g.L_pad_max, kRowsD) : 0;
  *total = a.cblocks + dblocks;
  return a;
}

}  // namespace

hipError_t launch_gather(const GatherLaunch& g, hipStream_t s) {
  int64_t total = 0;
  const GatherArgs a = make_gather_args(g, &total);
  if (total == 0) return hipSuccess;
  dim3 grid((unsigned)total);
  switch (g.in_dt) {
    case SBMM_F64: return dispatch_out<double>(a, g.out_dt, grid, s);
    case SBMM_F32: return dispatch_out<float>(a, g.out_dt, grid, s);
    case SBMM_BF16: return dispatch_out<uint16_t>(a, g.out_dt, grid, s);
    default: return hipErrorInvalidValue;
  }
}

size_t batch_gather_args_bytes() { return sizeof(GatherArgs); }

int64_t build_batch_gather_args(const GatherLaunch& g, void* out) {
  int64_t total = 0;
  const GatherArgs a = make_gather_args(g, &total);
  std::memcpy(out, &a, sizeof(a));
  return total;
}

hipError_t launch_batch_gather(const void* args, const int64_t* wg_off, int32_t count, int64_t total_wg,
                               hipStream_t s) {
  if (count <= 0 || total_wg <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_gather_kernel, dim3((unsigned)total_wg), dim3(kThreads), 0, s,
                     reinterpret_cast<const GatherArgs*>(args), wg_off, count);
  return hipGetLastError();
}
