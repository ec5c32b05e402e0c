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
constexpr int kColsC = 4;                  // consecutive sketch columns per thread
constexpr int kTileC = kThreads * kColsC;  // sketch columns per workgroup of C
constexpr int kRowsC = 16;                 // rows of C per workgroup
constexpr int kRowsD = 4;                  // rows of D per workgroup (one per wave)
constexpr int kBatch = 4;                  // loads a thread issues before their stores

// Four consecutive elements through one (or, for float64, two) vector
// memory instruction. Global vector accesses need only element alignment on
// this target, so these are used wherever the four elements are consecutive
// in memory.
template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef float type __attribute__((ext_vector_type(4), aligned(4))); };
template <> struct Vec4<double> { typedef double type __attribute__((ext_vector_type(4), aligned(8))); };
template <> struct Vec4<uint16_t> { typedef uint16_t type __attribute__((ext_vector_type(4), aligned(2))); };

template <typename T> __device__ __forceinline__ double to_d(T x) { return Elem<T>::to_double(x); }

template <typename T> __device__ __forceinline__ T from_d(double v);
template <> __device__ __forceinline__ double from_d<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_d<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ uint16_t from_d<uint16_t>(double v) { return float_to_bf16_bits((float)v); }

template <typename T> __device__ __forceinline__ void load4_raw(const T* p, T* v) {
  const typename Vec4<T>::type x = *reinterpret_cast<const typename Vec4<T>::type*>(p);
  v[0] = x[0]; v[1] = x[1]; v[2] = x[2]; v[3] = x[3];
}
template <typename T> __device__ __forceinline__ void store4(T* p, const double* v) {
  typename Vec4<T>::type x;
  x[0] = from_d<T>(v[0]); x[1] = from_d<T>(v[1]); x[2] = from_d<T>(v[2]); x[3] = from_d<T>(v[3]);
  *reinterpret_cast<typename Vec4<T>::type*>(p) = x;
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
// write C (1024 sketch columns x 16 rows each, four consecutive columns per
// thread: one vector load when they are four consecutive columns of M, as
// inside a drawn block, one vector store), the rest D (one row per wave, four
// consecutive elements per lane and step).
template <typename Tin, typename Tout>
__device__ __forceinline__ void gather_body(const GatherArgs& a, int64_t bid) {
  const int64_t L = *a.L_dev;
  const int64_t Lp = (L + SBMM_SKETCH_PAD - 1) / SBMM_SKETCH_PAD * SBMM_SKETCH_PAD;
  if (bid < a.cblocks) {
    if (!a.C) return;
    const int64_t lt = bid % a.ctiles;
    const int64_t hb = bid / a.ctiles;
    const int64_t l0 = lt * kTileC + (int64_t)threadIdx.x * kColsC;
    if (l0 >= Lp) return;          // Lp is a multiple of 32: the four columns are all in or all out
    int32_t j[4];
    double sc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      j[q] = a.colmap[l0 + q];
      sc[q] = a.colscale[l0 + q];
    }
    const bool run = j[0] >= 0 && j[1] == j[0] + 1 && j[2] == j[0] + 2 && j[3] == j[0] + 3;
    const bool vst = (a.ldc % 4 == 0) && ((uintptr_t)a.C % (4 * sizeof(Tout)) == 0);
    const Tin* M = reinterpret_cast<const Tin*>(a.M);
    Tout* C = reinterpret_cast<Tout*>(a.C);
    const int64_t h1 = min(a.m, (hb + 1) * kRowsC);
    // rows in groups of kBatch: every load of a group is issued before its
    // stores (C may not alias M, which the compiler cannot know), in one
    // branch per group with the raw values converted after it (a load whose
    // value is used inside its own branch is waited for there, one latency
    // each); a padding column reads column 0 and is zeroed afterwards
    int32_t jc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) jc[q] = j[q] >= 0 ? j[q] : 0;
    for (int64_t hg = hb * kRowsC; hg < h1; hg += kBatch) {
      Tin raw[kBatch][4];
      if (run) {
#pragma unroll
        for (int r = 0; r < kBatch; ++r)   // a short last group re-reads its last row
          load4_raw<Tin>(M + min(hg + r, h1 - 1) * a.ldm + j[0], raw[r]);
      } else {
#pragma unroll
        for (int r = 0; r < kBatch; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) raw[r][q] = M[min(hg + r, h1 - 1) * a.ldm + jc[q]];
      }
      double v[kBatch][4];
#pragma unroll
      for (int r = 0; r < kBatch; ++r) {
        const int64_t h = hg + r;
        if (h >= h1) break;
#pragma unroll
        for (int q = 0; q < 4; ++q) v[r][q] = j[q] >= 0 ? to_d<Tin>(raw[r][q]) * sc[q] : 0.0;
        if (vst) {
          store4<Tout>(C + h * a.ldc + l0, v[r]);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) C[h * a.ldc + l0 + q] = from_d<Tout>(v[r][q]);
        }
      }
    }
  } else {
    if (!a.D) return;
    const int64_t l = (bid - a.cblocks) * kRowsD + (threadIdx.x >> 6);
    if (l >= Lp) return;
    const int lane = threadIdx.x & 63;
    const int32_t j = a.colmap[l];
    const double sc = a.colscale[l];
    const Tin* src = reinterpret_cast<const Tin*>(a.N) + (int64_t)(j >= 0 ? j : 0) * a.ldn;
    Tout* dst = reinterpret_cast<Tout*>(a.D) + l * a.ldd;
    const bool vst = (a.ldd % 4 == 0) && ((uintptr_t)a.D % (4 * sizeof(Tout)) == 0);
    const int64_t p4 = vst ? a.p / 4 * 4 : 0;   // elements written four at a time
    // the loads unconditional (a lane past p4 re-reads the row's start, a
    // padding row reads row 0; both are zeroed), their values used only
    // after all of them are issued
    for (int64_t f0 = 4 * (int64_t)lane; f0 < p4; f0 += 256 * kBatch) {
      Tin raw[kBatch][4];
#pragma unroll
      for (int r = 0; r < kBatch; ++r) {
        const int64_t f = f0 + 256 * r;
        load4_raw<Tin>(src + (f < p4 ? f : 0), raw[r]);
      }
#pragma unroll
      for (int r = 0; r < kBatch; ++r) {
        const int64_t f = f0 + 256 * r;
        if (f >= p4) break;
        double v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = j >= 0 ? to_d<Tin>(raw[r][q]) * sc : 0.0;
        store4<Tout>(dst + f, v);
      }
    }
    for (int64_t f = p4 + lane; f < a.p; f += 64)
      dst[f] = from_d<Tout>(j >= 0 ? to_d<Tin>(src[f]) * sc : 0.0);
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
  const GatherArgs a = args[t];   // a copy: read once, not reloaded behind the kernel's stores
  gather_body<float, float>(a, bid - wg_off[t]);
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
  a.ctiles = ceil_div(g.L_pad_max, kTileC);
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
