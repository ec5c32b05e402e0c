// Internals of the C ABI shared by its source files: the handle, error
// reporting and the device status word.
#pragma once
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.h"

struct sbmm_handle_s {
  int device = 0;
  char err[512] = {0};
  char* ws = nullptr;
  size_t ws_bytes = 0;
  char* scratch = nullptr;     // this device's copy of the fixed scratch of sbmm_plan_noalloc
  int32_t* status = nullptr;   // device status word
  // device copy of the last block partition used, and its host shadow: a
  // call with the same partition enqueues no copy
  int64_t* off_dev = nullptr;
  size_t off_cap = 0;
  std::vector<int64_t> off_host;
};

namespace {

// A caller's enum argument or field as the int it stored. In C any int fits
// an enum object; in C++ reading a value outside the enumeration's range
// through the enum type is undefined, so caller-supplied enums are checked
// through their object representation before they are used as enums.
template <typename E> inline int enum_raw(const E& e) {
  static_assert(sizeof(E) == sizeof(int), "C enums of this ABI are int-sized");
  int v;
  std::memcpy(&v, &e, sizeof v);
  return v;
}

sbmm_status fail(sbmm_handle h, sbmm_status st, const char* fmt, ...) {
  if (h) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(h->err, sizeof(h->err), fmt, ap);
    va_end(ap);
  }
  return st;
}

#define HIP_TRY(h, expr)                                                        \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess)                                                       \
      return fail((h), SBMM_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

sbmm_status check_handle(sbmm_handle h) {
  if (!h || !h->status) return SBMM_E_STATE;
  h->err[0] = 0;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != h->device) {
    if (hipSetDevice(h->device) != hipSuccess)
      return fail(h, SBMM_E_STATE, "cannot select device %d", h->device);
  }
  return SBMM_OK;
}

sbmm_status status_from_device(sbmm_handle h, int32_t bits) {
  if (bits & SBMM_DEV_NONFINITE) return fail(h, SBMM_E_NONFINITE, "non-finite input norm or weight");
  if (bits & SBMM_DEV_BUDGET) return fail(h, SBMM_E_BUDGET, "c is below the number of strata with positive weight");
  if (bits & SBMM_DEV_USER_CK) return fail(h, SBMM_E_ARG, "user draw counts must be positive exactly on strata with positive weight");
  if (bits & SBMM_DEV_RNG) return fail(h, SBMM_E_HIP, "sampler exhausted its generator blocks");
  return SBMM_OK;
}

sbmm_status read_status(sbmm_handle h, hipStream_t s) {
  HIP_TRY(h, hipStreamSynchronize(s));
  int32_t bits = 0;
  HIP_TRY(h, hipMemcpy(&bits, h->status, sizeof(bits), hipMemcpyDeviceToHost));
  if (bits) {
    const int32_t zero = 0;
    HIP_TRY(h, hipMemcpy(h->status, &zero, sizeof(zero), hipMemcpyHostToDevice));
  }
  return status_from_device(h, bits);
}

}  // namespace
