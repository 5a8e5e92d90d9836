// The context of the C ABI (km_ctx) and the argument checks shared by the
// single-instance entry points and the batch engine.
#pragma once

#include <math.h>
#include <stdint.h>

#include <string>

#include "../../include/km.h"
#include "km_assign_kernel.h"
#include "km_ws.h"

using namespace km;

struct km_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  bool timing = false;

  void* arena = nullptr;
  size_t arena_bytes = 0;
  Shape shape;

  Ctl* ctl = nullptr;           // device
  Ctl* ctl_host = nullptr;      // pinned host mirror
  int* done_host = nullptr;     // pinned poll slots
  double* scal_host = nullptr;  // pinned scalars
  hipStream_t q = nullptr;      // internal stream
  hipEvent_t enter = nullptr;   // orders q after the caller's stream
  hipEvent_t poll_ev[2] = {nullptr, nullptr};   // end of an iteration (timing off)
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipEvent_t ta[2] = {nullptr, nullptr}, tb[2] = {nullptr, nullptr};  // start / end of an assignment dispatch

  // assignment tile shape per (precision, X type, padded width, K bucket)
  int8_t tile_shape[2][2][10][9] = {};

  Ws w;                         // workspace carve-up
};

inline km_status fail(km_ctx* c, km_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

inline km_status hip_fail(km_ctx* c, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(c, e == hipErrorOutOfMemory ? KM_ENOMEM : KM_EDEVICE, m);
}

#define HIP_TRY(c, expr, where)                       \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) return hip_fail(c, _e, where); \
  } while (0)

// The kernels read rows and centroids with 16-byte vector loads.
inline bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

inline bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

inline bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

// Tile-shape table index of (d, K): padded width class and K bucket.
inline bool tile_slot(int gemm_bf16, int32_t d, int32_t K, int* wi, int* kb) {
  static const int widths[] = {1, 2, 4, 8, 12, 16, 24, 32, 48, 64};
  if (d < 1 || d > kMaxD || K < 1 || K > kMaxK) return false;
  const int ks = pick_ks(d, gemm_bf16);
  *wi = -1;
  for (int i = 0; i < 10; ++i)
    if (widths[i] == ks) *wi = i;
  int b = 0;
  while ((16 << b) < K) ++b;
  *kb = b;
  return *wi >= 0 && b < 9;
}

inline int shape_for(const km_ctx* c, int gemm_bf16, int xbf, int32_t d, int32_t K) {
  int wi, kb;
  if (!tile_slot(gemm_bf16, d, K, &wi, &kb)) return 0;
  return c->tile_shape[gemm_bf16 ? 1 : 0][xbf ? 1 : 0][wi][kb];
}

inline km_status check_common(km_ctx* c, const void* X, int xt, int64_t N, int32_t d, int32_t K,
                              int prec) {
  if (!c) return KM_EINVAL;
  c->err.clear();
  if (N < 1 || d < 1 || K < 1) return fail(c, KM_EINVAL, "N, d and K must be positive");
  if (K > N) return fail(c, KM_EINVAL, "K must not exceed N");
  if (xt != KM_X_F32 && xt != KM_X_BF16) return fail(c, KM_EINVAL, "unknown X type");
  if (prec != KM_GEMM_F32 && prec != KM_GEMM_BF16) return fail(c, KM_EINVAL, "unknown precision");
  if (d > kMaxD) return fail(c, KM_EUNSUPPORTED, "d > 256 is not supported");
  if (K > kMaxK) return fail(c, KM_EUNSUPPORTED, "K > 4096 is not supported");
  if (N >= ((int64_t)1 << 31)) return fail(c, KM_EUNSUPPORTED, "N >= 2^31 is not supported");
  if (!is_device_ptr(X)) return fail(c, KM_EINVAL, "X is not a device pointer");
  if (!aligned16(X)) return fail(c, KM_EINVAL, "X must start on a 16-byte boundary");
  return KM_OK;
}

