// Assignment dispatch (shape choice, persistent grid, launches), centroid
// preparation, energy reduction and the controller kernel.  The assignment
// kernel itself is in km_assign_kernel.h.

#include <stdlib.h>

#include "km_assign_kernel.h"

namespace km {

// ---------------------------------------------------------------------------
// Host-side dispatch
// ---------------------------------------------------------------------------

// Kernel for an instance: the shape comes from the arguments (0 = default;
// KM_ASSIGN_SHAPE=<n> overrides it for tuning runs).
static int shape_override() {
  static int v = -2;
  if (v == -2) {
    const char* e = getenv("KM_ASSIGN_SHAPE");
    v = e ? atoi(e) : -1;
  }
  return v;
}

KernelPick assign_pick(const AssignArgs& a) {
  const int ks = pick_ks(a.d, a.gemm_bf16);
  if (ks < 0) return KernelPick();
  const int ov = shape_override();
  const int shape = ov >= 0 ? ov : a.shape;
  KernelPick p = a.gemm_bf16 ? pick_bf16(ks, a.xbf16 != 0, a.K, shape) : pick_f32(ks, a.xbf16 != 0, a.K, shape);
  // launches that keep row bounds run the bounds variant (more LDS: the row queues)
  if (a.lb && p.fn_bnd && p.resident) {
    p.fn = p.fn_bnd;
    p.lds = p.lds_bnd;
  }
  return p;
}

int assign_bounds_ok(const AssignArgs& a) {
  if (a.gemm_bf16) return 0;
  const int ks = pick_ks(a.d, 0);
  if (ks < 0) return 0;
  const int ov = shape_override();
  const KernelPick p = pick_f32(ks, a.xbf16 != 0, a.K, ov >= 0 ? ov : a.shape);
  return (p.fn_bnd && p.resident) ? 1 : 0;
}

int assign_list_mode(const AssignArgs& a) {
  const KernelPick p = assign_pick(a);
  if (!p.fn) return 0;
  const bool defer = a.gemm_bf16 || !p.resident;
  const int grid = assign_grid(a);
  return (defer && grid > 0 && grid <= kReMaxGrid) ? 1 : 0;
}

RecheckArgs recheck_args(const AssignArgs& a, double* e_part) {
  const KernelPick p = assign_pick(a);
  RecheckArgs r{};
  r.X = a.X; r.N = a.N; r.d = a.d; r.K = a.K; r.xbf16 = a.xbf16; r.C = a.C; r.nc = a.nc;
  r.lab = a.lab; r.lab_prev = a.lab_prev; r.flags = a.flags; r.fl_cnt = a.fl_cnt;
  r.grid = assign_grid(a);
  r.W = p.threads / 64;
  r.group_rows = p.rows;
  r.sb16 = p.rows / (p.threads / 64);
  r.e_part = e_part;
  r.ctl = a.ctl;
  return r;
}

// Kernels whose LDS budget exceeds the default 64 KB must say so once.
static hipError_t allow_lds(const KernelPick& p) {
  if (p.lds <= 64 * 1024) return hipSuccess;
  static const void* done[64];
  static int n_done = 0;
  for (int i = 0; i < n_done; ++i)
    if (done[i] == p.fn) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(p.fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e == hipSuccess && p.fn_batch && p.fn_batch != p.fn)
    e = hipFuncSetAttribute(p.fn_batch, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  if (n_done < 64) done[n_done++] = p.fn;
  return hipSuccess;
}

// Persistent grid: as many workgroups as fit on the device at once (queried
// once per kernel instance), never more than there are row groups.
int assign_grid(const AssignArgs& a) {
  if (a.N <= 0 || a.K <= 0 || a.d <= 0 || a.d > kMaxD || a.K > kMaxK) return -1;
  const KernelPick p = assign_pick(a);
  if (!p.fn) return -1;
  return (int)assign_resident(p, a.N, 1.0);
}

// Workgroups resident at once on the device for this kernel, scaled by frac
// and capped at the instance's row groups (at least 1).
int64_t assign_resident(const KernelPick& p, int64_t N, double frac) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
      clear_pending_error();
      cus = 256;
    }
  }
  if (allow_lds(p) != hipSuccess) clear_pending_error();
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, p.fn, p.threads, p.lds) != hipSuccess ||
      per_cu <= 0) {
    clear_pending_error();
    per_cu = 1;
  }
  const int64_t groups = (N + p.rows - 1) / p.rows;
  int64_t resident = (int64_t)per_cu * cus;
  if (const char* e = getenv("KM_ASSIGN_GRID_MULT")) resident *= atoi(e) > 0 ? atoi(e) : 1;
  int64_t g = (int64_t)(resident * frac);
  if (g < 1) g = 1;
  return groups < g ? groups : g;
}

hipError_t launch_assign(const AssignArgs& a, Role role, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (a.N <= 0 || a.K <= 0 || a.d <= 0 || a.d > kMaxD || a.K > kMaxK || !a.flags) return hipErrorInvalidValue;
  const KernelPick p = assign_pick(a);
  if (!p.fn) return hipErrorInvalidValue;
  const int grid = assign_grid(a);
  if (grid <= 0) return hipErrorInvalidValue;
  AssignArgs arg = a;
  arg.role = role;
  void* params[] = {&arg};
  hipError_t e = allow_lds(p);
  if (e != hipSuccess) return e;
  clear_pending_error();
  if (ev0 || ev1) return hipExtLaunchKernel(p.fn, dim3(grid), dim3(p.threads), params, p.lds, s, ev0, ev1, 0);
  return hipLaunchKernel(p.fn, dim3(grid), dim3(p.threads), params, p.lds, s);
}

// ---------------------------------------------------------------------------
// Centroid preparation: ||c_j||^2 (float64 sum, rounded), bf16 hi/lo pair, residual norms
// ---------------------------------------------------------------------------

__device__ __forceinline__ void prep_body(const float* C, int K, int d, float* nc, uint16_t* Cb, float* delta,
                                          int bx) {
  const int lane = threadIdx.x & 63;
  const int j = bx * 4 + (threadIdx.x >> 6);
  if (j >= K) return;
  const float* cr = C + (int64_t)j * d;
  const int64_t KD = (int64_t)K * d;
  double p = 0.0, e = 0.0;
  for (int k = lane; k < d; k += kWave) {
    const float c = cr[k];
    p = fma((double)c, (double)c, p);
    if (Cb) {
      uint16_t h, l;
      const double r = bf16_split(c, &h, &l);
      Cb[(int64_t)j * d + k] = h;
      Cb[KD + (int64_t)j * d + k] = l;
      e = fma(r, r, e);
    }
  }
  p = wave_sum(p);
  e = wave_sum(e);
  if (lane == 0) {
    nc[j] = (float)p;
    if (Cb) delta[j] = (float)sqrt(e);
  }
}

__global__ __launch_bounds__(256) void k_prep(const float* C, int K, int d, float* nc, uint16_t* Cb,
                                              float* delta) {
  prep_body(C, K, d, nc, Cb, delta, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_prep_batch(BatchRef<PrepArgs> t) {
  const int b = batch_find(t.prefix, t.n, blockIdx.x);
  const PrepArgs& p = t.tab[b];
  prep_body(p.C, p.K, p.d, p.nc, p.Cb, p.delta, blockIdx.x - t.prefix[b]);
}

hipError_t launch_prep_batch(const PrepArgs* tab, const int* prefix, int n, int blocks, hipStream_t s) {
  clear_pending_error();
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prep_batch, dim3(blocks), dim3(256), 0, s, BatchRef<PrepArgs>{tab, prefix, n});
  return hipGetLastError();
}

hipError_t launch_prep(const float* C, int K, int d, float* nc, uint16_t* Cb, float* delta,
                       hipStream_t s) {
  clear_pending_error();
  hipLaunchKernelGGL(k_prep, dim3((K + 3) / 4), dim3(256), 0, s, C, K, d, nc, Cb, delta);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_reduce_energy(const double* e_part, int n, double* out) {
  __shared__ double red[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += e_part[i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// One workgroup: the controller stage that closes a pass (stage 1 after the
// candidate, stage 2 after the optional fall-back).
__global__ __launch_bounds__(256) void k_controller(CtlArgs a) {
  __shared__ double red[256];
  if (a.ctl->done) return;
  controller_stage(a.ctl, a.e_part, a.n_part, a.stage, a.tr, red);
}

__global__ __launch_bounds__(256) void k_controller_batch(const CtlArgs* tab) {
  __shared__ double red[256];
  const CtlArgs& a = tab[blockIdx.x];
  if (a.ctl->done) return;
  controller_stage(a.ctl, a.e_part, a.n_part, a.stage, a.tr, red);
}

hipError_t launch_controller_batch(const CtlArgs* tab, int n, hipStream_t s) {
  clear_pending_error();
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_controller_batch, dim3(n), dim3(256), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_assign_batch(const KernelPick& p, const AssignArgs* tab, const int* prefix, int n, int blocks,
                               size_t lds, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (!p.fn_batch || blocks <= 0) return hipErrorInvalidValue;
  hipError_t e = allow_lds(p);
  if (e != hipSuccess) return e;
  BatchRef<AssignArgs> ref{tab, prefix, n};
  void* params[] = {&ref};
  clear_pending_error();
  return hipLaunchKernel(p.fn_batch, dim3(blocks), dim3(p.threads), params, lds, s);
}

hipError_t launch_controller(const CtlArgs& a, hipStream_t s) {
  clear_pending_error();
  hipLaunchKernelGGL(k_controller, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reduce_energy(const double* e_part, int n, double* out, hipStream_t s) {
  clear_pending_error();
  hipLaunchKernelGGL(k_reduce_energy, dim3(1), dim3(256), 0, s, e_part, n, out);
  return hipGetLastError();
}

}  // namespace km
