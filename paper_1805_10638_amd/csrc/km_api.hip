// C ABI of libkmaa (declared in include/km.h): argument checking, the
// context and its workspace, and the launch sequence of the solver.

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "km_ctx.h"


static km_status ensure_ws(km_ctx* c, const Shape& want) {
  if (c->arena && c->shape.fits(want)) return KM_OK;
  Shape s = want;
  if (c->arena) {  // grow monotonically
    s.N = s.N > c->shape.N ? s.N : c->shape.N;
    s.d = s.d > c->shape.d ? s.d : c->shape.d;
    s.K = s.K > c->shape.K ? s.K : c->shape.K;
    s.cap = s.cap > c->shape.cap ? s.cap : c->shape.cap;
    s.bf = s.bf > c->shape.bf ? s.bf : c->shape.bf;
    s.it = s.it > c->shape.it ? s.it : c->shape.it;
    s.bnd = s.bnd > c->shape.bnd ? s.bnd : c->shape.bnd;
    HIP_TRY(c, hipStreamSynchronize(c->q), "hipStreamSynchronize");
    HIP_TRY(c, hipFree(c->arena), "hipFree");
    c->arena = nullptr;
  }
  const size_t off = ws_layout(s, nullptr, nullptr);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, off);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    c->shape = Shape();
    c->arena_bytes = 0;
    return fail(c, KM_ENOMEM, "workspace allocation of " + std::to_string(off) + " bytes failed");
  }
  HIP_TRY(c, hipMemsetAsync(p, 0, off, c->q), "hipMemsetAsync");
  c->arena = p;
  c->arena_bytes = off;
  c->shape = s;
  ws_layout(s, (char*)p, &c->w);
  return KM_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free G (kmeans_g_noalloc)
// ---------------------------------------------------------------------------
// Every buffer of a kmeans_g_noalloc call beyond its inputs and outputs lives
// in this array; each device that runs the library holds its own copy until
// the process ends.  In host code the name is only a stand-in for the symbol:
// km_create looks up the array's address on the device (once per device,
// with that device current) and every host use goes through that address.
static __device__ __align__(256) unsigned char scratch[KM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices] = {};

// Address of device `device`'s copy of the scratch array (device current).
static hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_dev[device] = ptr;
  return hipSuccess;
}

static void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_dev[device];
}

// Clears n 32-bit words (a kernel rather than a memset node, so that the
// launch sequence can be recorded into a graph).
__global__ __launch_bounds__(256) void k_clear_words(unsigned* p, int n) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0u;
}

static hipError_t launch_clear(void* p, size_t bytes, hipStream_t s) {
  const int n = (int)(bytes / 4);
  clear_pending_error();
  hipLaunchKernelGGL(k_clear_words, dim3((n + 255) / 256 < 64 ? (n + 255) / 256 : 64), dim3(256), 0, s,
                     (unsigned*)p, n);
  return hipGetLastError();
}

// Argument checks of one G application (kmeans_g and kmeans_g_noalloc).
static km_status g_check(km_ctx* c, const void* X, km_xtype xt, int64_t N, int32_t d, int32_t K,
                         const float* C, km_prec prec, const int32_t* rho_prev, int32_t* rho, float* C_out,
                         double* E) {
  km_status s = check_common(c, X, xt, N, d, K, prec);
  if (s != KM_OK) return s;
  if (!E) return fail(c, KM_EINVAL, "E must be a host pointer");
  if (!is_device_ptr(C) || !is_device_ptr(rho) || !is_device_ptr(C_out))
    return fail(c, KM_EINVAL, "C, rho and C_out must be device pointers");
  if (!aligned16(C) || !aligned16(C_out)) return fail(c, KM_EINVAL, "C and C_out must start on a 16-byte boundary");
  if (rho_prev && !is_device_ptr(rho_prev)) return fail(c, KM_EINVAL, "rho_prev must be a device pointer");
  const size_t xbytes = (size_t)N * d * (xt == KM_X_BF16 ? 2 : 4);
  const size_t cbytes = (size_t)K * d * 4;
  if (overlap(C_out, cbytes, C, cbytes) || overlap(C_out, cbytes, X, xbytes) ||
      overlap(rho, (size_t)N * 4, X, xbytes) || overlap(rho, (size_t)N * 4, C_out, cbytes))
    return fail(c, KM_EINVAL, "outputs must not alias the inputs");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  return KM_OK;
}

// The launches of one G application on the buffers of w: prep, bound of
// |x|, assignment, energy, update, means; then the scalars come back through
// the context's pinned slots.
static km_status g_run(km_ctx* c, const Ws& w, const void* X, km_xtype xt, int64_t N, int32_t d, int32_t K,
                       const float* C, km_prec prec, const int32_t* rho_prev, int32_t* rho, float* C_out,
                       double* E, km_g_stats* st) {
  hipStream_t st_ = c->q;
  const bool gbf = prec == KM_GEMM_BF16;
  HIP_TRY(c, hipEventRecord(c->enter, c->stream), "hipEventRecord");
  HIP_TRY(c, hipStreamWaitEvent(st_, c->enter, 0), "hipStreamWaitEvent");

  HIP_TRY(c, launch_clear(w.ctl, sizeof(Ctl), st_), "clear control block");
  HIP_TRY(c, launch_prep(C, K, d, w.nc_tmp, gbf ? w.Cb_tmp : nullptr, gbf ? w.del_tmp : nullptr, st_), "prep");
  AssignArgs a{};
  a.X = X; a.N = N; a.d = d; a.K = K; a.C = C; a.nc = w.nc_tmp;
  a.Cb = gbf ? w.Cb_tmp : nullptr; a.delta = gbf ? w.del_tmp : nullptr;
  a.lab = rho; a.lab_prev = rho_prev; a.e_part = w.e_part; a.flags = w.flags; a.ctl = w.ctl;
  a.xbf16 = xt == KM_X_BF16; a.gemm_bf16 = gbf;
  a.shape = shape_for(c, gbf, xt == KM_X_BF16, d, K);
  a.fl_cnt = assign_list_mode(a) ? w.fl_cnt : nullptr;
  UpdateArgs u{};
  u.X = X; u.N = N; u.d = d; u.K = K; u.xbf16 = xt == KM_X_BF16;
  u.lab = rho; u.lab_from_ctl = 0; u.lrank = w.lrank; u.blockcount = w.blockcount;
  u.counts = w.counts; u.seg_start = w.seg_start; u.item_start = w.item_start;
  u.item_cluster = w.item_cluster; u.perm = w.perm; u.partial = w.partial;
  u.max_items = update_max_items(N, K); u.ctl = w.ctl; u.gated = 0;
  u.fx = fx_ok(K, d); u.xbound = w.xbound; u.fxpart = w.fxpart;
  // bound of |x| for the fixed-point sums: part of preparing X, outside the
  // phase times (a solve computes it once)
  HIP_TRY(c, launch_xbound(u, st_), "bound of |x|");
  // with timing on, the events take the times of the kernels' own dispatches
  HIP_TRY(c, launch_assign(a, kRolePlain, st_, c->timing ? c->ta[0] : nullptr,
                           (c->timing && !a.fl_cnt) ? c->tb[0] : nullptr),
          "assignment");
  const int grid = assign_grid(a);
  int n_part = grid;
  if (a.fl_cnt) {   // the listed rows: one re-check launch over the whole pass
    HIP_TRY(c, launch_recheck(recheck_args(a, w.e_part + grid), kRolePlain, st_, c->timing ? c->tb[0] : nullptr),
            "re-check");
    n_part = grid + kReGrid;
  }
  HIP_TRY(c, launch_reduce_energy(w.e_part, n_part, w.e_out, st_), "energy");
  HIP_TRY(c, launch_update_sums(u, st_, c->timing ? c->ta[1] : nullptr), "update");
  FinalizeArgs f{};
  f.d = d; f.K = K; f.cap = 0; f.partial = w.partial; f.item_start = w.item_start;
  f.counts = w.counts; f.C_in = C; f.C_out = C_out; f.ctl = w.ctl; f.mode = kFinG;
  f.fx = u.fx; f.fxpart = w.fxpart; f.xbound = w.xbound; f.N = N;
  f.C_cand = nullptr; f.C_fb = nullptr; f.G_last = nullptr; f.F_last = nullptr;
  f.ring_dF = nullptr; f.ring_dG = nullptr; f.dots = nullptr;
  HIP_TRY(c, launch_finalize(f, st_, c->timing ? c->tb[1] : nullptr), "finalize");
  HIP_TRY(c, hipMemcpyAsync(c->scal_host, w.e_out, 8, hipMemcpyDeviceToHost, st_), "copy E");
  HIP_TRY(c, hipMemcpyAsync(c->ctl_host, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st_), "copy ctl");
  HIP_TRY(c, hipStreamSynchronize(st_), "hipStreamSynchronize");
  *E = c->scal_host[0];
  if (st) {
    st->changed = rho_prev ? (int64_t)c->ctl_host->cnt_changed[0] : 0;
    st->recheck_rows = (int64_t)c->ctl_host->cnt_flagged[0];
    st->near_tie_rows = (int64_t)c->ctl_host->cnt_near[0];
    st->empty_clusters = c->ctl_host->empty;
    st->assign_ms = st->update_ms = -1.f;
    if (c->timing) {
      if (hipEventElapsedTime(&st->assign_ms, c->ta[0], c->tb[0]) != hipSuccess ||
          hipEventElapsedTime(&st->update_ms, c->ta[1], c->tb[1]) != hipSuccess) {
        clear_pending_error();
        st->assign_ms = st->update_ms = -1.f;
      }
    }
  }
  if (!isfinite(*E)) return fail(c, KM_ENONFINITE, "energy is not finite");
  return KM_OK;
}

extern "C" {

int km_version(void) { return 10000; }

const char* km_status_str(int s) {
  switch (s) {
    case KM_OK: return "ok";
    case KM_NOT_CONVERGED: return "not converged (max_iter reached)";
    case KM_EINVAL: return "invalid argument";
    case KM_ENOMEM: return "out of device memory";
    case KM_EDEVICE: return "HIP runtime error";
    case KM_EUNSUPPORTED: return "unsupported argument";
    case KM_ENONFINITE: return "non-finite energy";
  }
  return "unknown status";
}

const char* km_last_error(const km_ctx* c) { return c ? c->err.c_str() : ""; }

km_status km_create(int device, void* stream, km_ctx** out) {
  if (!out) return KM_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return KM_EINVAL;
  }
  if (hipSetDevice(device) != hipSuccess) return KM_EDEVICE;
  if (scratch_setup(device) != hipSuccess) {
    (void)hipGetLastError();
    return KM_EDEVICE;
  }
  km_ctx* c = new km_ctx();
  c->device = device;
  c->stream = (hipStream_t)stream;
  bool ok = hipStreamCreateWithFlags(&c->q, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&c->enter, hipEventDisableTiming) == hipSuccess &&
            hipEventCreate(&c->ta[0]) == hipSuccess && hipEventCreate(&c->ta[1]) == hipSuccess &&
            hipEventCreate(&c->tb[0]) == hipSuccess && hipEventCreate(&c->tb[1]) == hipSuccess &&
            hipHostMalloc((void**)&c->ctl_host, sizeof(Ctl), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&c->done_host, 2 * sizeof(int), hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&c->scal_host, 8 * sizeof(double), hipHostMallocDefault) == hipSuccess &&
            hipEventCreate(&c->poll_ev[0]) == hipSuccess && hipEventCreate(&c->poll_ev[1]) == hipSuccess &&
            hipEventCreate(&c->t0) == hipSuccess && hipEventCreate(&c->t1) == hipSuccess;
  if (!ok) {
    km_destroy(c);
    return KM_EDEVICE;
  }
  *out = c;
  return KM_OK;
}

void km_destroy(km_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->q) (void)hipStreamSynchronize(c->q);
  if (c->arena) (void)hipFree(c->arena);
  if (c->ctl_host) (void)hipHostFree(c->ctl_host);
  if (c->done_host) (void)hipHostFree(c->done_host);
  if (c->scal_host) (void)hipHostFree(c->scal_host);
  for (hipEvent_t e : c->poll_ev) if (e) (void)hipEventDestroy(e);
  if (c->t0) (void)hipEventDestroy(c->t0);
  if (c->t1) (void)hipEventDestroy(c->t1);
  for (hipEvent_t e : c->ta) if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->tb) if (e) (void)hipEventDestroy(e);
  if (c->enter) (void)hipEventDestroy(c->enter);
  if (c->q) (void)hipStreamDestroy(c->q);
  delete c;
}

km_status km_set_stream(km_ctx* c, void* stream) {
  if (!c) return KM_EINVAL;
  c->stream = (hipStream_t)stream;
  return KM_OK;
}

km_status km_set_tile_shape(km_ctx* c, km_prec prec, km_xtype xt, int32_t d, int32_t K, int32_t shape) {
  if (!c || (prec != KM_GEMM_F32 && prec != KM_GEMM_BF16) || (xt != KM_X_F32 && xt != KM_X_BF16) ||
      shape < 0 || shape >= KM_TILE_SHAPES)
    return KM_EINVAL;
  int wi, kb;
  if (!tile_slot(prec == KM_GEMM_BF16, d, K, &wi, &kb)) return KM_EINVAL;
  c->tile_shape[prec == KM_GEMM_BF16 ? 1 : 0][xt == KM_X_BF16 ? 1 : 0][wi][kb] = (int8_t)shape;
  return KM_OK;
}

int32_t km_get_tile_shape(const km_ctx* c, km_prec prec, km_xtype xt, int32_t d, int32_t K) {
  if (!c || (prec != KM_GEMM_F32 && prec != KM_GEMM_BF16) || (xt != KM_X_F32 && xt != KM_X_BF16)) return -1;
  int wi, kb;
  if (!tile_slot(prec == KM_GEMM_BF16, d, K, &wi, &kb)) return -1;
  return c->tile_shape[prec == KM_GEMM_BF16 ? 1 : 0][xt == KM_X_BF16 ? 1 : 0][wi][kb];
}

km_status km_set_timing(km_ctx* c, int enable) {
  if (!c) return KM_EINVAL;
  c->timing = enable != 0;
  return KM_OK;
}

void km_opts_default(km_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->eps1 = 0.02;
  o->eps2 = 0.5;
  o->ridge = 1e-10;
  o->m_init = 2;
  o->max_iter = 500;
  o->prec = KM_GEMM_F32;
  o->flags = 0;
  o->trace_C = nullptr;
  o->trace_rec = nullptr;
  o->m_traj = nullptr;
}

km_status kmeans_g(km_ctx* c, const void* X, km_xtype xt, int64_t N, int32_t d, int32_t K,
                   const float* C, km_prec prec, const int32_t* rho_prev, int32_t* rho, float* C_out,
                   double* E, km_g_stats* st) {
  km_status s = g_check(c, X, xt, N, d, K, C, prec, rho_prev, rho, C_out, E);
  if (s != KM_OK) return s;
  Shape want;
  want.N = N; want.d = d; want.K = K; want.cap = 0; want.bf = prec == KM_GEMM_BF16;
  s = ensure_ws(c, want);
  if (s != KM_OK) return s;
  return g_run(c, c->w, X, xt, N, d, K, C, prec, rho_prev, rho, C_out, E, st);
}

km_status kmeans_g_noalloc(km_ctx* c, const void* X, km_xtype xt, int64_t N, int32_t d, int32_t K,
                           const float* C, km_prec prec, const int32_t* rho_prev, int32_t* rho,
                           float* C_out, double* E, km_g_stats* st) {
  km_status s = g_check(c, X, xt, N, d, K, C, prec, rho_prev, rho, C_out, E);
  if (s != KM_OK) return s;
  char* base = (char*)scratch_ptr(c->device);
  if (!base) return fail(c, KM_EDEVICE, "the scratch array of this device was not set up by km_create");
  AssignArgs a{};
  a.N = N; a.d = d; a.K = K; a.xbf16 = xt == KM_X_BF16; a.gemm_bf16 = prec == KM_GEMM_BF16;
  a.shape = shape_for(c, a.gemm_bf16, a.xbf16, d, K);
  const int grid = assign_grid(a);
  if (grid <= 0) return fail(c, KM_EUNSUPPORTED, "no assignment kernel for this shape");
  const size_t need = ws_layout_g(N, d, K, a.gemm_bf16, grid, nullptr, nullptr);
  if (need > (size_t)KM_NOALLOC_SCRATCH_BYTES)
    return fail(c, KM_EUNSUPPORTED, "kmeans_g_noalloc needs " + std::to_string(need) +
                                        " bytes of scratch for this shape; the fixed array holds " +
                                        std::to_string((size_t)KM_NOALLOC_SCRATCH_BYTES));
  Ws w;
  ws_layout_g(N, d, K, a.gemm_bf16, grid, base, &w);
  return g_run(c, w, X, xt, N, d, K, C, prec, rho_prev, rho, C_out, E, st);
}

km_status kmeans_solve(km_ctx* c, const void* X, km_xtype xt, int64_t N, int32_t d, int32_t K,
                       const float* C0, int32_t m_max, double tol, const km_opts* opt_in,
                       float* C_out, int32_t* rho_out, double* E, int32_t* iters,
                       km_solve_stats* st) {
  km_opts opt;
  if (opt_in) opt = *opt_in; else km_opts_default(&opt);
  km_status s = check_common(c, X, xt, N, d, K, opt.prec);
  if (s != KM_OK) return s;
  if (m_max < 0 || m_max > KM_M_MAX_LIMIT) return fail(c, KM_EINVAL, "m_max must be in [0, 64]");
  if (!(tol >= 0.0) || !isfinite(tol)) return fail(c, KM_EINVAL, "tol must be finite and >= 0");
  if (opt.max_iter < 1) return fail(c, KM_EINVAL, "max_iter must be >= 1");
  if (opt.m_init < 0) return fail(c, KM_EINVAL, "m_init must be >= 0");
  if (!(opt.ridge >= 0.0) || !isfinite(opt.ridge) || !isfinite(opt.eps1) || !isfinite(opt.eps2))
    return fail(c, KM_EINVAL, "eps1, eps2 and ridge must be finite (ridge >= 0)");
  if (!E || !iters) return fail(c, KM_EINVAL, "E and iters must be host pointers");
  if (!is_device_ptr(C0) || !is_device_ptr(C_out) || !is_device_ptr(rho_out))
    return fail(c, KM_EINVAL, "C0, C_out and rho_out must be device pointers");
  if (!aligned16(C0) || !aligned16(C_out))
    return fail(c, KM_EINVAL, "C0 and C_out must start on a 16-byte boundary");
  if (opt.trace_C && !is_device_ptr(opt.trace_C)) return fail(c, KM_EINVAL, "trace_C must be a device pointer");
  if (opt.trace_rec && !is_device_ptr(opt.trace_rec))
    return fail(c, KM_EINVAL, "trace_rec must be a device pointer");
  const size_t xbytes = (size_t)N * d * (xt == KM_X_BF16 ? 2 : 4);
  const size_t cbytes = (size_t)K * d * 4;
  if (overlap(C_out, cbytes, X, xbytes) || overlap(rho_out, (size_t)N * 4, X, xbytes) ||
      overlap(rho_out, (size_t)N * 4, C_out, cbytes) || overlap(rho_out, (size_t)N * 4, C0, cbytes))
    return fail(c, KM_EINVAL, "outputs must not alias X or each other");
  HIP_TRY(c, hipSetDevice(c->device), "hipSetDevice");
  const bool gbf = opt.prec == KM_GEMM_BF16;
  // row bounds: float32 GEMM with the centroids resident in the kernel's LDS
  bool bnd = false;
  if (opt.flags & KM_FLAG_BOUNDS) {
    AssignArgs t{};
    t.N = N; t.d = d; t.K = K; t.xbf16 = xt == KM_X_BF16; t.gemm_bf16 = gbf;
    t.shape = shape_for(c, gbf, xt == KM_X_BF16, d, K);
    bnd = assign_bounds_ok(t) != 0;
  }
  Shape want;
  want.N = N; want.d = d; want.K = K; want.cap = m_max; want.bf = gbf;
  want.it = opt.m_traj ? opt.max_iter + 1 : 0;
  want.bnd = bnd ? 1 : 0;
  s = ensure_ws(c, want);
  if (s != KM_OK) return s;
  hipStream_t q = c->q;
  const bool xbf = xt == KM_X_BF16;
  const int cap = m_max;
  const int64_t KD = (int64_t)K * d;

  // controller state
  Ctl h;
  memset(&h, 0, sizeof(h));
  h.m = opt.m_init < m_max ? opt.m_init : m_max;
  h.cand_is_lloyd = 1;
  h.lab_prev = 0; h.lab_cand = 1; h.lab_fb = 2;
  h.max_iter = opt.max_iter;
  h.m_max = m_max;
  h.flags = (int32_t)opt.flags;
  h.eps1 = opt.eps1; h.eps2 = opt.eps2; h.tol = tol; h.ridge = opt.ridge;
  h.E1 = HUGE_VAL; h.E2 = HUGE_VAL;
  h.assign_passes = 1;
  *c->ctl_host = h;
  HIP_TRY(c, hipEventRecord(c->enter, c->stream), "hipEventRecord");
  HIP_TRY(c, hipStreamWaitEvent(q, c->enter, 0), "hipStreamWaitEvent");
  HIP_TRY(c, hipEventRecord(c->t0, q), "hipEventRecord");
  HIP_TRY(c, hipMemcpyAsync(c->w.ctl, c->ctl_host, sizeof(Ctl), hipMemcpyHostToDevice, q), "copy ctl");

  // ---- kernel arguments ----
  AssignArgs a{};
  a.X = X; a.N = N; a.d = d; a.K = K; a.C = c->w.C_tmp; a.nc = c->w.nc_tmp;
  a.Cb = gbf ? c->w.Cb_tmp : nullptr; a.delta = gbf ? c->w.del_tmp : nullptr;
  a.lab = c->w.labels; a.lab_prev = nullptr; a.e_part = c->w.e_part; a.flags = c->w.flags; a.ctl = c->w.ctl;
  a.xbf16 = xbf; a.gemm_bf16 = gbf;
  a.shape = shape_for(c, gbf, xbf, d, K);
  a.lb = bnd ? c->w.lb : nullptr; a.bounds = 0;
  // undecided rows of a deferring kernel: one re-check launch per pass
  a.fl_cnt = assign_list_mode(a) ? c->w.fl_cnt : nullptr;
  const bool relist = a.fl_cnt != nullptr;
  UpdateArgs u{};
  u.X = X; u.N = N; u.d = d; u.K = K; u.xbf16 = xbf;
  u.lab = c->w.labels; u.lab_from_ctl = 1; u.lrank = c->w.lrank; u.blockcount = c->w.blockcount;
  u.counts = c->w.counts; u.seg_start = c->w.seg_start; u.item_start = c->w.item_start;
  u.item_cluster = c->w.item_cluster; u.perm = c->w.perm; u.partial = c->w.partial;
  u.max_items = update_max_items(N, K); u.ctl = c->w.ctl; u.gated = 1;
  u.fx = fx_ok(K, d); u.xbound = c->w.xbound; u.fxpart = c->w.fxpart;
  FinalizeArgs f{};
  f.d = d; f.K = K; f.cap = cap; f.partial = c->w.partial; f.item_start = c->w.item_start;
  f.counts = c->w.counts; f.C_in = c->w.C_tmp; f.C_out = nullptr;
  f.C_cand = c->w.C_cand; f.C_fb = c->w.C_fb;
  f.G_last = c->w.G_last; f.F_last = c->w.F_last; f.ring_dF = c->w.ring_dF; f.ring_dG = c->w.ring_dG;
  f.dots = c->w.dots; f.ctl = c->w.ctl; f.mode = kFinInit;
  f.fx = u.fx; f.fxpart = c->w.fxpart; f.xbound = c->w.xbound; f.N = N;
  f.C_ref = bnd ? c->w.C_ref : nullptr;
  CombineArgs cb{};
  cb.ctl = c->w.ctl; cb.gated = 0; cb.G_last = c->w.G_last; cb.ring_dG = c->w.ring_dG;
  cb.K = K; cb.d = d; cb.cap = cap;
  cb.C_cand = c->w.C_cand; cb.nc_cand = c->w.nc_cand; cb.Cb_cand = gbf ? c->w.Cb_cand : nullptr;
  cb.delta_cand = gbf ? c->w.del_cand : nullptr;
  cb.C_fb = c->w.C_fb; cb.nc_fb = c->w.nc_fb; cb.Cb_fb = gbf ? c->w.Cb_fb : nullptr;
  cb.delta_fb = gbf ? c->w.del_fb : nullptr;
  if (bnd) {   // shifts of the new centroids against the bounds' reference
    cb.C_ref = c->w.C_ref; cb.sh_cand = c->w.shift; cb.sh_fb = c->w.shift + K;
  }

  // ---- prologue: P^0 = Assign(C^0), G^0 = Update(P^0), F^0 = G^0 - C^0, C^1 = G^0 ----
  HIP_TRY(c, hipMemcpyAsync(c->w.C_tmp, C0, cbytes, hipMemcpyDeviceToDevice, q), "copy C0");
  HIP_TRY(c, launch_prep(c->w.C_tmp, K, d, c->w.nc_tmp, gbf ? c->w.Cb_tmp : nullptr,
                         gbf ? c->w.del_tmp : nullptr, q), "prep");
  HIP_TRY(c, launch_assign(a, kRolePlain, q), "assignment");
  if (relist) HIP_TRY(c, launch_recheck(recheck_args(a, c->w.e_part), kRolePlain, q), "re-check");
  HIP_TRY(c, launch_xbound(u, q), "bound of |x|");
  HIP_TRY(c, launch_update_sums(u, q), "update");
  HIP_TRY(c, launch_finalize(f, q), "finalize");
  HIP_TRY(c, launch_combine(cb, q), "combine");
  // counters of the first candidate pass start from zero
  HIP_TRY(c, hipMemcpyAsync(c->w.ctl, c->ctl_host, sizeof(Ctl), hipMemcpyHostToDevice, q), "copy ctl");

  // ---- per-iteration launch sequence ----
  const int grid = assign_grid(a);
  if (grid <= 0) return fail(c, KM_EUNSUPPORTED, "no assignment kernel for this shape");
  // energy partials of a pass: the assignment's workgroups, then the re-check's
  const int n_part = grid + (relist ? kReGrid : 0);
  AssignArgs ac = a;
  ac.C = c->w.C_cand; ac.nc = c->w.nc_cand; ac.Cb = gbf ? c->w.Cb_cand : nullptr;
  ac.delta = gbf ? c->w.del_cand : nullptr; ac.e_part = c->w.e_part; ac.bounds = bnd ? 1 : 0;
  ac.shift = bnd ? c->w.shift : nullptr;
  AssignArgs af = a;
  af.C = c->w.C_fb; af.nc = c->w.nc_fb; af.Cb = gbf ? c->w.Cb_fb : nullptr;
  af.delta = gbf ? c->w.del_fb : nullptr; af.e_part = c->w.e_part + n_part; af.bounds = bnd ? 1 : 0;
  af.shift = bnd ? c->w.shift + K : nullptr;
  const RecheckArgs rc = recheck_args(ac, c->w.e_part + grid);
  const RecheckArgs rf = recheck_args(af, c->w.e_part + n_part + grid);
  FinalizeArgs fi = f;
  fi.mode = kFinIter; fi.C_in = nullptr;
  CombineArgs ci = cb;
  ci.gated = 1;
  ci.dots = c->w.dots; ci.n_dots = finalize_grid_for(u.fx, K, d); ci.gram = c->w.gram; ci.trace_rec = opt.trace_rec;

  // Each iteration is launched directly on the stream (a graph launch left
  // the device idle for about 13 us at every iteration boundary; kernels
  // launched back to back start without a gap while the host stays ahead).
  // The host keeps two iterations in flight.
  CtlArgs k1{};
  k1.ctl = c->w.ctl; k1.e_part = c->w.e_part; k1.n_part = n_part; k1.stage = 1;
  k1.tr.trace_C = opt.trace_C; k1.tr.trace_rec = opt.trace_rec; k1.tr.C_cand = c->w.C_cand;
  k1.tr.K = K; k1.tr.d = d;
  k1.tr.m_traj = opt.m_traj ? c->w.m_traj : nullptr;
  CtlArgs k2 = k1;
  k2.e_part = c->w.e_part + n_part; k2.stage = 2; k2.tr.trace_C = nullptr;

  // The combine kernel, last of the iteration, writes the done flag into
  // pinned slot p.  An event taken by a dispatch still idles the device for a
  // few microseconds, so one event per iteration tells the host that the
  // previous iteration is complete: with timing on, the start event of the
  // candidate assignment (which also times it); with timing off, the end
  // event of the combine.
  int* done_dev = nullptr;
  HIP_TRY(c, hipHostGetDevicePointer((void**)&done_dev, c->done_host, 0), "hipHostGetDevicePointer");
  auto enqueue_iteration = [&](int p) -> km_status {
    CombineArgs cp = ci;
    cp.done_out = done_dev + p;
    // with timing on, ta/tb take the candidate assignment's own start and end
    // (the end of its re-check in list mode)
    HIP_TRY(c, launch_assign(ac, kRoleCand, q, c->timing ? c->ta[p] : nullptr,
                             (c->timing && !relist) ? c->tb[p] : nullptr),
            "assignment");
    if (relist) HIP_TRY(c, launch_recheck(rc, kRoleCand, q, c->timing ? c->tb[p] : nullptr), "re-check");
    HIP_TRY(c, launch_controller(k1, q), "controller");
    HIP_TRY(c, launch_assign(af, kRoleFallback, q), "assignment");
    if (relist) HIP_TRY(c, launch_recheck(rf, kRoleFallback, q), "re-check");
    HIP_TRY(c, launch_controller(k2, q), "controller");
    HIP_TRY(c, launch_update_sums(u, q), "update");
    HIP_TRY(c, launch_finalize(fi, q), "finalize");
    HIP_TRY(c, launch_combine(cp, q, c->timing ? nullptr : c->poll_ev[p]), "combine");
    return KM_OK;
  };

  std::vector<float> it_ms;
  it_ms.reserve(64);
  int launched = 0;
  bool finished = false;
  while (launched < opt.max_iter && !finished) {
    const int it = launched;
    const int p = it & 1;
    const km_status es = enqueue_iteration(p);
    if (es != KM_OK) return es;
    if (it >= 1) {
      const int pp = (it - 1) & 1;
      // iteration it - 1 is complete once iteration it has started
      HIP_TRY(c, hipEventSynchronize(c->timing ? c->ta[p] : c->poll_ev[pp]), "hipEventSynchronize");
      if (c->timing) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ta[pp], c->tb[pp]) != hipSuccess) {
          clear_pending_error();
          ms = -1.f;
        }
        it_ms.push_back(ms);
      }
      if (((volatile int*)c->done_host)[pp]) finished = true;
    }
    ++launched;
  }
  HIP_TRY(c, hipMemcpyAsync(c->ctl_host, c->w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, q), "copy ctl");
  HIP_TRY(c, hipStreamSynchronize(q), "hipStreamSynchronize");
  if (c->timing && !finished) {  // the last launched iteration was not inspected in the loop
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ta[(launched - 1) & 1], c->tb[(launched - 1) & 1]) != hipSuccess) {
      clear_pending_error();
      ms = -1.f;
    }
    it_ms.push_back(ms);
  }
  Ctl r = *c->ctl_host;
  if (!r.done) return fail(c, KM_EDEVICE, "solver did not reach a final state");
  const float* Cres = r.acc_src == 1 ? c->w.C_fb : c->w.C_cand;
  HIP_TRY(c, hipMemcpyAsync(C_out, Cres, cbytes, hipMemcpyDeviceToDevice, q), "copy C");
  HIP_TRY(c, hipMemcpyAsync(rho_out, c->w.labels + (size_t)r.lab_prev * N, (size_t)N * 4,
                            hipMemcpyDeviceToDevice, q), "copy rho");
  if (opt.m_traj && r.t > 0)
    HIP_TRY(c, hipMemcpyAsync(opt.m_traj + 1, c->w.m_traj + 1, (size_t)r.t * 4, hipMemcpyDeviceToHost, q),
            "copy m trajectory");
  HIP_TRY(c, hipEventRecord(c->t1, q), "hipEventRecord");
  HIP_TRY(c, hipStreamSynchronize(q), "hipStreamSynchronize");
  *E = r.E_acc;
  *iters = r.t;
  if (opt.m_traj) opt.m_traj[0] = opt.m_init < m_max ? opt.m_init : m_max;
  if (st) {
    memset(st, 0, sizeof(*st));
    st->iters = r.t;
    st->accepted = r.accepted;
    st->rejected = r.rejected;
    st->assign_passes = r.assign_passes;
    st->m_final = r.m;
    st->recheck_rows = (int64_t)r.flagged_total;
    st->near_tie_rows = (int64_t)r.near_total;
    st->gemm_rows = (int64_t)r.gemm_total + N;   // the prologue pass assigns every row
    st->bounds = bnd ? 1 : 0;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->t0, c->t1) == hipSuccess) st->device_ms = ms;
    else clear_pending_error();
    if (c->timing) {
      double sum = 0.0;
      int n = 0;
      for (int it = 0; it < r.t && it < (int)it_ms.size(); ++it) {
        if (it_ms[it] >= 0.f) {
          sum += it_ms[it];
          ++n;
        }
      }
      st->assign_ms = sum;
      st->assign_launches = n;
    }
  }
  if (r.status == KM_ENONFINITE) return fail(c, KM_ENONFINITE, "energy is not finite");
  return (km_status)r.status;
}

}  // extern "C"
