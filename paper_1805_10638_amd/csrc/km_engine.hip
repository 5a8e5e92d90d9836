// Batch engine: many instances of Algorithm 1 advanced together (batched
// solving and continuous-batching service).
//
// Every active job owns a workspace (km_ws.h) and the argument structs of
// each kernel of the solver.  The structs of all active jobs are packed into
// device tables; one iteration is then a fixed sequence of batched launches
// whose grids are the concatenation of per-job slices (km_common.h,
// batch_find):
//   candidate assignment (one launch per assignment kernel variant),
//   controller stage 1, fall-back assignment, controller stage 2,
//   update (rank, scan, offsets, scatter, segmented sums), finalisation,
//   Anderson combination, and a gather of the jobs' done flags.
// A finished job's kernels return at once (they read its done flag), so
// the set only has to change when enough jobs have finished or a queued job
// can be admitted; the engine then drains its stream, frees the workspaces
// of finished jobs, admits queued jobs that fit the budget, runs their
// prologue (P^0 = Assign(C^0), G^0, C^1 = G^0) as batched launches and
// rebuilds the tables (and the two iteration graphs).

#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <vector>

#include "km_ctx.h"

namespace {

// Copy a finished job's accepted iterate and its labels to the job outputs.
__global__ __launch_bounds__(256) void k_finish(const Ctl* ctl, const float* C_cand, const float* C_fb,
                                                int64_t KD, const int* labels, int64_t N, float* C_out,
                                                int* rho_out) {
  const float* Cr = ctl->acc_src == 1 ? C_fb : C_cand;
  const int* L = labels + (int64_t)ctl->lab_prev * N;
  const int64_t stride = (int64_t)gridDim.x * 256;
  const int64_t t0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int64_t i = t0; i < KD; i += stride) C_out[i] = Cr[i];
  for (int64_t i = t0; i < N; i += stride) rho_out[i] = L[i];
}

__global__ __launch_bounds__(256) void k_gather_done(Ctl* const* ctls, int n, int* out) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) out[i] = ctls[i]->done;
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

enum JobState { kQueued = 0, kActive = 1, kFinishing = 2, kReady = 3 };

struct Job {
  km_job spec{};
  int64_t ticket = 0;
  Shape shape;
  bool gbf = false, xbf = false;
  size_t bytes = 0;       // workspace (allocated at admission)
  size_t footprint = 0;   // what the HBM budget counts: workspace + X + C0 + C_out + labels
  void* mem = nullptr;
  Ws w;
  KernelPick pick;
  int assign_blocks = 0;
  Ctl* ctl_host = nullptr;     // pinned: initial state, then the final state
  hipEvent_t ev = nullptr;     // finishing copies done
  JobState state = kQueued;
  bool done_dev = false;       // seen done on the device
  bool taken = false;          // result returned by km_engine_poll
  double t_submit = 0.0;
  km_job_result res{};
};

}  // namespace

struct km_engine {
  km_ctx* ctx = nullptr;
  hipStream_t q = nullptr;
  int m_max = 0;
  double tol = 0.0;
  km_opts opt{};
  int64_t budget = 0, used = 0;
  bool graphs = true;
  int64_t next_ticket = 0;

  std::deque<Job*> queued;
  std::vector<Job*> active;      // table order
  std::deque<Job*> finishing;
  std::deque<Job*> ready;
  bool change = true;            // membership must be rebuilt before the next launch

  // Device tables of the active set (and the prologue of newly admitted
  // jobs).  Two buffers alternate so that new tables can be uploaded while
  // iterations that read the previous ones are still in flight; tab_ev[k]
  // marks the end of the work that used buffer k.  Each has a pinned
  // staging buffer for the asynchronous upload.
  char* dtab = nullptr;          // current buffer
  char* dbuf[2] = {nullptr, nullptr};
  size_t dcap[2] = {0, 0};
  char* stage[2] = {nullptr, nullptr};
  size_t scap[2] = {0, 0};
  hipEvent_t tab_ev[2] = {nullptr, nullptr};
  int cur = 0;
  std::vector<hipGraphExec_t> old_graphs;   // replaced while possibly in flight
  int64_t drains = 0, appends = 0;
  double rebuild_ms = 0.0;
  struct Bucket {
    KernelPick pick;
    size_t o_cand = 0, o_fb = 0, o_pre = 0;
    int n = 0, blocks = 0;
    size_t lds = 0;
  };
  std::vector<Bucket> it_buckets;
  // pass-wide re-checks of the jobs whose assignment leaves listed rows
  size_t o_rc = 0, o_rf = 0, o_rpre = 0, rl_lds = 0;
  int n_rl = 0, rl_blocks = 0;
  size_t o_k1 = 0, o_k2 = 0, o_u = 0, o_upre[kUpdateKinds] = {}, o_fi = 0, o_fpre = 0, o_fxpre = 0, o_cb = 0, o_cpre = 0, o_ctls = 0;
  int ublocks[kUpdateKinds] = {}, fblocks = 0, fxblocks = 0, cblocks = 0, n_it = 0;

  // Up to kSlots iterations in flight, each with its slot of done flags
  // (pinned), its poll event and its graph.
  static constexpr int kSlots = 3;
  int* hdone = nullptr;
  int* ddone = nullptr;
  size_t done_cap = 0;
  hipEvent_t poll_ev[kSlots] = {};
  std::deque<std::pair<int, int>> inflight;   // (slot, jobs in its tables) of unharvested iterations
  int slot = 0;
  hipGraphExec_t gexec[kSlots] = {};
  int64_t iterations = 0;
  double share = 1.0;            // fraction of resident assignment workgroups to use
};

namespace {

km_status efail(km_engine* e, km_status s, const std::string& m) { return fail(e->ctx, s, m); }

void free_job(Job* j) {
  if (j->ev) (void)hipEventDestroy(j->ev);
  if (j->ctl_host) (void)hipHostFree(j->ctl_host);
  delete j;
}


#define ENG_TRY(e, expr, where)                              \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) return hip_fail((e)->ctx, _e, where); \
  } while (0)

// Host table under construction: arrays appended at 256-byte offsets.
struct Packer {
  std::vector<char> buf;
  template <class T>
  size_t add(const std::vector<T>& v) {
    const size_t o = ws_up(buf.size());
    buf.resize(o + std::max<size_t>(v.size() * sizeof(T), 1));
    if (!v.empty()) memcpy(buf.data() + o, v.data(), v.size() * sizeof(T));
    return o;
  }
};

std::vector<int> prefix_of(const std::vector<int>& sizes, int* total) {
  std::vector<int> p(sizes.size() + 1, 0);
  for (size_t i = 0; i < sizes.size(); ++i) p[i + 1] = p[i] + sizes[i];
  *total = p.back();
  return p;
}

Shape job_shape(const km_job& j, int m_max, bool gbf) {
  Shape s;
  s.N = j.N; s.d = j.d; s.K = j.K; s.cap = m_max; s.bf = gbf ? 1 : 0;
  return s;
}

// Workgroups of each job's assignment pass: a share of the device's resident
// workgroups for that kernel proportional to the job's work (rows x padded
// K), at least one, at most its row groups.  With frac = 1 the launches ask
// for twice the resident workgroups (balance); with frac < 1 for that
// fraction of them, leaving the rest of the device to other streams.
void size_assignment(const std::vector<Job*>& jobs, double frac) {
  struct Acc { double work = 0.0; int64_t cap = 0; };
  std::vector<std::pair<const void*, Acc>> acc;
  auto find = [&](const void* fn) -> Acc& {
    for (auto& p : acc) if (p.first == fn) return p.second;
    acc.push_back({fn, Acc()});
    return acc.back().second;
  };
  for (Job* j : jobs) {
    Acc& a = find(j->pick.fn);
    a.work += (double)j->spec.N * (double)((j->spec.K + 15) & ~15);
    if (a.cap == 0) a.cap = assign_resident(j->pick, (int64_t)1 << 40, 1.0);
  }
  for (Job* j : jobs) {
    const Acc& a = find(j->pick.fn);
    const int64_t groups = (j->spec.N + j->pick.rows - 1) / j->pick.rows;
    const double share = (double)j->spec.N * (double)((j->spec.K + 15) & ~15) / a.work;
    const double total = frac >= 1.0 ? 2.0 * (double)a.cap : frac * (double)a.cap;
    int64_t b = (int64_t)(total * share + 0.5);
    if (b < 1) b = 1;
    if (b > groups) b = groups;
    j->assign_blocks = (int)b;
  }
}

// Initial controller state of a job (the same as kmeans_solve's).
void init_ctl(km_engine* e, Job* j) {
  const int cap = e->m_max;
  Ctl h;
  memset(&h, 0, sizeof(h));
  h.m = e->opt.m_init < cap ? e->opt.m_init : cap;
  h.cand_is_lloyd = 1;
  h.lab_prev = 0; h.lab_cand = 1; h.lab_fb = 2;
  h.max_iter = e->opt.max_iter;
  h.m_max = cap;
  h.flags = (int32_t)e->opt.flags;
  h.eps1 = e->opt.eps1; h.eps2 = e->opt.eps2; h.tol = e->tol; h.ridge = e->opt.ridge;
  h.E1 = HUGE_VAL; h.E2 = HUGE_VAL;
  h.assign_passes = 1;
  *j->ctl_host = h;
}

struct JobArgs {
  AssignArgs plain, cand, fb;
  bool relist = false;    // candidate and fall-back rows the GEMM cannot decide go to a re-check launch
  int rgrid = 0;          // workgroups of its re-check (and energy partials it adds)
  RecheckArgs rc, rf;
  UpdateArgs u;
  FinalizeArgs f_init, f_iter;
  CombineArgs c0, c1;
  CtlArgs k1, k2;
  PrepArgs prep;
};

JobArgs job_args(const km_engine* e, const Job* j) {
  const km_job& s = j->spec;
  const Ws& w = j->w;
  const bool gbf = j->gbf;
  JobArgs r;
  AssignArgs a{};
  a.X = s.X; a.N = s.N; a.d = s.d; a.K = s.K; a.C = w.C_tmp; a.nc = w.nc_tmp;
  a.Cb = gbf ? w.Cb_tmp : nullptr; a.delta = gbf ? w.del_tmp : nullptr;
  a.lab = w.labels; a.lab_prev = nullptr; a.e_part = w.e_part; a.flags = w.flags; a.ctl = w.ctl;
  a.xbf16 = j->xbf; a.gemm_bf16 = gbf; a.shape = 0; a.role = kRolePlain;
  r.plain = a;
  r.cand = a;
  r.cand.C = w.C_cand; r.cand.nc = w.nc_cand; r.cand.Cb = gbf ? w.Cb_cand : nullptr;
  r.cand.delta = gbf ? w.del_cand : nullptr; r.cand.role = kRoleCand;
  r.fb = a;
  r.fb.C = w.C_fb; r.fb.nc = w.nc_fb; r.fb.Cb = gbf ? w.Cb_fb : nullptr;
  r.fb.delta = gbf ? w.del_fb : nullptr; r.fb.e_part = w.e_part + j->assign_blocks; r.fb.role = kRoleFallback;
  // Kernels that defer undecided rows (bfloat16 GEMM, centroids streamed
  // through LDS) leave them listed for one batched re-check per pass, as in
  // kmeans_solve, instead of re-checking them inside the assignment: the
  // re-check's float32 MFMA filter computes float64 distances for few
  // centroids.  The re-check gets a workgroup per 4096 rows (8 to kReGrid),
  // and the energy partials of a pass are the assignment's G and its rgrid.
  const int G = j->assign_blocks;
  int n_part = G;
  r.relist = (gbf || !j->pick.resident) && G <= kReMaxGrid;
  if (r.relist) {
    const int64_t rg = s.N / 4096;
    r.rgrid = rg < 8 ? 8 : (rg > kReGrid ? kReGrid : (int)rg);
    n_part = G + r.rgrid;
    r.cand.fl_cnt = w.fl_cnt;
    r.fb.fl_cnt = w.fl_cnt;
    r.fb.e_part = w.e_part + n_part;
    RecheckArgs rr{};
    rr.X = s.X; rr.N = s.N; rr.d = s.d; rr.K = s.K; rr.xbf16 = j->xbf;
    rr.lab = w.labels; rr.lab_prev = nullptr; rr.flags = w.flags; rr.fl_cnt = w.fl_cnt;
    rr.grid = G; rr.W = j->pick.threads / 64; rr.group_rows = j->pick.rows; rr.sb16 = j->pick.rows / rr.W;
    rr.ctl = w.ctl;
    r.rc = rr;
    r.rc.C = w.C_cand; r.rc.nc = w.nc_cand; r.rc.e_part = w.e_part + G; r.rc.role = kRoleCand;
    r.rf = rr;
    r.rf.C = w.C_fb; r.rf.nc = w.nc_fb; r.rf.e_part = w.e_part + n_part + G; r.rf.role = kRoleFallback;
  }

  UpdateArgs u{};
  u.X = s.X; u.N = s.N; u.d = s.d; u.K = s.K; u.xbf16 = j->xbf;
  u.lab = w.labels; u.lab_from_ctl = 1; u.lrank = w.lrank; u.blockcount = w.blockcount;
  u.counts = w.counts; u.seg_start = w.seg_start; u.item_start = w.item_start;
  u.item_cluster = w.item_cluster; u.perm = w.perm; u.partial = w.partial;
  u.max_items = update_max_items(s.N, s.K); u.ctl = w.ctl; u.gated = 1;
  u.fx = fx_ok(s.K, s.d); u.xbound = w.xbound; u.fxpart = w.fxpart;
  r.u = u;

  FinalizeArgs f{};
  f.d = s.d; f.K = s.K; f.cap = e->m_max; f.partial = w.partial; f.item_start = w.item_start;
  f.counts = w.counts; f.C_in = w.C_tmp; f.C_out = nullptr;
  f.C_cand = w.C_cand; f.C_fb = w.C_fb;
  f.G_last = w.G_last; f.F_last = w.F_last; f.ring_dF = w.ring_dF; f.ring_dG = w.ring_dG;
  f.dots = w.dots; f.ctl = w.ctl; f.mode = kFinInit;
  f.fx = u.fx; f.fxpart = w.fxpart; f.xbound = w.xbound; f.N = s.N;
  r.f_init = f;
  r.f_iter = f;
  r.f_iter.mode = kFinIter; r.f_iter.C_in = nullptr;

  CombineArgs cb{};
  cb.ctl = w.ctl; cb.gated = 0; cb.G_last = w.G_last; cb.ring_dG = w.ring_dG;
  cb.K = s.K; cb.d = s.d; cb.cap = e->m_max;
  cb.C_cand = w.C_cand; cb.nc_cand = w.nc_cand; cb.Cb_cand = gbf ? w.Cb_cand : nullptr;
  cb.delta_cand = gbf ? w.del_cand : nullptr;
  cb.C_fb = w.C_fb; cb.nc_fb = w.nc_fb; cb.Cb_fb = gbf ? w.Cb_fb : nullptr;
  cb.delta_fb = gbf ? w.del_fb : nullptr;
  r.c0 = cb;
  r.c1 = cb;
  r.c1.gated = 1; r.c1.dots = w.dots; r.c1.n_dots = finalize_grid_for(u.fx, s.K, s.d); r.c1.gram = w.gram;
  r.c1.trace_rec = nullptr;

  CtlArgs k{};
  k.ctl = w.ctl; k.e_part = w.e_part; k.n_part = n_part; k.stage = 1;
  k.tr.trace_C = nullptr; k.tr.trace_rec = nullptr; k.tr.C_cand = w.C_cand; k.tr.K = s.K; k.tr.d = s.d;
  r.k1 = k;
  r.k2 = k;
  r.k2.e_part = w.e_part + n_part; r.k2.stage = 2;

  r.prep = PrepArgs{w.C_tmp, s.K, s.d, w.nc_tmp, gbf ? w.Cb_tmp : nullptr, gbf ? w.del_tmp : nullptr};
  return r;
}

// Assignment buckets (one per kernel variant) of a job list.
struct HostBucket {
  KernelPick pick;
  std::vector<AssignArgs> a, b;
  std::vector<int> sizes;
  size_t lds = 0;
};

void add_bucket(std::vector<HostBucket>& bs, const KernelPick& p, const AssignArgs& a, const AssignArgs* b,
                int blocks) {
  HostBucket* hb = nullptr;
  for (auto& x : bs) if (x.pick.fn == p.fn) hb = &x;
  if (!hb) {
    bs.push_back(HostBucket());
    hb = &bs.back();
    hb->pick = p;
  }
  hb->a.push_back(a);
  if (b) hb->b.push_back(*b);
  hb->sizes.push_back(blocks);
  hb->lds = std::max(hb->lds, p.lds);
}

// Upload new tables into the other buffer, after the work that last used it.
km_status upload(km_engine* e, const Packer& pk) {
  const int k = e->cur ^ 1;
  ENG_TRY(e, hipEventRecord(e->tab_ev[e->cur], e->q), "hipEventRecord");
  ENG_TRY(e, hipEventSynchronize(e->tab_ev[k]), "hipEventSynchronize");
  const size_t need = pk.buf.size();
  if (need > e->dcap[k]) {
    if (e->dbuf[k]) ENG_TRY(e, hipFree(e->dbuf[k]), "hipFree");
    e->dbuf[k] = nullptr;
    const size_t cap = std::max<size_t>(need * 2, 1 << 20);
    ENG_TRY(e, hipMalloc((void**)&e->dbuf[k], cap), "hipMalloc");
    e->dcap[k] = cap;
  }
  if (need > e->scap[k]) {
    if (e->stage[k]) ENG_TRY(e, hipHostFree(e->stage[k]), "hipHostFree");
    e->stage[k] = nullptr;
    const size_t cap = std::max<size_t>(need * 2, 1 << 20);
    ENG_TRY(e, hipHostMalloc((void**)&e->stage[k], cap, hipHostMallocDefault), "hipHostMalloc");
    e->scap[k] = cap;
  }
  memcpy(e->stage[k], pk.buf.data(), need);
  ENG_TRY(e, hipMemcpyAsync(e->dbuf[k], e->stage[k], need, hipMemcpyHostToDevice, e->q), "table upload");
  e->cur = k;
  e->dtab = e->dbuf[k];
  return KM_OK;
}

template <class T>
const T* dptr(const km_engine* e, size_t o) { return (const T*)(e->dtab + o); }

// One iteration of every job in the tables; done flags into hdone[p].
km_status enqueue_iteration(km_engine* e, int p) {
  hipStream_t q = e->q;
  for (const auto& b : e->it_buckets)
    ENG_TRY(e, launch_assign_batch(b.pick, dptr<AssignArgs>(e, b.o_cand), dptr<int>(e, b.o_pre), b.n, b.blocks,
                                   b.lds, q), "batched assignment");
  if (e->n_rl > 0)
    ENG_TRY(e, launch_recheck_batch(dptr<RecheckArgs>(e, e->o_rc), dptr<int>(e, e->o_rpre), e->n_rl, e->rl_blocks,
                                    e->rl_lds, q), "batched re-check");
  ENG_TRY(e, launch_controller_batch(dptr<CtlArgs>(e, e->o_k1), e->n_it, q), "batched controller");
  for (const auto& b : e->it_buckets)
    ENG_TRY(e, launch_assign_batch(b.pick, dptr<AssignArgs>(e, b.o_fb), dptr<int>(e, b.o_pre), b.n, b.blocks,
                                   b.lds, q), "batched assignment");
  if (e->n_rl > 0)
    ENG_TRY(e, launch_recheck_batch(dptr<RecheckArgs>(e, e->o_rf), dptr<int>(e, e->o_rpre), e->n_rl, e->rl_blocks,
                                    e->rl_lds, q), "batched re-check");
  ENG_TRY(e, launch_controller_batch(dptr<CtlArgs>(e, e->o_k2), e->n_it, q), "batched controller");
  UpdateBatch ub;
  ub.tab = dptr<UpdateArgs>(e, e->o_u);
  for (int k = 0; k < kUpdateKinds; ++k) { ub.prefix[k] = dptr<int>(e, e->o_upre[k]); ub.blocks[k] = e->ublocks[k]; }
  ub.n = e->n_it;
  ENG_TRY(e, launch_update_sums_batch(ub, q), "batched update");
  ENG_TRY(e, launch_finalize_batch(dptr<FinalizeArgs>(e, e->o_fi), dptr<int>(e, e->o_fpre), e->fblocks,
                                   dptr<int>(e, e->o_fxpre), e->fxblocks, e->n_it, q),
          "batched finalize");
  ENG_TRY(e, launch_combine_batch(dptr<CombineArgs>(e, e->o_cb), dptr<int>(e, e->o_cpre), e->n_it, e->cblocks, q),
          "batched combine");
  clear_pending_error();
  hipLaunchKernelGGL(k_gather_done, dim3((e->n_it + 255) / 256), dim3(256), 0, q, (Ctl* const*)(e->dtab + e->o_ctls),
                     e->n_it, e->ddone);
  ENG_TRY(e, hipGetLastError(), "done flags");
  ENG_TRY(e, hipMemcpyAsync(e->hdone + (size_t)p * e->done_cap, e->ddone, (size_t)e->n_it * sizeof(int),
                            hipMemcpyDeviceToHost, q), "done flags copy");
  return KM_OK;
}

void drop_graphs(km_engine* e) {
  for (hipGraphExec_t& g : e->gexec) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  for (hipGraphExec_t g : e->old_graphs) (void)hipGraphExecDestroy(g);
  e->old_graphs.clear();
}

constexpr size_t kDoneCap = 4096;   // jobs in the tables between two drains

// Admit queued jobs, run their prologue and rebuild the iteration tables.
// drain = true: called with nothing in flight; the stream is drained and
// finished jobs are retired first.  drain = false: iterations may be in
// flight; admitted jobs are appended after the current ones (whose table
// positions stay valid for the iterations in flight) and nothing is freed.
km_status rebuild(km_engine* e, bool drain) {
  const double t_in = now_ms();
  if (drain) {
    ENG_TRY(e, hipStreamSynchronize(e->q), "hipStreamSynchronize");
    drop_graphs(e);
    // retire finished jobs (their finishing copies were enqueued before the drain)
    std::vector<Job*> keep;
    for (Job* j : e->active) {
      if (j->state == kActive) {
        keep.push_back(j);
        continue;
      }
      if (j->mem) {
        ENG_TRY(e, hipFreeAsync(j->mem, e->q), "hipFreeAsync");
        j->mem = nullptr;
        e->used -= (int64_t)j->footprint;
      }
      if (j->taken) free_job(j);
    }
    e->active.swap(keep);
  }
  if (!e->queued.empty()) {  // job inputs come from work on the context's stream
    km_ctx* c = e->ctx;
    ENG_TRY(e, hipEventRecord(c->enter, c->stream), "hipEventRecord");
    ENG_TRY(e, hipStreamWaitEvent(e->q, c->enter, 0), "hipStreamWaitEvent");
  }
  // admission in submission order while the workspace fits
  std::vector<Job*> admitted;
  while (!e->queued.empty() && e->active.size() + admitted.size() < kDoneCap) {
    Job* j = e->queued.front();
    if (e->budget > 0 && e->used + (int64_t)j->footprint > e->budget) break;
    e->queued.pop_front();
    hipError_t he = hipMallocAsync(&j->mem, j->bytes, e->q);
    if (he != hipSuccess) {
      clear_pending_error();
      e->queued.push_front(j);
      if (e->active.empty() && admitted.empty())
        return efail(e, KM_ENOMEM, "workspace allocation of a job failed");
      break;
    }
    ENG_TRY(e, hipMemsetAsync(j->mem, 0, j->bytes, e->q), "hipMemsetAsync");
    e->used += (int64_t)j->footprint;
    ws_layout(j->shape, (char*)j->mem, &j->w);
    j->state = kActive;
    admitted.push_back(j);
  }
  if (!drain && admitted.empty()) return KM_OK;
  std::vector<Job*> all = e->active;
  all.insert(all.end(), admitted.begin(), admitted.end());
  size_assignment(all, e->share);

  Packer pk;
  // ---- prologue tables of the admitted jobs ----
  const int na = (int)admitted.size();
  std::vector<JobArgs> aa;
  for (Job* j : admitted) aa.push_back(job_args(e, j));
  std::vector<HostBucket> pb;
  std::vector<PrepArgs> prep;
  std::vector<int> prep_sz;
  std::vector<UpdateArgs> pu;
  std::vector<int> pusz[kUpdateKinds];
  std::vector<FinalizeArgs> pf;
  std::vector<int> pfsz, pfxsz;   // finalisation workgroups: counting-sort, fixed-point instances
  std::vector<CombineArgs> pc;
  std::vector<int> pcsz;
  for (int i = 0; i < na; ++i) {
    Job* j = admitted[i];
    prep.push_back(aa[i].prep);
    prep_sz.push_back(prep_grid(j->spec.K));
    add_bucket(pb, j->pick, aa[i].plain, nullptr, j->assign_blocks);
    pu.push_back(aa[i].u);
    for (int k = 0; k < kUpdateKinds; ++k) pusz[k].push_back(update_grid(aa[i].u, k));
    pf.push_back(aa[i].f_init);
    pfsz.push_back(aa[i].u.fx ? 0 : finalize_grid_for(0, j->spec.K, j->spec.d));
    pfxsz.push_back(aa[i].u.fx ? finalize_grid_for(1, j->spec.K, j->spec.d) : 0);
    pc.push_back(aa[i].c0);
    pcsz.push_back(combine_grid(j->spec.K));
  }
  int prep_blocks = 0, pub[kUpdateKinds] = {}, pfb = 0, pfxb = 0, pcb = 0;
  const size_t o_prep = pk.add(prep), o_prep_pre = pk.add(prefix_of(prep_sz, &prep_blocks));
  std::vector<size_t> o_pb, o_pb_pre;
  std::vector<int> pb_blocks;
  for (auto& b : pb) {
    int t = 0;
    o_pb.push_back(pk.add(b.a));
    o_pb_pre.push_back(pk.add(prefix_of(b.sizes, &t)));
    pb_blocks.push_back(t);
  }
  const size_t o_pu = pk.add(pu);
  size_t o_pupre[kUpdateKinds];
  for (int k = 0; k < kUpdateKinds; ++k) o_pupre[k] = pk.add(prefix_of(pusz[k], &pub[k]));
  const size_t o_pf = pk.add(pf), o_pfpre = pk.add(prefix_of(pfsz, &pfb)), o_pfxpre = pk.add(prefix_of(pfxsz, &pfxb));
  const size_t o_pc = pk.add(pc), o_pcpre = pk.add(prefix_of(pcsz, &pcb));

  // ---- iteration tables of all jobs ----
  std::vector<HostBucket> ib;
  std::vector<CtlArgs> k1, k2;
  std::vector<UpdateArgs> iu;
  std::vector<int> iusz[kUpdateKinds];
  std::vector<FinalizeArgs> fi;
  std::vector<int> fisz, fixsz;
  std::vector<CombineArgs> ci;
  std::vector<int> cisz;
  std::vector<Ctl*> ctls;
  std::vector<RecheckArgs> rcs, rfs;
  std::vector<int> rlsz;
  size_t rl_lds = 0;
  for (Job* j : all) {
    const JobArgs r = job_args(e, j);
    add_bucket(ib, j->pick, r.cand, &r.fb, j->assign_blocks);
    if (r.relist) {
      rcs.push_back(r.rc);
      rfs.push_back(r.rf);
      rlsz.push_back(r.rgrid);
      rl_lds = std::max(rl_lds, recheck_lds(j->spec.d, j->assign_blocks));
    }
    k1.push_back(r.k1);
    k2.push_back(r.k2);
    iu.push_back(r.u);
    for (int k = 0; k < kUpdateKinds; ++k) iusz[k].push_back(update_grid(r.u, k));
    fi.push_back(r.f_iter);
    fisz.push_back(r.u.fx ? 0 : finalize_grid_for(0, j->spec.K, j->spec.d));
    fixsz.push_back(r.u.fx ? finalize_grid_for(1, j->spec.K, j->spec.d) : 0);
    ci.push_back(r.c1);
    cisz.push_back(combine_grid(j->spec.K));
    ctls.push_back(j->w.ctl);
  }
  e->it_buckets.clear();
  for (auto& b : ib) {
    km_engine::Bucket eb;
    eb.pick = b.pick;
    eb.o_cand = pk.add(b.a);
    eb.o_fb = pk.add(b.b);
    eb.o_pre = pk.add(prefix_of(b.sizes, &eb.blocks));
    eb.n = (int)b.a.size();
    eb.lds = b.lds;
    e->it_buckets.push_back(eb);
  }
  e->n_rl = (int)rcs.size();
  e->rl_lds = rl_lds;
  if (e->n_rl > 0) {
    e->o_rc = pk.add(rcs);
    e->o_rf = pk.add(rfs);
    e->o_rpre = pk.add(prefix_of(rlsz, &e->rl_blocks));
  }
  e->o_k1 = pk.add(k1);
  e->o_k2 = pk.add(k2);
  e->o_u = pk.add(iu);
  for (int k = 0; k < kUpdateKinds; ++k) e->o_upre[k] = pk.add(prefix_of(iusz[k], &e->ublocks[k]));
  e->o_fi = pk.add(fi);
  e->o_fpre = pk.add(prefix_of(fisz, &e->fblocks));
  e->o_fxpre = pk.add(prefix_of(fixsz, &e->fxblocks));
  e->o_cb = pk.add(ci);
  e->o_cpre = pk.add(prefix_of(cisz, &e->cblocks));
  e->o_ctls = pk.add(ctls);
  e->n_it = (int)all.size();
  km_status st = upload(e, pk);
  if (st != KM_OK) return st;

  // done-flag buffers (allocated once, for kDoneCap jobs)
  if (!e->hdone) {
    ENG_TRY(e, hipHostMalloc((void**)&e->hdone, km_engine::kSlots * kDoneCap * sizeof(int), hipHostMallocDefault),
            "hipHostMalloc");
    ENG_TRY(e, hipMalloc((void**)&e->ddone, kDoneCap * sizeof(int)), "hipMalloc");
    e->done_cap = kDoneCap;
  }

  // ---- prologue of the admitted jobs ----
  hipStream_t q = e->q;
  if (na > 0) {
    for (int i = 0; i < na; ++i) {
      Job* j = admitted[i];
      init_ctl(e, j);
      ENG_TRY(e, hipMemcpyAsync(j->w.ctl, j->ctl_host, sizeof(Ctl), hipMemcpyHostToDevice, q), "copy ctl");
      ENG_TRY(e, hipMemcpyAsync(j->w.C_tmp, j->spec.C0, (size_t)j->spec.K * j->spec.d * 4, hipMemcpyDeviceToDevice, q),
              "copy C0");
    }
    ENG_TRY(e, launch_prep_batch(dptr<PrepArgs>(e, o_prep), dptr<int>(e, o_prep_pre), na, prep_blocks, q), "batched prep");
    for (size_t b = 0; b < pb.size(); ++b)
      ENG_TRY(e, launch_assign_batch(pb[b].pick, dptr<AssignArgs>(e, o_pb[b]), dptr<int>(e, o_pb_pre[b]),
                                     (int)pb[b].a.size(), pb_blocks[b], pb[b].lds, q), "batched assignment");
    UpdateBatch ub;
    ub.tab = dptr<UpdateArgs>(e, o_pu);
    for (int k = 0; k < kUpdateKinds; ++k) { ub.prefix[k] = dptr<int>(e, o_pupre[k]); ub.blocks[k] = pub[k]; }
    ub.n = na;
    ENG_TRY(e, launch_xbound_batch(ub, q), "batched bound of |x|");
    ENG_TRY(e, launch_update_sums_batch(ub, q), "batched update");
    ENG_TRY(e, launch_finalize_batch(dptr<FinalizeArgs>(e, o_pf), dptr<int>(e, o_pfpre), pfb,
                                     dptr<int>(e, o_pfxpre), pfxb, na, q),
            "batched finalize");
    ENG_TRY(e, launch_combine_batch(dptr<CombineArgs>(e, o_pc), dptr<int>(e, o_pcpre), na, pcb, q),
            "batched combine");
    // counters of the first candidate pass start from zero
    for (Job* j : admitted)
      ENG_TRY(e, hipMemcpyAsync(j->w.ctl, j->ctl_host, sizeof(Ctl), hipMemcpyHostToDevice, q), "copy ctl");
  }
  e->active = all;

  // ---- iteration graphs ----
  for (hipGraphExec_t& g : e->gexec) {   // may still be in flight: destroyed at the next drain
    if (g) e->old_graphs.push_back(g);
    g = nullptr;
  }
  if (e->graphs && e->n_it > 0) {
    for (int p = 0; p < km_engine::kSlots; ++p) {
      hipGraph_t g = nullptr;
      ENG_TRY(e, hipStreamBeginCapture(q, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
      km_status es = enqueue_iteration(e, p);
      hipError_t ee = hipStreamEndCapture(q, &g);
      if (es != KM_OK) return es;
      if (ee != hipSuccess) return hip_fail(e->ctx, ee, "hipStreamEndCapture");
      ee = hipGraphInstantiate(&e->gexec[p], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ee != hipSuccess) return hip_fail(e->ctx, ee, "hipGraphInstantiate");
    }
  }
  if (drain) {
    e->change = false;
    ++e->drains;
  } else {
    ++e->appends;
  }
  e->rebuild_ms += now_ms() - t_in;
  return KM_OK;
}

// Results of the iteration in slot p (whose tables held the first n jobs):
// start the finishing copies of newly finished jobs.
km_status harvest(km_engine* e, std::pair<int, int> it) {
  const int p = it.first;
  ENG_TRY(e, hipEventSynchronize(e->poll_ev[p]), "hipEventSynchronize");
  const int* f = e->hdone + (size_t)p * e->done_cap;
  int done_in_tables = 0;
  for (int i = 0; i < it.second; ++i) {
    Job* j = e->active[i];
    if (f[i] && !j->done_dev) {
      j->done_dev = true;
      j->state = kFinishing;
      const int64_t KD = (int64_t)j->spec.K * j->spec.d;
      const int64_t n = std::max<int64_t>(KD, j->spec.N);
      const int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
      clear_pending_error();
      hipLaunchKernelGGL(k_finish, dim3(grid), dim3(256), 0, e->q, j->w.ctl, j->w.C_cand, j->w.C_fb, KD,
                         j->w.labels, j->spec.N, j->spec.C_out, j->spec.rho_out);
      ENG_TRY(e, hipGetLastError(), "finish");
      ENG_TRY(e, hipMemcpyAsync(j->ctl_host, j->w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, e->q), "copy ctl");
      ENG_TRY(e, hipEventRecord(j->ev, e->q), "hipEventRecord");
      e->finishing.push_back(j);
    }
    if (j->done_dev) ++done_in_tables;
  }
  for (int i = it.second; i < e->n_it; ++i) done_in_tables += e->active[i]->done_dev ? 1 : 0;
  const int live = e->n_it - done_in_tables;
  // a queued job that fits only once finished jobs are freed needs a drain
  bool admit_after_free = false;
  if (!e->queued.empty() && e->budget > 0 &&
      e->used + (int64_t)e->queued.front()->footprint > e->budget) {
    int64_t freed = 0;
    for (Job* j : e->active) if (j->done_dev) freed += (int64_t)j->footprint;
    admit_after_free = e->used - freed + (int64_t)e->queued.front()->footprint <= e->budget;
  }
  if (live == 0 || admit_after_free || (done_in_tables > 0 && done_in_tables * 4 >= e->n_it) ||
      (!e->queued.empty() && (size_t)e->n_it >= kDoneCap))
    e->change = true;
  return KM_OK;
}

// A queued job can join without a drain.
bool can_append(const km_engine* e) {
  if (e->queued.empty() || (size_t)e->active.size() >= kDoneCap) return false;
  return e->budget <= 0 || e->used + (int64_t)e->queued.front()->footprint <= e->budget;
}

void collect(km_engine* e) {
  while (!e->finishing.empty()) {
    Job* j = e->finishing.front();
    if (hipEventQuery(j->ev) != hipSuccess) {
      clear_pending_error();
      break;
    }
    e->finishing.pop_front();
    const Ctl& r = *j->ctl_host;
    km_job_result& o = j->res;
    o.ticket = j->ticket;
    o.status = r.status;
    o.iters = r.t;
    o.E = r.E_acc;
    o.accepted = r.accepted;
    o.rejected = r.rejected;
    o.assign_passes = r.assign_passes;
    o.m_final = r.m;
    o.recheck_rows = (int64_t)r.flagged_total;
    o.near_tie_rows = (int64_t)r.near_total;
    o.latency_ms = now_ms() - j->t_submit;
    j->state = kReady;
    e->ready.push_back(j);
  }
}

}  // namespace

extern "C" {

int64_t km_job_workspace_bytes(const km_job* job, int32_t m_max) {
  if (!job || job->N < 1 || job->d < 1 || job->K < 1 || m_max < 0 || m_max > KM_M_MAX_LIMIT) return -1;
  return (int64_t)ws_layout(job_shape(*job, m_max, job->prec == KM_GEMM_BF16), nullptr, nullptr);
}

km_status km_engine_create(km_ctx* c, int32_t m_max, double tol, const km_opts* opt_in, int64_t hbm_budget,
                           int32_t graphs, km_engine** out) {
  if (!c || !out) return KM_EINVAL;
  *out = nullptr;
  km_opts opt;
  if (opt_in) opt = *opt_in; else km_opts_default(&opt);
  if (m_max < 0 || m_max > KM_M_MAX_LIMIT) return fail(c, KM_EINVAL, "m_max must be in [0, 64]");
  if (!(tol >= 0.0) || !isfinite(tol)) return fail(c, KM_EINVAL, "tol must be finite and >= 0");
  if (opt.max_iter < 1 || opt.m_init < 0) return fail(c, KM_EINVAL, "max_iter must be >= 1 and m_init >= 0");
  if (!(opt.ridge >= 0.0) || !isfinite(opt.ridge) || !isfinite(opt.eps1) || !isfinite(opt.eps2))
    return fail(c, KM_EINVAL, "eps1, eps2 and ridge must be finite (ridge >= 0)");
  if (opt.trace_C || opt.trace_rec || opt.m_traj) return fail(c, KM_EINVAL, "the engine does not trace");
  if (hbm_budget < 0) return fail(c, KM_EINVAL, "hbm_budget must be >= 0");
  if (hipSetDevice(c->device) != hipSuccess) return hip_fail(c, hipGetLastError(), "hipSetDevice");
  km_engine* e = new km_engine();
  e->ctx = c;
  e->m_max = m_max;
  e->tol = tol;
  e->opt = opt;
  e->budget = hbm_budget;
  e->graphs = graphs != 0;
  bool ok = hipStreamCreateWithFlags(&e->q, hipStreamNonBlocking) == hipSuccess;
  for (int k = 0; k < km_engine::kSlots && ok; ++k)
    ok = hipEventCreateWithFlags(&e->poll_ev[k], hipEventDisableTiming) == hipSuccess;
  for (int k = 0; k < 2 && ok; ++k)
    ok = hipEventCreateWithFlags(&e->tab_ev[k], hipEventDisableTiming) == hipSuccess;
  if (ok) {  // order the engine after work already on the context's stream
    ok = hipEventRecord(c->enter, c->stream) == hipSuccess && hipStreamWaitEvent(e->q, c->enter, 0) == hipSuccess;
  }
  if (!ok) {
    clear_pending_error();
    km_engine_destroy(e);
    return fail(c, KM_EDEVICE, "engine stream or events could not be created");
  }
  *out = e;
  return KM_OK;
}

void km_engine_destroy(km_engine* e) {
  if (!e) return;
  if (e->q) (void)hipStreamSynchronize(e->q);
  drop_graphs(e);
  std::vector<Job*> all(e->queued.begin(), e->queued.end());
  all.insert(all.end(), e->active.begin(), e->active.end());
  all.insert(all.end(), e->finishing.begin(), e->finishing.end());
  all.insert(all.end(), e->ready.begin(), e->ready.end());
  std::sort(all.begin(), all.end());
  all.erase(std::unique(all.begin(), all.end()), all.end());
  for (Job* j : all) {
    if (j->mem) (void)hipFree(j->mem);
    free_job(j);
  }
  for (int k = 0; k < 2; ++k) {
    if (e->dbuf[k]) (void)hipFree(e->dbuf[k]);
    if (e->stage[k]) (void)hipHostFree(e->stage[k]);
    if (e->tab_ev[k]) (void)hipEventDestroy(e->tab_ev[k]);
  }
  if (e->ddone) (void)hipFree(e->ddone);
  if (e->hdone) (void)hipHostFree(e->hdone);
  for (hipEvent_t v : e->poll_ev) if (v) (void)hipEventDestroy(v);
  if (e->q) (void)hipStreamDestroy(e->q);
  clear_pending_error();
  delete e;
}

km_status km_engine_submit(km_engine* e, const km_job* job, int64_t* ticket) {
  if (!e || !job) return KM_EINVAL;
  km_ctx* c = e->ctx;
  km_status s = check_common(c, job->X, job->xt, job->N, job->d, job->K, job->prec);
  if (s != KM_OK) return s;
  if (!is_device_ptr(job->C0) || !is_device_ptr(job->C_out) || !is_device_ptr(job->rho_out))
    return fail(c, KM_EINVAL, "C0, C_out and rho_out must be device pointers");
  if (!aligned16(job->C0) || !aligned16(job->C_out))
    return fail(c, KM_EINVAL, "C0 and C_out must start on a 16-byte boundary");
  const size_t xbytes = (size_t)job->N * job->d * (job->xt == KM_X_BF16 ? 2 : 4);
  const size_t cbytes = (size_t)job->K * job->d * 4;
  if (overlap(job->C_out, cbytes, job->X, xbytes) || overlap(job->rho_out, (size_t)job->N * 4, job->X, xbytes) ||
      overlap(job->rho_out, (size_t)job->N * 4, job->C_out, cbytes) ||
      overlap(job->rho_out, (size_t)job->N * 4, job->C0, cbytes))
    return fail(c, KM_EINVAL, "outputs must not alias X or each other");
  const bool gbf = job->prec == KM_GEMM_BF16;
  Job* j = new Job();
  j->spec = *job;
  j->ticket = e->next_ticket;
  j->gbf = gbf;
  j->xbf = job->xt == KM_X_BF16;
  j->shape = job_shape(*job, e->m_max, gbf);
  j->bytes = ws_layout(j->shape, nullptr, nullptr);
  j->footprint = j->bytes + xbytes + 2 * cbytes + (size_t)job->N * 4;
  if (e->budget > 0 && (int64_t)j->footprint > e->budget) {
    delete j;
    return fail(c, KM_ENOMEM, "the job's device memory (workspace, X, centroids, labels) alone exceeds the HBM "
                              "budget");
  }
  AssignArgs probe{};
  probe.N = job->N; probe.d = job->d; probe.K = job->K; probe.xbf16 = j->xbf; probe.gemm_bf16 = gbf;
  probe.shape = shape_for(c, gbf, j->xbf, job->d, job->K);
  j->pick = assign_pick(probe);
  if (!j->pick.fn) {
    delete j;
    return fail(c, KM_EUNSUPPORTED, "no assignment kernel for this shape");
  }
  if (hipHostMalloc((void**)&j->ctl_host, sizeof(Ctl), hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&j->ev, hipEventDisableTiming) != hipSuccess) {
    clear_pending_error();
    free_job(j);
    return fail(c, KM_ENOMEM, "pinned host memory for a job failed");
  }
  j->t_submit = now_ms();
  e->queued.push_back(j);
  ++e->next_ticket;
  if (ticket) *ticket = j->ticket;
  return KM_OK;
}

km_status km_engine_set_share(km_engine* e, double frac) {
  if (!e || !(frac > 0.0) || frac > 1.0) return KM_EINVAL;
  e->share = frac;
  e->change = true;   // grids are sized at the next rebuild
  return KM_OK;
}

km_status km_engine_step(km_engine* e, int32_t wait, int32_t* n_active, int32_t* n_queued, int32_t* n_ready) {
  if (!e) return KM_EINVAL;
  km_ctx* c = e->ctx;
  c->err.clear();
  ENG_TRY(e, hipSetDevice(c->device), "hipSetDevice");
  km_status s = KM_OK;
  if (e->change) {
    // finish what is in flight first (its flags may start finishing copies)
    while (!e->inflight.empty()) {
      s = harvest(e, e->inflight.front());
      if (s != KM_OK) return s;
      e->inflight.pop_front();
    }
    s = rebuild(e, true);
    if (s != KM_OK) return s;
  } else if (can_append(e)) {
    s = rebuild(e, false);
    if (s != KM_OK) return s;
  }
  bool live = false;
  for (Job* j : e->active) live |= !j->done_dev;
  bool progressed = false;
  if (live && !e->change && (int)e->inflight.size() < km_engine::kSlots) {
    const int p = e->slot;
    e->slot = (e->slot + 1) % km_engine::kSlots;
    if (e->graphs) ENG_TRY(e, hipGraphLaunch(e->gexec[p], e->q), "hipGraphLaunch");
    else if ((s = enqueue_iteration(e, p)) != KM_OK) return s;
    ENG_TRY(e, hipEventRecord(e->poll_ev[p], e->q), "hipEventRecord");
    e->inflight.push_back({p, e->n_it});
    ++e->iterations;
    progressed = true;
  }
  // collect completed iterations without waiting
  while (!e->inflight.empty() && !e->change) {
    const hipError_t qe = hipEventQuery(e->poll_ev[e->inflight.front().first]);
    if (qe == hipErrorNotReady) {
      clear_pending_error();
      break;
    }
    if (qe != hipSuccess) return hip_fail(c, qe, "hipEventQuery");
    s = harvest(e, e->inflight.front());
    if (s != KM_OK) return s;
    e->inflight.pop_front();
    progressed = true;
  }
  if (wait && !progressed && !e->inflight.empty()) {
    s = harvest(e, e->inflight.front());
    if (s != KM_OK) return s;
    e->inflight.pop_front();
  }
  if (!live && e->inflight.empty()) {
    if (!e->queued.empty() || !e->active.empty()) e->change = true;
    ENG_TRY(e, hipStreamSynchronize(e->q), "hipStreamSynchronize");
  }
  collect(e);
  int act = 0;
  for (Job* j : e->active) act += j->state == kActive;
  if (n_active) *n_active = act;
  if (n_queued) *n_queued = (int32_t)e->queued.size();
  if (n_ready) *n_ready = (int32_t)e->ready.size();
  return KM_OK;
}

int32_t km_engine_poll(km_engine* e, km_job_result* res) {
  if (!e || e->ready.empty()) return 0;
  Job* j = e->ready.front();
  e->ready.pop_front();
  if (res) *res = j->res;
  // a job still in the tables leaves them at the next rebuild, which frees it
  j->taken = true;
  bool in_active = false;
  for (Job* a : e->active) in_active |= (a == j);
  if (!in_active) free_job(j);
  return 1;
}

km_status kmeans_solve_batch(km_ctx* c, const km_job* jobs, int32_t n, int32_t m_max, double tol,
                             const km_opts* opt, km_job_result* res) {
  if (!c || n < 0 || (n > 0 && (!jobs || !res))) return KM_EINVAL;
  km_engine* e = nullptr;
  km_status s = km_engine_create(c, m_max, tol, opt, 0, 1, &e);
  if (s != KM_OK) return s;
  for (int i = 0; i < n && s == KM_OK; ++i) s = km_engine_submit(e, &jobs[i], nullptr);
  int got = 0;
  while (s == KM_OK && got < n) {
    int32_t na = 0, nq = 0, nr = 0;
    s = km_engine_step(e, 1, &na, &nq, &nr);
    km_job_result r;
    while (s == KM_OK && km_engine_poll(e, &r)) {
      res[r.ticket] = r;
      ++got;
    }
  }
  // results are complete on the device; order the caller's stream after them
  if (s == KM_OK) {
    if (hipEventRecord(c->enter, e->q) != hipSuccess || hipStreamWaitEvent(c->stream, c->enter, 0) != hipSuccess)
      s = hip_fail(c, hipGetLastError(), "hipStreamWaitEvent");
  }
  km_engine_destroy(e);
  return s;
}

}  // extern "C"
