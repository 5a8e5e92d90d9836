// Host-side launch interface between the C ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "km_common.h"
#include "km_ctl.h"

namespace km {

// ----- assignment (Sec. 1, Eq. (3)) fused with the energy (Eq. (1)) -----
struct AssignArgs {
  const void* X;          // N x d rows, float32 or bfloat16 bits
  int64_t N;
  int d, K;
  const float* C;         // K x d float32 centroids
  const float* nc;        // K squared norms of C (float32)
  const uint16_t* Cb;     // bf16 GEMM only: 2 x K x d bfloat16 pair of C, hi rows then lo rows
  const float* delta;     // bf16 GEMM only: K residual norms ||c_j - hi_j - lo_j||
  int* lab;               // label buffers: 3 x N (solver roles) or N (plain role)
  const int* lab_prev;    // plain role: labels to count changes against, or null
  double* e_part;         // per-workgroup energy partials of this pass
  int* flags;             // N ints: per-wave lists of flagged rows (deferred re-check)
  Ctl* ctl;
  int xbf16;              // X stored as bfloat16
  int gemm_bf16;          // distance GEMM in bfloat16
  int role;               // Role of the launch (set by launch_assign / the batch tables)
  int shape;              // tile shape id (0 = default)
  // Row bounds (Hamerly-style, float32 GEMM with LDS-resident centroids only;
  // null / 0 elsewhere).  lb: lower bounds of the distance from each row to
  // every centroid other than its own, 3 x N (one slice per label buffer;
  // the plain role writes slice 0).  bounds = 1: candidate and fall-back
  // passes skip the rows whose bound proves the previous label; shift: K
  // upper bounds of ||c_j - c_ref_j|| of this pass's centroids against the
  // centroids the previous labels' bounds refer to.
  float* lb;
  int bounds;
  const double* shift;
  // List mode (single-instance launches): rows the GEMM bound cannot decide
  // stay in the per-wave lists for k_recheck, whose list lengths go to
  // fl_cnt[workgroup * 16 + wave]; null: the workgroups re-check their own.
  int* fl_cnt;
};
// 1 if launches for a's shape can keep row bounds (float32 GEMM, centroids
// resident in LDS); the solver enables them only then.
int assign_bounds_ok(const AssignArgs& a);
int assign_grid(const AssignArgs& a);   // workgroups of one launch (persistent grid)
// ev0 / ev1 (nullable): events that take the start and end time of this
// launch's own dispatch (no separate event record on the stream).
hipError_t launch_assign(const AssignArgs& a, Role role, hipStream_t s, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);
struct KernelPick;
KernelPick assign_pick(const AssignArgs& a);
// resident workgroups of kernel p on the device x frac, capped at N's row groups
int64_t assign_resident(const KernelPick& p, int64_t N, double frac);

// ||c_j||^2 (and the bfloat16 hi/lo pair with its residual norms when Cb != null).
hipError_t launch_prep(const float* C, int K, int d, float* nc, uint16_t* Cb, float* delta,
                       hipStream_t s);
struct PrepArgs {
  const float* C;
  int K, d;
  float* nc;
  uint16_t* Cb;
  float* delta;
};
inline int prep_grid(int K) { return (K + 3) / 4; }
hipError_t launch_prep_batch(const PrepArgs* tab, const int* prefix, int n, int blocks, hipStream_t s);
// Batched assignment: every instance of tab uses the kernel of p (same
// template), grid slices per prefix; lds = the largest LDS need of them.
hipError_t launch_assign_batch(const KernelPick& p, const AssignArgs* tab, const int* prefix, int n, int blocks,
                               size_t lds, hipStream_t s);

// ----- update step (Sec. 1, Eq. (4)): counting sort + segmented sum -----
struct UpdateArgs {
  const void* X;
  int64_t N;
  int d, K, xbf16;
  int* lab;               // label buffers base (3 x N) or the labels themselves
  int lab_from_ctl;       // 1: labels = lab + ctl->lab_prev * N
  int* lrank;             // N
  int* blockcount;        // K x nblk, overwritten with per-block offsets
  int* counts;            // K
  int* seg_start;         // K + 1
  int* item_start;        // K + 1
  int* item_cluster;      // max_items
  int* perm;              // N
  double* partial;        // max_items x d
  int max_items;
  Ctl* ctl;
  int gated;              // 1: skip when ctl->done
  int fx;                 // 1: fixed-point sums (fx_ok(K, d)) instead of the counting sort
  unsigned* xbound;       // kXBoundSlots per-workgroup maxima of the |x| bit patterns, then e
  unsigned long long* fxpart;  // fx_blocks(N) x (K*d + K) int64 partials
};
int update_max_items(int64_t N, int K);
// blockcount entries a workspace for (N, K) must hold: enough for any K' <= K
size_t update_blockcount_ints(int64_t N, int K);
// ev0 (nullable): takes the start time of the update's first kernel
hipError_t launch_update_sums(const UpdateArgs& u, hipStream_t s, hipEvent_t ev0 = nullptr);
// Bound of |x| over X and the scale exponent e of the fixed-point sums
// (u.fx only): once per X, before the first update with it.
hipError_t launch_xbound(const UpdateArgs& u, hipStream_t s);
// workgroups of update kernel `which` (0 rank, 1 scan, 2 scatter, 3 segsum,
// 4 fixed-point sums, 5 unused, 6 the |x| bound); 0 where the instance takes
// the other path
constexpr int kUpdateKinds = 7;
int update_grid(const UpdateArgs& u, int which);
// Batched update: tab (device) one UpdateArgs per instance; prefix[w]
// (device, n + 1 entries) the cumulative workgroups of kernel w; blocks[w]
// the launch size.  The offsets kernel runs one workgroup per instance.
struct UpdateBatch {
  const UpdateArgs* tab;
  const int* prefix[kUpdateKinds];
  int blocks[kUpdateKinds];
  int n;
};
hipError_t launch_update_sums_batch(const UpdateBatch& ub, hipStream_t s);
hipError_t launch_xbound_batch(const UpdateBatch& ub, hipStream_t s);

// Finalisation of the means and, in the solver, the residual/history push.
enum FinMode : int { kFinG = 0, kFinInit = 1, kFinIter = 2 };
struct FinalizeArgs {
  int d, K, cap;          // cap = m_max (history ring capacity)
  const double* partial;
  const int* item_start;
  const int* counts;
  const float* C_in;      // kFinG / kFinInit: centroids G was applied to
  float* C_out;           // kFinG: output means
  const float* C_cand;    // candidate C^t
  const float* C_fb;      // fall-back iterate, C^t when ctl->acc_src == 1
  double* G_last;         // K x d
  double* F_last;         // K x d
  double* ring_dF;        // cap x K x d
  double* ring_dG;        // cap x K x d
  double* dots;           // per-workgroup partial inner products (2 x cap each)
  Ctl* ctl;
  FinMode mode;
  // fixed-point sums (fx = 1): the finalisation also adds the per-workgroup
  // partials of k_fxsum (N rows, scale exponent in xbound[kXBoundSlots]);
  // partial, item_start and counts are then unused
  int fx;
  const unsigned long long* fxpart;
  const unsigned* xbound;
  int64_t N;
  float* C_ref;           // nullable: receives the accepted centroids (kFinInit: C_in), the
                          // reference of the next pass's row bounds
};
// workgroups of the finalisation (and rows of Gram partials it writes)
int finalize_grid(int64_t KD);                // counting-sort path
int finalize_grid_for(int fx, int K, int d);  // either path
// rows of Gram partials a workspace for K*d must hold (either path)
int finalize_grid_cap(int64_t KD);
// ev1 (nullable): takes the end time of the finalisation kernel
hipError_t launch_finalize(const FinalizeArgs& f, hipStream_t s, hipEvent_t ev1 = nullptr);
// Batched: tab one FinalizeArgs per instance; prefix/blocks for the
// counting-sort instances (256-thread workgroups) and fxprefix/fxblocks for
// the fixed-point ones (kFxThreads); an instance has 0 workgroups in the
// other launch.
hipError_t launch_finalize_batch(const FinalizeArgs* tab, const int* prefix, int blocks, const int* fxprefix,
                                 int fxblocks, int n, hipStream_t s);

// ----- controller (Algorithm 1) -----
struct CtlArgs {
  Ctl* ctl;
  const double* e_part;   // partials of the pass being decided
  int n_part;
  int stage;              // 1: after the candidate pass, 2: after the fall-back pass
  CtlTrace tr;
};
hipError_t launch_controller(const CtlArgs& a, hipStream_t s);
// one workgroup per instance
hipError_t launch_controller_batch(const CtlArgs* tab, int n, hipStream_t s);

// ----- Anderson step (Sec. 2.1, Eq. (7)-(8)) -----
struct CombineArgs {
  Ctl* ctl;
  int gated;              // 1: solver iteration (least squares + theta); 0: C^1 = G^0
  const double* G_last;
  const double* ring_dG;
  const double* dots;     // per-workgroup partial inner products of the finalize launch
  int n_dots;
  double* gram;           // cap x cap stored Gram entries of the history
  double* trace_rec;
  int K, d, cap;
  float* C_cand; float* nc_cand; uint16_t* Cb_cand; float* delta_cand;
  float* C_fb; float* nc_fb; uint16_t* Cb_fb; float* delta_fb;
  // row bounds (nullable): upper bounds of ||c_j - C_ref_j|| of the new
  // candidate and fall-back centroids (float64, K each)
  const float* C_ref; double* sh_cand; double* sh_fb;
  int* done_out;          // nullable: pinned host slot that receives ctl->done (solver iterations)
};
// ev1 (nullable): takes the end time of the combine's dispatch
hipError_t launch_combine(const CombineArgs& a, hipStream_t s, hipEvent_t ev1 = nullptr);
int combine_grid(int K);
hipError_t launch_combine_batch(const CombineArgs* tab, const int* prefix, int n, int blocks, hipStream_t s);

// ----- re-check of a pass's listed rows (list-mode assignment launches) -----
constexpr int kReGrid = 512;       // workgroups (and energy partials) of a re-check launch
constexpr int kReMaxGrid = 4096;   // largest assignment grid a re-check can follow
struct RecheckArgs {
  const void* X;
  int64_t N;
  int d, K, xbf16;
  const float* C;         // float32 centroids of the pass
  const float* nc;        // their squared norms (float32, as in AssignArgs)
  int* lab;               // as in AssignArgs
  const int* lab_prev;
  const int* flags;       // the pass's per-wave lists (slot layout of the assignment launch)
  const int* fl_cnt;      // grid x 16 list lengths written by the assignment launch
  int grid, W, sb16, group_rows;   // the assignment launch's workgroups, waves, 16 SB, rows per group
  double* e_part;         // kReGrid energy partials
  Ctl* ctl;
  int role;
};
// 1 if the assignment launch for a leaves undecided rows in lists (its kernel
// defers: bfloat16 GEMM or centroids streamed through LDS) and its grid fits a re-check.
int assign_list_mode(const AssignArgs& a);
// The re-check's arguments for the assignment launch a (role of the launch).
RecheckArgs recheck_args(const AssignArgs& a, double* e_part);
// ev1 (nullable): takes the end time of the re-check's own dispatch
hipError_t launch_recheck(const RecheckArgs& r, Role role, hipStream_t s, hipEvent_t ev1 = nullptr);
// LDS bytes of a re-check launch for width d after an assignment grid of `grid`
size_t recheck_lds(int d, int grid);
// Batched re-check: tab (device) one RecheckArgs per instance (role set in
// the entry), prefix (device, n + 1 entries) its workgroups (at most
// kReGrid; e_part of an instance holds that many partials); lds = the
// largest recheck_lds of the instances.
hipError_t launch_recheck_batch(const RecheckArgs* tab, const int* prefix, int n, int blocks, size_t lds,
                                hipStream_t s);

// Plain energy reduction for stand-alone G(C): sum of partials in fixed order.
hipError_t launch_reduce_energy(const double* e_part, int n, double* out, hipStream_t s);

}  // namespace km
