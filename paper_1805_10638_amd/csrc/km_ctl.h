// Device-side controller of the accelerated iteration (Algorithm 1).
//
// Run by one workgroup of 256 threads after each assignment pass.  The energy
// of the pass is the fixed-order sum of the per-workgroup partials.
//
// Stage 1 (after evaluating the candidate C^t):
//   convergence test on the assignment (an accelerated candidate whose
//   assignment repeats is not a fixed point and goes to the fall-back),
//   dynamic m (Sec. 2.2, cross-multiplied ratio test, skipped while E^{t-2}
//   is infinite), accept/reject by energy decrease (Sec. 2.1).
// Stage 2 (after the optional fall-back pass):
//   bookkeeping of the accepted iterate, fixed-point / tolerance / max_iter
//   stopping, and the shift E^{t-2} <- E^{t-1} <- E^t.
#pragma once

#include "km_common.h"

namespace km {

struct CtlTrace {
  float* trace_C;         // (max_iter + 1) x K x d, or null
  double* trace_rec;      // (max_iter + 1) x kTraceRec, or null
  int* m_traj;            // (max_iter + 1) ints: m after the dynamic-m rule at iteration t, or null
  const float* C_cand;    // candidate centroids (copied into trace_C)
  int K, d;
};

enum { kStopNone = 0, kStopFixedPoint = 1, kStopTol = 2, kStopMaxIter = 3, kStopNonFinite = 4 };

__device__ __forceinline__ void ctl_rotate_labels(Ctl* c, bool fb) {
  if (fb) {
    const int np = c->lab_fb;
    c->lab_fb = c->lab_prev;
    c->lab_prev = np;
  } else {
    const int np = c->lab_cand;
    c->lab_cand = c->lab_prev;
    c->lab_prev = np;
  }
}

__device__ __forceinline__ void ctl_finish(Ctl* c, int status, bool fb, double* rec, int stop) {
  c->done = 1;
  c->status = status;
  c->acc_src = fb ? 1 : 0;
  ctl_rotate_labels(c, fb);
  if (rec) rec[11] = stop;
}

// Decisions of one stage on the energy E of the pass (thread 0 only).
__device__ inline void controller_decide(Ctl* c, double E, int stage, int t_next, const CtlTrace& tr) {
  double* rec = tr.trace_rec ? tr.trace_rec + (int64_t)t_next * kTraceRec : nullptr;

  if (stage == 1) {
    c->t = t_next;
    c->E_cand = E;
    const unsigned long long changed = c->cnt_changed[0];
    c->assign_passes += 1;
    c->flagged_total += c->cnt_flagged[0];
    c->near_total += c->cnt_near[0];
    c->gemm_total += c->cnt_gemm[0];
    if (rec) {
      rec[0] = t_next; rec[1] = E; rec[2] = (double)changed; rec[10] = (double)c->cnt_flagged[0];
      rec[12] = (double)c->cnt_near[0];
      rec[13] = (double)c->cnt_gemm[0];
      rec[3] = c->m;
    }
    if (tr.m_traj) tr.m_traj[t_next] = c->m;
    if (!isfinite(E)) {
      c->E_acc = E;
      ctl_finish(c, -5, false, rec, kStopNonFinite);
      return;
    }
    const bool same = (changed == 0);
    if (same && (c->cand_is_lloyd || (c->flags & 2u))) {
      c->E_acc = E;
      if (rec) { rec[4] = kDecConverged; rec[7] = E; }
      ctl_finish(c, 0, false, rec, kStopFixedPoint);
      return;
    }
    if (!(c->flags & 1u) && isfinite(c->E2)) {          // dynamic m (Sec. 2.2)
      const double num = c->E1 - E, den = c->E2 - c->E1;
      if (num < c->eps1 * den) c->m = c->m - 1 > 0 ? c->m - 1 : 0;
      else if (num > c->eps2 * den) c->m = c->m + 1 < c->m_max ? c->m + 1 : c->m_max;
    }
    if (rec) rec[3] = c->m;
    if (tr.m_traj) tr.m_traj[t_next] = c->m;
    const bool reject = !c->cand_is_lloyd && (same || E >= c->E1);
    c->reject = reject ? 1 : 0;
    if (reject) {
      c->cnt_changed[1] = 0;
      c->cnt_flagged[1] = 0;
      c->cnt_near[1] = 0;
      c->cnt_gemm[1] = 0;
    }
    return;
  }

  // stage 2
  const int t = c->t;
  bool fb = false;
  if (c->reject) {
    fb = true;
    c->E_fb = E;
    const unsigned long long changed = c->cnt_changed[1];
    c->assign_passes += 1;
    c->flagged_total += c->cnt_flagged[1];
    c->near_total += c->cnt_near[1];
    c->gemm_total += c->cnt_gemm[1];
    c->rejected += 1;
    c->E_acc = E;
    if (rec) { rec[4] = kDecRejected; rec[5] = E; rec[6] = (double)changed; rec[7] = E; }
    if (!isfinite(E)) { ctl_finish(c, -5, true, rec, kStopNonFinite); return; }
    if (changed == 0) { ctl_finish(c, 0, true, rec, kStopFixedPoint); return; }
  } else {
    if (!c->cand_is_lloyd) c->accepted += 1;
    c->E_acc = c->E_cand;
    if (rec) { rec[4] = c->cand_is_lloyd ? kDecLloyd : kDecAccepted; rec[7] = c->E_cand; }
  }
  const double Ea = c->E_acc;
  if (c->tol > 0.0 && isfinite(c->E1) && (c->E1 - Ea) <= c->tol * c->E1) {
    ctl_finish(c, 0, fb, rec, kStopTol);
    return;
  }
  if (t >= c->max_iter) {
    ctl_finish(c, 1, fb, rec, kStopMaxIter);
    return;
  }
  c->acc_src = fb ? 1 : 0;
  ctl_rotate_labels(c, fb);
  c->E2 = c->E1;
  c->E1 = Ea;
  c->cnt_changed[0] = 0;
  c->cnt_flagged[0] = 0;
  c->cnt_near[0] = 0;
  c->cnt_gemm[0] = 0;
}

// red: 256 doubles of LDS.  Must be called by all 256 threads of the group.
// The control block is copied into LDS (one 8-byte word per thread), updated
// there by thread 0 and copied back, so that the decision logic does not
// wait on a global round trip per field.
__device__ inline void controller_stage(Ctl* cg, const double* e_part, int n_part, int stage,
                                        const CtlTrace& tr, double* red) {
  __shared__ Ctl lc;
  static_assert(sizeof(Ctl) % 8 == 0, "the control block is copied in 8-byte words");
  constexpr int kWords = (int)(sizeof(Ctl) / 8);
  const int tid = threadIdx.x;
  for (int i = tid; i < kWords; i += 256) ((unsigned long long*)&lc)[i] = ((const unsigned long long*)cg)[i];
  __syncthreads();
  Ctl* c = &lc;
  const bool need = (stage == 1) || c->reject;
  double v = 0.0;
  if (need) {   // partials tid, tid + 256, ... in order, four loads in flight
    for (int i0 = tid; i0 < n_part; i0 += 4 * 256) {
      double q[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) q[u] = i0 + u * 256 < n_part ? e_part[i0 + u * 256] : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i0 + u * 256 < n_part) v += q[u];
    }
  }
  red[tid] = v;
  const int t_next = c->t + (stage == 1 ? 1 : 0);
  if (stage == 1 && tr.trace_C) {
    const int64_t kd = (int64_t)tr.K * tr.d;
    for (int64_t e = tid; e < kd; e += 256) tr.trace_C[(int64_t)t_next * kd + e] = tr.C_cand[e];
  }
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) controller_decide(c, red[0], stage, t_next, tr);
  __syncthreads();
  for (int i = tid; i < kWords; i += 256) ((unsigned long long*)cg)[i] = ((const unsigned long long*)&lc)[i];
}

}  // namespace km
