// Controller, least-squares solve and accelerated iterate
// (Sec. 2.1 Eq. (7)-(8), Sec. 2.2, Algorithm 1).
//
// All decisions are taken on the device by single-workgroup kernels, so the
// host only enqueues a fixed sequence of launches per iteration and polls a
// flag; every kernel returns at once when the solve is done (or, for the
// fall-back assignment, when the candidate was kept).
//
// Readings of points the paper leaves open (the CPU reference follows the
// same ones):
//  * P^0 is the assignment of C^0; the iteration starts from C^1 = G(C^0).
//  * An accelerated candidate whose assignment repeats is replaced by the
//    Lloyd iterate; the run ends when a Lloyd iterate repeats the previous
//    assignment (KM_FLAG_LITERAL_RETURN restores the printed early return).
//  * The m-rule is skipped while E^{t-2} is infinite and is evaluated in
//    cross-multiplied form with the candidate's energy.
//  * Optional energy tolerance on the accepted energies.
//  * Least squares: normal equations of the norm-scaled columns, ridge, float64
//    Cholesky; zero columns dropped.  C^{t+1} = G^t - sum_j theta_j dG_j.

#include "km_launch.h"

namespace km {

__device__ __forceinline__ void rotate_labels(Ctl* c, bool fb) {
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

__device__ __forceinline__ void finish(Ctl* c, int status, bool fb, double* rec, int stop) {
  c->done = 1;
  c->status = status;
  c->acc_src = fb ? 1 : 0;
  rotate_labels(c, fb);
  if (rec) rec[11] = stop;
}

// stop codes in record slot 11
enum { kStopNone = 0, kStopFixedPoint = 1, kStopTol = 2, kStopMaxIter = 3, kStopNonFinite = 4 };

__global__ __launch_bounds__(256) void k_controller(CtlArgs a) {
  Ctl* c = a.ctl;
  if (c->done) return;
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const bool need = (a.stage == 1) || c->reject;
  double v = 0.0;
  if (need)
    for (int i = tid; i < a.n_part; i += 256) v += a.e_part[i];
  red[tid] = v;
  const int t_next = c->t + (a.stage == 1 ? 1 : 0);
  if (a.stage == 1 && a.trace_C) {
    const int64_t kd = (int64_t)a.K * a.d;
    for (int64_t e = tid; e < kd; e += 256) a.trace_C[(int64_t)t_next * kd + e] = a.C_cand[e];
  }
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid != 0) return;
  const double E = red[0];
  double* rec = a.trace_rec ? a.trace_rec + (int64_t)t_next * kTraceRec : nullptr;

  if (a.stage == 1) {
    c->t = t_next;
    c->E_cand = E;
    const unsigned long long changed = c->cnt_changed[0];
    c->assign_passes += 1;
    c->flagged_total += c->cnt_flagged[0];
    if (rec) {
      rec[0] = t_next; rec[1] = E; rec[2] = (double)changed; rec[10] = (double)c->cnt_flagged[0];
      rec[3] = c->m;
    }
    if (!isfinite(E)) {
      c->E_acc = E;
      finish(c, -5, false, rec, kStopNonFinite);
      return;
    }
    const bool same = (changed == 0);
    if (same && (c->cand_is_lloyd || (c->flags & 2u))) {
      c->E_acc = E;
      if (rec) { rec[4] = kDecConverged; rec[7] = E; }
      finish(c, 0, false, rec, kStopFixedPoint);
      return;
    }
    if (!(c->flags & 1u) && isfinite(c->E2)) {          // dynamic m (Sec. 2.2)
      const double num = c->E1 - E, den = c->E2 - c->E1;
      if (num < c->eps1 * den) c->m = c->m - 1 > 0 ? c->m - 1 : 0;
      else if (num > c->eps2 * den) c->m = c->m + 1 < c->m_max ? c->m + 1 : c->m_max;
    }
    if (rec) rec[3] = c->m;
    const bool reject = !c->cand_is_lloyd && (same || E >= c->E1);
    c->reject = reject ? 1 : 0;
    if (reject) {
      c->cnt_changed[1] = 0;
      c->cnt_flagged[1] = 0;
    }
    return;
  }

  // stage 2: accept or fall back, stopping rules, advance the state
  const int t = c->t;
  bool fb = false;
  if (c->reject) {
    fb = true;
    c->E_fb = E;
    const unsigned long long changed = c->cnt_changed[1];
    c->assign_passes += 1;
    c->flagged_total += c->cnt_flagged[1];
    c->rejected += 1;
    c->E_acc = E;
    if (rec) { rec[4] = kDecRejected; rec[5] = E; rec[6] = (double)changed; rec[7] = E; }
    if (!isfinite(E)) { finish(c, -5, true, rec, kStopNonFinite); return; }
    if (changed == 0) { finish(c, 0, true, rec, kStopFixedPoint); return; }
  } else {
    if (!c->cand_is_lloyd) c->accepted += 1;
    c->E_acc = c->E_cand;
    if (rec) { rec[4] = c->cand_is_lloyd ? kDecLloyd : kDecAccepted; rec[7] = c->E_cand; }
  }
  const double Ea = c->E_acc;
  if (c->tol > 0.0 && isfinite(c->E1) && (c->E1 - Ea) <= c->tol * c->E1) {
    finish(c, 0, fb, rec, kStopTol);
    return;
  }
  if (t >= c->max_iter) {
    finish(c, 1, fb, rec, kStopMaxIter);
    return;
  }
  c->acc_src = fb ? 1 : 0;
  rotate_labels(c, fb);
  c->E2 = c->E1;
  c->E1 = Ea;
  c->cnt_changed[0] = 0;
  c->cnt_flagged[0] = 0;
}

hipError_t launch_controller(const CtlArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_controller, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Least squares (Eq. (7)) on the newest m_t history columns.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ls_solve(SolveArgs a) {
  Ctl* c = a.ctl;
  if (c->done) return;
  const int cap = a.cap;
  const int tid = threadIdx.x;
  if (cap == 0) {
    if (tid == 0) { c->mt = 0; c->used = 0; c->cand_is_lloyd = 1; }
    return;
  }
  __shared__ double bvec[kMaxM];
  __shared__ double Am[kMaxM * kMaxM];
  __shared__ double sc[kMaxM], rhs[kMaxM], y[kMaxM];
  __shared__ int cols[kMaxM];
  const int s_new = (c->hist_len == 0) ? 0 : (c->hist_head + 1) % cap;
  const int len_new = c->hist_len + 1 < cap ? c->hist_len + 1 : cap;

  for (int q = tid; q < len_new; q += 256) {
    const int sl = (s_new - q + cap) % cap;
    double ga = 0.0, gb = 0.0;
    for (int w = 0; w < a.n_dots; ++w) {
      ga += a.dots[(int64_t)w * 2 * cap + sl];
      gb += a.dots[(int64_t)w * 2 * cap + cap + sl];
    }
    a.gram[s_new * cap + sl] = ga;
    a.gram[sl * cap + s_new] = ga;
    bvec[sl] = gb;
  }
  __threadfence_block();
  __syncthreads();
  if (tid != 0) return;

  int mt = c->m < c->t ? c->m : c->t;
  if (mt > len_new) mt = len_new;
  double* rec = a.trace_rec ? a.trace_rec + (int64_t)c->t * kTraceRec : nullptr;
  int n = 0;
  for (int q = 0; q < mt; ++q) {
    const int sl = (s_new - q + cap) % cap;
    const double nrm = sqrt(a.gram[sl * cap + sl]);
    c->theta[q] = 0.0;
    if (nrm > 0.0) { cols[n] = q; sc[n] = nrm; ++n; }
  }
  bool ok = true;
  if (n > 0) {
    for (int r = 0; r < n; ++r) {
      const int sr = (s_new - cols[r] + cap) % cap;
      for (int q = 0; q < n; ++q) {
        const int sq = (s_new - cols[q] + cap) % cap;
        Am[r * n + q] = a.gram[sr * cap + sq] / (sc[r] * sc[q]) + (r == q ? c->ridge : 0.0);
      }
      rhs[r] = bvec[sr] / sc[r];
    }
    // Cholesky A = L L^T, L stored in the lower triangle of Am
    for (int i = 0; i < n && ok; ++i) {
      for (int k = 0; k <= i; ++k) {
        double s = Am[i * n + k];
        for (int p = 0; p < k; ++p) s -= Am[i * n + p] * Am[k * n + p];
        if (i == k) {
          if (!(s > 0.0)) { ok = false; break; }
          Am[i * n + i] = sqrt(s);
        } else {
          Am[i * n + k] = s / Am[k * n + k];
        }
      }
    }
    if (ok) {
      for (int i = 0; i < n; ++i) {            // L z = rhs
        double s = rhs[i];
        for (int p = 0; p < i; ++p) s -= Am[i * n + p] * y[p];
        y[i] = s / Am[i * n + i];
      }
      for (int i = n - 1; i >= 0; --i) {       // L^T w = z
        double s = y[i];
        for (int p = i + 1; p < n; ++p) s -= Am[p * n + i] * y[p];
        y[i] = s / Am[i * n + i];
      }
      for (int r = 0; r < n; ++r) c->theta[cols[r]] = y[r] / sc[r];
    }
  }
  if (!ok) n = 0;
  c->mt = mt;
  c->used = n;
  c->cand_is_lloyd = (n == 0) ? 1 : 0;
  c->hist_head = s_new;
  c->hist_len = len_new;
  if (rec) {
    rec[8] = mt;
    rec[9] = n;
    for (int q = 0; q < mt; ++q) rec[16 + q] = c->theta[q];
  }
}

hipError_t launch_ls_solve(const SolveArgs& a, hipStream_t s) {
  if (a.cap > kMaxM) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ls_solve, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Accelerated iterate (Eq. (8), sign of Algorithm 1) and its centroid prep.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_combine(CombineArgs a) {
  Ctl* c = a.ctl;
  if (c->done) return;
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= a.K) return;
  const int d = a.d, cap = a.cap;
  const int mt = (c->used > 0) ? c->mt : 0;
  const int head = c->hist_head;
  const int64_t KD = (int64_t)a.K * d;
  double nsq = 0.0, e2 = 0.0;
  for (int k = lane; k < d; k += kWave) {
    const int64_t e = (int64_t)j * d + k;
    double v = a.G_last[e];
    for (int q = 0; q < mt; ++q) {
      const int sl = (head - q + cap) % cap;
      v -= c->theta[q] * a.ring_dG[(int64_t)sl * KD + e];
    }
    const float f = (float)v;
    a.C_cand[e] = f;
    nsq = fma((double)f, (double)f, nsq);
    if (a.Cb_cand) {
      uint32_t x = __float_as_uint(f);
      x += 0x7FFFu + ((x >> 16) & 1u);
      const uint16_t b = (uint16_t)(x >> 16);
      a.Cb_cand[e] = b;
      const double df = (double)f - (double)__uint_as_float(((uint32_t)b) << 16);
      e2 = fma(df, df, e2);
    }
  }
  nsq = wave_sum(nsq);
  e2 = wave_sum(e2);
  if (lane == 0) {
    a.nc_cand[j] = (float)nsq;
    if (a.Cb_cand) a.delta_cand[j] = (float)sqrt(e2);
  }
}

hipError_t launch_combine(const CombineArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, dim3((a.K + 3) / 4), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace km
