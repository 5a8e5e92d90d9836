// Least-squares solve and accelerated iterate (Sec. 2.1, Eq. (7)-(8)).
//
// The history keeps the newest m_max differences dF_j = F^{t-j+1} - F^{t-j}
// and dG_j = G^{t-j+1} - G^{t-j} in a ring, plus the Gram entries
// <dF_a, dF_b> of the stored differences: every iteration adds one row of
// m inner products (computed by the finalisation kernel) and the right-hand
// side <dF_j, F^t>.  The m_t x m_t system is solved here by one wave:
// normal equations of the norm-scaled columns plus a ridge, float64
// Cholesky (zero columns dropped), then theta_j = y_j / ||dF_j||.
// C^{t+1} = G^t - sum_j theta_j dG_j (the sign of Algorithm 1).

#include "km_launch.h"

namespace km {

__global__ __launch_bounds__(64) void k_ls_solve(SolveArgs a) {
  Ctl* c = a.ctl;
  if (c->done) return;
  const int cap = a.cap;
  const int lane = threadIdx.x;
  if (cap == 0) {
    if (lane == 0) { c->mt = 0; c->used = 0; c->cand_is_lloyd = 1; }
    return;
  }
  __shared__ double bvec[kMaxM];
  __shared__ double L[kMaxM * kMaxM];
  __shared__ double sc[kMaxM], y[kMaxM];
  __shared__ int cols[kMaxM];
  __shared__ int n_sh, ok_sh;

  const int s_new = (c->hist_len == 0) ? 0 : (c->hist_head + 1) % cap;
  const int len_new = c->hist_len + 1 < cap ? c->hist_len + 1 : cap;
  int mt = c->m < c->t ? c->m : c->t;
  if (mt > len_new) mt = len_new;

  // new Gram row and right-hand side: fixed-order sums of per-workgroup partials
  for (int q = lane; q < len_new; q += 64) {
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

  // columns with nonzero norm, newest first
  if (lane == 0) {
    int n = 0;
    for (int q = 0; q < mt; ++q) {
      const int sl = (s_new - q + cap) % cap;
      const double nrm = sqrt(a.gram[sl * cap + sl]);
      if (nrm > 0.0) { cols[n] = q; sc[n] = nrm; ++n; }
    }
    n_sh = n;
    ok_sh = 1;
  }
  __syncthreads();
  const int n = n_sh;

  // A = S^-1 Gram S^-1 + ridge I (lane r owns row r), rhs = S^-1 b
  if (lane < n) {
    const int sr = (s_new - cols[lane] + cap) % cap;
    for (int q = 0; q < n; ++q) {
      const int sq = (s_new - cols[q] + cap) % cap;
      L[lane * kMaxM + q] = a.gram[sr * cap + sq] / (sc[lane] * sc[q]) + (lane == q ? c->ridge : 0.0);
    }
    y[lane] = bvec[sr] / sc[lane];
  }
  __syncthreads();
  // right-looking Cholesky, one row per lane
  for (int k = 0; k < n; ++k) {
    if (lane == 0) {
      const double p = L[k * kMaxM + k];
      if (!(p > 0.0)) ok_sh = 0;
      L[k * kMaxM + k] = sqrt(p > 0.0 ? p : 1.0);
    }
    __syncthreads();
    if (lane > k && lane < n) L[lane * kMaxM + k] /= L[k * kMaxM + k];
    __syncthreads();
    if (lane > k && lane < n) {
      const double lik = L[lane * kMaxM + k];
      for (int j = k + 1; j <= lane; ++j) L[lane * kMaxM + j] -= lik * L[j * kMaxM + k];
    }
    __syncthreads();
  }
  // forward (L z = rhs) and backward (L^T w = z) substitution, dot products over lanes
  for (int i = 0; i < n; ++i) {
    double part = (lane < i) ? L[i * kMaxM + lane] * y[lane] : 0.0;
    part = wave_sum(part);
    __syncthreads();
    if (lane == 0) y[i] = (y[i] - part) / L[i * kMaxM + i];
    __syncthreads();
  }
  for (int i = n - 1; i >= 0; --i) {
    double part = (lane > i && lane < n) ? L[lane * kMaxM + i] * y[lane] : 0.0;
    part = wave_sum(part);
    __syncthreads();
    if (lane == 0) y[i] = (y[i] - part) / L[i * kMaxM + i];
    __syncthreads();
  }
  const bool ok = ok_sh != 0;
  for (int q = lane; q < mt; q += 64) c->theta[q] = 0.0;
  __syncthreads();
  if (ok && lane < n) c->theta[cols[lane]] = y[lane] / sc[lane];
  __syncthreads();
  if (lane == 0) {
    const int used = ok ? n : 0;
    c->mt = mt;
    c->used = used;
    c->cand_is_lloyd = (used == 0) ? 1 : 0;
    c->hist_head = s_new;
    c->hist_len = len_new;
    if (a.trace_rec) {
      double* rec = a.trace_rec + (int64_t)c->t * kTraceRec;
      rec[8] = mt;
      rec[9] = used;
      for (int q = 0; q < mt; ++q) rec[16 + q] = c->theta[q];
    }
  }
}

hipError_t launch_ls_solve(const SolveArgs& a, hipStream_t s) {
  if (a.cap > kMaxM) return hipErrorInvalidValue;
  clear_pending_error();
  hipLaunchKernelGGL(k_ls_solve, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// C^{t+1} = G^t - sum_j theta_j dG_j and the fall-back iterate fl32(G^t),
// each with its squared norms (and bfloat16 shadows): one wave per centroid.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float put_centroid(float* C, uint16_t* Cb, int64_t e, double v, double* nsq,
                                              double* e2) {
  const float f = (float)v;
  C[e] = f;
  *nsq = fma((double)f, (double)f, *nsq);
  if (Cb) {
    uint32_t x = __float_as_uint(f);
    x += 0x7FFFu + ((x >> 16) & 1u);
    const uint16_t b = (uint16_t)(x >> 16);
    Cb[e] = b;
    const double df = (double)f - (double)__uint_as_float(((uint32_t)b) << 16);
    *e2 = fma(df, df, *e2);
  }
  return f;
}

__global__ __launch_bounds__(256) void k_combine(CombineArgs a) {
  Ctl* c = a.ctl;
  if (a.gated && c->done) return;
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= a.K) return;
  const int d = a.d, cap = a.cap;
  const int mt = (a.gated && c->used > 0) ? c->mt : 0;
  const int head = a.gated ? c->hist_head : 0;
  const int64_t KD = (int64_t)a.K * d;
  double n_c = 0.0, e_c = 0.0, n_f = 0.0, e_f = 0.0;
  for (int k = lane; k < d; k += kWave) {
    const int64_t e = (int64_t)j * d + k;
    const double g = a.G_last[e];
    double v = g;
    for (int q = 0; q < mt; ++q) {
      const int sl = (head - q + cap) % cap;
      v -= c->theta[q] * a.ring_dG[(int64_t)sl * KD + e];
    }
    put_centroid(a.C_cand, a.Cb_cand, e, v, &n_c, &e_c);
    put_centroid(a.C_fb, a.Cb_fb, e, g, &n_f, &e_f);
  }
  n_c = wave_sum(n_c);
  e_c = wave_sum(e_c);
  n_f = wave_sum(n_f);
  e_f = wave_sum(e_f);
  if (lane == 0) {
    a.nc_cand[j] = (float)n_c;
    a.nc_fb[j] = (float)n_f;
    if (a.Cb_cand) a.delta_cand[j] = (float)sqrt(e_c);
    if (a.Cb_fb) a.delta_fb[j] = (float)sqrt(e_f);
  }
}

hipError_t launch_combine(const CombineArgs& a, hipStream_t s) {
  clear_pending_error();
  hipLaunchKernelGGL(k_combine, dim3((a.K + 3) / 4), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace km
