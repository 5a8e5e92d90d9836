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

constexpr int kSmallLs = 12;   // systems up to this size are solved in registers

// Least squares of Eq. (7) on the newest m_t history columns, solved by
// wave 0 of the calling workgroup (every workgroup of the combine launch
// solves the same tiny system; results are identical).  Column q (0-based,
// newest first) lives in ring slot (s_new - q) mod cap.  Entries of the Gram
// matrix that involve the newest column come from this iteration's partial
// inner products; older entries from the stored Gram matrix.  Writes theta
// (zero for dropped columns) to th[0..mt) and returns the number of columns
// used (0 when the factorisation fails).
__device__ int ls_solve_group(const CombineArgs& a, int s_new, int len_new, int mt, double ridge,
                              double* th, double* newrow, double* bvec, double* Lm, double* sc, double* diag,
                              int* cols, int* misc) {
  const int cap = a.cap;
  const int tid = threadIdx.x;
  // Fixed-order sums of the per-workgroup partials: new Gram row (sums
  // 0..len_new) and rhs (len_new..2 len_new).  Eight lanes share a sum: lane
  // r adds partials r, r + 8, ... in order (up to eight loads in flight),
  // then the eight lane sums are added by a fixed shuffle tree.
  for (int p0 = 0; p0 < 2 * len_new; p0 += (int)blockDim.x / 8) {
    const int p = p0 + tid / 8, r = tid & 7;
    double v = 0.0;
    if (p < 2 * len_new) {
      const int q = p < len_new ? p : p - len_new;
      const int col = (p < len_new ? 0 : cap) + (s_new - q + cap) % cap;
      for (int w0 = r; w0 < a.n_dots; w0 += 64) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int w = w0 + 8 * u;
          t[u] = w < a.n_dots ? a.dots[(int64_t)w * 2 * cap + col] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) v += t[u];
      }
    }
    v += __shfl_xor(v, 1, 8);
    v += __shfl_xor(v, 2, 8);
    v += __shfl_xor(v, 4, 8);
    if (p < 2 * len_new && r == 0) {
      if (p < len_new) newrow[p] = v;
      else bvec[p - len_new] = v;
    }
  }
  __syncthreads();
  auto gram = [&](int q, int r) -> double {   // Gram entry of columns q, r
    if (q == 0) return newrow[r];
    if (r == 0) return newrow[q];
    const int sq = (s_new - q + cap) % cap, sr = (s_new - r + cap) % cap;
    return a.gram[sq * cap + sr];
  };
  for (int q = tid; q < mt; q += blockDim.x) diag[q] = gram(q, q);   // loaded in parallel
  __syncthreads();
  if (tid == 0) {
    int n = 0;
    for (int q = 0; q < mt; ++q) {
      const double nrm = sqrt(diag[q]);
      if (nrm > 0.0) { cols[n] = q; sc[n] = nrm; ++n; }
    }
    misc[0] = n;
    misc[1] = 1;
  }
  __syncthreads();
  const int n = misc[0];
  for (int e = tid; e < n * n; e += blockDim.x) {
    const int r = e / n, q = e - r * n;
    Lm[r * kMaxM + q] = gram(cols[r], cols[q]) / (sc[r] * sc[q]) + (r == q ? ridge : 0.0);
  }
  for (int r = tid; r < n; r += blockDim.x) th[r] = bvec[cols[r]] / sc[r];
  __syncthreads();
  if (n <= kSmallLs) {
    // small systems: Cholesky and both substitutions by one lane in registers
    if (tid == 0) {
      double A[kSmallLs][kSmallLs], z[kSmallLs];
#pragma unroll
      for (int i = 0; i < kSmallLs; ++i) {
        z[i] = i < n ? th[i] : 0.0;
#pragma unroll
        for (int j = 0; j <= i; ++j) A[i][j] = (i < n && j < n) ? Lm[i * kMaxM + j] : (i == j ? 1.0 : 0.0);
      }
      bool good = true;
#pragma unroll
      for (int k = 0; k < kSmallLs; ++k) {
        double p = A[k][k];
#pragma unroll
        for (int q = 0; q < k; ++q) p -= A[k][q] * A[k][q];
        good = good && (p > 0.0);
        const double lkk = sqrt(p > 0.0 ? p : 1.0);
        A[k][k] = lkk;
#pragma unroll
        for (int i = k + 1; i < kSmallLs; ++i) {
          double v = A[i][k];
#pragma unroll
          for (int q = 0; q < k; ++q) v -= A[i][q] * A[k][q];
          A[i][k] = v / lkk;
        }
      }
#pragma unroll
      for (int i = 0; i < kSmallLs; ++i) {        // L z = rhs
        double v = z[i];
#pragma unroll
        for (int q = 0; q < i; ++q) v -= A[i][q] * z[q];
        z[i] = v / A[i][i];
      }
#pragma unroll
      for (int i = kSmallLs - 1; i >= 0; --i) {   // L^T w = z
        double v = z[i];
#pragma unroll
        for (int q = i + 1; q < kSmallLs; ++q) v -= A[q][i] * z[q];
        z[i] = v / A[i][i];
      }
#pragma unroll
      for (int i = 0; i < kSmallLs; ++i) if (i < n) th[i] = z[i];
      if (!good) misc[1] = 0;
    }
    __syncthreads();
  } else {
    // right-looking Cholesky in LDS, one row per thread
    for (int k = 0; k < n; ++k) {
      if (tid == 0) {
        const double p = Lm[k * kMaxM + k];
        if (!(p > 0.0)) misc[1] = 0;
        Lm[k * kMaxM + k] = sqrt(p > 0.0 ? p : 1.0);
      }
      __syncthreads();
      if (tid > k && tid < n) Lm[tid * kMaxM + k] /= Lm[k * kMaxM + k];
      __syncthreads();
      if (tid > k && tid < n) {
        const double lik = Lm[tid * kMaxM + k];
        for (int j = k + 1; j <= tid; ++j) Lm[tid * kMaxM + j] -= lik * Lm[j * kMaxM + k];
      }
      __syncthreads();
    }
    if (tid == 0) {
      for (int i = 0; i < n; ++i) {
        double v = th[i];
        for (int q = 0; q < i; ++q) v -= Lm[i * kMaxM + q] * th[q];
        th[i] = v / Lm[i * kMaxM + i];
      }
      for (int i = n - 1; i >= 0; --i) {
        double v = th[i];
        for (int q = i + 1; q < n; ++q) v -= Lm[q * kMaxM + i] * th[q];
        th[i] = v / Lm[i * kMaxM + i];
      }
    }
    __syncthreads();
  }
  // scatter back to column positions (cols[] is increasing), undo the scaling
  const bool ok = misc[1] != 0;
  if (tid == 0) {
    for (int r = n - 1; r >= 0; --r) {
      const double v = ok ? th[r] / sc[r] : 0.0;
      for (int q = (r + 1 < n ? cols[r + 1] : mt) - 1; q > cols[r]; --q) th[q] = 0.0;
      th[cols[r]] = v;
    }
    for (int q = (n > 0 ? cols[0] : mt) - 1; q >= 0; --q) th[q] = 0.0;
  }
  __syncthreads();
  return ok ? n : 0;
}

// ---------------------------------------------------------------------------
// C^{t+1} = G^t - sum_j theta_j dG_j and the fall-back iterate fl32(G^t),
// each with its squared norms (and bfloat16 hi/lo pairs): one wave per centroid.
// In the solver (gated) each workgroup first solves the least-squares
// problem; workgroup 0 also records the new Gram row and the results.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float put_centroid(float* C, uint16_t* Cb, int64_t KD, int64_t e, double v,
                                              double* nsq, double* e2) {
  const float f = (float)v;
  C[e] = f;
  *nsq = fma((double)f, (double)f, *nsq);
  if (Cb) {
    uint16_t h, l;
    const double r = bf16_split(f, &h, &l);
    Cb[e] = h;
    Cb[KD + e] = l;
    *e2 = fma(r, r, *e2);
  }
  return f;
}

__device__ __forceinline__ void combine_body(const CombineArgs& a, int bx) {
  Ctl* c = a.ctl;
  __shared__ double th[kMaxM], newrow[kMaxM], bvec[kMaxM], sc[kMaxM], diag[kMaxM];
  __shared__ double Lm[kMaxM * kMaxM];
  __shared__ int cols[kMaxM], misc[2];
  int mt = 0, head = 0;
  const int cap = a.cap;
  if (a.gated) {
    if (a.done_out && bx == 0 && threadIdx.x == 0) {   // the host polls this slot
      *(volatile int*)a.done_out = c->done;
      __threadfence_system();
    }
    if (c->done) return;
    const int t = c->t;
    if (cap > 0) {
      const int s_new = (t - 1) % cap;
      const int len_new = t < cap ? t : cap;
      int m = c->m < t ? c->m : t;
      if (m > len_new) m = len_new;
      const int used = ls_solve_group(a, s_new, len_new, m, c->ridge, th, newrow, bvec, Lm, sc, diag, cols, misc);
      if (bx == 0) {
        for (int q = threadIdx.x; q < len_new; q += blockDim.x) {
          const int sl = (s_new - q + cap) % cap;
          a.gram[s_new * cap + sl] = newrow[q];
          a.gram[sl * cap + s_new] = newrow[q];
        }
        if (threadIdx.x == 0) {
          for (int q = 0; q < m; ++q) c->theta[q] = th[q];
          c->mt = m;
          c->used = used;
          c->cand_is_lloyd = (used == 0) ? 1 : 0;
          if (a.trace_rec) {
            double* rec = a.trace_rec + (int64_t)t * kTraceRec;
            rec[8] = m;
            rec[9] = used;
            for (int q = 0; q < m; ++q) rec[16 + q] = th[q];
          }
        }
      }
      mt = used > 0 ? m : 0;
      head = s_new;
    } else if (bx == 0 && threadIdx.x == 0) {
      c->mt = 0;
      c->used = 0;
      c->cand_is_lloyd = 1;
    }
  }
  const int lane = threadIdx.x & 63;
  const int j = bx * 4 + (threadIdx.x >> 6);
  if (j >= a.K) return;
  const int d = a.d;
  const int64_t KD = (int64_t)a.K * d;
  double n_c = 0.0, e_c = 0.0, n_f = 0.0, e_f = 0.0, s_c = 0.0, s_f = 0.0;
  for (int k = lane; k < d; k += kWave) {
    const int64_t e = (int64_t)j * d + k;
    const double g = a.G_last[e];
    double v = g;
    for (int q0 = 0; q0 < mt; q0 += 8) {   // history columns in order, 8 loads in flight
      double r[8];
#pragma unroll
      for (int q8 = 0; q8 < 8; ++q8) {
        const int sl = (head - (q0 + q8) + cap) % cap;
        r[q8] = q0 + q8 < mt ? a.ring_dG[(int64_t)sl * KD + e] : 0.0;
      }
#pragma unroll
      for (int q8 = 0; q8 < 8; ++q8)
        if (q0 + q8 < mt) v -= th[q0 + q8] * r[q8];
    }
    const float fc = put_centroid(a.C_cand, a.Cb_cand, KD, e, v, &n_c, &e_c);
    const float ff = put_centroid(a.C_fb, a.Cb_fb, KD, e, g, &n_f, &e_f);
    if (a.C_ref) {   // shifts of the stored float32 values against the reference
      const double r = a.C_ref[e];
      s_c = fma((double)fc - r, (double)fc - r, s_c);
      s_f = fma((double)ff - r, (double)ff - r, s_f);
    }
  }
  n_c = wave_sum(n_c);
  e_c = wave_sum(e_c);
  n_f = wave_sum(n_f);
  e_f = wave_sum(e_f);
  if (a.C_ref) {
    s_c = wave_sum(s_c);
    s_f = wave_sum(s_f);
  }
  if (lane == 0) {
    a.nc_cand[j] = (float)n_c;
    a.nc_fb[j] = (float)n_f;
    if (a.Cb_cand) a.delta_cand[j] = (float)sqrt(e_c);
    if (a.Cb_fb) a.delta_fb[j] = (float)sqrt(e_f);
    if (a.C_ref) {   // rounded up: upper bounds of the shifts
      a.sh_cand[j] = sqrt(s_c) * (1.0 + 1e-12);
      a.sh_fb[j] = sqrt(s_f) * (1.0 + 1e-12);
    }
  }
}

__global__ __launch_bounds__(256) void k_combine(CombineArgs a) { combine_body(a, blockIdx.x); }

__global__ __launch_bounds__(256) void k_combine_batch(BatchRef<CombineArgs> t) {
  const int b = batch_find(t.prefix, t.n, blockIdx.x);
  combine_body(t.tab[b], blockIdx.x - t.prefix[b]);
}

int combine_grid(int K) { return (K + 3) / 4; }

hipError_t launch_combine_batch(const CombineArgs* tab, const int* prefix, int n, int blocks, hipStream_t s) {
  clear_pending_error();
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine_batch, dim3(blocks), dim3(256), 0, s, BatchRef<CombineArgs>{tab, prefix, n});
  return hipGetLastError();
}

hipError_t launch_combine(const CombineArgs& a, hipStream_t s, hipEvent_t ev1) {
  if (a.cap > kMaxM) return hipErrorInvalidValue;
  clear_pending_error();
  if (ev1)
    hipExtLaunchKernelGGL(k_combine, dim3((a.K + 3) / 4), dim3(256), 0, s, nullptr, ev1, 0, a);
  else
    hipLaunchKernelGGL(k_combine, dim3((a.K + 3) / 4), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace km
