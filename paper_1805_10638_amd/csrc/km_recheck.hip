// Re-check of the rows an assignment pass could not decide (Sec. 1, Eq. (3)
// exactly): one launch over the whole pass's flagged rows.
//
// An assignment launch in list mode (AssignArgs::fl_cnt set) leaves the rows
// whose two best GEMM scores lie within the rounding bound in its per-wave
// lists (the p-th row wave w of workgroup b flags is stored in the slot of
// the p-th row that wave owns) and writes the list lengths.  This kernel
// numbers the listed rows in (workgroup, wave, position) order and takes them
// in batches of kReRows (kReMR per wave), so that a few thousand listed rows
// still spread over every CU.  A batch's rows are staged in LDS as float64
// and float32; the float32 centroids stream through LDS in chunks of 64 (one
// per lane) and every chunk serves the whole batch.
//
// For every listed row the result is that of float64 direct differences to
// all K centroids: the lowest index among the smallest distances, and the
// second smallest distance (near ties by the float64 definition are counted).
// The float64 distance is computed only for candidates: each wave first
// scores a 16-centroid tile of the chunk against the batch's 16 rows with
// float32 MFMA, s_j = x.c_j - ||c_j||^2 / 2 (the assignment kernel's float32
// tile product), whose error is at most B = gamma_{dp+3} (||x|| + max ||c||)^2
// (plus an absolute term for underflow); the squared distance is
// ||x||^2 - 2 s_j.  With M the largest
// float32 score seen so far, every centroid scored below
// M - 2B - 0.51e-6 (||x|| + max ||c||)^2 is farther than the best by more
// than the near-tie margin, so it is neither the argmin nor a near tie and
// its distance is not needed; the others get float64 distances (lanes split
// the dimensions, then a fixed-order wave sum).  The smallest distance with
// the lowest index and the second smallest are kept per wave and row, then
// merged over the waves.
// Non-finite scores or bounds make every centroid a candidate.  The energy
// terms of the rows are added in batch and row order into one partial per
// workgroup, so the pass's energy does not depend on timing.

#include "km_assign_kernel.h"

namespace km {

constexpr int kReThreads = 256;
constexpr int kReWaves = kReThreads / 64;
constexpr int kReMR = 4;                     // rows per wave and batch
constexpr int kReRows = kReWaves * kReMR;    // rows per batch
constexpr int kReCRows = 64;                 // centroid rows per LDS chunk (one per lane)
constexpr int kReBatch = 8;                  // 16-byte loads in flight per thread while staging

// Four consecutive values of a row of X from element e (all inside the row),
// as float32.
__device__ __forceinline__ float4 ld_x4(const void* X, int64_t e, bool bf) {
  if (bf) {
    const uint2 v = *(const uint2*)((const uint16_t*)X + e);
    return make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xFFFF0000u),
                       __uint_as_float(v.y << 16), __uint_as_float(v.y & 0xFFFF0000u));
  }
  return *(const float4*)((const float*)X + e);
}

// LDS bytes of k_recheck for width d and an assignment grid of `grid`.
size_t recheck_lds(int d, int grid) {
  const int dp = (d + 15) & ~15;
  return (size_t)kReRows * dp * 8 + (size_t)kReRows * 8 + (size_t)kReRows * (dp + 4) * 4 +
         (size_t)kReCRows * (dp + 4) * 4 + (size_t)kReCRows * 4 + (size_t)kReRows * 8 +
         (size_t)kReWaves * kReRows * (8 + 8 + 4 + 4) + (size_t)kReRows * 4 + (size_t)kReWaves * 4 +
         (size_t)(grid + 1) * 4;
}

// bx / gx: this workgroup's index and the workgroups of this instance
__device__ __forceinline__ void recheck_body(const RecheckArgs& r, int bx, int gx) {
  Ctl* ctl = r.ctl;
  if (r.role != kRolePlain) {
    if (ctl->done) return;
    if (r.role == kRoleFallback && !ctl->reject) return;
  }
  int* rho;
  const int* prev;
  if (r.role == kRoleCand) {
    rho = r.lab + (int64_t)ctl->lab_cand * r.N;
    prev = r.lab + (int64_t)ctl->lab_prev * r.N;
  } else if (r.role == kRoleFallback) {
    rho = r.lab + (int64_t)ctl->lab_fb * r.N;
    prev = r.lab + (int64_t)ctl->lab_prev * r.N;
  } else {
    rho = r.lab;
    prev = r.lab_prev;
  }
  const int slot = (r.role == kRoleFallback) ? 1 : 0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // rows padded with zeros to dp (a multiple of 16: the MFMA tile takes dp / 4
  // dimensions per lane group, four at a time); LDS row stride dp + 4
  const int d = r.d, K = r.K, dp = (d + 15) & ~15, LDc = dp + 4;
  const int grid = r.grid;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* xs = (double*)smem_raw;                            // kReRows x dp
  double* rowterm = xs + (size_t)kReRows * dp;               // kReRows
  float* xsf = (float*)(rowterm + kReRows);                  // kReRows x (dp + 4) (float32 copies)
  float* cc = xsf + (size_t)kReRows * LDc;                   // kReCRows x (dp + 4)
  float* ncc = cc + (size_t)kReCRows * LDc;                  // kReCRows: -||c||^2 / 2 of the chunk
  double* margs = (double*)(ncc + kReCRows);                 // kReRows: margin of the score test
  double* st_bd = margs + kReRows;                           // kReWaves x kReRows: smallest distance
  double* st_bd2 = st_bd + kReWaves * kReRows;               //   second smallest
  int* st_bj = (int*)(st_bd2 + kReWaves * kReRows);          //   index of the smallest
  float* smx = (float*)(st_bj + kReWaves * kReRows);         // kReWaves x kReRows: tile maxima
  int* rowidx = (int*)(smx + kReWaves * kReRows);            // kReRows
  int* wsum = rowidx + kReRows;                              // kReWaves
  int* pre = wsum + kReWaves;                                // grid + 1

  // flagged rows before workgroup b of the assignment launch: pre[b]
  // (each thread sums a run of workgroups, then one scan over the threads)
  {
    const int per = (grid + kReThreads - 1) / kReThreads;
    const int b0 = tid * per, b1 = (b0 + per) < grid ? (b0 + per) : grid;
    int s = 0;
    for (int b = b0; b < b1; ++b) {
      int c = 0;
      for (int w = 0; w < r.W; ++w) c += r.fl_cnt[b * 16 + w];
      pre[b + 1] = c;
      s += c;
    }
    int incl = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int o = __shfl_up(incl, off, kWave);
      if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int run = incl - s;
    for (int w = 0; w < wave; ++w) run += wsum[w];
    for (int b = b0; b < b1; ++b) {
      run += pre[b + 1];
      pre[b + 1] = run;
    }
    if (tid == 0) pre[0] = 0;
    __syncthreads();
  }
  const int F = pre[grid];
  const int nbatch = (F + kReRows - 1) / kReRows;
  if (bx >= nbatch) {   // no rows for this workgroup
    if (tid == 0) r.e_part[bx] = 0.0;
    return;
  }
  // largest centroid norm (from the float32 squared norms, rounded up)
  double cmax;
  {
    float mx = 0.f;
    for (int j = tid; j < K; j += kReThreads) mx = fmaxf(mx, r.nc[j]);
    mx = wave_max(mx);
    __syncthreads();
    if (lane == 0) wsum[wave] = __float_as_int(mx);
    __syncthreads();
    for (int w = 0; w < kReWaves; ++w) mx = fmaxf(mx, __int_as_float(wsum[w]));
    cmax = sqrt((double)mx) * (1.0 + 1e-6);
    __syncthreads();
  }
  // error bound factor of a float32 MFMA score of dp terms and the start value
  const double gam = (double)(dp + 3) * 0x1p-24 / (1.0 - (double)(dp + 3) * 0x1p-24);

  double e_sum = 0.0;
  unsigned n_changed = 0, n_near = 0;
  const int q4 = dp / 4;
  const bool xbf = r.xbf16 != 0;
  for (int bt = bx; bt < nbatch; bt += gx) {
    const int rb = (F - bt * kReRows) < kReRows ? (F - bt * kReRows) : kReRows;
    if (tid < rb) {   // listed row number f: its workgroup, wave, list position, slot
      const int f = bt * kReRows + tid;
      int lo = 0, hi = grid;   // largest b with pre[b] <= f
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= f) lo = mid; else hi = mid;
      }
      int q = f - pre[lo], w = 0;
      while (w < r.W - 1 && q >= r.fl_cnt[lo * 16 + w]) { q -= r.fl_cnt[lo * 16 + w]; ++w; }
      const int64_t own = ((int64_t)lo + (int64_t)(q / r.sb16) * grid) * r.group_rows + (int64_t)w * r.sb16 +
                          q % r.sb16;
      rowidx[tid] = r.flags[own];
    }
    __syncthreads();
    // the batch's rows as float64 (exact for float32 and bfloat16 storage)
    // and float32, zero beyond d and rb; 16-byte loads when d is a multiple of 4
    if ((d & 3) == 0) {
      for (int e = tid; e < kReRows * q4; e += kReThreads) {
        const int u = e / q4, k = (e - u * q4) * 4;
        const float4 v = (u < rb && k < d) ? ld_x4(r.X, (int64_t)rowidx[u] * d + k, xbf)
                                           : make_float4(0.f, 0.f, 0.f, 0.f);
        double2* dst = (double2*)(xs + (size_t)u * dp + k);
        dst[0] = make_double2(v.x, v.y);
        dst[1] = make_double2(v.z, v.w);
        *(float4*)(xsf + (size_t)u * LDc + k) = v;
      }
    } else {
      for (int e = tid; e < kReRows * dp; e += kReThreads) {
        const int u = e / dp, k = e - u * dp;
        float v = 0.f;
        if (u < rb && k < d) v = ld_x(r.X, (int64_t)rowidx[u] * d + k, xbf);
        xs[e] = v;
        xsf[(size_t)u * LDc + k] = v;
      }
    }
    __syncthreads();   // rows staged
    // per row: the margin 2B + 0.51e-6 (||x|| + max||c||)^2 of the score
    // test; per wave and row: the float64 result so far
    if (tid < kReRows) {
      double q = 0.0;
      for (int k = 0; k < dp; ++k) q = fma(xs[tid * dp + k], xs[tid * dp + k], q);
      const double nb = sqrt(q) * (1.0 + 1e-12) + cmax;
      margs[tid] = 2.0 * (1.01 * gam * nb * nb + (double)(dp + 3) * 0x1p-125) + 0.51e-6 * nb * nb;
    }
    if (tid < kReWaves * kReRows) {
      st_bd[tid] = __builtin_inf();
      st_bd2[tid] = __builtin_inf();
      st_bj[tid] = -1;
    }
    __syncthreads();
    // this lane's tile position: centroid row 16 * wave + r16 (A operand),
    // row r16 of the batch (B operand), dimensions g * KS ... g * KS + KS - 1
    const int g = lane >> 4, r16 = lane & 15, KS = dp >> 2;
    const float* brow = xsf + (size_t)r16 * LDc + g * KS;
    const double marg = margs[r16];
    float smax = -__builtin_inff();   // largest score of row r16 so far
    for (int c0 = 0; c0 < K; c0 += kReCRows) {
      const int rows = (K - c0) < kReCRows ? (K - c0) : kReCRows;
      __syncthreads();
      if ((d & 3) == 0) {   // 16-byte loads, kReBatch in flight per thread
        for (int e0 = tid; e0 < kReCRows * q4; e0 += kReBatch * kReThreads) {
          float4 v[kReBatch];
#pragma unroll
          for (int t = 0; t < kReBatch; ++t) {
            const int e = e0 + t * kReThreads, jj = e / q4, k = (e - jj * q4) * 4;
            v[t] = (e < kReCRows * q4 && jj < rows && k < d) ? *(const float4*)(r.C + (int64_t)(c0 + jj) * d + k)
                                                             : make_float4(0.f, 0.f, 0.f, 0.f);
          }
#pragma unroll
          for (int t = 0; t < kReBatch; ++t) {
            const int e = e0 + t * kReThreads, jj = e / q4, k = (e - jj * q4) * 4;
            if (e < kReCRows * q4) *(float4*)(cc + jj * LDc + k) = v[t];
          }
        }
      } else {
        for (int e = tid; e < kReCRows * dp; e += kReThreads) {
          const int jj = e / dp, k = e - jj * dp;
          cc[jj * LDc + k] = (jj < rows && k < d) ? r.C[(int64_t)(c0 + jj) * d + k] : 0.f;
        }
      }
      if (tid < kReCRows) ncc[tid] = tid < rows ? -0.5f * r.nc[c0 + tid] : -__builtin_inff();
      __syncthreads();
      // float32 scores of centroids 16 * wave + 4 g + i (i < 4) for row r16
      const int jt = 16 * wave + 4 * g;
      f32x4 acc = *(const f32x4*)(ncc + jt);
      const float* arow = cc + (size_t)(16 * wave + r16) * LDc + g * KS;
      for (int q = 0; q < KS; q += 4) {
        const float4 a4 = *(const float4*)(arow + q);
        const float4 b4 = *(const float4*)(brow + q);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.x, b4.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.y, b4.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.z, b4.z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.w, b4.w, acc, 0, 0, 0);
      }
      float t[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) t[i] = (jt + i < rows) ? acc[i] : -__builtin_inff();
      // largest score of each row over the chunk: lane, lane groups, waves
      float m = fmaxf(fmaxf(t[0], t[1]), fmaxf(t[2], t[3]));
      m = fmaxf(m, __shfl_xor(m, 16, kWave));
      m = fmaxf(m, __shfl_xor(m, 32, kWave));
      if (g == 0) smx[wave * kReRows + r16] = m;
      __syncthreads();
#pragma unroll
      for (int w = 0; w < kReWaves; ++w) smax = fmaxf(smax, smx[w * kReRows + r16]);
      const double thr = (isfinite(smax) && isfinite(marg)) ? (double)smax - marg : -__builtin_inf();
      // candidates: float64 distance, lanes split the dimensions; the wave's
      // result for the row is updated by lane 0 (the same on every lane)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        unsigned long long cand = __ballot(r16 < rb && jt + i < rows && !((double)t[i] < thr));
        while (cand) {
          const int l = __ffsll((long long)cand) - 1;
          cand &= cand - 1;
          const int u = l & 15, jj = 16 * wave + 4 * (l >> 4) + i;
          const float* cr = cc + (size_t)jj * LDc;
          double p = 0.0;
          for (int k = lane; k < dp; k += kWave) {
            const double df = xs[u * dp + k] - (double)cr[k];
            p = fma(df, df, p);
          }
          const double dist = wave_sum(p);
          if (lane == 0) {
            const int o = wave * kReRows + u, j = c0 + jj;
            const double b = st_bd[o];
            if (dist < b || (dist == b && j < st_bj[o])) {
              st_bd2[o] = fmin(st_bd2[o], b);
              st_bd[o] = dist;
              st_bj[o] = j;
            } else {
              st_bd2[o] = fmin(st_bd2[o], dist);
            }
          }
        }
      }
    }
    __syncthreads();
    // merge the waves' results per row: lowest index among the smallest
    // distances, second smallest distance
    bool ch = false, nt = false;
    if (tid < rb) {
      double bd = st_bd[tid], bd2 = st_bd2[tid];
      int bj = st_bj[tid];
      for (int w = 1; w < kReWaves; ++w) {
        const double ob = st_bd[w * kReRows + tid], ob2 = st_bd2[w * kReRows + tid];
        const int oj = st_bj[w * kReRows + tid];
        const bool take = (ob < bd) || (ob == bd && (unsigned)oj < (unsigned)bj);
        const double hi = bd < ob ? ob : bd, lo2 = bd2 < ob2 ? bd2 : ob2;
        bd2 = hi < lo2 ? hi : lo2;
        bd = take ? ob : bd;
        bj = take ? oj : bj;
      }
      const int i = rowidx[tid];
      const int jl = bj >= 0 ? bj : 0;
      rho[i] = jl;
      ch = (prev != nullptr) && (prev[i] != jl);
      nt = near_tie(bd, bd2);
      rowterm[tid] = bd;
    }
    if (wave == 0) {
      n_changed += (unsigned)__popcll(__ballot(ch));
      n_near += (unsigned)__popcll(__ballot(nt));
    }
    __syncthreads();
    if (tid == 0)
      for (int u = 0; u < rb; ++u) e_sum += rowterm[u];
  }
  if (lane == 0) {
    if (n_changed) atomicAdd(&ctl->cnt_changed[slot], (unsigned long long)n_changed);
    if (n_near) atomicAdd(&ctl->cnt_near[slot], (unsigned long long)n_near);
  }
  if (tid == 0) r.e_part[bx] = e_sum;
}

__global__ __launch_bounds__(kReThreads) void k_recheck(RecheckArgs r) { recheck_body(r, blockIdx.x, gridDim.x); }

// Batched: instance b gets prefix[b + 1] - prefix[b] workgroups.
__global__ __launch_bounds__(kReThreads) void k_recheck_batch(BatchRef<RecheckArgs> t) {
  const int b = batch_find(t.prefix, t.n, blockIdx.x);
  const RecheckArgs r = t.tab[b];   // a copy: no reloads after stores that could alias the table
  recheck_body(r, blockIdx.x - t.prefix[b], t.prefix[b + 1] - t.prefix[b]);
}

hipError_t launch_recheck_batch(const RecheckArgs* tab, const int* prefix, int n, int blocks, size_t lds,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  static bool attr = false;
  if (!attr) {
    const hipError_t e = hipFuncSetAttribute((const void*)&k_recheck_batch,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  clear_pending_error();
  hipLaunchKernelGGL(k_recheck_batch, dim3(blocks), dim3(kReThreads), lds, s,
                     BatchRef<RecheckArgs>{tab, prefix, n});
  return hipGetLastError();
}

hipError_t launch_recheck(const RecheckArgs& a, Role role, hipStream_t s, hipEvent_t ev1) {
  if (a.d <= 0 || a.d > kMaxD || a.K <= 0 || a.grid <= 0 || a.grid > kReMaxGrid || a.W <= 0 || a.W > 16)
    return hipErrorInvalidValue;
  RecheckArgs arg = a;
  arg.role = role;
  const size_t lds = recheck_lds(a.d, a.grid);
  static bool attr = false;
  if (!attr) {
    const hipError_t e = hipFuncSetAttribute((const void*)&k_recheck, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  clear_pending_error();
  if (ev1) {
    void* params[] = {&arg};
    return hipExtLaunchKernel((const void*)&k_recheck, dim3(kReGrid), dim3(kReThreads), params, lds, s, nullptr,
                              ev1, 0);
  }
  hipLaunchKernelGGL(k_recheck, dim3(kReGrid), dim3(kReThreads), lds, s, arg);
  return hipGetLastError();
}

}  // namespace km
