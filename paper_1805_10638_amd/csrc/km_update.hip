// Update step (Sec. 1, Eq. (4)): c_j = mean of the samples labelled j.
//
// Deterministic and atomic-free in floating point:
//   1. k_rank     stable within-block ranks of every label (wave match by
//                 ballots, per-wave LDS counters) and a per-block histogram;
//   2. k_scan     per-label exclusive prefix of the block histograms;
//   3. k_offsets  segment starts and the list of work items, each item being
//                 at most kSegRows consecutive samples of one cluster;
//   4. k_scatter  perm[segment start + block offset + rank] = i  (a stable
//                 counting sort by label);
//   5. k_segsum   one workgroup per item gathers its rows and sums them in
//                 float64, reducing across row groups through LDS in a fixed
//                 order;
//   6. k_finalize sums the items of each cluster in order and divides by the
//                 count (an empty cluster keeps its centroid).  In the solver
//                 it also forms the residual F = G - C, pushes the newest
//                 differences of F and G into the history ring and emits the
//                 partial inner products of the Anderson Gram matrix.

#include "km_launch.h"

namespace km {

__device__ __forceinline__ const int* labels_of(const UpdateArgs& u) {
  return u.lab_from_ctl ? u.lab + (int64_t)u.ctl->lab_prev * u.N : u.lab;
}

// ---------------------------------------------------------------------------
// 1. ranks within blocks of kRankRows rows
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_rank(UpdateArgs u) {
  if (u.gated && u.ctl->done) return;
  __shared__ int cnt[4][kMaxK];
  const int* L = labels_of(u);
  const int K = u.K;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int j = tid; j < 4 * K; j += 256) cnt[j / K][j % K] = 0;
  __syncthreads();

  int nbits = 0;
  while ((1 << nbits) < K) ++nbits;
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  constexpr int kChunks = kRankRows / 256;   // 64-row chunks per wave
  int labs[kChunks], rk[kChunks];
  const int64_t base = (int64_t)blockIdx.x * kRankRows + (int64_t)w * (kChunks * 64);
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const int64_t i = base + c * 64 + lane;
    const bool valid = i < u.N;
    int lab = valid ? L[i] : 0;
    if (lab < 0 || lab >= K) lab = 0;
    unsigned long long m = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
      const bool bit = (lab >> b) & 1;
      const unsigned long long bb = __ballot(valid && bit);
      m &= bit ? bb : ~bb;
    }
    if (!valid) m = 0;
    const int before = __popcll(m & lt);
    const int tot = __popcll(m);
    const int prior = valid ? cnt[w][lab] : 0;
    rk[c] = prior + before;
    labs[c] = lab;
    if (valid && before == tot - 1) cnt[w][lab] = prior + tot;
  }
  __syncthreads();
  for (int j = tid; j < K; j += 256) {
    int s = 0;
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) {
      const int v = cnt[ww][j];
      cnt[ww][j] = s;
      s += v;
    }
    u.blockcount[(int64_t)blockIdx.x * K + j] = s;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const int64_t i = base + c * 64 + lane;
    if (i < u.N) u.lrank[i] = rk[c] + cnt[w][labs[c]];
  }
}

// ---------------------------------------------------------------------------
// 2. per-label prefix over blocks (64 labels x 4 block ranges per workgroup)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scan(UpdateArgs u, int nblk) {
  if (u.gated && u.ctl->done) return;
  __shared__ int part[4][64];
  const int K = u.K;
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const int p = threadIdx.x >> 6;
  const int b0 = (int)((int64_t)nblk * p / 4), b1 = (int)((int64_t)nblk * (p + 1) / 4);
  int s = 0;
  if (j < K)
    for (int b = b0; b < b1; ++b) s += u.blockcount[(int64_t)b * K + j];
  part[p][threadIdx.x & 63] = s;
  __syncthreads();
  int run = 0;
  for (int q = 0; q < p; ++q) run += part[q][threadIdx.x & 63];
  if (j < K) {
    for (int b = b0; b < b1; ++b) {
      const int64_t idx = (int64_t)b * K + j;
      const int v = u.blockcount[idx];
      u.blockcount[idx] = run;
      run += v;
    }
    if (p == 3) u.counts[j] = run;
  }
}

// ---------------------------------------------------------------------------
// 3. segment starts and work items (one workgroup of 1024 threads)
// ---------------------------------------------------------------------------
__device__ int block_exclusive_scan_1024(int v, int* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int add = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  const int incl = sh[t];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(1024) void k_offsets(UpdateArgs u) {
  if (u.gated && u.ctl->done) return;
  __shared__ int sh[1024];
  const int K = u.K;
  const int per = (K + 1023) / 1024;
  const int j0 = threadIdx.x * per;
  int csum = 0, isum = 0, empty = 0;
  for (int j = j0; j < j0 + per && j < K; ++j) {
    const int c = u.counts[j];
    csum += c;
    isum += (c + kSegRows - 1) / kSegRows;
    empty += (c == 0);
  }
  int cbase = block_exclusive_scan_1024(csum, sh);
  int ibase = block_exclusive_scan_1024(isum, sh);
  int etot = block_exclusive_scan_1024(empty, sh) + empty;   // inclusive at the last thread
  for (int j = j0; j < j0 + per && j < K; ++j) {
    const int c = u.counts[j];
    const int ni = (c + kSegRows - 1) / kSegRows;
    u.seg_start[j] = cbase;
    u.item_start[j] = ibase;
    for (int q = 0; q < ni; ++q)
      if (ibase + q < u.max_items) u.item_cluster[ibase + q] = j;
    cbase += c;
    ibase += ni;
  }
  if (threadIdx.x == 1023) {
    u.seg_start[K] = cbase;
    u.item_start[K] = ibase;
    u.ctl->total_items = ibase < u.max_items ? ibase : u.max_items;
    u.ctl->empty = etot;
  }
}

// ---------------------------------------------------------------------------
// 4. stable scatter
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scatter(UpdateArgs u) {
  if (u.gated && u.ctl->done) return;
  const int* L = labels_of(u);
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= u.N) return;
  int lab = L[i];
  if (lab < 0 || lab >= u.K) lab = 0;
  const int64_t b = i / kRankRows;
  const int64_t pos = (int64_t)u.seg_start[lab] + u.blockcount[b * u.K + lab] + u.lrank[i];
  if (pos >= 0 && pos < u.N) u.perm[pos] = (int)i;
}

// ---------------------------------------------------------------------------
// 5. segmented sums: one workgroup per work item
// ---------------------------------------------------------------------------
template <bool XBF>
__global__ __launch_bounds__(256) void k_segsum(UpdateArgs u) {
  if (u.gated && u.ctl->done) return;
  const int item = blockIdx.x;
  if (item >= u.ctl->total_items) return;
  __shared__ double red[256 * 4];
  const int d = u.d;
  const int j = u.item_cluster[item];
  const int c = item - u.item_start[j];
  const int64_t p0 = (int64_t)u.seg_start[j] + (int64_t)c * kSegRows;
  const int64_t pend = (int64_t)u.seg_start[j] + u.counts[j];
  const int64_t p1 = (p0 + kSegRows < pend) ? p0 + kSegRows : pend;

  // threads per row: power of two covering ceil(d/4) float4 columns (<= 64)
  int tpr = 1;
  while (tpr * 4 < d) tpr <<= 1;
  const int rpp = 256 / tpr;                 // rows per pass
  const int col = threadIdx.x % tpr, rg = threadIdx.x / tpr;
  const int k0 = col * 4;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const bool vec = (d % 4) == 0 && k0 + 4 <= d;
  for (int64_t p = p0 + rg; p < p1; p += rpp) {
    const int64_t i = u.perm[p];
    if (XBF) {
      const uint16_t* xr = (const uint16_t*)u.X + i * d;
      if (vec) {
        const uint2 v = *(const uint2*)(xr + k0);
        acc[0] += (double)__uint_as_float(v.x << 16);
        acc[1] += (double)__uint_as_float(v.x & 0xFFFF0000u);
        acc[2] += (double)__uint_as_float(v.y << 16);
        acc[3] += (double)__uint_as_float(v.y & 0xFFFF0000u);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (k0 + e < d) acc[e] += (double)__uint_as_float(((uint32_t)xr[k0 + e]) << 16);
      }
    } else {
      const float* xr = (const float*)u.X + i * d;
      if (vec) {
        const float4 v = *(const float4*)(xr + k0);
        acc[0] += (double)v.x;
        acc[1] += (double)v.y;
        acc[2] += (double)v.z;
        acc[3] += (double)v.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (k0 + e < d) acc[e] += (double)xr[k0 + e];
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) red[(rg * tpr + col) * 4 + e] = acc[e];
  __syncthreads();
  for (int k = threadIdx.x; k < d; k += 256) {
    const int cc = k / 4, e = k % 4;
    double s = 0.0;
    for (int r = 0; r < rpp; ++r) s += red[(r * tpr + cc) * 4 + e];
    u.partial[(int64_t)item * d + k] = s;
  }
}

int update_rank_blocks(int64_t N) { return (int)((N + kRankRows - 1) / kRankRows); }
int update_max_items(int64_t N, int K) { return (int)((N + kSegRows - 1) / kSegRows) + K; }

hipError_t launch_update_sums(const UpdateArgs& u, hipStream_t s) {
  if (u.K > kMaxK || u.d > kMaxD) return hipErrorInvalidValue;
  const int nblk = update_rank_blocks(u.N);
  hipLaunchKernelGGL(k_rank, dim3(nblk), dim3(256), 0, s, u);
  hipLaunchKernelGGL(k_scan, dim3((u.K + 63) / 64), dim3(256), 0, s, u, nblk);
  hipLaunchKernelGGL(k_offsets, dim3(1), dim3(1024), 0, s, u);
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)((u.N + 255) / 256)), dim3(256), 0, s, u);
  if (u.xbf16)
    hipLaunchKernelGGL(k_segsum<true>, dim3(u.max_items), dim3(256), 0, s, u);
  else
    hipLaunchKernelGGL(k_segsum<false>, dim3(u.max_items), dim3(256), 0, s, u);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 6. means, residual, history push and Gram partials (one wave per cluster)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t x = __float_as_uint(f);
  x += 0x7FFFu + ((x >> 16) & 1u);
  return (uint16_t)(x >> 16);
}

// Writes fl32(v) into C and returns its float32 value; also the bf16 shadow.
__device__ __forceinline__ float store_centroid(float* C, uint16_t* Cb, int64_t idx, double v,
                                                double* err2) {
  const float f = (float)v;
  C[idx] = f;
  if (Cb) {
    const uint16_t b = f32_to_bf16(f);
    Cb[idx] = b;
    const double df = (double)f - (double)__uint_as_float(((uint32_t)b) << 16);
    *err2 = fma(df, df, *err2);
  }
  return f;
}

__global__ __launch_bounds__(256) void k_finalize(FinalizeArgs f) {
  Ctl* ctl = f.ctl;
  if (f.mode == kFinIter && ctl->done) return;
  __shared__ double wsum[4][2 * kMaxM];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.x * 4 + w;
  const int d = f.d, cap = f.cap;
  const bool active = j < f.K;

  int s_new = 0, len_new = 0, head = 0;
  if (f.mode == kFinIter && cap > 0) {
    head = ctl->hist_head;
    s_new = (ctl->hist_len == 0) ? 0 : (head + 1) % cap;
    len_new = ctl->hist_len + 1 < cap ? ctl->hist_len + 1 : cap;
  }
  const float* Cacc = (f.mode == kFinIter && ctl->acc_src == 1) ? f.C_fb : f.C_cand;
  const int64_t KD = (int64_t)f.K * d;

  if (active) {
    const int n = f.counts[j];
    const int i0 = f.item_start[j], i1 = f.item_start[j + 1];
    double nsq_fb = 0.0, e_fb = 0.0, nsq_c = 0.0, e_c = 0.0;
    for (int k = lane; k < d; k += kWave) {
      double sum = 0.0;
      for (int it = i0; it < i1; ++it) sum += f.partial[(int64_t)it * d + k];
      const int64_t e = (int64_t)j * d + k;
      if (f.mode == kFinG) {
        const double gv = n > 0 ? sum / (double)n : (double)f.C_in[e];
        f.C_out[e] = (float)gv;
        continue;
      }
      const double cin = (f.mode == kFinInit) ? (double)f.C_in[e] : (double)Cacc[e];
      const double gv = n > 0 ? sum / (double)n : cin;
      const double fv = gv - cin;
      if (f.mode == kFinIter && cap > 0) {
        f.ring_dF[(int64_t)s_new * KD + e] = fv - f.F_last[e];
        f.ring_dG[(int64_t)s_new * KD + e] = gv - f.G_last[e];
      }
      f.G_last[e] = gv;
      f.F_last[e] = fv;
      const float gf = store_centroid(f.C_fb, f.Cb_fb, e, gv, &e_fb);
      nsq_fb = fma((double)gf, (double)gf, nsq_fb);
      if (f.mode == kFinInit) {
        const float cf = store_centroid(f.C_cand_w, f.Cb_cand, e, gv, &e_c);
        nsq_c = fma((double)cf, (double)cf, nsq_c);
      }
    }
    if (f.mode != kFinG) {
      nsq_fb = wave_sum(nsq_fb);
      e_fb = wave_sum(e_fb);
      if (lane == 0) {
        f.nc_fb[j] = (float)nsq_fb;
        if (f.Cb_fb) f.delta_fb[j] = (float)sqrt(e_fb);
      }
      if (f.mode == kFinInit) {
        nsq_c = wave_sum(nsq_c);
        e_c = wave_sum(e_c);
        if (lane == 0) {
          f.nc_cand[j] = (float)nsq_c;
          if (f.Cb_cand) f.delta_cand[j] = (float)sqrt(e_c);
        }
      }
    }
  }
  if (f.mode != kFinIter || cap == 0) return;

  // Partial inner products for the Gram matrix: for every valid slot s,
  // <dF_new, dF_s> (index s) and <dF_s, F^t> (index cap + s).  Each lane
  // reads back only elements it wrote above.
  for (int q = 0; q < len_new; ++q) {
    const int sl = (s_new - q + cap) % cap;
    double a = 0.0, b = 0.0;
    if (active) {
      for (int k = lane; k < d; k += kWave) {
        const int64_t e = (int64_t)j * d + k;
        const double dfs = f.ring_dF[(int64_t)sl * KD + e];
        a = fma(f.ring_dF[(int64_t)s_new * KD + e], dfs, a);
        b = fma(dfs, f.F_last[e], b);
      }
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) {
      wsum[w][sl] = a;
      wsum[w][cap + sl] = b;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < len_new; q += 256) {
    const int sl = (s_new - q + cap) % cap;
    f.dots[(int64_t)blockIdx.x * 2 * cap + sl] =
        ((wsum[0][sl] + wsum[1][sl]) + wsum[2][sl]) + wsum[3][sl];
    f.dots[(int64_t)blockIdx.x * 2 * cap + cap + sl] =
        ((wsum[0][cap + sl] + wsum[1][cap + sl]) + wsum[2][cap + sl]) + wsum[3][cap + sl];
  }
}

int finalize_grid(int K) { return (K + 3) / 4; }

hipError_t launch_finalize(const FinalizeArgs& f, hipStream_t s) {
  if (f.cap > kMaxM) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_finalize, dim3(finalize_grid(f.K)), dim3(256), 0, s, f);
  return hipGetLastError();
}

}  // namespace km
