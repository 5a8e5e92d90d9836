// Update step (Sec. 1, Eq. (4)): c_j = mean of the samples labelled j.
//
// Two paths, both deterministic and free of floating-point atomics; which
// one runs depends only on (K, d).
//
// Fixed-point sums, when K * (d | 1) + K int64 accumulators fit in LDS
// (fx_ok), described at k_fxsum below:
//   k_xbound, k_xexp  once per X: bound of |x| and the scale exponent;
//   k_fxsum           one pass over X into per-workgroup int64 partials;
//   k_fxfinal         adds the partials and does the work of k_finalize.
//
// Counting sort otherwise:
//   1. k_rank     stable within-block ranks of every label (wave match by
//                 ballots, per-wave LDS counters) and each block's histogram,
//                 stored label-major: blockcount[j][b];
//   2. k_scan     one workgroup per label: exclusive prefix of its block
//                 counts (the offset of block b inside segment j) and the
//                 cluster size N_j;
//   3. k_offsets  segment starts and the list of work items, each item being
//                 at most kSegRows consecutive sorted samples of one cluster;
//   4. k_scatter  perm[start_j + offset_jb + rank] = i: a stable counting sort;
//   5. k_segsum   one workgroup per item gathers its rows and sums them in
//                 float64, reducing across row groups through LDS in a fixed
//                 order;
//   6. k_finalize one thread per centroid element: sums the items of its
//                 cluster in order and divides by N_j (an empty cluster keeps
//                 its centroid).  In the solver it also forms the residual
//                 F = G - C, pushes the newest differences of F and G into the
//                 history ring and emits per-workgroup partial inner products
//                 for the Anderson Gram matrix.

#include "km_launch.h"

namespace km {

__device__ __forceinline__ const int* labels_of(const UpdateArgs& u) {
  return u.lab_from_ctl ? u.lab + (int64_t)u.ctl->lab_prev * u.N : u.lab;
}

// ---------------------------------------------------------------------------
// 1. ranks within blocks of rank_rows(N, K) rows
// ---------------------------------------------------------------------------
template <int RR>
__device__ __forceinline__ void rank_rows_body(const UpdateArgs& u, int bx, int (&cnt)[4][kMaxK]) {
  const int* L = labels_of(u);
  const int K = u.K;
  const int nblk = (int)((u.N + RR - 1) / RR);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  constexpr int kChunks = RR / 256;   // 64-row chunks per wave
  const int64_t base = (int64_t)bx * RR + (int64_t)w * (kChunks * 64);
  int labs[kChunks], rk[kChunks];
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const int64_t i = base + c * 64 + lane;
    int lab = (i < u.N) ? L[i] : 0;
    labs[c] = (lab < 0 || lab >= K) ? 0 : lab;
  }
  for (int j = tid; j < 4 * K; j += 256) cnt[j / K][j % K] = 0;
  __syncthreads();

  int nbits = 0;
  while ((1 << nbits) < K) ++nbits;
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const int64_t i = base + c * 64 + lane;
    const bool valid = i < u.N;
    const int lab = labs[c];
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
    u.blockcount[(int64_t)j * nblk + bx] = s;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const int64_t i = base + c * 64 + lane;
    if (i < u.N) u.lrank[i] = rk[c] + cnt[w][labs[c]];
  }
}

__device__ __forceinline__ void rank_body(const UpdateArgs& u, int bx) {
  if (u.gated && u.ctl->done) return;
  __shared__ int cnt[4][kMaxK];
  if (rank_rows(u.N, u.K) == kRankRowsLarge) rank_rows_body<kRankRowsLarge>(u, bx, cnt);
  else rank_rows_body<kRankRowsSmall>(u, bx, cnt);
}

// ---------------------------------------------------------------------------
// Workgroup-wide exclusive scan of one int per thread (256 threads).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(v, off, kWave);
    if (lane >= off) v += o;
  }
  return v;
}

// ---------------------------------------------------------------------------
// 2. per-label prefix over blocks: one workgroup per label
// ---------------------------------------------------------------------------
__device__ __forceinline__ void scan_body(const UpdateArgs& u, int bx) {
  if (u.gated && u.ctl->done) return;
  __shared__ int wsum[4];
  __shared__ int carry;
  constexpr int V = 8;   // consecutive block counts per thread and pass
  const int j = bx;
  const int nblk = update_rank_blocks(u.N, u.K);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int* row = u.blockcount + (int64_t)j * nblk;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int b0 = 0; b0 < nblk; b0 += 256 * V) {
    const int bb = b0 + tid * V;
    int v[V], loc = 0;
#pragma unroll
    for (int q = 0; q < V; ++q) {
      v[q] = (bb + q < nblk) ? row[bb + q] : 0;
      loc += v[q];
    }
    const int inc = wave_incl_scan(loc, lane);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int before = carry;
    for (int q = 0; q < w; ++q) before += wsum[q];
    int run = before + inc - loc;   // exclusive prefix of this thread's first entry
#pragma unroll
    for (int q = 0; q < V; ++q) {
      if (bb + q < nblk) row[bb + q] = run;
      run += v[q];
    }
    __syncthreads();
    if (tid == 255) carry = before + inc;
    __syncthreads();
  }
  if (tid == 0) u.counts[j] = carry;
}

// ---------------------------------------------------------------------------
// 3. segment starts and work items (one workgroup of 1024 threads)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void offsets_body(const UpdateArgs& u) {
  if (u.gated && u.ctl->done) return;
  __shared__ int wc[16], wi[16];
  __shared__ int empty_sh;
  __shared__ int ist[kMaxK + 1];   // item starts, for the item list below
  const int K = u.K;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int per = (K + 1023) / 1024;
  const int j0 = tid * per;
  if (tid == 0) empty_sh = 0;
  int csum = 0, isum = 0, empty = 0;
  for (int j = j0; j < j0 + per && j < K; ++j) {
    const int c = u.counts[j];
    csum += c;
    isum += (c + kSegRows - 1) / kSegRows;
    empty += (c == 0);
  }
  const int ci = wave_incl_scan(csum, lane);
  const int ii = wave_incl_scan(isum, lane);
  if (lane == 63) { wc[w] = ci; wi[w] = ii; }
  __syncthreads();
  if (empty) atomicAdd(&empty_sh, empty);
  int cbase = ci - csum, ibase = ii - isum;
  for (int q = 0; q < w; ++q) { cbase += wc[q]; ibase += wi[q]; }
  for (int j = j0; j < j0 + per && j < K; ++j) {
    const int c = u.counts[j];
    const int ni = (c + kSegRows - 1) / kSegRows;
    u.seg_start[j] = cbase;
    u.item_start[j] = ibase;
    ist[j] = ibase;
    cbase += c;
    ibase += ni;
  }
  if (tid == 1023) ist[K] = ibase;
  __syncthreads();
  if (tid == 1023) {
    u.seg_start[K] = cbase;
    u.item_start[K] = ibase;
    u.ctl->total_items = ibase < u.max_items ? ibase : u.max_items;
    u.ctl->empty = empty_sh;
  }
  // item list: wave w writes the items of clusters w, w + 16, ... with
  // consecutive lanes on consecutive items (coalesced stores)
  for (int j = w; j < K; j += 16) {
    const int i1 = ist[j + 1] < u.max_items ? ist[j + 1] : u.max_items;
    for (int q = ist[j] + lane; q < i1; q += 64) u.item_cluster[q] = j;
  }
}

// ---------------------------------------------------------------------------
// 4. stable scatter
// ---------------------------------------------------------------------------
__device__ __forceinline__ void scatter_body(const UpdateArgs& u, int bx) {
  if (u.gated && u.ctl->done) return;
  const int* L = labels_of(u);
  const int64_t i = (int64_t)bx * 256 + threadIdx.x;
  if (i >= u.N) return;
  const int nblk = update_rank_blocks(u.N, u.K);
  int lab = L[i];
  if (lab < 0 || lab >= u.K) lab = 0;
  const int64_t b = i / rank_rows(u.N, u.K);
  const int64_t pos = (int64_t)u.seg_start[lab] + u.blockcount[(int64_t)lab * nblk + b] + u.lrank[i];
  if (pos >= 0 && pos < u.N) u.perm[pos] = (int)i;
}

// ---------------------------------------------------------------------------
// 5. segmented sums: one workgroup per work item
// ---------------------------------------------------------------------------
__device__ __forceinline__ void segsum_body(const UpdateArgs& u, int bx) {
  if (u.gated && u.ctl->done) return;
  const int item = bx;
  const bool XBF = u.xbf16 != 0;
  if (item >= u.ctl->total_items) return;
  __shared__ double red[256 * 4];
  const int d = u.d;
  const int j = u.item_cluster[item];
  const int c = item - u.item_start[j];
  const int64_t p0 = (int64_t)u.seg_start[j] + (int64_t)c * kSegRows;
  const int64_t pend = (int64_t)u.seg_start[j] + u.counts[j];
  const int64_t p1 = (p0 + kSegRows < pend) ? p0 + kSegRows : pend;

  // threads per row: power of two covering ceil(d/4) four-element columns
  int tpr = 1;
  while (tpr * 4 < d) tpr <<= 1;
  const int rpp = 256 / tpr;                 // rows per pass
  const int col = threadIdx.x % tpr, rg = threadIdx.x / tpr;
  const int k0 = col * 4;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const bool vec = (d % 4) == 0 && k0 + 4 <= d;
  // Rows p, p + rpp, ... of the item, four per step: the four row loads are
  // issued together and the permutation entries of the next step are fetched
  // meanwhile; the rows are still added in order.
  constexpr int kU = 4;
  auto row4 = [&](int64_t i, bool ok, double (&v)[4]) {
    v[0] = v[1] = v[2] = v[3] = 0.0;
    if (!ok) return;
    if (XBF) {   // uniform per workgroup
      const uint16_t* xr = (const uint16_t*)u.X + i * d;
      if (vec) {
        const uint2 t = *(const uint2*)(xr + k0);
        v[0] = (double)__uint_as_float(t.x << 16);
        v[1] = (double)__uint_as_float(t.x & 0xFFFF0000u);
        v[2] = (double)__uint_as_float(t.y << 16);
        v[3] = (double)__uint_as_float(t.y & 0xFFFF0000u);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (k0 + e < d) v[e] = (double)__uint_as_float(((uint32_t)xr[k0 + e]) << 16);
      }
    } else {
      const float* xr = (const float*)u.X + i * d;
      if (vec) {
        const float4 t = *(const float4*)(xr + k0);
        v[0] = (double)t.x;
        v[1] = (double)t.y;
        v[2] = (double)t.z;
        v[3] = (double)t.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (k0 + e < d) v[e] = (double)xr[k0 + e];
      }
    }
  };
  const int64_t pbase = p0 + rg;
  int nxt[kU];
#pragma unroll
  for (int q = 0; q < kU; ++q) {
    const int64_t pp = pbase + (int64_t)q * rpp;
    nxt[q] = pp < p1 ? u.perm[pp] : 0;
  }
  for (int64_t p = pbase; p < p1; p += (int64_t)kU * rpp) {
    int cur[kU];
#pragma unroll
    for (int q = 0; q < kU; ++q) cur[q] = nxt[q];
#pragma unroll
    for (int q = 0; q < kU; ++q) {
      const int64_t pp = p + (int64_t)(kU + q) * rpp;
      nxt[q] = pp < p1 ? u.perm[pp] : 0;
    }
    double v[kU][4];
#pragma unroll
    for (int q = 0; q < kU; ++q) row4(cur[q], p + (int64_t)q * rpp < p1, v[q]);
#pragma unroll
    for (int q = 0; q < kU; ++q) {
      if (p + (int64_t)q * rpp < p1) {
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] += v[q][e];
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

size_t update_blockcount_ints(int64_t N, int K) {
  // largest nblk(N', K') * K' over N' <= N, K' <= K: small blocks at the
  // largest N' below the row split and K' = min(K, split), or large blocks at
  // N and K
  const int ks = K < kRankSplitK ? K : kRankSplitK;
  const int64_t ns = N < kRankSplitN ? N : kRankSplitN - 1;
  const size_t a = (size_t)((ns + kRankRowsSmall - 1) / kRankRowsSmall) * ks;
  const size_t b = (size_t)((N + kRankRowsLarge - 1) / kRankRowsLarge) * K;
  return a > b ? a : b;
}
// ---------------------------------------------------------------------------
// Fixed-point sums (fx_ok(K, d)): X is read once, in row order
// ---------------------------------------------------------------------------
// Each workgroup of k_fxsum adds its share of the rows into int64
// accumulators in LDS (sums of the scaled, rounded coordinates, then the
// cluster sizes) and writes them as partials; the finalisation (k_fxfinal)
// adds the per-workgroup partials and converts the sums back.  Integer
// addition is associative, so the order of the LDS atomics does not change
// the result: runs are bitwise reproducible, and the sums do not depend on
// how the rows are split between workgroups.
//
// Scale: 2^e with n * max|x| * 2^e < 2^62, so no partial sum of at most n
// scaled values overflows, and max|x| * 2^e < 2^51 (below).  e is the largest
// such integer up to the powers of two that bound n and max|x|, so for
// n >= 2048, 2^-e <= n * max|x| * 2^-60.  Each coordinate is rounded to the
// nearest multiple of 2^-e; a cluster mean then differs from the exact mean
// of the float32 values by at most 2^-(e+1) <= n * max|x| * 2^-61 (about
// 4e-12 max|x| at n = 1e7; max|x| * 2^-51 for smaller n), far below float32
// rounding of the centroids.
//
// Rounding: with |v * 2^e| < 2^51, t = fma(v, 2^e, 1.5 * 2^52) lies in
// [2^52, 2^53), where float64 spacing is 1, so t is v * 2^e rounded to the
// nearest integer q, and the bit pattern of t is q + bits(1.5 * 2^52).  The
// accumulators add bit patterns (modulo 2^64); each workgroup subtracts
// (rows of cluster j) * bits(1.5 * 2^52) from the sums of cluster j when it
// writes its partials, which leaves the exact integer sums.

__device__ __forceinline__ unsigned wave_umax(unsigned v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, o, 64));
  return v;
}

// Per-workgroup maxima of |x| over X, as float32 bit patterns (non-negative
// floats order like their bits; NaN lies above infinity).  bfloat16 bits are
// the high half of the float32 pattern.
// largest |x| pattern of a 16-byte word: 4 float32, or 8 bfloat16 (16-bit result)
__device__ __forceinline__ unsigned xb_half(unsigned w) {
  w &= 0x7fff7fffu;
  return max(w >> 16, w & 0xffffu);
}
__device__ __forceinline__ unsigned xb_word(uint4 v, bool bf) {
  if (bf) return max(max(xb_half(v.x), xb_half(v.y)), max(xb_half(v.z), xb_half(v.w)));
  return max(max(v.x & 0x7fffffffu, v.y & 0x7fffffffu), max(v.z & 0x7fffffffu, v.w & 0x7fffffffu));
}

__device__ __forceinline__ void xbound_body(const UpdateArgs& u, int bx) {
  __shared__ unsigned wm[4];
  const int tid = threadIdx.x;
  const int64_t n = u.N * u.d;
  const int64_t stride = (int64_t)kXBoundSlots * 256;
  const uint4* x4 = (const uint4*)u.X;     // X starts on a 16-byte boundary
  const bool bf = u.xbf16 != 0;
  const int es = bf ? 8 : 4;               // elements per 16-byte word
  const int64_t nw = n / es;
  unsigned m = 0;
  int64_t q = (int64_t)bx * 256 + tid;
  for (; q + 3 * stride < nw; q += 4 * stride) {   // four loads in flight
    const uint4 a = x4[q], b = x4[q + stride], c = x4[q + 2 * stride], e = x4[q + 3 * stride];
    m = max(m, max(max(xb_word(a, bf), xb_word(b, bf)), max(xb_word(c, bf), xb_word(e, bf))));
  }
  for (; q < nw; q += stride) m = max(m, xb_word(x4[q], bf));
  if (bf) {
    const uint16_t* x = (const uint16_t*)u.X;
    for (int64_t i = nw * es + (int64_t)bx * 256 + tid; i < n; i += stride) m = max(m, (unsigned)(x[i] & 0x7fffu));
    m <<= 16;
  } else {
    const unsigned* x = (const unsigned*)u.X;
    for (int64_t i = nw * es + (int64_t)bx * 256 + tid; i < n; i += stride) m = max(m, x[i] & 0x7fffffffu);
  }
  m = wave_umax(m);
  if ((tid & 63) == 0) wm[tid >> 6] = m;
  __syncthreads();
  if (tid == 0) u.xbound[bx] = max(max(wm[0], wm[1]), max(wm[2], wm[3]));
}

// e for the bound pattern `bits` and n rows; 0 for all-zero or non-finite X
// (non-finite data makes the energy non-finite, which the caller reports).
__device__ __forceinline__ int fx_exponent(unsigned bits, int64_t n) {
  if (bits == 0u || bits >= 0x7f800000u) return 0;
  const int E = (int)(bits >> 23);
  const int eb = E == 0 ? -126 : E - 126;                 // max|x| < 2^eb
  const int ln = 64 - __clzll((unsigned long long)n);     // n < 2^ln
  const int e = 62 - eb - ln;
  return e < 51 - eb ? e : 51 - eb;
}

constexpr double kFxMagic = 0x1.8p52;                      // 1.5 * 2^52
constexpr unsigned long long kFxMagicBits = 0x4338000000000000ull;

// One workgroup of kFxThreads: the bound over all slots, then e into slot
// kXBoundSlots (once per X, so the sums read one word instead of reducing
// the slots behind a barrier).
__device__ __forceinline__ void xexp_body(const UpdateArgs& u) {
  __shared__ unsigned sh[kFxThreads / 64];
  const int tid = threadIdx.x;
  unsigned m = tid < kXBoundSlots ? u.xbound[tid] : 0u;
  m = wave_umax(m);
  if ((tid & 63) == 0) sh[tid >> 6] = m;
  __syncthreads();
  if (tid == 0) {
    unsigned b = 0;
    for (int w = 0; w < kFxThreads / 64; ++w) b = max(b, sh[w]);
    u.xbound[kXBoundSlots] = (unsigned)fx_exponent(b, u.N);
  }
}

__device__ __forceinline__ int fx_exp_of(const UpdateArgs& u) { return (int)u.xbound[kXBoundSlots]; }

// round(v * s) + bits(1.5 * 2^52), |v * s| < 2^51 (see above)
__device__ __forceinline__ unsigned long long fx_quant(float v, double s) {
  return (unsigned long long)__double_as_longlong(fma((double)v, s, kFxMagic));
}

__device__ __forceinline__ int fx_label(const int* lab, int64_t r, int K) {
  const int j = lab[r];
  return (j < 0 || j >= K) ? 0 : j;
}

__device__ __forceinline__ float4 fx_load4(const UpdateArgs& u, int64_t i) {
  if (u.xbf16) {
    const uint2 v = *(const uint2*)((const uint16_t*)u.X + i);
    return make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xffff0000u),
                       __uint_as_float(v.y << 16), __uint_as_float(v.y & 0xffff0000u));
  }
  return *(const float4*)((const float*)u.X + i);
}

__device__ __forceinline__ float fx_load1(const UpdateArgs& u, int64_t i) {
  return u.xbf16 ? __uint_as_float((unsigned)((const uint16_t*)u.X)[i] << 16) : ((const float*)u.X)[i];
}

// Workgroup bx of P.  The workgroups sweep X together: step t of workgroup
// bx takes the T coordinate groups starting at group (t * P + bx) * T.  Any
// split of the rows gives the same integer sums.  The lane that holds
// coordinate group 0 of a row also adds the row to its cluster's size, so the
// labels are read once.
__device__ __forceinline__ void fxsum_body(const UpdateArgs& u, int bx, int P, unsigned long long* acc) {
  if (u.gated && u.ctl->done) return;
  constexpr int T = kFxThreads;
  const int tid = threadIdx.x;
  const int d = u.d, K = u.K, KD = K * d, L = KD + K;
  const int S = fx_stride(d), KS = K * S;   // LDS: sums of cluster j at j*S, sizes at KS
  const int* lab = labels_of(u);
  for (int i = tid; i < KS + K; i += T) acc[i] = 0ull;
  if (bx == 0 && tid == 0) u.ctl->empty = 0;     // the reduction adds the empty clusters
  const double s = ldexp(1.0, fx_exp_of(u));
  __syncthreads();                                // accumulators cleared
  // consecutive threads take consecutive groups of g coordinates; (row, col)
  // of a thread's group advances by P * T groups per step
  const int g = (d & 3) == 0 ? 4 : 1;
  const int qd = d / g;
  const int64_t ng = u.N * qd;
  const int64_t stride = (int64_t)P * T;
  const int64_t g0 = (int64_t)bx * T + tid;
  const int64_t drow = stride / qd;
  const int dcol = (int)(stride % qd);
  int64_t row = g0 / qd;
  int col = (int)(g0 % qd);
  int64_t q = g0;
  if (g == 4) {
    for (; q + stride < ng; q += 2 * stride) {
      int64_t rowb = row + drow;
      int colb = col + dcol;
      if (colb >= qd) { colb -= qd; ++rowb; }
      const float4 va = fx_load4(u, row * d + 4 * col), vb = fx_load4(u, rowb * d + 4 * colb);
      const int ja = fx_label(lab, row, K), jb = fx_label(lab, rowb, K);
      unsigned long long* a = acc + ja * S + 4 * col;
      atomicAdd(a + 0, fx_quant(va.x, s)); atomicAdd(a + 1, fx_quant(va.y, s));
      atomicAdd(a + 2, fx_quant(va.z, s)); atomicAdd(a + 3, fx_quant(va.w, s));
      if (col == 0) atomicAdd(acc + KS + ja, 1ull);
      unsigned long long* b = acc + jb * S + 4 * colb;
      atomicAdd(b + 0, fx_quant(vb.x, s)); atomicAdd(b + 1, fx_quant(vb.y, s));
      atomicAdd(b + 2, fx_quant(vb.z, s)); atomicAdd(b + 3, fx_quant(vb.w, s));
      if (colb == 0) atomicAdd(acc + KS + jb, 1ull);
      row = rowb + drow;
      col = colb + dcol;
      if (col >= qd) { col -= qd; ++row; }
    }
    if (q < ng) {
      const float4 va = fx_load4(u, row * d + 4 * col);
      const int ja = fx_label(lab, row, K);
      unsigned long long* a = acc + ja * S + 4 * col;
      atomicAdd(a + 0, fx_quant(va.x, s)); atomicAdd(a + 1, fx_quant(va.y, s));
      atomicAdd(a + 2, fx_quant(va.z, s)); atomicAdd(a + 3, fx_quant(va.w, s));
      if (col == 0) atomicAdd(acc + KS + ja, 1ull);
    }
  } else {
    for (; q < ng; q += stride) {
      const int j = fx_label(lab, row, K);
      atomicAdd(acc + j * S + col, fx_quant(fx_load1(u, row * d + col), s));
      if (col == 0) atomicAdd(acc + KS + j, 1ull);   // the row's size, once per row
      row += drow;
      col += dcol;
      if (col >= qd) { col -= qd; ++row; }
    }
  }
  __syncthreads();
  // partials dense: sums (K x d) then sizes (K)
  unsigned long long* part = u.fxpart + (int64_t)bx * L;
  for (int i = tid; i < L; i += T) {
    if (i < KD) {
      const int j = (int)((unsigned)i / (unsigned)d), k = i - j * d;
      part[i] = acc[j * S + k] - acc[KS + j] * kFxMagicBits;
    } else {
      part[i] = acc[KS + i - KD];
    }
  }
}

int update_max_items(int64_t N, int K) { return (int)((N + kSegRows - 1) / kSegRows) + K; }

__global__ __launch_bounds__(256) void k_rank(UpdateArgs u) { rank_body(u, blockIdx.x); }
__global__ __launch_bounds__(256) void k_scan(UpdateArgs u) { scan_body(u, blockIdx.x); }
__global__ __launch_bounds__(1024) void k_offsets(UpdateArgs u) { offsets_body(u); }
__global__ __launch_bounds__(256) void k_scatter(UpdateArgs u) { scatter_body(u, blockIdx.x); }
__global__ __launch_bounds__(256) void k_segsum(UpdateArgs u) { segsum_body(u, blockIdx.x); }

__global__ __launch_bounds__(256) void k_rank_batch(BatchRef<UpdateArgs> t) {
  const int b = batch_find(t.prefix, t.n, blockIdx.x);
  rank_body(t.tab[b], blockIdx.x - t.prefix[b]);
}
__global__ __launch_bounds__(256) void k_scan_batch(BatchRef<UpdateArgs> t) {
  const int b = batch_find(t.prefix, t.n, blockIdx.x);
  scan_body(t.tab[b], blockIdx.x - t.prefix[b]);
}
__global__ __launch_bounds__(1024) void k_offsets_batch(BatchRef<UpdateArgs> t) {
  const UpdateArgs& u = t.tab[blockIdx.x];   // one workgroup per instance
  if (!u.fx) offsets_body(u);
}
__global__ __launch_bounds__(256) void k_scatter_batch(BatchRef<UpdateArgs> t) {
  const int b = batch_find(t.prefix, t.n, blockIdx.x);
  scatter_body(t.tab[b], blockIdx.x - t.prefix[b]);
}
__global__ __launch_bounds__(256) void k_segsum_batch(BatchRef<UpdateArgs> t) {
  const int b = batch_find(t.prefix, t.n, blockIdx.x);
  segsum_body(t.tab[b], blockIdx.x - t.prefix[b]);
}

__global__ __launch_bounds__(256) void k_xbound(UpdateArgs u) { xbound_body(u, blockIdx.x); }
__global__ __launch_bounds__(kFxThreads) void k_fxsum(UpdateArgs u) {
  extern __shared__ unsigned long long fx_acc[];
  fxsum_body(u, blockIdx.x, gridDim.x, fx_acc);
}
__global__ __launch_bounds__(kFxThreads) void k_xexp(UpdateArgs u) { xexp_body(u); }
__global__ __launch_bounds__(kFxThreads) void k_xexp_batch(BatchRef<UpdateArgs> t) {
  const UpdateArgs& u = t.tab[blockIdx.x];   // one workgroup per instance
  if (u.fx) xexp_body(u);
}

__global__ __launch_bounds__(256) void k_xbound_batch(BatchRef<UpdateArgs> t) {
  const int b = batch_find(t.prefix, t.n, blockIdx.x);
  xbound_body(t.tab[b], blockIdx.x - t.prefix[b]);
}
__global__ __launch_bounds__(kFxThreads) void k_fxsum_batch(BatchRef<UpdateArgs> t) {
  extern __shared__ unsigned long long fx_acc[];
  const int b = batch_find(t.prefix, t.n, blockIdx.x);
  fxsum_body(t.tab[b], blockIdx.x - t.prefix[b], t.prefix[b + 1] - t.prefix[b], fx_acc);
}

// Dynamic LDS of the fixed-point sums: kFxMaxL accumulators (above the
// default 64 KB limit, so the attribute is raised once per process).
constexpr size_t kFxLds = (size_t)kFxMaxL * 8;
static hipError_t fx_lds_attr() {
  static hipError_t st = [] {
    hipError_t a = hipFuncSetAttribute((const void*)k_fxsum, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFxLds);
    hipError_t b = hipFuncSetAttribute((const void*)k_fxsum_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kFxLds);
    return a != hipSuccess ? a : b;
  }();
  return st;
}

hipError_t launch_xbound(const UpdateArgs& u, hipStream_t s) {
  if (!u.fx) return hipSuccess;
  clear_pending_error();
  hipLaunchKernelGGL(k_xbound, dim3(kXBoundSlots), dim3(256), 0, s, u);
  hipLaunchKernelGGL(k_xexp, dim3(1), dim3(kFxThreads), 0, s, u);
  return hipGetLastError();
}

hipError_t launch_xbound_batch(const UpdateBatch& ub, hipStream_t s) {
  clear_pending_error();
  if (ub.n <= 0 || ub.blocks[6] <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_xbound_batch, dim3(ub.blocks[6]), dim3(256), 0, s, BatchRef<UpdateArgs>{ub.tab, ub.prefix[6], ub.n});
  hipLaunchKernelGGL(k_xexp_batch, dim3(ub.n), dim3(kFxThreads), 0, s, BatchRef<UpdateArgs>{ub.tab, nullptr, ub.n});
  return hipGetLastError();
}

hipError_t launch_update_sums(const UpdateArgs& u, hipStream_t s, hipEvent_t ev0) {
  if (u.K > kMaxK || u.d > kMaxD) return hipErrorInvalidValue;
  if (u.fx) {
    if (!fx_ok(u.K, u.d)) return hipErrorInvalidValue;
    const hipError_t a = fx_lds_attr();
    if (a != hipSuccess) return a;
    clear_pending_error();
    if (ev0)
      hipExtLaunchKernelGGL(k_fxsum, dim3(fx_blocks(u.N)), dim3(kFxThreads), kFxLds, s, ev0, nullptr, 0, u);
    else
      hipLaunchKernelGGL(k_fxsum, dim3(fx_blocks(u.N)), dim3(kFxThreads), kFxLds, s, u);
    return hipGetLastError();   // the finalisation adds the partials
  }
  const int nblk = update_rank_blocks(u.N, u.K);
  clear_pending_error();
  if (ev0)
    hipExtLaunchKernelGGL(k_rank, dim3(nblk), dim3(256), 0, s, ev0, nullptr, 0, u);
  else
    hipLaunchKernelGGL(k_rank, dim3(nblk), dim3(256), 0, s, u);
  hipLaunchKernelGGL(k_scan, dim3(u.K), dim3(256), 0, s, u);
  hipLaunchKernelGGL(k_offsets, dim3(1), dim3(1024), 0, s, u);
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)((u.N + 255) / 256)), dim3(256), 0, s, u);
  hipLaunchKernelGGL(k_segsum, dim3(u.max_items), dim3(256), 0, s, u);
  return hipGetLastError();
}

// Instances on the counting sort get workgroups in kernels 0-3 (and the
// offsets kernel, one workgroup per instance, returns at once for the others);
// fixed-point instances in kernel 4 (their partials are added by the
// finalisation).
hipError_t launch_update_sums_batch(const UpdateBatch& ub, hipStream_t s) {
  clear_pending_error();
  if (ub.n <= 0) return hipSuccess;
  if (ub.blocks[0] > 0) {
    hipLaunchKernelGGL(k_rank_batch, dim3(ub.blocks[0]), dim3(256), 0, s, BatchRef<UpdateArgs>{ub.tab, ub.prefix[0], ub.n});
    hipLaunchKernelGGL(k_scan_batch, dim3(ub.blocks[1]), dim3(256), 0, s, BatchRef<UpdateArgs>{ub.tab, ub.prefix[1], ub.n});
    hipLaunchKernelGGL(k_offsets_batch, dim3(ub.n), dim3(1024), 0, s, BatchRef<UpdateArgs>{ub.tab, nullptr, ub.n});
    hipLaunchKernelGGL(k_scatter_batch, dim3(ub.blocks[2]), dim3(256), 0, s, BatchRef<UpdateArgs>{ub.tab, ub.prefix[2], ub.n});
    hipLaunchKernelGGL(k_segsum_batch, dim3(ub.blocks[3]), dim3(256), 0, s, BatchRef<UpdateArgs>{ub.tab, ub.prefix[3], ub.n});
  }
  if (ub.blocks[4] > 0) {
    const hipError_t a = fx_lds_attr();
    if (a != hipSuccess) return a;
    hipLaunchKernelGGL(k_fxsum_batch, dim3(ub.blocks[4]), dim3(kFxThreads), kFxLds, s,
                       BatchRef<UpdateArgs>{ub.tab, ub.prefix[4], ub.n});
  }
  return hipGetLastError();
}

int update_grid(const UpdateArgs& u, int which) {
  if (which <= 3 && u.fx) return 0;
  if (which >= 4 && !u.fx) return 0;
  switch (which) {
    case 0: return update_rank_blocks(u.N, u.K);
    case 1: return u.K;
    case 2: return (int)((u.N + 255) / 256);
    case 3: return u.max_items;
    case 4: return fx_blocks(u.N);
    case 6: return kXBoundSlots;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// 6. means, residual, history push and Gram partials (one thread per element)
// ---------------------------------------------------------------------------
constexpr int kDotGroup = 12;   // history slots reduced per pass over the elements (m_max <= 12 in one pass)

__device__ __forceinline__ void finalize_body(const FinalizeArgs& f, int bx, int gx) {
  Ctl* ctl = f.ctl;
  if (f.mode == kFinIter && ctl->done) return;
  __shared__ double red[2 * kDotGroup][4];
  const int tid = threadIdx.x;
  const int d = f.d, cap = f.cap;
  const int64_t KD = (int64_t)f.K * d;
  const int64_t stride = (int64_t)gx * 256;

  int s_new = 0, len_new = 0;
  if (f.mode == kFinIter && cap > 0) {
    // the difference created at iteration t goes to ring slot (t - 1) mod cap
    const int t = ctl->t;
    s_new = (t - 1) % cap;
    len_new = t < cap ? t : cap;
  }
  const float* Cacc = (f.mode == kFinIter && ctl->acc_src == 1) ? f.C_fb : f.C_cand;

  for (int64_t e = (int64_t)bx * 256 + tid; e < KD; e += stride) {
    const int j = (int)((uint32_t)e / (uint32_t)d);   // K*d < 2^31
    const int n = f.counts[j];
    const int i0 = f.item_start[j], i1 = f.item_start[j + 1];
    const int k = (int)(e - (int64_t)j * d);
    // item partials in order, eight loads in flight
    double sum = 0.0;
    int it = i0;
    for (; it + 8 <= i1; it += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = f.partial[(int64_t)(it + q) * d + k];
#pragma unroll
      for (int q = 0; q < 8; ++q) sum += v[q];
    }
    for (; it < i1; ++it) sum += f.partial[(int64_t)it * d + k];
    if (f.mode == kFinG) {
      f.C_out[e] = (float)(n > 0 ? sum / (double)n : (double)f.C_in[e]);
      continue;
    }
    const double cin = (f.mode == kFinInit) ? (double)f.C_in[e] : (double)Cacc[e];
    if (f.C_ref) f.C_ref[e] = (float)cin;   // exact: cin is a float32 value
    const double gv = n > 0 ? sum / (double)n : cin;
    const double fv = gv - cin;
    if (f.mode == kFinIter && cap > 0) {
      f.ring_dF[(int64_t)s_new * KD + e] = fv - f.F_last[e];
      f.ring_dG[(int64_t)s_new * KD + e] = gv - f.G_last[e];
    }
    f.G_last[e] = gv;
    f.F_last[e] = fv;
  }
  if (f.mode != kFinIter || cap == 0) return;

  // Gram partials: for each valid slot sl, <dF_new, dF_sl> (index sl) and
  // <dF_sl, F^t> (index cap + sl).  Each thread reads back only the elements
  // it wrote above.  Reduction: waves by shuffles, then the 4 wave partials
  // in order.
  const int lane = tid & 63, w = tid >> 6;
  for (int q0 = 0; q0 < len_new; q0 += kDotGroup) {
    double pa[kDotGroup], pb[kDotGroup];
#pragma unroll
    for (int g = 0; g < kDotGroup; ++g) { pa[g] = 0.0; pb[g] = 0.0; }
    for (int64_t e = (int64_t)bx * 256 + tid; e < KD; e += stride) {
      const double dfn = f.ring_dF[(int64_t)s_new * KD + e];
      const double fv = f.F_last[e];
#pragma unroll
      for (int g = 0; g < kDotGroup; ++g) {
        if (q0 + g < len_new) {
          const int sl = (s_new - (q0 + g) + cap) % cap;
          const double dfs = f.ring_dF[(int64_t)sl * KD + e];
          pa[g] = fma(dfn, dfs, pa[g]);
          pb[g] = fma(dfs, fv, pb[g]);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < kDotGroup; ++g) {
      pa[g] = wave_sum(pa[g]);
      pb[g] = wave_sum(pb[g]);
    }
    if (lane == 0) {
#pragma unroll
      for (int g = 0; g < kDotGroup; ++g) {
        red[g][w] = pa[g];
        red[kDotGroup + g][w] = pb[g];
      }
    }
    __syncthreads();
    if (tid < kDotGroup && q0 + tid < len_new) {
      const int sl = (s_new - (q0 + tid) + cap) % cap;
      f.dots[(int64_t)bx * 2 * cap + sl] = ((red[tid][0] + red[tid][1]) + red[tid][2]) + red[tid][3];
      f.dots[(int64_t)bx * 2 * cap + cap + sl] =
          ((red[kDotGroup + tid][0] + red[kDotGroup + tid][1]) + red[kDotGroup + tid][2]) + red[kDotGroup + tid][3];
    }
    __syncthreads();
  }
}

// Fixed-point path: the addition of the k_fxsum partials fused with the
// finalisation.  Workgroup bx (kFxThreads threads) owns the centroid elements
// e0 = 64 bx ... e0 + 63 and the sizes of the clusters they span.  Its 16
// waves add the partials (wave w takes partials w, w + 16, ...; then the 16
// wave sums in order; integer sums, so any order gives the same bits); wave 0
// then does the work of finalize_body for its 64 elements and writes one row
// of Gram partials (the combine adds finalize_grid_for rows).
__device__ __forceinline__ void fxfinal_body(const FinalizeArgs& f, int bx) {
  Ctl* ctl = f.ctl;
  if (f.mode == kFinIter && ctl->done) return;
  constexpr int NW = kFxThreads / 64;
  __shared__ unsigned long long rs[NW][64], rc[NW][64];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int d = f.d, K = f.K, cap = f.cap;
  const int KD = K * d, L = KD + K;
  const int P = fx_blocks(f.N);
  const int e0 = bx * 64, e = e0 + lane;
  const int j0 = e0 / d;                                   // first cluster spanned
  const int jlast = min((e0 + 63) / d, K - 1);
  const int jl = j0 + lane;                                // size column of this lane
  const bool has_e = e < KD, has_c = jl <= jlast;
  // wave 0 issues its element loads before the reduction (they do not depend on it)
  int s_new = 0, len_new = 0;
  double cin = 0.0, flast = 0.0, glast = 0.0;
  if (w == 0 && has_e) {
    if (f.mode == kFinIter) {
      const float* Cacc = ctl->acc_src == 1 ? f.C_fb : f.C_cand;
      cin = (double)Cacc[e];
      if (cap > 0) {
        flast = f.F_last[e];
        glast = f.G_last[e];
      }
    } else {
      cin = (double)f.C_in[e];
    }
  }
  unsigned long long ts = 0, tc = 0;
  {
    const unsigned long long* ps = f.fxpart + (has_e ? e : 0);
    const unsigned long long* pc = f.fxpart + KD + (has_c ? jl : 0);
    for (int p = w; p < P; p += 8 * NW) {                  // up to sixteen loads in flight
      unsigned long long a[8], c[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool in = p + u * NW < P;
        a[u] = (has_e && in) ? ps[(int64_t)(p + u * NW) * L] : 0ull;
        c[u] = (has_c && in) ? pc[(int64_t)(p + u * NW) * L] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        ts += a[u];
        tc += c[u];
      }
    }
  }
  rs[w][lane] = ts;
  rc[w][lane] = tc;
  __syncthreads();
  if (w != 0) return;
  ts = 0;
  tc = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    ts += rs[i][lane];
    tc += rc[i][lane];
  }
  // lane l holds the size of cluster j0 + l; this workgroup owns (counts as
  // empty) the clusters whose first element it holds
  const bool owned = has_c && jl * d >= e0;
  const unsigned long long em = __ballot(owned && tc == 0);
  if (lane == 0 && em) atomicAdd(&ctl->empty, (int)__popcll(em));
  const int je = has_e ? e / d : j0;
  const int n = __shfl((int)tc, je - j0, 64);
  const double sum = (double)(long long)ts * ldexp(1.0, -(int)f.xbound[kXBoundSlots]);

  if (f.mode == kFinIter && cap > 0) {
    // the difference created at iteration t goes to ring slot (t - 1) mod cap
    const int t = ctl->t;
    s_new = (t - 1) % cap;
    len_new = t < cap ? t : cap;
  }
  double dfn = 0.0, fv = 0.0;
  if (has_e) {
    if (f.mode == kFinG) {
      f.C_out[e] = (float)(n > 0 ? sum / (double)n : cin);
      return;
    }
    if (f.C_ref) f.C_ref[e] = (float)cin;   // exact: cin is a float32 value
    const double gv = n > 0 ? sum / (double)n : cin;
    fv = gv - cin;
    if (f.mode == kFinIter && cap > 0) {
      dfn = fv - flast;
      f.ring_dF[(int64_t)s_new * KD + e] = dfn;
      f.ring_dG[(int64_t)s_new * KD + e] = gv - glast;
    }
    f.G_last[e] = gv;
    f.F_last[e] = fv;
  }
  if (f.mode != kFinIter || cap == 0) return;
  // Gram partials of this workgroup's elements: <dF_new, dF_sl> (index sl)
  // and <dF_sl, F^t> (index cap + sl)
  for (int q0 = 0; q0 < len_new; q0 += kDotGroup) {
    double pa[kDotGroup], pb[kDotGroup];
#pragma unroll
    for (int g = 0; g < kDotGroup; ++g) {
      pa[g] = 0.0;
      pb[g] = 0.0;
      if (has_e && q0 + g < len_new) {
        const int sl = (s_new - (q0 + g) + cap) % cap;
        const double dfs = (q0 + g == 0) ? dfn : f.ring_dF[(int64_t)sl * KD + e];
        pa[g] = dfn * dfs;
        pb[g] = dfs * fv;
      }
    }
#pragma unroll
    for (int g = 0; g < kDotGroup; ++g) {
      pa[g] = wave_sum(pa[g]);
      pb[g] = wave_sum(pb[g]);
    }
    if (lane < kDotGroup && q0 + lane < len_new) {
      const int sl = (s_new - (q0 + lane) + cap) % cap;
      double va = 0.0, vb = 0.0;
#pragma unroll
      for (int g = 0; g < kDotGroup; ++g)
        if (g == lane) { va = pa[g]; vb = pb[g]; }
      f.dots[(int64_t)bx * 2 * cap + sl] = va;
      f.dots[(int64_t)bx * 2 * cap + cap + sl] = vb;
    }
  }
}

int finalize_grid(int64_t KD) {
  const int64_t g = (KD + 255) / 256;
  return (int)(g < 128 ? (g > 0 ? g : 1) : 128);
}
int finalize_grid_for(int fx, int K, int d) {
  const int64_t KD = (int64_t)K * d;
  return fx ? (int)((KD + 63) / 64) : finalize_grid(KD);
}
int finalize_grid_cap(int64_t KD) {
  const int64_t fx = ((KD < kFxMaxL ? KD : kFxMaxL) + 63) / 64;
  const int64_t g = finalize_grid(KD);
  return (int)(g > fx ? g : fx);
}

__global__ __launch_bounds__(256) void k_finalize(FinalizeArgs f) { finalize_body(f, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(kFxThreads) void k_fxfinal(FinalizeArgs f) { fxfinal_body(f, blockIdx.x); }

__global__ __launch_bounds__(256) void k_finalize_batch(BatchRef<FinalizeArgs> t) {
  const int b = batch_find(t.prefix, t.n, blockIdx.x);
  const int b0 = t.prefix[b];
  finalize_body(t.tab[b], blockIdx.x - b0, t.prefix[b + 1] - b0);
}
__global__ __launch_bounds__(kFxThreads) void k_fxfinal_batch(BatchRef<FinalizeArgs> t) {
  const int b = batch_find(t.prefix, t.n, blockIdx.x);
  fxfinal_body(t.tab[b], blockIdx.x - t.prefix[b]);
}

hipError_t launch_finalize_batch(const FinalizeArgs* tab, const int* prefix, int blocks, const int* fxprefix,
                                 int fxblocks, int n, hipStream_t s) {
  clear_pending_error();
  if (n <= 0) return hipSuccess;
  if (blocks > 0)
    hipLaunchKernelGGL(k_finalize_batch, dim3(blocks), dim3(256), 0, s, BatchRef<FinalizeArgs>{tab, prefix, n});
  if (fxblocks > 0)
    hipLaunchKernelGGL(k_fxfinal_batch, dim3(fxblocks), dim3(kFxThreads), 0, s,
                       BatchRef<FinalizeArgs>{tab, fxprefix, n});
  return hipGetLastError();
}

hipError_t launch_finalize(const FinalizeArgs& f, hipStream_t s, hipEvent_t ev1) {
  if (f.cap > kMaxM) return hipErrorInvalidValue;
  clear_pending_error();
  const dim3 grid(f.fx ? finalize_grid_for(1, f.K, f.d) : finalize_grid((int64_t)f.K * f.d));
  const dim3 block(f.fx ? kFxThreads : 256);
  if (ev1) {
    if (f.fx) hipExtLaunchKernelGGL(k_fxfinal, grid, block, 0, s, nullptr, ev1, 0, f);
    else hipExtLaunchKernelGGL(k_finalize, grid, block, 0, s, nullptr, ev1, 0, f);
  } else {
    if (f.fx) hipLaunchKernelGGL(k_fxfinal, grid, block, 0, s, f);
    else hipLaunchKernelGGL(k_finalize, grid, block, 0, s, f);
  }
  return hipGetLastError();
}

}  // namespace km
