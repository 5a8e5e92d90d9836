// Assignment step (Sec. 1, Eq. (3)) fused with the energy of Eq. (1).
//
// The squared distance ||x - c_j||^2 = ||x||^2 - 2 (x.c_j - ||c_j||^2 / 2), so
// the argmin over j is the argmax of s_j = x.c_j - ||c_j||^2 / 2.  The s_j
// of a 16-centroid x 16-sample tile come out of MFMA (v_mfma_f32_16x16x4f32)
// with the accumulator pre-loaded with -||c_j||^2 / 2; the running best and
// second-best s_j of each sample stay in registers across the whole K loop.
//
// Operand layout of the 16x16x4 MFMA: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; it receives D[4*(l/16)+r][l%16], r = 0..3.  A is a tile of
// 16 centroids, B a tile of 16 samples, so each lane accumulates 4 centroids
// of one sample.  The reduction index k is permuted so that lane group
// g = l/16 owns the contiguous dimensions [g*KS, g*KS+KS): sample rows are
// read with wide contiguous loads and kept in registers for the whole K loop.
//
// Exactness.  With u = 2^-24 and dp the padded dimension, every computed s_j
// is within gamma/2 * (||x|| + max_j ||c_j||)^2 of its exact value, gamma =
// (dp + 3) u / (1 - (dp + 3) u).  A sample whose best and second-best s_j
// differ by at most twice that bound (with a further factor 2 of margin) is
// re-checked: all K distances are recomputed as float64 sums of squared
// float64 differences, ties to the lowest index.  Every other sample's label
// is provably the exact argmin.  The energy term of every sample is the
// float64 direct-difference distance to its label.
//
// bfloat16 GEMM.  Centroids are rounded to bfloat16 (Cb); then s_j carries an
// extra error of at most ||x|| * delta_j with delta_j = ||c_j - Cb_j||, which
// is added to the bound.  X stored as bfloat16 is exact in both modes.

#include "km_launch.h"

namespace km {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short i16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __uint_as_float(((uint32_t)b) << 16);
}

__device__ __forceinline__ float ld_x(const void* X, int64_t idx, bool bf) {
  return bf ? bf16_to_f32(((const uint16_t*)X)[idx]) : ((const float*)X)[idx];
}

// Load dims [k0, k0 + KS) of row i as float32 (zero beyond d).
template <int KS, bool XBF>
__device__ __forceinline__ void load_chunk(const void* X, int64_t i, int d, int k0, bool vec,
                                           float (&out)[KS]) {
  if constexpr (KS % 4 == 0) {
    if (vec) {
      if constexpr (XBF) {
        const uint2* p = (const uint2*)((const uint16_t*)X + i * d + k0);
#pragma unroll
        for (int q = 0; q < KS / 4; ++q) {
          uint2 v = p[q];
          out[4 * q + 0] = __uint_as_float(v.x << 16);
          out[4 * q + 1] = __uint_as_float(v.x & 0xFFFF0000u);
          out[4 * q + 2] = __uint_as_float(v.y << 16);
          out[4 * q + 3] = __uint_as_float(v.y & 0xFFFF0000u);
        }
      } else {
        const float4* p = (const float4*)((const float*)X + i * d + k0);
#pragma unroll
        for (int q = 0; q < KS / 4; ++q) {
          float4 v = p[q];
          out[4 * q + 0] = v.x;
          out[4 * q + 1] = v.y;
          out[4 * q + 2] = v.z;
          out[4 * q + 3] = v.w;
        }
      }
      return;
    }
  }
#pragma unroll
  for (int q = 0; q < KS; ++q) {
    const int k = k0 + q;
    out[q] = (k < d) ? ld_x(X, i * d + k, XBF) : 0.f;
  }
}

// Exact re-check of one flagged sample by the whole wave: float64 direct
// differences to all K centroids, lowest index on ties.  Returns the label
// (or -1 if every distance is NaN) and its distance in *dist.
template <bool XBF>
__device__ __forceinline__ int exact_argmin(const void* X, int64_t i, int d, const float* C, int K,
                                            int lane, double* dist) {
  double bd = __builtin_inf();
  int bj = -1;
  for (int j = lane; j < K; j += kWave) {
    const float* cr = C + (int64_t)j * d;
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
      const double df = (double)ld_x(X, i * d + k, XBF) - (double)cr[k];
      s = fma(df, df, s);
    }
    if (s < bd) { bd = s; bj = j; }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ob = __shfl_xor(bd, off, kWave);
    const int oj = __shfl_xor(bj, off, kWave);
    const bool take = (ob < bd) || (ob == bd && (unsigned)oj < (unsigned)bj);
    bd = take ? ob : bd;
    bj = take ? oj : bj;
  }
  *dist = bd;
  return bj;
}

// One 16x16 tile: s = nc4 + C_tile . x_tile over the padded dimension.
template <int KS, bool GBF>
__device__ __forceinline__ f32x4 tile_dot(const float (&av)[KS], const float (&xv)[KS],
                                          const i16x8 (&ab)[KS / 8 > 0 ? KS / 8 : 1],
                                          const i16x8 (&xbv)[KS / 8 > 0 ? KS / 8 : 1], f32x4 acc) {
  if constexpr (GBF) {
#pragma unroll
    for (int q = 0; q < KS / 8; ++q)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, ab[q]),
                                                    __builtin_bit_cast(bf16x8, xbv[q]), acc, 0, 0, 0);
  } else {
#pragma unroll
    for (int q = 0; q < KS; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[q], xv[q], acc, 0, 0, 0);
  }
  return acc;
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// KS: padded dims per lane group (dp = 4*KS for f32 MFMA; for the bf16 MFMA
// the per-lane chunk is KS dims with KS a multiple of 8 and dp = 4*KS).
// SB: 16-sample blocks per wave.
template <int KS, int SB, int ROLE, bool XBF, bool GBF>
__global__ __launch_bounds__(256) void k_assign(AssignArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Ctl* ctl = a.ctl;
  if (ROLE != kRolePlain) {
    if (ctl->done) return;
    if (ROLE == kRoleFallback && !ctl->reject) return;
  }
  int* rho;
  const int* prev;
  if (ROLE == kRoleCand) {
    rho = a.lab + (int64_t)ctl->lab_cand * a.N;
    prev = a.lab + (int64_t)ctl->lab_prev * a.N;
  } else if (ROLE == kRoleFallback) {
    rho = a.lab + (int64_t)ctl->lab_fb * a.N;
    prev = a.lab + (int64_t)ctl->lab_prev * a.N;
  } else {
    rho = a.lab;
    prev = a.lab_prev;
  }
  const int slot = (ROLE == kRoleFallback) ? 1 : 0;

  constexpr int DP = 4 * KS;        // padded dimension
  constexpr int LD = DP + 4;        // LDS row stride (floats) of the f32 tile
  constexpr int LDB = DP + 8;       // LDS row stride (bf16) of the bf16 tile
  constexpr int NB = KS / 8 > 0 ? KS / 8 : 1;
  const int d = a.d, K = a.K;
  const int Kpad = (K + 15) & ~15;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r16 = lane & 15;

  // LDS: centroid tile, -||c||^2/2 per row, small reduction scratch.
  const int chunk = GBF ? (int)(65536 / (LDB * 2 + 4)) & ~15 : (int)(65536 / (LD * 4 + 4)) & ~15;
  const int kchunk = chunk < Kpad ? chunk : Kpad;
  float* Cs = (float*)smem_raw;                                  // kchunk x LD (f32 path)
  uint16_t* Cbs = (uint16_t*)smem_raw;                           // kchunk x LDB (bf16 path)
  float* ncs = (float*)(smem_raw + (GBF ? (size_t)kchunk * LDB * 2 : (size_t)kchunk * LD * 4));
  float* fred = ncs + kchunk;          // 8 floats
  double* dred = (double*)(fred + 8);  // 4 doubles

  // max_j ||c_j||^2 and max_j delta_j over the real centroids
  float mx = 0.f, mdel = 0.f;
  for (int j = tid; j < K; j += 256) {
    mx = fmaxf(mx, a.nc[j]);
    if (GBF) mdel = fmaxf(mdel, a.delta[j]);
  }
  mx = wave_max(mx);
  mdel = wave_max(mdel);
  if (lane == 0) { fred[wave] = mx; fred[4 + wave] = mdel; }
  __syncthreads();
  const float cmax = sqrtf(fmaxf(fmaxf(fred[0], fred[1]), fmaxf(fred[2], fred[3]))) * 1.0001f;
  const float dmax = GBF ? fmaxf(fmaxf(fred[4], fred[5]), fmaxf(fred[6], fred[7])) * 1.0001f : 0.f;

  // Sample rows of this wave, kept in registers.
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * SB);
  const bool vec = (d == DP);
  float xv[SB][KS];
  i16x8 xbv[SB][NB];
  float xerr[SB];  // ||x - bf16(x)||^2 partial when float32 X feeds the bf16 GEMM
#pragma unroll
  for (int s = 0; s < SB; ++s) {
    xerr[s] = 0.f;
    const int64_t i = row0 + 16 * s + r16;
    if (i < a.N) {
      load_chunk<KS, XBF>(a.X, i, d, g * KS, vec, xv[s]);
    } else {
#pragma unroll
      for (int q = 0; q < KS; ++q) xv[s][q] = 0.f;
    }
    if constexpr (GBF) {
      // X values are exact in bfloat16 when stored so; otherwise this rounds.
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint16_t hb = f32_to_bf16_rne(xv[s][8 * q + e]);
          xbv[s][q][e] = (short)hb;
          if (!XBF) {
            const float df = xv[s][8 * q + e] - bf16_to_f32(hb);
            xerr[s] = fmaf(df, df, xerr[s]);
          }
        }
    }
  }

  float best[SB], sec[SB];
  int bidx[SB];
#pragma unroll
  for (int s = 0; s < SB; ++s) { best[s] = -__builtin_inff(); sec[s] = -__builtin_inff(); bidx[s] = 0; }

  for (int c0 = 0; c0 < Kpad; c0 += kchunk) {
    const int rows = (Kpad - c0) < kchunk ? (Kpad - c0) : kchunk;
    __syncthreads();
    if constexpr (GBF) {
      for (int e = tid; e < rows * DP; e += 256) {
        const int rr = e / DP, col = e - rr * DP, j = c0 + rr;
        Cbs[rr * LDB + col] = (j < K && col < d) ? a.Cb[(int64_t)j * d + col] : (uint16_t)0;
      }
    } else {
      for (int e = tid; e < rows * DP; e += 256) {
        const int rr = e / DP, col = e - rr * DP, j = c0 + rr;
        Cs[rr * LD + col] = (j < K && col < d) ? a.C[(int64_t)j * d + col] : 0.f;
      }
    }
    for (int rr = tid; rr < rows; rr += 256) {
      const int j = c0 + rr;
      ncs[rr] = (j < K) ? -0.5f * a.nc[j] : -__builtin_inff();
    }
    __syncthreads();

    for (int tt = 0; tt < rows; tt += 16) {
      float av[KS];
      i16x8 ab[NB];
      if constexpr (GBF) {
        const i16x8* cr = (const i16x8*)(Cbs + (tt + r16) * LDB + g * KS);
#pragma unroll
        for (int q = 0; q < NB; ++q) ab[q] = cr[q];
      } else {
        const float* cr = Cs + (tt + r16) * LD + g * KS;
        if constexpr (KS % 4 == 0) {
#pragma unroll
          for (int q = 0; q < KS; q += 4) {
            const float4 v = *(const float4*)(cr + q);
            av[q] = v.x; av[q + 1] = v.y; av[q + 2] = v.z; av[q + 3] = v.w;
          }
        } else {
#pragma unroll
          for (int q = 0; q < KS; ++q) av[q] = cr[q];
        }
      }
      const f32x4 n4 = *(const f32x4*)(ncs + tt + 4 * g);
      const int jb = c0 + tt;
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const f32x4 acc = tile_dot<KS, GBF>(av, xv[s], ab, xbv[s], n4);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float v = acc[r];
          const bool gt = v > best[s];
          sec[s] = fmaxf(sec[s], fminf(v, best[s]));
          best[s] = fmaxf(best[s], v);
          bidx[s] = gt ? (jb + r) : bidx[s];
        }
      }
    }
  }

  // Epilogue: combine the 4 lane groups, flag near ties, exact energy terms.
  const float u = 5.9604644775390625e-8f;  // 2^-24
  const float gam = 2.0f * ((float)(DP + 3) * u) / (1.0f - (float)(DP + 3) * u) * 1.001f;
  double e_wave = 0.0;
  unsigned n_changed = 0, n_flag = 0;
#pragma unroll
  for (int s = 0; s < SB; ++s) {
    const int64_t i = row0 + 16 * s + r16;
    const bool valid = i < a.N;
    float b = best[s], sc = sec[s];
    int bi = bidx[s] + 4 * g;
#pragma unroll
    for (int off = 16; off <= 32; off <<= 1) {
      const float ob = __shfl_xor(b, off, kWave);
      const int oi = __shfl_xor(bi, off, kWave);
      const float os = __shfl_xor(sc, off, kWave);
      const float ns = fmaxf(fmaxf(sc, os), fminf(b, ob));
      const bool take = (ob > b) || (ob == b && oi < bi);
      b = take ? ob : b;
      bi = take ? oi : bi;
      sc = ns;
    }
    if (bi < 0 || bi >= K) bi = 0;
    float xs = 0.f;
#pragma unroll
    for (int q = 0; q < KS; ++q) xs = fmaf(xv[s][q], xv[s][q], xs);
    xs += __shfl_xor(xs, 16, kWave);
    xs += __shfl_xor(xs, 32, kWave);
    const float nx = sqrtf(xs) * 1.0001f;
    float bound;
    if (GBF) {
      // s_j is computed from bf16(x) . bf16(c_j): |x.c - x^.c^| <= ex ||c|| + ||x^|| delta_j
      float ex = 0.f;
      if (!XBF) {
        float e2 = xerr[s];
        e2 += __shfl_xor(e2, 16, kWave);
        e2 += __shfl_xor(e2, 32, kWave);
        ex = sqrtf(e2) * 1.0001f;
      }
      const float cb = cmax + dmax;
      bound = gam * (nx + ex + cb) * (nx + ex + cb) + 4.0f * (ex * cb + (nx + ex) * dmax);
    } else {
      bound = gam * (nx + cmax) * (nx + cmax);
    }
    const bool flag = valid && !((b - sc) > bound);

    // exact energy term of the provisional label
    double term;
    {
      const float* cr = a.C + (int64_t)bi * d + g * KS;
      double p = 0.0;
#pragma unroll
      for (int q = 0; q < KS; ++q) {
        if (g * KS + q < d) {
          const double df = (double)xv[s][q] - (double)cr[q];
          p = fma(df, df, p);
        }
      }
      p += __shfl_xor(p, 16, kWave);
      p += __shfl_xor(p, 32, kWave);
      term = p;
    }

    unsigned long long fm = __ballot(flag) & 0xFFFFull;
    n_flag += (unsigned)__popcll(fm);
    while (fm) {
      const int f = __ffsll((long long)fm) - 1;
      fm &= fm - 1;
      double dist;
      const int j = exact_argmin<XBF>(a.X, row0 + 16 * s + f, d, a.C, K, lane, &dist);
      if (j >= 0 && r16 == f) { bi = j; term = dist; }
    }

    bool ch = false;
    if (valid && g == 0) {
      rho[i] = bi;
      ch = (prev != nullptr) && (prev[i] != bi);
    }
    n_changed += (unsigned)__popcll(__ballot(ch));
    e_wave += wave_sum((valid && g == 0) ? term : 0.0);
  }

  if (lane == 0) {
    dred[wave] = e_wave;
    if (n_changed) atomicAdd(&ctl->cnt_changed[slot], (unsigned long long)n_changed);
    if (n_flag) atomicAdd(&ctl->cnt_flagged[slot], (unsigned long long)n_flag);
  }
  __syncthreads();
  if (tid == 0) a.e_part[blockIdx.x] = ((dred[0] + dred[1]) + dred[2]) + dred[3];
}

// ---------------------------------------------------------------------------
// Host-side dispatch
// ---------------------------------------------------------------------------

static int pick_ks(int d, int gemm_bf16) {
  static const int f32_ks[] = {1, 2, 4, 8, 12, 16, 24, 32, 48, 64};
  static const int bf_ks[] = {8, 16, 24, 32, 48, 64};
  const int need = (d + 3) / 4;
  if (gemm_bf16) {
    for (int k : bf_ks) if (k >= need) return k;
  } else {
    for (int k : f32_ks) if (k >= need) return k;
  }
  return -1;
}

static int pick_sb(int ks) { return ks <= 16 ? 4 : (ks <= 32 ? 2 : 1); }

int assign_grid(int64_t N, int d, int gemm_bf16) {
  const int ks = pick_ks(d, gemm_bf16);
  if (ks < 0) return -1;
  const int64_t rows = 64 * pick_sb(ks);
  return (int)((N + rows - 1) / rows);
}

static size_t assign_lds(int ks, int K, int gbf) {
  const int DP = 4 * ks;
  const int Kpad = (K + 15) & ~15;
  if (gbf) {
    const int LDB = DP + 8;
    int chunk = (65536 / (LDB * 2 + 4)) & ~15;
    if (chunk > Kpad) chunk = Kpad;
    return (size_t)chunk * LDB * 2 + (size_t)chunk * 4 + 8 * 4 + 4 * 8;
  }
  const int LD = DP + 4;
  int chunk = (65536 / (LD * 4 + 4)) & ~15;
  if (chunk > Kpad) chunk = Kpad;
  return (size_t)chunk * LD * 4 + (size_t)chunk * 4 + 8 * 4 + 4 * 8;
}

template <int KS, int ROLE, bool XBF, bool GBF>
static hipError_t go(const AssignArgs& a, hipStream_t s) {
  constexpr int SB = KS <= 16 ? 4 : (KS <= 32 ? 2 : 1);
  const int64_t rows = 64 * SB;
  const int grid = (int)((a.N + rows - 1) / rows);
  const size_t lds = assign_lds(KS, a.K, GBF);
  hipLaunchKernelGGL((k_assign<KS, SB, ROLE, XBF, GBF>), dim3(grid), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <int ROLE, bool XBF, bool GBF>
static hipError_t dispatch_ks(const AssignArgs& a, hipStream_t s) {
  const int ks = pick_ks(a.d, GBF);
  if constexpr (GBF) {
    switch (ks) {
      case 8: return go<8, ROLE, XBF, GBF>(a, s);
      case 16: return go<16, ROLE, XBF, GBF>(a, s);
      case 24: return go<24, ROLE, XBF, GBF>(a, s);
      case 32: return go<32, ROLE, XBF, GBF>(a, s);
      case 48: return go<48, ROLE, XBF, GBF>(a, s);
      case 64: return go<64, ROLE, XBF, GBF>(a, s);
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (ks) {
      case 1: return go<1, ROLE, XBF, GBF>(a, s);
      case 2: return go<2, ROLE, XBF, GBF>(a, s);
      case 4: return go<4, ROLE, XBF, GBF>(a, s);
      case 8: return go<8, ROLE, XBF, GBF>(a, s);
      case 12: return go<12, ROLE, XBF, GBF>(a, s);
      case 16: return go<16, ROLE, XBF, GBF>(a, s);
      case 24: return go<24, ROLE, XBF, GBF>(a, s);
      case 32: return go<32, ROLE, XBF, GBF>(a, s);
      case 48: return go<48, ROLE, XBF, GBF>(a, s);
      case 64: return go<64, ROLE, XBF, GBF>(a, s);
      default: return hipErrorInvalidValue;
    }
  }
}

template <int ROLE>
static hipError_t dispatch_types(const AssignArgs& a, hipStream_t s) {
  if (a.gemm_bf16) {
    return a.xbf16 ? dispatch_ks<ROLE, true, true>(a, s) : dispatch_ks<ROLE, false, true>(a, s);
  }
  return a.xbf16 ? dispatch_ks<ROLE, true, false>(a, s) : dispatch_ks<ROLE, false, false>(a, s);
}

hipError_t launch_assign(const AssignArgs& a, Role role, hipStream_t s) {
  if (a.N <= 0 || a.K <= 0 || a.d <= 0 || a.d > kMaxD || a.K > kMaxK) return hipErrorInvalidValue;
  switch (role) {
    case kRolePlain: return dispatch_types<kRolePlain>(a, s);
    case kRoleCand: return dispatch_types<kRoleCand>(a, s);
    case kRoleFallback: return dispatch_types<kRoleFallback>(a, s);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Centroid preparation: ||c_j||^2 (float64 sum, rounded), bf16 shadow, delta_j
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_prep(const float* C, int K, int d, float* nc, uint16_t* Cb,
                                              float* delta) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= K) return;
  const float* cr = C + (int64_t)j * d;
  double p = 0.0, e = 0.0;
  for (int k = lane; k < d; k += kWave) {
    const float c = cr[k];
    p = fma((double)c, (double)c, p);
    if (Cb) {
      const uint16_t b = f32_to_bf16_rne(c);
      Cb[(int64_t)j * d + k] = b;
      const double df = (double)c - (double)bf16_to_f32(b);
      e = fma(df, df, e);
    }
  }
  p = wave_sum(p);
  e = wave_sum(e);
  if (lane == 0) {
    nc[j] = (float)p;
    if (Cb) delta[j] = (float)sqrt(e);
  }
}

hipError_t launch_prep(const float* C, int K, int d, float* nc, uint16_t* Cb, float* delta,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_prep, dim3((K + 3) / 4), dim3(256), 0, s, C, K, d, nc, Cb, delta);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_reduce_energy(const double* e_part, int n, double* out) {
  __shared__ double red[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += e_part[i];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_reduce_energy(const double* e_part, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_energy, dim3(1), dim3(256), 0, s, e_part, n, out);
  return hipGetLastError();
}

}  // namespace km
