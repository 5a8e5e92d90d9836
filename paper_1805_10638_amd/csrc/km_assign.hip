// Assignment step (Sec. 1, Eq. (3)) fused with the energy of Eq. (1).
//
// The squared distance ||x - c_j||^2 = ||x||^2 - 2 (x.c_j - ||c_j||^2 / 2), so
// the argmin over j is the argmax of s_j = x.c_j - ||c_j||^2 / 2.  The s_j
// of a 16-centroid x 16-sample tile come out of MFMA (v_mfma_f32_16x16x4f32,
// or v_mfma_f32_16x16x32_bf16) with the accumulator pre-loaded with
// -||c_j||^2 / 2; the running best and second-best s_j of each sample stay in
// registers across the whole K loop.
//
// Operand layout of the 16x16 MFMAs: lane l supplies row l%16 of A and
// column l%16 of B for the k-slice owned by lane group g = l/16, and
// receives D[4g+r][l%16], r = 0..3.  A is a tile of 16 centroids, B a tile of
// 16 samples, so each lane accumulates 4 centroids of one sample.  The
// reduction index is permuted so that lane group g owns the contiguous
// dimensions [g*KS, g*KS+KS): sample rows are read with wide contiguous loads
// and kept in registers for the whole K loop.
//
// Workgroups are persistent: each stages the centroids into LDS once (when
// they fit) and then walks row groups gridDim.x apart.
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
// bfloat16 GEMM.  Each centroid is held as a bfloat16 pair hi + lo (hi the
// rounding of c, lo the rounding of c - hi) and s_j accumulates x.hi + x.lo in
// float32: bf16 x bf16 products are exact, so the error is the float32
// summation of 2 dp + 3 terms plus ||x|| r_j, r_j = ||c_j - hi_j - lo_j|| <=
// 2^-16 ||c_j||.  A single bfloat16 copy of c would leave an error near
// 2^-9 ||x|| ||c||, about a hundred times the float32 bound, and the re-check
// would then dominate.  Float32 rows are split the same way (x.hi + x.lo ~ x,
// three products per slice, x_lo . c_lo and the residuals added to the bound).
// X stored as bfloat16 is exact in both modes.

#include <stdlib.h>

#include "km_launch.h"

namespace km {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short i16x8 __attribute__((ext_vector_type(8)));

constexpr int kAssignLdsBudget = 60 * 1024;   // bytes of LDS for the centroid tile

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
__device__ __forceinline__ int wave_argmin(double bd, int bj, double* dist) {
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

// Centroids from global memory, the sample staged in LDS (xrow, zero-padded
// to DP): float64 differences over the d real dimensions.
template <int DP>
__device__ __forceinline__ int exact_argmin(const float* xrow, int d, const float* C, int K, int lane,
                                            double* dist) {
  double bd = __builtin_inf();
  int bj = -1;
  const bool v4 = (d % 4) == 0;
  for (int j = lane; j < K; j += kWave) {
    const float* cr = C + (int64_t)j * d;
    double s = 0.0;
    if (v4) {
      for (int k = 0; k < d; k += 4) {
        const float4 x4 = *(const float4*)(xrow + k);
        const float4 c4 = *(const float4*)(cr + k);
        double df = (double)x4.x - (double)c4.x; s = fma(df, df, s);
        df = (double)x4.y - (double)c4.y; s = fma(df, df, s);
        df = (double)x4.z - (double)c4.z; s = fma(df, df, s);
        df = (double)x4.w - (double)c4.w; s = fma(df, df, s);
      }
    } else {
      for (int k = 0; k < d; ++k) {
        const double df = (double)xrow[k] - (double)cr[k];
        s = fma(df, df, s);
      }
    }
    if (s < bd) { bd = s; bj = j; }
  }
  return wave_argmin(bd, bj, dist);
}

// Centroids resident in LDS (row stride ld, zero-padded to DP) and the
// sample staged in LDS (xrow, zero-padded to DP).
template <int DP>
__device__ __forceinline__ int exact_argmin_lds(const float* xrow, const float* Cs, int ld, int K, int lane,
                                             double* dist) {
  double bd = __builtin_inf();
  int bj = -1;
  for (int j = lane; j < K; j += kWave) {
    const float* cr = Cs + j * ld;
    double s = 0.0;
    if constexpr (DP % 4 == 0) {
#pragma unroll 4
      for (int k = 0; k < DP; k += 4) {
        const float4 x4 = *(const float4*)(xrow + k);
        const float4 c4 = *(const float4*)(cr + k);
        double df = (double)x4.x - (double)c4.x; s = fma(df, df, s);
        df = (double)x4.y - (double)c4.y; s = fma(df, df, s);
        df = (double)x4.z - (double)c4.z; s = fma(df, df, s);
        df = (double)x4.w - (double)c4.w; s = fma(df, df, s);
      }
    } else {
      for (int k = 0; k < DP; ++k) {
        const double df = (double)xrow[k] - (double)cr[k];
        s = fma(df, df, s);
      }
    }
    if (s < bd) { bd = s; bj = j; }
  }
  return wave_argmin(bd, bj, dist);
}

template <int KS, bool GBF>
struct Tile {
  static constexpr int DP = 4 * KS;                    // padded dimension
  static constexpr int NB = GBF ? KS / 8 : 1;          // bf16 MFMAs per tile and operand half
  static constexpr int LD = DP + 4;                    // f32 LDS row stride (floats)
  static constexpr int LDB = 2 * DP + 8;               // bf16 LDS row stride: hi[DP], lo[DP], pad
  static constexpr int ROW_BYTES = GBF ? LDB * 2 : LD * 4;
  // centroid rows per LDS chunk (multiple of 16) for a given K
  static __host__ __device__ int chunk_rows(int K) {
    const int kpad = (K + 15) & ~15;
    int c = ((kAssignLdsBudget - 16 * DP * 4) / (ROW_BYTES + 4)) & ~15;
    return c < kpad ? c : kpad;
  }
  static __host__ __device__ size_t lds_bytes(int K) {
    const int c = chunk_rows(K);
    return (size_t)c * ROW_BYTES + (size_t)c * 4 + 32 * 4 + 16 * 8 + (size_t)16 * DP * 4;
  }
};

// MFMAs of one 16-centroid tile (rows [tt, tt+16) of the LDS chunk) against
// the SB sample blocks of this wave; accumulators start at -||c||^2/2.
// bf16: x.hi + x.lo per slice (and x_lo.hi for float32 rows, XLO).
template <int KS, int SB, bool GBF, bool XLO, typename XV>
__device__ __forceinline__ void tile_mfma(const float* Cs, const uint16_t* Cbs, const float* ncs,
                                          int tt, int g, int r16, const XV& xv,
                                          const i16x8 (&xbv)[SB][Tile<KS, GBF>::NB],
                                          const i16x8 (&xlv)[SB][XLO ? Tile<KS, GBF>::NB : 1],
                                          f32x4 (&acc)[SB]) {
  using T = Tile<KS, GBF>;
  const f32x4 n4 = *(const f32x4*)(ncs + tt + 4 * g);
#pragma unroll
  for (int s = 0; s < SB; ++s) acc[s] = n4;
  if constexpr (GBF) {
    i16x8 ah[T::NB], al[T::NB];
    const uint16_t* cr = Cbs + (tt + r16) * T::LDB + g * KS;
#pragma unroll
    for (int q = 0; q < T::NB; ++q) {
      ah[q] = *(const i16x8*)(cr + 8 * q);
      al[q] = *(const i16x8*)(cr + T::DP + 8 * q);
    }
#pragma unroll
    for (int q = 0; q < T::NB; ++q) {
#pragma unroll
      for (int s = 0; s < SB; ++s)
        acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf16x8, ah[q]), __builtin_bit_cast(bf16x8, xbv[s][q]), acc[s], 0, 0, 0);
#pragma unroll
      for (int s = 0; s < SB; ++s)
        acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf16x8, al[q]), __builtin_bit_cast(bf16x8, xbv[s][q]), acc[s], 0, 0, 0);
      if constexpr (XLO) {
#pragma unroll
        for (int s = 0; s < SB; ++s)
          acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              __builtin_bit_cast(bf16x8, ah[q]), __builtin_bit_cast(bf16x8, xlv[s][q]), acc[s], 0, 0, 0);
      }
    }
  } else {
    float av[KS];
    const float* cr = Cs + (tt + r16) * T::LD + g * KS;
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
#pragma unroll
    for (int q = 0; q < KS; ++q)
#pragma unroll
      for (int s = 0; s < SB; ++s)
        acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[q], xv[s][q], acc[s], 0, 0, 0);
  }
}

// bfloat16 bits -> float32 of element q of a lane's bf16 chunk
__device__ __forceinline__ float bf_elem(const i16x8& v, int e) {
  return bf16_to_f32((uint16_t)v[e]);
}

// KS: padded dims per lane group; SB: 16-sample blocks per wave; W: waves
// per workgroup (they share one LDS copy of the centroids).
template <int KS, int SB, int W, int ROLE, bool XBF, bool GBF>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu((!GBF && KS * SB <= 32) ? 4 : 1))) void k_assign(AssignArgs a) {
  constexpr int NT = 64 * W;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using T = Tile<KS, GBF>;
  constexpr int DP = T::DP, LD = T::LD, LDB = T::LDB, NB = T::NB;
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

  const int d = a.d, K = a.K;
  const int Kpad = (K + 15) & ~15;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r16 = lane & 15;

  // LDS: centroid tile, -||c||^2/2 per row, small reduction scratch.
  const int kchunk = T::chunk_rows(K);
  const bool resident = kchunk >= Kpad;
  float* Cs = (float*)smem_raw;                                  // kchunk x LD (f32 path)
  uint16_t* Cbs = (uint16_t*)smem_raw;                           // kchunk x LDB (bf16 path)
  float* ncs = (float*)(smem_raw + (size_t)kchunk * T::ROW_BYTES);
  float* fred = ncs + kchunk;          // 2 W floats (W <= 16)
  double* dred = (double*)(fred + 32); // W doubles

  // max_j ||c_j||^2 and max_j r_j over the real centroids
  float mx = 0.f, mdel = 0.f;
  for (int j = tid; j < K; j += NT) {
    mx = fmaxf(mx, a.nc[j]);
    if (GBF) mdel = fmaxf(mdel, a.delta[j]);
  }
  mx = wave_max(mx);
  mdel = wave_max(mdel);
  if (lane == 0) { fred[wave] = mx; fred[16 + wave] = mdel; }
  __syncthreads();
  float cm2 = 0.f, dm = 0.f;
#pragma unroll
  for (int w = 0; w < W; ++w) { cm2 = fmaxf(cm2, fred[w]); dm = fmaxf(dm, fred[16 + w]); }
  const float cmax = sqrtf(cm2) * 1.0001f;
  const float rmax = GBF ? dm * 1.0001f : 0.f;
  // float32 summation terms per s_j: dp products (f32), 2 dp or 3 dp exact
  // bf16 products, plus the accumulator start and two roundings of margin
  constexpr int NTERM = GBF ? (XBF ? 2 * DP + 3 : 3 * DP + 3) : DP + 3;
  const float u = 5.9604644775390625e-8f;  // 2^-24
  const float gam = 2.0f * ((float)NTERM * u) / (1.0f - (float)NTERM * u) * 1.001f;
  // ||hi_j|| + ||lo_j|| <= (1 + 2^-7 + 2^-16) ||c_j||
  const float cb = GBF ? cmax * 1.008f : cmax;

  // Stage centroid rows [c0, c0 + rows) into LDS (zero padding beyond d and K).
  auto stage = [&](int c0, int rows) {
    if constexpr (GBF) {
      const bool v8 = (d % 8) == 0;
      const int64_t KD = (int64_t)K * d;
      constexpr int V = DP / 8;   // 8-element vectors per half row
      for (int e = tid; e < rows * 2 * V; e += NT) {
        const int rr = e / (2 * V), rem = e - rr * (2 * V);
        const int half = rem >= V ? 1 : 0, c8 = (rem - half * V) * 8, j = c0 + rr;
        const uint16_t* src = a.Cb + half * KD + (int64_t)j * d;
        i16x8 v;
        if (v8 && j < K && c8 < d) {
          v = *(const i16x8*)(src + c8);
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q)
            v[q] = (j < K && c8 + q < d) ? (short)src[c8 + q] : (short)0;
        }
        *(i16x8*)(Cbs + rr * LDB + half * DP + c8) = v;
      }
    } else {
      const bool v4 = (d % 4) == 0;
      for (int e = tid; e < rows * (DP / 4); e += NT) {
        const int rr = e / (DP / 4), c4 = (e - rr * (DP / 4)) * 4, j = c0 + rr;
        float4 v;
        if (v4 && j < K && c4 < d) {
          v = *(const float4*)(a.C + (int64_t)j * d + c4);
        } else {
          v.x = (j < K && c4 + 0 < d) ? a.C[(int64_t)j * d + c4 + 0] : 0.f;
          v.y = (j < K && c4 + 1 < d) ? a.C[(int64_t)j * d + c4 + 1] : 0.f;
          v.z = (j < K && c4 + 2 < d) ? a.C[(int64_t)j * d + c4 + 2] : 0.f;
          v.w = (j < K && c4 + 3 < d) ? a.C[(int64_t)j * d + c4 + 3] : 0.f;
        }
        *(float4*)(Cs + rr * LD + c4) = v;
      }
    }
    for (int rr = tid; rr < rows; rr += NT) {
      const int j = c0 + rr;
      ncs[rr] = (j < K) ? -0.5f * a.nc[j] : -__builtin_inff();
    }
  };
  if (resident) {
    stage(0, Kpad);
    __syncthreads();
  }
  float* xrow = fred + 32 + 2 * 16 + wave * DP;   // per-wave row of a flagged sample

  const int64_t group_rows = 16 * SB * W;
  const int64_t groups = (a.N + group_rows - 1) / group_rows;
  const bool vec = (d == DP);
  double e_wave = 0.0;
  unsigned n_changed = 0, n_flag = 0;
  // float32 copy of the rows in registers only for the float32 GEMM; bf16 rows
  // are exact as bf16; float32 rows on the bf16 GEMM keep hi and lo (XLO)
  constexpr bool KF = !GBF;
  constexpr bool XLO = GBF && !XBF;

  for (int64_t grp = blockIdx.x; grp < groups; grp += gridDim.x) {
    // Sample rows of this wave, kept in registers.
    const int64_t row0 = grp * group_rows + (int64_t)wave * (16 * SB);
    float xv[SB][KF ? KS : 1];
    i16x8 xbv[SB][NB];
    i16x8 xlv[SB][XLO ? NB : 1];
    float xres[SB];  // ||x - hi - lo||^2 lane partial (XLO)
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      xres[s] = 0.f;
      const int64_t i = row0 + 16 * s + r16;
      if constexpr (GBF && XBF) {
        const uint16_t* xr = (const uint16_t*)a.X + i * d + g * KS;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          if (i < a.N && vec) {
            xbv[s][q] = *(const i16x8*)(xr + 8 * q);
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int k = g * KS + 8 * q + e;
              xbv[s][q][e] = (i < a.N && k < d) ? (short)xr[8 * q + e] : (short)0;
            }
          }
        }
      } else if constexpr (XLO) {
        float t[KS];
        if (i < a.N) {
          load_chunk<KS, XBF>(a.X, i, d, g * KS, vec, t);
        } else {
#pragma unroll
          for (int q = 0; q < KS; ++q) t[q] = 0.f;
        }
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            uint16_t h, l;
            const float r = (float)bf16_split(t[8 * q + e], &h, &l);
            xbv[s][q][e] = (short)h;
            xlv[s][q][e] = (short)l;
            xres[s] = fmaf(r, r, xres[s]);
          }
      } else {
        if (i < a.N) {
          load_chunk<KS, XBF>(a.X, i, d, g * KS, vec, xv[s]);
        } else {
#pragma unroll
          for (int q = 0; q < KS; ++q) xv[s][q] = 0.f;
        }
      }
    }

    float best[SB], sec[SB];
    int bidx[SB];
#pragma unroll
    for (int s = 0; s < SB; ++s) { best[s] = -__builtin_inff(); sec[s] = -__builtin_inff(); bidx[s] = 0; }

    for (int c0 = 0; c0 < Kpad; c0 += kchunk) {
      const int rows = (Kpad - c0) < kchunk ? (Kpad - c0) : kchunk;
      if (!resident) {
        __syncthreads();
        stage(c0, rows);
        __syncthreads();
      }
      for (int tt = 0; tt < rows; tt += 16) {
        f32x4 acc[SB];
        tile_mfma<KS, SB, GBF, XLO>(Cs, Cbs, ncs, tt, g, r16, xv, xbv, xlv, acc);
        const int jb = c0 + tt;
#pragma unroll
        for (int s = 0; s < SB; ++s) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float v = acc[s][r];
            const bool gt = v > best[s];
            // second best = median of (v, best, second) since second <= best;
            // best and its index follow the one compare (two selects).  No
            // inline asm may read these MFMA results: the compiler inserts the
            // MFMA-to-VALU wait states only for instructions it can see.
            sec[s] = __builtin_amdgcn_fmed3f(v, best[s], sec[s]);
            best[s] = gt ? v : best[s];
            bidx[s] = gt ? (jb + r) : bidx[s];
          }
        }
      }
    }

    // Epilogue: combine the 4 lane groups, flag near ties, exact energy terms.
    double e_lane = 0.0;
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
      // this lane's float32 values of its KS dimensions of the row
      float xe[KS];
      if constexpr (KF) {
#pragma unroll
        for (int q = 0; q < KS; ++q) xe[q] = xv[s][q];
      } else if constexpr (XBF) {
#pragma unroll
        for (int q = 0; q < KS; ++q) xe[q] = bf_elem(xbv[s][q >> 3], q & 7);
      } else {
        if (valid) {
          load_chunk<KS, XBF>(a.X, i, d, g * KS, vec, xe);
        } else {
#pragma unroll
          for (int q = 0; q < KS; ++q) xe[q] = 0.f;
        }
      }
      float xs = 0.f;
#pragma unroll
      for (int q = 0; q < KS; ++q) xs = fmaf(xe[q], xe[q], xs);
      xs += __shfl_xor(xs, 16, kWave);
      xs += __shfl_xor(xs, 32, kWave);
      const float nx = sqrtf(xs) * 1.0001f;
      float bound;
      if constexpr (GBF && XBF) {
        // per s_j: summation error + ||x|| r_j; gap error twice that, margin 2
        bound = gam * (nx + cb) * (nx + cb) + 4.0f * nx * rmax;
      } else if constexpr (XLO) {
        // x = xh + xl + rx: the dropped products are xh.r_j + xl.lo_j + xl.r_j
        // + rx.c_j, with ||xh|| + ||xl|| <= 1.008 ||x||, ||xl|| <= 2^-8 1.004 ||x||
        // and ||lo_j|| <= 2^-8 1.004 ||c_j||
        float e2 = xres[s];
        e2 += __shfl_xor(e2, 16, kWave);
        e2 += __shfl_xor(e2, 32, kWave);
        const float nrx = sqrtf(e2) * 1.0001f;
        const float nxs = nx * 1.008f;
        bound = gam * (nxs + cb) * (nxs + cb) + 4.0f * (nxs * rmax + nx * 1.6e-5f * cmax + nrx * cmax);
      } else {
        bound = gam * (nx + cmax) * (nx + cmax);
      }
      const bool flag = valid && !((b - sc) > bound);

      // exact energy term of the provisional label
      double term;
      {
        const float* cr = (resident && !GBF) ? Cs + bi * LD + g * KS : a.C + (int64_t)bi * d + g * KS;
        double p = 0.0;
#pragma unroll
        for (int q = 0; q < KS; ++q) {
          if (g * KS + q < d) {
            const double df = (double)xe[q] - (double)cr[q];
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
        // the flagged row is spread over lanes r16 == f of the 4 lane groups
        if (r16 == f) {
#pragma unroll
          for (int q = 0; q < KS; ++q) xrow[g * KS + q] = xe[q];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double dist;
        int j;
        if (!GBF && resident) j = exact_argmin_lds<DP>(xrow, Cs, LD, K, lane, &dist);
        else j = exact_argmin<DP>(xrow, d, a.C, K, lane, &dist);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (j >= 0 && r16 == f) { bi = j; term = dist; }
      }

      bool ch = false;
      if (valid && g == 0) {
        rho[i] = bi;
        ch = (prev != nullptr) && (prev[i] != bi);
      }
      n_changed += (unsigned)__popcll(__ballot(ch));
      e_lane += (valid && g == 0) ? term : 0.0;
    }
    e_wave += wave_sum(e_lane);
  }

  if (lane == 0) {
    dred[wave] = e_wave;
    if (n_changed) atomicAdd(&ctl->cnt_changed[slot], (unsigned long long)n_changed);
    if (n_flag) atomicAdd(&ctl->cnt_flagged[slot], (unsigned long long)n_flag);
  }
  __syncthreads();
  if (tid == 0) {
    double e = dred[0];
#pragma unroll
    for (int w = 1; w < W; ++w) e += dred[w];
    a.e_part[blockIdx.x] = e;
  }
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

struct KernelPick {
  const void* fn = nullptr;
  int rows = 0;        // samples per row group (16 * SB * W)
  int threads = 0;     // 64 * W
  size_t lds = 0;
};

// Tile shapes (SB sample blocks per wave, W waves per workgroup) per KS.
// The default comes from measurements on MI355X; KM_ASSIGN_SHAPE=<n>
// selects an alternative for tuning runs.
template <int KS, int ROLE, bool XBF, bool GBF, int SB, int W>
static KernelPick make_pick(int K) {
  KernelPick p;
  p.fn = (const void*)&k_assign<KS, SB, W, ROLE, XBF, GBF>;
  p.rows = 16 * SB * W;
  p.threads = 64 * W;
  p.lds = Tile<KS, GBF>::lds_bytes(K);
  return p;
}

static int shape_override() {
  static int v = -2;
  if (v == -2) {
    const char* e = getenv("KM_ASSIGN_SHAPE");
    v = e ? atoi(e) : -1;
  }
  return v;
}

template <int KS, int ROLE, bool XBF, bool GBF>
static KernelPick pick_one(int K) {
  // default: two 16-sample blocks per wave up to 64 padded dimensions per
  // lane group (measured best for d = 32: 190 us vs 213 us with four blocks
  // at N = 1e6, K = 256), one block beyond.
  // The bf16 GEMM on bf16 rows streams centroid chunks through LDS for large
  // K: 16 waves of two 16-sample blocks share each staged chunk (three blocks
  // exceed the 128 registers of a 1024-thread workgroup).  Float32 rows on
  // the bf16 GEMM hold hi and lo operands: one block per wave.
  constexpr bool BIG = GBF && XBF && KS <= 32;
  constexpr int SB0 = BIG ? 2 : (GBF ? 1 : (KS <= 32 ? 2 : 1));
  constexpr int W0 = BIG ? 16 : 4;
  // alternative shapes are only built for the benchmark widths (d = 32 in
  // float32, d = 128 in bfloat16) and the candidate role
  if constexpr (ROLE == kRoleCand && KS == 8 && !GBF) {
    switch (shape_override()) {
      case 1: return make_pick<KS, ROLE, XBF, GBF, SB0, 8>(K);
      case 2: return make_pick<KS, ROLE, XBF, GBF, 4, 4>(K);
      case 3: return make_pick<KS, ROLE, XBF, GBF, 1, 8>(K);
      default: break;
    }
  }
  if constexpr (ROLE == kRoleCand && KS == 32 && BIG) {
    switch (shape_override()) {
      case 1: return make_pick<KS, ROLE, XBF, GBF, 3, 8>(K);
      case 2: return make_pick<KS, ROLE, XBF, GBF, 2, 8>(K);
      case 3: return make_pick<KS, ROLE, XBF, GBF, 1, 16>(K);
      default: break;
    }
  }
  return make_pick<KS, ROLE, XBF, GBF, SB0, W0>(K);
}

template <int ROLE, bool XBF, bool GBF>
static KernelPick pick_ks_role(int d, int K) {
  const int ks = pick_ks(d, GBF);
  if constexpr (GBF) {
    switch (ks) {
      case 8: return pick_one<8, ROLE, XBF, GBF>(K);
      case 16: return pick_one<16, ROLE, XBF, GBF>(K);
      case 24: return pick_one<24, ROLE, XBF, GBF>(K);
      case 32: return pick_one<32, ROLE, XBF, GBF>(K);
      case 48: return pick_one<48, ROLE, XBF, GBF>(K);
      case 64: return pick_one<64, ROLE, XBF, GBF>(K);
    }
  } else {
    switch (ks) {
      case 1: return pick_one<1, ROLE, XBF, GBF>(K);
      case 2: return pick_one<2, ROLE, XBF, GBF>(K);
      case 4: return pick_one<4, ROLE, XBF, GBF>(K);
      case 8: return pick_one<8, ROLE, XBF, GBF>(K);
      case 12: return pick_one<12, ROLE, XBF, GBF>(K);
      case 16: return pick_one<16, ROLE, XBF, GBF>(K);
      case 24: return pick_one<24, ROLE, XBF, GBF>(K);
      case 32: return pick_one<32, ROLE, XBF, GBF>(K);
      case 48: return pick_one<48, ROLE, XBF, GBF>(K);
      case 64: return pick_one<64, ROLE, XBF, GBF>(K);
    }
  }
  return KernelPick();
}

template <int ROLE>
static KernelPick pick_types(const AssignArgs& a) {
  if (a.gemm_bf16)
    return a.xbf16 ? pick_ks_role<ROLE, true, true>(a.d, a.K) : pick_ks_role<ROLE, false, true>(a.d, a.K);
  return a.xbf16 ? pick_ks_role<ROLE, true, false>(a.d, a.K) : pick_ks_role<ROLE, false, false>(a.d, a.K);
}

static KernelPick pick(const AssignArgs& a, Role role) {
  switch (role) {
    case kRolePlain: return pick_types<kRolePlain>(a);
    case kRoleCand: return pick_types<kRoleCand>(a);
    case kRoleFallback: return pick_types<kRoleFallback>(a);
  }
  return KernelPick();
}

// Persistent grid: as many workgroups as fit on the device at once (queried
// once per kernel instance), never more than there are row groups.
int assign_grid(const AssignArgs& a) {
  if (a.N <= 0 || a.K <= 0 || a.d <= 0 || a.d > kMaxD || a.K > kMaxK) return -1;
  const KernelPick p = pick(a, kRoleCand);
  if (!p.fn) return -1;
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
      clear_pending_error();
      cus = 256;
    }
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, p.fn, p.threads, p.lds) != hipSuccess ||
      per_cu <= 0) {
    clear_pending_error();
    per_cu = 1;
  }
  const int64_t groups = (a.N + p.rows - 1) / p.rows;
  int64_t resident = (int64_t)per_cu * cus;
  if (const char* e = getenv("KM_ASSIGN_GRID_MULT")) resident *= atoi(e) > 0 ? atoi(e) : 1;
  return (int)(groups < resident ? groups : resident);
}

hipError_t launch_assign(const AssignArgs& a, Role role, hipStream_t s) {
  if (a.N <= 0 || a.K <= 0 || a.d <= 0 || a.d > kMaxD || a.K > kMaxK) return hipErrorInvalidValue;
  const KernelPick p = pick(a, role);
  if (!p.fn) return hipErrorInvalidValue;
  const int grid = assign_grid(a);
  if (grid <= 0) return hipErrorInvalidValue;
  AssignArgs arg = a;
  void* params[] = {&arg};
  clear_pending_error();
  return hipLaunchKernel(p.fn, dim3(grid), dim3(p.threads), params, p.lds, s);
}

// ---------------------------------------------------------------------------
// Centroid preparation: ||c_j||^2 (float64 sum, rounded), bf16 hi/lo pair, residual norms
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_prep(const float* C, int K, int d, float* nc, uint16_t* Cb,
                                              float* delta) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= K) return;
  const float* cr = C + (int64_t)j * d;
  const int64_t KD = (int64_t)K * d;
  double p = 0.0, e = 0.0;
  for (int k = lane; k < d; k += kWave) {
    const float c = cr[k];
    p = fma((double)c, (double)c, p);
    if (Cb) {
      uint16_t h, l;
      const double r = bf16_split(c, &h, &l);
      Cb[(int64_t)j * d + k] = h;
      Cb[KD + (int64_t)j * d + k] = l;
      e = fma(r, r, e);
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
  clear_pending_error();
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

// One workgroup: the controller stage that closes a pass (stage 1 after the
// candidate, stage 2 after the optional fall-back).
__global__ __launch_bounds__(256) void k_controller(CtlArgs a) {
  __shared__ double red[256];
  if (a.ctl->done) return;
  controller_stage(a.ctl, a.e_part, a.n_part, a.stage, a.tr, red);
}

hipError_t launch_controller(const CtlArgs& a, hipStream_t s) {
  clear_pending_error();
  hipLaunchKernelGGL(k_controller, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reduce_energy(const double* e_part, int n, double* out, hipStream_t s) {
  clear_pending_error();
  hipLaunchKernelGGL(k_reduce_energy, dim3(1), dim3(256), 0, s, e_part, n, out);
  return hipGetLastError();
}

}  // namespace km
