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
// they fit, else in chunks per row group) and then walks row groups a grid
// apart.  The same body serves one instance (the launch grid) and batched
// launches (a slice of the grid per instance).
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

#pragma once

#include <type_traits>

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

// load_chunk for U rows at once (ic: valid row indices; callers map rows
// past N to row 0 and discard their results).  The choice between 16-byte
// and per-column loads is made once for all rows, so every load of the U
// rows is in flight before the first is used; a branch per row would make
// the compiler wait for each row's loads before issuing the next row's.
template <int U, int KS, bool XBF>
__device__ __forceinline__ void load_rows(const void* X, const int64_t (&ic)[U], int d, int k0, bool vec,
                                          float (&out)[U][KS]) {
  if constexpr (KS % 4 == 0) {
    if (vec) {
#pragma unroll
      for (int s = 0; s < U; ++s) {
        if constexpr (XBF) {
          const uint2* p = (const uint2*)((const uint16_t*)X + ic[s] * d + k0);
#pragma unroll
          for (int q = 0; q < KS / 4; ++q) {
            const uint2 v = p[q];
            out[s][4 * q + 0] = __uint_as_float(v.x << 16);
            out[s][4 * q + 1] = __uint_as_float(v.x & 0xFFFF0000u);
            out[s][4 * q + 2] = __uint_as_float(v.y << 16);
            out[s][4 * q + 3] = __uint_as_float(v.y & 0xFFFF0000u);
          }
        } else {
          const float4* p = (const float4*)((const float*)X + ic[s] * d + k0);
#pragma unroll
          for (int q = 0; q < KS / 4; ++q) {
            const float4 v = p[q];
            out[s][4 * q + 0] = v.x;
            out[s][4 * q + 1] = v.y;
            out[s][4 * q + 2] = v.z;
            out[s][4 * q + 3] = v.w;
          }
        }
      }
      return;
    }
  }
  // other widths: one row at a time, which keeps the registers of the
  // loads in flight to one row's.  The wait at the end keeps these loads
  // from being pending where the two paths join: the compiler would
  // otherwise wait for every outstanding memory operation (the previous
  // unit's label stores included) before the 16-byte path's first load.
#pragma unroll
  for (int s = 0; s < U; ++s) load_chunk<KS, XBF>(X, ic[s], d, k0, false, out[s]);
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
}

// Wave reduction of per-lane (smallest distance bd, its index bj, second
// smallest distance bd2): lowest index on ties; the second smallest counts a
// second centroid at the smallest distance (then it equals the smallest).
// Every lane returns the label (-1 if every distance is NaN), with the two
// distances in *dist and *dist2.
__device__ __forceinline__ int wave_argmin2(double bd, double bd2, int bj, double* dist, double* dist2) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ob = __shfl_xor(bd, off, kWave);
    const double ob2 = __shfl_xor(bd2, off, kWave);
    const int oj = __shfl_xor(bj, off, kWave);
    const bool take = (ob < bd) || (ob == bd && (unsigned)oj < (unsigned)bj);
    const double hi = bd < ob ? ob : bd, lo2 = bd2 < ob2 ? bd2 : ob2;
    bd2 = hi < lo2 ? hi : lo2;
    bd = take ? ob : bd;
    bj = take ? oj : bj;
  }
  *dist = bd;
  *dist2 = bd2;
  return bj;
}

// Running smallest / second smallest distance of a lane (indices ascend).
__device__ __forceinline__ void keep_two(double s, int j, double& bd, double& bd2, int& bj) {
  if (s < bd) { bd2 = bd; bd = s; bj = j; }
  else if (s < bd2) bd2 = s;
}

// Near tie as the float64 oracle defines it: relative gap between the two
// smallest squared distances below 1e-6, or both zero.
__device__ __forceinline__ bool near_tie(double d1, double d2) {
  return (d2 - d1) < 1e-6 * d2 || d2 == 0.0;
}

// Largest float32 not above v (v >= 0 or +inf).
__device__ __forceinline__ float f32_down(double v) {
  float f = (float)v;
  if ((double)f > v) f = __uint_as_float(__float_as_uint(f) - 1u);
  return f;
}

// A float32 lower bound of sqrt(l2) (0 when l2 is not positive).
__device__ __forceinline__ float sqrt_down(double l2) {
  if (!(l2 > 0.0)) return 0.f;
  return f32_down(sqrt(l2) * (1.0 - 1e-15));
}

// Squared float64 distance between a sample and a centroid row, this lane's
// KS dimensions (xe: the sample's, cr: the centroid's), summed over the four
// lane groups: float64 differences of the float32 values, squares added in
// dimension order, then lane groups 16 and 32 apart.  Every lane holds the
// result.
template <int KS>
__device__ __forceinline__ double row_dist2(const float (&xe)[KS], const float* cr, int d, int g, bool vec) {
  double p = 0.0;
  bool done4 = false;
  if constexpr (KS % 4 == 0) {
    if (vec) {  // whole chunk real: 16-byte loads of the centroid row
#pragma unroll
      for (int q = 0; q < KS; q += 4) {
        const float4 c4 = *(const float4*)(cr + q);
        double df = (double)xe[q] - (double)c4.x; p = fma(df, df, p);
        df = (double)xe[q + 1] - (double)c4.y; p = fma(df, df, p);
        df = (double)xe[q + 2] - (double)c4.z; p = fma(df, df, p);
        df = (double)xe[q + 3] - (double)c4.w; p = fma(df, df, p);
      }
      done4 = true;
    }
  }
  if (!done4) {
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      if (g * KS + q < d) {
        const double df = (double)xe[q] - (double)cr[q];
        p = fma(df, df, p);
      }
    }
  }
  p += __shfl_xor(p, 16, kWave);
  p += __shfl_xor(p, 32, kWave);
  return p;
}

// Centroids resident in LDS (row stride ld, zero-padded to DP) and the
// sample staged in LDS (xrow, zero-padded to DP).
template <int DP>
__device__ __forceinline__ int exact_argmin_lds(const float* xrow, const float* Cs, int ld, int K, int lane,
                                             double* dist, double* dist2) {
  double bd = __builtin_inf(), bd2 = __builtin_inf();
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
    keep_two(s, j, bd, bd2, bj);
  }
  return wave_argmin2(bd, bd2, bj, dist, dist2);
}

// LDS layout.  HEAD: workgroup scratch (maxima: 32 floats; energy partials:
// 16 doubles; flagged-row list lengths: 2 x 16 ints; re-checked counts: 16
// ints, padded) and one staged row per wave
// for immediate re-checks (16 x DP floats).  AREA: the centroid chunk and its
// -||c||^2/2 values during the row groups; after the last row group the
// deferred re-check reuses it for RX sample rows (float64), per-wave
// reduction slots and float32 centroid rows.
constexpr int kAssignScratch = 128 + 128 + 128 + 128;

// LB: bytes of LDS a workgroup may use for the centroid chunk.
template <int KS, bool GBF, int LB>
struct Tile {
  static constexpr int DP = 4 * KS;                    // padded dimension
  static constexpr int NB = GBF ? KS / 8 : 1;          // bf16 MFMAs per tile and operand half
  static constexpr int LD = DP + 4;                    // f32 LDS row stride (floats)
  static constexpr int LDB = 2 * DP + 8;               // bf16 LDS row stride: hi[DP], lo[DP], pad
  static constexpr int ROW_BYTES = GBF ? LDB * 2 : LD * 4;
  static constexpr int HEAD = kAssignScratch + 16 * DP * 4;
  static constexpr int RX = DP <= 128 ? 16 : 8;        // rows per deferred re-check batch
  static constexpr int DEF_FIXED = RX * DP * 8 + RX * 16 * 24;
  static constexpr int DEF_MIN = DEF_FIXED + 16 * LD * 4;
  // centroid rows per LDS chunk (multiple of 16) for a given K
  static __host__ __device__ int chunk_rows(int K) {
    const int kpad = (K + 15) & ~15;
    int c = ((LB - HEAD) / (ROW_BYTES + 4)) & ~15;
    return c < kpad ? c : kpad;
  }
  static __host__ __device__ size_t area_bytes(int K) {
    const size_t c = (size_t)chunk_rows(K) * (ROW_BYTES + 4);
    return c > (size_t)DEF_MIN ? c : (size_t)DEF_MIN;
  }
  static __host__ __device__ size_t lds_bytes(int K) { return HEAD + area_bytes(K); }
  // float32 centroid rows per chunk of the deferred re-check (at least 16)
  static __host__ __device__ int def_rows(int K) { return (int)((area_bytes(K) - DEF_FIXED) / (LD * 4)); }
};

// A operand of one 16-centroid tile (rows [tt, tt+16) of the LDS chunk): this
// lane's centroid row r16, lane group g's dimensions, and the tile's
// -||c||^2/2 start values.  The tile loop loads the next tile's operand while
// the current tile's MFMAs run, so the LDS latency is not paid per tile.
template <int KS, bool GBF, int LB>
struct AOp {
  static constexpr int NB = Tile<KS, GBF, LB>::NB;
  f32x4 n4;
  i16x8 ah[GBF ? NB : 1], al[GBF ? NB : 1];  // bf16 hi and lo halves
  float av[GBF ? 1 : KS];                     // float32 row
};

template <int KS, bool GBF, int LB>
__device__ __forceinline__ void load_aop(const float* Cs, const uint16_t* Cbs, const float* ncs, int tt,
                                         int g, int r16, AOp<KS, GBF, LB>& o) {
  using T = Tile<KS, GBF, LB>;
  o.n4 = *(const f32x4*)(ncs + tt + 4 * g);
  if constexpr (GBF) {
    const uint16_t* cr = Cbs + (tt + r16) * T::LDB + g * KS;
#pragma unroll
    for (int q = 0; q < T::NB; ++q) {
      o.ah[q] = *(const i16x8*)(cr + 8 * q);
      o.al[q] = *(const i16x8*)(cr + T::DP + 8 * q);
    }
  } else {
    const float* cr = Cs + (tt + r16) * T::LD + g * KS;
    if constexpr (KS % 4 == 0) {
#pragma unroll
      for (int q = 0; q < KS; q += 4) {
        const float4 v = *(const float4*)(cr + q);
        o.av[q] = v.x; o.av[q + 1] = v.y; o.av[q + 2] = v.z; o.av[q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < KS; ++q) o.av[q] = cr[q];
    }
  }
}

// MFMAs of one tile against the SB sample blocks of this wave; accumulators
// start at -||c||^2/2.  bf16: x.hi + x.lo per slice (and x_lo.hi for float32
// rows, XLO).  A scheduling barrier after every group of SB independent MFMAs
// keeps the blocks in round-robin order, so that an MFMA never waits on the
// accumulator written just before it (the compiler otherwise pairs dependent
// MFMAs and pads them with wait states).
template <int KS, int SB, bool GBF, bool XLO, int LB, typename XV>
__device__ __forceinline__ void tile_mfma(const AOp<KS, GBF, LB>& o, const XV& xv,
                                          const i16x8 (&xbv)[SB][Tile<KS, GBF, LB>::NB],
                                          const i16x8 (&xlv)[SB][XLO ? Tile<KS, GBF, LB>::NB : 1],
                                          f32x4 (&acc)[SB]) {
  using T = Tile<KS, GBF, LB>;
#pragma unroll
  for (int s = 0; s < SB; ++s) acc[s] = o.n4;
  if constexpr (GBF) {
#pragma unroll
    for (int q = 0; q < T::NB; ++q) {
#pragma unroll
      for (int s = 0; s < SB; ++s)
        acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf16x8, o.ah[q]), __builtin_bit_cast(bf16x8, xbv[s][q]), acc[s], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int s = 0; s < SB; ++s)
        acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf16x8, o.al[q]), __builtin_bit_cast(bf16x8, xbv[s][q]), acc[s], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (XLO) {
#pragma unroll
        for (int s = 0; s < SB; ++s)
          acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              __builtin_bit_cast(bf16x8, o.ah[q]), __builtin_bit_cast(bf16x8, xlv[s][q]), acc[s], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < KS; ++q) {
#pragma unroll
      for (int s = 0; s < SB; ++s)
        acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(o.av[q], xv[s][q], acc[s], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// bfloat16 bits -> float32 of element q of a lane's bf16 chunk
__device__ __forceinline__ float bf_elem(const i16x8& v, int e) {
  return bf16_to_f32((uint16_t)v[e]);
}

// Waves per SIMD the register allocation must leave room for: 16-wave
// workgroups need 4; small float32 tiles run best at 4 (latency hiding),
// float32 tiles up to 32 dims x blocks at 3 (VGPRs come in blocks of 8, so
// 169 of them would already leave room for only 2);
// wide tiles (float32 rows on the bf16 GEMM, 8 sample blocks, d > 128 in
// bf16, more than 64 dims x blocks in float32) get the whole register file;
// the rest run 2 waves per SIMD.
template <int KS, int SB, int W, bool XBF, bool GBF>
constexpr int assign_wpe() {
  if (W >= 16) return 4;
  if (!GBF) {
    if (KS * SB <= 16 && SB <= 2) return 4;
    if (KS * SB <= 32 && KS <= 16) return 3;   // fits 168 VGPRs: 3 waves per SIMD
    return KS * SB > 64 ? 1 : 2;
  }
  if (!XBF || KS >= 48 || SB >= 8) return 1;
  return 2;
}

// KS: padded dims per lane group; SB: 16-sample blocks per wave; W: waves
// per workgroup (they share one LDS copy of the centroids); LB: LDS bytes.
// bx / gx: this workgroup's index and the number of workgroups working on
// this instance.
template <int KS, int SB, int W, bool XBF, bool GBF, int LB, bool BND = false>
__device__ __forceinline__ void assign_body(const AssignArgs& a, int bx, int gx) {
  constexpr int NT = 64 * W;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using T = Tile<KS, GBF, LB>;
  constexpr int DP = T::DP, LD = T::LD, LDB = T::LDB, NB = T::NB;
  Ctl* ctl = a.ctl;
  const int role = a.role;
  if (role != kRolePlain) {
    if (ctl->done) return;
    if (role == kRoleFallback && !ctl->reject) return;
  }
  int* rho;
  const int* prev;
  if (role == kRoleCand) {
    rho = a.lab + (int64_t)ctl->lab_cand * a.N;
    prev = a.lab + (int64_t)ctl->lab_prev * a.N;
  } else if (role == kRoleFallback) {
    rho = a.lab + (int64_t)ctl->lab_fb * a.N;
    prev = a.lab + (int64_t)ctl->lab_prev * a.N;
  } else {
    rho = a.lab;
    prev = a.lab_prev;
  }
  const int slot = (role == kRoleFallback) ? 1 : 0;
  // row bounds: written for this pass's labels (lbo), read for the previous ones (lbi)
  float* lbo = nullptr;
  const float* lbi = nullptr;
  if constexpr (BND) {
    if (a.lb) {
      if (role == kRoleCand) {
        lbo = a.lb + (int64_t)ctl->lab_cand * a.N;
        lbi = a.lb + (int64_t)ctl->lab_prev * a.N;
      } else if (role == kRoleFallback) {
        lbo = a.lb + (int64_t)ctl->lab_fb * a.N;
        lbi = a.lb + (int64_t)ctl->lab_prev * a.N;
      } else {
        lbo = a.lb;
      }
    }
  }

  const int d = a.d, K = a.K;
  const int Kpad = (K + 15) & ~15;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, r16 = lane & 15;

  // LDS (layout at Tile): scratch, per-wave rows, centroid chunk + norms.
  const int kchunk = T::chunk_rows(K);
  const bool resident = kchunk >= Kpad;
  float* fred = (float*)smem_raw;                            // 2 x 16 floats
  double* dred = (double*)(smem_raw + 128);                  // W doubles
  int* wcnt = (int*)(smem_raw + 256);                        // 2 x 16 list lengths
  int* pw = (int*)(smem_raw + 384);                          // 16 re-checked counts
  float* xrows = (float*)(smem_raw + kAssignScratch);        // 16 x DP floats
  unsigned char* area = smem_raw + T::HEAD;
  float* Cs = (float*)area;                                  // kchunk x LD (f32 path)
  uint16_t* Cbs = (uint16_t*)area;                           // kchunk x LDB (bf16 path)
  float* ncs = (float*)(area + (size_t)kchunk * T::ROW_BYTES);

  if (tid < 16) pw[tid] = 0;   // published by the barrier below

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
  // When every vector of a row is real (d = dp), each thread issues several
  // 16-byte loads before it writes any of them, so a chunk costs a few L2
  // round trips instead of one per vector: 8, or for chunks staged inside
  // the row-group loop 2 where registers are short there (float32 rows on
  // the bf16 GEMM at 256 dims, 4-wave-per-SIMD tiles, and float32 tiles up to
  // 64 dims, which would otherwise lose a wave per SIMD).  Other widths take
  // one vector at a time with per-element bounds.
  constexpr int kWpe = assign_wpe<KS, SB, W, XBF, GBF>();
  constexpr bool kShortRegs = (GBF && !XBF && KS >= 64) || kWpe >= 4 || (!GBF && KS <= 16);
  constexpr int kStageBatch = kShortRegs ? 2 : 8;
  // The one staging of resident centroids runs before any row is in
  // registers, so it always keeps 8 loads in flight.
  using StageAll = std::integral_constant<int, 8>;
  using StageLoop = std::integral_constant<int, kStageBatch>;
  // float32 rows [c0, c0 + rows) of C into dst (row stride LD, zero beyond d);
  // bt: 16-byte loads in flight per thread
  auto stage_f32 = [&](auto bt, float* dst, int c0, int rows) {
    constexpr int SBt = decltype(bt)::value;
    const int total = rows * (DP / 4);
    if (d == DP) {
      for (int e0 = tid; e0 < total; e0 += SBt * NT) {
        float4 v[SBt];
#pragma unroll
        for (int b = 0; b < SBt; ++b) {
          const int e = e0 + b * NT;
          const int rr = e / (DP / 4), c4 = (e - rr * (DP / 4)) * 4, j = c0 + rr;
          v[b] = (e < total && j < K) ? *(const float4*)(a.C + (int64_t)j * d + c4)
                                      : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int b = 0; b < SBt; ++b) {
          const int e = e0 + b * NT;
          if (e < total) {
            const int rr = e / (DP / 4), c4 = (e - rr * (DP / 4)) * 4;
            *(float4*)(dst + rr * LD + c4) = v[b];
          }
        }
      }
    } else {
      for (int e = tid; e < total; e += NT) {
        const int rr = e / (DP / 4), c4 = (e - rr * (DP / 4)) * 4, j = c0 + rr;
        const float* src = a.C + (int64_t)j * d;
        float4 v;
        v.x = (j < K && c4 + 0 < d) ? src[c4 + 0] : 0.f;
        v.y = (j < K && c4 + 1 < d) ? src[c4 + 1] : 0.f;
        v.z = (j < K && c4 + 2 < d) ? src[c4 + 2] : 0.f;
        v.w = (j < K && c4 + 3 < d) ? src[c4 + 3] : 0.f;
        *(float4*)(dst + rr * LD + c4) = v;
      }
    }
  };
  auto stage = [&](auto bt, int c0, int rows) {
    constexpr int SBt = decltype(bt)::value;
    // bfloat16 pair chunks of bfloat16 rows from 64 dims (streamed per row
    // group): the first NT rows' -||c||^2/2 are loaded before the row vectors
    // so that its latency overlaps theirs (an unconditional load at a clamped
    // index: a load inside a branch would be waited for before going on).
    // Elsewhere the extra register would cost an occupancy step.
    constexpr bool kNcEarly = GBF && XBF && KS >= 16;
    const int jn = c0 + tid;
    float nc0 = 0.f;
    if constexpr (kNcEarly) {
      const float ncv = a.nc[jn < K ? jn : K - 1];
      nc0 = jn < K ? -0.5f * ncv : -__builtin_inff();
    }
    if constexpr (GBF) {
      const int64_t KD = (int64_t)K * d;
      constexpr int V = DP / 8;   // 8-element vectors per half row
      const int total = rows * 2 * V;
      if (d == DP) {
        for (int e0 = tid; e0 < total; e0 += SBt * NT) {
          i16x8 v[SBt];
#pragma unroll
          for (int b = 0; b < SBt; ++b) {
            const int e = e0 + b * NT;
            const int rr = e / (2 * V), rem = e - rr * (2 * V);
            const int half = rem >= V ? 1 : 0, c8 = (rem - half * V) * 8, j = c0 + rr;
            v[b] = (e < total && j < K) ? *(const i16x8*)(a.Cb + half * KD + (int64_t)j * d + c8)
                                        : i16x8{0, 0, 0, 0, 0, 0, 0, 0};
          }
#pragma unroll
          for (int b = 0; b < SBt; ++b) {
            const int e = e0 + b * NT;
            if (e < total) {
              const int rr = e / (2 * V), rem = e - rr * (2 * V);
              const int half = rem >= V ? 1 : 0, c8 = (rem - half * V) * 8;
              *(i16x8*)(Cbs + rr * LDB + half * DP + c8) = v[b];
            }
          }
        }
      } else {
        for (int e = tid; e < total; e += NT) {
          const int rr = e / (2 * V), rem = e - rr * (2 * V);
          const int half = rem >= V ? 1 : 0, c8 = (rem - half * V) * 8, j = c0 + rr;
          const uint16_t* src = a.Cb + half * KD + (int64_t)j * d;
          i16x8 v;
#pragma unroll
          for (int q = 0; q < 8; ++q) v[q] = (j < K && c8 + q < d) ? (short)src[c8 + q] : (short)0;
          *(i16x8*)(Cbs + rr * LDB + half * DP + c8) = v;
        }
      }
    } else {
      stage_f32(bt, Cs, c0, rows);
    }
    if constexpr (kNcEarly) {
      if (tid < rows) ncs[tid] = nc0;
    }
    for (int rr = kNcEarly ? tid + NT : tid; rr < rows; rr += NT) {
      const int j = c0 + rr;
      ncs[rr] = (j < K) ? -0.5f * a.nc[j] : -__builtin_inff();
    }
  };
  if (resident) {
    stage(StageAll{}, 0, Kpad);
    __syncthreads();
  }
  // Row bounds in use (candidate and fall-back passes, centroids resident):
  // the largest and second largest centroid shift ||c_j - c_ref_j|| (upper
  // bounds, float64, written by the step that formed this pass's centroids)
  // and the index of the largest.  A row whose previous label is j1 moved
  // away from every other centroid by at most sm2, any other row by at most
  // sm1.
  const bool use_in = BND && lbi != nullptr && a.bounds && resident;
  double sm1 = 0.0, sm2 = 0.0;
  int sj1 = -1;
  if constexpr (BND) {
    if (use_in) {
      double m1 = 0.0, m2 = 0.0;
      int j1 = -1;
      for (int j = tid; j < K; j += NT) {
        const double sh = a.shift[j];
        if (sh > m1) { m2 = m1; m1 = sh; j1 = j; }
        else if (sh > m2) m2 = sh;
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const double o1 = __shfl_xor(m1, off, kWave), o2 = __shfl_xor(m2, off, kWave);
        const int oj = __shfl_xor(j1, off, kWave);
        const double lo = o1 < m1 ? o1 : m1, hi2 = o2 > m2 ? o2 : m2;
        m2 = lo > hi2 ? lo : hi2;
        if (o1 > m1 || (o1 == m1 && (unsigned)oj < (unsigned)j1)) { m1 = o1; j1 = oj; }
      }
      double* t1 = dred;                        // W doubles
      double* t2 = (double*)(smem_raw + 256);   // W doubles (the list-length slots, unused here)
      int* tj = pw;                             // W ints
      if (lane == 0) { t1[wave] = m1; t2[wave] = m2; tj[wave] = j1; }
      __syncthreads();
      for (int w = 0; w < W; ++w) {
        const double o1 = t1[w], o2 = t2[w];
        const int oj = tj[w];
        const double lo = o1 < sm1 ? o1 : sm1, hi2 = o2 > sm2 ? o2 : sm2;
        sm2 = lo > hi2 ? lo : hi2;
        if (o1 > sm1 || (o1 == sm1 && (unsigned)oj < (unsigned)sj1)) { sm1 = o1; sj1 = oj; }
      }
      __syncthreads();
      if (tid < 16) pw[tid] = 0;
    }
  }
  // Flagged rows.  With float32 centroids resident in LDS a wave re-checks a
  // row at once from the LDS copy (xrow: its staged row).  Otherwise each
  // wave appends the rows it flags to its own list, and the workgroup
  // re-checks them together in batches (recheck_batches below): at the end
  // of every row group when a full batch is pending and the centroids are
  // streamed, and after the last row group; the centroids are read once per
  // batch of rows rather than once per row.
  // The p-th row a wave flags is stored in the slot of the p-th row it owns
  // (its rows of row groups bx, bx + gx, ...), so every list fits in N ints
  // and its order is fixed.
  float* xrow = xrows + wave * DP;
  const bool defer = GBF || !resident;             // uniform per launch
  int nfl = 0;                                     // rows this wave has listed

  const int64_t group_rows = 16 * SB * W;
  const int64_t groups = (a.N + group_rows - 1) / group_rows;
  const bool vec = (d == DP);
  double e_wave = 0.0;
  unsigned n_changed = 0, n_flag = 0, n_near = 0, n_gemm = 0;
  // float32 copy of the rows in registers only for the float32 GEMM; bf16 rows
  // are exact as bf16; float32 rows on the bf16 GEMM keep hi and lo (XLO)
  constexpr bool KF = !GBF;
  constexpr bool XLO = GBF && !XBF;
  using AO = AOp<KS, GBF, LB>;
  // float32 rows on the bf16 GEMM at 256 dims and float32 tiles beyond 128
  // dims have no registers for a second operand buffer (it would spill)
  constexpr bool kPairOps = !(XLO && KS >= 64) && !(!GBF && KS >= 48);

  // Re-check of the listed rows: float64 direct differences to all K
  // centroids (dimensions in order), the lowest distance wins, ties to the
  // lowest index.  Rows go in batches of RX (staged as float64), centroids in
  // chunks of def_rows(K) float32 rows.  Thread t scores centroid slots
  // t % S, t % S + S, ... of a chunk against rows rg, rg + G, ... of the
  // batch (rg = t / S, G = NT / S >= 2; S is a multiple of 64, so a wave
  // shares its rows and reduces them with shuffles).  The energy terms of the
  // batch are added in row order by thread 0.  Called by all threads after a
  // barrier that published the waves' list lengths wc; pw[w] counts the rows
  // of wave w's list already re-checked, and batches take pending rows with
  // the waves in order, so the batches depend on the data only.  Without
  // final only full batches run.
  double e_def = 0.0;
  // rows per batch: the layout's RX, or 8 where registers are short
  constexpr int RX = kShortRegs && T::RX > 8 ? 8 : T::RX;
  constexpr int MR = RX / 2;
  constexpr bool kInterleave = GBF && !(XLO && KS >= 64);
  auto recheck_batches = [&](const int* wc, bool final) {
    double* xb = (double*)area;                          // RX x DP
    double* redd = (double*)(area + RX * DP * 8);        // RX x 16 waves
    double* redd2 = redd + RX * 16;                      // RX x 16 waves: second smallest
    int* redj = (int*)(redd2 + RX * 16);                 // RX x 16 waves
    int* rowidx = redj + RX * 16;                        // RX
    double* rowdist = (double*)(rowidx + RX);            // RX
    float* cc = (float*)(area + T::DEF_FIXED);           // def_rows(K) x LD
    const int crows = T::def_rows(K);
    const int want = crows < NT / 2 ? crows : NT / 2;
    int S = 64;
    while (S < want) S <<= 1;
    const int G = NT / S;
    const int cs = tid % S, rg = tid / S;
    int pending = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) pending += wc[w] - pw[w];
    while (pending >= RX || (final && pending > 0)) {
      const int rb = pending < RX ? pending : RX;
      if (tid < rb) {   // the tid-th pending row, waves in order
        int r = tid, w = 0;
        while (r >= wc[w] - pw[w]) { r -= wc[w] - pw[w]; ++w; }
        const int q = pw[w] + r;
        const int64_t own = (bx + (int64_t)(q / (16 * SB)) * gx) * group_rows + w * (16 * SB) + q % (16 * SB);
        rowidx[tid] = a.flags[own];
      }
      __syncthreads();
      for (int e = tid; e < RX * DP; e += NT) {
        const int u = e / DP, k = e - u * DP;
        double v = 0.0;
        if (u < rb && k < d) v = (double)ld_x(a.X, (int64_t)rowidx[u] * d + k, XBF);
        xb[e] = v;
      }
      // second smallest distance per row kept in float32 (it only decides
      // whether a re-checked row counts as a near tie), saving registers
      double bd[MR];
      float bd2[MR];
      int bj[MR];
#pragma unroll
      for (int m = 0; m < MR; ++m) { bd[m] = __builtin_inf(); bd2[m] = __builtin_inff(); bj[m] = -1; }
      for (int c0 = 0; c0 < K; c0 += crows) {
        const int rows = (K - c0) < crows ? (K - c0) : crows;
        __syncthreads();
        stage_f32(StageLoop{}, cc, c0, rows);
        __syncthreads();
        for (int jj = cs; jj < rows; jj += S) {
          const float* cr = cc + jj * LD;
          const int j = c0 + jj;
#pragma unroll
          for (int m0 = 0; m0 < MR; m0 += 4) {
            if (rg + G * m0 >= rb) break;
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int k = 0; k < DP; k += 4) {
              const float4 c4 = *(const float4*)(cr + k);
              const double cx = c4.x, cy = c4.y, cz = c4.z, cw = c4.w;
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int u = rg + G * (m0 + r);
                if (u < rb) {
                  const double* xr = xb + u * DP + k;
                  double df = xr[0] - cx; acc[r] = fma(df, df, acc[r]);
                  df = xr[1] - cy; acc[r] = fma(df, df, acc[r]);
                  df = xr[2] - cz; acc[r] = fma(df, df, acc[r]);
                  df = xr[3] - cw; acc[r] = fma(df, df, acc[r]);
                }
              }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int m = m0 + r;
              if (acc[r] < bd[m]) { bd2[m] = (float)bd[m]; bd[m] = acc[r]; bj[m] = j; }
              else bd2[m] = fminf(bd2[m], (float)acc[r]);
            }
          }
        }
      }
#pragma unroll
      for (int m = 0; m < MR; ++m) {
        const int u = rg + G * m;
        if (u < rb) {
          double dist, dist2;
          const int j = wave_argmin2(bd[m], (double)bd2[m], bj[m], &dist, &dist2);
          if (lane == 0) { redd[u * 16 + wave] = dist; redd2[u * 16 + wave] = dist2; redj[u * 16 + wave] = j; }
        }
      }
      __syncthreads();
      bool ch = false, nt = false;
      if (tid < rb) {
        const int w0 = (tid % G) * (S / 64), w1 = w0 + S / 64;
        double bdist = redd[tid * 16 + w0], bdist2 = redd2[tid * 16 + w0];
        int bjj = redj[tid * 16 + w0];
        for (int w = w0 + 1; w < w1; ++w) {
          const double od = redd[tid * 16 + w], od2 = redd2[tid * 16 + w];
          const int oj = redj[tid * 16 + w];
          const bool take = (od < bdist) || (od == bdist && (unsigned)oj < (unsigned)bjj);
          const double hi = bdist < od ? od : bdist, lo2 = bdist2 < od2 ? bdist2 : od2;
          bdist2 = hi < lo2 ? hi : lo2;
          bdist = take ? od : bdist;
          bjj = take ? oj : bjj;
        }
        const int i = rowidx[tid];
        const int jl = bjj >= 0 ? bjj : 0;
        rho[i] = jl;
        ch = (prev != nullptr) && (prev[i] != jl);
        nt = near_tie(bdist, bdist2);
        rowdist[tid] = bdist;
      }
      if (wave == 0) {
        n_changed += (unsigned)__popcll(__ballot(ch));
        n_near += (unsigned)__popcll(__ballot(nt));
      }
      __syncthreads();
      if (tid == 0) {
        for (int u = 0; u < rb; ++u) e_def += rowdist[u];
        int c = rb;   // consume the batch from the waves' pending ranges
        for (int w = 0; w < W && c > 0; ++w) {
          const int av = wc[w] - pw[w];
          const int take = av < c ? av : c;
          pw[w] += take;
          c -= take;
        }
      }
      __syncthreads();
      pending -= rb;
    }
  };

  // One unit of work of this wave: U 16-sample blocks from row row0 (U = SB
  // inside a row group; U = 1 for the single blocks that end a balanced
  // range).
  auto unit = [&](auto ut, const int64_t row0, const int* qrows, const int qcnt) {
    constexpr int U = decltype(ut)::value;
    // rows of the unit: consecutive from row0, or the first qcnt entries of
    // an LDS queue (positions past qcnt are not rows: index N)
    int64_t ii[U];
#pragma unroll
    for (int s = 0; s < U; ++s) {
      if (qrows) ii[s] = (16 * s + r16 < qcnt) ? (int64_t)qrows[16 * s + r16] : a.N;
      else ii[s] = row0 + 16 * s + r16;
    }
    // Sample rows of this wave, kept in registers.  Rows past N load row 0
    // (their results are discarded), so no load waits behind a branch and
    // the loads of all U blocks are in flight together.
    int64_t ic[U];
#pragma unroll
    for (int s = 0; s < U; ++s) ic[s] = ii[s] < a.N ? ii[s] : 0;
    float xv[U][KF ? KS : 1];
    i16x8 xbv[U][NB];
    i16x8 xlv[U][XLO ? NB : 1];
    float xres[U];  // ||x - hi - lo||^2 lane partial (XLO)
#pragma unroll
    for (int s = 0; s < U; ++s) xres[s] = 0.f;
    if constexpr (GBF && XBF) {
#pragma unroll
      for (int s = 0; s < U; ++s) {
        const uint16_t* xr = (const uint16_t*)a.X + ic[s] * d + g * KS;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          if (vec) {
            xbv[s][q] = *(const i16x8*)(xr + 8 * q);
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int k = g * KS + 8 * q + e;
              xbv[s][q][e] = (k < d) ? (short)xr[8 * q + e] : (short)0;
            }
          }
        }
      }
    } else if constexpr (XLO) {
#pragma unroll
      for (int s = 0; s < U; ++s) {
        float t[KS];
        load_chunk<KS, XBF>(a.X, ic[s], d, g * KS, vec, t);
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
      }
    } else {
      load_rows<U, KS, XBF>(a.X, ic, d, g * KS, vec, xv);
    }

    // Previous labels (changed-row count): for units of 4 or more blocks of
    // float32 rows they are loaded here, with the rows, so that the tile loop
    // hides their latency (4 registers; smaller units would lose an occupancy
    // step); otherwise at the start of the epilogue.
    // Without previous labels this pass's own label buffer is read instead
    // (the values are not used): no branch around the loads, which would
    // make the compiler wait for them before going on.
    constexpr bool kEarlyPrev = U >= 4 && !GBF;
    int pv[U];
    if constexpr (kEarlyPrev) {
      const int* pvsrc = prev != nullptr ? prev : rho;
#pragma unroll
      for (int s = 0; s < U; ++s) pv[s] = pvsrc[ic[s]];
    }
    float best[U], sec[U];
    int bidx[U];
#pragma unroll
    for (int s = 0; s < U; ++s) { best[s] = -__builtin_inff(); sec[s] = -__builtin_inff(); bidx[s] = 0; }

    for (int c0 = 0; c0 < Kpad; c0 += kchunk) {
      const int rows = (Kpad - c0) < kchunk ? (Kpad - c0) : kchunk;
      if (!resident) {
        __syncthreads();
        stage(StageLoop{}, c0, rows);
        __syncthreads();
      }
      // Tiles in pairs with two operand buffers: the loads of tile t + 1 are
      // issued (and pinned there by a scheduling barrier) before the MFMAs of
      // tile t.  The index of a load past the chunk's last tile is clamped to
      // a tile of the chunk; that operand is then not used.
      auto step = [&](const AO& op, int tt) {
        f32x4 acc[U];
        tile_mfma<KS, U, GBF, XLO, LB>(op, xv, xbv, xlv, acc);
        const int jb = c0 + tt;
#pragma unroll
        for (int s = 0; s < U; ++s) {
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
      };
      AO opa;
      if constexpr (kPairOps) {
        AO opb;
        load_aop<KS, GBF, LB>(Cs, Cbs, ncs, 0, g, r16, opa);
        for (int tt = 0; tt < rows; tt += 32) {
          load_aop<KS, GBF, LB>(Cs, Cbs, ncs, tt + 16 < rows ? tt + 16 : tt, g, r16, opb);
          __builtin_amdgcn_sched_barrier(0);
          step(opa, tt);
          if (tt + 16 >= rows) break;
          load_aop<KS, GBF, LB>(Cs, Cbs, ncs, tt + 32 < rows ? tt + 32 : tt + 16, g, r16, opa);
          __builtin_amdgcn_sched_barrier(0);
          step(opb, tt + 16);
        }
      } else {
        for (int tt = 0; tt < rows; tt += 16) {
          load_aop<KS, GBF, LB>(Cs, Cbs, ncs, tt, g, r16, opa);
          step(opa, tt);
        }
      }
    }

    // Epilogue: combine the 4 lane groups, flag near ties, exact energy terms.
    if constexpr (!kEarlyPrev) {   // all U blocks' previous labels together, used at the end
#pragma unroll
      for (int s = 0; s < U; ++s) pv[s] = prev != nullptr ? prev[ic[s]] : -1;
    }
    int bi_s[U];
    bool fl_s[U];
    double term_s[U];
    double l2_s[BND ? U : 1];   // squared lower bound of the distance to every other centroid
#pragma unroll
    for (int s = 0; s < U; ++s) {
      const int64_t i = ii[s];
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
        load_chunk<KS, XBF>(a.X, i < a.N ? i : 0, d, g * KS, vec, xe);
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
      // Re-check when the gap is within the bound, or so small that the row
      // could be a float64 near tie: a gap above bound/2 + 5.1e-7 (|x| +
      // max|c|)^2 leaves an exact squared-distance gap above 1.02e-6
      // (|x| + max|c|)^2, at least 1.02e-6 times the second distance, so
      // every near tie is among the re-checked rows (and counted there).
      const float nb2 = (nx + cb) * (nx + cb);
      const float thr = fmaxf(bound, 0.5f * bound + 5.1e-7f * nb2);
      const bool flag = valid && !((b - sc) > thr);
      // Lower bound for the row bounds: every other centroid j has exact score
      // s_j <= sc + e with e <= bound / 4, so its squared distance is at least
      // ||x||^2 - 2 sc - bound / 2; taken with a factor 2 of margin, and
      // ||x||^2 in float64 less 1e-12 of itself for its rounding.
      double l2 = 0.0;
      if constexpr (BND) {
        double x2 = 0.0;
#pragma unroll
        for (int q = 0; q < KS; ++q) x2 = fma((double)xe[q], (double)xe[q], x2);
        x2 += __shfl_xor(x2, 16, kWave);
        x2 += __shfl_xor(x2, 32, kWave);
        l2 = x2 * (1.0 - 1e-12) - 2.0 * (double)sc - (double)bound;
      }

      // exact energy term of the provisional label
      double term = row_dist2<KS>(xe, (resident && !GBF) ? Cs + bi * LD + g * KS : a.C + (int64_t)bi * d + g * KS,
                                  d, g, vec);

      unsigned long long fm = __ballot(flag) & 0xFFFFull;
      n_flag += (unsigned)__popcll(fm);
      bool listed = false;
      if constexpr (U == SB) listed = defer;   // lists exist in row-group mode only
      if (listed) {
        if (flag && g == 0) {
          const int pos = nfl + __popcll(fm & ((1ull << r16) - 1ull));
          const int64_t own = (bx + (int64_t)(pos / (16 * SB)) * gx) * group_rows + wave * (16 * SB) +
                              pos % (16 * SB);
          a.flags[own] = (int)i;
        }
        nfl += __popcll(fm);
      } else {
        // immediate: the row is spread over lanes r16 == f of the 4 lane groups
        while (fm) {
          const int f = __ffsll((long long)fm) - 1;
          fm &= fm - 1;
          if (r16 == f) {
#pragma unroll
            for (int q = 0; q < KS; ++q) xrow[g * KS + q] = xe[q];
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          double dist, dist2;
          const int j = exact_argmin_lds<DP>(xrow, Cs, LD, K, lane, &dist, &dist2);
          n_near += near_tie(dist, dist2) ? 1u : 0u;   // the same on every lane
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          if (j >= 0 && r16 == f) {
            bi = j;
            term = dist;
            if constexpr (BND) l2 = dist2 * (1.0 - 1e-12);
          }
        }
      }
      bi_s[s] = bi;
      term_s[s] = term;
      fl_s[s] = listed && flag;
      if constexpr (BND) l2_s[s] = listed ? 0.0 : l2;
    }

    // Changed labels of all blocks are counted before the first label
    // store: a previous label compared after a store inside a branch makes
    // the compiler wait for the outstanding stores (it cannot count them).
#pragma unroll
    for (int s = 0; s < U; ++s) {
      const bool mine = ii[s] < a.N && g == 0 && !fl_s[s];
      n_changed += (unsigned)__popcll(__ballot(mine && prev != nullptr && pv[s] != bi_s[s]));
    }
    double e_lane = 0.0;
#pragma unroll
    for (int s = 0; s < U; ++s) {
      const int64_t i = ii[s];
      const bool valid = i < a.N;
      const bool mine = valid && g == 0 && !fl_s[s];   // deferred rows are written later
      if (mine) {
        rho[i] = bi_s[s];
        if constexpr (BND) {
          if (lbo) lbo[i] = sqrt_down(l2_s[s]);
        }
      }
      if constexpr (BND) {   // listed rows get no bound (they are re-checked later)
        if (lbo && valid && g == 0 && fl_s[s]) lbo[i] = 0.f;
      }
      n_gemm += (unsigned)__popcll(__ballot(valid && g == 0));
      e_lane += mine ? term_s[s] : 0.0;
    }
    e_wave += wave_sum(e_lane);
  };

  // Bounds pass over blocks [b, b1) of this wave (row bounds in use): each
  // row's exact float64 distance d1 to the new centroid of its previous
  // label is compared with its bound lp = lb - (largest shift of another
  // centroid).  Every other centroid is then at least lp away, so if
  // d1 (1 + 2.1e-6) < lp^2 the previous label is the exact argmin, by a
  // relative margin wider than a near tie: the row keeps its label, its
  // energy term is d1 and its bound lp.  The other rows are queued in LDS
  // (in row order) and go through the distance GEMM in units of SB blocks,
  // the rest in single blocks.
  auto bounds_pass = [&](int64_t b, const int64_t b1) {
    if constexpr (BND) {
      int* q = (int*)(smem_raw + T::lds_bytes(K)) + wave * (32 * SB);
      int nq = 0;
      double e_skip = 0.0;
      auto wave_sync = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      };
      // drop the first `used` entries of the queue (fewer than 64 remain)
      auto consume = [&](int used) {
        const int rest = nq - used;
        wave_sync();
        const int v = lane < rest ? q[used + lane] : 0;
        wave_sync();
        if (lane < rest) q[lane] = v;
        wave_sync();
        nq = rest;
      };
      for (; b < b1; b += SB) {
        // rows past the range load row 0 (not used): no load behind a branch
        float xr[SB][KS];
        int ar[SB];
        float lr[SB];
        int64_t ir[SB], ic[SB];
#pragma unroll
        for (int s = 0; s < SB; ++s) {
          const int64_t i = (b + s) * 16 + r16;
          const bool valid = b + s < b1 && i < a.N;
          ir[s] = valid ? i : a.N;
          ic[s] = valid ? i : 0;
        }
        load_rows<SB, KS, XBF>(a.X, ic, d, g * KS, vec, xr);
#pragma unroll
        for (int s = 0; s < SB; ++s) {
          ar[s] = prev[ic[s]];
          lr[s] = lbi[ic[s]];
        }
#pragma unroll
        for (int s = 0; s < SB; ++s) {
          const bool valid = ir[s] < a.N;
          const int la = (ar[s] >= 0 && ar[s] < K) ? ar[s] : 0;
          const double d1 = row_dist2<KS>(xr[s], Cs + la * LD + g * KS, d, g, vec);
          const double lp = (double)lr[s] - (la == sj1 ? sm2 : sm1);
          const bool skip = valid && lp > 0.0 && d1 * (1.0 + 2.1e-6) < lp * lp * (1.0 - 1e-9);
          if (skip && g == 0) {
            rho[ir[s]] = la;
            lbo[ir[s]] = f32_down(lp * (1.0 - 1e-15));
            e_skip += d1;
          }
          const bool act = valid && !skip && g == 0;
          const unsigned long long am = __ballot(act);
          if (act) q[nq + __popcll(am & ((1ull << r16) - 1ull))] = (int)ir[s];
          nq += (int)__popcll(am);
        }
        wave_sync();
        if (nq >= 16 * SB) {
          unit(std::integral_constant<int, SB>{}, 0, q, 16 * SB);
          consume(16 * SB);
        }
      }
      while (nq > 0) {
        const int c = nq < 16 ? nq : 16;
        unit(std::integral_constant<int, 1>{}, 0, q, c);
        consume(c);
      }
      e_wave += wave_sum(e_skip);
    }
  };

  int nb = 0;   // row-group boundaries passed (selects the wc buffer)
  bool balanced = false;
  if constexpr (!GBF) balanced = resident;   // then defer is false: no lists, no barriers
  if (balanced) {
    // Float32 centroids resident in LDS: the waves are independent, so the
    // 16-sample blocks are split evenly over every wave of the launch (wave
    // gw takes blocks [gw B / GW, (gw + 1) B / GW)), in units of SB blocks
    // and single blocks for the rest.  With row groups a grid apart the last
    // round would run on a fraction of the waves (at N = 1e6 and 768
    // workgroups of 256 rows: 5.09 rounds of work take 6).
    const int64_t nblk = (a.N + 15) / 16;
    const int64_t GW = (int64_t)gx * W, gw = (int64_t)bx * W + wave;
    const int64_t b1 = (gw + 1) * nblk / GW;
    int64_t b = gw * nblk / GW;
    bool filtered = false;
    if constexpr (BND) {
      if (use_in) {
        bounds_pass(b, b1);
        filtered = true;
      }
    }
    if (!filtered) {
      for (; b + SB <= b1; b += SB) unit(std::integral_constant<int, SB>{}, b * 16, nullptr, 0);
      if constexpr (SB > 1)
        for (; b < b1; ++b) unit(std::integral_constant<int, 1>{}, b * 16, nullptr, 0);
    }
  } else {
    for (int64_t grp = bx; grp < groups; grp += gx) {
      unit(std::integral_constant<int, SB>{}, grp * group_rows + (int64_t)wave * (16 * SB), nullptr, 0);
      // With streamed centroids the chunk area is free here: re-check full
      // batches now, so that the re-check overlaps other workgroups' MFMA work
      // instead of piling up after the last row group (bf16 GEMM kernels; in
      // the float32 kernels the extra live registers of this call would spill).
      if (kInterleave && defer && !resident && !a.fl_cnt) {
        int* wc = wcnt + (nb & 1) * 16;   // two buffers: a slow wave may still read the previous one
        if (lane == 0) wc[wave] = nfl;
        __syncthreads();
        recheck_batches(wc, false);
        ++nb;
      }
    }
  }

  if (a.fl_cnt) {   // list mode: the rows stay listed for k_recheck
    if (lane == 0) a.fl_cnt[bx * 16 + wave] = defer ? nfl : 0;
  } else if (defer) {   // the remaining listed rows
    int* wc = wcnt + (nb & 1) * 16;
    if (lane == 0) wc[wave] = nfl;
    __syncthreads();
    recheck_batches(wc, true);
  }

  if (lane == 0) {
    dred[wave] = e_wave;
    if (n_changed) atomicAdd(&ctl->cnt_changed[slot], (unsigned long long)n_changed);
    if (n_flag) atomicAdd(&ctl->cnt_flagged[slot], (unsigned long long)n_flag);
    if (n_near) atomicAdd(&ctl->cnt_near[slot], (unsigned long long)n_near);
    if (n_gemm) atomicAdd(&ctl->cnt_gemm[slot], (unsigned long long)n_gemm);
  }
  __syncthreads();
  if (tid == 0) {
    double e = dred[0];
#pragma unroll
    for (int w = 1; w < W; ++w) e += dred[w];
    a.e_part[bx] = e + e_def;
  }
}

template <int KS, int SB, int W, bool XBF, bool GBF, int LB>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(assign_wpe<KS, SB, W, XBF, GBF>())))
void k_assign(AssignArgs a) {
  assign_body<KS, SB, W, XBF, GBF, LB>(a, blockIdx.x, gridDim.x);
}

// Single instance with row bounds (float32 GEMM; the bounds are used when the
// centroids are resident in LDS, which the host ensures).
template <int KS, int SB, int W, bool XBF, bool GBF, int LB>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(assign_wpe<KS, SB, W, XBF, GBF>())))
void k_assign_bnd(AssignArgs a) {
  assign_body<KS, SB, W, XBF, GBF, LB, true>(a, blockIdx.x, gridDim.x);
}

// Batched launch: the grid is the concatenation of every instance's slice.
template <int KS, int SB, int W, bool XBF, bool GBF, int LB>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(assign_wpe<KS, SB, W, XBF, GBF>())))
void k_assign_batch(BatchRef<AssignArgs> t) {
  const int b = batch_find(t.prefix, t.n, blockIdx.x);
  const int b0 = t.prefix[b];
  if constexpr (GBF && XBF && KS >= 16) {
    // a copy of the instance's arguments: read through the table pointer,
    // fields are loaded again after stores to global memory (the stores
    // could alias the table); the other kernels keep the reference, where
    // the copy's registers would cost an occupancy step or spill
    const AssignArgs a = t.tab[b];
    assign_body<KS, SB, W, XBF, GBF, LB>(a, blockIdx.x - b0, t.prefix[b + 1] - b0);
  } else {
    assign_body<KS, SB, W, XBF, GBF, LB>(t.tab[b], blockIdx.x - b0, t.prefix[b + 1] - b0);
  }
}

// Host view of one kernel instantiation.
struct KernelPick {
  const void* fn = nullptr;        // k_assign
  const void* fn_batch = nullptr;  // k_assign_batch
  const void* fn_bnd = nullptr;    // k_assign_bnd (float32 GEMM only)
  bool resident = false;           // the K centroids fit the LDS budget at once
  size_t lds_bnd = 0;              // LDS bytes of k_assign_bnd (lds + the row queues)
  int rows = 0;                    // samples per row group (16 * SB * W)
  int threads = 0;                 // 64 * W
  int lb = 0;                      // LDS budget (bytes)
  size_t lds = 0;                  // LDS bytes for the K of the call
};

template <int KS, bool XBF, bool GBF, int SB, int W, int LB>
KernelPick make_pick(int K) {
  KernelPick p;
  p.fn = (const void*)&k_assign<KS, SB, W, XBF, GBF, LB>;
  p.fn_batch = (const void*)&k_assign_batch<KS, SB, W, XBF, GBF, LB>;
  p.rows = 16 * SB * W;
  p.threads = 64 * W;
  p.lb = LB;
  p.lds = Tile<KS, GBF, LB>::lds_bytes(K);
  p.resident = Tile<KS, GBF, LB>::chunk_rows(K) >= ((K + 15) & ~15);
  if constexpr (!GBF) {
    p.fn_bnd = (const void*)&k_assign_bnd<KS, SB, W, XBF, GBF, LB>;
    p.lds_bnd = p.lds + (size_t)W * 32 * SB * 4;
  }
  return p;
}

// Padded dimensions per lane group for d (-1 beyond the supported range).
inline int pick_ks(int d, int gemm_bf16) {
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

// Kernel of the given tile shape (0 = default; see the per-family tables).
KernelPick pick_f32(int ks, bool xbf, int K, int shape);
KernelPick pick_bf16(int ks, bool xbf, int K, int shape);

}  // namespace km
