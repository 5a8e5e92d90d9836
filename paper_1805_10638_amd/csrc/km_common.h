// Shared device-side definitions of libkmaa (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace km {

constexpr int kWave = 64;
constexpr int kMaxK = 4096;          // labels per LDS histogram row in the rank kernel
constexpr int kMaxD = 256;           // register-resident sample rows in the assignment
constexpr int kMaxM = 64;            // Anderson history bound
// Rows per block of the counting sort: 4096 for more than 512 clusters (each
// block clears and writes a K-entry histogram, so large K wants fewer blocks)
// or at least 4M rows (longer runs of consecutive permutation entries per
// cluster, so the scatter's stores coalesce), else 1024 (enough blocks to
// fill the device).
constexpr int kRankRowsSmall = 1024;
constexpr int kRankRowsLarge = 4096;
constexpr int kRankSplitK = 512;
constexpr int64_t kRankSplitN = 4 << 20;
__host__ __device__ inline int rank_rows(int64_t N, int K) {
  return (K > kRankSplitK || N >= kRankSplitN) ? kRankRowsLarge : kRankRowsSmall;
}
__host__ __device__ inline int update_rank_blocks(int64_t N, int K) {
  const int rr = rank_rows(N, K);
  return (int)((N + rr - 1) / rr);
}
constexpr int kSegRows = 512;        // rows per work item of the segmented sum
constexpr int kTraceRec = 80;        // doubles per trace record

// Fixed-point update: the cluster sums and sizes of a contiguous row range
// are int64 accumulators in LDS (integer addition is associative, so the
// result does not depend on the order of the LDS atomics).  A cluster's sums
// take fx_stride(d) entries: an odd stride puts the rows of different
// clusters on different banks.  Used when K * fx_stride(d) + K entries fit in
// kFxMaxL (80 KB); larger K*d takes the counting sort.
constexpr int kFxThreads = 1024;
constexpr int kFxMaxL = 10240;
constexpr int kFxMaxBlocks = 256;    // one workgroup per compute unit (fewer partials to add)
constexpr int kFxMinRows = 4096;     // rows per workgroup before the grid grows
constexpr int kXBoundSlots = 1024;   // per-workgroup maxima of |x| (one per thread of a fixed-point workgroup)
__host__ __device__ inline int fx_stride(int d) { return d | 1; }
__host__ __device__ inline bool fx_ok(int K, int d) { return (int64_t)K * fx_stride(d) + K <= kFxMaxL; }
__host__ __device__ inline int fx_blocks(int64_t N) {
  const int64_t p = N / kFxMinRows;
  return p < 1 ? 1 : (p > kFxMaxBlocks ? kFxMaxBlocks : (int)p);
}
// int64 entries of the per-workgroup partials a workspace for (N, K, d) holds
// (enough for any shape it fits: fewer rows, clusters or K*d)
__host__ __device__ inline int64_t fx_part_entries(int64_t N, int K, int d) {
  const int64_t L = (int64_t)K * d + K;
  return (int64_t)fx_blocks(N) * (L < kFxMaxL ? L : kFxMaxL);
}

// Roles of an assignment launch.
enum Role : int {
  kRolePlain = 0,      // stand-alone G(C): explicit label pointers, no gating
  kRoleCand = 1,       // candidate C^t of an iteration
  kRoleFallback = 2,   // Lloyd fall-back iterate, runs only when ctl->reject
};

// Decision codes written to trace records.
enum Decision : int {
  kDecLloyd = 0, kDecAccepted = 1, kDecRejected = 2, kDecConverged = 3,
  kDecTol = 4, kDecMaxIter = 5,
};

// Solver state, resident in device memory for the whole solve.  Written only
// by the single-workgroup controller kernels (and counters by atomics).
struct Ctl {
  int32_t t;               // current iteration (0 during the prologue)
  int32_t done;            // 1 once the solve has finished
  int32_t status;          // km_status at finish
  int32_t m;               // current m of the dynamic rule
  int32_t cand_is_lloyd;   // candidate C^t equals the Lloyd iterate
  int32_t reject;          // candidate of this iteration rejected
  int32_t lab_prev;        // label buffer (0..2) of the accepted P^{t-1}
  int32_t lab_cand;        // label buffer of the candidate's assignment
  int32_t lab_fb;          // label buffer of the fall-back assignment
  int32_t acc_src;         // accepted centroids: 0 candidate buffer, 1 fall-back buffer
  int32_t mt;              // m_t used this iteration
  int32_t used;            // columns that entered the least squares
  int32_t accepted, rejected, assign_passes, max_iter;
  int32_t m_max, flags;
  int32_t total_items;     // work items of the segmented sum
  int32_t empty;           // empty clusters of the last update
  double eps1, eps2, tol, ridge;
  double E1, E2;           // accepted energies E^{t-1}, E^{t-2}
  double E_cand, E_fb, E_acc;
  unsigned long long cnt_changed[2];   // [candidate/plain, fall-back]
  unsigned long long cnt_flagged[2];   // rows re-checked in float64
  unsigned long long flagged_total;
  unsigned long long cnt_near[2];      // re-checked rows that are float64 near ties
  unsigned long long near_total;
  unsigned long long cnt_gemm[2];      // rows that went through the distance GEMM (not skipped by bounds)
  unsigned long long gemm_total;
  double theta[kMaxM];
};

// ---------------------------------------------------------------------------
// Wave helpers (fixed reduction order, hence deterministic)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, kWave));
  return v;
}

// Drop a pending error of an unrelated earlier runtime call so that the
// check after a launch reports that launch only.
// bfloat16 pair for the distance GEMM: hi = rne(f), lo = rne(f - hi) (the
// difference is exact in float32).  Returns the residual f - hi - lo, exact in
// float64; |residual| <= 2^-16 |f| for normal values.
__device__ __forceinline__ uint16_t bf16_rne_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ double bf16_split(float f, uint16_t* hi, uint16_t* lo) {
  const uint16_t h = bf16_rne_bits(f);
  const float fh = __uint_as_float(((uint32_t)h) << 16);
  const float r1 = f - fh;
  const uint16_t l = bf16_rne_bits(r1);
  *hi = h;
  *lo = l;
  return (double)r1 - (double)__uint_as_float(((uint32_t)l) << 16);
}

// Batched launches: the grid is the concatenation of per-instance slices;
// workgroup bx belongs to instance b with prefix[b] <= bx < prefix[b + 1]
// (prefix has n + 1 entries; empty slices are skipped by the search).
template <class A>
struct BatchRef {
  const A* tab;
  const int* prefix;
  int n;
};

__device__ __forceinline__ int batch_find(const int* prefix, int n, int bx) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= bx) lo = mid; else hi = mid;
  }
  return lo;
}

inline void clear_pending_error() { (void)hipGetLastError(); }

__device__ __forceinline__ unsigned popc64(unsigned long long m) { return __popcll(m); }

}  // namespace km
