// Workspace of one solve: the device buffers of Algorithm 1 for one
// instance, carved out of a single allocation.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "km_launch.h"

namespace km {

constexpr size_t kWsAlign = 256;
inline size_t ws_up(size_t v) { return (v + kWsAlign - 1) & ~(kWsAlign - 1); }

// Sizes that determine the workspace layout.
struct Shape {
  int64_t N = 0;
  int d = 0, K = 0, cap = 0, bf = 0;
  int it = 0;   // entries of the m trajectory (max_iter + 1 when requested)
  int bnd = 0;  // row bounds kept (3 x N lower bounds and the reference centroids)
  bool fits(const Shape& o) const {
    return N >= o.N && d >= o.d && K >= o.K && cap >= o.cap && bf >= o.bf && it >= o.it && bnd >= o.bnd &&
           (int64_t)K * d >= (int64_t)o.K * o.d;
  }
};

struct Ws {
  Ctl* ctl = nullptr;
  int* labels = nullptr;        // 3 x N
  int* lrank = nullptr;         // N
  int* perm = nullptr;          // N
  int* flags = nullptr;         // N (flagged rows of an assignment pass)
  int* blockcount = nullptr;    // nblk x K
  int* counts = nullptr;        // K
  int* seg_start = nullptr;     // K + 1
  int* item_start = nullptr;    // K + 1
  int* item_cluster = nullptr;  // max_items
  double* e_part = nullptr;     // 2 x (N / 64 + 1 + kReGrid): partials of the candidate and fall-back
                                //   passes (assignment workgroups, then the re-check's)
  int* fl_cnt = nullptr;        // kReMaxGrid x 16 list lengths of a list-mode assignment launch
  double* partial = nullptr;    // max_items x d
  unsigned* xbound = nullptr;   // kXBoundSlots + 1 (fixed-point update: maxima, then e)
  unsigned long long* fxpart = nullptr;  // fx_part_entries(N, K, d)
  double* G_last = nullptr;     // K x d
  double* F_last = nullptr;     // K x d
  double* ring_dF = nullptr;    // cap x K x d
  double* ring_dG = nullptr;    // cap x K x d
  double* gram = nullptr;       // cap x cap
  double* dots = nullptr;       // fin_grid x 2 cap
  double* e_out = nullptr;      // 1
  float* C_cand = nullptr;      // K x d
  float* C_fb = nullptr;        // K x d
  float* C_tmp = nullptr;       // K x d (kmeans_g / prologue input copy)
  float* nc_cand = nullptr;
  float* nc_fb = nullptr;
  float* nc_tmp = nullptr;
  uint16_t* Cb_cand = nullptr;  // bf16 hi/lo pairs, 2 x K x d (bf16 GEMM only)
  uint16_t* Cb_fb = nullptr;
  uint16_t* Cb_tmp = nullptr;
  float* del_cand = nullptr;
  float* del_fb = nullptr;
  float* del_tmp = nullptr;
  int* m_traj = nullptr;        // it ints (m after the dynamic-m rule per iteration)
  float* lb = nullptr;          // 3 x N row bounds (bnd only)
  float* C_ref = nullptr;       // K x d reference centroids of the row bounds (bnd only)
  double* shift = nullptr;      // 2 x K centroid shifts against C_ref: candidate, fall-back (bnd only)
  int max_items = 0, nblk = 0, fin_grid = 0;
};

// Bytes of the workspace for s; with base != null also fills w.
inline size_t ws_layout(const Shape& s, char* base, Ws* w) {
  const int64_t N = s.N;
  const int64_t KD = (int64_t)s.K * s.d;
  const int64_t grid = N / 64 + 1;   // upper bound of an assignment grid
  const int max_items = update_max_items(N, s.K);
  const int nblk = update_rank_blocks(N, s.K);
  const int fin_grid = finalize_grid_cap(KD);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += ws_up(bytes); return o; };
  const size_t o_ctl = take(sizeof(Ctl));
  const size_t o_lab = take(3 * N * 4);
  const size_t o_lr = take(N * 4);
  const size_t o_perm = take(N * 4);
  const size_t o_flags = take(N * 4);
  const size_t o_bc = take(update_blockcount_ints(N, s.K) * 4);
  const size_t o_cnt = take((size_t)s.K * 4);
  const size_t o_ss = take((size_t)(s.K + 1) * 4);
  const size_t o_is = take((size_t)(s.K + 1) * 4);
  const size_t o_ic = take((size_t)max_items * 4);
  const size_t o_ep = take((size_t)2 * (grid + kReGrid) * 8);
  const size_t o_fc = take((size_t)kReMaxGrid * 16 * 4);
  const size_t o_pa = take((size_t)max_items * s.d * 8);
  const size_t o_xb = take((size_t)(kXBoundSlots + 1) * 4);
  const size_t o_fx = take((size_t)fx_part_entries(N, s.K, s.d) * 8);
  const size_t o_gl = take(KD * 8);
  const size_t o_fl = take(KD * 8);
  const size_t o_rf = take((size_t)s.cap * KD * 8);
  const size_t o_rg = take((size_t)s.cap * KD * 8);
  const size_t o_gr = take((size_t)s.cap * s.cap * 8 + 8);
  const size_t o_dt = take((size_t)fin_grid * 2 * s.cap * 8 + 8);
  const size_t o_eo = take(8);
  const size_t o_cc = take(KD * 4);
  const size_t o_cf = take(KD * 4);
  const size_t o_ct = take(KD * 4);
  const size_t o_nc = take((size_t)s.K * 4);
  const size_t o_nf = take((size_t)s.K * 4);
  const size_t o_nt = take((size_t)s.K * 4);
  const size_t o_bcand = take(s.bf ? KD * 4 : 0);
  const size_t o_bfb = take(s.bf ? KD * 4 : 0);
  const size_t o_btmp = take(s.bf ? KD * 4 : 0);
  const size_t o_dc = take(s.bf ? s.K * 4 : 0);
  const size_t o_df = take(s.bf ? s.K * 4 : 0);
  const size_t o_dtmp = take(s.bf ? s.K * 4 : 0);
  const size_t o_mt = take((size_t)s.it * 4);
  const size_t o_lb = take(s.bnd ? (size_t)3 * N * 4 : 0);
  const size_t o_cr = take(s.bnd ? (size_t)KD * 4 : 0);
  const size_t o_sh = take(s.bnd ? (size_t)2 * s.K * 8 : 0);
  if (base && w) {
    char* b = base;
    w->ctl = (Ctl*)(b + o_ctl);
    w->labels = (int*)(b + o_lab);
    w->lrank = (int*)(b + o_lr);
    w->perm = (int*)(b + o_perm);
    w->flags = (int*)(b + o_flags);
    w->blockcount = (int*)(b + o_bc);
    w->counts = (int*)(b + o_cnt);
    w->seg_start = (int*)(b + o_ss);
    w->item_start = (int*)(b + o_is);
    w->item_cluster = (int*)(b + o_ic);
    w->e_part = (double*)(b + o_ep);
    w->fl_cnt = (int*)(b + o_fc);
    w->partial = (double*)(b + o_pa);
    w->xbound = (unsigned*)(b + o_xb);
    w->fxpart = (unsigned long long*)(b + o_fx);
    w->G_last = (double*)(b + o_gl);
    w->F_last = (double*)(b + o_fl);
    w->ring_dF = (double*)(b + o_rf);
    w->ring_dG = (double*)(b + o_rg);
    w->gram = (double*)(b + o_gr);
    w->dots = (double*)(b + o_dt);
    w->e_out = (double*)(b + o_eo);
    w->C_cand = (float*)(b + o_cc);
    w->C_fb = (float*)(b + o_cf);
    w->C_tmp = (float*)(b + o_ct);
    w->nc_cand = (float*)(b + o_nc);
    w->nc_fb = (float*)(b + o_nf);
    w->nc_tmp = (float*)(b + o_nt);
    w->Cb_cand = s.bf ? (uint16_t*)(b + o_bcand) : nullptr;
    w->Cb_fb = s.bf ? (uint16_t*)(b + o_bfb) : nullptr;
    w->Cb_tmp = s.bf ? (uint16_t*)(b + o_btmp) : nullptr;
    w->del_cand = s.bf ? (float*)(b + o_dc) : nullptr;
    w->del_fb = s.bf ? (float*)(b + o_df) : nullptr;
    w->del_tmp = s.bf ? (float*)(b + o_dtmp) : nullptr;
    w->m_traj = s.it ? (int*)(b + o_mt) : nullptr;
    w->lb = s.bnd ? (float*)(b + o_lb) : nullptr;
    w->C_ref = s.bnd ? (float*)(b + o_cr) : nullptr;
    w->shift = s.bnd ? (double*)(b + o_sh) : nullptr;
    w->max_items = max_items;
    w->nblk = nblk;
    w->fin_grid = fin_grid;
  }
  return off;
}

}  // namespace km

namespace km {

// Buffers of one stand-alone G application (kmeans_g): the control block,
// the prepared centroids, the energy partials of `grid` workgroups, the
// flagged-row lists and the update's scratch for the path (K, d) takes.  No
// solver state.  Bytes for the shape; with base != null also fills the G
// fields of w (the rest stay null).
inline size_t ws_layout_g(int64_t N, int d, int K, int bf, int grid, char* base, Ws* w) {
  const int64_t KD = (int64_t)K * d;
  const bool fx = fx_ok(K, d);
  const int max_items = fx ? 0 : update_max_items(N, K);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += ws_up(bytes); return o; };
  const size_t o_ctl = take(sizeof(Ctl));
  const size_t o_nc = take((size_t)K * 4);
  const size_t o_cb = take(bf ? (size_t)KD * 4 : 0);
  const size_t o_del = take(bf ? (size_t)K * 4 : 0);
  const size_t o_ep = take((size_t)(grid + kReGrid) * 8);
  const size_t o_fc = take((size_t)kReMaxGrid * 16 * 4);
  const size_t o_eo = take(8);
  const size_t o_flags = take((size_t)N * 4);
  const size_t o_xb = take(fx ? (size_t)(kXBoundSlots + 1) * 4 : 0);
  const size_t o_fx = take(fx ? (size_t)fx_part_entries(N, K, d) * 8 : 0);
  const size_t o_lr = take(fx ? 0 : (size_t)N * 4);
  const size_t o_perm = take(fx ? 0 : (size_t)N * 4);
  const size_t o_bc = take(fx ? 0 : update_blockcount_ints(N, K) * 4);
  const size_t o_cnt = take(fx ? 0 : (size_t)K * 4);
  const size_t o_ss = take(fx ? 0 : (size_t)(K + 1) * 4);
  const size_t o_is = take(fx ? 0 : (size_t)(K + 1) * 4);
  const size_t o_ic = take((size_t)max_items * 4);
  const size_t o_pa = take((size_t)max_items * d * 8);
  if (base && w) {
    char* b = base;
    *w = Ws();
    w->ctl = (Ctl*)(b + o_ctl);
    w->nc_tmp = (float*)(b + o_nc);
    w->Cb_tmp = bf ? (uint16_t*)(b + o_cb) : nullptr;
    w->del_tmp = bf ? (float*)(b + o_del) : nullptr;
    w->e_part = (double*)(b + o_ep);
    w->fl_cnt = (int*)(b + o_fc);
    w->e_out = (double*)(b + o_eo);
    w->flags = (int*)(b + o_flags);
    w->xbound = fx ? (unsigned*)(b + o_xb) : nullptr;
    w->fxpart = fx ? (unsigned long long*)(b + o_fx) : nullptr;
    w->lrank = fx ? nullptr : (int*)(b + o_lr);
    w->perm = fx ? nullptr : (int*)(b + o_perm);
    w->blockcount = fx ? nullptr : (int*)(b + o_bc);
    w->counts = fx ? nullptr : (int*)(b + o_cnt);
    w->seg_start = fx ? nullptr : (int*)(b + o_ss);
    w->item_start = fx ? nullptr : (int*)(b + o_is);
    w->item_cluster = fx ? nullptr : (int*)(b + o_ic);
    w->partial = fx ? nullptr : (double*)(b + o_pa);
    w->max_items = max_items;
  }
  return off;
}

}  // namespace km
