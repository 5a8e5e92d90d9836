// Float32 distance-GEMM instantiations of the assignment kernel.
//
// Tile shapes (SB 16-sample blocks per wave, W waves, LDS budget):
//   0  SB = 2 (1 beyond 32 dims per lane group), W = 4, 60 KB  (default)
//   1  SB = 1, W = 4, 60 KB
//   2  default SB, W = 8, 60 KB
//   3  SB = 4, W = 4, 60 KB (up to 8 dims per lane group; else the default)
// The autotuner picks the shape per (width, K bucket) from measured times
// (tiles_gfx950.json); at N = 1e6, d = 32, K = 256 it picks shape 3.
// float32 rows are instantiated here, bfloat16-stored rows in
// km_assign_f32x.hip (the same source with KM_F32_XBF), so that the two
// halves compile in parallel.

#include "km_assign_kernel.h"

namespace km {

template <int KS, bool XBF>
static KernelPick f32_shape(int K, int shape) {
  constexpr int SB0 = KS <= 32 ? 2 : 1;
  constexpr int L = 60 * 1024;
  switch (shape) {
    case 1: return make_pick<KS, XBF, false, 1, 4, L>(K);
    case 2: return make_pick<KS, XBF, false, SB0, 8, L>(K);
    case 3:
      if constexpr (KS <= 8) return make_pick<KS, XBF, false, 4, 4, L>(K);
      else return make_pick<KS, XBF, false, SB0, 4, L>(K);
    default: return make_pick<KS, XBF, false, SB0, 4, L>(K);
  }
}

template <bool XBF>
static KernelPick f32_ks(int ks, int K, int shape) {
  switch (ks) {
    case 1: return f32_shape<1, XBF>(K, shape);
    case 2: return f32_shape<2, XBF>(K, shape);
    case 4: return f32_shape<4, XBF>(K, shape);
    case 8: return f32_shape<8, XBF>(K, shape);
    case 12: return f32_shape<12, XBF>(K, shape);
    case 16: return f32_shape<16, XBF>(K, shape);
    case 24: return f32_shape<24, XBF>(K, shape);
    case 32: return f32_shape<32, XBF>(K, shape);
    case 48: return f32_shape<48, XBF>(K, shape);
    case 64: return f32_shape<64, XBF>(K, shape);
  }
  return KernelPick();
}

#ifdef KM_F32_XBF
// bfloat16-stored rows (compiled as km_assign_f32x.hip)
KernelPick pick_f32_xbf(int ks, int K, int shape) { return f32_ks<true>(ks, K, shape); }
#else
KernelPick pick_f32_xbf(int ks, int K, int shape);
KernelPick pick_f32(int ks, bool xbf, int K, int shape) {
  return xbf ? pick_f32_xbf(ks, K, shape) : f32_ks<false>(ks, K, shape);
}
#endif

}  // namespace km
