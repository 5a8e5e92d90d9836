// bfloat16 distance-GEMM instantiations of the assignment kernel.
//
// Tile shapes for bfloat16 rows up to 32 dims per lane group (SB 16-sample
// blocks per wave, W waves, LDS budget):
//   0  SB = 4, W = 8, 144 KB  (default: one workgroup per CU, few chunks)
//   1  SB = 2, W = 8, 72 KB
//   2  SB = 4, W = 4, 72 KB   (two workgroups per CU)
//   3  SB = 8, W = 4, 144 KB
// Each 16x16x32 MFMA reads a 1 KB A operand (hi or lo) from LDS and reuses
// it for SB sample blocks; at SB = 2 the LDS port would have to deliver
// 128 B/clk per CU at full MFMA rate, SB >= 4 halves that.
// Wider rows, and float32 rows (which carry hi and lo operands), use 4-wave
// workgroups with 60 KB: shape 0 SB = 1, any other SB = 2.

#include "km_assign_kernel.h"

namespace km {

template <int KS, bool XBF>
static KernelPick bf16_shape(int K, int shape) {
  if constexpr (XBF && KS <= 32) {
    switch (shape) {
      case 1: return make_pick<KS, XBF, true, 2, 8, 72 * 1024>(K);
      case 2: return make_pick<KS, XBF, true, 4, 4, 72 * 1024>(K);
      case 3: return make_pick<KS, XBF, true, 8, 4, 144 * 1024>(K);
      default: return make_pick<KS, XBF, true, 4, 8, 144 * 1024>(K);
    }
  } else {
    if (shape != 0) return make_pick<KS, XBF, true, 2, 4, 60 * 1024>(K);
    return make_pick<KS, XBF, true, 1, 4, 60 * 1024>(K);
  }
}

template <bool XBF>
static KernelPick bf16_ks(int ks, int K, int shape) {
  switch (ks) {
    case 8: return bf16_shape<8, XBF>(K, shape);
    case 16: return bf16_shape<16, XBF>(K, shape);
    case 24: return bf16_shape<24, XBF>(K, shape);
    case 32: return bf16_shape<32, XBF>(K, shape);
    case 48: return bf16_shape<48, XBF>(K, shape);
    case 64: return bf16_shape<64, XBF>(K, shape);
  }
  return KernelPick();
}

KernelPick pick_bf16(int ks, bool xbf, int K, int shape) {
  return xbf ? bf16_ks<true>(ks, K, shape) : bf16_ks<false>(ks, K, shape);
}

}  // namespace km
