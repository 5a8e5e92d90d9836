// Float32 distance-GEMM instantiations of the assignment kernel for
// bfloat16-stored rows: km_assign_f32.hip compiled with KM_F32_XBF.
#define KM_F32_XBF 1
#include "km_assign_f32.hip"
