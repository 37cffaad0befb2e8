// Launches across shapes, float: column passes and row inverse passes.
#include "firls_inst.h"
#include "firls_multi.h"
namespace firls {
template <int M>
hipError_t LM_col_f32(const MultiArgs& A, int items, size_t lds, hipStream_t st) {
  return launch_multi_kernel(km_col<float, M>, A, items, lds, st);
}
template <int M>
hipError_t LM_rowinv_f32(const MultiArgs& A, int items, size_t lds, hipStream_t st) {
  return launch_multi_kernel(km_rowinv<float, M>, A, items, lds, st);
}
void fill_multi_f32_col(MultiKernels& k) {
  const size_t most_c = lds_col_bytes<float, 512>(), most_r = lds_bytes<float, 512>();
#define FIRLS_COL(M)                                   \
  allow_multi_lds(km_col<float, M>, most_c);           \
  k.fn[MC_COL][M] = LM_col_f32<M>;
#define FIRLS_INV(M)                                   \
  allow_multi_lds(km_rowinv<float, M>, most_r);        \
  k.fn[MC_ROWINV][M] = LM_rowinv_f32<M>;
  FIRLS_COL(COL_SP) FIRLS_COL(COL_R0) FIRLS_COL(COL_SP_PQ)
  FIRLS_INV(RI_SP_HAAR) FIRLS_INV(RI_SP_TV) FIRLS_INV(RI_R0_HAAR) FIRLS_INV(RI_R0_TV) FIRLS_INV(RI_R0_HAAR_P0)
#undef FIRLS_COL
#undef FIRLS_INV
}
}  // namespace firls
