// Launches across shapes, double: row forward passes.
#include "firls_inst.h"
#include "firls_multi.h"
namespace firls {
template <int M>
hipError_t LM_rowfwd_f64(const MultiArgs& A, int items, size_t lds, hipStream_t st) {
  return launch_multi_kernel(km_rowfwd<double, M>, A, items, lds, st);
}
void fill_multi_f64_row(MultiKernels& k) {
  const size_t most = lds_bytes<double, 512>();
#define FIRLS_MODE(M)                                  \
  allow_multi_lds(km_rowfwd<double, M>, most);          \
  k.fn[MC_ROWFWD][M] = LM_rowfwd_f64<M>;
  FIRLS_MODE(RF_PLAIN) FIRLS_MODE(RF_PCG_HAAR) FIRLS_MODE(RF_PCG_Z) FIRLS_MODE(RF_STEP_HAAR)
  FIRLS_MODE(RF_SQ_HAAR) FIRLS_MODE(RF_SQW_HAAR)
#undef FIRLS_MODE
}
}  // namespace firls
