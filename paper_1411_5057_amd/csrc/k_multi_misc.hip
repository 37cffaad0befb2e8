// Launches across shapes: the paired PCG pass, the Haar update
// kernels of the textbook PCG order, the TV and group kernels and the outer
// check (both precisions), and the LDS sizes of every class.
#include "firls_inst.h"
#include "firls_multi.h"
namespace firls {

template <typename T>
hipError_t LM_pair(const MultiArgs& A, int items, size_t lds, hipStream_t st) {
  return launch_multi_kernel(km_pair<T>, A, items, lds, st);
}
template <typename T>
hipError_t LM_pair_wide(const MultiArgs& A, int items, size_t lds, hipStream_t st) {
  return launch_multi_kernel(km_pair_wide<T>, A, items, lds, st);
}
template <typename T, int CLS>
hipError_t LM_haar(const MultiArgs& A, int items, size_t lds, hipStream_t st) {
  return launch_multi_kernel(km_haar<T, CLS>, A, items, lds, st);
}
template <typename T, int CLS, int MODE>
hipError_t LM_prec(const MultiArgs& A, int items, size_t lds, hipStream_t st) {
  return launch_multi_kernel(km_prec<T, CLS, MODE>, A, items, lds, st);
}

template <typename T>
void fill_multi_misc(MultiKernels& k) {
  allow_multi_lds(km_pair<T>, lds_bytes<T, 256>());
  k.fn[MC_PAIR][0] = LM_pair<T>;
  if constexpr (sizeof(T) == 4) {
    allow_multi_lds(km_pair_wide<T>, lds_bytes<T, 512>());
    k.fn[MC_PAIR][1] = LM_pair_wide<T>;
  }
  k.fn[MC_PSI_SQ_HAAR][0] = LM_haar<T, MC_PSI_SQ_HAAR>;
  k.fn[MC_UPDATE_HAAR][0] = LM_haar<T, MC_UPDATE_HAAR>;
  k.fn[MC_LAST_X][0] = LM_haar<T, MC_LAST_X>;
  k.fn[MC_PSI_SQ_TV][0] = LM_prec<T, MC_PSI_SQ_TV, 0>;
  k.fn[MC_GROUP_W][0] = LM_prec<T, MC_GROUP_W, 0>;
  k.fn[MC_GROUP_D][0] = LM_prec<T, MC_GROUP_D, 0>;
  k.fn[MC_UPDATE_TV][UP_INIT] = LM_prec<T, MC_UPDATE_TV, UP_INIT>;
  k.fn[MC_UPDATE_TV][UP_STEP] = LM_prec<T, MC_UPDATE_TV, UP_STEP>;
  k.fn[MC_OUTER_CHECK][0] = LM_prec<T, MC_OUTER_CHECK, 0>;
}

void fill_multi_f32_row(MultiKernels& k);
void fill_multi_f32_col(MultiKernels& k);
void fill_multi_f64_row(MultiKernels& k);
void fill_multi_f64_col(MultiKernels& k);

const MultiKernels* multi_kernels(bool fp64) {
  static MultiKernels t32 = [] {
    MultiKernels k{};
    fill_multi_f32_row(k);
    fill_multi_f32_col(k);
    fill_multi_misc<float>(k);
    return k;
  }();
  static MultiKernels t64 = [] {
    MultiKernels k{};
    fill_multi_f64_row(k);
    fill_multi_f64_col(k);
    fill_multi_misc<double>(k);
    return k;
  }();
  return fp64 ? &t64 : &t32;
}

template <typename T>
size_t multi_lds_of(int cls, int n) {
  switch (n) {
#define FIRLS_CASE(NN)                                                              \
  case NN:                                                                          \
    if (cls == MC_ROWFWD || cls == MC_ROWINV || cls == MC_PAIR) return lds_bytes<T, NN>(); \
    if (cls == MC_COL) return lds_col_bytes<T, NN>();                               \
    return 0;
    FIRLS_SIZES(FIRLS_CASE)
#undef FIRLS_CASE
  }
  return 0;
}

size_t multi_lds_bytes(bool fp64, int cls, int n) { return fp64 ? multi_lds_of<double>(cls, n) : multi_lds_of<float>(cls, n); }

}  // namespace firls
