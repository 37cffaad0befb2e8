// Launchers for one (precision, size) instantiation (internal).
#pragma once
#include "firls_kernels.h"
#include "firls_registry.h"

namespace firls {

// Dynamic LDS of the row passes (band_rows(N) lines) and of the column
// pass (strip_cols lines), each followed by the N twiddles.
template <typename T, int N>
constexpr size_t lds_bytes() {
  return ((size_t)band_rows(N) * LdsLayout<N>::LS + N) * sizeof(cplx<T>);
}
template <typename T, int N>
constexpr size_t lds_col_bytes() {
  return ((size_t)Geo<T, N>::COLS * LdsLayout<N>::LS + N) * sizeof(cplx<T>);
}

template <class K>
hipError_t launch_dyn(K kern, size_t lds, const Params& P, dim3 g, hipStream_t st) {
  const LaunchTiming& t = launch_timing();
  launch_kernel(kern, g, dim3(NT), lds, st, t.start, t.stop, P);
  return hipGetLastError();
}

#define FIRLS_DYN_LAUNCHER(NAME, KERNEL)                                       \
  template <typename T, int N, int M>                                          \
  hipError_t NAME(const Params& P, dim3 g, hipStream_t st) {                   \
    return launch_dyn(KERNEL<T, N, M>, lds_bytes<T, N>(), P, g, st);           \
  }
FIRLS_DYN_LAUNCHER(L_rowfwd, k_rowfwd)
FIRLS_DYN_LAUNCHER(L_rowinv, k_rowinv)
#undef FIRLS_DYN_LAUNCHER

template <typename T, int N, int M>
hipError_t L_col(const Params& P, dim3 g, hipStream_t st) {
  return launch_dyn(k_col<T, N, M>, lds_col_bytes<T, N>(), P, g, st);
}
template <typename T, int N>
hipError_t L_update_haar(const Params& P, dim3 g, hipStream_t st) {
  return launch_dyn(k_update_haar<T, N>, 0, P, g, st);
}
template <typename T, int N>
hipError_t L_last_x(const Params& P, dim3 g, hipStream_t st) {
  return launch_dyn(k_last_x<T, N>, 0, P, g, st);
}
template <typename T, int N>
hipError_t L_pcg_pair(const Params& P, dim3 g, hipStream_t st) {
  return launch_dyn(k_pcg_pair<T, N>, lds_bytes<T, N>(), P, g, st);
}
template <typename T, int N>
hipError_t L_psi_sq_haar(const Params& P, dim3 g, hipStream_t st) {
  return launch_dyn(k_psi_sq_haar<T, N>, 0, P, g, st);
}

template <class K>
void allow_lds(K kern, size_t bytes) {
  if (bytes > 64 * 1024) (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename T, int N>
SizeKernels make_size_kernels() {
  const size_t b = lds_bytes<T, N>();
  allow_lds(k_rowfwd<T, N, RF_PLAIN>, b);
  allow_lds(k_rowfwd<T, N, RF_PCG_HAAR>, b);
  allow_lds(k_rowfwd<T, N, RF_PCG_Z>, b);
  allow_lds(k_rowfwd<T, N, RF_STEP_HAAR>, b);
  allow_lds(k_rowfwd<T, N, RF_SQ_HAAR>, b);
  allow_lds(k_rowfwd<T, N, RF_SQW_HAAR>, b);
  allow_lds(k_rowfwd<T, N, RF_PEN_HAAR>, b);
  const size_t bc = lds_col_bytes<T, N>();
  allow_lds(k_col<T, N, COL_SP>, bc);
  allow_lds(k_col<T, N, COL_R0>, bc);
  allow_lds(k_col<T, N, COL_AHB>, bc);
  allow_lds(k_col<T, N, COL_DC>, bc);
  allow_lds(k_col<T, N, COL_SP_PQ>, bc);
  allow_lds(k_rowinv<T, N, RI_PLAIN>, b);
  allow_lds(k_rowinv<T, N, RI_SP_HAAR>, b);
  allow_lds(k_rowinv<T, N, RI_SP_TV>, b);
  allow_lds(k_rowinv<T, N, RI_R0_HAAR>, b);
  allow_lds(k_rowinv<T, N, RI_R0_TV>, b);
  allow_lds(k_rowinv<T, N, RI_R0_HAAR_P0>, b);
  // one tile column per thread in both precisions (FP64 at two workgroups
  // per CU, as its fused step); two in FP32 (sides 384 and 512)
  constexpr bool pair = Units<N, band_rows(N)>::PER == 1 || (Units<N, band_rows(N)>::PER == 2 && sizeof(T) == 4);
  if constexpr (pair) allow_lds(k_pcg_pair<T, N>, b);
  SizeKernels k{};
  k.rowfwd[RF_PLAIN] = L_rowfwd<T, N, RF_PLAIN>;
  k.rowfwd[RF_PCG_HAAR] = L_rowfwd<T, N, RF_PCG_HAAR>;
  k.rowfwd[RF_PCG_Z] = L_rowfwd<T, N, RF_PCG_Z>;
  k.rowfwd[RF_STEP_HAAR] = L_rowfwd<T, N, RF_STEP_HAAR>;
  k.rowfwd[RF_SQ_HAAR] = L_rowfwd<T, N, RF_SQ_HAAR>;
  k.rowfwd[RF_SQW_HAAR] = L_rowfwd<T, N, RF_SQW_HAAR>;
  k.rowfwd[RF_PEN_HAAR] = L_rowfwd<T, N, RF_PEN_HAAR>;
  k.col[COL_SP] = L_col<T, N, COL_SP>;
  k.col[COL_R0] = L_col<T, N, COL_R0>;
  k.col[COL_AHB] = L_col<T, N, COL_AHB>;
  k.col[COL_DC] = L_col<T, N, COL_DC>;
  k.col[COL_SP_PQ] = L_col<T, N, COL_SP_PQ>;
  k.rowinv[RI_PLAIN] = L_rowinv<T, N, RI_PLAIN>;
  k.rowinv[RI_SP_HAAR] = L_rowinv<T, N, RI_SP_HAAR>;
  k.rowinv[RI_SP_TV] = L_rowinv<T, N, RI_SP_TV>;
  k.rowinv[RI_R0_HAAR] = L_rowinv<T, N, RI_R0_HAAR>;
  k.rowinv[RI_R0_TV] = L_rowinv<T, N, RI_R0_TV>;
  k.rowinv[RI_R0_HAAR_P0] = L_rowinv<T, N, RI_R0_HAAR_P0>;
  k.psi_sq_haar = L_psi_sq_haar<T, N>;
  k.last_x = L_last_x<T, N>;
  k.update_haar = L_update_haar<T, N>;
  if constexpr (pair) k.pcg_pair = L_pcg_pair<T, N>;
  return k;
}

}  // namespace firls
