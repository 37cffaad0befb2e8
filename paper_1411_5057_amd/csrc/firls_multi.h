// Launches across shapes: one grid covers the slices of every shape of a
// batch for one kernel class and mode.  Each workgroup reads its work item
// (slice, block within the slice, Params entry) and runs that shape's
// kernel body, chosen by the image side, so a batch of uneven slices takes
// one launch per class and position of the outer iteration instead of one
// per shape (internal).
#pragma once
#include "firls_kernels.h"
#include "firls_registry.h"

namespace firls {

#define FIRLS_MULTI_PROLOGUE                          \
  const MultiItem it = A.items[blockIdx.x];           \
  const Params& P = A.table[it.p];                    \
  const Blk B{it.x, it.s};

template <typename T, int MODE>
__global__ __launch_bounds__(NT) void km_rowfwd(MultiArgs A) {
  FIRLS_MULTI_PROLOGUE
  switch (P.n) {
#define FIRLS_CASE(NN) case NN: rowfwd_body<T, NN, MODE>(P, B); break;
    FIRLS_SIZES(FIRLS_CASE)
#undef FIRLS_CASE
  }
}

template <typename T, int MODE>
__global__ __launch_bounds__(NT) void km_col(MultiArgs A) {
  FIRLS_MULTI_PROLOGUE
  switch (P.n) {
#define FIRLS_CASE(NN) case NN: col_body<T, NN, MODE>(P, B); break;
    FIRLS_SIZES(FIRLS_CASE)
#undef FIRLS_CASE
  }
}

template <typename T, int MODE>
__global__ __launch_bounds__(NT) void km_rowinv(MultiArgs A) {
  FIRLS_MULTI_PROLOGUE
  switch (P.n) {
#define FIRLS_CASE(NN) case NN: rowinv_body<T, NN, MODE>(P, B); break;
    FIRLS_SIZES(FIRLS_CASE)
#undef FIRLS_CASE
  }
}

// the paired PCG pass exists where a thread holds one tile column (sides up
// to 256); here without the last iteration's regulariser sum (the sequence
// recorded for launches across shapes keeps that iteration's row inverse)
#define FIRLS_PAIR_SIZES(X) X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256)
template <typename T>
__global__ __launch_bounds__(NT, sizeof(T) == 4 ? 4 : 2) void km_pair(MultiArgs A) {
  FIRLS_MULTI_PROLOGUE
  switch (P.n) {
#define FIRLS_CASE(NN) case NN: pcg_pair_body<T, NN, false>(P, B); break;
    FIRLS_PAIR_SIZES(FIRLS_CASE)
#undef FIRLS_CASE
  }
}
// FP32 sides 384 and 512 (two tile columns per thread, two workgroups per
// CU): mode 1 of the paired class
template <typename T>
__global__ __launch_bounds__(NT, 2) void km_pair_wide(MultiArgs A) {
  FIRLS_MULTI_PROLOGUE
  switch (P.n) {
    case 384: pcg_pair_body<T, 384, false>(P, B); break;
    case 512: pcg_pair_body<T, 512, false>(P, B); break;
  }
}

template <typename T, int CLS>
__global__ __launch_bounds__(NT) void km_haar(MultiArgs A) {
  FIRLS_MULTI_PROLOGUE
  switch (P.n) {
#define FIRLS_CASE(NN)                                          \
  case NN:                                                      \
    if constexpr (CLS == MC_PSI_SQ_HAAR) psi_sq_haar_body<T, NN>(P, B); \
    else if constexpr (CLS == MC_UPDATE_HAAR) update_haar_body<T, NN>(P, B); \
    else last_x_body<T, NN>(P, B);                              \
    break;
    FIRLS_SIZES(FIRLS_CASE)
#undef FIRLS_CASE
  }
}

template <typename T, int CLS, int MODE>
__global__ __launch_bounds__(NT) void km_prec(MultiArgs A) {
  FIRLS_MULTI_PROLOGUE
  if constexpr (CLS == MC_PSI_SQ_TV) psi_sq_tv_body<T>(P, B);
  else if constexpr (CLS == MC_GROUP_W) group_w_body<T>(P, B);
  else if constexpr (CLS == MC_GROUP_D) group_d_body<T>(P, B);
  else if constexpr (CLS == MC_UPDATE_TV) update_tv_body<T, MODE>(P, B);
  else {
    if (P.state[B.s].active) outer_check_wg(P, B.s);
  }
}

template <class K>
hipError_t launch_multi_kernel(K kern, const MultiArgs& A, int items, size_t lds, hipStream_t st) {
  const LaunchTiming& t = launch_timing();
  launch_kernel(kern, dim3(items), dim3(NT), lds, st, t.start, t.stop, A);
  return hipGetLastError();
}

template <class K>
void allow_multi_lds(K kern, size_t bytes) {
  (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace firls
