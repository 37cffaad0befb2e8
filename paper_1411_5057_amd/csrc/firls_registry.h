// Host-side tables of kernel launchers (internal).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include "firls_types.h"

namespace firls {

// Opt-in per-launch timing: while ``start`` is set (the handle's profiling
// mode, one launcher call at a time on the calling thread), launches record
// the kernel's own GPU start and end times in these events, the interval a
// kernel trace reports, with no launch gap in it.
struct LaunchTiming {
  hipEvent_t start, stop;
};
LaunchTiming& launch_timing();

template <class K, class... A>
void launch_kernel(K kern, dim3 g, dim3 b, size_t lds, hipStream_t st, hipEvent_t start, hipEvent_t stop, A... args) {
  if (start || stop) hipExtLaunchKernelGGL(kern, g, b, (uint32_t)lds, st, start, stop, 0u, args...);
  else hipLaunchKernelGGL(kern, g, b, lds, st, args...);
}

using Launcher = hipError_t (*)(const Params&, dim3, hipStream_t);

// Kernels that depend on the image side (FFT length).
struct SizeKernels {
  Launcher rowfwd[7];
  Launcher col[5];
  Launcher rowinv[6];
  Launcher psi_sq_haar;
  Launcher last_x;
  Launcher update_haar;
  Launcher pcg_pair;   // null in FP64 where a thread holds more than one tile column (sides above 256)
};

// Kernels that depend on the precision only.
struct PrecKernels {
  Launcher psi_sq_tv;
  Launcher group_w;
  Launcher group_d;
  Launcher update_tv[2];
  Launcher export_d;
  Launcher slice_init;
  Launcher outer_check;
};

// Dense sensing matrix products (GemmMode order).
struct GemmKernels {
  Launcher g[4];
};
const GemmKernels* gemm_kernels(bool fp64);

// Saves the final states of stopped slices, points their slots at new
// slices and starts those (as k_slice_init does); one workgroup per record.
hipError_t launch_refill(const RefillArgs& A, hipStream_t st);

// Launches across shapes (MultiClass x mode); null where not built.
using MultiLauncher = hipError_t (*)(const MultiArgs&, int items, size_t lds, hipStream_t);
struct MultiKernels {
  MultiLauncher fn[MC_COUNT][MC_MODES];
};
const MultiKernels* multi_kernels(bool fp64);
// Dynamic LDS a kernel of class cls needs for image side n (0: none).
size_t multi_lds_bytes(bool fp64, int cls, int n);

// nullptr if the size is not built for that precision.
const SizeKernels* size_kernels(bool fp64, int n);
const PrecKernels* prec_kernels(bool fp64);
bool size_supported(int n);

}  // namespace firls
