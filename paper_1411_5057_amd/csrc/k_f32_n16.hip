// Kernel instantiation: float, n = 16.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f32_16() { return make_size_kernels<float, 16>(); }
}  // namespace firls
