// Kernel instantiation: float, n = 32.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f32_32() { return make_size_kernels<float, 32>(); }
}  // namespace firls
