// Kernel instantiation: float, n = 64.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f32_64() { return make_size_kernels<float, 64>(); }
}  // namespace firls
