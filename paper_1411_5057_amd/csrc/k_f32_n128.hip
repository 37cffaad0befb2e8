// Kernel instantiation: float, n = 128.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f32_128() { return make_size_kernels<float, 128>(); }
}  // namespace firls
