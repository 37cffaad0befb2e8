// Kernel instantiation: float, n = 256.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f32_256() { return make_size_kernels<float, 256>(); }
}  // namespace firls
