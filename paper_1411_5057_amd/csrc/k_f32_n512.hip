// Kernel instantiation: float, n = 512.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f32_512() { return make_size_kernels<float, 512>(); }
}  // namespace firls
