// Kernel instantiation: float, n = 48.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f32_48() { return make_size_kernels<float, 48>(); }
}  // namespace firls
