// Kernel instantiation: float, n = 192.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f32_192() { return make_size_kernels<float, 192>(); }
}  // namespace firls
