// Kernel instantiation: float, n = 96.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f32_96() { return make_size_kernels<float, 96>(); }
}  // namespace firls
