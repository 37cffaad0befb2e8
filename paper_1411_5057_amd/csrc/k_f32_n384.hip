// Kernel instantiation: float, n = 384.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f32_384() { return make_size_kernels<float, 384>(); }
}  // namespace firls
