// Kernel instantiation: double, n = 384.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f64_384() { return make_size_kernels<double, 384>(); }
}  // namespace firls
