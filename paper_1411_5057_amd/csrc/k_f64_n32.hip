// Kernel instantiation: double, n = 32.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f64_32() { return make_size_kernels<double, 32>(); }
}  // namespace firls
