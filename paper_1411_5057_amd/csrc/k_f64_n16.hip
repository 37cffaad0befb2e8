// Kernel instantiation: double, n = 16.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f64_16() { return make_size_kernels<double, 16>(); }
}  // namespace firls
