// Kernel instantiation: double, n = 64.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f64_64() { return make_size_kernels<double, 64>(); }
}  // namespace firls
