// Kernel instantiation: double, n = 256.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f64_256() { return make_size_kernels<double, 256>(); }
}  // namespace firls
