// Kernel instantiation: double, n = 512.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f64_512() { return make_size_kernels<double, 512>(); }
}  // namespace firls
