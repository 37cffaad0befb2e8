// Kernel instantiation: double, n = 48.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f64_48() { return make_size_kernels<double, 48>(); }
}  // namespace firls
