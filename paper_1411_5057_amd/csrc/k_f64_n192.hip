// Kernel instantiation: double, n = 192.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f64_192() { return make_size_kernels<double, 192>(); }
}  // namespace firls
