// Kernel instantiation: double, n = 96.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f64_96() { return make_size_kernels<double, 96>(); }
}  // namespace firls
