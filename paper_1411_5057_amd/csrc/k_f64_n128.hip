// Kernel instantiation: double, n = 128.
#include "firls_inst.h"
namespace firls {
SizeKernels make_size_f64_128() { return make_size_kernels<double, 128>(); }
}  // namespace firls
