// Stockham pass kernels, complex128 data: passes with the c2r untwist fused into the loads.
#include "pass_device.h"

namespace mifft {
const void *pass_kernel_f64_c2r(int shape) { return pass_kernel_table<double, PRO_C2R, EPI_PLAIN>(shape); }
} // namespace mifft
