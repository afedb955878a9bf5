// Stockham pass kernels, complex128 data: passes with the r2c twist fused into the stores.
#include "pass_device.h"

namespace mifft {
const void *pass_kernel_f64_r2c(int shape) { return pass_kernel_table<double, PRO_PLAIN, EPI_R2C>(shape); }
} // namespace mifft
