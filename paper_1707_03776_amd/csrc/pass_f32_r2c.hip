// Stockham pass kernels, complex64 data: passes with the r2c twist fused into the stores.
#include "pass_device.h"

namespace mifft {
const void *pass_kernel_f32_r2c(int shape) { return pass_kernel_table<float, PRO_PLAIN, EPI_R2C>(shape); }
} // namespace mifft
