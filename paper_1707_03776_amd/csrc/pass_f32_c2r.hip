// Stockham pass kernels, complex64 data: passes with the c2r untwist fused into the loads.
#include "pass_device.h"

namespace mifft {
const void *pass_kernel_f32_c2r(int shape) { return pass_kernel_table<float, PRO_C2R, EPI_PLAIN>(shape); }
} // namespace mifft
