// Stockham pass kernels, complex64 data: complex passes, plain loads and stores.
#include "pass_device.h"

namespace mifft {
const void *pass_kernel_f32_plain(int shape) { return pass_kernel_table<float, PRO_PLAIN, EPI_PLAIN>(shape); }
} // namespace mifft
