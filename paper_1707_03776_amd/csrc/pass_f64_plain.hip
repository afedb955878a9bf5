// Stockham pass kernels, complex128 data: complex passes, plain loads and stores.
#include "pass_device.h"

namespace mifft {
const void *pass_kernel_f64_plain(int shape) { return pass_kernel_table<double, PRO_PLAIN, EPI_PLAIN>(shape); }
} // namespace mifft
