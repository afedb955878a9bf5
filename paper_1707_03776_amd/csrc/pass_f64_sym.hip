// Stockham pass kernels, complex128 data: plain loads scaled by a real separable symbol
// (PRO_SYM), plain stores; specialised shapes only.
#include "pass_device.h"

namespace mifft {
const void *pass_kernel_f64_sym(int shape) { return fixed_kernel_table<double, PRO_SYM, EPI_PLAIN>(shape); }
} // namespace mifft
