// Stockham pass kernels, complex64 data: plain loads scaled by a real separable symbol
// (PRO_SYM), plain stores; specialised shapes only.
#include "pass_device.h"

namespace mifft {
const void *pass_kernel_f32_sym(int shape) { return fixed_kernel_table<float, PRO_SYM, EPI_PLAIN>(shape); }
} // namespace mifft
