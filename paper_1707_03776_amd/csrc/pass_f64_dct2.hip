// Stockham pass kernels, complex128 data: first-stage loads of Makhoul-reordered input reals
// (PRO_DCT2, the DCT-II reordering folded into the real transform's first pass), plain
// stores; specialised shapes only.
#include "pass_device.h"

namespace mifft {
const void *pass_kernel_f64_dct2(int shape) { return fixed_kernel_table<double, PRO_DCT2, EPI_PLAIN>(shape); }
} // namespace mifft
