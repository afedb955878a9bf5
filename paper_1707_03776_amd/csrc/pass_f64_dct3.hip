// Stockham pass kernels, complex128 data: plain loads, last-stage stores that put the two reals
// of each point back in natural order (EPI_DCT3, the DCT-III inverse reordering folded
// into the real inverse transform's last pass); specialised shapes only.
#include "pass_device.h"

namespace mifft {
const void *pass_kernel_f64_dct3(int shape) { return fixed_kernel_table<double, PRO_PLAIN, EPI_DCT3>(shape); }
} // namespace mifft
