// Stockham pass kernels, complex128 data: plain loads in mirrored tiles, the real transform's twist folded into the last pass of a staged real transform (EPI_RTWIST); specialised
// shapes only.
#include "pass_device.h"

namespace mifft {
const void *pass_kernel_f64_rtwist(int shape) { return fixed_kernel_table<double, PRO_PLAIN, EPI_RTWIST>(shape); }
} // namespace mifft
