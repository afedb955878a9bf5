// Stockham pass kernels, complex64 data: plain loads in mirrored tiles, the real transform's twist and the DCT-II rotation folded into the last pass of a staged real transform (EPI_DTWIST); specialised
// shapes only.
#include "pass_device.h"

namespace mifft {
const void *pass_kernel_f32_dtwist(int shape) { return fixed_kernel_table<float, PRO_PLAIN, EPI_DTWIST>(shape); }
} // namespace mifft
