// Stockham pass kernels, complex64 data: mirrored tiles whose c2r untwist of the bins runs
// into LDS before the first stage (PRO_CUNTWIST, the first pass of a staged real inverse);
// specialised shapes only.
#include "pass_device.h"

namespace mifft {
const void *pass_kernel_f32_cuntwist(int shape) { return fixed_kernel_table<float, PRO_CUNTWIST, EPI_PLAIN>(shape); }
} // namespace mifft
