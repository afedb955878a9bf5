// Launchers of the gfx950 kernels (kernels.hip), called by the plan executor.
#pragma once

#include <hip/hip_runtime.h>

#include "fft_args.h"

namespace mifft {

// element-wise kernel ids (match planner OpType order after OP_PASS)
enum LineKernel : int {
    LINE_CHIRP_PAD = 1,
    LINE_MUL_CONJ,
    LINE_CHIRP_EXTRACT,
    LINE_R2C_TWIST,
    LINE_C2R_UNTWIST,
    LINE_REAL_TO_CPLX,
    LINE_HALF_COPY,
    LINE_HERM_EXPAND,
    LINE_CPLX_TO_REAL
};

struct StagesArg {
    int32_t nst, pad_;
    StageInfo st[kMaxStages];
};

// Per-plan preparation of a pass launch (LDS opt-in); call once at plan creation.
hipError_t prepare_pass(const PassArgs &a, bool f64);
hipError_t launch_pass(const PassArgs &a, bool f64, const void *in, void *out, hipStream_t st);
hipError_t launch_line(int type, const LineArgs &l, bool f64, const void *in, void *out, int64_t grid, int block,
                       hipStream_t st);

// FP64 table generators (plan time)
hipError_t gen_range(double2 *dst, int64_t N, int64_t e0, int64_t step, int64_t count, hipStream_t st);
hipError_t gen_inner(double2 *dst, const StagesArg &s, int64_t count, hipStream_t st);
hipError_t gen_chirp(double2 *dst, int64_t n, int64_t count, hipStream_t st);
hipError_t gen_bwrap(double2 *dst, const double2 *chirp, int64_t n, int64_t M, hipStream_t st);
hipError_t convert_d2f(float2 *dst, const double2 *src, int64_t count, hipStream_t st);

} // namespace mifft
