// Launchers of the gfx950 kernels (kernels.hip), called by the plan executor.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "fft_args.h"

struct fft_plan_s; // the C ABI's plan (include/mifft.h)

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
    LINE_CPLX_TO_REAL,
    LINE_DCT2_PRE,
    LINE_DCT2_POST,
    LINE_DCT3_PRE,
    LINE_DCT3_POST,
    LINE_DCT2_TWPOST,
    LINE_DCT3_PREUNTWIST
};

// Elements an element-wise op covers: lines x per-line length.
__host__ __device__ inline int64_t line_total(int type, const LineArgs &l)
{
    switch (type) {
    case LINE_CHIRP_PAD:
    case LINE_MUL_CONJ: return l.nlines * l.M;
    case LINE_R2C_TWIST:
    case LINE_HALF_COPY: return l.nlines * (l.n / 2 + 1);
    case LINE_C2R_UNTWIST: return l.nlines * (l.n / 2);
    case LINE_DCT3_PRE: return l.nlines * (l.n / 2 + 1);
    case LINE_DCT2_TWPOST:
    case LINE_DCT3_PREUNTWIST: return l.nlines * (l.n / 4 + 1);
    default: return l.nlines * l.n; // chirp extract, real/complex staging, Hermitian expand
    }
}

// Ragged batch: a short sequence of launches (phases) over a table of blocks.  A block
// either runs one whole small transform (every op of its length's plan, in one
// workgroup) or one part of one op of a large transform: a tile of a pass, or a chunk
// of an element-wise op.  Op k of a large transform runs in phase k, so the launch
// boundary orders it after op k-1; blocks of one phase never depend on each other.
constexpr int B_NBUF_DEV = 7;           // buffers an op may name: in, out, five scratch regions
constexpr int kRagLineChunk = 256 * 16; // elements of an element-wise op per block

struct RagOp {                        // one op of one length's plan
    int32_t type, src, dst, tiles;    // type 0: pass (pa, `tiles` tiles), otherwise the element-wise kernel id (la)
    PassArgs pa;
    LineArgs la;
};
struct RagClass {                     // the plan shared by every transform of one length
    int32_t first_op, nops;
    int64_t sofs[B_NBUF_DEV];         // scratch region offsets (elements) within a transform's scratch
};
// Everything a block needs, so its first loads do not depend on each other.
// Part block: op = global op index, off[0] / off[1] = element offsets of the op's
// source / destination within the buffer the op names (in, out or the scratch arena).
// Whole block: op = class index, off = the transform's in, out and scratch offsets.
constexpr uint32_t kRagWhole = 0x80000000u;
struct RagBlock {
    int64_t off[3];
    uint32_t op;
    uint32_t part;                    // tile of a pass, or chunk of an element-wise op; kRagWhole: whole
};
struct RaggedArgs {
    const void *blocks, *classes, *ops;
    const void *in;
    void *out, *scratch;
};

const void *ragged_kernel(bool f64);

struct StagesArg {
    int32_t nst, pad_;
    StageInfo st[kMaxStages];
};

// Device allocation of plan and operator creation (api.cpp): hipMalloc, except that
// the test hook MIFFT_TEST_FAIL_ALLOC=k makes the k-th allocation of the outermost
// creation call on this thread fail with hipErrorOutOfMemory.  Every creation entry
// point holds a CreateScope for its duration (it starts the count).
hipError_t dev_malloc(void **ptr, size_t bytes);
struct CreateScope {
    CreateScope();
    ~CreateScope();
    CreateScope(const CreateScope &) = delete;
    CreateScope &operator=(const CreateScope &) = delete;
};

// Per-plan preparation of a pass launch (LDS opt-in); call once at plan creation.
hipError_t prepare_pass(PassArgs &a, bool f64);

// For operators that fuse a step into a plan they own (api.cpp): the first op of each
// of the plan's op lists (chunk lists included) when every one is a pass, else empty;
// and the plan's description rebuilt after such a change.
std::vector<PassArgs *> plan_first_passes(::fft_plan_s *p);
void plan_refresh_description(::fft_plan_s *p);
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
