// The ragged batch kernel (fft_plan_create_many).
#include <hip/hip_runtime.h>

#include "line_device.h"
#include "pass_device.h"

namespace mifft {

// ----------------------------------------------------------------------------- ragged batch

// A ragged batch runs as a few launches (phases) over a block table built on the host.
// A whole block runs every op of a small transform's plan in order, with a workgroup
// barrier between steps; a part block runs one tile (or element chunk) of op k of a
// large transform in phase k, after the launch boundary has ordered it behind op k-1.
// No block ever waits on another, so no device-scope synchronisation is needed.

// One op of a ragged transform, or one part of it: tiles [t0, t1) of a pass, or
// elements [e0, e1) of an element-wise op.
template <typename R>
__device__ __forceinline__ void ragged_op(const RagOp &op, typename Cplx<R>::T *lds, const void *src, void *dst,
                                          int64_t lo, int64_t hi)
{
    using C = typename Cplx<R>::T;
    if (op.type == 0) {
        constexpr int E = RaggedElems<R>::v;
        const C *s = static_cast<const C *>(src);
        C *d = static_cast<C *>(dst);
        for (int64_t tile = lo; tile < hi; ++tile) {
            const uint32_t col0 = uint32_t(tile) * uint32_t(op.pa.c);
            const int ncl = int(min(int64_t(op.pa.c), op.pa.ncols - int64_t(col0)));
            // plain and fused Bluestein passes alike (the flavour is read from op.pa)
            generic_pass_tile<R, PRO_PLAIN, EPI_PLAIN, E>(op.pa, lds, s, d, col0, ncl);
            __syncthreads(); // the next tile reuses LDS; the next op reads this one's output
        }
    } else {
        for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) line_elem_dispatch<R>(op.type, op.la, e, src, dst);
        __syncthreads();
    }
}

// One phase of a ragged batch: block b runs blocks[b] (a whole small transform, or
// one part of one op of a large one).
template <typename R>
__global__ void __launch_bounds__(256) k_ragged(const RaggedArgs g)
{
    using C = typename Cplx<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const RagBlock bk = static_cast<const RagBlock *>(g.blocks)[blockIdx.x];
    const RagOp *ops = static_cast<const RagOp *>(g.ops);
    C *const scratch = static_cast<C *>(g.scratch);
    // The op descriptor is copied into LDS in one coalesced read before use.  Read in
    // place, each field became a separate vector load and full wait on the way to the
    // data loads (the kernel's stores keep the compiler from using scalar loads), a
    // chain of L2 round trips per block.
    __shared__ RagOp sop;
    auto stage = [&](const RagOp &src) {
        static_assert(sizeof(RagOp) % 8 == 0, "RagOp is copied in 8-byte words");
        for (int i = threadIdx.x; i < int(sizeof(RagOp) / 8); i += blockDim.x)
            reinterpret_cast<uint2 *>(&sop)[i] = reinterpret_cast<const uint2 *>(&src)[i];
        __syncthreads();
    };
    if (bk.part & kRagWhole) {
        const RagClass &cl = static_cast<const RagClass *>(g.classes)[bk.op];
        const void *bases[B_NBUF_DEV];
        bases[0] = static_cast<const C *>(g.in) + bk.off[0];
        bases[1] = static_cast<C *>(g.out) + bk.off[1];
        for (int b = 2; b < B_NBUF_DEV; ++b) bases[b] = scratch + bk.off[2] + cl.sofs[b];
        for (int o = 0; o < cl.nops; ++o) {
            stage(ops[cl.first_op + o]);
            const RagOp &op = sop;
            const int64_t n = op.type == 0 ? int64_t(op.tiles) : line_total(op.type, op.la);
            ragged_op<R>(op, lds, bases[op.src], const_cast<void *>(bases[op.dst]), 0, n);
        }
    } else {
        stage(ops[bk.op]);
        const RagOp &op = sop;
        const C *src = (op.src == 0 ? static_cast<const C *>(g.in) : op.src == 1 ? static_cast<const C *>(g.out)
                                                                                 : scratch) + bk.off[0];
        C *dst = (op.dst == 1 ? static_cast<C *>(g.out) : scratch) + bk.off[1];
        int64_t lo = bk.part, hi = int64_t(bk.part) + 1;
        if (op.type != 0) {
            lo = int64_t(bk.part) * kRagLineChunk;
            hi = min(lo + kRagLineChunk, line_total(op.type, op.la));
        }
        ragged_op<R>(op, lds, src, dst, lo, hi);
    }
}

const void *ragged_kernel(bool f64)
{
    return f64 ? reinterpret_cast<const void *>(&k_ragged<double>) : reinterpret_cast<const void *>(&k_ragged<float>);
}

} // namespace mifft
