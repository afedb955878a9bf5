// Allocation-free execution (include/mifft.h, fft_execute_noalloc): one transform
// request planned on the host and run on `stream` with every device buffer the plan
// would own — its FP64 and FP32 tables and its scratch — placed in one static device
// array per GPU instead of memory from hipMalloc.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "kernels.h"
#include "mifft.h"
#include "planner.h"

namespace {

using namespace mifft;

// Bytes of the static array (every GPU the library runs on holds one until the process
// ends).
constexpr size_t kNoallocBytes = size_t(64) << 20;

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

// The array's device address on each GPU, taken once per device with that device
// current.  In host code `scratch` names a host-side stand-in, never the device memory.
constexpr int kMaxDevices = 64;
std::mutex g_addr_mutex;
void *g_addr[kMaxDevices] = {};

int scratch_address(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= kMaxDevices) return set_error(FFT_ERR_UNSUPPORTED, "device index beyond 64");
    std::lock_guard<std::mutex> lock(g_addr_mutex);
    if (!g_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(FFT_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_addr[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_addr[dev]);
    return FFT_OK;
}

int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

// Bytes the plan needs in the array: FP64 tables, FP32 copies (FP32 plans), scratch.
int64_t needed_bytes(const PlanSpec &sp, int64_t *scratch_off)
{
    const int64_t eb = sp.f64 ? 16 : 8;
    int64_t off = align256(sp.table_elems * 16);
    if (!sp.f64) off += align256(sp.table_elems * 8);
    for (int b = B_S0; b < B_NBUF; ++b) {
        scratch_off[b] = off;
        off += align256(sp.scratch_elems[b] * eb);
    }
    return off;
}

} // namespace

extern "C" int fft_execute_noalloc(int rank, const int64_t *dims, int64_t batch, int kind, int direction,
                                   int dtype, const void *in, void *out, hipStream_t stream)
{
    if (!in || !out) return set_error(FFT_ERR_INVALID_ARG, "NULL buffer");
    if (kind != FFT_C2C && in == out) return set_error(FFT_ERR_INVALID_ARG, "only C2C transforms run in place");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(FFT_ERR_HIP, "hipGetDevice");
    unsigned char *base = nullptr;
    int st = scratch_address(dev, &base);
    if (st != FFT_OK) return st;

    // plan on the host; if the plan's tables and scratch exceed the array, run the batch
    // in smaller chunks (the scratch is chunk-sized), down to one transform per chunk
    PlanSpec sp;
    std::string err;
    int64_t off[B_NBUF] = {};
    int64_t need = 0;
    for (int64_t target = -1;;) {
        sp = PlanSpec();
        sp.chunk_target = target;
        st = build_plan(rank, dims, batch, kind, direction, dtype, sp, err);
        if (st != FFT_OK) return set_error(st, err);
        need = needed_bytes(sp, off);
        // fits, or no smaller chunk exists (one transform per chunk, or a plan that
        // does not run in chunks at all)
        if (need <= int64_t(kNoallocBytes) || sp.batch == 1 || sp.chunk == 1 || (target >= 0 && sp.chunk == 0))
            break;
        target = target < 0 ? int64_t(kNoallocBytes) / 4 : std::max<int64_t>(1, target / 2);
    }
    for (const TableReq &t : sp.tables)
        if (t.kind == TableReq::BFILTER)
            return set_error(FFT_ERR_UNSUPPORTED, "the allocation-free entry point does not take lengths with a "
                                                  "prime factor above 7 (Bluestein's filter needs its own plan)");
    if (need > int64_t(kNoallocBytes))
        return set_error(FFT_ERR_UNSUPPORTED, "transform needs " + std::to_string(need) +
                                                  " bytes of tables and scratch; the allocation-free entry point "
                                                  "holds at most " + std::to_string(kNoallocBytes));

    // tables: generated in FP64 into the array on `stream`, rounded once for FP32 plans
    const int64_t eb = sp.f64 ? 16 : 8;
    double2 *t64 = reinterpret_cast<double2 *>(base);
    void *tabs = sp.f64 ? static_cast<void *>(t64) : static_cast<void *>(base + align256(sp.table_elems * 16));
    for (const TableReq &t : sp.tables) {
        double2 *dst = t64 + t.offset;
        hipError_t e = hipSuccess;
        if (t.kind == TableReq::INNER) {
            StagesArg sa{};
            sa.nst = t.nst;
            for (int s = 0; s < t.nst; ++s) sa.st[s] = t.st[s];
            e = gen_inner(dst, sa, t.count, stream);
        } else if (t.kind == TableReq::RANGE) {
            e = gen_range(dst, t.N, t.e0, t.step, t.count, stream);
        } else if (t.kind == TableReq::CHIRP) {
            e = gen_chirp(dst, t.N, t.count, stream);
        }
        if (e != hipSuccess) return set_error(FFT_ERR_HIP, std::string("table generation: ") + hipGetErrorString(e));
    }
    if (!sp.f64 && sp.table_elems > 0) {
        const hipError_t e = convert_d2f(static_cast<float2 *>(tabs), t64, sp.table_elems, stream);
        if (e != hipSuccess) return set_error(FFT_ERR_HIP, std::string("table rounding: ") + hipGetErrorString(e));
    }

    // the op lists with table pointers into the array, run chunk by chunk as fft_execute does
    const bool inplace = in == out;
    const int64_t chunk = sp.chunk > 0 ? sp.chunk : sp.batch;
    const int64_t rb = sp.f64 ? 8 : 4;
    const int64_t in_eb = (kind == FFT_C2C || kind == FFT_C2R) ? 2 * rb : rb;
    const int64_t out_eb = (kind == FFT_C2C || kind == FFT_R2C) ? 2 * rb : rb;
    auto table_ptr = [&](int id, bool fp64) -> const void * {
        if (id < 0) return nullptr;
        const int64_t o = sp.tables[size_t(id)].offset;
        return fp64 ? static_cast<const void *>(t64 + o) : static_cast<const char *>(tabs) + o * eb;
    };
    for (int64_t first = 0; first < sp.batch; first += chunk) {
        const bool tail = sp.batch - first < chunk;
        std::vector<Op> &plain = tail ? sp.tail_ops : sp.ops;
        std::vector<Op> &inpl = tail ? sp.tail_ops_inplace : sp.ops_inplace;
        std::vector<Op> &ops = (inplace && !inpl.empty()) ? inpl : plain;
        void *buf[B_NBUF];
        buf[B_IN] = static_cast<char *>(const_cast<void *>(in)) + first * sp.in_dist * in_eb;
        buf[B_OUT] = static_cast<char *>(out) + first * sp.out_dist * out_eb;
        for (int b = B_S0; b < B_NBUF; ++b) buf[b] = base + off[b];
        for (Op &op : ops) {
            hipError_t e;
            if (op.type == OP_PASS) {
                op.pa.itw = table_ptr(op.t_itw, sp.f64);
                op.pa.tw_lo = table_ptr(op.t_lo, true);
                op.pa.tw_hi = table_ptr(op.t_hi, true);
                op.pa.aux = table_ptr(op.t_aux, sp.f64);
                op.pa.aux2 = table_ptr(op.t_aux2, sp.f64);
                e = prepare_pass(op.pa, sp.f64);
                if (e == hipSuccess) e = launch_pass(op.pa, sp.f64, buf[op.src], buf[op.dst], stream);
            } else {
                op.la.tab = table_ptr(op.t_tab, sp.f64);
                op.la.tab2 = table_ptr(op.t_tab2, sp.f64);
                e = launch_line(op.type, op.la, sp.f64, buf[op.src], buf[op.dst], op.grid, op.block, stream);
            }
            if (e != hipSuccess) return set_error(FFT_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
        }
    }
    return FFT_OK;
}
