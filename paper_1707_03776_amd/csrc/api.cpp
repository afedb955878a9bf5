// C ABI of the library (include/mifft.h): plan creation (planner + FP64 table
// generation on the GPU + scratch), execution (one launch per planned op on the
// caller's stream), destruction, and the thread-local error state.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <new>
#include <sstream>
#include <vector>
#include <string>

#include "kernels.h"
#include "mifft.h"
#include "planner.h"

using namespace mifft;

struct fft_plan_s {
    PlanSpec spec;
    int device = 0;
    void *tables = nullptr;   // in the plan's precision
    void *tables64 = nullptr; // FP64 originals (the multi-pass twiddles are read from here)
    void *scratch[B_NBUF] = {};
    int64_t device_bytes = 0;
    std::string desc;
    // ragged batch (fft_plan_create_many)
    struct Many *many = nullptr;
};

struct Many {
    ManySpec ms;
    RagOp *ops = nullptr;
    RagClass *classes = nullptr;
    RagBlock *blocks = nullptr;              // every phase's blocks, phase after phase
    std::vector<uint32_t> phase_first, phase_blocks;
    uint32_t count = 0;
    void *scratch = nullptr;
    int block = 256;
    size_t lds = 0;
    hipGraph_t graph = nullptr;                 // one kernel node per phase, instantiated at creation
    hipGraphExec_t exec = nullptr;
    std::vector<hipGraphNode_t> nodes;
    const void *g_in = nullptr;                 // buffers the exec's nodes are bound to
    void *g_out = nullptr;
};

namespace mifft {

std::vector<PassArgs *> plan_first_passes(fft_plan p)
{
    std::vector<PassArgs *> out;
    if (!p || p->many) return out;
    for (std::vector<Op> *list : {&p->spec.ops, &p->spec.ops_inplace, &p->spec.tail_ops, &p->spec.tail_ops_inplace}) {
        if (list->empty()) continue;
        if (list->front().type != OP_PASS) return {};
        out.push_back(&list->front().pa);
    }
    return out;
}

void plan_refresh_description(fft_plan p)
{
    if (p && !p->many) p->desc = p->spec.describe();
}

} // namespace mifft

namespace {

thread_local int g_status = FFT_OK;
thread_local std::string g_msg;

// Allocation-failure injection for tests: with MIFFT_TEST_FAIL_ALLOC=k set, the k-th
// device allocation of a plan or operator creation call fails as if the device were
// out of memory (allocations of nested creations, such as a Bluestein filter's
// sub-plan, count towards their outermost call).
thread_local int g_create_depth = 0;
thread_local int64_t g_alloc_seq = 0, g_fail_at = 0;

int fail(int status, const std::string &msg)
{
    g_status = status;
    g_msg = msg;
    return status;
}

#define HIP_TRY(expr)                                                                                       \
    do {                                                                                                    \
        hipError_t e__ = (expr);                                                                            \
        if (e__ != hipSuccess) {                                                                            \
            fail(e__ == hipErrorOutOfMemory ? FFT_ERR_ALLOC : FFT_ERR_HIP,                                  \
                 std::string(#expr) + ": " + hipGetErrorString(e__));                                       \
            goto fail_label;                                                                                \
        }                                                                                                   \
    } while (0)

void free_many(Many *m)
{
    if (!m) return;
    if (m->exec) (void)hipGraphExecDestroy(m->exec);
    if (m->graph) (void)hipGraphDestroy(m->graph);
    for (void *q : {(void *)m->ops, (void *)m->classes, (void *)m->blocks, m->scratch})
        if (q) (void)hipFree(q);
    delete m;
}

void free_plan(fft_plan p)
{
    if (!p) return;
    free_many(p->many);
    if (p->tables && p->tables != p->tables64) (void)hipFree(p->tables);
    if (p->tables64) (void)hipFree(p->tables64);
    for (int b = 0; b < B_NBUF; ++b)
        if (p->scratch[b]) (void)hipFree(p->scratch[b]);
    delete p;
}

size_t elem_bytes(const PlanSpec &s) { return s.f64 ? 16 : 8; }

// Generate every table in FP64 into `t64` (complex128 arena).
int generate_tables(const std::vector<TableReq> &tables, double2 *t64)
{
    for (const TableReq &t : tables) {
        double2 *dst = t64 + t.offset;
        hipError_t e = hipSuccess;
        switch (t.kind) {
        case TableReq::INNER: {
            StagesArg sa{};
            sa.nst = t.nst;
            for (int s = 0; s < t.nst; ++s) sa.st[s] = t.st[s];
            e = gen_inner(dst, sa, t.count, nullptr);
            break;
        }
        case TableReq::RANGE: e = gen_range(dst, t.N, t.e0, t.step, t.count, nullptr); break;
        case TableReq::CHIRP: e = gen_chirp(dst, t.N, t.count, nullptr); break;
        case TableReq::BFILTER: {
            // FFT_M of the wrapped conjugate chirp, computed with an FP64 plan of this library
            const int64_t n = t.N, M = t.count;
            double2 *tmp = nullptr;
            if (dev_malloc(reinterpret_cast<void **>(&tmp), size_t(M + n) * sizeof(double2)) != hipSuccess)
                return fail(FFT_ERR_ALLOC, "Bluestein filter scratch");
            double2 *chirp = tmp + M;
            e = gen_chirp(chirp, n, n, nullptr);
            if (e == hipSuccess) e = gen_bwrap(tmp, chirp, n, M, nullptr);
            int st = FFT_OK;
            if (e == hipSuccess) {
                fft_plan sub = fft_plan_create(1, &M, 1, FFT_C2C, FFT_FORWARD, FFT_F64);
                if (!sub) {
                    st = g_status;
                } else {
                    st = fft_execute(sub, tmp, dst, nullptr);
                    if (st == FFT_OK && hipStreamSynchronize(nullptr) != hipSuccess) st = FFT_ERR_HIP;
                    fft_plan_destroy(sub);
                }
            }
            (void)hipFree(tmp);
            if (st != FFT_OK) return fail(st, "Bluestein filter: " + g_msg);
            break;
        }
        }
        if (e != hipSuccess) return fail(FFT_ERR_HIP, std::string("table generation: ") + hipGetErrorString(e));
    }
    return FFT_OK;
}

fft_plan create_from_spec(PlanSpec &&spec)
{
    fft_plan p = new (std::nothrow) fft_plan_s();
    if (!p) {
        fail(FFT_ERR_ALLOC, "host allocation");
        return nullptr;
    }
    p->spec = std::move(spec);
    PlanSpec &sp = p->spec;
    const size_t eb = elem_bytes(sp);
    double2 *t64 = nullptr;
    HIP_TRY(hipGetDevice(&p->device));
    if (sp.table_elems > 0) {
        HIP_TRY(dev_malloc(reinterpret_cast<void **>(&t64), size_t(sp.table_elems) * sizeof(double2)));
        if (generate_tables(sp.tables, t64) != FFT_OK) goto fail_label;
        p->tables64 = t64;
        t64 = nullptr;
        if (sp.f64) {
            p->tables = p->tables64;
        } else {
            HIP_TRY(dev_malloc(&p->tables, size_t(sp.table_elems) * eb));
            HIP_TRY(convert_d2f(static_cast<float2 *>(p->tables), static_cast<const double2 *>(p->tables64),
                                sp.table_elems, nullptr));
            p->device_bytes += sp.table_elems * int64_t(eb);
        }
        p->device_bytes += sp.table_elems * int64_t(sizeof(double2));
    }
    for (int b = B_S0; b < B_NBUF; ++b)
        if (sp.scratch_elems[b] > 0) {
            HIP_TRY(dev_malloc(&p->scratch[b], size_t(sp.scratch_elems[b]) * eb));
            p->device_bytes += sp.scratch_elems[b] * int64_t(eb);
        }
    // bind table pointers into the launch arguments
    for (std::vector<Op> *list : {&sp.ops, &sp.ops_inplace, &sp.tail_ops, &sp.tail_ops_inplace})
        for (Op &op : *list) {
            auto ptr = [&](int id) -> const void * {
                return id < 0 ? nullptr : static_cast<const char *>(p->tables) + sp.tables[id].offset * int64_t(eb);
            };
            auto ptr64 = [&](int id) -> const void * {
                return id < 0 ? nullptr
                              : static_cast<const char *>(p->tables64) +
                                    sp.tables[id].offset * int64_t(sizeof(double2));
            };
            op.pa.itw = ptr(op.t_itw);
            op.pa.tw_lo = ptr64(op.t_lo);
            op.pa.tw_hi = ptr64(op.t_hi);
            op.pa.aux = ptr(op.t_aux);
            op.pa.aux2 = ptr(op.t_aux2);
            op.la.tab = ptr(op.t_tab);
            op.la.tab2 = ptr(op.t_tab2);
            if (op.type == OP_PASS) HIP_TRY(prepare_pass(op.pa, sp.f64));
        }
    HIP_TRY(hipStreamSynchronize(nullptr));
    if (t64) (void)hipFree(t64);
    t64 = nullptr;
    p->desc = sp.describe();
    g_status = FFT_OK;
    g_msg.clear();
    return p;
fail_label:
    if (t64) (void)hipFree(t64);
    free_plan(p);
    return nullptr;
}

// Kernel-node parameters of ragged phase `ph` with buffers in / out bound.  `ga` and
// `kargs` are the caller's storage for the argument block (hipGraph copies them).
hipKernelNodeParams phase_params(const fft_plan p, size_t ph, const void *in, void *out, RaggedArgs &ga,
                                 void **kargs)
{
    const Many *m = p->many;
    ga = RaggedArgs{};
    ga.blocks = m->blocks + m->phase_first[ph];
    ga.classes = m->classes;
    ga.ops = m->ops;
    ga.in = in;
    ga.out = out;
    ga.scratch = m->scratch;
    kargs[0] = &ga;
    hipKernelNodeParams kp{};
    kp.func = const_cast<void *>(ragged_kernel(p->spec.f64));
    kp.gridDim = dim3(m->phase_blocks[ph]);
    kp.blockDim = dim3(uint32_t(m->block));
    kp.sharedMemBytes = unsigned(m->lds);
    kp.kernelParams = kargs;
    kp.extra = nullptr;
    return kp;
}

// The ragged plan's graph, recorded and instantiated once at plan creation: one
// kernel node per phase, in order, with no buffers bound yet.
int build_many_graph(fft_plan p)
{
    Many *m = p->many;
    if (hipGraphCreate(&m->graph, 0) != hipSuccess) return fail(FFT_ERR_HIP, "hipGraphCreate");
    hipGraphNode_t prev = nullptr;
    for (size_t ph = 0; ph < m->phase_first.size(); ++ph) {
        RaggedArgs ga;
        void *kargs[1];
        const hipKernelNodeParams kp = phase_params(p, ph, nullptr, nullptr, ga, kargs);
        hipGraphNode_t node = nullptr;
        if (hipGraphAddKernelNode(&node, m->graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp) != hipSuccess)
            return fail(FFT_ERR_HIP, "hipGraphAddKernelNode (ragged phase)");
        m->nodes.push_back(node);
        prev = node;
    }
    if (hipGraphInstantiate(&m->exec, m->graph, nullptr, nullptr, 0) != hipSuccess)
        return fail(FFT_ERR_HIP, "hipGraphInstantiate");
    return FFT_OK;
}

// Runs the phases on `stream`.  Outside a stream capture: one launch of the plan's
// instantiated graph, its kernel nodes re-bound in place (hipGraphExecKernelNodeSetParams)
// when the buffers differ from the previous call's.  Inside a capture (a graph cannot
// be launched into a capturing stream): the same phase kernels launched one by one, so
// the caller's graph records them as its own nodes.  Nothing is allocated either way.
int execute_many(fft_plan p, const void *in, void *out, hipStream_t stream)
{
    Many *m = p->many;
    if (in == out) return fail(FFT_ERR_INVALID_ARG, "ragged plans run out of place");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
        return fail(FFT_ERR_INVALID_ARG, "plan was created on another device");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cs) != hipSuccess) return fail(FFT_ERR_HIP, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone) {
        for (size_t ph = 0; ph < m->phase_first.size(); ++ph) {
            RaggedArgs ga;
            void *kargs[1];
            const hipKernelNodeParams kp = phase_params(p, ph, in, out, ga, kargs);
            const hipError_t e = hipLaunchKernel(kp.func, kp.gridDim, kp.blockDim, kp.kernelParams,
                                                 kp.sharedMemBytes, stream);
            if (e != hipSuccess) return fail(FFT_ERR_HIP, std::string("ragged phase launch: ") + hipGetErrorString(e));
        }
        return FFT_OK;
    }
    if (m->g_in != in || m->g_out != out) {
        for (size_t ph = 0; ph < m->nodes.size(); ++ph) {
            RaggedArgs ga;
            void *kargs[1];
            hipKernelNodeParams kp = phase_params(p, ph, in, out, ga, kargs);
            if (hipGraphExecKernelNodeSetParams(m->exec, m->nodes[ph], &kp) != hipSuccess) {
                m->g_in = nullptr; // some nodes may be re-bound: bind every node next time
                m->g_out = nullptr;
                return fail(FFT_ERR_HIP, "hipGraphExecKernelNodeSetParams (ragged phase)");
            }
        }
        m->g_in = in;
        m->g_out = out;
    }
    const hipError_t e = hipGraphLaunch(m->exec, stream);
    if (e != hipSuccess) return fail(FFT_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    return FFT_OK;
}

} // namespace

namespace mifft {
// the thread-local error state, for entry points defined in other sources
int set_error(int status, const std::string &msg) { return fail(status, msg); }

CreateScope::CreateScope()
{
    if (g_create_depth++ == 0) {
        const char *e = std::getenv("MIFFT_TEST_FAIL_ALLOC");
        g_fail_at = e ? std::atoll(e) : 0;
        g_alloc_seq = 0;
    }
}
CreateScope::~CreateScope() { --g_create_depth; }

hipError_t dev_malloc(void **ptr, size_t bytes)
{
    if (g_fail_at > 0 && ++g_alloc_seq == g_fail_at) {
        *ptr = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(ptr, bytes);
}
} // namespace mifft

extern "C" {

fft_plan fft_plan_create(int rank, const int64_t *dims, int64_t batch, int kind, int direction, int dtype)
{
    const CreateScope scope;
    PlanSpec spec;
    std::string err;
    const int st = build_plan(rank, dims, batch, kind, direction, dtype, spec, err);
    if (st != FFT_OK) {
        fail(st, err);
        return nullptr;
    }
    return create_from_spec(std::move(spec));
}

int fft_execute(fft_plan p, const void *in, void *out, hipStream_t stream)
{
    if (!p) return fail(FFT_ERR_INVALID_ARG, "NULL plan");
    if (!in || !out) return fail(FFT_ERR_INVALID_ARG, "NULL buffer");
    if (p->many) return execute_many(p, in, out, stream);
    const PlanSpec &sp = p->spec;
    if (sp.kind != FFT_C2C && in == out) return fail(FFT_ERR_INVALID_ARG, "only C2C plans run in place");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
        return fail(FFT_ERR_INVALID_ARG, "plan was created on another device");
    // a chunked plan runs its op list once per chunk of transforms, each chunk's buffers
    // offset by the chunk's first transform; the scratch is shared by the chunks
    const bool inplace = in == out;
    const int64_t chunk = sp.chunk > 0 ? sp.chunk : sp.batch;
    const int64_t rb = sp.f64 ? 8 : 4;
    const int64_t in_eb = (sp.kind == FFT_C2C || sp.kind == FFT_C2R) ? 2 * rb : rb;
    const int64_t out_eb = (sp.kind == FFT_C2C || sp.kind == FFT_R2C) ? 2 * rb : rb;
    for (int64_t first = 0; first < sp.batch; first += chunk) {
        const bool tail = sp.batch - first < chunk;
        const std::vector<Op> &plain = tail ? sp.tail_ops : sp.ops;
        const std::vector<Op> &inpl = tail ? sp.tail_ops_inplace : sp.ops_inplace;
        const std::vector<Op> &ops = (inplace && !inpl.empty()) ? inpl : plain;
        void *buf[B_NBUF];
        buf[B_IN] = static_cast<char *>(const_cast<void *>(in)) + first * sp.in_dist * in_eb;
        buf[B_OUT] = static_cast<char *>(out) + first * sp.out_dist * out_eb;
        for (int b = B_S0; b < B_NBUF; ++b) buf[b] = p->scratch[b];
        for (const Op &op : ops) {
            hipError_t e;
            if (op.type == OP_PASS)
                e = launch_pass(op.pa, sp.f64, buf[op.src], buf[op.dst], stream);
            else
                e = launch_line(op.type, op.la, sp.f64, buf[op.src], buf[op.dst], op.grid, op.block, stream);
            if (e != hipSuccess) return fail(FFT_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
        }
    }
    return FFT_OK;
}

void fft_plan_destroy(fft_plan p) { free_plan(p); }

fft_plan fft_plan_create_many(int64_t count, const int64_t *lengths, const int64_t *in_offsets,
                              const int64_t *out_offsets, int kind, int direction, int dtype)
{
    const CreateScope scope;
    if (count < 1 || count > (int64_t(1) << 30) || !lengths || !in_offsets || !out_offsets) {
        fail(FFT_ERR_INVALID_ARG, "count must be in [1, 2^30] and lengths/offsets non-NULL");
        return nullptr;
    }
    for (int64_t t = 0; t < count; ++t)
        if (in_offsets[t] < 0 || out_offsets[t] < 0 || lengths[t] < 1 ||
            in_offsets[t] + lengths[t] > (int64_t(1) << 32) || out_offsets[t] + lengths[t] > (int64_t(1) << 32)) {
            fail(FFT_ERR_INVALID_ARG, "lengths must be >= 1 and offsets non-negative, below 2^32 elements");
            return nullptr;
        }
    fft_plan p = new (std::nothrow) fft_plan_s();
    Many *m = new (std::nothrow) Many();
    if (!p || !m) {
        delete p;
        delete m;
        fail(FFT_ERR_ALLOC, "host allocation");
        return nullptr;
    }
    p->many = m;
    std::string err;
    int st = build_many(count, lengths, kind, direction, dtype, m->ms, err);
    if (st != FFT_OK) {
        fail(st, err);
        free_plan(p);
        return nullptr;
    }
    ManySpec &ms = m->ms;
    p->spec.kind = FFT_C2C;
    p->spec.dtype = dtype;
    p->spec.f64 = ms.f64;
    const size_t eb = ms.f64 ? 16 : 8;
    double2 *t64 = nullptr;
    std::vector<RagOp> hops;
    std::vector<RagClass> hcls;
    std::vector<int64_t> scr_off;
    std::vector<RagBlock> hblocks;
    RaggedSchedule sched;
    int64_t scr_total = 0;
    int64_t max_lds = 16;
    HIP_TRY(hipGetDevice(&p->device));
    if (ms.table_elems > 0) {
        HIP_TRY(dev_malloc(reinterpret_cast<void **>(&t64), size_t(ms.table_elems) * sizeof(double2)));
        p->tables64 = t64;
        t64 = nullptr;
        if (generate_tables(ms.tables, static_cast<double2 *>(p->tables64)) != FFT_OK) goto fail_label;
        if (ms.f64) {
            p->tables = p->tables64;
        } else {
            HIP_TRY(dev_malloc(&p->tables, size_t(ms.table_elems) * eb));
            HIP_TRY(convert_d2f(static_cast<float2 *>(p->tables), static_cast<const double2 *>(p->tables64),
                                ms.table_elems, nullptr));
        }
    }
    // ops with bound tables
    for (const Op &op : ms.ops) {
        RagOp r{};
        r.type = op.type;
        r.src = op.src;
        r.dst = op.dst;
        r.pa = op.pa;
        r.la = op.la;
        auto ptr = [&](int id) -> const void * {
            return id < 0 ? nullptr : static_cast<const char *>(p->tables) + ms.tables[id].offset * int64_t(eb);
        };
        auto ptr64 = [&](int id) -> const void * {
            return id < 0 ? nullptr
                          : static_cast<const char *>(p->tables64) + ms.tables[id].offset * int64_t(sizeof(double2));
        };
        r.pa.itw = ptr(op.t_itw);
        r.pa.tw_lo = ptr64(op.t_lo);
        r.pa.tw_hi = ptr64(op.t_hi);
        r.pa.aux = ptr(op.t_aux);
        r.pa.aux2 = ptr(op.t_aux2);
        r.la.tab = ptr(op.t_tab);
        r.la.tab2 = ptr(op.t_tab2);
        if (op.type == OP_PASS) {
            r.tiles = int32_t(op.pa.ntiles);
            max_lds = std::max<int64_t>(max_lds, op.pa.lds_bytes);
        } else {
            r.tiles = 1;
        }
        hops.push_back(r);
    }
    for (const ManySpec::Class &c : ms.classes) {
        RagClass rc{};
        rc.first_op = c.first_op;
        rc.nops = c.nops;
        for (int b = 0; b < B_NBUF; ++b) rc.sofs[b] = c.sofs[b];
        hcls.push_back(rc);
    }
    for (int64_t t = 0; t < count; ++t) {
        scr_off.push_back(scr_total);
        scr_total += ms.classes[size_t(ms.xform_class[size_t(t)])].scratch;
    }
    {
        std::string serr;
        const int sst = schedule_many(ms, sched, serr);
        if (sst != FFT_OK) {
            fail(sst, serr);
            goto fail_label;
        }
    }
    // device blocks carry the offsets they need (no lookups through the transform)
    for (const RaggedSchedule::Block &sb : sched.blocks) {
        const int cls = ms.xform_class[sb.t];
        const ManySpec::Class &c = ms.classes[size_t(cls)];
        const int64_t offs[B_NBUF] = {in_offsets[sb.t], out_offsets[sb.t], 0, 0, 0, 0, 0};
        auto off = [&](int b) { return b < 2 ? offs[b] : scr_off[sb.t] + c.sofs[b]; };
        RagBlock rb{};
        if (sb.whole) {
            rb.off[0] = in_offsets[sb.t];
            rb.off[1] = out_offsets[sb.t];
            rb.off[2] = scr_off[sb.t];
            rb.op = uint32_t(cls);
            rb.part = kRagWhole;
        } else {
            const Op &op = ms.ops[size_t(c.first_op) + sb.op];
            rb.off[0] = off(op.src);
            rb.off[1] = off(op.dst);
            rb.op = uint32_t(c.first_op) + sb.op;
            rb.part = sb.part;
            if (op.dst == B_IN || (rb.part & kRagWhole)) {
                fail(FFT_ERR_INTERNAL, "ragged op writes its input or has too many parts");
                goto fail_label;
            }
        }
        hblocks.push_back(rb);
    }
    m->phase_first = sched.phase_first;
    m->phase_blocks = sched.phase_blocks;
    m->count = uint32_t(count);
    HIP_TRY(dev_malloc(reinterpret_cast<void **>(&m->ops), hops.size() * sizeof(RagOp)));
    HIP_TRY(hipMemcpy(m->ops, hops.data(), hops.size() * sizeof(RagOp), hipMemcpyHostToDevice));
    HIP_TRY(dev_malloc(reinterpret_cast<void **>(&m->classes), hcls.size() * sizeof(RagClass)));
    HIP_TRY(hipMemcpy(m->classes, hcls.data(), hcls.size() * sizeof(RagClass), hipMemcpyHostToDevice));
    HIP_TRY(dev_malloc(reinterpret_cast<void **>(&m->blocks), hblocks.size() * sizeof(RagBlock)));
    HIP_TRY(hipMemcpy(m->blocks, hblocks.data(), hblocks.size() * sizeof(RagBlock), hipMemcpyHostToDevice));
    if (scr_total > 0) HIP_TRY(dev_malloc(&m->scratch, size_t(scr_total) * eb));
    m->lds = size_t(max_lds);
    if (m->lds > 64 * 1024)
        HIP_TRY(hipFuncSetAttribute(ragged_kernel(ms.f64), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    int(m->lds)));
    p->device_bytes = ms.table_elems * int64_t(eb + (ms.f64 ? 0 : 16)) + scr_total * int64_t(eb) +
                      int64_t(hblocks.size() * sizeof(RagBlock));
    HIP_TRY(hipStreamSynchronize(nullptr));
    if (build_many_graph(p) != FFT_OK) goto fail_label;
    {
        std::ostringstream o;
        o << ms.describe() << sched.describe() << "  block=" << m->block << " lds=" << m->lds
          << " scratch_bytes=" << scr_total * int64_t(eb) << "\n";
        p->desc = o.str();
    }
    g_status = FFT_OK;
    g_msg.clear();
    return p;
fail_label:
    if (t64) (void)hipFree(t64);
    free_plan(p);
    return nullptr;
}

int fft_last_error(void) { return g_status; }

const char *fft_last_error_message(void) { return g_msg.c_str(); }

const char *fft_plan_describe(fft_plan p) { return p ? p->desc.c_str() : ""; }

int fft_plan_inspect(int rank, const int64_t *dims, int64_t batch, int kind, int direction, int dtype, char *buf,
                     size_t len)
{
    PlanSpec spec;
    std::string err;
    const int st = build_plan(rank, dims, batch, kind, direction, dtype, spec, err);
    const std::string s = st == FFT_OK ? spec.describe() : err;
    if (buf && len) {
        const size_t k = s.size() < len - 1 ? s.size() : len - 1;
        std::memcpy(buf, s.data(), k);
        buf[k] = '\0';
    }
    if (st != FFT_OK) fail(st, err);
    return st;
}

int fft_plan_inspect_many(int64_t count, const int64_t *lengths, int kind, int direction, int dtype, char *buf,
                          size_t len)
{
    ManySpec ms;
    RaggedSchedule sched;
    std::string err;
    int st = FFT_ERR_INVALID_ARG;
    if (count < 1 || count > (int64_t(1) << 30) || !lengths)
        err = "count must be in [1, 2^30] and lengths non-NULL";
    else
        st = build_many(count, lengths, kind, direction, dtype, ms, err);
    if (st == FFT_OK) st = schedule_many(ms, sched, err);
    const std::string s = st == FFT_OK ? ms.describe() + sched.describe() : err;
    if (buf && len) {
        const size_t k = s.size() < len - 1 ? s.size() : len - 1;
        std::memcpy(buf, s.data(), k);
        buf[k] = '\0';
    }
    if (st != FFT_OK) fail(st, err);
    return st;
}

int fft_tune_set(const char *entries, int replace) { return tune_set(entries, replace); }

int fft_tune_get(char *buf, size_t len)
{
    const std::string s = tune_dump();
    if (!buf || len == 0) return fail(FFT_ERR_INVALID_ARG, "buffer is NULL or empty");
    const size_t k = s.size() < len - 1 ? s.size() : len - 1;
    std::memcpy(buf, s.data(), k);
    buf[k] = '\0';
    if (s.size() > len - 1) return fail(FFT_ERR_INVALID_ARG, "tuning table does not fit the buffer");
    return FFT_OK;
}

int64_t fft_plan_device_bytes(fft_plan p) { return p ? p->device_bytes : 0; }

} // extern "C"
