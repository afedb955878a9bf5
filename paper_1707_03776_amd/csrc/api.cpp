// C ABI of the library (include/mifft.h): plan creation (planner + FP64 table
// generation on the GPU + scratch), execution (one launch per planned op on the
// caller's stream), destruction, and the thread-local error state.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
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
    void *many = nullptr;
};

namespace {

thread_local int g_status = FFT_OK;
thread_local std::string g_msg;

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

void free_plan(fft_plan p)
{
    if (!p) return;
    if (p->tables && p->tables != p->tables64) (void)hipFree(p->tables);
    if (p->tables64) (void)hipFree(p->tables64);
    for (int b = 0; b < B_NBUF; ++b)
        if (p->scratch[b]) (void)hipFree(p->scratch[b]);
    delete p;
}

size_t elem_bytes(const PlanSpec &s) { return s.f64 ? 16 : 8; }

// Generate every table in FP64 into `t64` (complex128 arena).
int generate_tables(const PlanSpec &sp, double2 *t64)
{
    for (const TableReq &t : sp.tables) {
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
            if (hipMalloc(&tmp, size_t(M + n) * sizeof(double2)) != hipSuccess)
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
        HIP_TRY(hipMalloc(&t64, size_t(sp.table_elems) * sizeof(double2)));
        if (generate_tables(sp, t64) != FFT_OK) goto fail_label;
        p->tables64 = t64;
        t64 = nullptr;
        if (sp.f64) {
            p->tables = p->tables64;
        } else {
            HIP_TRY(hipMalloc(&p->tables, size_t(sp.table_elems) * eb));
            HIP_TRY(convert_d2f(static_cast<float2 *>(p->tables), static_cast<const double2 *>(p->tables64),
                                sp.table_elems, nullptr));
            p->device_bytes += sp.table_elems * int64_t(eb);
        }
        p->device_bytes += sp.table_elems * int64_t(sizeof(double2));
    }
    for (int b = B_S0; b < B_NBUF; ++b)
        if (sp.scratch_elems[b] > 0) {
            HIP_TRY(hipMalloc(&p->scratch[b], size_t(sp.scratch_elems[b]) * eb));
            p->device_bytes += sp.scratch_elems[b] * int64_t(eb);
        }
    // bind table pointers into the launch arguments
    for (Op &op : sp.ops_inplace) {
        auto ptr = [&](int id) -> const void * {
            return id < 0 ? nullptr : static_cast<const char *>(p->tables) + sp.tables[id].offset * int64_t(eb);
        };
        auto ptr64 = [&](int id) -> const void * {
            return id < 0 ? nullptr
                          : static_cast<const char *>(p->tables64) + sp.tables[id].offset * int64_t(sizeof(double2));
        };
        op.pa.itw = ptr(op.t_itw);
        op.pa.tw_lo = ptr64(op.t_lo);
        op.pa.tw_hi = ptr64(op.t_hi);
        op.pa.aux = ptr(op.t_aux);
        op.la.tab = ptr(op.t_tab);
        op.la.tab2 = ptr(op.t_tab2);
    }
    for (Op &op : sp.ops) {
        auto ptr = [&](int id) -> const void * {
            return id < 0 ? nullptr : static_cast<const char *>(p->tables) + sp.tables[id].offset * int64_t(eb);
        };
        auto ptr64 = [&](int id) -> const void * {
            return id < 0 ? nullptr
                          : static_cast<const char *>(p->tables64) + sp.tables[id].offset * int64_t(sizeof(double2));
        };
        op.pa.itw = ptr(op.t_itw);
        op.pa.tw_lo = ptr64(op.t_lo);
        op.pa.tw_hi = ptr64(op.t_hi);
        op.pa.aux = ptr(op.t_aux);
        op.la.tab = ptr(op.t_tab);
        op.la.tab2 = ptr(op.t_tab2);
    }
    for (const std::vector<Op> *list : {&sp.ops, &sp.ops_inplace})
        for (const Op &op : *list)
            if (op.type == OP_PASS) HIP_TRY(prepare_pass(op.pa, sp.f64));
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

} // namespace

extern "C" {

fft_plan fft_plan_create(int rank, const int64_t *dims, int64_t batch, int kind, int direction, int dtype)
{
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
    if (p->many) return fail(FFT_ERR_UNSUPPORTED, "ragged plans are not available in this build");
    if (!in || !out) return fail(FFT_ERR_INVALID_ARG, "NULL buffer");
    const PlanSpec &sp = p->spec;
    if (sp.kind != FFT_C2C && in == out) return fail(FFT_ERR_INVALID_ARG, "R2C/C2R cannot run in place");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
        return fail(FFT_ERR_INVALID_ARG, "plan was created on another device");
    void *buf[B_NBUF];
    buf[B_IN] = const_cast<void *>(in);
    buf[B_OUT] = out;
    for (int b = B_S0; b < B_NBUF; ++b) buf[b] = p->scratch[b];
    const std::vector<Op> &ops = (in == out && !sp.ops_inplace.empty()) ? sp.ops_inplace : sp.ops;
    for (const Op &op : ops) {
        hipError_t e;
        if (op.type == OP_PASS)
            e = launch_pass(op.pa, sp.f64, buf[op.src], buf[op.dst], stream);
        else
            e = launch_line(op.type, op.la, sp.f64, buf[op.src], buf[op.dst], op.grid, op.block, stream);
        if (e != hipSuccess) return fail(FFT_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
    }
    return FFT_OK;
}

void fft_plan_destroy(fft_plan p) { free_plan(p); }

fft_plan fft_plan_create_many(int64_t count, const int64_t *lengths, const int64_t *in_offsets,
                              const int64_t *out_offsets, int kind, int direction, int dtype)
{
    (void)count;
    (void)lengths;
    (void)in_offsets;
    (void)out_offsets;
    (void)kind;
    (void)direction;
    (void)dtype;
    fail(FFT_ERR_UNSUPPORTED, "ragged plans are not available in this build");
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

int64_t fft_plan_device_bytes(fft_plan p) { return p ? p->device_bytes : 0; }

} // extern "C"
