// Pseudo-spectral Laplacian (include/mifft.h, fft_laplacian_*): an r2c plan, one
// element-wise multiply of the half spectrum by -|kappa|^2, a c2r plan.  The
// Laplacian is the operator of the paper's "Laplace equation" example and the
// spatial term of its acoustic wave equation ("Seismic Inversion Example"); here
// it is applied through its Fourier symbol rather than a stencil.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <new>
#include <string>
#include <vector>

#include "kernels.h"
#include "mifft.h"
#include "planner.h"

using mifft::set_error;

namespace {

// floor(n / d) for n, d < 2^32 with one 64-bit high product: m = ceil(2^64 / d) makes
// the error term n (m d - 2^64) / (d 2^64) smaller than 1/d, so the floor is exact
// (d = 1 would need m = 2^64 and is taken apart).
struct Divisor {
    uint32_t d;
    uint64_t m;
};

Divisor make_divisor(uint32_t d) { return Divisor{d, d > 1 ? ~uint64_t(0) / d + 1 : 0}; }

__device__ __forceinline__ uint32_t div_by(uint32_t n, const Divisor &v)
{
    return v.d == 1 ? n : uint32_t(__umul64hi(uint64_t(n), v.m));
}

__device__ __forceinline__ double freq_sq(uint32_t j, uint32_t n)
{
    const double f = 2u * j <= n ? double(j) : double(j) - double(n);
    return f * f;
}

template <typename R> struct Cplx;
template <> struct Cplx<float> { using T = float2; };
template <> struct Cplx<double> { using T = double2; };

__device__ __forceinline__ double symbol(uint32_t e, const Divisor &dh, const Divisor &d1, const Divisor &d0,
                                         double c0, double c1, double c2)
{
    const uint32_t r = div_by(e, dh);
    const uint32_t j = e - r * dh.d;
    const uint32_t r1 = div_by(r, d1);
    const uint32_t i1 = r - r1 * d1.d;
    const uint32_t i0 = r1 - div_by(r1, d0) * d0.d;
    // the last axis holds only j = 0..n/2: its frequency is j itself
    return -(c0 * freq_sq(i0, d0.d) + c1 * freq_sq(i1, d1.d) + c2 * double(j) * double(j));
}

// Bins per thread: 16 bytes per lane (two complex64 bins, one complex128 bin).
template <typename R> constexpr uint32_t kBinsPerThread = 16 / (2 * sizeof(R));

// spec: [batch][n0][n1][h] complex (the r2c layout of a rank-3 field; lower ranks
// take n0 = n1 = 1).  c[a] = (2 pi / L_a)^2.
template <typename R>
__global__ __launch_bounds__(256) void k_laplace_symbol(typename Cplx<R>::T *__restrict__ spec, uint32_t total,
                                                        Divisor dh, Divisor d1, Divisor d0, double c0, double c1,
                                                        double c2)
{
    constexpr uint32_t B = kBinsPerThread<R>;
    const uint64_t e64 = (uint64_t(blockIdx.x) * 256u + threadIdx.x) * B; // no wrap near 2^32
    if (e64 >= total) return;
    const uint32_t e = uint32_t(e64);
    if constexpr (B == 2) {
        if (e + 1u < total) {
            // e is even and the buffer 256-byte aligned: one 16-byte access for two bins
            float4 v = reinterpret_cast<float4 *>(spec)[e / 2u];
            const float s0 = float(symbol(e, dh, d1, d0, c0, c1, c2));
            const float s1 = float(symbol(e + 1u, dh, d1, d0, c0, c1, c2));
            v.x *= s0;
            v.y *= s0;
            v.z *= s1;
            v.w *= s1;
            reinterpret_cast<float4 *>(spec)[e / 2u] = v;
            return;
        }
    }
    const R s = R(symbol(e, dh, d1, d0, c0, c1, c2));
    typename Cplx<R>::T v = spec[e];
    v.x *= s;
    v.y *= s;
    spec[e] = v;
}

} // namespace

struct fft_laplacian_s {
    fft_plan fwd = nullptr, inv = nullptr;
    void *spec = nullptr;
    void *sym = nullptr; // symbol tables of the fused form (null: the multiply runs on its own)
    uint32_t spec_elems = 0;
    int f64 = 0, device = 0;
    Divisor dh{}, d1{}, d0{};
    double c[3] = {0, 0, 0};
    std::string desc;
};

namespace {

// Fuses the multiply into the first pass of the c2r plan when that pass is a
// specialised kernel over one whole axis of the half spectrum and its columns run over
// the other axes (then the batch): the symbol is separable, -|kappa|^2 = sum over axes
// of -c_a f_a^2, so the pass scales each point it loads by S_p[p] + S_0[d0] (+ S_1[d1])
// from three small FP64 tables.  Returns false (and leaves the plan alone) otherwise.
bool fuse_symbol(fft_laplacian op, const int64_t n[3], int64_t h, hipError_t &err)
{
    err = hipSuccess;
    std::vector<mifft::PassArgs *> firsts = mifft::plan_first_passes(op->inv);
    if (firsts.empty()) return false;
    // the half-spectrum layout [batch][n0][n1][h]: axis sizes and strides (elements)
    const int64_t sz[3] = {n[0], n[1], h}, st[3] = {n[1] * h, h, 1}, field = n[0] * n[1] * h;
    // the axis a dim of `size` points `stride` apart runs over: the whole axis, or the
    // outermost axis merged with the batch (the planner folds dims whose strides chain)
    auto axis_of = [&](int64_t stride, int64_t size, bool exact) {
        for (int a = 0; a < 3; ++a)
            if (sz[a] > 1 && st[a] == stride &&
                (size == sz[a] || (!exact && size % sz[a] == 0 && st[a] * sz[a] == field)))
                return a;
        return -1;
    };
    int ap = -1, a0 = -1, a1 = -1, cd = 0;
    int64_t c0 = 0, c1max = 0;
    for (const mifft::PassArgs *pa : firsts) {
        if (pa->pro != mifft::PRO_PLAIN || pa->epi != mifft::EPI_PLAIN || pa->shape < 0 || pa->mode != 0 ||
            pa->tw_dim >= 0 || pa->ncd < 1 || pa->ncd > 3)
            return false;
        const int p = axis_of(pa->rin, pa->L, true), q0 = axis_of(pa->cin[0], pa->csz[0], false);
        const int q1 = pa->ncd > 1 ? axis_of(pa->cin[1], pa->csz[1], false) : -1;
        const int c = q1 >= 0 ? 2 : 1;
        // every dim past the symbol's column dims is the batch
        for (int d = c; d < pa->ncd; ++d)
            if (pa->cin[d] != field) return false;
        if (p < 0 || q0 < 0 || (cd && (p != ap || q0 != a0 || q1 != a1 || c != cd || pa->csz[0] != c0)))
            return false;
        ap = p;
        a0 = q0;
        a1 = q1;
        cd = c;
        c0 = pa->csz[0];
        if (c == 2) c1max = std::max<int64_t>(c1max, pa->csz[1]);
    }
    // the three axes named once each, and every axis longer than 1 among them
    for (int a = 0; a < 3; ++a) {
        const int hits = (ap == a) + (a0 == a) + (a1 == a);
        if (hits > 1 || (sz[a] > 1 && hits != 1)) return false;
    }
    // S_p over the pass's points, S_0 over csz[0] columns, S_1 over the widest csz[1];
    // a dim merged with the batch repeats its axis' values
    std::vector<double> tab;
    auto axis_table = [&](int a, int64_t count) {
        for (int64_t i = 0; i < count; ++i) {
            const int64_t j = i % sz[a];
            // the last axis holds only j = 0..n/2: its frequency is j itself
            const double f = a == 2 || 2 * j <= sz[a] ? double(j) : double(j) - double(sz[a]);
            tab.push_back(-(op->c[a] * f * f));
        }
    };
    axis_table(ap, sz[ap]);
    axis_table(a0, c0);
    if (cd == 2) axis_table(a1, c1max);
    err = mifft::dev_malloc(&op->sym, tab.size() * sizeof(double));
    if (err == hipSuccess) err = hipMemcpy(op->sym, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice);
    if (err != hipSuccess) return false;
    for (mifft::PassArgs *pa : firsts) {
        mifft::PassArgs t = *pa;
        t.pro = mifft::PRO_SYM;
        t.aux = op->sym;
        t.sym_cd = cd;
        err = mifft::prepare_pass(t, op->f64);
        if (err != hipSuccess) return false;
        *pa = t;
    }
    mifft::plan_refresh_description(op->inv);
    return true;
}

} // namespace

extern "C" {

void fft_laplacian_destroy(fft_laplacian op)
{
    if (!op) return;
    fft_plan_destroy(op->fwd);
    fft_plan_destroy(op->inv);
    if (op->spec) (void)hipFree(op->spec);
    if (op->sym) (void)hipFree(op->sym);
    delete op;
}

fft_laplacian fft_laplacian_create(int rank, const int64_t *dims, int64_t batch, const double *lengths, int dtype)
{
    const mifft::CreateScope scope; // the test hook's allocation count spans both plans and the buffer
    if (rank < 1 || rank > 3 || !dims || !lengths) {
        set_error(FFT_ERR_INVALID_ARG, "rank must be 1, 2 or 3 and dims/lengths non-NULL");
        return nullptr;
    }
    if (dtype != FFT_F32 && dtype != FFT_F64) {
        set_error(FFT_ERR_INVALID_ARG, "the Laplacian takes FFT_F32 or FFT_F64");
        return nullptr;
    }
    for (int a = 0; a < rank; ++a)
        if (!(std::isfinite(lengths[a]) && lengths[a] > 0.0)) {
            set_error(FFT_ERR_INVALID_ARG, "periods must be finite and positive");
            return nullptr;
        }
    fft_laplacian op = new (std::nothrow) fft_laplacian_s();
    if (!op) {
        set_error(FFT_ERR_ALLOC, "host allocation");
        return nullptr;
    }
    // the two plans validate dims and batch and enforce the element limits
    op->fwd = fft_plan_create(rank, dims, batch, FFT_R2C, FFT_FORWARD, dtype);
    if (op->fwd) op->inv = fft_plan_create(rank, dims, batch, FFT_C2R, FFT_INVERSE, dtype);
    if (!op->inv) {
        const int st = fft_last_error();
        const std::string msg = fft_last_error_message();
        fft_laplacian_destroy(op);
        set_error(st, msg);
        return nullptr;
    }
    int64_t n[3] = {1, 1, 1};
    double L[3] = {1, 1, 1};
    for (int a = 0; a < rank; ++a) {
        n[3 - rank + a] = dims[a];
        L[3 - rank + a] = lengths[a];
    }
    const int64_t h = n[2] / 2 + 1;
    const int64_t elems = batch * n[0] * n[1] * h; // below 2^32 - 1: the r2c plan exists
    op->spec_elems = uint32_t(elems);
    op->f64 = dtype == FFT_F64;
    op->dh = make_divisor(uint32_t(h));
    op->d1 = make_divisor(uint32_t(n[1]));
    op->d0 = make_divisor(uint32_t(n[0]));
    for (int a = 0; a < 3; ++a) {
        const double w = 2.0 * M_PI / L[a];
        op->c[a] = w * w;
    }
    hipError_t e = hipGetDevice(&op->device);
    if (e == hipSuccess) e = mifft::dev_malloc(&op->spec, size_t(elems) * (op->f64 ? sizeof(double2) : sizeof(float2)));
    if (e != hipSuccess) {
        fft_laplacian_destroy(op);
        set_error(e == hipErrorOutOfMemory ? FFT_ERR_ALLOC : FFT_ERR_HIP,
                  std::string("half-spectrum buffer: ") + hipGetErrorString(e));
        return nullptr;
    }
    // the multiply fused into the c2r plan's first pass where that pass allows it
    // (MIFFT_LAPLACE_UNFUSED=1 keeps it a kernel of its own)
    const bool fused = std::getenv("MIFFT_LAPLACE_UNFUSED") == nullptr && fuse_symbol(op, n, h, e);
    if (e != hipSuccess) {
        fft_laplacian_destroy(op);
        set_error(e == hipErrorOutOfMemory ? FFT_ERR_ALLOC : FFT_ERR_HIP,
                  std::string("symbol tables: ") + hipGetErrorString(e));
        return nullptr;
    }
    op->desc = std::string("laplacian: r2c, multiply by -|kappa|^2 (") + std::to_string(elems) +
               " half-spectrum elements" + (fused ? ", in the c2r plan's first pass" : "") + "), c2r\n" +
               fft_plan_describe(op->fwd) + fft_plan_describe(op->inv);
    return op;
}

int fft_laplacian_execute(fft_laplacian op, const void *in, void *out, hipStream_t stream)
{
    if (!op) return set_error(FFT_ERR_INVALID_ARG, "NULL operator");
    if (!in || !out) return set_error(FFT_ERR_INVALID_ARG, "NULL buffer");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != op->device)
        return set_error(FFT_ERR_INVALID_ARG, "operator was created on another device");
    int st = fft_execute(op->fwd, in, op->spec, stream);
    if (st != FFT_OK) return st;
    if (op->sym) return fft_execute(op->inv, op->spec, out, stream); // the multiply rides in its first pass
    const uint64_t per_block = 256u * uint64_t(op->f64 ? kBinsPerThread<double> : kBinsPerThread<float>);
    const uint32_t blocks = uint32_t((uint64_t(op->spec_elems) + per_block - 1) / per_block);
    if (op->f64)
        hipLaunchKernelGGL(k_laplace_symbol<double>, dim3(blocks), dim3(256), 0, stream,
                           static_cast<double2 *>(op->spec), op->spec_elems, op->dh, op->d1, op->d0, op->c[0],
                           op->c[1], op->c[2]);
    else
        hipLaunchKernelGGL(k_laplace_symbol<float>, dim3(blocks), dim3(256), 0, stream,
                           static_cast<float2 *>(op->spec), op->spec_elems, op->dh, op->d1, op->d0, op->c[0],
                           op->c[1], op->c[2]);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(FFT_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
    return fft_execute(op->inv, op->spec, out, stream);
}

const char *fft_laplacian_describe(fft_laplacian op) { return op ? op->desc.c_str() : ""; }

} // extern "C"
