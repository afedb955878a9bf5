// gfx950 kernels around the Stockham passes: the element-wise steps (Bluestein,
// real-data staging, DCT reordering and twists), the FP64 table generators, and
// the launchers of every kernel family (the pass kernels themselves are
// instantiated in pass_*.hip, mfma.hip and ragged.hip).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "line_device.h"
#include "shapes.h"

#include <algorithm>

namespace mifft {

// kernel tables of the pass flavours (pass_*.hip, mfma.hip)
const void *pass_kernel_f32_plain(int shape);
const void *pass_kernel_f32_c2r(int shape);
const void *pass_kernel_f32_r2c(int shape);
const void *pass_kernel_f64_plain(int shape);
const void *pass_kernel_f64_c2r(int shape);
const void *pass_kernel_f64_r2c(int shape);
const void *mfma_kernel(int nsplit, int shape);

template <typename R, int TYPE>
__global__ void __launch_bounds__(256) k_line(const LineArgs l, const void *in, void *out)
{
    const int64_t total = line_total(TYPE, l);
    for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += int64_t(gridDim.x) * blockDim.x)
        line_elem<R, TYPE>(l, g, in, out);
}

// ----------------------------------------------------------------------------- FP64 tables

// exp(-2 pi i e / N) in FP64, the exponent reduced exactly to (-N/2, N/2]
__device__ __forceinline__ double2 root_fp64(int64_t N, int64_t e)
{
    e %= N;
    if (e < 0) e += N;
    if (2 * e > N) e -= N;
    double s, c;
    sincospi(-2.0 * double(e) / double(N), &s, &c);
    return double2{c, s};
}

__global__ void k_gen_range(double2 *dst, int64_t N, int64_t e0, int64_t step, int64_t count)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = root_fp64(N, e0 + i * step);
}

__global__ void k_gen_inner(double2 *dst, StagesArg st)
{
    for (int s = 1; s < st.nst; ++s) {
        const int r = st.st[s].r, ns = st.st[s].ns;
        const int64_t cnt = int64_t(ns) * (r - 1);
        for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt;
             i += int64_t(gridDim.x) * blockDim.x) {
            const int64_t m = i / (r - 1), k = i % (r - 1) + 1;
            dst[st.st[s].tw + i] = root_fp64(int64_t(ns) * r, k * m);
        }
    }
}

// Bluestein chirp w_j = exp(-pi i j^2 / n) = W_{2n}^{j^2 mod 2n}, j^2 reduced exactly
__global__ void k_gen_chirp(double2 *dst, int64_t n, int64_t count)
{
    for (int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < count; j += int64_t(gridDim.x) * blockDim.x) {
        const uint64_t jj = uint64_t(j) % uint64_t(2 * n);
        const uint64_t e = (jj * jj) % uint64_t(2 * n);
        dst[j] = root_fp64(2 * n, int64_t(e));
    }
}

// b_m = conj(w_m) for m < n, wrapped so b_{M-m} = b_m, zero elsewhere
__global__ void k_gen_bwrap(double2 *dst, const double2 *chirp, int64_t n, int64_t M)
{
    for (int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; m < M; m += int64_t(gridDim.x) * blockDim.x) {
        double2 v{0.0, 0.0};
        if (m < n)
            v = double2{chirp[m].x, -chirp[m].y};
        else if (M - m < n)
            v = double2{chirp[M - m].x, -chirp[M - m].y};
        dst[m] = v;
    }
}

__global__ void k_d2f(float2 *dst, const double2 *src, int64_t count)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = float2{float(src[i].x), float(src[i].y)};
}

// ----------------------------------------------------------------------------- launchers

namespace {
template <typename R> const void *pass_kernel_for(const PassArgs &a);
template <> const void *pass_kernel_for<float>(const PassArgs &a)
{
    if (a.mode >= 2 && a.mshape >= 0) return mfma_kernel(a.mode, a.mshape);
    // fused Bluestein steps: the runtime-radix kernel, which reads the flavour from a
    if (a.pro == PRO_BPAD || a.epi == EPI_BMUL || a.epi == EPI_BEXT) return pass_kernel_f32_plain(-1);
    if (a.pro == PRO_C2R) return pass_kernel_f32_c2r(a.shape);
    if (a.epi == EPI_R2C) return pass_kernel_f32_r2c(a.shape);
    return pass_kernel_f32_plain(a.shape);
}
template <> const void *pass_kernel_for<double>(const PassArgs &a)
{
    if (a.pro == PRO_BPAD || a.epi == EPI_BMUL || a.epi == EPI_BEXT) return pass_kernel_f64_plain(-1);
    if (a.pro == PRO_C2R) return pass_kernel_f64_c2r(a.shape);
    if (a.epi == EPI_R2C) return pass_kernel_f64_r2c(a.shape);
    return pass_kernel_f64_plain(a.shape);
}

template <typename R>
hipError_t launch_pass_t(const PassArgs &a, const void *in, void *out, hipStream_t st)
{
    const void *k = pass_kernel_for<R>(a);
    PassArgs args = a;
    const void *pin = in;
    void *pout = out;
    void *kargs[] = {&args, &pin, &pout};
    const uint32_t grid = uint32_t(a.grid > 0 ? a.grid : a.ntiles);
    return hipLaunchKernel(k, dim3(grid), dim3(uint32_t(a.threads)), kargs, size_t(a.lds_bytes), st);
}

template <typename R>
hipError_t launch_line_t(int type, const LineArgs &l, const void *in, void *out, int64_t grid, int block,
                         hipStream_t st)
{
    const dim3 g{uint32_t(grid)}, b{uint32_t(block)};
    switch (type) {
    case LINE_CHIRP_PAD: hipLaunchKernelGGL((k_line<R, LINE_CHIRP_PAD>), g, b, 0, st, l, in, out); break;
    case LINE_MUL_CONJ: hipLaunchKernelGGL((k_line<R, LINE_MUL_CONJ>), g, b, 0, st, l, in, out); break;
    case LINE_CHIRP_EXTRACT: hipLaunchKernelGGL((k_line<R, LINE_CHIRP_EXTRACT>), g, b, 0, st, l, in, out); break;
    case LINE_R2C_TWIST: hipLaunchKernelGGL((k_line<R, LINE_R2C_TWIST>), g, b, 0, st, l, in, out); break;
    case LINE_C2R_UNTWIST: hipLaunchKernelGGL((k_line<R, LINE_C2R_UNTWIST>), g, b, 0, st, l, in, out); break;
    case LINE_REAL_TO_CPLX: hipLaunchKernelGGL((k_line<R, LINE_REAL_TO_CPLX>), g, b, 0, st, l, in, out); break;
    case LINE_HALF_COPY: hipLaunchKernelGGL((k_line<R, LINE_HALF_COPY>), g, b, 0, st, l, in, out); break;
    case LINE_HERM_EXPAND: hipLaunchKernelGGL((k_line<R, LINE_HERM_EXPAND>), g, b, 0, st, l, in, out); break;
    case LINE_CPLX_TO_REAL: hipLaunchKernelGGL((k_line<R, LINE_CPLX_TO_REAL>), g, b, 0, st, l, in, out); break;
    case LINE_DCT2_PRE: hipLaunchKernelGGL((k_line<R, LINE_DCT2_PRE>), g, b, 0, st, l, in, out); break;
    case LINE_DCT2_POST: hipLaunchKernelGGL((k_line<R, LINE_DCT2_POST>), g, b, 0, st, l, in, out); break;
    case LINE_DCT3_PRE: hipLaunchKernelGGL((k_line<R, LINE_DCT3_PRE>), g, b, 0, st, l, in, out); break;
    case LINE_DCT3_POST: hipLaunchKernelGGL((k_line<R, LINE_DCT3_POST>), g, b, 0, st, l, in, out); break;
    case LINE_DCT2_TWPOST: hipLaunchKernelGGL((k_line<R, LINE_DCT2_TWPOST>), g, b, 0, st, l, in, out); break;
    case LINE_DCT3_PREUNTWIST:
        hipLaunchKernelGGL((k_line<R, LINE_DCT3_PREUNTWIST>), g, b, 0, st, l, in, out);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

inline uint32_t gen_grid(int64_t count) { return uint32_t(std::min<int64_t>((count + 255) / 256, 4096)); }
} // namespace

hipError_t prepare_pass(PassArgs &a, bool f64)
{
    const void *k = f64 ? pass_kernel_for<double>(a) : pass_kernel_for<float>(a);
    if (a.lds_bytes > 64 * 1024) {
        // dynamic LDS beyond 64 KiB (gfx950 has 160 KiB per CU) needs an opt-in per kernel
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
    }
    // one tile per workgroup: measured faster than persistent workgroups looping over
    // tiles (a pipelined form that kept the next tile's loads in flight needed more
    // than the 128 VGPRs a 1024-thread group may hold, and spilled) -- except the
    // radix-64 matrix-core kernels, whose groups build an LDS table once and then walk
    // their tiles: as many groups as are resident at once
    a.grid = a.ntiles;
    bool r64 = false;
    for (int s = 0; s < a.nst; ++s) r64 = r64 || a.st[s].r == 64;
    if (r64 && a.mode >= 2 && a.mshape >= 0) {
        int per_cu = 0, dev = 0, cus = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, a.threads, size_t(a.lds_bytes));
        if (e == hipSuccess) e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        const int64_t g = int64_t(std::max(per_cu, 1)) * cus;
        if (g < a.ntiles) a.grid = g;
    }
    return hipSuccess;
}

hipError_t launch_pass(const PassArgs &a, bool f64, const void *in, void *out, hipStream_t st)
{
    return f64 ? launch_pass_t<double>(a, in, out, st) : launch_pass_t<float>(a, in, out, st);
}

hipError_t launch_line(int type, const LineArgs &l, bool f64, const void *in, void *out, int64_t grid, int block,
                       hipStream_t st)
{
    return f64 ? launch_line_t<double>(type, l, in, out, grid, block, st)
               : launch_line_t<float>(type, l, in, out, grid, block, st);
}


hipError_t gen_range(double2 *dst, int64_t N, int64_t e0, int64_t step, int64_t count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gen_range, dim3(gen_grid(count)), dim3(256), 0, st, dst, N, e0, step, count);
    return hipGetLastError();
}

hipError_t gen_inner(double2 *dst, const StagesArg &s, int64_t count, hipStream_t st)
{
    hipLaunchKernelGGL(k_gen_inner, dim3(gen_grid(count)), dim3(256), 0, st, dst, s);
    return hipGetLastError();
}

hipError_t gen_chirp(double2 *dst, int64_t n, int64_t count, hipStream_t st)
{
    hipLaunchKernelGGL(k_gen_chirp, dim3(gen_grid(count)), dim3(256), 0, st, dst, n, count);
    return hipGetLastError();
}

hipError_t gen_bwrap(double2 *dst, const double2 *chirp, int64_t n, int64_t M, hipStream_t st)
{
    hipLaunchKernelGGL(k_gen_bwrap, dim3(gen_grid(M)), dim3(256), 0, st, dst, chirp, n, M);
    return hipGetLastError();
}

hipError_t convert_d2f(float2 *dst, const double2 *src, int64_t count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_d2f, dim3(gen_grid(count)), dim3(256), 0, st, dst, src, count);
    return hipGetLastError();
}

} // namespace mifft
