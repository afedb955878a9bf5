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
const void *pass_kernel_f32_sym(int shape);
const void *pass_kernel_f64_sym(int shape);
const void *pass_kernel_f32_dct2(int shape);
const void *pass_kernel_f64_dct2(int shape);
const void *pass_kernel_f32_dct3(int shape);
const void *pass_kernel_f64_dct3(int shape);
const void *pass_kernel_f32_rtwist(int shape);
const void *pass_kernel_f64_rtwist(int shape);
const void *pass_kernel_f32_dtwist(int shape);
const void *pass_kernel_f32_cuntwist(int shape);
const void *pass_kernel_f64_cuntwist(int shape);
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

// Element-wise steps over long rows (the DCT reorderings and rotations, the real
// transforms' twist and untwist): lane k of a row handles the bin or sample pair (or
// quad) k, and each thread walks kRowLines rows with the twiddles of its k loaded once.
// The per-element form (k_line) loaded every twiddle once per row element, so for
// 2^20-point rows the tables (W_4n^k for k < n, W_n^k for k <= n/2: 12 MiB in FP32) were
// streamed again for every row; it also read the reordered samples in two half-used
// strided sweeps, where here x_2k and x_2k+1 come in one pair, and it read each bin of a
// twist's pair (k, h-k) twice, where here one thread reads both and writes both.
constexpr int kRowLines = 8;

template <typename R, int TYPE, bool QUAD = false>
__global__ void __launch_bounds__(256) k_line_rows(const LineArgs l, const void *vin, void *vout)
{
    using C = typename Cplx<R>::T;
    const uint32_t n = uint32_t(l.n), h = n / 2u;
    const uint32_t q = QUAD ? n / 4u : (TYPE == LINE_DCT2_PRE || TYPE == LINE_DCT3_POST) ? (n + 1u) / 2u : h / 2u + 1u;
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= q) return;
    if constexpr (QUAD) {
        // n a multiple of 4 and rows aligned to 4 samples: lane k takes two sample pairs,
        // x_4k..x_4k+3 <-> (v_2k, v_2k+1) and (v_{n-2-2k}, v_{n-1-2k}), in 4- and 2-sample
        // accesses
        using V2 = R __attribute__((ext_vector_type(2)));
        using V4 = R __attribute__((ext_vector_type(4)));
        for (int64_t f0 = int64_t(blockIdx.y) * kRowLines; f0 < l.nlines; f0 += int64_t(gridDim.y) * kRowLines) {
            const int64_t f1 = f0 + kRowLines < l.nlines ? f0 + kRowLines : l.nlines;
#pragma unroll 4
            for (int64_t f = f0; f < f1; ++f) {
                int64_t bi, bo;
                line_bases(l, uint32_t(f), bi, bo);
                if constexpr (TYPE == LINE_DCT2_PRE) {
                    const V4 x = *reinterpret_cast<const V4 *>(static_cast<const R *>(vin) + bi + 4u * k);
                    R *v = static_cast<R *>(vout) + bo;
                    *reinterpret_cast<V2 *>(v + 2u * k) = V2{x.x, x.z};
                    *reinterpret_cast<V2 *>(v + (n - 2u - 2u * k)) = V2{x.w, x.y};
                } else {
                    const R *v = static_cast<const R *>(vin) + bi;
                    const V2 a = *reinterpret_cast<const V2 *>(v + 2u * k);
                    const V2 b = *reinterpret_cast<const V2 *>(v + (n - 2u - 2u * k));
                    *reinterpret_cast<V4 *>(static_cast<R *>(vout) + bo + 4u * k) = V4{a.x, b.y, a.y, b.x};
                }
            }
        }
        return;
    }
    const C *tab = static_cast<const C *>(l.tab);  // DCT steps: W_4n^k, k < n; twist / untwist: W_n^k, k <= n/2
    const C *tw = static_cast<const C *>(l.tab2);  // DCT steps: W_n^k, k <= n/2
    const int64_t nl = l.nlines;
    if constexpr (TYPE == LINE_DCT2_PRE) {
        // v_k = x_2k and v_{n-1-k} = x_2k+1 (the second only while 2k+1 < n)
        const R *x = static_cast<const R *>(vin);
        R *v = static_cast<R *>(vout);
        const bool two = 2u * k + 1u < n;
        for (int64_t f0 = int64_t(blockIdx.y) * kRowLines; f0 < nl; f0 += int64_t(gridDim.y) * kRowLines) {
            const int64_t f1 = f0 + kRowLines < nl ? f0 + kRowLines : nl;
#pragma unroll 4
            for (int64_t f = f0; f < f1; ++f) {
                int64_t bi, bo;
                line_bases(l, uint32_t(f), bi, bo);
                v[bo + k] = x[bi + 2u * k];
                if (two) v[bo + (n - 1u - k)] = x[bi + 2u * k + 1u];
            }
        }
    } else if constexpr (TYPE == LINE_DCT3_POST) {
        // y_2k = v_k and y_2k+1 = v_{n-1-k} (the second only while 2k+1 < n)
        const R *v = static_cast<const R *>(vin);
        R *y = static_cast<R *>(vout);
        const bool two = 2u * k + 1u < n;
        for (int64_t f0 = int64_t(blockIdx.y) * kRowLines; f0 < nl; f0 += int64_t(gridDim.y) * kRowLines) {
            const int64_t f1 = f0 + kRowLines < nl ? f0 + kRowLines : nl;
#pragma unroll 4
            for (int64_t f = f0; f < f1; ++f) {
                int64_t bi, bo;
                line_bases(l, uint32_t(f), bi, bo);
                y[bo + 2u * k] = v[bi + k];
                if (two) y[bo + 2u * k + 1u] = v[bi + (n - 1u - k)];
            }
        }
    } else if constexpr (TYPE == LINE_DCT2_TWPOST) {
        // the twist of the n/2-point spectrum Z into V and y_k = 2 Re(W_4n^k V_k),
        // y_{n-k} = 2 Re(W_4n^{n-k} conj V_k), for the bin pair (k, h-k) of every row
        R *y = static_cast<R *>(vout);
        const C *z = static_cast<const C *>(vin);
        const uint32_t kb = h - k;
        const C twa = tw[k], twb = tw[kb];
        const C wa = tab[k], wb = tab[kb];
        const bool a2 = k >= 1u && k < h, b2 = kb >= 1u && kb < h, bb = kb != k;
        const C wa2 = a2 ? tab[n - k] : C{}, wb2 = b2 ? tab[n - kb] : C{};
        const uint32_t ia = k == h ? 0u : k, ib = kb == h ? 0u : kb;
        const R half = R(0.5);
        auto twist = [&](const C zk, const C zm, const C w) {
            const C s = C{zk.x + zm.x, zk.y - zm.y};
            const C d = C{zk.x - zm.x, zk.y + zm.y};
            const C wd = c_mul(w, d);
            return C{(s.x + wd.y) * half, (s.y - wd.x) * half};
        };
        for (int64_t f0 = int64_t(blockIdx.y) * kRowLines; f0 < nl; f0 += int64_t(gridDim.y) * kRowLines) {
            const int64_t f1 = f0 + kRowLines < nl ? f0 + kRowLines : nl;
#pragma unroll 2
            for (int64_t f = f0; f < f1; ++f) {
                int64_t bi, bo;
                line_bases(l, uint32_t(f), bi, bo);
                const C za = z[bi + ia], zb = z[bi + ib];
                const C va = twist(za, zb, twa);
                y[bo + k] = R(2) * (va.x * wa.x - va.y * wa.y);
                if (a2) y[bo + (n - k)] = R(2) * (va.x * wa2.x + va.y * wa2.y);
                if (bb) {
                    const C vb = twist(zb, za, twb);
                    y[bo + kb] = R(2) * (vb.x * wb.x - vb.y * wb.y);
                    if (b2) y[bo + (n - kb)] = R(2) * (vb.x * wb2.x + vb.y * wb2.y);
                }
            }
        }
    } else if constexpr (TYPE == LINE_R2C_TWIST) {
        // X_k = (Z_k + conj Z_{h-k})/2 - (i/2) W_n^k (Z_k - conj Z_{h-k}) (Z_h = Z_0) for the
        // bin pair (k, h-k): both from the same two loads
        const C *z = static_cast<const C *>(vin);
        C *out = static_cast<C *>(vout);
        const uint32_t kb = h - k;
        const C wa = tab[k], wb = tab[kb];
        const uint32_t ia = k == h ? 0u : k, ib = kb == h ? 0u : kb;
        const R half = R(0.5);
        auto twist = [&](const C zk, const C zm, const C w) {
            const C s = C{zk.x + zm.x, zk.y - zm.y};
            const C d = C{zk.x - zm.x, zk.y + zm.y};
            const C wd = c_mul(w, d);
            return C{(s.x + wd.y) * half, (s.y - wd.x) * half};
        };
        for (int64_t f0 = int64_t(blockIdx.y) * kRowLines; f0 < nl; f0 += int64_t(gridDim.y) * kRowLines) {
            const int64_t f1 = f0 + kRowLines < nl ? f0 + kRowLines : nl;
#pragma unroll 2
            for (int64_t f = f0; f < f1; ++f) {
                int64_t bi, bo;
                line_bases(l, uint32_t(f), bi, bo);
                const C za = z[bi + ia], zb = z[bi + ib];
                out[bo + k] = twist(za, zb, wa);
                if (kb != k) out[bo + kb] = twist(zb, za, wb);
            }
        }
    } else if constexpr (TYPE == LINE_C2R_UNTWIST) {
        // P_k = (Y_k + conj Y_{h-k}) - i W_n^k (Y_k - conj Y_{h-k}) for the bin pair (k, h-k),
        // k < h (Y = conj X for a true spectrum in; Y_0 and Y_h with their real parts only)
        const C *y = static_cast<const C *>(vin);
        C *out = static_cast<C *>(vout);
        const uint32_t kb = h - k;
        const C wa = tab[k], wb = tab[kb];
        const bool bb = kb != k && kb < h;
        const R cs = l.conj_in ? R(-1) : R(1);
        for (int64_t f0 = int64_t(blockIdx.y) * kRowLines; f0 < nl; f0 += int64_t(gridDim.y) * kRowLines) {
            const int64_t f1 = f0 + kRowLines < nl ? f0 + kRowLines : nl;
#pragma unroll 2
            for (int64_t f = f0; f < f1; ++f) {
                int64_t bi, bo;
                line_bases(l, uint32_t(f), bi, bo);
                C ya = y[bi + k], yb = y[bi + kb];
                ya.y *= cs;
                yb.y *= cs;
                if (k == 0u) {
                    ya.y = R(0);
                    yb.y = R(0);
                }
                out[bo + k] = c2r_untwist_point(ya, yb, wa);
                if (bb) out[bo + kb] = c2r_untwist_point(yb, ya, wb);
            }
        }
    } else if constexpr (TYPE == LINE_DCT3_PREUNTWIST) {
        // the DCT-III rotation of input reals into Y = conj V and the c2r untwist of the
        // bin pair (k, h-k) of every row (Y_0 and Y_h with their real parts only)
        const R *x = static_cast<const R *>(vin);
        C *out = static_cast<C *>(vout);
        const uint32_t kb = h - k;
        const C twa = tw[k], twb = tw[kb];
        const C wa = tab[k], wb = tab[kb];
        const bool bb = kb != k && kb < h;
        for (int64_t f0 = int64_t(blockIdx.y) * kRowLines; f0 < nl; f0 += int64_t(gridDim.y) * kRowLines) {
            const int64_t f1 = f0 + kRowLines < nl ? f0 + kRowLines : nl;
#pragma unroll 2
            for (int64_t f = f0; f < f1; ++f) {
                int64_t bi, bo;
                line_bases(l, uint32_t(f), bi, bo);
                const R a0 = x[bi + k], b0 = k == 0u ? R(0) : x[bi + (n - k)];
                const R a1 = x[bi + kb], b1 = kb == 0u ? R(0) : x[bi + (n - kb)];
                C ya = C{wa.x * a0 - wa.y * b0, wa.x * b0 + wa.y * a0};
                C yb = C{wb.x * a1 - wb.y * b1, wb.x * b1 + wb.y * a1};
                if (k == 0u) {
                    ya.y = R(0);
                    yb.y = R(0);
                }
                out[bo + k] = c2r_untwist_point(ya, yb, twa);
                if (bb) out[bo + kb] = c2r_untwist_point(yb, ya, twb);
            }
        }
    }
}

// Rows long enough for k_line_rows to fill its workgroups: at least 256 pairs or quads.
bool line_rows_form(int type, const LineArgs &l)
{
    const int64_t n = l.n;
    if (type == LINE_DCT2_PRE || type == LINE_DCT3_POST) return (n + 1) / 2 >= 256;
    if (type == LINE_DCT2_TWPOST || type == LINE_DCT3_PREUNTWIST || type == LINE_R2C_TWIST ||
        type == LINE_C2R_UNTWIST)
        return n % 2 == 0 && n / 4 + 1 >= 256;
    return false;
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
    if (a.pro == PRO_SYM) return pass_kernel_f32_sym(a.shape); // null unless a specialised shape
    if (a.pro == PRO_DCT2) return pass_kernel_f32_dct2(a.shape);
    if (a.pro == PRO_CUNTWIST) return pass_kernel_f32_cuntwist(a.shape);
    if (a.epi == EPI_DCT3) return pass_kernel_f32_dct3(a.shape);
    if (a.epi == EPI_RTWIST) return pass_kernel_f32_rtwist(a.shape);
    if (a.epi == EPI_DTWIST) return pass_kernel_f32_dtwist(a.shape);
    if (a.pro == PRO_BPAD || a.epi == EPI_BMUL || a.epi == EPI_BEXT) return pass_kernel_f32_plain(-1);
    if (a.pro == PRO_C2R) return pass_kernel_f32_c2r(a.shape);
    if (a.epi == EPI_R2C) return pass_kernel_f32_r2c(a.shape);
    return pass_kernel_f32_plain(a.shape);
}
template <> const void *pass_kernel_for<double>(const PassArgs &a)
{
    if (a.pro == PRO_SYM) return pass_kernel_f64_sym(a.shape);
    if (a.pro == PRO_DCT2) return pass_kernel_f64_dct2(a.shape);
    if (a.pro == PRO_CUNTWIST) return pass_kernel_f64_cuntwist(a.shape);
    if (a.epi == EPI_DCT3) return pass_kernel_f64_dct3(a.shape);
    if (a.epi == EPI_RTWIST) return pass_kernel_f64_rtwist(a.shape);
    if (a.epi == EPI_DTWIST) return nullptr; // float32 only (the planner never asks for it)
    if (a.pro == PRO_BPAD || a.epi == EPI_BMUL || a.epi == EPI_BEXT) return pass_kernel_f64_plain(-1);
    if (a.pro == PRO_C2R) return pass_kernel_f64_c2r(a.shape);
    if (a.epi == EPI_R2C) return pass_kernel_f64_r2c(a.shape);
    return pass_kernel_f64_plain(a.shape);
}

template <typename R>
hipError_t launch_pass_t(const PassArgs &a, const void *in, void *out, hipStream_t st)
{
    const void *k = pass_kernel_for<R>(a);
    if (!k) return hipErrorInvalidDeviceFunction;
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
    if (line_rows_form(type, l)) {
        const int64_t q = (type == LINE_DCT2_PRE || type == LINE_DCT3_POST) ? (l.n + 1) / 2 : l.n / 4 + 1;
        const dim3 rg{uint32_t((q + 255) / 256),
                      uint32_t(std::min<int64_t>((l.nlines + kRowLines - 1) / kRowLines, 65535))};
        // the reorders in 4-sample accesses where the rows allow (n a multiple of 4, plain
        // rows a multiple of 4 samples apart, buffers aligned to 4 samples)
        constexpr uintptr_t a4 = 4 * sizeof(R);
        const bool quad = (type == LINE_DCT2_PRE || type == LINE_DCT3_POST) && l.n % 4 == 0 &&
                          l.csz[1] == 1 && l.csz[2] == 1 && l.csz[3] == 1 && l.cin[0] % 4 == 0 &&
                          l.cout[0] % 4 == 0 && reinterpret_cast<uintptr_t>(in) % a4 == 0 &&
                          reinterpret_cast<uintptr_t>(out) % a4 == 0;
        if (quad) {
            const dim3 qg{uint32_t((l.n / 4 + 255) / 256), rg.y};
            if (type == LINE_DCT2_PRE)
                hipLaunchKernelGGL((k_line_rows<R, LINE_DCT2_PRE, true>), qg, dim3(256), 0, st, l, in, out);
            else
                hipLaunchKernelGGL((k_line_rows<R, LINE_DCT3_POST, true>), qg, dim3(256), 0, st, l, in, out);
            return hipGetLastError();
        }
        switch (type) {
        case LINE_DCT2_PRE: hipLaunchKernelGGL((k_line_rows<R, LINE_DCT2_PRE>), rg, dim3(256), 0, st, l, in, out); break;
        case LINE_DCT3_POST: hipLaunchKernelGGL((k_line_rows<R, LINE_DCT3_POST>), rg, dim3(256), 0, st, l, in, out); break;
        case LINE_DCT2_TWPOST:
            hipLaunchKernelGGL((k_line_rows<R, LINE_DCT2_TWPOST>), rg, dim3(256), 0, st, l, in, out);
            break;
        case LINE_R2C_TWIST:
            hipLaunchKernelGGL((k_line_rows<R, LINE_R2C_TWIST>), rg, dim3(256), 0, st, l, in, out);
            break;
        case LINE_C2R_UNTWIST:
            hipLaunchKernelGGL((k_line_rows<R, LINE_C2R_UNTWIST>), rg, dim3(256), 0, st, l, in, out);
            break;
        default: hipLaunchKernelGGL((k_line_rows<R, LINE_DCT3_PREUNTWIST>), rg, dim3(256), 0, st, l, in, out); break;
        }
        return hipGetLastError();
    }
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
    if (!k) return hipErrorInvalidDeviceFunction; // a flavour with no kernel for this shape
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
