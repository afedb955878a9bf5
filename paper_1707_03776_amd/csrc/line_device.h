// Device code of the element-wise steps (Bluestein, real-data staging, DCT
// reordering and twists), shared by k_line and the ragged batch kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "dft_small.h"
#include "fft_args.h"
#include "kernels.h"

namespace mifft {

__device__ __forceinline__ void line_bases(const LineArgs &l, uint32_t f, int64_t &bin, int64_t &bout)
{
    if (l.csz[1] == 1 && l.csz[2] == 1 && l.csz[3] == 1) {
        // plain rows (uniform branch): f < nlines = csz[0] is the row itself
        bin = int64_t(f) * l.cin[0];
        bout = int64_t(f) * l.cout[0];
        return;
    }
    uint32_t d0 = f % uint32_t(l.csz[0]);
    f /= uint32_t(l.csz[0]);
    uint32_t d1 = f % uint32_t(l.csz[1]);
    f /= uint32_t(l.csz[1]);
    uint32_t d2 = f % uint32_t(l.csz[2]);
    uint32_t d3 = f / uint32_t(l.csz[2]);
    bin = int64_t(d0) * l.cin[0] + int64_t(d1) * l.cin[1] + int64_t(d2) * l.cin[2] + int64_t(d3) * l.cin[3];
    bout = int64_t(d0) * l.cout[0] + int64_t(d1) * l.cout[1] + int64_t(d2) * l.cout[2] + int64_t(d3) * l.cout[3];
}

// (Y_k + conj Y_{h-k}) - i W (Y_k - conj Y_{h-k}): one untwisted point of a c2r.
template <typename C> __device__ __forceinline__ C c2r_untwist_point(const C yk, const C ym, const C w)
{
    const C s = C{yk.x + ym.x, yk.y - ym.y};
    const C d = C{yk.x - ym.x, yk.y + ym.y};
    const C wd = c_mul(w, d);
    return C{s.x + wd.y, s.y - wd.x};
}

template <typename C> __device__ __forceinline__ C maybe_conj(C x, int c)
{
    if (c) x.y = -x.y;
    return x;
}

// One element g (< line_total) of an element-wise op.
template <typename R, int TYPE>
__device__ __forceinline__ void line_elem(const LineArgs &l, int64_t g, const void *vin, void *vout)
{
    using C = typename Cplx<R>::T;
    // every element-wise op covers fewer than 2^32 elements (the planner's limits)
    const uint32_t g32 = uint32_t(g);
    const C *in = static_cast<const C *>(vin);
    C *out = static_cast<C *>(vout);
    const C *tab = static_cast<const C *>(l.tab);
    int64_t bi, bo;
    if constexpr (TYPE == LINE_CHIRP_PAD) {
        // Bluestein: a_j = x_j w_j, zero-padded to M
        const uint32_t f = (g32 / uint32_t(l.M)), j = (g32 % uint32_t(l.M));
        line_bases(l, f, bi, bo);
        C v = C{R(0), R(0)};
        if (j < l.n) v = c_mul(maybe_conj(in[bi + int64_t(j) * l.es_in], l.conj_in), tab[j]);
        out[bo + int64_t(j) * l.es_out] = v;
    } else if constexpr (TYPE == LINE_MUL_CONJ) {
        // Bluestein: A <- conj(A * B), in place (the inverse transform as a conjugated forward one)
        const C *bf = static_cast<const C *>(l.tab2);
        out[g] = c_conj(c_mul(out[g], bf[g32 % uint32_t(l.M)]));
    } else if constexpr (TYPE == LINE_CHIRP_EXTRACT) {
        // Bluestein: X_k = w_k conj(E_k) / M (scale carries the 1/M and any inverse scale)
        const uint32_t f = (g32 / uint32_t(l.n)), k = (g32 % uint32_t(l.n));
        line_bases(l, f, bi, bo);
        C y = c_scale(c_mul(tab[k], c_conj(in[bi + int64_t(k) * l.es_in])), R(l.scale));
        out[bo + int64_t(k) * l.es_out] = maybe_conj(y, l.conj_out);
    } else if constexpr (TYPE == LINE_R2C_TWIST) {
        const int64_t h = l.n / 2;
        const uint32_t f = (g32 / uint32_t((h + 1))), k = (g32 % uint32_t((h + 1)));
        line_bases(l, f, bi, bo);
        const C zk = in[bi + (k == h ? 0 : k)];
        const C zm = in[bi + (k == 0 ? 0 : h - k)];
        const C s = C{zk.x + zm.x, zk.y - zm.y};
        const C d = C{zk.x - zm.x, zk.y + zm.y};
        const C wd = c_mul(tab[k], d);
        const R half = R(0.5);
        out[bo + k] = C{(s.x + wd.y) * half, (s.y - wd.x) * half};
    } else if constexpr (TYPE == LINE_C2R_UNTWIST) {
        const int64_t h = l.n / 2;
        const uint32_t f = (g32 / uint32_t(h)), k = (g32 % uint32_t(h));
        line_bases(l, f, bi, bo);
        C yk = in[bi + k];
        C ym = in[bi + (h - k)];
        if (l.conj_in) { // true spectrum in: Y = conj(X)
            yk.y = -yk.y;
            ym.y = -ym.y;
        }
        if (k == 0) {
            yk.y = R(0);
            ym.y = R(0);
        }
        const C s = C{yk.x + ym.x, yk.y - ym.y};
        const C d = C{yk.x - ym.x, yk.y + ym.y};
        const C wd = c_mul(tab[k], d);
        out[bo + k] = C{s.x + wd.y, s.y - wd.x};
    } else if constexpr (TYPE == LINE_REAL_TO_CPLX) {
        const R *rin = static_cast<const R *>(vin);
        const uint32_t f = (g32 / uint32_t(l.n)), j = (g32 % uint32_t(l.n));
        line_bases(l, f, bi, bo);
        out[bo + j] = C{rin[bi + j], R(0)};
    } else if constexpr (TYPE == LINE_HALF_COPY) {
        const int64_t h1 = l.n / 2 + 1;
        const uint32_t f = (g32 / uint32_t(h1)), k = (g32 % uint32_t(h1));
        line_bases(l, f, bi, bo);
        out[bo + k] = in[bi + k];
    } else if constexpr (TYPE == LINE_HERM_EXPAND) {
        const int64_t n = l.n, h = n / 2;
        const uint32_t f = (g32 / uint32_t(n)), k = (g32 % uint32_t(n));
        line_bases(l, f, bi, bo);
        C y;
        if (k <= h) {
            y = maybe_conj(in[bi + k], l.conj_in);
            if (k == 0 || 2 * int64_t(k) == n) y.y = R(0);
        } else {
            y = c_conj(maybe_conj(in[bi + (n - k)], l.conj_in));
        }
        out[bo + k] = y;
    } else if constexpr (TYPE == LINE_CPLX_TO_REAL) {
        R *rout = static_cast<R *>(vout);
        const uint32_t f = (g32 / uint32_t(l.n)), j = (g32 % uint32_t(l.n));
        line_bases(l, f, bi, bo);
        rout[bo + j] = in[bi + j].x * R(l.scale);
    } else if constexpr (TYPE == LINE_DCT2_PRE) {
        // DCT-II via the real DFT of v: v_j = x_2j for j < ceil(n/2), v_{n-1-j} = x_{2j+1}
        const R *rin = static_cast<const R *>(vin);
        R *rout = static_cast<R *>(vout);
        const uint32_t f = (g32 / uint32_t(l.n)), j = (g32 % uint32_t(l.n)), n = uint32_t(l.n);
        line_bases(l, f, bi, bo);
        const uint32_t src = 2u * j < n ? 2u * j : 2u * (n - 1u - j) + 1u;
        rout[bo + j] = rin[bi + src];
    } else if constexpr (TYPE == LINE_DCT2_POST) {
        // y_k = 2 Re(W_4n^k V_k) from the half spectrum (V_k = conj V_{n-k} above n/2)
        R *rout = static_cast<R *>(vout);
        const uint32_t f = (g32 / uint32_t(l.n)), k = (g32 % uint32_t(l.n)), n = uint32_t(l.n);
        line_bases(l, f, bi, bo);
        C v;
        if (2u * k <= n) {
            v = in[bi + k];
        } else {
            v = in[bi + (n - k)];
            v.y = -v.y;
        }
        const C w = tab[k];
        rout[bo + k] = R(2) * (v.x * w.x - v.y * w.y);
    } else if constexpr (TYPE == LINE_DCT3_PRE) {
        // DCT-III via the real inverse DFT: V_k = conj(W_4n^k) (y_k - i y_{n-k}) for
        // k = 0..n/2 with y_n = 0 (the unnormalised inverse of V is Makhoul's reordered line)
        const R *rin = static_cast<const R *>(vin);
        const uint32_t n = uint32_t(l.n), hb = n / 2u + 1u;
        const uint32_t f = g32 / hb, k = g32 % hb;
        line_bases(l, f, bi, bo);
        const R a = rin[bi + k];
        const R b = k == 0u ? R(0) : rin[bi + (n - k)];
        const C w = tab[k];
        out[bo + k] = C{w.x * a - w.y * b, -(w.x * b + w.y * a)};
    } else if constexpr (TYPE == LINE_DCT2_TWPOST) {
        // DCT-II straight from the n/2-point spectrum Z of z_m = v_2m + i v_2m+1 (v the
        // reordered line): V_k = (Z_k + conj Z_{h-k})/2 - (i/2) W_n^k (Z_k - conj Z_{h-k})
        // (Z_h = Z_0), y_k = 2 Re(W_4n^k V_k) and y_{n-k} = 2 Re(W_4n^{n-k} conj V_k).
        // Element g covers the bin pair (k, h-k), k <= h/2: both V from the same two loads.
        R *rout = static_cast<R *>(vout);
        const C *tw = static_cast<const C *>(l.tab2); // W_n^k, k <= h
        const uint32_t n = uint32_t(l.n), h = n / 2u, q = h / 2u + 1u;
        const uint32_t f = g32 / q, k = g32 % q;
        line_bases(l, f, bi, bo);
        const C za = in[bi + (k == h ? 0u : k)];
        const C zb = in[bi + (h - k == h ? 0u : h - k)];
        const R half = R(0.5);
        auto twist = [&](const C zk, const C zm, const C w) {
            const C s = C{zk.x + zm.x, zk.y - zm.y};
            const C d = C{zk.x - zm.x, zk.y + zm.y};
            const C wd = c_mul(w, d);
            return C{(s.x + wd.y) * half, (s.y - wd.x) * half};
        };
        auto emit = [&](uint32_t kk, const C v) {
            const C w = tab[kk];
            rout[bo + kk] = R(2) * (v.x * w.x - v.y * w.y);
            if (kk >= 1u && kk < h) {
                const C w2 = tab[n - kk]; // conj V for bin n - k
                rout[bo + (n - kk)] = R(2) * (v.x * w2.x + v.y * w2.y);
            }
        };
        emit(k, twist(za, zb, tw[k]));
        if (h - k != k) emit(h - k, twist(zb, za, tw[h - k]));
    } else if constexpr (TYPE == LINE_DCT3_PREUNTWIST) {
        // DCT-III's rotation V_k = conj(W_4n^k) (y_k - i y_{n-k}) (y_n = 0) and the c2r
        // untwist of its conjugate, P_k = (Y_k + conj Y_{h-k}) - i W_n^k (Y_k - conj Y_{h-k})
        // with Y = conj V and the imaginary parts of Y_0 and Y_h dropped, for k < h.
        // Element g covers the bin pair (k, h-k), k <= h/2: both V from four input reals.
        const R *rin = static_cast<const R *>(vin);
        const C *tw = static_cast<const C *>(l.tab2); // W_n^k, k <= h
        const uint32_t n = uint32_t(l.n), h = n / 2u, q = h / 2u + 1u;
        const uint32_t f = g32 / q, k = g32 % q;
        line_bases(l, f, bi, bo);
        auto rot = [&](uint32_t kk) { // conj V_kk = Y_kk
            const R a = rin[bi + kk];
            const R b = kk == 0u ? R(0) : rin[bi + (n - kk)];
            const C w = tab[kk];
            return C{w.x * a - w.y * b, w.x * b + w.y * a};
        };
        C ya = rot(k), yb = rot(h - k);
        if (k == 0u) { // Y_0 and Y_h enter with their real parts only
            ya.y = R(0);
            yb.y = R(0);
        }
        out[bo + k] = c2r_untwist_point(ya, yb, tw[k]);
        if (h - k != k && h - k < h) out[bo + (h - k)] = c2r_untwist_point(yb, ya, tw[h - k]);
    } else if constexpr (TYPE == LINE_DCT3_POST) {
        // undo the reordering: y_2m = v_m, y_2m+1 = v_{n-1-m}
        const R *rin = static_cast<const R *>(vin);
        R *rout = static_cast<R *>(vout);
        const uint32_t n = uint32_t(l.n);
        const uint32_t f = g32 / n, k = g32 % n;
        line_bases(l, f, bi, bo);
        const uint32_t src = (k & 1u) == 0u ? k / 2u : n - 1u - k / 2u;
        rout[bo + k] = rin[bi + src];
    }
}

template <typename R>
__device__ __forceinline__ void line_elem_dispatch(int type, const LineArgs &l, int64_t g, const void *in, void *out)
{
    switch (type) {
    case LINE_CHIRP_PAD: line_elem<R, LINE_CHIRP_PAD>(l, g, in, out); break;
    case LINE_MUL_CONJ: line_elem<R, LINE_MUL_CONJ>(l, g, in, out); break;
    case LINE_CHIRP_EXTRACT: line_elem<R, LINE_CHIRP_EXTRACT>(l, g, in, out); break;
    case LINE_R2C_TWIST: line_elem<R, LINE_R2C_TWIST>(l, g, in, out); break;
    case LINE_C2R_UNTWIST: line_elem<R, LINE_C2R_UNTWIST>(l, g, in, out); break;
    case LINE_REAL_TO_CPLX: line_elem<R, LINE_REAL_TO_CPLX>(l, g, in, out); break;
    case LINE_HALF_COPY: line_elem<R, LINE_HALF_COPY>(l, g, in, out); break;
    case LINE_HERM_EXPAND: line_elem<R, LINE_HERM_EXPAND>(l, g, in, out); break;
    case LINE_CPLX_TO_REAL: line_elem<R, LINE_CPLX_TO_REAL>(l, g, in, out); break;
    case LINE_DCT2_PRE: line_elem<R, LINE_DCT2_PRE>(l, g, in, out); break;
    case LINE_DCT2_POST: line_elem<R, LINE_DCT2_POST>(l, g, in, out); break;
    case LINE_DCT3_PRE: line_elem<R, LINE_DCT3_PRE>(l, g, in, out); break;
    case LINE_DCT3_POST: line_elem<R, LINE_DCT3_POST>(l, g, in, out); break;
    case LINE_DCT2_TWPOST: line_elem<R, LINE_DCT2_TWPOST>(l, g, in, out); break;
    case LINE_DCT3_PREUNTWIST: line_elem<R, LINE_DCT3_PREUNTWIST>(l, g, in, out); break;
    default: break;
    }
}

} // namespace mifft
