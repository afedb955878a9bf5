// Device code of the Stockham pass kernels, included by the translation units that
// instantiate them (pass_*.hip for the plain passes, mfma.hip, ragged.hip).
//
// k_pass computes, for each of `ncols` independent columns, one length-L DFT of
// the Stockham factorisation (Stockham autosort: no bit reversal; outputs land in
// natural order).  A workgroup owns `c` consecutive columns.  Inner stage s with
// radix r and Ns = product of the earlier radices maps butterfly b (< L/r) of a
// column from points b + k*L/r (k < r), multiplied by W_{Ns r}^{k (b mod Ns)}, through
// an r-point DFT to points (b/Ns)*Ns*r + (b mod Ns) + k*Ns.  The first stage reads
// global memory directly and the last writes it directly; the stages between
// exchange through LDS.  Stage 1 of a pass is therefore also where the multi-pass
// twiddle (four-step, in Stockham form) is applied, and the last stage is where the
// conjugation/scale of an inverse transform is folded in.
#pragma once

#include <hip/hip_runtime.h>

#include "dft_small.h"
#include "fft_args.h"
#include "kernels.h"
#include "shapes.h"

#include <algorithm>
#include <cstdlib>
#include <utility>

namespace mifft {

template <typename R> struct PadShift;
template <> struct PadShift<float> { static constexpr int v = kLdsPadShiftF32; };
template <> struct PadShift<double> { static constexpr int v = kLdsPadShiftF64; };

// Workgroup -> tile: the hardware deals workgroups round-robin over the 8 XCDs;
// give each XCD a contiguous range of tiles so neighbouring tiles (which share
// cache lines at their edges) run on the same L2.
__device__ __forceinline__ uint32_t tile_of_block()
{
    const uint32_t nb = gridDim.x, b = blockIdx.x;
    const uint32_t q = nb >> 3, rem = nb & 7, x = b & 7, s = b >> 3;
    return x * q + min(x, rem) + s;
}

struct ColBase {
    uint32_t in, out; // element offsets (every buffer holds fewer than 2^32 elements)
    uint32_t twi;     // column index along the twiddle dim
};

template <typename R> __device__ __forceinline__ int lds_index(int col, int q, int lp)
{
    return col * lp + q + (q >> PadShift<R>::v);
}

// W_N^e in FP64 from the two-level table (FP64 in every plan): hi[e >> bits] * lo[e & mask]
__device__ __forceinline__ double2 pass_root(const PassArgs &a, uint32_t e)
{
    const double2 *lo = static_cast<const double2 *>(a.tw_lo);
    const double2 *hi = static_cast<const double2 *>(a.tw_hi);
    const uint32_t mask = (1u << a.tw_bits) - 1u;
    return c_mul(hi[e >> a.tw_bits], lo[e & mask]);
}

template <typename C> __device__ __forceinline__ C to_c(double2 w);
template <> __device__ __forceinline__ float2 to_c<float2>(double2 w) { return float2{float(w.x), float(w.y)}; }
template <> __device__ __forceinline__ double2 to_c<double2>(double2 w) { return w; }

// Global loads and stores, optionally nontemporal (streamed once: marked for early
// eviction so they do not push intermediates out of the caches).  A uniform branch.
template <typename C> struct NtVec;
template <> struct NtVec<float2> { typedef float T __attribute__((ext_vector_type(2))); };
template <> struct NtVec<double2> { typedef double T __attribute__((ext_vector_type(2))); };
template <typename C> __device__ __forceinline__ C gload(const C *p, int nt)
{
    if (nt) {
        const typename NtVec<C>::T v = __builtin_nontemporal_load(reinterpret_cast<const typename NtVec<C>::T *>(p));
        return C{v.x, v.y};
    }
    return *p;
}
template <typename C> __device__ __forceinline__ void gstore(C *p, C x, int nt)
{
    if (nt) {
        const typename NtVec<C>::T v = {x.x, x.y};
        __builtin_nontemporal_store(v, reinterpret_cast<typename NtVec<C>::T *>(p));
    } else {
        *p = x;
    }
}

// n / d for n < 2^32 via the FP64 reciprocal (the product is within 2^-20 of n/d, so one
// correction step makes it exact)
__device__ __forceinline__ uint32_t div_rcp(uint32_t n, uint32_t d, double rcp)
{
    uint32_t q = uint32_t(double(n) * rcp);
    const int64_t r = int64_t(n) - int64_t(q) * int64_t(d);
    if (r < 0) --q;
    else if (r >= int64_t(d)) ++q;
    return q;
}

// Column offsets, decomposing f only over the dims in use (none for a single dim).
__device__ __forceinline__ ColBase col_base_fast(const PassArgs &a, uint32_t f)
{
    ColBase cb{0u, 0u, 0u};
#pragma unroll
    for (int d = 0; d < kColDims; ++d) {
        if (d < a.ncd) {
            uint32_t r = f, q = 0u;
            if (d + 1 < a.ncd) {
                q = div_rcp(f, uint32_t(a.csz[d]), a.crcp[d]);
                r = f - q * uint32_t(a.csz[d]);
            }
            cb.in += r * uint32_t(a.cin[d]);
            cb.out += r * uint32_t(a.cout[d]);
            if (d == a.tw_dim) cb.twi = r;
            f = q;
        }
    }
    return cb;
}

// Column of slot `slot` of the tile starting at column col0 in a mirrored-tile pass
// (EPI_RTWIST / EPI_DTWIST): tile t of a line holds columns t*c/2 + i (slots i < c/2) and
// their mirrors J - (t*c/2 + i) (slots c/2 + i), column 0's slot taking J/2 instead.
__device__ __forceinline__ uint32_t mirror_col(const PassArgs &a, uint32_t col0, int slot)
{
    const uint32_t J = uint32_t(a.csz[0]), c = uint32_t(a.c), half = c >> 1;
    const uint32_t line = a.ncd > 1 ? div_rcp(col0, J, a.crcp[0]) : 0u;
    const uint32_t t = (col0 - line * J) / c;
    const bool low = uint32_t(slot) < half;
    const uint32_t jl = t * half + (low ? uint32_t(slot) : uint32_t(slot) - half);
    const uint32_t j = low ? jl : (jl == 0u ? J >> 1 : J - jl);
    return line * J + j;
}

template <int X> struct IsPow2 { static constexpr bool v = X > 0 && (X & (X - 1)) == 0; };

// LDS slot of point q of a column: one spare slot every 2^PadShift points.
template <typename R> __device__ __forceinline__ int lds_pad(int q) { return q + (q >> PadShift<R>::v); }

// W^{k m}, k = 1..RADIX-1, from the table row m (which holds all of them): entries at
// k = 1, 2, 4, 8 are read, the others are products of at most three of those.
// row_twiddle_loads reads the four entries (issued early, before a barrier);
// row_twiddle_products fills in the rest.
template <int RADIX, typename C> __device__ __forceinline__ void row_twiddle_loads(const C *row, C *w4)
{
    w4[0] = row[0];
    if constexpr (RADIX > 2) w4[1] = row[1];
    if constexpr (RADIX > 4) w4[2] = row[3];
    if constexpr (RADIX > 8) w4[3] = row[7];
}
template <int RADIX, typename C> __device__ __forceinline__ void row_twiddle_products(const C *w4, C *w)
{
    w[1] = w4[0];
    if constexpr (RADIX > 2) w[2] = w4[1];
    if constexpr (RADIX > 4) w[4] = w4[2];
    if constexpr (RADIX > 8) w[8] = w4[3];
    if constexpr (RADIX > 3) w[3] = c_mul(w[1], w[2]);
    if constexpr (RADIX > 5) w[5] = c_mul(w[1], w[4]);
    if constexpr (RADIX > 6) w[6] = c_mul(w[2], w[4]);
    if constexpr (RADIX > 7) w[7] = c_mul(w[3], w[4]);
    if constexpr (RADIX > 9) w[9] = c_mul(w[1], w[8]);
    if constexpr (RADIX > 10) w[10] = c_mul(w[2], w[8]);
    if constexpr (RADIX > 11) w[11] = c_mul(w[3], w[8]);
    if constexpr (RADIX > 12) w[12] = c_mul(w[4], w[8]);
    if constexpr (RADIX > 13) w[13] = c_mul(w[5], w[8]);
    if constexpr (RADIX > 14) w[14] = c_mul(w[6], w[8]);
    if constexpr (RADIX > 15) w[15] = c_mul(w[7], w[8]);
}
template <int RADIX, typename C> __device__ __forceinline__ void row_twiddles(const C *row, C *w)
{
    w[1] = row[0];
    if constexpr (RADIX > 2) w[2] = row[1];
    if constexpr (RADIX > 4) w[4] = row[3];
    if constexpr (RADIX > 8) w[8] = row[7];
    if constexpr (RADIX > 3) w[3] = c_mul(w[1], w[2]);
    if constexpr (RADIX > 5) w[5] = c_mul(w[1], w[4]);
    if constexpr (RADIX > 6) w[6] = c_mul(w[2], w[4]);
    if constexpr (RADIX > 7) w[7] = c_mul(w[3], w[4]);
    if constexpr (RADIX > 9) w[9] = c_mul(w[1], w[8]);
    if constexpr (RADIX > 10) w[10] = c_mul(w[2], w[8]);
    if constexpr (RADIX > 11) w[11] = c_mul(w[3], w[8]);
    if constexpr (RADIX > 12) w[12] = c_mul(w[4], w[8]);
    if constexpr (RADIX > 13) w[13] = c_mul(w[5], w[8]);
    if constexpr (RADIX > 14) w[14] = c_mul(w[6], w[8]);
    if constexpr (RADIX > 15) w[15] = c_mul(w[7], w[8]);
}

// Line and position of offset e in a layout of lines M apart: shift and mask for a power
// of two (the planner's choice), the FP64-reciprocal division otherwise.
__device__ __forceinline__ uint32_t line_of(uint32_t e, uint32_t M, double rcp)
{
    return (M & (M - 1u)) == 0u ? e >> __builtin_ctz(M) : div_rcp(e, M, rcp);
}

// n / d for small non-negative n, d (n < 2^20) from a float reciprocal and one correction.
__device__ __forceinline__ int div_small(int n, int d, float rcp)
{
    int q = int(float(n) * rcp);
    const int r = n - q * d;
    if (r < 0) --q;
    else if (r >= d) ++q;
    return q;
}

// One Stockham stage over the tile with runtime shape: nb = L/RADIX butterflies per
// column, ns = product of the earlier radices, tw_off = this stage's twiddle rows.
// MAXI items (butterflies) per thread; src_g / dst_g say whether the stage reads /
// writes global memory (first / last stage of a plain pass) instead of LDS; cf
// selects column-fast lane order for those accesses (the tile is c columns wide, c a
// power of two).  Same arithmetic as the specialised stages: inner twiddles from the
// table rows at k = 1, 2, 4, 8 and products, the multi-pass twiddle from two FP64
// anchors and an FP64 multiplication chain.
// The global load follows a.pro (PRO_PLAIN, or PRO_BPAD) and the global store a.epi
// (EPI_PLAIN, EPI_BMUL, EPI_BEXT): uniform branches, so one instantiation serves the
// plain and the fused Bluestein passes.  The Bluestein flavours address the padded
// length-M lines and map them onto the length-n lines of the input / output.
template <typename R, int RADIX, int MAXI>
__device__ __forceinline__ void stage_body(const PassArgs &a, int nb, int ns, int tw_off, bool src_g, bool dst_g,
                                           int cf, typename Cplx<R>::T *lds, const typename Cplx<R>::T *in,
                                           typename Cplx<R>::T *out, uint32_t col0, int ncl)
{
    using C = typename Cplx<R>::T;
    const int tid = threadIdx.x, T = blockDim.x;
    const int lp = a.lp;
    const float rnb = 1.0f / float(nb), rns = 1.0f / float(ns);
    const int cmask = a.c - 1;

    C v[MAXI][RADIX];
    int icol[MAXI], ib[MAXI];
    bool ok[MAXI];
#pragma unroll
    for (int i = 0; i < MAXI; ++i) {
        const int it = tid + i * T;
        int col, b;
        if (cf) {
            col = it & cmask;
            b = it >> a.logc;
        } else {
            col = div_small(it, nb, rnb);
            b = it - col * nb;
        }
        icol[i] = col;
        ib[i] = b;
        ok[i] = col < ncl && b < nb;
    }
    if (src_g) {
        const uint32_t rin = uint32_t(a.rin);
#pragma unroll
        for (int i = 0; i < MAXI; ++i) {
            if (ok[i]) {
                const ColBase cb = col_base_fast(a, col0 + uint32_t(icol[i]));
                if (a.pro == PRO_BPAD) {
                    // point e of the padded layout: line e / M, position j = e mod M
                    const C *chirp = static_cast<const C *>(a.aux);
                    const uint32_t M = uint32_t(a.bm), n = uint32_t(a.nreal);
#pragma unroll
                    for (int k = 0; k < RADIX; ++k) {
                        const uint32_t e = cb.in + uint32_t(ib[i] + k * nb) * rin;
                        const uint32_t line = line_of(e, M, a.brcp), j = e - line * M;
                        C x = C{R(0), R(0)};
                        if (j < n) {
                            x = in[line * n + j];
                            if (a.conj_in) x.y = -x.y;
                            x = c_mul(x, chirp[j]);
                        }
                        v[i][k] = x;
                    }
                } else {
                    const C *src = in + (cb.in + uint32_t(ib[i]) * rin);
#pragma unroll
                    for (int k = 0; k < RADIX; ++k) v[i][k] = gload(src + uint32_t(k * nb) * rin, a.nt_in);
                    if (a.conj_in) {
#pragma unroll
                        for (int k = 0; k < RADIX; ++k) v[i][k].y = -v[i][k].y;
                    }
                }
                if (a.tw_dim >= 0) {
                    const uint32_t j = cb.twi;
                    double2 t = pass_root(a, uint32_t(ib[i]) * j);
                    const double2 u = pass_root(a, uint32_t(nb) * j);
#pragma unroll
                    for (int k = 0; k < RADIX; ++k) {
                        if (k > 0) t = c_mul(t, u);
                        v[i][k] = c_mul(v[i][k], to_c<C>(t));
                    }
                }
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < MAXI; ++i) {
            if (ok[i]) {
                const int base = icol[i] * lp;
#pragma unroll
                for (int k = 0; k < RADIX; ++k) v[i][k] = lds[base + lds_pad<R>(ib[i] + k * nb)];
            }
        }
    }
    // this stage's twiddle rows and output positions, requested before the barrier
    const C *itw = static_cast<const C *>(a.itw) + tw_off;
    C w4[MAXI][4];
    int iq0[MAXI];
#pragma unroll
    for (int i = 0; i < MAXI; ++i) {
        const int b = ib[i];
        const int hi = div_small(b, ns, rns), lo = b - hi * ns;
        iq0[i] = hi * ns * RADIX + lo;
        if (ns > 1 && ok[i]) row_twiddle_loads<RADIX>(itw + lo * (RADIX - 1), w4[i]);
    }
    // everyone has read before anyone overwrites: LDS -> LDS stages, and a single
    // global -> global stage, which may run in place
    if (src_g == dst_g) __syncthreads();

#pragma unroll
    for (int i = 0; i < MAXI; ++i) {
        if (ok[i]) {
            if (ns > 1) {
                C w[RADIX > 1 ? RADIX : 2];
                row_twiddle_products<RADIX>(w4[i], w);
#pragma unroll
                for (int k = 1; k < RADIX; ++k) v[i][k] = c_mul(v[i][k], w[k]);
            }
            dft<RADIX>(v[i]);
            const int q0 = iq0[i];
            if (dst_g) {
                const ColBase cb = col_base_fast(a, col0 + uint32_t(icol[i]));
                const uint32_t rout = uint32_t(a.rout);
                const R sc = R(a.scale);
                if (a.epi == EPI_BMUL) {
                    // conj(Y_e B_e): the inverse transform that follows runs as a forward one
                    const C *bf = static_cast<const C *>(a.aux2);
                    const uint32_t M = uint32_t(a.bm);
#pragma unroll
                    for (int k = 0; k < RADIX; ++k) {
                        const uint32_t e = cb.out + uint32_t(q0 + k * ns) * rout;
                        out[e] = c_conj(c_mul(v[i][k], bf[e - line_of(e, M, a.brcp) * M]));
                    }
                } else if (a.epi == EPI_BEXT) {
                    // X_j = scale * w_j * conj(E_j) for positions j < n of each padded line
                    const C *chirp = static_cast<const C *>(a.aux);
                    const uint32_t M = uint32_t(a.bm), n = uint32_t(a.nreal);
#pragma unroll
                    for (int k = 0; k < RADIX; ++k) {
                        const uint32_t e = cb.out + uint32_t(q0 + k * ns) * rout;
                        const uint32_t line = line_of(e, M, a.brcp), j = e - line * M;
                        if (j < n) {
                            C y = c_scale(c_mul(chirp[j], c_conj(v[i][k])), sc);
                            if (a.conj_out) y.y = -y.y;
                            out[line * n + j] = y;
                        }
                    }
                } else {
                    C *dst = out + (cb.out + uint32_t(q0) * rout);
#pragma unroll
                    for (int k = 0; k < RADIX; ++k) {
                        C y = v[i][k];
                        if (a.conj_out) y.y = -y.y;
                        if (a.scale != 1.0) y = c_scale(y, sc);
                        gstore(dst + uint32_t(k * ns) * rout, y, a.nt_out);
                    }
                }
            } else {
                const int base = icol[i] * lp;
#pragma unroll
                for (int k = 0; k < RADIX; ++k) lds[base + lds_pad<R>(q0 + k * ns)] = v[i][k];
            }
        }
    }
    if (!dst_g) __syncthreads();
}

// One untwisted point: (Y_k + conj Y_{h-k}) - i W (Y_k - conj Y_{h-k}) with W = W_n^k.
template <typename C>
__device__ __forceinline__ C c2r_untwist(const C yk, const C ym, const C w)
{
    const C s = C{yk.x + ym.x, yk.y - ym.y};
    const C d = C{yk.x - ym.x, yk.y + ym.y};
    const C wd = c_mul(w, d);
    return C{s.x + wd.y, s.y - wd.x};
}

// Half spectrum -> conj of the z = x[2m] + i x[2m+1] spectrum into LDS:
// P_k = (Y_k + conj Y_{h-k}) - i W_n^k (Y_k - conj Y_{h-k}), Y = conj(X) (the transform
// then runs forward and conjugates on the way out).  The imaginary parts of X_0 and
// X_{n/2} do not enter (numpy semantics).  A thread owns the pair (k, h-k), so each
// bin is loaded once: P_k and P_{h-k} use the same two values.  A thread takes its pairs
// kC2rBatch at a time and issues all of their loads (bins and twiddles) before it uses
// any, so that a row pass waits on memory once per batch rather than once per pair.
constexpr int kC2rBatch = 4;
constexpr int kR2cBatch = 8;

template <typename R>
__device__ __forceinline__ void c2r_prologue(const PassArgs &a, int h, typename Cplx<R>::T *lds,
                                             const typename Cplx<R>::T *in, uint32_t col0, int ncl)
{
    using C = typename Cplx<R>::T;
    const C *wt = static_cast<const C *>(a.aux);
    const int tid = threadIdx.x, T = blockDim.x;
    const int hp = h / 2 + 1; // k = 0..h/2
    const int total = ncl * hp;
    const uint32_t rin = uint32_t(a.rin);
    for (int it0 = tid; it0 < total; it0 += kC2rBatch * T) {
        C yk[kC2rBatch], ym[kC2rBatch], wk[kC2rBatch], wm[kC2rBatch];
#pragma unroll
        for (int u = 0; u < kC2rBatch; ++u) {
            const int it = it0 + u * T;
            if (it < total) {
                const int col = it / hp, k = it % hp;
                const ColBase cb = col_base_fast(a, col0 + uint32_t(col));
                yk[u] = in[cb.in + uint32_t(k) * rin];
                ym[u] = in[cb.in + uint32_t(h - k) * rin];
                wk[u] = wt[k];
                // k = 0 has no partner below h; k = h/2 (h even) is its own partner
                if (k != 0 && 2 * k != h) wm[u] = wt[h - k];
            }
        }
#pragma unroll
        for (int u = 0; u < kC2rBatch; ++u) {
            const int it = it0 + u * T;
            if (it < total) {
                const int col = it / hp, k = it % hp;
                C y0 = yk[u], y1 = ym[u];
                if (a.conj_in) { // true spectrum in: Y = conj(X); already conjugated data passes as is
                    y0.y = -y0.y;
                    y1.y = -y1.y;
                }
                if (k == 0) {
                    y0.y = R(0);
                    y1.y = R(0);
                }
                lds[lds_index<R>(col, k, a.lp)] = c2r_untwist(y0, y1, wk[u]);
                if (k != 0 && 2 * k != h) lds[lds_index<R>(col, h - k, a.lp)] = c2r_untwist(y1, y0, wm[u]);
            }
        }
    }
    __syncthreads();
}

// z spectrum Z (length h, in LDS) -> X_k = (Z_k + conj Z_{h-k})/2 - (i/2) W_n^k (Z_k - conj Z_{h-k}),
// k = 0..h, with Z_h = Z_0.  Bins go kR2cBatch at a time per thread, their twiddle loads
// issued first.
template <typename R>
__device__ __forceinline__ void r2c_epilogue(const PassArgs &a, int h, const typename Cplx<R>::T *lds,
                                             typename Cplx<R>::T *out, uint32_t col0, int ncl)
{
    using C = typename Cplx<R>::T;
    const C *wt = static_cast<const C *>(a.aux);
    const int tid = threadIdx.x, T = blockDim.x;
    const int total = ncl * (h + 1);
    const uint32_t rout = uint32_t(a.rout);
    for (int it0 = tid; it0 < total; it0 += kR2cBatch * T) {
        C w[kR2cBatch];
#pragma unroll
        for (int u = 0; u < kR2cBatch; ++u) {
            const int it = it0 + u * T;
            if (it < total) w[u] = wt[it % (h + 1)];
        }
#pragma unroll
        for (int u = 0; u < kR2cBatch; ++u) {
            const int it = it0 + u * T;
            if (it < total) {
                const int col = it / (h + 1), k = it % (h + 1);
                const C zk = lds[lds_index<R>(col, k == h ? 0 : k, a.lp)];
                const C zm = lds[lds_index<R>(col, k == 0 ? 0 : h - k, a.lp)];
                const C s = C{zk.x + zm.x, zk.y - zm.y};
                const C d = C{zk.x - zm.x, zk.y + zm.y};
                const C wd = c_mul(w[u], d);
                const R half = R(0.5);
                const ColBase cb = col_base_fast(a, col0 + uint32_t(col));
                out[cb.out + uint32_t(k) * rout] = C{(s.x + wd.y) * half, (s.y - wd.x) * half};
            }
        }
    }
}

// ----------------------------------------------------------------------------- generic pass kernel

template <typename R, int RADIX, int PRO, int EPI, int ELEMS>
__device__ __forceinline__ void generic_stage(const PassArgs &a, int s, typename Cplx<R>::T *lds,
                                              const typename Cplx<R>::T *in, typename Cplx<R>::T *out,
                                              uint32_t col0, int ncl)
{
    constexpr int MAXI = RADIX == 1 ? 8 : (ELEMS / RADIX > 0 ? ELEMS / RADIX : 1);
    const bool first = (s == 0), last = (s == a.nst - 1);
    const int cf = first ? a.load_cf : (last ? a.store_cf : 0);
    stage_body<R, RADIX, MAXI>(a, a.L / RADIX, a.st[s].ns, a.st[s].tw, first && PRO != PRO_C2R,
                               last && EPI != EPI_R2C, cf, lds, in, out, col0, ncl);
}

// One tile (columns col0 .. col0+ncl-1) of a pass with runtime radices; ELEMS complex
// values per thread per stage (the planner sizes the group to match).
template <typename R, int PRO, int EPI, int ELEMS = RegBudget<R>::kElems>
__device__ __forceinline__ void generic_pass_tile(const PassArgs &a, typename Cplx<R>::T *lds,
                                                  const typename Cplx<R>::T *in, typename Cplx<R>::T *out,
                                                  uint32_t col0, int ncl)
{
    if constexpr (PRO == PRO_C2R) c2r_prologue<R>(a, a.L, lds, in, col0, ncl);
    for (int s = 0; s < a.nst; ++s) {
        switch (a.st[s].r) {
        case 16: generic_stage<R, 16, PRO, EPI, ELEMS>(a, s, lds, in, out, col0, ncl); break;
        case 8: generic_stage<R, 8, PRO, EPI, ELEMS>(a, s, lds, in, out, col0, ncl); break;
        case 4: generic_stage<R, 4, PRO, EPI, ELEMS>(a, s, lds, in, out, col0, ncl); break;
        case 2: generic_stage<R, 2, PRO, EPI, ELEMS>(a, s, lds, in, out, col0, ncl); break;
        case 3: generic_stage<R, 3, PRO, EPI, ELEMS>(a, s, lds, in, out, col0, ncl); break;
        case 9: generic_stage<R, 9, PRO, EPI, ELEMS>(a, s, lds, in, out, col0, ncl); break;
        case 5: generic_stage<R, 5, PRO, EPI, ELEMS>(a, s, lds, in, out, col0, ncl); break;
        case 7: generic_stage<R, 7, PRO, EPI, ELEMS>(a, s, lds, in, out, col0, ncl); break;
        case 6: generic_stage<R, 6, PRO, EPI, ELEMS>(a, s, lds, in, out, col0, ncl); break;
        case 10: generic_stage<R, 10, PRO, EPI, ELEMS>(a, s, lds, in, out, col0, ncl); break;
        case 12: generic_stage<R, 12, PRO, EPI, ELEMS>(a, s, lds, in, out, col0, ncl); break;
        case 14: generic_stage<R, 14, PRO, EPI, ELEMS>(a, s, lds, in, out, col0, ncl); break;
        case 15: generic_stage<R, 15, PRO, EPI, ELEMS>(a, s, lds, in, out, col0, ncl); break;
        default: generic_stage<R, 1, PRO, EPI, ELEMS>(a, s, lds, in, out, col0, ncl); break;
        }
    }
    if constexpr (EPI == EPI_R2C) r2c_epilogue<R>(a, a.L, lds, out, col0, ncl);
}

template <typename R, int PRO, int EPI>
__global__ void __launch_bounds__(256) k_pass(const PassArgs a, const typename Cplx<R>::T *in,
                                              typename Cplx<R>::T *out)
{
    using C = typename Cplx<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const uint32_t col0 = tile_of_block() * uint32_t(a.c);
    const int ncl = int(min(int64_t(a.c), a.ncols - int64_t(col0)));
    generic_pass_tile<R, PRO, EPI>(a, lds, in, out, col0, ncl);
}

// ----------------------------------------------------------------------------- specialised pass kernels

// Lane -> butterfly items of a specialised stage: MAXI items per thread, column-fast
// (cf) or point-fast; the tile is always c columns wide (c a power of two), items of
// columns beyond the tile's last valid one idle.
template <int RADIX, int L, int MAXI>
__device__ __forceinline__ void map_items(const PassArgs &a, int cf, int ncl, int *icol, int *ib, bool *ok)
{
    constexpr int NB = L / RADIX;
    const int tid = threadIdx.x, T = blockDim.x;
    const int cmask = a.c - 1;
#pragma unroll
    for (int i = 0; i < MAXI; ++i) {
        const int it = tid + i * T;
        int col, b;
        if (cf) {
            col = it & cmask;
            b = it >> a.logc;
        } else {
            col = it / NB;
            b = it - col * NB;
        }
        icol[i] = col;
        ib[i] = b;
        ok[i] = col < ncl && b < NB;
    }
}

// First-stage loads from global memory: points b + k*NB of each item's column (raw values;
// conj and the multi-pass twiddle are applied by fix_loaded once the loads are needed).
template <typename R, int RADIX, int L, int MAXI, bool MIR = false>
__device__ __forceinline__ void load_global(const PassArgs &a, typename Cplx<R>::T (*v)[RADIX], const int *icol,
                                            const int *ib, const bool *ok, uint32_t col0,
                                            const typename Cplx<R>::T *in)
{
    using C = typename Cplx<R>::T;
    constexpr int NB = L / RADIX;
    const uint32_t rin = uint32_t(a.rin);
#pragma unroll
    for (int i = 0; i < MAXI; ++i) {
        if (ok[i]) {
            const ColBase cb =
                col_base_fast(a, MIR ? mirror_col(a, col0, icol[i]) : col0 + uint32_t(icol[i]));
            const C *src = in + (cb.in + uint32_t(ib[i]) * rin);
#pragma unroll
            for (int k = 0; k < RADIX; ++k) v[i][k] = gload(src + uint32_t(k * NB) * rin, a.nt_in);
        }
    }
}

template <typename R, int RADIX, int L, int MAXI, bool MIR = false>
__device__ __forceinline__ void fix_loaded(const PassArgs &a, typename Cplx<R>::T (*v)[RADIX], const int *icol,
                                           const int *ib, const bool *ok, uint32_t col0)
{
    using C = typename Cplx<R>::T;
    constexpr int NB = L / RADIX;
    if (a.conj_in) {
#pragma unroll
        for (int i = 0; i < MAXI; ++i)
#pragma unroll
            for (int k = 0; k < RADIX; ++k) v[i][k].y = -v[i][k].y;
    }
    if (a.tw_dim >= 0) {
        // multi-pass twiddle W_N^{p j}, p = b + k*NB, j the column index along the twiddle
        // dim: two FP64 anchors W^{b j} and W^{NB j} from the table, then an FP64
        // multiplication chain over k (error ~k * 1e-16), rounded once to the data type
#pragma unroll
        for (int i = 0; i < MAXI; ++i) {
            if (ok[i]) {
                const uint32_t j =
                    col_base_fast(a, MIR ? mirror_col(a, col0, icol[i]) : col0 + uint32_t(icol[i])).twi;
                double2 t = pass_root(a, uint32_t(ib[i]) * j);
                const double2 u = pass_root(a, uint32_t(NB) * j);
#pragma unroll
                for (int k = 0; k < RADIX; ++k) {
                    if (k > 0) t = c_mul(t, u);
                    v[i][k] = c_mul(v[i][k], to_c<C>(t));
                }
            }
        }
    }
}

// PRO_DCT2 first-stage loads: point m = d0 + p * rin of line d1 is z_m = (v_2m, v_2m+1),
// v the reordered reals of the line (v_j = x_2j for j < n/2, else x_{2(n-1-j)+1}), read
// straight from the input reals, so the reordering never makes a pass of its own.  A tile
// reads every other real of its line segments and the mirrored tile the rest, so these
// loads stay ordinary ones whatever nt_in says: nontemporal ones evicted the lines before
// the mirror read them (DCT-II no faster, DCT-III with the same for its stores 0.94 ->
// 1.18 ms on 128 lines of 2^20 float32).
template <typename R, int RADIX, int L, int MAXI>
__device__ __forceinline__ void load_dct2(const PassArgs &a, typename Cplx<R>::T (*v)[RADIX], const int *icol,
                                          const int *ib, const bool *ok, uint32_t col0,
                                          const typename Cplx<R>::T *in)
{
    using C = typename Cplx<R>::T;
    constexpr int NB = L / RADIX;
    const R *x = reinterpret_cast<const R *>(in);
    const uint32_t n = uint32_t(a.nreal), h = n / 2u, c0 = uint32_t(a.csz[0]), rin = uint32_t(a.rin);
    auto src = [&](uint32_t j) { return j < h ? 2u * j : 2u * (n - 1u - j) + 1u; };
#pragma unroll
    for (int i = 0; i < MAXI; ++i) {
        if (ok[i]) {
            const uint32_t f = col0 + uint32_t(icol[i]);
            const uint32_t line = a.ncd > 1 ? div_rcp(f, c0, a.crcp[0]) : 0u;
            const R *xl = x + uint64_t(line) * n;
            const uint32_t d0 = f - line * c0;
#pragma unroll
            for (int k = 0; k < RADIX; ++k) {
                const uint32_t m = d0 + uint32_t(ib[i] + k * NB) * rin;
                v[i][k] = C{xl[src(2u * m)], xl[src(2u * m + 1u)]};
            }
        }
    }
}

// PRO_SYM: scale each loaded point by the real symbol S_p[p] + S_0[d0] (+ S_1[d1]), p the
// point's index along the pass and d0, d1 its column's first digits (FP64 tables in
// aux: S_p over the L points, then S_0 over csz[0], then S_1 over csz[1]); the sum is
// rounded once to the data type.
template <typename R, int RADIX, int L, int MAXI>
__device__ __forceinline__ void apply_symbol(const PassArgs &a, typename Cplx<R>::T (*v)[RADIX], const int *icol,
                                             const int *ib, const bool *ok, uint32_t col0)
{
    constexpr int NB = L / RADIX;
    const double *S = static_cast<const double *>(a.aux);
    const uint32_t c0 = uint32_t(a.csz[0]);
#pragma unroll
    for (int i = 0; i < MAXI; ++i) {
        if (ok[i]) {
            const uint32_t f = col0 + uint32_t(icol[i]);
            const uint32_t q = a.ncd > 1 ? div_rcp(f, c0, a.crcp[0]) : 0u;
            double base = S[L + (f - q * c0)];
            if (a.sym_cd == 2) {
                const uint32_t c1 = uint32_t(a.csz[1]);
                const uint32_t d1 = a.ncd > 2 ? q - div_rcp(q, c1, a.crcp[1]) * c1 : q;
                base += S[L + c0 + d1];
            }
#pragma unroll
            for (int k = 0; k < RADIX; ++k) {
                const R s = R(S[ib[i] + k * NB] + base);
                v[i][k].x *= s;
                v[i][k].y *= s;
            }
        }
    }
}

// Inner twiddles, butterflies and the scatter to points (b/NS)*NS*RADIX + b%NS + k*NS of
// LDS or (DST_G) global memory, there as complex values or (LEPI == EPI_DCT3) as the two
// reals of each point put back in natural order.
template <typename R, int RADIX, int L, int NS, int TWOFF, int MAXI, bool DST_G, int LEPI = EPI_PLAIN,
          bool MIR = false>
__device__ __forceinline__ void compute_scatter(const PassArgs &a, typename Cplx<R>::T (*v)[RADIX], const int *icol,
                                                const int *ib, const bool *ok, typename Cplx<R>::T *lds,
                                                typename Cplx<R>::T *out, uint32_t col0)
{
    using C = typename Cplx<R>::T;
    constexpr bool LIN = IsPow2<L>::v;
    const int lp = a.lp;
    if constexpr (NS > 1) {
        const C *itw = static_cast<const C *>(a.itw) + TWOFF;
#pragma unroll
        for (int i = 0; i < MAXI; ++i) {
            if (ok[i]) {
                C w[RADIX];
                row_twiddles<RADIX>(itw + (ib[i] % NS) * (RADIX - 1), w);
#pragma unroll
                for (int k = 1; k < RADIX; ++k) v[i][k] = c_mul(v[i][k], w[k]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < MAXI; ++i)
        if (ok[i]) dft<RADIX>(v[i]);
    if constexpr (DST_G) {
        if (a.conj_out) {
#pragma unroll
            for (int i = 0; i < MAXI; ++i)
#pragma unroll
                for (int k = 0; k < RADIX; ++k) v[i][k].y = -v[i][k].y;
        }
        if (a.scale != 1.0) {
            const R sc = R(a.scale);
#pragma unroll
            for (int i = 0; i < MAXI; ++i)
#pragma unroll
                for (int k = 0; k < RADIX; ++k) v[i][k] = c_scale(v[i][k], sc);
        }
        const uint32_t rout = uint32_t(a.rout);
        if constexpr (LEPI == EPI_DCT3) {
            // point m = d0 + q * rout of line d1 holds (v_2m, v_2m+1); ordinary stores
            // whatever nt_out says (the mirrored tile writes the other half of each line)
            R *y = reinterpret_cast<R *>(out);
            const uint32_t n = uint32_t(a.nreal), h = n / 2u, c0 = uint32_t(a.csz[0]);
            auto dst = [&](uint32_t j) { return j < h ? 2u * j : 2u * (n - 1u - j) + 1u; };
#pragma unroll
            for (int i = 0; i < MAXI; ++i) {
                if (ok[i]) {
                    const int b = ib[i];
                    const int q0 = (b / NS) * NS * RADIX + (b % NS);
                    const uint32_t f = col0 + uint32_t(icol[i]);
                    const uint32_t line = a.ncd > 1 ? div_rcp(f, c0, a.crcp[0]) : 0u;
                    R *yl = y + uint64_t(line) * n;
                    const uint32_t d0 = f - line * c0;
#pragma unroll
                    for (int k = 0; k < RADIX; ++k) {
                        const uint32_t m = d0 + uint32_t(q0 + k * NS) * rout;
                        yl[dst(2u * m)] = v[i][k].x;
                        yl[dst(2u * m + 1u)] = v[i][k].y;
                    }
                }
            }
            return;
        }
#pragma unroll
        for (int i = 0; i < MAXI; ++i) {
            if (ok[i]) {
                const int b = ib[i];
                const int q0 = (b / NS) * NS * RADIX + (b % NS);
                const ColBase cb =
                    col_base_fast(a, MIR ? mirror_col(a, col0, icol[i]) : col0 + uint32_t(icol[i]));
                C *dst = out + (cb.out + uint32_t(q0) * rout);
#pragma unroll
                for (int k = 0; k < RADIX; ++k) gstore(dst + uint32_t(k * NS) * rout, v[i][k], a.nt_out);
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < MAXI; ++i) {
            if (ok[i]) {
                const int b = ib[i];
                const int q0 = (b / NS) * NS * RADIX + (b % NS);
                const int base = icol[i] * lp;
                if constexpr (LIN) {
                    const int s0 = base + lds_pad<R>(q0);
#pragma unroll
                    for (int k = 0; k < RADIX; ++k) lds[s0 + lds_pad<R>(k * NS)] = v[i][k];
                } else {
#pragma unroll
                    for (int k = 0; k < RADIX; ++k) lds[base + lds_pad<R>(q0 + k * NS)] = v[i][k];
                }
            }
        }
    }
}

// One stage of a specialised kernel.  NB = L/RADIX butterflies per column, NS = product of
// the earlier radices, TWOFF = offset of this stage's twiddle rows.  SRC_G / DST_G: the
// stage reads / writes global memory rather than LDS; LPRO / LEPI: the prologue of those
// loads (PRO_PLAIN, PRO_SYM or PRO_DCT2) and the epilogue of those stores (EPI_PLAIN or
// EPI_DCT3).
template <typename R, int RADIX, int L, int NS, int TWOFF, bool SRC_G, bool DST_G, int LPRO = PRO_PLAIN,
          int LEPI = EPI_PLAIN, bool MIR = false>
__device__ __forceinline__ void fixed_stage_body(const PassArgs &a, int cf, typename Cplx<R>::T *lds,
                                                 const typename Cplx<R>::T *in, typename Cplx<R>::T *out,
                                                 uint32_t col0, int ncl)
{
    using C = typename Cplx<R>::T;
    constexpr int NB = L / RADIX;
    constexpr int MAXI = RADIX == 1 ? 8 : kFixedElems / RADIX;
    constexpr bool LIN = IsPow2<L>::v;
    const int lp = a.lp;
    C v[MAXI][RADIX];
    int icol[MAXI], ib[MAXI];
    bool ok[MAXI];
    map_items<RADIX, L, MAXI>(a, cf, ncl, icol, ib, ok);
    if constexpr (SRC_G) {
        if constexpr (LPRO == PRO_DCT2)
            load_dct2<R, RADIX, L, MAXI>(a, v, icol, ib, ok, col0, in);
        else
            load_global<R, RADIX, L, MAXI, MIR>(a, v, icol, ib, ok, col0, in);
        fix_loaded<R, RADIX, L, MAXI, MIR>(a, v, icol, ib, ok, col0);
        if constexpr (LPRO == PRO_SYM) apply_symbol<R, RADIX, L, MAXI>(a, v, icol, ib, ok, col0);
    } else {
#pragma unroll
        for (int i = 0; i < MAXI; ++i) {
            if (ok[i]) {
                const int b = ib[i];
                const int base = icol[i] * lp;
                if constexpr (LIN) {
                    const int q0 = base + lds_pad<R>(b);
#pragma unroll
                    for (int k = 0; k < RADIX; ++k) v[i][k] = lds[q0 + lds_pad<R>(k * NB)];
                } else {
#pragma unroll
                    for (int k = 0; k < RADIX; ++k) v[i][k] = lds[base + lds_pad<R>(b + k * NB)];
                }
            }
        }
    }
    // everyone has read before anyone overwrites: LDS -> LDS stages, and a single
    // global -> global stage, which may run in place
    if constexpr (SRC_G == DST_G) __syncthreads();
    compute_scatter<R, RADIX, L, NS, TWOFF, MAXI, DST_G, LEPI, MIR>(a, v, icol, ib, ok, lds, out, col0);
    if constexpr (!DST_G) __syncthreads();
}

template <int... Rs> struct Seq {
    static constexpr int n = sizeof...(Rs);
    static constexpr int r[n] = {Rs...};
    static constexpr int L = (Rs * ... * 1);
    static constexpr int ns(int s) { return s == 0 ? 1 : ns(s - 1) * r[s - 1]; }
    static constexpr int tw(int s) { return s == 0 ? 0 : tw(s - 1) + ns(s - 1) * (r[s - 1] - 1); }
};

template <typename R, int PRO, int EPI, typename S, int s>
__device__ __forceinline__ void fixed_stage(const PassArgs &a, typename Cplx<R>::T *lds,
                                            const typename Cplx<R>::T *in, typename Cplx<R>::T *out, uint32_t col0,
                                            int ncl)
{
    constexpr int RADIX = S::r[s];
    constexpr bool first = s == 0, last = s == S::n - 1;
    const int cf = first ? a.load_cf : (last ? a.store_cf : 0);
    constexpr bool src_g = first && (PRO == PRO_PLAIN || PRO == PRO_SYM || PRO == PRO_DCT2);
    constexpr bool dst_g = last && (EPI == EPI_PLAIN || EPI == EPI_DCT3);
    constexpr bool mir = EPI == EPI_RTWIST || EPI == EPI_DTWIST || PRO == PRO_CUNTWIST;
    fixed_stage_body<R, RADIX, S::L, S::ns(s), S::tw(s), src_g, dst_g, first ? PRO : PRO_PLAIN,
                     last ? EPI : EPI_PLAIN, mir>(a, cf, lds, in, out, col0, ncl);
}

template <typename R, int PRO, int EPI, typename S, int... I>
__device__ __forceinline__ void fixed_stages(const PassArgs &a, typename Cplx<R>::T *lds,
                                             const typename Cplx<R>::T *in, typename Cplx<R>::T *out,
                                             uint32_t col0, int ncl, std::integer_sequence<int, I...>)
{
    (fixed_stage<R, PRO, EPI, S, I>(a, lds, in, out, col0, ncl), ...);
}

// The c2r untwist of a mirrored-tile first pass (PRO_CUNTWIST) into LDS: a thread takes a
// bin pair (Y_m, Y_{h-m}), m = j + J p, and writes P_m to slot s, point p and P_{h-m} to
// the partner (point L-1-p of the mirror slot; for column J/2 of the same slot; for
// column 0 point L-p of the same slot, and Y_h with Y_0).  The low slots of a tile take
// L pairs each; the tile holding column 0 runs column 0 (L/2 + 1 pairs) and column J/2
// (L/2 pairs) in a second loop.
template <typename R>
__device__ __forceinline__ void cuntwist_prologue(const PassArgs &a, int L, typename Cplx<R>::T *lds,
                                                  const typename Cplx<R>::T *in, uint32_t col0)
{
    using C = typename Cplx<R>::T;
    const C *wn = static_cast<const C *>(a.aux);
    const uint32_t J = uint32_t(a.csz[0]), half = uint32_t(a.c) >> 1;
    const uint32_t line = a.ncd > 1 ? div_rcp(col0, J, a.crcp[0]) : 0u;
    const uint32_t t = (col0 - line * J) / uint32_t(a.c);
    const uint32_t h = uint32_t(a.nreal) >> 1, rin = uint32_t(a.rin);
    const C *y = in + uint64_t(line) * uint64_t(a.cin[1]);
    const R cs = a.conj_in ? R(-1) : R(1);
    auto pair = [&](uint32_t m, uint32_t mm, int s, int p, int s2, int p2, bool both) {
        C ya = y[m], yb = y[mm];
        ya.y *= cs;
        yb.y *= cs;
        if (m == 0u) {
            ya.y = R(0);
            yb.y = R(0);
        }
        lds[lds_index<R>(s, p, a.lp)] = c2r_untwist(ya, yb, wn[m]);
        if (both) lds[lds_index<R>(s2, p2, a.lp)] = c2r_untwist(yb, ya, wn[mm]);
    };
    const int lowL = int(half) * L;
    for (int it = threadIdx.x; it < lowL; it += blockDim.x) {
        const int s = it & int(half - 1u), p = it >> (a.logc - 1); // c/2 a power of two
        const uint32_t j = t * half + uint32_t(s);
        if (j == 0u) continue; // column 0 and its partner column J/2: the loop below
        const uint32_t m = j + J * uint32_t(p);
        pair(m, h - m, s, p, s + int(half), L - 1 - p, true);
    }
    if (t == 0u) {
        for (int q = threadIdx.x; q <= L; q += blockDim.x) {
            if (q <= L / 2) { // column 0, slot 0: (p, L-p); p = 0 with Y_h; p = L/2 itself
                const uint32_t m = J * uint32_t(q);
                pair(m, h - m, 0, q, 0, L - q, q != 0 && 2 * q != L);
            } else { // column J/2, slot c/2: (p, L-1-p)
                const int p = q - L / 2 - 1;
                const uint32_t m = (J >> 1) + J * uint32_t(p);
                pair(m, h - m, int(half), p, int(half), L - 1 - p, true);
            }
        }
    }
    __syncthreads();
}

// The twist of a mirrored-tile pass (EPI_RTWIST / EPI_DTWIST) from the tile in LDS: slot s,
// point p holds Z_m, m = j + J p (j the slot's column); its partner Z_{h-m} is point
// L-1-p of the mirror slot, or of the same slot for j = J/2, or point (L-p) mod L of the
// same slot for j = 0 (Z_h = Z_0).  Every point gives X_m; the point m = 0 also X_h.
template <typename R, int EPI>
__device__ __forceinline__ void twist_epilogue(const PassArgs &a, int L, const typename Cplx<R>::T *lds,
                                               typename Cplx<R>::T *out, uint32_t col0)
{
    using C = typename Cplx<R>::T;
    const C *wn = static_cast<const C *>(a.aux);
    const uint32_t J = uint32_t(a.csz[0]), c = uint32_t(a.c), half = c >> 1;
    const uint32_t line = a.ncd > 1 ? div_rcp(col0, J, a.crcp[0]) : 0u;
    const uint32_t t = (col0 - line * J) / c;
    const uint32_t n = uint32_t(a.nreal), h = n >> 1;
    const int total = int(c) * L;
    const R hf = R(0.5);
    for (int it = threadIdx.x; it < total; it += blockDim.x) {
        const int s = it & int(c - 1u), p = it >> a.logc;
        const bool low = uint32_t(s) < half;
        const uint32_t jl = t * half + (low ? uint32_t(s) : uint32_t(s) - half);
        const uint32_t j = low ? jl : (jl == 0u ? J >> 1 : J - jl);
        int sp = s, pp = L - 1 - p;
        if (j == 0u)
            pp = p == 0 ? 0 : L - p;
        else if (j != (J >> 1))
            sp = low ? s + int(half) : s - int(half);
        const C zk = lds[lds_index<R>(s, p, a.lp)];
        const C zm = lds[lds_index<R>(sp, pp, a.lp)];
        const uint32_t m = j + J * uint32_t(p);
        const C w = wn[m];
        const C sm = C{zk.x + zm.x, zk.y - zm.y};
        const C d = C{zk.x - zm.x, zk.y + zm.y};
        const C wd = c_mul(w, d);
        const C x = C{(sm.x + wd.y) * hf, (sm.y - wd.x) * hf};
        if constexpr (EPI == EPI_RTWIST) {
            C *o = out + uint64_t(line) * uint64_t(a.bm);
            o[m] = x;
            if (m == 0u) o[h] = C{zk.x - zk.y, R(0)};
        } else {
            const C *w4 = static_cast<const C *>(a.aux2);
            R *y = reinterpret_cast<R *>(out) + uint64_t(line) * uint64_t(a.bm);
            const C wa = w4[m];
            y[m] = R(2) * (x.x * wa.x - x.y * wa.y);
            if (m != 0u) {
                const C wb = w4[n - m];
                y[n - m] = R(2) * (x.x * wb.x + x.y * wb.y);
            } else {
                const C wh = w4[h];
                y[h] = R(2) * (zk.x - zk.y) * wh.x;
            }
        }
    }
}

template <typename R, int PRO, int EPI, int... Rs>
__global__ void __launch_bounds__(FixedMaxThreads<R>::v) k_pass_fixed(const PassArgs a, const typename Cplx<R>::T *in,
                                                                 typename Cplx<R>::T *out)
{
    using C = typename Cplx<R>::T;
    using S = Seq<Rs...>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *lds = reinterpret_cast<C *>(smem_raw);
    const uint32_t col0 = tile_of_block() * uint32_t(a.c);
    const int ncl = int(min(int64_t(a.c), a.ncols - int64_t(col0)));
    if constexpr (PRO == PRO_C2R) c2r_prologue<R>(a, S::L, lds, in, col0, ncl);
    if constexpr (PRO == PRO_CUNTWIST) cuntwist_prologue<R>(a, S::L, lds, in, col0);
    fixed_stages<R, PRO, EPI, S>(a, lds, in, out, col0, ncl, std::make_integer_sequence<int, S::n>{});
    if constexpr (EPI == EPI_R2C) r2c_epilogue<R>(a, S::L, lds, out, col0, ncl);
    if constexpr (EPI == EPI_RTWIST || EPI == EPI_DTWIST) twist_epilogue<R, EPI>(a, S::L, lds, out, col0);
}

// Specialised kernels only, in MIFFT_FIXED_SHAPES order (null for any other shape): for
// flavours the runtime-radix kernel does not implement.
template <typename R, int PRO, int EPI> const void *fixed_kernel_table(int shape)
{
#define MIFFT_KPTR(...) reinterpret_cast<const void *>(&k_pass_fixed<R, PRO, EPI, __VA_ARGS__>),
    static const void *const table[] = {MIFFT_FIXED_SHAPES(MIFFT_KPTR)};
#undef MIFFT_KPTR
    const int count = int(sizeof(table) / sizeof(table[0]));
    return shape >= 0 && shape < count ? table[shape] : nullptr;
}

// Kernel table of one (type, prologue, epilogue) flavour: the specialised kernels in
// MIFFT_FIXED_SHAPES order, and the runtime-radix kernel for any other shape.
template <typename R, int PRO, int EPI> const void *pass_kernel_table(int shape)
{
#define MIFFT_KPTR(...) reinterpret_cast<const void *>(&k_pass_fixed<R, PRO, EPI, __VA_ARGS__>),
    static const void *const table[] = {MIFFT_FIXED_SHAPES(MIFFT_KPTR)};
#undef MIFFT_KPTR
    const int count = int(sizeof(table) / sizeof(table[0]));
    if (shape >= 0 && shape < count) return table[shape];
    return reinterpret_cast<const void *>(&k_pass<R, PRO, EPI>);
}

} // namespace mifft
