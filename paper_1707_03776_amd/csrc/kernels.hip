// gfx950 kernels of the transform: the Stockham pass (k_pass), the element-wise
// kernels around it (Bluestein, real-data staging) and the FP64 table generators.
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

__device__ __forceinline__ ColBase col_base(const PassArgs &a, uint32_t f)
{
    ColBase cb;
    uint32_t d[kColDims];
    d[0] = f % uint32_t(a.csz[0]);
    f /= uint32_t(a.csz[0]);
    d[1] = f % uint32_t(a.csz[1]);
    f /= uint32_t(a.csz[1]);
    d[2] = f % uint32_t(a.csz[2]);
    d[3] = f / uint32_t(a.csz[2]);
    cb.in = d[0] * uint32_t(a.cin[0]) + d[1] * uint32_t(a.cin[1]) + d[2] * uint32_t(a.cin[2]) +
            d[3] * uint32_t(a.cin[3]);
    cb.out = d[0] * uint32_t(a.cout[0]) + d[1] * uint32_t(a.cout[1]) + d[2] * uint32_t(a.cout[2]) +
             d[3] * uint32_t(a.cout[3]);
    cb.twi = a.tw_dim >= 0 ? d[a.tw_dim] : 0u;
    return cb;
}

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
                    for (int k = 0; k < RADIX; ++k) v[i][k] = src[uint32_t(k * nb) * rin];
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
                        dst[uint32_t(k * ns) * rout] = y;
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
// bin is loaded once: P_k and P_{h-k} use the same two values.
template <typename R>
__device__ __forceinline__ void c2r_prologue(const PassArgs &a, int h, typename Cplx<R>::T *lds,
                                             const typename Cplx<R>::T *in, uint32_t col0, int ncl)
{
    using C = typename Cplx<R>::T;
    const C *wt = static_cast<const C *>(a.aux);
    const int tid = threadIdx.x, T = blockDim.x;
    const int hp = h / 2 + 1; // k = 0..h/2
    for (int it = tid; it < ncl * hp; it += T) {
        const int col = it / hp, k = it % hp;
        const ColBase cb = col_base(a, col0 + uint32_t(col));
        C yk = in[cb.in + uint32_t(k) * uint32_t(a.rin)];
        C ym = in[cb.in + uint32_t(h - k) * uint32_t(a.rin)];
        if (a.conj_in) { // true spectrum in: Y = conj(X); already conjugated data passes as is
            yk.y = -yk.y;
            ym.y = -ym.y;
        }
        if (k == 0) {
            yk.y = R(0);
            ym.y = R(0);
        }
        lds[lds_index<R>(col, k, a.lp)] = c2r_untwist(yk, ym, wt[k]);
        // k = 0 has no partner below h; k = h/2 (h even) is its own partner
        if (k != 0 && 2 * k != h) lds[lds_index<R>(col, h - k, a.lp)] = c2r_untwist(ym, yk, wt[h - k]);
    }
    __syncthreads();
}

// z spectrum Z (length h, in LDS) -> X_k = (Z_k + conj Z_{h-k})/2 - (i/2) W_n^k (Z_k - conj Z_{h-k}),
// k = 0..h, with Z_h = Z_0.
template <typename R>
__device__ __forceinline__ void r2c_epilogue(const PassArgs &a, int h, const typename Cplx<R>::T *lds,
                                             typename Cplx<R>::T *out, uint32_t col0, int ncl)
{
    using C = typename Cplx<R>::T;
    const C *wt = static_cast<const C *>(a.aux);
    const int tid = threadIdx.x, T = blockDim.x;
    for (int it = tid; it < ncl * (h + 1); it += T) {
        const int col = it / (h + 1), k = it % (h + 1);
        const C zk = lds[lds_index<R>(col, k == h ? 0 : k, a.lp)];
        const C zm = lds[lds_index<R>(col, k == 0 ? 0 : h - k, a.lp)];
        const C s = C{zk.x + zm.x, zk.y - zm.y};
        const C d = C{zk.x - zm.x, zk.y + zm.y};
        const C wd = c_mul(wt[k], d);
        const R half = R(0.5);
        const ColBase cb = col_base(a, col0 + uint32_t(col));
        out[cb.out + uint32_t(k) * uint32_t(a.rout)] = C{(s.x + wd.y) * half, (s.y - wd.x) * half};
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
template <typename R, int RADIX, int L, int MAXI>
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
            const ColBase cb = col_base_fast(a, col0 + uint32_t(icol[i]));
            const C *src = in + (cb.in + uint32_t(ib[i]) * rin);
#pragma unroll
            for (int k = 0; k < RADIX; ++k) v[i][k] = src[uint32_t(k * NB) * rin];
        }
    }
}

template <typename R, int RADIX, int L, int MAXI>
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
                const uint32_t j = col_base_fast(a, col0 + uint32_t(icol[i])).twi;
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

// Inner twiddles, butterflies and the scatter to points (b/NS)*NS*RADIX + b%NS + k*NS of
// LDS or (DST_G) global memory.
template <typename R, int RADIX, int L, int NS, int TWOFF, int MAXI, bool DST_G>
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
#pragma unroll
        for (int i = 0; i < MAXI; ++i) {
            if (ok[i]) {
                const int b = ib[i];
                const int q0 = (b / NS) * NS * RADIX + (b % NS);
                const ColBase cb = col_base_fast(a, col0 + uint32_t(icol[i]));
                C *dst = out + (cb.out + uint32_t(q0) * rout);
#pragma unroll
                for (int k = 0; k < RADIX; ++k) dst[uint32_t(k * NS) * rout] = v[i][k];
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
// stage reads / writes global memory rather than LDS.
template <typename R, int RADIX, int L, int NS, int TWOFF, bool SRC_G, bool DST_G>
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
        load_global<R, RADIX, L, MAXI>(a, v, icol, ib, ok, col0, in);
        fix_loaded<R, RADIX, L, MAXI>(a, v, icol, ib, ok, col0);
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
    compute_scatter<R, RADIX, L, NS, TWOFF, MAXI, DST_G>(a, v, icol, ib, ok, lds, out, col0);
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
    fixed_stage_body<R, RADIX, S::L, S::ns(s), S::tw(s), first && PRO == PRO_PLAIN, last && EPI == EPI_PLAIN>(
        a, cf, lds, in, out, col0, ncl);
}

template <typename R, int PRO, int EPI, typename S, int... I>
__device__ __forceinline__ void fixed_stages(const PassArgs &a, typename Cplx<R>::T *lds,
                                             const typename Cplx<R>::T *in, typename Cplx<R>::T *out,
                                             uint32_t col0, int ncl, std::integer_sequence<int, I...>)
{
    (fixed_stage<R, PRO, EPI, S, I>(a, lds, in, out, col0, ncl), ...);
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
    fixed_stages<R, PRO, EPI, S>(a, lds, in, out, col0, ncl, std::make_integer_sequence<int, S::n>{});
    if constexpr (EPI == EPI_R2C) r2c_epilogue<R>(a, S::L, lds, out, col0, ncl);
}

// ----------------------------------------------------------------------------- split-BF16 MFMA radix-16

// A radix-16 butterfly Y = F16 X is a product with the real 32x32 matrix acting on the
// interleaved vector (x0.re, x0.im, x1.re, ..., x15.im): row 2k of block [Y_k.re] holds
// (cos, sin)(2 pi jk/16) against (x_j.re, x_j.im), row 2k+1 [Y_k.im] holds (-sin, cos).
// v_mfma_f32_16x16x32_bf16 computes D(16x16) = A(16x32) B(32x16) + D with, per lane l,
// A[l%16][8(l/16)+i], B[8(l/16)+i][l%16], D[4(l/16)+i][l%16] (i < 8, 8, 4).  With 16
// butterflies as the 16 columns of B, lane (n, g) = (l%16, l/16) supplies the 4 complex
// points 4g..4g+3 of butterfly n and receives complete complex outputs 2g, 2g+1 (block
// of outputs 0..7) and 8+2g, 9+2g (block 8..15).  Operands are split x = hi + lo
// (+ mid) in BF16; the products with combined weight above 2^-24 are accumulated in FP32:
// 3 per block for the two-term split, 6 for the three-term one.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// x = parts[0] + parts[1] (+ parts[2]), each rounded to nearest-even BF16 from what
// remains (the casts are gfx950's packed FP32 -> BF16 conversion)
template <int NSPLIT> __device__ __forceinline__ void split_bf16(float x, __bf16 *parts)
{
    float r = x;
#pragma unroll
    for (int t = 0; t < NSPLIT; ++t) {
        parts[t] = __bf16(r);
        if (t + 1 < NSPLIT) r -= float(parts[t]);
    }
}

// cos/sin(2 pi m/16), m = 0..15
__device__ __forceinline__ float cos16(int m)
{
    const float c1 = 0.92387953251128675613f, c2 = 0.70710678118654752440f, c3 = 0.38268343236508977173f;
    const float t[16] = {1.f, c1, c2, c3, 0.f, -c3, -c2, -c1, -1.f, -c1, -c2, -c3, 0.f, c3, c2, c1};
    return t[m & 15];
}
__device__ __forceinline__ float sin16(int m) { return cos16(m - 4); }

template <int NSPLIT> struct Mfma16Operands {
    bf16x8 a1[NSPLIT], a2[NSPLIT]; // DFT matrix rows for outputs 0..7 and 8..15, split
};

template <int NSPLIT> __device__ __forceinline__ Mfma16Operands<NSPLIT> dft16_operands(int lane)
{
    Mfma16Operands<NSPLIT> op;
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        const int k = blk * 8 + (r >> 1), comp = r & 1;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int j = 4 * g + (i >> 1), ic = i & 1;
            const int m = (j * k) & 15;
            const float c = cos16(m), sn = sin16(m);
            const float v = comp == 0 ? (ic == 0 ? c : sn) : (ic == 0 ? -sn : c);
            __bf16 parts[NSPLIT];
            split_bf16<NSPLIT>(v, parts);
#pragma unroll
            for (int t = 0; t < NSPLIT; ++t) {
                if (blk == 0) op.a1[t][i] = parts[t];
                else op.a2[t][i] = parts[t];
            }
        }
    }
    return op;
}

template <int NSPLIT>
__device__ __forceinline__ f32x4 mfma16_block(const bf16x8 *a, const bf16x8 *b)
{
    f32x4 d = {0.f, 0.f, 0.f, 0.f};
    if constexpr (NSPLIT == 2) {
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], d, 0, 0, 0);
    } else {
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1], d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0], d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2], d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], d, 0, 0, 0);
    }
    return d;
}

// One radix-16 stage on the matrix cores.  Same data movement contract as
// fixed_stage_body<float, 16, ...>: butterfly b of a column reads points b + k*NB
// (twiddled by W_{16 NS}^{k (b mod NS)}, or by the multi-pass twiddle in a first
// stage) and writes points (b/NS)*16*NS + b%NS + k*NS.  A wave handles 16 butterflies
// at a time; the MFMA runs for the whole wave (lanes without a butterfly feed zeros).
template <int NSPLIT, int L, int NS, int TWOFF, bool SRC_G, bool DST_G>
__device__ __forceinline__ void mfma16_stage(const PassArgs &a, int cf, float2 *lds, const float2 *in, float2 *out,
                                             uint32_t col0, int ncl)
{
    constexpr int NB = L / 16;
    constexpr int MAXG = kFixedElems / 4; // groups of 16 butterflies per wave
    constexpr bool LIN = IsPow2<L>::v;
    const int tid = threadIdx.x, T = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwaves = T >> 6;
    const int n = lane & 15, g = lane >> 4;
    const int lp = a.lp, cmask = a.c - 1;
    const int nbt = a.c * NB; // butterflies in a full tile

    const Mfma16Operands<NSPLIT> A = dft16_operands<NSPLIT>(lane);

    float2 x[MAXG][4];
    int icol[MAXG], ib[MAXG];
    bool ok[MAXG];
#pragma unroll
    for (int it = 0; it < MAXG; ++it) {
        const int bt = (wave + it * nwaves) * 16 + n;
        int col, b;
        if (cf) {
            col = bt & cmask;
            b = bt >> a.logc;
        } else {
            col = bt / NB;
            b = bt - col * NB;
        }
        icol[it] = col;
        ib[it] = b;
        ok[it] = bt < nbt && col < ncl;
#pragma unroll
        for (int t = 0; t < 4; ++t) x[it][t] = float2{0.f, 0.f};
        if (ok[it]) {
            if constexpr (SRC_G) {
                const ColBase cb = col_base_fast(a, col0 + uint32_t(col));
                const uint32_t rin = uint32_t(a.rin);
                const float2 *src = in + (cb.in + uint32_t(b) * rin);
#pragma unroll
                for (int t = 0; t < 4; ++t) x[it][t] = src[uint32_t((4 * g + t) * NB) * rin];
                if (a.conj_in) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) x[it][t].y = -x[it][t].y;
                }
                if (a.tw_dim >= 0) {
                    double2 w = pass_root(a, uint32_t(b + 4 * g * NB) * cb.twi);
                    const double2 u = pass_root(a, uint32_t(NB) * cb.twi);
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        if (t > 0) w = c_mul(w, u);
                        x[it][t] = c_mul(x[it][t], to_c<float2>(w));
                    }
                }
            } else {
                const int base = col * lp;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int q = b + (4 * g + t) * NB;
                    x[it][t] = LIN ? lds[base + lds_pad<float>(b) + lds_pad<float>((4 * g + t) * NB)]
                                   : lds[base + lds_pad<float>(q)];
                }
            }
            if constexpr (NS > 1) {
                const float2 *row = static_cast<const float2 *>(a.itw) + TWOFF + (b % NS) * 15;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int k = 4 * g + t;
                    if (k > 0) x[it][t] = c_mul(x[it][t], row[k - 1]);
                }
            }
        }
    }
    if constexpr (SRC_G == DST_G) __syncthreads();

    // all products first (independent accumulation chains overlap in the matrix
    // pipeline), then the scatter
    f32x4 d1s[MAXG], d2s[MAXG];
#pragma unroll
    for (int it = 0; it < MAXG; ++it) {
        if ((wave + it * nwaves) * 16 >= nbt) continue; // uniform per wave
        bf16x8 bsp[NSPLIT];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            __bf16 pr[NSPLIT], pi[NSPLIT];
            split_bf16<NSPLIT>(x[it][t].x, pr);
            split_bf16<NSPLIT>(x[it][t].y, pi);
#pragma unroll
            for (int u = 0; u < NSPLIT; ++u) {
                bsp[u][2 * t] = pr[u];
                bsp[u][2 * t + 1] = pi[u];
            }
        }
        d1s[it] = mfma16_block<NSPLIT>(A.a1, bsp);
        d2s[it] = mfma16_block<NSPLIT>(A.a2, bsp);
    }
#pragma unroll
    for (int it = 0; it < MAXG; ++it) {
        if (!ok[it]) continue;
        const f32x4 d1 = d1s[it], d2 = d2s[it];
        float2 y[4] = {float2{d1[0], d1[1]}, float2{d1[2], d1[3]}, float2{d2[0], d2[1]}, float2{d2[2], d2[3]}};
        const int ks[4] = {2 * g, 2 * g + 1, 8 + 2 * g, 9 + 2 * g};
        const int b = ib[it];
        const int q0 = (b / NS) * NS * 16 + (b % NS);
        if constexpr (DST_G) {
            if (a.conj_out) {
#pragma unroll
                for (int t = 0; t < 4; ++t) y[t].y = -y[t].y;
            }
            if (a.scale != 1.0) {
                const float sc = float(a.scale);
#pragma unroll
                for (int t = 0; t < 4; ++t) y[t] = c_scale(y[t], sc);
            }
            const ColBase cb = col_base_fast(a, col0 + uint32_t(icol[it]));
            const uint32_t rout = uint32_t(a.rout);
            float2 *dst = out + (cb.out + uint32_t(q0) * rout);
#pragma unroll
            for (int t = 0; t < 4; ++t) dst[uint32_t(ks[t] * NS) * rout] = y[t];
        } else {
            const int base = icol[it] * lp;
#pragma unroll
            for (int t = 0; t < 4; ++t) lds[base + lds_pad<float>(q0 + ks[t] * NS)] = y[t];
        }
    }
    if constexpr (!DST_G) __syncthreads();
}

template <int NSPLIT, typename S, int s>
__device__ __forceinline__ void mfma_pass_stage(const PassArgs &a, float2 *lds, const float2 *in, float2 *out,
                                                uint32_t col0, int ncl)
{
    constexpr int RADIX = S::r[s];
    constexpr bool first = s == 0, last = s == S::n - 1;
    const int cf = first ? a.load_cf : (last ? a.store_cf : 0);
    if constexpr (RADIX == 16)
        mfma16_stage<NSPLIT, S::L, S::ns(s), S::tw(s), first, last>(a, cf, lds, in, out, col0, ncl);
    else
        fixed_stage_body<float, RADIX, S::L, S::ns(s), S::tw(s), first, last>(a, cf, lds, in, out, col0, ncl);
}

template <int NSPLIT, typename S, int... I>
__device__ __forceinline__ void mfma_pass_stages(const PassArgs &a, float2 *lds, const float2 *in, float2 *out,
                                                 uint32_t col0, int ncl, std::integer_sequence<int, I...>)
{
    (mfma_pass_stage<NSPLIT, S, I>(a, lds, in, out, col0, ncl), ...);
}

// Complex64 pass whose radix-16 stages run as split-BF16 MFMA products (NSPLIT = 2 or 3).
template <int NSPLIT, int... Rs>
__global__ void __launch_bounds__(1024) k_pass_mfma(const PassArgs a, const float2 *in, float2 *out)
{
    using S = Seq<Rs...>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2 *lds = reinterpret_cast<float2 *>(smem_raw);
    const uint32_t col0 = tile_of_block() * uint32_t(a.c);
    const int ncl = int(min(int64_t(a.c), a.ncols - int64_t(col0)));
    mfma_pass_stages<NSPLIT, S>(a, lds, in, out, col0, ncl, std::make_integer_sequence<int, S::n>{});
}

// ----------------------------------------------------------------------------- element-wise

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
    default: break;
    }
}

template <typename R, int TYPE>
__global__ void __launch_bounds__(256) k_line(const LineArgs l, const void *in, void *out)
{
    const int64_t total = line_total(TYPE, l);
    for (int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total; g += int64_t(gridDim.x) * blockDim.x)
        line_elem<R, TYPE>(l, g, in, out);
}

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
    if (bk.part & kRagWhole) {
        const RagClass &cl = static_cast<const RagClass *>(g.classes)[bk.op];
        const void *bases[B_NBUF_DEV];
        bases[0] = static_cast<const C *>(g.in) + bk.off[0];
        bases[1] = static_cast<C *>(g.out) + bk.off[1];
        for (int b = 2; b < B_NBUF_DEV; ++b) bases[b] = scratch + bk.off[2] + cl.sofs[b];
        for (int o = 0; o < cl.nops; ++o) {
            const RagOp &op = ops[cl.first_op + o];
            const int64_t n = op.type == 0 ? int64_t(op.tiles) : line_total(op.type, op.la);
            ragged_op<R>(op, lds, bases[op.src], const_cast<void *>(bases[op.dst]), 0, n);
        }
    } else {
        const RagOp &op = ops[bk.op];
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
// Kernel table: the specialised kernels in MIFFT_FIXED_SHAPES order.
template <typename R, int PRO, int EPI> const void *pass_kernel(int shape)
{
#define MIFFT_KPTR(...) reinterpret_cast<const void *>(&k_pass_fixed<R, PRO, EPI, __VA_ARGS__>),
    static const void *const table[] = {MIFFT_FIXED_SHAPES(MIFFT_KPTR)};
#undef MIFFT_KPTR
    const int count = int(sizeof(table) / sizeof(table[0]));
    if (shape >= 0 && shape < count) return table[shape];
    return reinterpret_cast<const void *>(&k_pass<R, PRO, EPI>);
}

const void *mfma_kernel(int nsplit, int shape)
{
#define MIFFT_MPTR2(...) reinterpret_cast<const void *>(&k_pass_mfma<2, __VA_ARGS__>),
#define MIFFT_MPTR3(...) reinterpret_cast<const void *>(&k_pass_mfma<3, __VA_ARGS__>),
    static const void *const t2[] = {MIFFT_MFMA_SHAPES(MIFFT_MPTR2)};
    static const void *const t3[] = {MIFFT_MFMA_SHAPES(MIFFT_MPTR3)};
#undef MIFFT_MPTR2
#undef MIFFT_MPTR3
    const int count = int(sizeof(t2) / sizeof(t2[0]));
    if (shape < 0 || shape >= count) return nullptr;
    return nsplit == 2 ? t2[shape] : t3[shape];
}

template <typename R> const void *pass_kernel_for(const PassArgs &a)
{
    if (a.mode >= 2 && a.mshape >= 0) return mfma_kernel(a.mode, a.mshape);
    // fused Bluestein steps: the runtime-radix kernel, which reads the flavour from a
    if (a.pro == PRO_BPAD || a.epi == EPI_BMUL || a.epi == EPI_BEXT)
        return reinterpret_cast<const void *>(&k_pass<R, PRO_PLAIN, EPI_PLAIN>);
    if (a.pro == PRO_C2R) return pass_kernel<R, PRO_C2R, EPI_PLAIN>(a.shape);
    if (a.epi == EPI_R2C) return pass_kernel<R, PRO_PLAIN, EPI_R2C>(a.shape);
    return pass_kernel<R, PRO_PLAIN, EPI_PLAIN>(a.shape);
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
    // one tile per workgroup: measured faster here than persistent workgroups looping over
    // tiles (with or without prefetching the next tile, which also costs registers)
    a.grid = a.ntiles;
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

const void *ragged_kernel(bool f64)
{
    return f64 ? reinterpret_cast<const void *>(&k_ragged<double>) : reinterpret_cast<const void *>(&k_ragged<float>);
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
