// Split-BF16 matrix-core radix-16 pass kernels (complex64).
#include <hip/hip_runtime.h>

#include "pass_device.h"

namespace mifft {

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

// ----------------------------------------------------------------------------- split-BF16 MFMA radix-64

// A radix-64 butterfly Y = F64 X is the product with the real 128x128 matrix acting on
// the interleaved vector, computed as 8 x 4 blocks of v_mfma_f32_16x16x32_bf16: output
// block rb (reals 16 rb .. 16 rb + 15, complex outputs 8 rb .. 8 rb + 7) accumulates four
// input blocks kb (reals 32 kb .. 32 kb + 31, complex inputs 16 kb .. 16 kb + 15).  With 16
// butterflies as the 16 columns, lane (n, g) = (l%16, l/16) supplies complex inputs
// 16 kb + 4 g + t (t < 4) of butterfly n for every kb, and receives complex outputs
// 8 rb + 2 g and 8 rb + 2 g + 1 for every rb: sixteen points in, sixteen out.  The split
// DFT matrix (NSPLIT x 32 operand vectors of 16 bytes per lane, kMfma64PartBytes = 32 KiB
// per split part)
// is too large for registers; each workgroup builds it once in LDS, behind its tile.

// cos(2 pi m / 64), m = 0..63, from the exact first-octant-and-a-bit values
__device__ __forceinline__ float cos64(int m)
{
    const float c[17] = {1.0f, 0.9951847266721968862448f, 0.9807852804032304491262f, 0.9569403357322088649358f,
                         0.9238795325112867561282f, 0.8819212643483550297128f, 0.8314696123025452370788f,
                         0.7730104533627369608109f, 0.7071067811865475244008f, 0.6343932841636454982152f,
                         0.5555702330196022247428f, 0.4713967368259976485564f, 0.3826834323650897717285f,
                         0.2902846772544623676362f, 0.1950903220161282678483f, 0.0980171403295606019942f, 0.0f};
    m &= 63;
    if (m <= 16) return c[m];
    if (m <= 32) return -c[32 - m];
    if (m <= 48) return -c[m - 32];
    return c[64 - m];
}
__device__ __forceinline__ float sin64(int m) { return cos64(m - 16); }


// LDS table of the split radix-64 DFT operands: entry ((p * 8 + rb) * 4 + kb) * 64 + lane
// holds part p of the A operand lane `lane` feeds to block (rb, kb).
template <int NSPLIT> __device__ __forceinline__ void build_dft64_table(uint4 *tbl)
{
    const int T = blockDim.x;
    for (int e = threadIdx.x; e < NSPLIT * 2048; e += T) {
        const int p = e >> 11, rem = e & 2047;
        const int rb = rem >> 8, kb = (rem >> 6) & 3, ln = rem & 63;
        const int r = ln & 15, g = ln >> 4;
        const int k = 8 * rb + (r >> 1), comp = r & 1;
        bf16x8 v;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int j = 16 * kb + 4 * g + (i >> 1), ic = i & 1;
            const int m = (j * k) & 63;
            const float c = cos64(m), sn = sin64(m);
            const float x = comp == 0 ? (ic == 0 ? c : sn) : (ic == 0 ? -sn : c);
            __bf16 parts[NSPLIT];
            split_bf16<NSPLIT>(x, parts);
            v[i] = parts[p];
        }
        tbl[e] = __builtin_bit_cast(uint4, v);
    }
}

// One radix-64 stage on the matrix cores; same data movement contract as the other
// stages (butterfly b of a column reads points b + j*NB, twiddled by W_{64 NS}^{j (b mod NS)}
// or by the multi-pass twiddle in a first stage, and writes points (b/NS)*64*NS + b%NS +
// k*NS).  Each wave takes one group of 16 butterflies (the planner sizes the group so).
template <int NSPLIT, int L, int NS, int TWOFF, bool SRC_G, bool DST_G>
__device__ __forceinline__ void mfma64_stage(const PassArgs &a, int cf, float2 *lds, const uint4 *tbl,
                                             const float2 *in, float2 *out, uint32_t col0, int ncl)
{
    constexpr int NB = L / 64;
    constexpr bool LIN = IsPow2<L>::v;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int n = lane & 15, g = lane >> 4;
    const int lp = a.lp, cmask = a.c - 1;
    const int nbt = a.c * NB;
    const int bt = wave * 16 + n;
    int col, b;
    if (cf) {
        col = bt & cmask;
        b = bt >> a.logc;
    } else {
        col = bt / NB;
        b = bt - col * NB;
    }
    const bool active = wave * 16 < nbt;       // uniform per wave
    const bool ok = bt < nbt && col < ncl;
    float2 x[4][4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int t = 0; t < 4; ++t) x[kb][t] = float2{0.f, 0.f};
    if (ok) {
        if constexpr (SRC_G) {
            const ColBase cb = col_base_fast(a, col0 + uint32_t(col));
            const uint32_t rin = uint32_t(a.rin);
            const float2 *src = in + (cb.in + uint32_t(b) * rin);
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
#pragma unroll
                for (int t = 0; t < 4; ++t) x[kb][t] = gload(src + uint32_t((16 * kb + 4 * g + t) * NB) * rin, a.nt_in);
            if (a.conj_in) {
#pragma unroll
                for (int kb = 0; kb < 4; ++kb)
#pragma unroll
                    for (int t = 0; t < 4; ++t) x[kb][t].y = -x[kb][t].y;
            }
            if (a.tw_dim >= 0) {
                const double2 u = pass_root(a, uint32_t(NB) * cb.twi);
#pragma unroll
                for (int kb = 0; kb < 4; ++kb) {
                    double2 w = pass_root(a, uint32_t(b + (16 * kb + 4 * g) * NB) * cb.twi);
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        if (t > 0) w = c_mul(w, u);
                        x[kb][t] = c_mul(x[kb][t], to_c<float2>(w));
                    }
                }
            }
        } else {
            const int base = col * lp;
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int j = 16 * kb + 4 * g + t;
                    x[kb][t] = LIN ? lds[base + lds_pad<float>(b) + lds_pad<float>(j * NB)]
                                   : lds[base + lds_pad<float>(b + j * NB)];
                }
        }
        if constexpr (NS > 1) {
            const float2 *row = static_cast<const float2 *>(a.itw) + TWOFF + (b % NS) * 63;
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int j = 16 * kb + 4 * g + t;
                    if (j > 0) x[kb][t] = c_mul(x[kb][t], row[j - 1]);
                }
        }
    }
    if constexpr (SRC_G == DST_G) __syncthreads();

    f32x4 d[8];
    if (active) {
        bf16x8 bsp[4][NSPLIT];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                __bf16 pr[NSPLIT], pi[NSPLIT];
                split_bf16<NSPLIT>(x[kb][t].x, pr);
                split_bf16<NSPLIT>(x[kb][t].y, pi);
#pragma unroll
                for (int u = 0; u < NSPLIT; ++u) {
                    bsp[kb][u][2 * t] = pr[u];
                    bsp[kb][u][2 * t + 1] = pi[u];
                }
            }
        // eight independent accumulators (one per output block), input blocks outermost,
        // so consecutive products never wait on each other in the matrix pipeline
#pragma unroll
        for (int rb = 0; rb < 8; ++rb) d[rb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
#pragma unroll
            for (int rb = 0; rb < 8; ++rb) {
                bf16x8 av[NSPLIT];
#pragma unroll
                for (int p = 0; p < NSPLIT; ++p)
                    av[p] = __builtin_bit_cast(bf16x8, tbl[((p * 8 + rb) * 4 + kb) * 64 + lane]);
                f32x4 acc = d[rb];
                if constexpr (NSPLIT == 2) {
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1], bsp[kb][0], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], bsp[kb][1], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], bsp[kb][0], acc, 0, 0, 0);
                } else {
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1], bsp[kb][1], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[2], bsp[kb][0], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], bsp[kb][2], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[1], bsp[kb][0], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], bsp[kb][1], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[0], bsp[kb][0], acc, 0, 0, 0);
                }
                d[rb] = acc;
            }
        }
    }
    if (ok) {
        const int q0 = (b / NS) * NS * 64 + (b % NS);
        if constexpr (DST_G) {
            const ColBase cb = col_base_fast(a, col0 + uint32_t(col));
            const uint32_t rout = uint32_t(a.rout);
            float2 *dst = out + (cb.out + uint32_t(q0) * rout);
            const float sc = float(a.scale);
#pragma unroll
            for (int rb = 0; rb < 8; ++rb)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    float2 y{d[rb][2 * h], d[rb][2 * h + 1]};
                    if (a.conj_out) y.y = -y.y;
                    if (a.scale != 1.0) y = c_scale(y, sc);
                    gstore(dst + uint32_t((8 * rb + 2 * g + h) * NS) * rout, y, a.nt_out);
                }
        } else {
            const int base = col * lp;
#pragma unroll
            for (int rb = 0; rb < 8; ++rb)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    lds[base + lds_pad<float>(q0 + (8 * rb + 2 * g + h) * NS)] =
                        float2{d[rb][2 * h], d[rb][2 * h + 1]};
        }
    }
    if constexpr (!DST_G) __syncthreads();
}

template <int NSPLIT, typename S, int s>
__device__ __forceinline__ void mfma64_pass_stage(const PassArgs &a, float2 *lds, const uint4 *tbl, const float2 *in,
                                                  float2 *out, uint32_t col0, int ncl)
{
    constexpr int RADIX = S::r[s];
    constexpr bool first = s == 0, last = s == S::n - 1;
    const int cf = first ? a.load_cf : (last ? a.store_cf : 0);
    if constexpr (RADIX == 64)
        mfma64_stage<NSPLIT, S::L, S::ns(s), S::tw(s), first, last>(a, cf, lds, tbl, in, out, col0, ncl);
    else
        mfma_pass_stage<NSPLIT, S, s>(a, lds, in, out, col0, ncl);
}

template <int NSPLIT, typename S, int... I>
__device__ __forceinline__ void mfma64_pass_stages(const PassArgs &a, float2 *lds, const uint4 *tbl,
                                                   const float2 *in, float2 *out, uint32_t col0, int ncl,
                                                   std::integer_sequence<int, I...>)
{
    (mfma64_pass_stage<NSPLIT, S, I>(a, lds, tbl, in, out, col0, ncl), ...);
}

// Complex64 pass with a radix-64 matrix-core stage: persistent workgroups (at most 256
// threads, so a wave may hold the 16 points, their split operands and eight
// accumulators) build the split DFT matrix in LDS once and then walk their tiles; the
// tiles are split into 8 contiguous ranges, one per XCD, taken in turn by the
// workgroups on that XCD.
template <int NSPLIT, int... Rs>
__global__ void __launch_bounds__(256) k_pass_mfma64(const PassArgs a, const float2 *in, float2 *out)
{
    using S = Seq<Rs...>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float2 *lds = reinterpret_cast<float2 *>(smem_raw);
    uint4 *tbl = reinterpret_cast<uint4 *>(smem_raw + (a.lds_bytes - NSPLIT * kMfma64PartBytes));
    build_dft64_table<NSPLIT>(tbl);
    __syncthreads();
    const uint32_t nb = gridDim.x, blk = blockIdx.x, x = blk & 7u, sb = blk >> 3;
    const uint32_t nbx = (nb >> 3) + (x < (nb & 7u) ? 1u : 0u);
    const uint32_t ntiles = uint32_t(a.ntiles), q = ntiles >> 3, rem = ntiles & 7u;
    const uint32_t start = x * q + min(x, rem), end = start + q + (x < rem ? 1u : 0u);
    for (uint32_t t = start + sb; t < end; t += nbx) {
        const uint32_t col0 = t * uint32_t(a.c);
        const int ncl = int(min(int64_t(a.c), a.ncols - int64_t(col0)));
        mfma64_pass_stages<NSPLIT, S>(a, lds, tbl, in, out, col0, ncl, std::make_integer_sequence<int, S::n>{});
        __syncthreads(); // the next tile's first stage rewrites the exchange
    }
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

// The kernel of a radix sequence: the radix-64 form when a stage has radix 64.
template <int NSPLIT, int... Rs> const void *mfma_kernel_of()
{
    if constexpr (((Rs == 64) || ...))
        return reinterpret_cast<const void *>(&k_pass_mfma64<NSPLIT, Rs...>);
    else
        return reinterpret_cast<const void *>(&k_pass_mfma<NSPLIT, Rs...>);
}

const void *mfma_kernel(int nsplit, int shape)
{
#define MIFFT_MPTR2(...) mfma_kernel_of<2, __VA_ARGS__>(),
#define MIFFT_MPTR3(...) mfma_kernel_of<3, __VA_ARGS__>(),
    static const void *const t2[] = {MIFFT_MFMA_SHAPES(MIFFT_MPTR2)};
    static const void *const t3[] = {MIFFT_MFMA_SHAPES(MIFFT_MPTR3)};
#undef MIFFT_MPTR2
#undef MIFFT_MPTR3
    const int count = int(sizeof(t2) / sizeof(t2[0]));
    if (shape < 0 || shape >= count) return nullptr;
    return nsplit == 2 ? t2[shape] : t3[shape];
}

} // namespace mifft
