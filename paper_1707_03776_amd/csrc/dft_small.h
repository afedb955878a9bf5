// Small forward DFTs held in registers (W_R = exp(-2 pi i / R)), the butterflies of
// the Stockham stages.  Outputs overwrite inputs in natural order: after dft<R>(v),
// v[k] = sum_j v_in[j] W_R^{jk}.  Radix 4, 8 and 16 are built from radix-2/4 steps
// (16 = 4 x 4 with the W_16 twiddles between), 9 = 3 x 3 likewise, 6, 10, 12, 14 and
// 15 by the twiddle-free prime-factor split of two coprime radices; 5 and 7 use the
// symmetric pairing X_k = v0 + sum_j [cos(2 pi jk/R) (v_j + v_{R-j}) - i sin(2 pi jk/R) (v_j - v_{R-j})].
#pragma once

#include <hip/hip_runtime.h>

namespace mifft {

template <typename R> struct Cplx;
template <> struct Cplx<float> { using T = float2; };
template <> struct Cplx<double> { using T = double2; };

template <typename C> __device__ __forceinline__ C c_add(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C c_sub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C c_mul(C a, C b)
{
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C> __device__ __forceinline__ C c_conj(C a) { return C{a.x, -a.y}; }
template <typename C> __device__ __forceinline__ C c_mul_mi(C a) { return C{a.y, -a.x}; } // * (-i)
template <typename C> __device__ __forceinline__ C c_mul_pi(C a) { return C{-a.y, a.x}; } // * (+i)
template <typename C, typename S> __device__ __forceinline__ C c_scale(C a, S s) { return C{a.x * s, a.y * s}; }

// (1 - i)/sqrt(2) * a  and  (-1 - i)/sqrt(2) * a
template <typename C> __device__ __forceinline__ C c_mul_w8_1(C a)
{
    using S = decltype(a.x);
    const S h = S(0.70710678118654752440084436210485);
    return C{(a.x + a.y) * h, (a.y - a.x) * h};
}
template <typename C> __device__ __forceinline__ C c_mul_w8_3(C a)
{
    using S = decltype(a.x);
    const S h = S(0.70710678118654752440084436210485);
    return C{(a.y - a.x) * h, -(a.x + a.y) * h};
}

template <typename C> __device__ __forceinline__ void dft2(C &a, C &b)
{
    C t = a;
    a = c_add(t, b);
    b = c_sub(t, b);
}

template <typename C> __device__ __forceinline__ void dft4(C &a0, C &a1, C &a2, C &a3)
{
    C t0 = c_add(a0, a2), t1 = c_sub(a0, a2);
    C t2 = c_add(a1, a3), t3 = c_mul_mi(c_sub(a1, a3));
    a0 = c_add(t0, t2);
    a2 = c_sub(t0, t2);
    a1 = c_add(t1, t3);
    a3 = c_sub(t1, t3);
}

template <typename C> __device__ __forceinline__ void dft8(C *v)
{
    // even/odd halves, then X_k = E_k + W8^k O_k, X_{k+4} = E_k - W8^k O_k
    dft4(v[0], v[2], v[4], v[6]);
    dft4(v[1], v[3], v[5], v[7]);
    C o1 = c_mul_w8_1(v[3]), o2 = c_mul_mi(v[5]), o3 = c_mul_w8_3(v[7]);
    C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    v[0] = c_add(e0, v[1]);
    v[4] = c_sub(e0, v[1]);
    v[1] = c_add(e1, o1);
    v[5] = c_sub(e1, o1);
    v[2] = c_add(e2, o2);
    v[6] = c_sub(e2, o2);
    v[3] = c_add(e3, o3);
    v[7] = c_sub(e3, o3);
}

template <typename C> __device__ __forceinline__ void dft16(C *v)
{
    using S = decltype(v[0].x);
    const S c1 = S(0.92387953251128675612818318939679); // cos(pi/8)
    const S s1 = S(0.38268343236508977172845998403040); // sin(pi/8)
    // 4-point transforms over m of v[j + 4m]; results stay in place: v[j + 4 k1]
    dft4(v[0], v[4], v[8], v[12]);
    dft4(v[1], v[5], v[9], v[13]);
    dft4(v[2], v[6], v[10], v[14]);
    dft4(v[3], v[7], v[11], v[15]);
    // twiddles W16^{j k1}
    v[5] = c_mul(v[5], C{c1, -s1});   // W^1
    v[9] = c_mul_w8_1(v[9]);          // W^2
    v[13] = c_mul(v[13], C{s1, -c1}); // W^3
    v[6] = c_mul_w8_1(v[6]);          // W^2
    v[10] = c_mul_mi(v[10]);          // W^4
    v[14] = c_mul_w8_3(v[14]);        // W^6
    v[7] = c_mul(v[7], C{s1, -c1});   // W^3
    v[11] = c_mul_w8_3(v[11]);        // W^6
    v[15] = c_mul(v[15], C{-c1, s1}); // W^9
    // 4-point transforms over j for each k1: X[k1 + 4 k2]
    C t[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        C a0 = v[4 * k1 + 0], a1 = v[4 * k1 + 1], a2 = v[4 * k1 + 2], a3 = v[4 * k1 + 3];
        dft4(a0, a1, a2, a3);
        t[k1 + 0] = a0;
        t[k1 + 4] = a1;
        t[k1 + 8] = a2;
        t[k1 + 12] = a3;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = t[k];
}

// cos/sin(2 pi m / R) for the odd radices
template <int R> struct OddConst;
template <> struct OddConst<3> {
    static constexpr double c[2] = {1.0, -0.5};
    static constexpr double s[2] = {0.0, 0.86602540378443864676372317075294};
};
template <> struct OddConst<5> {
    static constexpr double c[3] = {1.0, 0.30901699437494742410229341718282, -0.80901699437494742410229341718282};
    static constexpr double s[3] = {0.0, 0.95105651629515357211643933337938, 0.58778525229247312916870595463907};
};
template <> struct OddConst<7> {
    static constexpr double c[4] = {1.0, 0.62348980185873353052500488400424, -0.22252093395631440428890256449680,
                                    -0.90096886790241912623610231950745};
    static constexpr double s[4] = {0.0, 0.78183148246802980870844452667406, 0.97492791218182360701813168299393,
                                    0.43388373911755812047576833284836};
};

template <int R, typename C> __device__ __forceinline__ void dft_odd(C *v)
{
    using S = decltype(v[0].x);
    constexpr int H = (R - 1) / 2;
    C t[H + 1], d[H + 1];
#pragma unroll
    for (int j = 1; j <= H; ++j) {
        t[j] = c_add(v[j], v[R - j]);
        d[j] = c_sub(v[j], v[R - j]);
    }
    C x0 = v[0];
    C out[R];
    C sum = x0;
#pragma unroll
    for (int j = 1; j <= H; ++j) sum = c_add(sum, t[j]);
    out[0] = sum;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        C a = x0, b = C{S(0), S(0)};
#pragma unroll
        for (int j = 1; j <= H; ++j) {
            const int m = (j * k) % R;
            // cos(2 pi m/R) = cos(2 pi (R-m)/R); sin(2 pi m/R) = -sin(2 pi (R-m)/R)
            const S cs = S(OddConst<R>::c[m <= H ? m : R - m]);
            const S sn = m <= H ? S(OddConst<R>::s[m]) : -S(OddConst<R>::s[R - m]);
            a.x += cs * t[j].x;
            a.y += cs * t[j].y;
            b.x += sn * d[j].x;
            b.y += sn * d[j].y;
        }
        // X_k = a - i b,  X_{R-k} = a + i b
        out[k] = C{a.x + b.y, a.y - b.x};
        out[R - k] = C{a.x - b.y, a.y + b.x};
    }
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = out[k];
}

// 3-point DFT in place: X1,2 = a - (b+c)/2 -/+ i (sqrt(3)/2)(b-c)
template <typename C> __device__ __forceinline__ void dft3(C &a, C &b, C &c)
{
    using S = decltype(a.x);
    const S h = S(0.86602540378443864676372317075294); // sqrt(3)/2
    const C t = c_add(b, c), d = c_sub(b, c);
    const C m = C{a.x - S(0.5) * t.x, a.y - S(0.5) * t.y};
    a = c_add(a, t);
    b = C{m.x + h * d.y, m.y - h * d.x};
    c = C{m.x - h * d.y, m.y + h * d.x};
}

// 9 = 3 x 3: 3-point transforms over v[j1 + 3 j2], twiddles W9^{j1 k1}, 3-point transforms over j1
template <typename C> __device__ __forceinline__ void dft9(C *v)
{
    using S = decltype(v[0].x);
    const S c1 = S(0.76604444311897803520239265055542), s1 = S(0.64278760968653932632264340990726); // 2pi/9
    const S c2 = S(0.17364817766693034885171662676931), s2 = S(0.98480775301220805936674302458952); // 4pi/9
    const S c4 = S(-0.93969262078590838405410927732473), s4 = S(0.34202014332566873304409961468226); // 8pi/9
    dft3(v[0], v[3], v[6]);
    dft3(v[1], v[4], v[7]);
    dft3(v[2], v[5], v[8]);
    // v[j1 + 3 k1] *= W9^{j1 k1}
    v[4] = c_mul(v[4], C{c1, -s1});
    v[7] = c_mul(v[7], C{c2, -s2});
    v[5] = c_mul(v[5], C{c2, -s2});
    v[8] = c_mul(v[8], C{c4, -s4});
    C t[9];
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
        C a = v[3 * k1], b = v[3 * k1 + 1], c = v[3 * k1 + 2];
        dft3(a, b, c);
        t[k1] = a;
        t[k1 + 3] = b;
        t[k1 + 6] = c;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k] = t[k];
}

// Output slot of the prime-factor mapping: the k in [0, P*Q) with k = k1 (mod P) and
// k = k2 (mod Q) (Chinese remainder theorem; P and Q coprime).
constexpr int crt_index(int P, int Q, int k1, int k2)
{
    for (int k = 0; k < P * Q; ++k)
        if (k % P == k1 && k % Q == k2) return k;
    return 0;
}

template <int R, typename C> __device__ __forceinline__ void dft(C *v);

// R = P*Q with P, Q coprime, by the prime-factor (Good-Thomas) algorithm: with
// x indexed j = (Q j1 + P j2) mod R and X indexed by k = CRT(k1, k2), W_R^{jk} factors
// into W_P^{j1 k1} W_Q^{j2 k2}, so Q-point transforms over j2 followed by P-point
// transforms over j1 need no twiddles; both index maps are compile-time permutations.
template <int P, int Q, typename C> __device__ __forceinline__ void dft_pfa(C *v)
{
    constexpr int R = P * Q;
    C y[R];
#pragma unroll
    for (int j1 = 0; j1 < P; ++j1) {
        C t[Q];
#pragma unroll
        for (int j2 = 0; j2 < Q; ++j2) t[j2] = v[(Q * j1 + P * j2) % R];
        dft<Q>(t);
#pragma unroll
        for (int k2 = 0; k2 < Q; ++k2) y[j1 * Q + k2] = t[k2];
    }
#pragma unroll
    for (int k2 = 0; k2 < Q; ++k2) {
        C t[P];
#pragma unroll
        for (int j1 = 0; j1 < P; ++j1) t[j1] = y[j1 * Q + k2];
        dft<P>(t);
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) v[crt_index(P, Q, k1, k2)] = t[k1];
    }
}

template <int R, typename C> __device__ __forceinline__ void dft(C *v)
{
    if constexpr (R == 1) {
    } else if constexpr (R == 2) {
        dft2(v[0], v[1]);
    } else if constexpr (R == 4) {
        dft4(v[0], v[1], v[2], v[3]);
    } else if constexpr (R == 8) {
        dft8(v);
    } else if constexpr (R == 16) {
        dft16(v);
    } else if constexpr (R == 9) {
        dft9(v);
    } else if constexpr (R == 3) {
        dft3(v[0], v[1], v[2]);
    } else if constexpr (R == 6) {
        dft_pfa<2, 3>(v);
    } else if constexpr (R == 10) {
        dft_pfa<2, 5>(v);
    } else if constexpr (R == 12) {
        dft_pfa<4, 3>(v);
    } else if constexpr (R == 14) {
        dft_pfa<2, 7>(v);
    } else if constexpr (R == 15) {
        dft_pfa<3, 5>(v);
    } else {
        dft_odd<R>(v);
    }
}

} // namespace mifft
