// Launch-argument structures shared by the host planner and the gfx950 kernels.
// Plain data only: no HIP types, so the planner compiles and is tested without a GPU.
#pragma once

#include <stdint.h>

namespace mifft {

constexpr int kMaxStages = 10;    // inner (in-workgroup) Stockham stages per pass
constexpr int kColDims = 4;       // column index decomposes into up to 4 strided dims
constexpr int kMaxThreads = 1024; // workgroup size limit
constexpr int kLdsBudget = 80 * 1024; // LDS per workgroup the planner aims for (2 groups per CU)

// LDS column layout: one spare slot every 2^kLdsPadShift{F32,F64} points of a column.
constexpr int kLdsPadShiftF32 = 5;
constexpr int kLdsPadShiftF64 = 4;

// Elements each thread may hold per stage (registers): 32 complex64 / 16 complex128
// (64 VGPRs of data either way).
template <typename R> struct RegBudget;
template <> struct RegBudget<float> { static constexpr int kElems = 32; };
template <> struct RegBudget<double> { static constexpr int kElems = 16; };

// Elements per thread per stage of the generic stages inside the ragged batch kernel
// (fewer registers -> more resident workgroups).
template <typename R> struct RaggedElems;
template <> struct RaggedElems<float> { static constexpr int v = 16; };
template <> struct RaggedElems<double> { static constexpr int v = 8; };

// Prologue / epilogue kinds of a pass.
enum Prologue : int32_t {
    PRO_PLAIN = 0, // complex loads from global memory (optional conj, optional pass twiddle)
    PRO_C2R = 1,   // half spectrum -> z = x[2m] + i x[2m+1] spectrum (Hermitian untwist) in LDS
    PRO_BPAD = 2,  // Bluestein: point j of a length-M line is x_j w_j (j < n) or 0, read from
                   // the length-n lines of the input (x conjugated first when conj_in)
    PRO_SYM = 3,   // complex loads as PRO_PLAIN, each point then scaled by a real separable
                   // symbol s = S_p[p] + S_0[d0] (+ S_1[d1]), FP64 tables in aux (specialised
                   // kernels only; sym_cd = column dims the symbol covers)
    PRO_DCT2 = 4,  // point m of a line is z_m = v_2m + i v_2m+1, v the Makhoul reordering of the
                   // nreal input reals of that line (v_j = x_2j below nreal/2, else
                   // x_{2(nreal-1-j)+1}); columns: d0 within the line, d1 the line (specialised
                   // kernels only)
    PRO_CUNTWIST = 5 // first pass of a staged real inverse (h = nreal/2 points, J = csz[0]
                     // columns per line, point p of column j is P_{j + J p}): mirrored tiles
                     // as EPI_RTWIST; the c2r untwist of the bins Y_m, Y_{h-m} (line of h+1
                     // bins, cin[1] apart; W_n^m, m <= h, in aux) goes straight into LDS
};
enum Epilogue : int32_t {
    EPI_PLAIN = 0, // complex stores to global memory (optional conj, scale)
    EPI_R2C = 1,   // z spectrum in LDS -> half spectrum of the real row (twist)
    EPI_BMUL = 2,  // Bluestein: store conj(Y_k B_k) (B = the filter spectrum, aux2)
    EPI_BEXT = 3,  // Bluestein: for k < n store scale * w_k * conj(Y_k) (optional conj) into the
                   // length-n lines of the output; points k >= n are dropped
    EPI_DCT3 = 4,  // point m of a line is z_m = v_2m + i v_2m+1 (after conj and scale); v_j goes
                   // to the nreal output reals of the line undoing the Makhoul reordering
                   // (y_2j = v_j below nreal/2, else y_{2(nreal-1-j)+1} = v_j); columns: d0
                   // within the line, d1 the line (specialised kernels only)
    EPI_RTWIST = 5, // last pass of a staged real transform (h = nreal/2 points, J = csz[0]
                    // columns per line, point p of column j is Z_{j + J p}): tiles hold c/2
                    // columns and their mirrors J - j (0 and J/2 are their own), so the twist
                    // X_m from Z_m and Z_{h-m} runs from LDS; X_0..X_h go to the line's output
                    // (bm complex apart; W_n^m, m <= h, in aux)
    EPI_DTWIST = 6  // as EPI_RTWIST, then the DCT-II rotation: y_m = 2 Re(W_4n^m X_m) and
                    // y_{n-m} = 2 Re(W_4n^{n-m} conj X_m) into the line's nreal output reals
                    // (bm reals apart; W_4n^k, k < n, in aux2); float32 kernels only
};

// One inner Stockham stage: radix r, Ns = product of the radices before it,
// tw = offset (complex elements) of its twiddles W_{Ns*r}^{k*m} (m < Ns,
// k = 1..r-1, stored at tw + m*(r-1) + k-1) in the pass's inner table.
struct StageInfo {
    int32_t r, ns, tw, pad_;
};

// One pass: `ncols` independent length-L sub-transforms ("columns").  Column
// index f (0 <= f < ncols) decomposes as f = d0 + csz[0]*(d1 + csz[1]*(d2 + csz[2]*d3));
// its input starts at sum(d_i*cin[i]) and its point p at + p*rin (elements);
// likewise for output with cout/rout.  A workgroup takes `c` consecutive columns.
struct PassArgs {
    int32_t L, nst;
    int32_t shape, mshape;             // specialised kernel (MIFFT_FIXED_SHAPES / MIFFT_MFMA_SHAPES) or -1
    int32_t mode;                      // 0: FP32/FP64 vector units; 2/3: radix-16 stages as split-BF16 MFMA
    int32_t sym_cd;                    // PRO_SYM: column dims (1 or 2) with a symbol table after S_p
    int32_t nt_in, nt_out;             // global loads / stores of this pass are nontemporal (streamed
                                       // data read or written once per call: input of the first pass,
                                       // output of the last), keeping the caches for intermediates
    StageInfo st[kMaxStages];
    int32_t c, threads, lp, lds_bytes; // columns per tile, group size, LDS column pitch, LDS bytes
    int32_t load_cf, store_cf;         // 1: first/last stage maps consecutive lanes to consecutive columns
    int32_t pro, epi;
    int32_t conj_in, conj_out;
    int32_t tw_dim, tw_bits;           // pass twiddle W_{twN}^{p*d[tw_dim]} on the input; -1 = none
    int64_t twN;
    int64_t ncols, ntiles;
    int64_t grid;                      // workgroups launched (specialised kernels loop over tiles)
    int64_t csz[kColDims], cin[kColDims], cout[kColDims];
    double crcp[kColDims];             // 1/csz[d], for division by multiplication
    int32_t ncd, logc;                 // column dims in use; log2(c)
    int64_t rin, rout;
    double scale;                      // multiplies every stored value (1.0 = none)
    int64_t nreal;                     // real row length for PRO_C2R / EPI_R2C; Bluestein length n
    int64_t bm;                        // Bluestein: padded length M (lines of the padded layout are M apart)
    double brcp;                       // 1/M, for the division of padded offsets by M
    const void *itw;                   // inner twiddle table
    const void *tw_lo, *tw_hi;         // two-level pass twiddles, FP64: W^e = hi[e >> bits] * lo[e & mask]
    const void *aux;                   // W_n^k, k = 0..n/2 for the real twist kinds; chirp w_j for Bluestein
    const void *aux2;                  // Bluestein filter spectrum B (EPI_BMUL)
};

// Elementwise kernels (Bluestein, real-data staging).  Lines are addressed like
// pass columns; element e of line f sits at base(f) + e*es.
struct LineArgs {
    int64_t nlines;
    int64_t csz[kColDims], cin[kColDims], cout[kColDims];
    int64_t es_in, es_out;
    int64_t n, M;        // logical length, padded length
    int32_t conj_in, conj_out;
    double scale;
    const void *tab;     // chirp w_j (Bluestein) or twist table
    const void *tab2;    // Bluestein filter spectrum
};

} // namespace mifft
