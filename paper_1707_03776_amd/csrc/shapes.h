// Radix sequences that have compile-time-specialised pass kernels (kernels.hip).
// A pass whose inner decomposition matches one of these runs a kernel in which L,
// every stage's radix, Ns and butterfly count are constants; any other sequence
// runs the runtime-generic kernel.  Plain data: the host planner reads it too.
#pragma once

// Powers of two up to 8192 in the planner's decomposition, the odd pass shapes of
// the 1-D size sweep (3*2^18 = 768*1024, 5*2^16 = 640*512, 7*3^9 = 567*243 with
// 567 = 9*9*7 and 243 = 9*9*3), and a few neighbours of those.
#define MIFFT_FIXED_SHAPES(X)                                                                                   \
    X(1)                                                                                                        \
    X(2)                                                                                                        \
    X(4)                                                                                                        \
    X(8)                                                                                                        \
    X(16)                                                                                                       \
    X(8, 4)                                                                                                     \
    X(8, 8)                                                                                                     \
    X(16, 8)                                                                                                    \
    X(16, 16)                                                                                                   \
    X(8, 8, 8)                                                                                                  \
    X(16, 8, 8)                                                                                                 \
    X(16, 16, 8)                                                                                                \
    X(16, 16, 16)                                                                                               \
    X(16, 8, 8, 8)                                                                                              \
    X(16, 16, 3)                                                                                                \
    X(16, 8, 3)                                                                                                 \
    X(8, 8, 3)                                                                                                  \
    X(16, 8, 5)                                                                                                 \
    X(8, 8, 5)                                                                                                  \
    X(8, 8, 7)                                                                                                  \
    X(9, 9, 7)                                                                                                  \
    X(9, 9, 3)                                                                                                  \
    X(9, 9, 9)                                                                                                  \
    X(16, 16, 9)                                                                                                \
    X(16, 9)                                                                                                    \
    X(8, 8, 9)

// Radix sequences with split-BF16 MFMA kernels (complex64; every radix-16 and
// radix-64 stage on the matrix cores, other radices on the FP32 vector units).
#define MIFFT_MFMA_SHAPES(X)                                                                                    \
    X(16)                                                                                                       \
    X(16, 4)                                                                                                    \
    X(16, 8)                                                                                                    \
    X(16, 16)                                                                                                   \
    X(16, 16, 4)                                                                                                \
    X(16, 16, 8)                                                                                                \
    X(16, 16, 16)                                                                                               \
    X(64)                                                                                                       \
    X(64, 4)                                                                                                    \
    X(64, 8)                                                                                                    \
    X(64, 16)                                                                                                   \
    X(16, 64)                                                                                                   \
    X(64, 64)

namespace mifft {

// Index of the sequence in MIFFT_MFMA_SHAPES, or -1.
int mfma_shape_id(const int *radices, int nst);

// Radix-64 matrix-core passes: persistent groups of at most 256 threads, with the split
// DFT matrix (32 KiB per split part) in LDS behind the tile.
constexpr int kMfma64MaxThreads = 256;
constexpr int kMfma64PartBytes = 32 * 1024;

// Elements one thread holds per stage in the specialised kernels (registers):
// an item of radix r is r elements, so a stage gives each thread kFixedElems / r items.
constexpr int kFixedElems = 16;
template <typename R> struct FixedMaxThreads;
template <> struct FixedMaxThreads<float> { static constexpr int v = 1024; };
template <> struct FixedMaxThreads<double> { static constexpr int v = 512; };

// Index of the sequence in MIFFT_FIXED_SHAPES, or -1.
int fixed_shape_id(const int *radices, int nst);

} // namespace mifft
