// Allocation-failure injection through the C ABI, host only (tests/fake_hip.cpp stands
// in for the HIP runtime), built with AddressSanitizer by tests/test_fail_alloc.py.
// For each plan kind: count the device allocations a creation makes, then for every k
// make the k-th one fail (MIFFT_TEST_FAIL_ALLOC=k) and require NULL, FFT_ERR_ALLOC and
// no device allocation or graph left behind; LeakSanitizer checks host memory.
#include <cstdio>
#include <cstdlib>
#include <string>

#include "mifft.h"

long fake_live();
long fake_made();

namespace {
int failures = 0;

template <typename F> void exercise(const char *name, F create)
{
    unsetenv("MIFFT_TEST_FAIL_ALLOC");
    const long made0 = fake_made();
    fft_plan p = create();
    const long allocs = fake_made() - made0;
    if (!p || allocs < 1) {
        std::printf("%s: creation failed without injection (%s)\n", name, fft_last_error_message());
        ++failures;
        return;
    }
    fft_plan_destroy(p);
    if (fake_live() != 0) {
        std::printf("%s: destroy left %ld objects\n", name, fake_live());
        ++failures;
    }
    for (long k = 1; k <= allocs; ++k) {
        setenv("MIFFT_TEST_FAIL_ALLOC", std::to_string(k).c_str(), 1);
        fft_plan q = create();
        const int st = fft_last_error();
        if (q || st != FFT_ERR_ALLOC || fake_live() != 0) {
            std::printf("%s: k=%ld plan=%p status=%d live=%ld (%s)\n", name, k, static_cast<void *>(q), st,
                        fake_live(), fft_last_error_message());
            ++failures;
            fft_plan_destroy(q);
        }
    }
    unsetenv("MIFFT_TEST_FAIL_ALLOC");
    std::printf("%s: %ld allocations, each failure cleaned up\n", name, allocs);
}
} // namespace

int main()
{
    exercise("c2c 2^20 x2", [] {
        const int64_t n = int64_t(1) << 20;
        return fft_plan_create(1, &n, 2, FFT_C2C, FFT_FORWARD, FFT_F32);
    });
    exercise("c2c bluestein 65521", [] {
        const int64_t n = 65521;
        return fft_plan_create(1, &n, 1, FFT_C2C, FFT_INVERSE, FFT_F64);
    });
    exercise("r2c 64x48x40", [] {
        const int64_t d[3] = {64, 48, 40};
        return fft_plan_create(3, d, 2, FFT_R2C, FFT_FORWARD, FFT_F32);
    });
    exercise("dct2 1000", [] {
        const int64_t n = 1000;
        return fft_plan_create(1, &n, 3, FFT_DCT2, FFT_FORWARD, FFT_F32);
    });
    exercise("ragged", [] {
        const int64_t len[5] = {64, 97, 4096, 65536, 30011};
        int64_t off[5], pos = 0;
        for (int t = 0; t < 5; ++t) {
            off[t] = pos;
            pos += len[t];
        }
        return fft_plan_create_many(5, len, off, off, FFT_C2C, FFT_FORWARD, FFT_F32);
    });
    std::printf("failures=%d\n", failures);
    return failures != 0;
}
