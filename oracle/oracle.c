/*
 * FP64 CPU oracle for the discrete Fourier transform.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the GPU
 * library is checked against.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the library itself never calls it,
 * shares no source with it and has no fallback to it.
 *
 * What it computes (the definition; the paper has no Fourier transform,
 * so the conventions are numpy.fft's):
 *
 *   X[k] = s * sum_{j=0}^{n-1} x[j] * exp(sigma * 2*pi*i * j*k / n),  k = 0..n-1
 *
 * with sigma = -1, s = 1 for the forward transform and sigma = +1, s = 1/n for the
 * inverse.  A d-dimensional transform applies the 1-D transform along every axis
 * with the same sigma, and the inverse scale is 1/prod(dims).
 *
 * How: the recursive decimation-in-time factorisation of Cooley and Tukey (1965),
 * taking the smallest prime factor p of n at each level, splitting x into the p
 * subsequences x[r + p*t], transforming each, and recombining with a plain p-point
 * sum against exact roots of unity.  A prime length is a direct O(p^2) sum.  No
 * radix tricks, no reordering beyond that factorisation, no recurrences for the
 * roots of unity.
 *
 * Parity pins (tests/test_oracle_*.py): brute-force O(n^2) sums in FP64 and in
 * 50-digit mpmath, closed forms (delta, constant, pure tones), Parseval,
 * linearity, the shift and convolution theorems, adjointness, inverse round
 * trip, Hermitian symmetry of real input, and hand-worked fixtures.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double re, im;
} cplx;

/* Status codes returned to the ctypes wrapper. */
enum { ORACLE_OK = 0, ORACLE_BAD_ARG = 1, ORACLE_NO_MEM = 2 };

/*
 * exp(sigma * 2*pi*i * m / n), computed on the argument reduced to the first
 * octant.  m is reduced modulo n in exact integer arithmetic first, and 8m is
 * split into an octant number o and a remainder r (0 <= r < n), so that the
 * angle is (pi/4)*(o + r/n).  Each octant is mapped back to [0, pi/4] through the
 * usual sine/cosine symmetries.  Multiples of n/4 (and n/8) therefore come out
 * exactly as 1, i, -1, -i (and exactly symmetric at pi/4).
 */
static cplx unit_root(int64_t n, int64_t m, int sigma)
{
    m %= n;
    if (m < 0) m += n;
    /* 8*m fits comfortably in int64 for every n this oracle is asked for (< 2^59). */
    int64_t o = (8 * m) / n;
    int64_t r = 8 * m - o * n;
    double phi = (M_PI / 4.0) * ((double)r / (double)n);       /* distance from octant start */
    double psi = (M_PI / 4.0) * ((double)(n - r) / (double)n); /* distance to octant end */
    double c = 0.0, s = 0.0;
    if (r == 0 && (o & 1)) {
        /* odd multiple of pi/4: both parts are sqrt(1/2), correctly rounded */
        c = (o == 1 || o == 7) ? M_SQRT1_2 : -M_SQRT1_2;
        s = (o == 1 || o == 3) ? M_SQRT1_2 : -M_SQRT1_2;
        cplx w = {c, sigma > 0 ? s : -s};
        return w;
    }
    switch (o) {
    case 0: c = cos(phi);  s = sin(phi);  break;
    case 1: c = sin(psi);  s = cos(psi);  break;
    case 2: c = -sin(phi); s = cos(phi);  break;
    case 3: c = -cos(psi); s = sin(psi);  break;
    case 4: c = -cos(phi); s = -sin(phi); break;
    case 5: c = -sin(psi); s = -cos(psi); break;
    case 6: c = sin(phi);  s = -cos(phi); break;
    default: c = cos(psi); s = -sin(psi); break;
    }
    cplx w = {c, sigma > 0 ? s : -s};
    return w;
}

static int64_t smallest_prime_factor(int64_t n)
{
    if (n % 2 == 0) return 2;
    for (int64_t p = 3; p * p <= n; p += 2)
        if (n % p == 0) return p;
    return n;
}

/* Table of the N-th roots of unity w[e] = exp(sigma*2*pi*i*e/N), e = 0..N-1.  A
 * sub-transform of length n | N uses w[(e mod n) * (N/n)]. */
typedef struct {
    int64_t N;
    cplx *w;
} roots_t;

static int roots_make(roots_t *R, int64_t N, int sigma)
{
    R->N = N;
    R->w = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    if (!R->w) return ORACLE_NO_MEM;
    for (int64_t e = 0; e < N; ++e) R->w[e] = unit_root(N, e, sigma);
    return ORACLE_OK;
}

static void roots_free(roots_t *R)
{
    free(R->w);
    R->w = NULL;
}

static inline cplx cmul(cplx a, cplx b)
{
    cplx z = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return z;
}

/*
 * Length-n DFT of x[0], x[s], ..., x[(n-1)s] into out[0..n-1] (contiguous).
 * ws is scratch for at least 2n elements.  Recursive Cooley-Tukey:
 *   n = p*m,  Y_r[k] = DFT_m( x[r + p*t] )[k]            (r < p, k < m)
 *   X[k + q*m] = sum_{r<p} w_n^{r*(k+q*m)} * Y_r[k]       (q < p)
 */
static void ct(const cplx *x, int64_t n, int64_t s, cplx *out, cplx *ws, const roots_t *R)
{
    if (n == 1) {
        out[0] = x[0];
        return;
    }
    const int64_t step = R->N / n; /* w_n^e = w_N^{e*step} */
    const int64_t p = smallest_prime_factor(n);
    if (p == n) {
        /* prime length: the definition, with the exponent reduced exactly mod n */
        for (int64_t k = 0; k < n; ++k) {
            double ar = 0.0, ai = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                cplx t = cmul(R->w[((j * k) % n) * step], x[j * s]);
                ar += t.re;
                ai += t.im;
            }
            out[k].re = ar;
            out[k].im = ai;
        }
        return;
    }
    const int64_t m = n / p;
    cplx *Y = ws; /* p blocks of m values; children use the scratch above */
    for (int64_t r = 0; r < p; ++r) ct(x + r * s, m, s * p, Y + r * m, ws + n, R);
    for (int64_t q = 0; q < p; ++q) {
        for (int64_t k = 0; k < m; ++k) {
            const int64_t idx = k + q * m;
            double ar = 0.0, ai = 0.0;
            for (int64_t r = 0; r < p; ++r) {
                cplx t = cmul(R->w[((r * idx) % n) * step], Y[r * m + k]);
                ar += t.re;
                ai += t.im;
            }
            out[idx].re = ar;
            out[idx].im = ai;
        }
    }
}

static int bad_geometry(int rank, const int64_t *dims, int64_t batch)
{
    if (rank < 1 || rank > 3 || !dims || batch < 0) return 1;
    for (int a = 0; a < rank; ++a)
        if (dims[a] < 1) return 1;
    return 0;
}

/*
 * In-place 1-D transforms along axis `a` of every [dims] block of `data`
 * (batch blocks, row-major, last axis contiguous).  One roots table per call;
 * OpenMP over the independent lines only.
 */
static int along_axis(cplx *data, int rank, const int64_t *dims, int64_t batch, int a, int sigma)
{
    const int64_t n = dims[a];
    int64_t inner = 1, outer = batch;
    for (int b = a + 1; b < rank; ++b) inner *= dims[b];
    for (int b = 0; b < a; ++b) outer *= dims[b];
    const int64_t lines = outer * inner;
    if (n == 1 || lines == 0) return ORACLE_OK;
    roots_t R;
    if (roots_make(&R, n, sigma) != ORACLE_OK) return ORACLE_NO_MEM;
    int status = ORACLE_OK;
#pragma omp parallel
    {
        cplx *line = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        cplx *res = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        cplx *ws = (cplx *)malloc(sizeof(cplx) * (size_t)(2 * n));
        const int ok = line && res && ws;
        if (!ok) {
#pragma omp atomic write
            status = ORACLE_NO_MEM;
        }
        /* every thread reaches the work-sharing loop; one without buffers idles */
#pragma omp for schedule(dynamic, 1)
        for (int64_t l = 0; l < lines; ++l) {
            if (!ok) continue;
            const int64_t o = l / inner, i = l % inner;
            cplx *base = data + o * n * inner + i;
            for (int64_t j = 0; j < n; ++j) line[j] = base[j * inner];
            ct(line, n, 1, res, ws, &R);
            for (int64_t k = 0; k < n; ++k) base[k * inner] = res[k];
        }
        free(line);
        free(res);
        free(ws);
    }
    roots_free(&R);
    return status;
}

/*
 * Complex-to-complex transform of `batch` row-major blocks of shape dims[0..rank).
 * in/out hold interleaved (re, im) doubles; they may be the same buffer.
 * sigma = -1: forward, unscaled.  sigma = +1: inverse, scaled by 1/prod(dims).
 */
int oracle_c2c(int rank, const int64_t *dims, int64_t batch, int sigma, const double *in, double *out)
{
    if (bad_geometry(rank, dims, batch) || (sigma != -1 && sigma != 1) || !in || !out)
        return ORACLE_BAD_ARG;
    int64_t per = 1;
    for (int a = 0; a < rank; ++a) per *= dims[a];
    const int64_t total = per * batch;
    if (out != in) memmove(out, in, sizeof(cplx) * (size_t)total);
    cplx *d = (cplx *)out;
    for (int a = rank - 1; a >= 0; --a) {
        int st = along_axis(d, rank, dims, batch, a, sigma);
        if (st != ORACLE_OK) return st;
    }
    if (sigma > 0) {
        const double sc = 1.0 / (double)per;
#pragma omp parallel for
        for (int64_t e = 0; e < total; ++e) {
            d[e].re *= sc;
            d[e].im *= sc;
        }
    }
    return ORACLE_OK;
}

/*
 * Real-to-complex forward transform (numpy rfftn layout): the forward c2c of the
 * real input (zero imaginary part), keeping k = 0..dims[rank-1]/2 along the last
 * axis.  in: batch*prod(dims) doubles.  out: batch*prod(dims[:-1])*(dims[-1]/2+1)
 * interleaved complex.
 */
int oracle_r2c(int rank, const int64_t *dims, int64_t batch, const double *in, double *out)
{
    if (bad_geometry(rank, dims, batch) || !in || !out) return ORACLE_BAD_ARG;
    int64_t per = 1;
    for (int a = 0; a < rank; ++a) per *= dims[a];
    const int64_t n = dims[rank - 1], h = n / 2 + 1;
    const int64_t rows = batch * (per / n);
    cplx *full = (cplx *)malloc(sizeof(cplx) * (size_t)(per * batch > 0 ? per * batch : 1));
    if (!full) return ORACLE_NO_MEM;
#pragma omp parallel for
    for (int64_t e = 0; e < per * batch; ++e) {
        full[e].re = in[e];
        full[e].im = 0.0;
    }
    int st = oracle_c2c(rank, dims, batch, -1, (const double *)full, (double *)full);
    if (st == ORACLE_OK) {
        cplx *o = (cplx *)out;
#pragma omp parallel for
        for (int64_t r = 0; r < rows; ++r)
            for (int64_t k = 0; k < h; ++k) o[r * h + k] = full[r * n + k];
    }
    free(full);
    return st;
}

/*
 * Complex-to-real inverse transform with numpy irfftn semantics: a scaled inverse
 * c2c along every axis but the last, then along the last axis the 1-D c2r
 *   x[j] = (1/n) * ( Re X[0] + (-1)^j Re X[n/2] [n even]
 *                    + 2 * sum_{k=1}^{ceil(n/2)-1} Re(X[k] exp(2 pi i j k / n)) ).
 * That sum equals the inverse DFT of the Hermitian extension Y[k] = X[k] (k <= n/2),
 * Y[n-k] = conj X[k], with the imaginary parts of X[0] and X[n/2] (n even) dropped,
 * which is how it is evaluated here.  in: batch*prod(dims[:-1])*(n/2+1) complex.
 * out: batch*prod(dims) doubles.
 */
int oracle_c2r(int rank, const int64_t *dims, int64_t batch, const double *in, double *out)
{
    if (bad_geometry(rank, dims, batch) || !in || !out) return ORACLE_BAD_ARG;
    int64_t per = 1;
    for (int a = 0; a < rank; ++a) per *= dims[a];
    const int64_t n = dims[rank - 1], h = n / 2 + 1;
    const int64_t rows = batch * (per / n);
    cplx *half = (cplx *)malloc(sizeof(cplx) * (size_t)(rows * h > 0 ? rows * h : 1));
    cplx *full = (cplx *)malloc(sizeof(cplx) * (size_t)(rows * n > 0 ? rows * n : 1));
    if (!half || !full) {
        free(half);
        free(full);
        return ORACLE_NO_MEM;
    }
    memcpy(half, in, sizeof(cplx) * (size_t)(rows * h));
    int st = ORACLE_OK;
    if (rank > 1) {
        /* leading axes: scaled inverse c2c on the half-spectrum array */
        int64_t hd[3];
        for (int a = 0; a < rank; ++a) hd[a] = dims[a];
        hd[rank - 1] = h;
        for (int a = rank - 2; a >= 0 && st == ORACLE_OK; --a) st = along_axis(half, rank, hd, batch, a, +1);
        const double sc = (double)n / (double)per; /* 1/prod(leading dims) */
        for (int64_t e = 0; e < rows * h; ++e) {
            half[e].re *= sc;
            half[e].im *= sc;
        }
    }
    if (st == ORACLE_OK) {
#pragma omp parallel for
        for (int64_t r = 0; r < rows; ++r) {
            cplx *y = full + r * n;
            const cplx *x = half + r * h;
            for (int64_t k = 0; k < n; ++k) {
                y[k].re = 0.0;
                y[k].im = 0.0;
            }
            y[0].re = x[0].re;
            for (int64_t k = 1; k < h; ++k) {
                if (2 * k == n) {
                    y[k].re = x[k].re; /* Nyquist: real part only */
                } else {
                    y[k] = x[k];
                    y[n - k].re = x[k].re;
                    y[n - k].im = -x[k].im;
                }
            }
        }
        const int64_t d1 = n;
        st = oracle_c2c(1, &d1, rows, +1, (const double *)full, (double *)full);
    }
    if (st == ORACLE_OK)
        for (int64_t e = 0; e < rows * n; ++e) out[e] = full[e].re;
    free(half);
    free(full);
    return st;
}

/*
 * Discrete cosine transforms by their definitions (unnormalised, scipy.fft.dct norm=None):
 *   type 2: y_k = 2 sum_{j<n} x_j cos(pi k (2j+1) / (2n))
 *   type 3: y_k = x_0 + 2 sum_{1<=j<n} x_j cos(pi j (2k+1) / (2n))
 * so that type 3 applied to type 2 gives 2n x.  Each cosine is the real part of the exact
 * root exp(-2 pi i m / (4n)) with the index m reduced modulo 4n.  O(n^2) per transform;
 * OpenMP over the transforms of the batch.
 */
int oracle_dct(int type, int64_t n, int64_t batch, const double *in, double *out)
{
    if (n < 1 || batch < 0 || (type != 2 && type != 3)) return 1;
    const int64_t N4 = 4 * n;
#pragma omp parallel for schedule(dynamic)
    for (int64_t b = 0; b < batch; ++b) {
        const double *x = in + b * n;
        double *y = out + b * n;
        for (int64_t k = 0; k < n; ++k) {
            double acc = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                if (type == 2) {
                    acc += 2.0 * x[j] * unit_root(N4, (k * (2 * j + 1)) % N4, -1).re;
                } else {
                    const double wj = j == 0 ? 1.0 : 2.0;
                    acc += wj * x[j] * unit_root(N4, (j * (2 * k + 1)) % N4, -1).re;
                }
            }
            y[k] = acc;
        }
    }
    return 0;
}

/* exp(sigma*2*pi*i*m/n) exactly as the oracle evaluates it; exported for the pins. */
void oracle_unit_root(int64_t n, int64_t m, int sigma, double *re_im)
{
    cplx w = unit_root(n, m, sigma);
    re_im[0] = w.re;
    re_im[1] = w.im;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads this calling thread's later oracle calls may use (n >= 1); lets a test run
 * many small single-threaded calls side by side from its own worker threads. */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
