/*
 * mifft — discrete Fourier transforms on one MI355X (gfx950), C ABI.
 *
 * The operation (numpy.fft conventions; the paper, a finite-difference
 * code generator, defines no Fourier transform, so these follow the DFT's
 * definition and numpy's documented layout):
 *
 *   forward   X[k] = sum_{j<n} x[j] * exp(-2*pi*i*j*k/n)                (unscaled)
 *   inverse   x[j] = (1/n) * sum_{k<n} X[k] * exp(+2*pi*i*j*k/n)
 *
 * applied along every axis of a rank-1..3 array; the inverse scale is
 * 1/prod(dims).  Real transforms keep dims[rank-1]/2+1 bins along the last axis
 * (numpy rfftn/irfftn layout, "Hermitian-packed").
 *
 * Execution model (plan once, execute many; buffers bound per call — the same
 * split as the paper's Operator, built once and then called with its data,
 * Sections "Design and API" and "Fluid Dynamics Examples"):
 *   fft_plan_create    validates, factorises, builds twiddle/chirp tables on the
 *                      GPU in FP64, allocates plan-owned scratch; may synchronise.
 *   fft_execute        enqueues kernels on `stream`; no allocation, no host
 *                      synchronisation, no host reads: safe to capture in a
 *                      hipGraph.  (A ragged plan owns a graph instantiated at
 *                      creation and launches it, re-binding its kernel nodes in
 *                      place when the buffers change; under a stream capture it
 *                      launches the same kernels one by one instead.)
 *   fft_plan_destroy   frees everything the plan owns (NULL-safe).
 *
 * Layouts.  `dims` are row-major (C order) logical sizes; the last dim is
 * contiguous.  The batch is the outermost index: transform b starts at element
 * b*dist, dist = prod(dims) for complex c2c data, prod(dims) reals for real
 * data, prod(dims[:-1])*(dims[rank-1]/2+1) complex for half spectra.
 * FFT_F32* data is complex64 (interleaved float re, im) / float32 reals;
 * FFT_F64 data is complex128 / float64.
 *
 * Ownership.  `in` and `out` are caller-owned device pointers and are never
 * freed or retained.  `in` is never written for any kind.  Tables and scratch
 * belong to the plan.  One plan must not be executed concurrently with itself
 * (its scratch is shared); use two plans for overlapping work.
 *
 * Errors.  Nothing aborts and no exception crosses the ABI.  fft_plan_create*
 * return NULL and set a thread-local status and message (fft_last_error,
 * fft_last_error_message); fft_execute returns the status and sets the same.
 */
#ifndef MIFFT_H
#define MIFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* hipStream_t as HIP defines it (an identical typedef is legal in C11/C++). */
typedef struct ihipStream_t *hipStream_t;

typedef struct fft_plan_s *fft_plan; /* opaque, library-owned */

enum fft_kind {
    FFT_C2C = 0,  /* complex -> complex, either direction */
    FFT_R2C = 1,  /* real -> half spectrum, FORWARD only */
    FFT_C2R = 2,  /* half spectrum -> real, INVERSE only (numpy irfftn semantics) */
    FFT_DCT2 = 3, /* real -> real DCT-II, rank 1, FORWARD only:
                     y_k = 2 sum_j x_j cos(pi k (2j+1) / (2n))  (scipy.fft.dct type 2, norm=None) */
    FFT_DCT3 = 4  /* real -> real DCT-III, rank 1, FORWARD only:
                     y_k = x_0 + 2 sum_{j>=1} x_j cos(pi j (2k+1) / (2n));  DCT-III(DCT-II(x)) = 2n x */
};

enum fft_direction {
    FFT_FORWARD = -1, /* sign of the exponent */
    FFT_INVERSE = +1
};

enum fft_dtype {
    FFT_F32 = 0,        /* complex64 data, FP32 arithmetic */
    FFT_F64 = 1,        /* complex128 data, FP64 arithmetic */
    FFT_F32_BF16X2 = 2, /* complex64 data; radix-16 stages as BF16 MFMA DFT-matrix
                           products, operands split hi+lo, FP32 accumulation */
    FFT_F32_BF16X3 = 3  /* as above with a hi+mid+lo split (FP32-level accuracy) */
};

enum fft_status {
    FFT_OK = 0,
    FFT_ERR_INVALID_ARG = 1, /* bad rank/dims/batch/kind/direction/dtype, NULL or aliased buffers */
    FFT_ERR_UNSUPPORTED = 2, /* valid request this library does not implement */
    FFT_ERR_ALLOC = 3,       /* device or host allocation failed */
    FFT_ERR_HIP = 4,         /* a HIP runtime call or kernel launch failed */
    FFT_ERR_INTERNAL = 5
};

/*
 * Plan a batched transform.
 *   rank       1, 2 or 3.
 *   dims       rank logical sizes, each >= 1 (for real kinds: the real length).
 *   batch      number of transforms, >= 1.
 *   kind       enum fft_kind.
 *   direction  enum fft_direction; R2C requires FORWARD, C2R requires INVERSE.
 *   dtype      enum fft_dtype; the BF16 forms accept C2C, rank 1 only.
 * Elements per call (input and output, and Bluestein's padded lines) must stay
 * below 2^32 - 1 (32-bit element indexing; larger requests return
 * FFT_ERR_UNSUPPORTED).  Every length is handled: lengths with a prime factor
 * above 7 go through Bluestein's chirp-z algorithm.
 * Returns NULL on error (see fft_last_error).  Binds to the current HIP device.
 */
fft_plan fft_plan_create(int rank, const int64_t *dims, int64_t batch, int kind, int direction, int dtype);

/*
 * Run the planned transform: in -> out on `stream` (NULL = the null stream).
 * C2C allows in == out (in place); the other kinds do not (FFT_ERR_INVALID_ARG).
 * Partially overlapping buffers are undefined.  Asynchronous; returns FFT_OK
 * once every kernel is enqueued.
 */
int fft_execute(fft_plan plan, const void *in, void *out, hipStream_t stream);

/* Free the plan's tables, scratch and graphs. NULL-safe. */
void fft_plan_destroy(fft_plan plan);

/*
 * Plan `count` independent 1-D transforms of uneven lengths, executed together
 * (the ragged batch).  Transform t has length lengths[t] >= 1 and reads
 * in[in_offsets[t] .. +lengths[t]) and writes out[out_offsets[t] .. +lengths[t])
 * (offsets in complex elements).  C2C only; dtype FFT_F32 or FFT_F64.
 * fft_execute(plan, in, out, stream) then runs all of them with one
 * hipGraphLaunch: the graph, instantiated when the plan is created, holds a few
 * kernel nodes, one per phase, whose buffer arguments are re-bound in place
 * (hipGraphExecKernelNodeSetParams) when a call passes other buffers than the
 * previous one; under a stream capture the phase kernels are launched one by
 * one, so the caller's graph records them.  A small transform
 * runs whole inside one workgroup; a large one runs op k of its plan (a
 * Stockham pass, or an element-wise Bluestein step) in phase k, spread over
 * many workgroups.  No workgroup waits on another.  Out of place only
 * (in == out is FFT_ERR_INVALID_ARG); output ranges must not overlap each
 * other or the input.  Two executions of one plan must not overlap in time
 * (the plan's scratch is shared).
 */
fft_plan fft_plan_create_many(int64_t count, const int64_t *lengths, const int64_t *in_offsets,
                              const int64_t *out_offsets, int kind, int direction, int dtype);

/* Status and message of the last failing call on this thread (FFT_OK / "" if none). */
int fft_last_error(void);
const char *fft_last_error_message(void);

/*
 * Human-readable description of a plan: passes, radices, tiles, LDS bytes,
 * scratch bytes.  The string is owned by the plan and lives until it is
 * destroyed.
 */
const char *fft_plan_describe(fft_plan plan);

/*
 * Host-only planner dry run: writes the same description fft_plan_describe
 * would give, without touching any GPU, into buf (at most len bytes, NUL
 * terminated).  Returns FFT_OK or the status plan creation would fail with.
 */
int fft_plan_inspect(int rank, const int64_t *dims, int64_t batch, int kind, int direction, int dtype,
                     char *buf, size_t len);

/*
 * Host-only dry run of fft_plan_create_many: the description (per-length
 * plans and the phase schedule) without touching any GPU, into buf as for
 * fft_plan_inspect.  Offsets are not needed.
 */
int fft_plan_inspect_many(int64_t count, const int64_t *lengths, int kind, int direction, int dtype, char *buf,
                          size_t len);

/*
 * Tuning table: per-shape overrides picked by the autotuner
 * (paper_1707_03776_amd/autotune.py), read by the planner when a plan is
 * created (plans that exist are unaffected).  `entries` holds "key=value"
 * items separated by ';' or newlines ('#' starts a comment line):
 *   pass key  "f32:L1024:16x8x8:CC:tw1"  -> c<cols>,p<pitch residue>,t<threads>
 *   radix key "f32:L1024:radix"          -> r16.8.8
 *   split key "f32:n1048576:S1:split"    -> s1024.1024
 *   "rag:schedule"                       -> w<parts> (ragged: largest number of
 *                                           parts a transform runs whole in one block)
 * (keys of ragged plans start with "rag:"; fft_plan_describe prints every
 * pass's key).  replace != 0 clears the table first.  Entries that do not
 * apply to a plan, or that it cannot honour, leave the planner's default.
 * The table starts with the file named by MIFFT_TUNE_FILE, if set.
 * Thread-safe.  Returns FFT_OK.
 */
int fft_tune_set(const char *entries, int replace);

/* Writes the table as "key=value" lines into buf (NUL terminated); returns
 * FFT_ERR_INVALID_ARG if buf is NULL/empty or the table does not fit. */
int fft_tune_get(char *buf, size_t len);

/*
 * For callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): plan and run one transform in a
 * single call that allocates nothing on the device.  Arguments as for
 * fft_plan_create followed by fft_execute (in, out caller-owned device buffers; C2C
 * may run in place).  The plan's FP64/FP32 tables and its scratch live in one static
 * device array of 64 MiB per GPU (held by each GPU the library runs on until the
 * process ends); the tables are regenerated on `stream` by every call, and nothing
 * there needs to start at zero.  A batch whose scratch would exceed the array runs in
 * smaller chunks; a request that still does not fit, or any length with a prime
 * factor above 7 (Bluestein's filter would need a plan of its own), returns
 * FFT_ERR_UNSUPPORTED.  Every call on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (other streams, other threads) race and must not be
 * issued.  Same results as fft_plan_create + fft_execute.  Returns the status
 * (fft_last_error / fft_last_error_message as for the other calls).
 */
int fft_execute_noalloc(int rank, const int64_t *dims, int64_t batch, int kind, int direction, int dtype,
                        const void *in, void *out, hipStream_t stream);

/* Device bytes the plan owns (tables + scratch), for accounting. */
int64_t fft_plan_device_bytes(fft_plan plan);

/*
 * Pseudo-spectral Laplacian of real fields on a periodic grid: the operator of
 * the "Laplace equation" example (Section "Fluid Dynamics Examples") and the
 * Laplacian term of the acoustic wave equation (Section "Seismic Inversion
 * Example"), evaluated spectrally instead of by a finite-difference stencil:
 *
 *   lap u = c2r( -|kappa|^2 * r2c(u) ),   kappa_a = 2*pi*f_a / L_a,
 *
 * f_a the signed frequency of bin j along axis a (j for j <= n_a/2, else
 * j - n_a; the last axis holds j = 0..n/2), L_a the period of axis a (grid
 * spacing L_a / n_a).  The inverse transform carries the 1/prod(dims) scale.
 *   rank, dims, batch  as for fft_plan_create (dims are the real sizes).
 *   lengths            rank finite periods L_a > 0.
 *   dtype              FFT_F32 (float32 fields) or FFT_F64 (float64 fields).
 * Layout: batch fields of prod(dims) reals, C order, field b at b*prod(dims).
 * The operator owns an r2c plan, a c2r plan and one half-spectrum buffer
 * (batch * prod(dims[:-1]) * (dims[rank-1]/2+1) complex elements); where the c2r
 * plan's first pass is a specialised kernel over one whole axis, the wavenumber
 * multiply is done by that pass as it loads the spectrum (small FP64 tables of
 * -c_a f_a^2 per axis, owned by the operator), else by a kernel of its own
 * (MIFFT_LAPLACE_UNFUSED=1 at creation forces the latter).
 * fft_laplacian_execute enqueues r2c, the wavenumber multiply and c2r on
 * `stream`; it allocates nothing and never synchronises.  in == out is
 * allowed (the input is fully read before the output is written); `in` is
 * otherwise never written.  Errors as for plans: NULL / a status, with
 * fft_last_error and fft_last_error_message set.  One operator must not be
 * executed concurrently with itself.
 */
typedef struct fft_laplacian_s *fft_laplacian;
fft_laplacian fft_laplacian_create(int rank, const int64_t *dims, int64_t batch, const double *lengths, int dtype);
int fft_laplacian_execute(fft_laplacian op, const void *in, void *out, hipStream_t stream);
void fft_laplacian_destroy(fft_laplacian op); /* NULL-safe */
/* Description of both plans and the multiply; owned by the operator. */
const char *fft_laplacian_describe(fft_laplacian op);

#ifdef __cplusplus
}
#endif

#endif /* MIFFT_H */
