// Host-side planner: turns (rank, dims, batch, kind, direction, dtype) into an
// ordered list of kernel launches ("ops") and the tables they need.  No HIP calls
// here, so the whole decision logic runs (and is tested) on a machine without a GPU.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "fft_args.h"

namespace mifft {

// Buffers an op reads or writes: the caller's two, and plan-owned scratch.
// S0/S1: temporaries of multi-pass chains; S2: Bluestein work lines;
// S3: staged real rows; S4: c2r half-spectrum staging.
enum BufId : int { B_IN = 0, B_OUT = 1, B_S0 = 2, B_S1 = 3, B_S2 = 4, B_S3 = 5, B_S4 = 6, B_NBUF = 7 };

enum OpType : int {
    OP_PASS = 0,          // one Stockham pass (kernel k_pass)
    OP_CHIRP_PAD,         // Bluestein: a = x * w, zero-padded to M
    OP_MUL_CONJ,          // Bluestein: A <- conj(A * B_filter)   (in place)
    OP_CHIRP_EXTRACT,     // Bluestein: X = w * conj(E) * scale
    OP_R2C_TWIST,         // real even n, staged: half spectrum from the n/2-point z spectrum
    OP_C2R_UNTWIST,       // real even n, staged: z spectrum from the half spectrum
    OP_REAL_TO_CPLX,      // real odd n, staged: x -> x + 0i
    OP_HALF_COPY,         // real odd n, staged: keep k <= n/2
    OP_HERM_EXPAND,       // real odd n, staged: half spectrum -> full Hermitian spectrum
    OP_CPLX_TO_REAL,      // real odd n, staged: keep the real part
    OP_DCT2_PRE,          // DCT-II: v = (x_0, x_2, ..., x_3, x_1) as complex
    OP_DCT2_POST,         // DCT-II: y_k = 2 Re(W_4n^k V_k)
    OP_DCT3_PRE,          // DCT-III: z_k = w_k x_k W_4n^k (w_0 = 1, else 2)
    OP_DCT3_POST,         // DCT-III: y_2m = Re Z_m, y_2m+1 = Re Z_{n-1-m}
    OP_DCT2_TWPOST,       // DCT-II, staged real transform: the r2c twist and the DCT-II rotation in one
                          // pass over the n/2-point spectrum
    OP_DCT3_PREUNTWIST,   // DCT-III, staged real transform: the DCT-III rotation and the c2r untwist
                          // (of the conjugate) in one pass
    OP_NTYPES
};

const char *op_name(int type);

// A table the plan needs on the device, generated in FP64 on the GPU.
struct TableReq {
    enum Kind : int {
        INNER = 0, // inner Stockham twiddles of one pass decomposition (stages in `st`)
        RANGE = 1, // W_N^{e0 + i*step}, i < count
        CHIRP = 2, // w_j = exp(-pi i (j^2 mod 2N)/N), j < count   (N = Bluestein length)
        BFILTER = 3 // FFT_M of the wrapped conjugate chirp of length N (count = M)
    } kind;
    int64_t N = 0, e0 = 0, step = 1, count = 0;
    int nst = 0;
    StageInfo st[kMaxStages] = {};
    int64_t offset = 0; // complex elements into the plan's table arena
    std::string key() const;
};

struct Op {
    int type = OP_PASS;
    int src = B_IN, dst = B_OUT;
    int src_real = 0, dst_real = 0; // buffer holds reals rather than complex (offsets in reals)
    PassArgs pa{};
    LineArgs la{};
    // table ids (index into PlanSpec::tables) for the pointer fields, -1 = none
    int t_itw = -1, t_lo = -1, t_hi = -1, t_aux = -1, t_aux2 = -1, t_tab = -1, t_tab2 = -1;
    int64_t grid = 0;
    int block = 0;
    std::string note;
};

struct PlanSpec {
    int rank = 0;
    int64_t dims[3] = {1, 1, 1};
    int64_t batch = 0;
    int kind = 0, direction = -1, dtype = 0;
    bool f64 = false;
    // The batch runs in chunks of `chunk` transforms (0: all at once).  `ops` and
    // `ops_inplace` then cover one chunk, and `tail_ops` / `tail_ops_inplace` the last
    // batch % chunk transforms (empty when the chunk divides the batch); chunk c reads
    // at in + c * chunk * in_dist and writes at out + c * chunk * out_dist.
    std::vector<Op> ops;
    std::vector<Op> ops_inplace; // c2c with in == out (empty when `ops` is already safe for that)
    int64_t chunk = 0;
    std::vector<Op> tail_ops, tail_ops_inplace;
    int64_t in_dist = 0, out_dist = 0;   // elements of the input's / output's type per transform
    std::vector<TableReq> tables;
    int64_t table_elems = 0;            // complex elements of the table arena
    int64_t scratch_elems[B_NBUF] = {}; // complex elements per scratch buffer (S0..S3)
    int64_t in_elems = 0, out_elems = 0; // per call, in the buffer's own element type
    bool generic_only = false;           // plan every pass for the runtime-generic kernel
    int64_t chunk_target = -1;           // input bytes per batch chunk forced by the caller (-1: the
                                         // planner's rules, tuning table and MIFFT_CHUNK_BYTES)
    bool ragged = false;                 // part of a ragged batch: one workgroup runs the whole plan,
                                         // so keep LDS small (occupancy) and skip the in-place op list
    std::string describe() const;
};

// Ragged batch: one plan per distinct length, shared by the transforms of that length.
struct ManySpec {
    bool f64 = false;
    int direction = -1, dtype = 0;
    struct Class {
        int64_t n = 0;
        int first_op = 0, nops = 0;
        int64_t sofs[B_NBUF] = {}; // scratch region offsets within one transform's scratch
        int64_t scratch = 0;       // scratch elements per transform of this length
        int64_t count = 0;         // transforms of this length
    };
    std::vector<Class> classes;
    std::vector<Op> ops;             // every class's ops (out-of-place list), table ids global
    std::vector<TableReq> tables;
    int64_t table_elems = 0;
    std::vector<int> xform_class;    // class of each transform
    std::string describe() const;
};

int build_many(int64_t count, const int64_t *lengths, int kind, int direction, int dtype, ManySpec &ms,
               std::string &err);

// Launch schedule of a ragged batch.  A transform whose plan has few parts (tiles of
// its passes plus chunks of its element-wise ops) runs whole in one block; a larger
// one puts part j of its op k in phase k, one block per part, so every pass of it is
// spread over the GPU and the launch boundary orders its ops.  Whole transforms go to
// the phase with the least work so far; blocks of a phase are ordered by cost, largest
// first, and dealt to the XCDs in runs of consecutive blocks.
struct RaggedSchedule {
    struct Block {
        uint32_t t, op, part, whole; // transform, op within its class, part, whole flag
    };
    std::vector<Block> blocks;       // phase after phase
    std::vector<uint32_t> phase_first, phase_blocks;
    int64_t whole_transforms = 0, split_transforms = 0;
    std::string describe() const;
};

// Parts a transform may have and still run whole in one block (default; the tuning
// table's "rag:schedule" entry overrides it).
constexpr int64_t kRagWholeParts = 8;

// XCDs of the device (workgroups are dealt to them round-robin), and the number of
// consecutive ragged blocks given to one XCD (default; "rag:schedule" c<group>).
constexpr uint32_t kXcds = 8;
constexpr int64_t kRagXcdGroup = 8;

int schedule_many(const ManySpec &ms, RaggedSchedule &rs, std::string &err);

// Input bytes per chunk when a plan runs its batch in chunks (its intermediates then
// stay in the 256 MB last-level cache between passes); MIFFT_CHUNK_BYTES overrides.
constexpr int64_t kChunkBytes = int64_t(128) << 20;

// Status codes match include/mifft.h.
int build_plan(int rank, const int64_t *dims, int64_t batch, int kind, int direction, int dtype,
               PlanSpec &spec, std::string &err);

// Process-wide tuning table (see the tuning section of planner.cpp): merge or replace
// entries, and dump the table as "key=value" lines.
int tune_set(const char *entries, int replace);
std::string tune_dump();

// Factorisation helpers (exposed for the planner tests through fft_plan_inspect).
bool is_smooth7(int64_t n);
std::vector<int> base_radices(int64_t L);
std::vector<int> inner_radices(int64_t L);
std::vector<int64_t> pass_lengths(int64_t n, int64_t max_len);

// Sets the thread-local status and message that fft_last_error* report; returns status.
int set_error(int status, const std::string &msg);

} // namespace mifft
