// Host-side planner (see planner.h).  Decides, for every axis of the request,
// how the transform splits into workgroup-sized Stockham passes (or Bluestein's
// chirp-z when a prime factor above 7 remains), which buffers each pass reads and
// writes, how a workgroup tiles its columns, and which tables are needed.
#include "planner.h"
#include "kernels.h"
#include "shapes.h"

#include <algorithm>
#include <cctype>
#include <cstdlib>
#include <fstream>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <sstream>
#include <tuple>

namespace mifft {

std::vector<int> inner_radices16(int64_t L);

namespace {

constexpr int kOK = 0, kInvalid = 1, kUnsupported = 2, kInternal = 5;

int64_t pow2_ceil(int64_t v)
{
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

int64_t pow2_floor(int64_t v)
{
    int64_t p = 1;
    while (p * 2 <= v) p <<= 1;
    return p;
}

int ilog2_ceil(int64_t v)
{
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

std::vector<int64_t> prime_factors(int64_t n)
{
    std::vector<int64_t> f;
    for (int64_t p = 2; p * p <= n; ++p)
        while (n % p == 0) {
            f.push_back(p);
            n /= p;
        }
    if (n > 1) f.push_back(n);
    return f;
}

struct Ctx {
    PlanSpec &sp;
    std::map<std::string, int> table_ids;
    int elem;  // bytes per complex element
    int maxe;  // register budget (complex elements per thread per stage)
    int shift; // LDS padding: one spare slot every 2^shift elements
    bool route_scratch = false; // chains keep every intermediate in plan scratch (chunked plans)
    int64_t force_c = 0;        // tile_pass: columns per tile asked for (0: its own choice)

    explicit Ctx(PlanSpec &s) : sp(s)
    {
        elem = s.f64 ? 16 : 8;
        maxe = s.f64 ? RegBudget<double>::kElems : RegBudget<float>::kElems;
        shift = s.f64 ? kLdsPadShiftF64 : kLdsPadShiftF32;
    }

    int table(const TableReq &t)
    {
        std::string k = t.key();
        auto it = table_ids.find(k);
        if (it != table_ids.end()) return it->second;
        TableReq c = t;
        c.offset = sp.table_elems;
        sp.table_elems += (c.count + 31) / 32 * 32; // keep every table 256-byte aligned (FP32) or better
        sp.tables.push_back(c);
        int id = int(sp.tables.size()) - 1;
        table_ids[k] = id;
        return id;
    }

    int64_t lds_pitch(int64_t L) const { return L + (L >> shift) + 1; }

    void need_scratch(int buf, int64_t elems)
    {
        if (buf >= B_S0) sp.scratch_elems[buf] = std::max(sp.scratch_elems[buf], elems);
    }
};

// Drop size-1 column dims (keeping order) and remember where the twiddle dim went.
void compact_cols(PassArgs &pa, int tw_dim_in)
{
    int64_t sz[kColDims], ci[kColDims], co[kColDims];
    int m = 0, tw = -1;
    for (int d = 0; d < kColDims; ++d) {
        if (pa.csz[d] == 1 && d != tw_dim_in) continue;
        sz[m] = pa.csz[d];
        ci[m] = pa.cin[d];
        co[m] = pa.cout[d];
        if (d == tw_dim_in) tw = m;
        ++m;
    }
    for (int d = 0; d < kColDims; ++d) {
        pa.csz[d] = d < m ? sz[d] : 1;
        pa.cin[d] = d < m ? ci[d] : 0;
        pa.cout[d] = d < m ? co[d] : 0;
    }
    pa.tw_dim = tw;
}

// ----------------------------------------------------------------------------- tuning table

// Overrides written by the autotuner (paper_1707_03776_amd/autotune.py) and read by the
// planner.  One process-wide table of "key=value" items; values are comma-separated
// knobs:
//   pass keys (pass_key, "rag:"-prefixed inside ragged plans):
//       c<cols>  columns per workgroup (power of two; T and LDS follow)
//       p<res>   LDS column pitch residue modulo the padding unit
//       t<thr>   minimum workgroup size (multiple of 64)
//   radix keys ("<dt>:L<L>:radix", "rag:"-prefixed inside ragged plans):
//       r<r1>.<r2>...   inner radix sequence of every pass of length L
//   split keys ("<dt>:n<n>:S1:split" for contiguous axes, ":Sx:" for strided ones):
//       s<L1>.<L2>...   pass lengths of the axis, first pass first
//   "rag:schedule":
//       w<parts>        largest number of parts a ragged transform may have and still
//                       run whole in one block
//       c<group>        consecutive blocks of a phase (in cost order) dealt to one XCD
//   chunk keys ("<dt>:<kind>:<dims, x-separated>:chunk"):
//       b<bytes>        input bytes per batch chunk (0: the whole batch at once)
// Sources, later ones overriding: the file named by MIFFT_TUNE_FILE (read once),
// fft_tune_set, and the MIFFT_TUNE environment variable (read at every plan).
// Invalid or unusable entries are ignored (the planner's default is used).
struct Tune {
    int c = 0;              // 0: planner default
    int lp_mod = -1;        // -1: planner default
    int t = 0;              // 0: planner default
    std::vector<int> r;     // empty: planner default
    std::vector<int64_t> s; // empty: planner default
    int w = 0;              // 0: planner default
    int64_t b = -1;         // -1: planner default
};

std::string dt_name(const PlanSpec &sp)
{
    return std::string(sp.ragged ? "rag:" : "") +
           (sp.f64 ? "f64" : sp.dtype == 2 ? "bf2" : sp.dtype == 3 ? "bf3" : "f32");
}

std::string pass_key(const PlanSpec &sp, const PassArgs &pa)
{
    std::ostringstream o;
    o << dt_name(sp) << ":L" << pa.L << ":";
    for (int s = 0; s < pa.nst; ++s) o << (s ? "x" : "") << pa.st[s].r;
    o << ":" << (pa.load_cf ? 'C' : 'P') << (pa.store_cf ? 'C' : 'P') << ":tw" << (pa.tw_dim >= 0 ? 1 : 0);
    if (pa.pro == PRO_C2R) o << ":c2r";
    if (pa.pro == PRO_BPAD) o << ":bpad";
    if (pa.epi == EPI_R2C) o << ":r2c";
    if (pa.epi == EPI_BMUL) o << ":bmul";
    if (pa.epi == EPI_BEXT) o << ":bext";
    return o.str();
}

std::string radix_key(const PlanSpec &sp, int64_t L) { return dt_name(sp) + ":L" + std::to_string(L) + ":radix"; }

std::string chunk_key(const PlanSpec &sp)
{
    static const char *kinds[5] = {"c2c", "r2c", "c2r", "dct2", "dct3"};
    std::string k = dt_name(sp) + ":" + kinds[sp.kind >= 0 && sp.kind < 5 ? sp.kind : 0] + ":";
    for (int a = 0; a < sp.rank; ++a) k += (a ? "x" : "") + std::to_string(sp.dims[a]);
    return k + ":chunk";
}

std::string split_key(const PlanSpec &sp, int64_t n, int64_t S)
{
    return dt_name(sp) + ":n" + std::to_string(n) + (S == 1 ? ":S1" : ":Sx") + ":split";
}

template <typename T> std::vector<T> parse_dotted(const std::string &f)
{
    std::vector<T> v;
    std::stringstream ss(f);
    std::string x;
    while (std::getline(ss, x, '.'))
        if (!x.empty()) v.push_back(T(std::atoll(x.c_str())));
    return v;
}

std::string trim(const std::string &x)
{
    size_t i = 0, j = x.size();
    while (i < j && isspace((unsigned char)x[i])) ++i;
    while (j > i && isspace((unsigned char)x[j - 1])) --j;
    return x.substr(i, j - i);
}

void parse_tune_items(std::string text, std::map<std::string, Tune> &out)
{
    for (char &ch : text)
        if (ch == '\n' || ch == '\r') ch = ';';
    std::stringstream ss(text);
    std::string item;
    while (std::getline(ss, item, ';')) {
        item = trim(item);
        if (item.empty() || item[0] == '#') continue;
        const size_t eq = item.find('=');
        if (eq == std::string::npos) continue;
        const std::string key = trim(item.substr(0, eq));
        Tune t;
        std::stringstream vs(item.substr(eq + 1));
        std::string f;
        while (std::getline(vs, f, ',')) {
            f = trim(f);
            if (f.size() < 2) continue;
            const std::string v = f.substr(1);
            if (f[0] == 'c') t.c = std::atoi(v.c_str());
            if (f[0] == 'p') t.lp_mod = std::atoi(v.c_str());
            if (f[0] == 't') t.t = std::atoi(v.c_str());
            if (f[0] == 'r') t.r = parse_dotted<int>(v);
            if (f[0] == 's') t.s = parse_dotted<int64_t>(v);
            if (f[0] == 'w') t.w = std::atoi(v.c_str());
            if (f[0] == 'b') t.b = std::atoll(v.c_str());
        }
        out[key] = t;
    }
}

std::string format_tune(const Tune &t)
{
    std::ostringstream o;
    const char *sep = "";
    if (t.c > 0) { o << sep << "c" << t.c; sep = ","; }
    if (t.lp_mod >= 0) { o << sep << "p" << t.lp_mod; sep = ","; }
    if (t.t > 0) { o << sep << "t" << t.t; sep = ","; }
    if (!t.r.empty()) {
        o << sep << "r";
        for (size_t i = 0; i < t.r.size(); ++i) o << (i ? "." : "") << t.r[i];
        sep = ",";
    }
    if (!t.s.empty()) {
        o << sep << "s";
        for (size_t i = 0; i < t.s.size(); ++i) o << (i ? "." : "") << t.s[i];
        sep = ",";
    }
    if (t.w > 0) { o << sep << "w" << t.w; sep = ","; }
    if (t.b >= 0) o << sep << "b" << t.b;
    return o.str();
}

std::mutex &tune_mutex()
{
    static std::mutex m;
    return m;
}

std::map<std::string, Tune> &tune_table_locked()
{
    static std::map<std::string, Tune> table = [] {
        std::map<std::string, Tune> t;
        const char *path = std::getenv("MIFFT_TUNE_FILE");
        if (path && *path) {
            std::ifstream f(path);
            std::stringstream buf;
            buf << f.rdbuf();
            parse_tune_items(buf.str(), t);
        }
        return t;
    }();
    return table;
}

bool find_tune(const std::string &key, Tune &out)
{
    std::map<std::string, Tune> env;
    if (const char *e = std::getenv("MIFFT_TUNE")) parse_tune_items(e, env);
    auto it = env.find(key);
    if (it != env.end()) {
        out = it->second;
        return true;
    }
    std::lock_guard<std::mutex> lock(tune_mutex());
    const std::map<std::string, Tune> &tab = tune_table_locked();
    const auto jt = tab.find(key);
    if (jt != tab.end()) {
        out = jt->second;
        return true;
    }
    return false;
}

Tune lookup_tune(const PlanSpec &sp, const PassArgs &pa)
{
    Tune t;
    if (find_tune(pass_key(sp, pa), t)) return t;
    if (find_tune(sp.ragged ? "rag:*" : "*", t)) return t;
    return Tune{};
}

// The specialised kernels give each thread kFixedElems / r butterflies of radix r
// per stage (and up to FixedMaxThreads threads); the generic one RegBudget / r
// (and up to 256 threads).
int stage_items(const Ctx &cx, const PassArgs &pa, int r)
{
    if (r == 1) return 8;
    if (cx.sp.ragged) return std::max(1, (cx.sp.f64 ? RaggedElems<double>::v : RaggedElems<float>::v) / r);
    return (pa.shape >= 0 || pa.mshape >= 0 ? kFixedElems : cx.maxe) / r;
}

// Bytes of adjacent columns a strided pass's tile covers (the contiguous run of each of
// its global accesses): 128 bytes, 256 in ragged plans; MIFFT_COLFAST_BYTES overrides.
int64_t colfast_bytes(bool ragged)
{
    if (const char *e = std::getenv("MIFFT_COLFAST_BYTES")) {
        const int64_t v = std::atoll(e);
        if (v >= 16 && v <= 4096) return v;
    }
    // ragged passes: wider runs fill the short passes' tiles (the LDS budget still
    // caps c): 20,000-length batch 2.45 -> 2.34 ms with 256-byte runs
    return ragged ? 256 : 128;
}

// LDS per workgroup the tile choice aims for, and the largest group of a specialised
// pass kernel it picks by default (MIFFT_LDS_BUDGET, MIFFT_TILE_THREADS override).
int64_t lds_budget()
{
    if (const char *e = std::getenv("MIFFT_LDS_BUDGET")) {
        const int64_t v = std::atoll(e);
        if (v >= 1024 && v <= 160 * 1024) return v;
    }
    return kLdsBudget;
}
int64_t tile_threads()
{
    if (const char *e = std::getenv("MIFFT_TILE_THREADS")) {
        const int64_t v = std::atoll(e);
        if (v >= 64 && v <= 1024) return v;
    }
    return 512;
}

// Choose columns per workgroup, workgroup size and LDS for a pass.  Returns false
// if the pass cannot be tiled (L too large for one workgroup).
bool tile_pass(Ctx &cx, PassArgs &pa)
{
    const int64_t L = pa.L;
    if (pa.nst < 1 || pa.nst > kMaxStages) return false; // no in-workgroup decomposition
    pa.load_cf = (pa.pro != PRO_C2R && pa.rin != 1) ? 1 : 0;
    pa.store_cf = (pa.epi != EPI_R2C && pa.rout != 1) ? 1 : 0;
    const bool colfast = pa.load_cf || pa.store_cf;
    int64_t c;
    if (colfast)
        c = colfast_bytes(cx.sp.ragged) / cx.elem; // runs of that many bytes along the contiguous column index
    else
        c = std::max<int64_t>(1, pow2_floor(std::max<int64_t>(1, (cx.sp.f64 ? 2048 : 4096) / L)));
    Tune tune = lookup_tune(cx.sp, pa);
    if (tune.c == 0 && cx.force_c > 0) tune.c = int(cx.force_c);
    if (tune.c > 0) c = pow2_floor(tune.c);
    c = std::min<int64_t>(c, pow2_ceil(std::max<int64_t>(1, pa.ncols)));
    const int pad_unit = 1 << cx.shift;
    auto pitch = [&](int64_t L0) {
        int64_t lp = cx.lds_pitch(L0);
        if (tune.lp_mod >= 0)
            while (lp % pad_unit != tune.lp_mod % pad_unit) ++lp;
        return lp;
    };
    const bool uses_lds = pa.nst > 1 || pa.pro == PRO_C2R || pa.epi == EPI_R2C;
    for (; c >= 1; c /= 2) {
        int64_t lds = uses_lds ? c * pitch(L) * cx.elem : 0;
        // the budget keeps two groups per CU unless the tuning asks for wider tiles
        const int64_t budget = cx.sp.ragged ? 36 * 1024 : lds_budget();
        if (lds > 160 * 1024 || (lds > budget && c > 1 && tune.c == 0)) continue;
        // smallest group size (multiple of 64) that fits every stage in registers
        const bool special = pa.shape >= 0 || pa.mshape >= 0;
        bool r64 = false;
        for (int s = 0; s < pa.nst; ++s) r64 = r64 || pa.st[s].r == 64;
        if (r64 && pa.mshape >= 0) {
            // the split radix-64 DFT matrix sits in LDS behind the tile
            lds = (lds + 15) / 16 * 16 + int64_t(pa.mode) * kMfma64PartBytes;
            if (lds > 160 * 1024) continue;
        }
        const int64_t tmax = r64 ? kMfma64MaxThreads
                                 : special ? (cx.sp.f64 ? FixedMaxThreads<double>::v : FixedMaxThreads<float>::v)
                                           : 256;
        const int64_t tdef = special ? std::min(tmax, tile_threads()) : 256; // default cap; wider only when tuned
        int64_t T = 64;
        for (int s = 0; s < pa.nst; ++s) {
            const int r = pa.st[s].r;
            // a radix-64 matrix-core stage gives each lane 16 points (a quarter butterfly)
            const int64_t maxi = r == 64 ? 1 : stage_items(cx, pa, r);
            const int64_t items = r == 64 ? c * L / 16 : c * (L / r);
            int64_t need = (items + maxi - 1) / maxi;
            need = (need + 63) / 64 * 64;
            T = std::max(T, need);
        }
        if (tune.t > 0) T = std::max<int64_t>(T, (int64_t(tune.t) + 63) / 64 * 64);
        if (T > tmax || (T > tdef && tune.c == 0 && tune.t == 0)) continue;
        pa.c = int32_t(c);
        pa.logc = 0;
        while ((int64_t(1) << pa.logc) < c) ++pa.logc;
        pa.ncd = 1;
        for (int d = 0; d < kColDims; ++d) {
            if (pa.csz[d] > 1) pa.ncd = d + 1;
            pa.crcp[d] = 1.0 / double(pa.csz[d] > 0 ? pa.csz[d] : 1);
        }
        if (pa.tw_dim >= pa.ncd) pa.ncd = pa.tw_dim + 1;
        pa.threads = int32_t(T);
        pa.lp = int32_t(pitch(L));
        pa.lds_bytes = int32_t(lds);
        pa.ntiles = (pa.ncols + c - 1) / c;
        return true;
    }
    return false;
}

// Inner radix sequence of a pass of length L: the tuned one if the table has a valid
// entry, else the planner's default.
std::vector<int> choose_radices(const Ctx &cx, int64_t L, int mode)
{
    Tune t;
    if (find_tune(radix_key(cx.sp, L), t) && !t.r.empty() && int(t.r.size()) <= kMaxStages) {
        int64_t prod = 1;
        bool ok = true;
        for (int r : t.r) {
            ok = ok && (r == 2 || r == 3 || r == 4 || r == 5 || r == 6 || r == 7 || r == 8 || r == 9 || r == 10 ||
                        r == 12 || r == 14 || r == 15 || r == 16 || (r == 64 && mode >= 2));
            prod *= r;
        }
        // a matrix-core plan takes only sequences it has kernels for
        if (ok && prod == L && (mode < 2 || mfma_shape_id(t.r.data(), int(t.r.size())) >= 0)) return t.r;
    }
    if (mode >= 2) return inner_radices16(L);
    return inner_radices(L);
}

// Fill the inner stages of a pass of length L.
void set_stages(Ctx &cx, PassArgs &pa, Op &op)
{
    std::vector<int> rad = choose_radices(cx, pa.L, pa.mode);
    int64_t prod = 1;
    for (int r : rad) prod *= r;
    if (prod != pa.L) rad.clear(); // no valid decomposition: the pass will not tile
    pa.nst = int32_t(rad.size());
    pa.shape = (rad.empty() || cx.sp.generic_only) ? -1 : fixed_shape_id(rad.data(), int(rad.size()));
    pa.mshape = (pa.mode >= 2 && !rad.empty() && !cx.sp.generic_only) ? mfma_shape_id(rad.data(), int(rad.size()))
                                                                       : -1;
    int ns = 1, tw = 0;
    for (size_t s = 0; s < rad.size(); ++s) {
        pa.st[s].r = rad[s];
        pa.st[s].ns = ns;
        pa.st[s].tw = tw;
        tw += ns * (rad[s] - 1);
        ns *= rad[s];
    }
    if (pa.nst > 1 || (pa.nst == 1 && pa.st[0].ns > 1)) {
        TableReq t{};
        t.kind = TableReq::INNER;
        t.nst = pa.nst;
        for (int s = 0; s < pa.nst; ++s) t.st[s] = pa.st[s];
        t.count = std::max(1, tw);
        t.N = pa.L;
        op.t_itw = cx.table(t);
    }
}

void set_pass_twiddle(Ctx &cx, PassArgs &pa, Op &op, int64_t twN)
{
    pa.twN = twN;
    pa.tw_bits = (ilog2_ceil(twN) + 1) / 2;
    const int64_t B = int64_t(1) << pa.tw_bits;
    TableReq lo{};
    lo.kind = TableReq::RANGE;
    lo.N = twN;
    lo.e0 = 0;
    lo.step = 1;
    lo.count = std::min(B, twN);
    TableReq hi = lo;
    hi.step = B;
    hi.count = (twN + B - 1) / B;
    op.t_lo = cx.table(lo);
    op.t_hi = cx.table(hi);
}

std::string fmt_pass(const PassArgs &pa)
{
    std::ostringstream o;
    o << "L=" << pa.L << " radices=";
    for (int s = 0; s < pa.nst; ++s) o << (s ? "x" : "") << pa.st[s].r;
    o << (pa.mshape >= 0 ? (pa.mode == 3 ? " mfma-bf16x3" : " mfma-bf16x2") : pa.shape >= 0 ? " fixed" : " generic")
      << " c=" << pa.c << " T=" << pa.threads << " lds=" << pa.lds_bytes << " tiles=" << pa.ntiles
      << " cols=" << pa.ncols << " rin=" << pa.rin << " rout=" << pa.rout << " map=" << (pa.load_cf ? "C" : "P")
      << (pa.store_cf ? "C" : "P");
    if (pa.tw_dim >= 0) o << " twN=" << pa.twN;
    if (pa.pro == PRO_C2R) o << " pro=c2r";
    if (pa.pro == PRO_BPAD) o << " pro=bpad";
    if (pa.pro == PRO_SYM) o << " pro=sym";
    if (pa.pro == PRO_DCT2) o << " pro=dct2";
    if (pa.pro == PRO_CUNTWIST) o << " pro=cuntwist";
    if (pa.epi == EPI_DCT3) o << " epi=dct3";
    if (pa.epi == EPI_RTWIST) o << " epi=rtwist";
    if (pa.epi == EPI_DTWIST) o << " epi=dtwist";
    if (pa.epi == EPI_R2C) o << " epi=r2c";
    if (pa.epi == EPI_BMUL) o << " epi=bmul";
    if (pa.epi == EPI_BEXT) o << " epi=bext";
    return o.str();
}

// One Stockham pass over an axis of length n, inner count S (stride 1), outer
// count O (stride n*S): pass length L, Ns = product of earlier pass lengths.
bool add_axis_pass(Ctx &cx, int64_t n, int64_t S, int64_t O, int64_t L, int64_t Ns, int src, int dst,
                   std::string &err, int pro = PRO_PLAIN, int epi = EPI_PLAIN)
{
    Op op;
    op.type = OP_PASS;
    op.src = src;
    op.dst = dst;
    PassArgs &pa = op.pa;
    pa.L = int32_t(L);
    pa.scale = 1.0;
    pa.pro = pro;
    pa.epi = epi;
    pa.mode = cx.sp.dtype >= 2 ? cx.sp.dtype : 0;
    set_stages(cx, pa, op);
    if (pro == PRO_BPAD || epi == EPI_BMUL || epi == EPI_BEXT) {
        // the fused Bluestein steps exist in the runtime-radix kernel only
        pa.shape = -1;
        pa.mshape = -1;
    }
    const int64_t J = n / (L * Ns);
    pa.csz[0] = S;  pa.cin[0] = 1;          pa.cout[0] = 1;
    pa.csz[1] = Ns; pa.cin[1] = S;          pa.cout[1] = S;
    pa.csz[2] = J;  pa.cin[2] = Ns * S;     pa.cout[2] = Ns * L * S;
    pa.csz[3] = O;  pa.cin[3] = n * S;      pa.cout[3] = n * S;
    pa.rin = (n / L) * S;
    pa.rout = Ns * S;
    pa.ncols = S * Ns * J * O;
    compact_cols(pa, Ns > 1 ? 1 : -1);
    if (Ns > 1) set_pass_twiddle(cx, pa, op, Ns * L);
    if (!tile_pass(cx, pa)) {
        err = "cannot tile a pass of length " + std::to_string(L);
        return false;
    }
    op.grid = pa.ntiles;
    op.block = pa.threads;
    op.note = "axis n=" + std::to_string(n) + " Ns=" + std::to_string(Ns);
    cx.need_scratch(src, n * S * O);
    cx.need_scratch(dst, n * S * O);
    cx.sp.ops.push_back(op);
    return true;
}

// Longest strided pass a multi-pass chain uses (MIFFT_STRIDED_CAP overrides).
int64_t strided_cap(const Ctx &cx)
{
    if (cx.sp.ragged) return 512;
    if (const char *e = std::getenv("MIFFT_STRIDED_CAP")) {
        const int64_t v = std::atoll(e);
        if (v >= 16) return pow2_floor(v);
    }
    return 1024;
}

int64_t max_pass_len(const Ctx &cx, int64_t n, int64_t S)
{
    // a single pass over contiguous rows may use a whole workgroup per row;
    // strided passes need several adjacent columns per workgroup for coalescing
    (void)n;
    if (cx.sp.ragged) return S == 1 ? (cx.sp.f64 ? 1024 : 2048) : 512;
    if (S == 1) return cx.sp.f64 ? 4096 : 8192;
    return strided_cap(cx);
}

// Whether one workgroup can hold a length-L pass (registers, LDS) in the column
// layout a pass over an axis with inner count S would use.
bool pass_fits(Ctx &cx, int64_t L, int64_t S)
{
    PassArgs pa{};
    Op op;
    pa.L = int32_t(L);
    std::vector<int> rad = choose_radices(cx, L, 0);
    pa.nst = int32_t(rad.size());
    if (pa.nst < 1 || pa.nst > kMaxStages) return false;
    for (int s = 0; s < pa.nst; ++s) pa.st[s].r = rad[s];
    pa.shape = cx.sp.generic_only ? -1 : fixed_shape_id(rad.data(), int(rad.size()));
    pa.mshape = -1;
    pa.rin = S == 1 ? 1 : S;
    pa.rout = pa.rin;
    pa.ncols = 1 << 20;
    pa.pro = PRO_PLAIN;
    pa.epi = EPI_PLAIN;
    return tile_pass(cx, pa);
}

// Pass lengths of an axis of length n (inner count S): a tuned split if the table has a
// usable one, else a single pass when it fits, else strided passes of bounded length.
std::vector<int64_t> chain_lengths(Ctx &cx, int64_t n, int64_t S)
{
    std::vector<int64_t> Ls;
    Tune tsp;
    if (find_tune(split_key(cx.sp, n, S), tsp) && !tsp.s.empty() && tsp.s.size() <= 8) {
        int64_t prod = 1;
        bool ok = true;
        for (int64_t L : tsp.s) {
            ok = ok && L >= 2 && L <= 16384 && pass_fits(cx, L, tsp.s.size() == 1 ? S : 2);
            prod *= L;
        }
        if (ok && prod == n) Ls = tsp.s;
    }
    if (Ls.empty() && n <= max_pass_len(cx, n, S) && pass_fits(cx, n, S)) Ls.push_back(n);
    bool balanced = false;
    for (int64_t cap = strided_cap(cx); cap >= 16 && Ls.empty(); cap /= 2) {
        Ls = pass_lengths(n, cap);
        for (int64_t L : Ls)
            if (!pass_fits(cx, L, 2)) Ls.clear();
        balanced = !Ls.empty();
    }
    if (balanced && Ls.size() == 2 && !tsp.s.size()) {
        // two passes: among the splits within the same cap, take the fewest inner stages
        // (then the most specialised passes, then the size balance); the balanced split
        // wins ties
        const int64_t cap = std::max(Ls[0], Ls[1]) <= strided_cap(cx) ? strided_cap(cx) : std::max(Ls[0], Ls[1]);
        auto score = [&](int64_t a, int64_t b) {
            const std::vector<int> ra = inner_radices(a), rb = inner_radices(b);
            const int nfixed = (fixed_shape_id(ra.data(), int(ra.size())) >= 0) +
                               (fixed_shape_id(rb.data(), int(rb.size())) >= 0);
            return std::make_tuple(int(ra.size() + rb.size()), -nfixed);
        };
        auto best = score(Ls[0], Ls[1]);
        // short passes make small tiles: no candidate below 64 points (or the balanced
        // split's shorter pass, if that is shorter)
        const int64_t lmin = std::min<int64_t>(64, std::min(Ls[0], Ls[1]));
        for (int64_t a = lmin; a <= cap; ++a) {
            if (n % a != 0 || n / a > a || n / a < lmin || n / a > cap) continue;
            const int64_t b = n / a;
            const auto sc = score(a, b);
            if (sc < best && pass_fits(cx, a, 2) && pass_fits(cx, b, 2)) {
                best = sc;
                Ls = {a, b};
            }
        }
    }
    return Ls;
}

bool add_chain(Ctx &cx, int64_t n, int64_t S, int64_t O, int A, int B, const int temps[2], std::string &err)
{
    const std::vector<int64_t> Ls = chain_lengths(cx, n, S);
    const int p = int(Ls.size());
    if (p == 0) {
        err = "no pass decomposition for n=" + std::to_string(n);
        return false;
    }
    // buffer sequence: pass 1 reads A; the last pass runs in place on B (its read
    // and write sets coincide); the passes between alternate over the temps
    std::vector<int> seq(p + 1);
    seq[0] = A;
    if (p == 1) {
        seq[1] = B;
    } else if (cx.route_scratch) {
        // chunked plan: every intermediate in (chunk-sized) scratch, which stays in the
        // last-level cache between passes; only the first read and the last write touch
        // the caller's buffers
        for (int i = 1; i < p; ++i) seq[i] = temps[(i - 1) & 1];
        seq[p] = B;
    } else if (p == 2) {
        seq[1] = (A != B) ? B : temps[0];
        seq[2] = B;
    } else {
        for (int i = 1; i < p - 1; ++i) seq[i] = temps[(i - 1) & 1];
        seq[p - 1] = B;
        seq[p] = B;
    }
    int64_t Ns = 1;
    for (int i = 0; i < p; ++i) {
        if (!add_axis_pass(cx, n, S, O, Ls[i], Ns, seq[i], seq[i + 1], err)) return false;
        Ns *= Ls[i];
    }
    return true;
}

Op line_op(int type, int src, int dst)
{
    Op op;
    op.type = type;
    op.src = src;
    op.dst = dst;
    op.la.scale = 1.0;
    op.block = 256;
    return op;
}

void set_lines_axis(LineArgs &la, int64_t n, int64_t S, int64_t O, bool in_side)
{
    // lines of an axis: inner index (stride 1), outer index (stride n*S); element stride S
    la.csz[0] = S;
    la.csz[1] = O;
    la.csz[2] = 1;
    la.csz[3] = 1;
    if (in_side) {
        la.cin[0] = 1;
        la.cin[1] = n * S;
        la.es_in = S;
    } else {
        la.cout[0] = 1;
        la.cout[1] = n * S;
        la.es_out = S;
    }
    la.nlines = S * O;
}

void set_lines_rows(LineArgs &la, int64_t rows, int64_t din, int64_t dout)
{
    la.csz[0] = rows;
    la.csz[1] = la.csz[2] = la.csz[3] = 1;
    la.cin[0] = din;
    la.cout[0] = dout;
    la.es_in = la.es_out = 1;
    la.nlines = rows;
}

int64_t grid_for(int64_t work, int block)
{
    int64_t g = (work + block - 1) / block;
    return std::max<int64_t>(1, std::min<int64_t>(g, 256 * 64));
}

// Padded length of Bluestein's convolution: the next power of two at or above 2n - 1.
// The passes accept any M >= 2n - 1; smaller 2^a 3^b 5^c lengths were measured slower
// (their mixed-radix passes cost more per point than the power-of-two ones save).
int64_t bluestein_m(int64_t n) { return pow2_ceil(2 * n - 1); }

// Bluestein over contiguous lines (inner count 1) with the element-wise steps fused into
// the passes: the first pass of the forward M-point transform builds x_j w_j on its loads
// (PRO_BPAD), the last one multiplies by the filter spectrum and conjugates on its stores
// (EPI_BMUL), and the last pass of the second transform writes w_k conj(.)/M straight into
// the length-n output lines (EPI_BEXT).  Four sweeps of the M-point data instead of seven.
// Returns false (and adds nothing) if a fused pass cannot be tiled.
bool add_bluestein_fused(Ctx &cx, int64_t n, int64_t M, int64_t lines, int A, int B, int t_chirp, int t_filter,
                         std::string &err)
{
    const std::vector<int64_t> Ls = chain_lengths(cx, M, 1);
    const int p = int(Ls.size());
    if (p == 0) return false;
    const size_t mark = cx.sp.ops.size();
    for (int half = 0; half < 2; ++half) {
        // sequence: first buffer, the temps between, last buffer
        const int first = half == 0 ? A : B_S2, last = half == 0 ? B_S2 : B;
        int64_t Ns = 1;
        for (int i = 0; i < p; ++i) {
            const int src = i == 0 ? first : (i - 1) % 2 == 0 ? B_S0 : B_S1;
            const int dst = i == p - 1 ? last : i % 2 == 0 ? B_S0 : B_S1;
            const int pro = (half == 0 && i == 0) ? PRO_BPAD : PRO_PLAIN;
            const int epi = i == p - 1 ? (half == 0 ? EPI_BMUL : EPI_BEXT) : EPI_PLAIN;
            std::string e2;
            if (!add_axis_pass(cx, M, 1, lines, Ls[i], Ns, src, dst, e2, pro, epi)) {
                cx.sp.ops.resize(mark);
                return false;
            }
            Op &op = cx.sp.ops.back();
            op.pa.nreal = n;
            op.pa.bm = M;
            op.pa.brcp = 1.0 / double(M);
            if (pro == PRO_BPAD || epi == EPI_BEXT) op.t_aux = t_chirp;
            if (epi == EPI_BMUL) op.t_aux2 = t_filter;
            if (epi == EPI_BEXT) op.pa.scale = 1.0 / double(M);
            if (half == 0 && i == 0) op.note = "bluestein n=" + std::to_string(n) + " M=" + std::to_string(M);
            Ns *= Ls[i];
        }
    }
    (void)err;
    cx.need_scratch(B_S2, lines * M);
    cx.need_scratch(B, n * lines);
    return true;
}

// c2c transform of length n along an axis (inner S, outer O), from buffer A to B
// (same layout).  Lengths with a prime factor above 7 go through Bluestein.
bool add_c2c_axis(Ctx &cx, int64_t n, int64_t S, int64_t O, int A, int B, std::string &err)
{
    static const int main_temps[2] = {B_S0, B_S1};
    if (is_smooth7(n)) return add_chain(cx, n, S, O, A, B, main_temps, err);

    // Bluestein (chirp-z): X_k = w_k * sum_j (x_j w_j) conj(w_{k-j}), w_j = exp(-pi i j^2/n),
    // the convolution done with length-M FFTs, M >= 2n-1 (no wrap-around aliasing).
    const int64_t M = bluestein_m(n);
    const int64_t lines = S * O;
    TableReq ch{};
    ch.kind = TableReq::CHIRP;
    ch.N = n;
    ch.count = n;
    const int t_chirp = cx.table(ch);
    TableReq bf{};
    bf.kind = TableReq::BFILTER;
    bf.N = n;
    bf.count = M;
    const int t_filter = cx.table(bf);

    if (lines * M >= (int64_t(1) << 32)) {
        err = "Bluestein padded length times lines exceeds 32-bit indexing";
        return false;
    }
    if (S == 1 && add_bluestein_fused(cx, n, M, lines, A, B, t_chirp, t_filter, err)) return true;

    Op pad = line_op(OP_CHIRP_PAD, A, B_S2);
    set_lines_axis(pad.la, n, S, O, true);
    pad.la.cout[0] = M; // destination lines are contiguous, M apart, in line order
    pad.la.cout[1] = S * M;
    pad.la.es_out = 1;
    pad.la.n = n;
    pad.la.M = M;
    pad.t_tab = t_chirp;
    pad.grid = grid_for(lines * M, pad.block);
    pad.note = "bluestein n=" + std::to_string(n) + " M=" + std::to_string(M);
    cx.sp.ops.push_back(pad);
    cx.need_scratch(B_S2, lines * M);

    const int inner_temps[2] = {B_S0, B_S1};
    if (!add_chain(cx, M, 1, lines, B_S2, B_S2, inner_temps, err)) return false;

    Op mul = line_op(OP_MUL_CONJ, B_S2, B_S2);
    set_lines_rows(mul.la, lines, M, M);
    mul.la.n = M;
    mul.la.M = M;
    mul.t_tab2 = t_filter;
    mul.grid = grid_for(lines * M, mul.block);
    cx.sp.ops.push_back(mul);

    if (!add_chain(cx, M, 1, lines, B_S2, B_S2, inner_temps, err)) return false;

    Op ex = line_op(OP_CHIRP_EXTRACT, B_S2, B);
    set_lines_axis(ex.la, n, S, O, false);
    // the source lines are contiguous in S2, M apart, in line order
    ex.la.cin[0] = M;
    ex.la.cin[1] = S * M;
    ex.la.es_in = 1;
    ex.la.n = n;
    ex.la.M = M;
    ex.la.scale = 1.0 / double(M);
    ex.t_tab = t_chirp;
    ex.grid = grid_for(lines * n, ex.block);
    cx.sp.ops.push_back(ex);
    cx.need_scratch(B, n * S * O);
    return true;
}

// ----------------------------------------------------------------------------- real rows

// r2c along the last axis: rows of n reals (distance din reals) -> rows of h+1
// complex (distance dout complex), h = n/2.
bool add_r2c_rows(Ctx &cx, int64_t n, int64_t rows, int A, int B, std::string &err, bool fold_twist = true)
{
    const int64_t h = n / 2;
    if (n % 2 == 0 && is_smooth7(h) && h <= (cx.sp.f64 ? 4096 : 8192)) {
        // fused: the n/2-point transform of z = x[2m] + i x[2m+1], then the twist, one kernel
        Op op;
        op.type = OP_PASS;
        op.src = A;
        op.dst = B;
        op.src_real = 1;
        PassArgs &pa = op.pa;
        pa.L = int32_t(h);
        pa.scale = 1.0;
        pa.pro = PRO_PLAIN;
        pa.epi = EPI_R2C;
        pa.nreal = n;
        set_stages(cx, pa, op);
        pa.csz[0] = rows;
        pa.cin[0] = h;      // complex (z) units
        pa.cout[0] = h + 1; // complex units
        for (int d = 1; d < kColDims; ++d) pa.csz[d] = 1;
        pa.rin = 1;
        pa.rout = 1;
        pa.ncols = rows;
        pa.tw_dim = -1;
        TableReq tw{};
        tw.kind = TableReq::RANGE;
        tw.N = n;
        tw.count = h + 1;
        op.t_aux = cx.table(tw);
        if (!tile_pass(cx, pa)) {
            err = "cannot tile r2c rows";
            return false;
        }
        op.grid = pa.ntiles;
        op.block = pa.threads;
        op.note = "r2c rows n=" + std::to_string(n);
        cx.sp.ops.push_back(op);
        return true;
    }
    if (n % 2 == 0) {
        // staged: c2c on the z view into S3, then the twist kernel
        const size_t first = cx.sp.ops.size();
        if (!add_c2c_axis(cx, h, 1, rows, A, B_S3, err)) return false;
        cx.sp.ops[first].src_real = 1;
        TableReq t{};
        t.kind = TableReq::RANGE;
        t.N = n;
        t.count = h + 1;
        // the twist folded into the last pass when that pass is a specialised kernel over
        // J = csz[0] columns per line (point p of column j is Z_{j + J p}) whose tiles can
        // be paired with their mirrors: the tile holds both bins of every twist pair.  A
        // mirrored tile is two runs of c/2 columns, so it takes twice the columns of a
        // plain one where they fit (each run as long as a plain tile's): 2^20-point float32
        // rows 0.64 -> 0.62 ms, and 0.74 ms with the twist as its own op
        if (fold_twist && std::getenv("MIFFT_TWIST_UNFUSED") == nullptr && cx.sp.ops.size() - first >= 2) {
            Op &last = cx.sp.ops.back();
            PassArgs &la = last.pa;
            const int64_t J = la.csz[0];
            auto foldable = [&]() {
                return last.type == OP_PASS && last.dst == B_S3 && la.shape >= 0 && la.mshape < 0 && la.mode == 0 &&
                       la.pro == PRO_PLAIN && la.epi == EPI_PLAIN && la.scale == 1.0 && !la.conj_out && la.c >= 2 &&
                       J % 2 == 0 && J % la.c == 0 && J * la.L == h && la.cin[0] == 1 && la.cout[0] == 1 &&
                       la.rin == J && la.rout == J &&
                       (la.ncd == 1 || (la.ncd == 2 && la.cin[1] == h && la.cout[1] == h));
            };
            if (foldable()) {
                const PassArgs plain = la;
                cx.force_c = 2 * int64_t(la.c);
                const bool wide = tile_pass(cx, la);
                cx.force_c = 0;
                if (!wide || !foldable()) la = plain;
                last.grid = la.ntiles;
                last.block = la.threads;
                last.dst = B;
                la.epi = EPI_RTWIST;
                la.nreal = n;
                la.bm = h + 1;
                last.t_aux = cx.table(t);
                last.note += ", r2c twist in the stores";
                return true;
            }
        }
        cx.need_scratch(B_S3, rows * h);
        Op tw = line_op(OP_R2C_TWIST, B_S3, B);
        set_lines_rows(tw.la, rows, h, h + 1);
        tw.la.n = n;
        tw.t_tab = cx.table(t);
        tw.grid = grid_for(rows * (h + 1), tw.block);
        cx.sp.ops.push_back(tw);
        return true;
    }
    // odd n: full complex transform of x + 0i, keep k <= n/2
    Op ex = line_op(OP_REAL_TO_CPLX, A, B_S3);
    ex.src_real = 1;
    set_lines_rows(ex.la, rows, n, n);
    ex.la.n = n;
    ex.grid = grid_for(rows * n, ex.block);
    cx.sp.ops.push_back(ex);
    cx.need_scratch(B_S3, rows * n);
    if (!add_c2c_axis(cx, n, 1, rows, B_S3, B_S3, err)) return false;
    Op hc = line_op(OP_HALF_COPY, B_S3, B);
    set_lines_rows(hc.la, rows, n, h + 1);
    hc.la.n = n;
    hc.grid = grid_for(rows * (h + 1), hc.block);
    cx.sp.ops.push_back(hc);
    return true;
}

// c2r along the last axis: rows of h+1 complex (distance din) -> rows of n reals.
bool add_c2r_rows(Ctx &cx, int64_t n, int64_t rows, int A, int B, std::string &err, bool fold_untwist = true)
{
    const int64_t h = n / 2;
    if (n % 2 == 0 && is_smooth7(h) && h <= (cx.sp.f64 ? 4096 : 8192)) {
        Op op;
        op.type = OP_PASS;
        op.src = A;
        op.dst = B;
        op.dst_real = 1;
        PassArgs &pa = op.pa;
        pa.L = int32_t(h);
        pa.scale = 1.0;
        pa.pro = PRO_C2R;
        pa.epi = EPI_PLAIN;
        pa.nreal = n;
        set_stages(cx, pa, op);
        pa.csz[0] = rows;
        pa.cin[0] = h + 1;
        pa.cout[0] = h;
        for (int d = 1; d < kColDims; ++d) pa.csz[d] = 1;
        pa.rin = 1;
        pa.rout = 1;
        pa.ncols = rows;
        pa.tw_dim = -1;
        TableReq tw{};
        tw.kind = TableReq::RANGE;
        tw.N = n;
        tw.count = h + 1;
        op.t_aux = cx.table(tw);
        if (!tile_pass(cx, pa)) {
            err = "cannot tile c2r rows";
            return false;
        }
        op.grid = pa.ntiles;
        op.block = pa.threads;
        op.note = "c2r rows n=" + std::to_string(n);
        cx.sp.ops.push_back(op);
        return true;
    }
    if (n % 2 == 0) {
        Op un = line_op(OP_C2R_UNTWIST, A, B_S3);
        set_lines_rows(un.la, rows, h + 1, h);
        un.la.n = n;
        TableReq t{};
        t.kind = TableReq::RANGE;
        t.N = n;
        t.count = h + 1;
        un.t_tab = cx.table(t);
        un.grid = grid_for(rows * h, un.block);
        cx.sp.ops.push_back(un);
        cx.need_scratch(B_S3, rows * h);
        const size_t at = cx.sp.ops.size();
        if (!add_c2c_axis(cx, h, 1, rows, B_S3, B, err)) return false;
        for (size_t i = at; i < cx.sp.ops.size(); ++i)
            if (cx.sp.ops[i].dst == B) cx.sp.ops[i].dst_real = 1;
        for (size_t i = at; i < cx.sp.ops.size(); ++i)
            if (cx.sp.ops[i].src == B) cx.sp.ops[i].src_real = 1;
        // the untwist folded into the chain's first pass when that pass is a specialised
        // kernel over J = csz[0] columns per line whose tiles can hold their mirrors (the
        // same pairing as the r2c twist in the last pass): the bins go straight from the
        // input into LDS and the untwisted spectrum never reaches HBM
        Op &fp = cx.sp.ops[at];
        PassArgs &fa = fp.pa;
        const int64_t J = fa.csz[0];
        if (fold_untwist && std::getenv("MIFFT_TWIST_UNFUSED") == nullptr && cx.sp.ops.size() - at >= 2 &&
            fp.type == OP_PASS &&
            fp.src == B_S3 && fa.shape >= 0 && fa.mshape < 0 && fa.mode == 0 && fa.pro == PRO_PLAIN &&
            fa.tw_dim < 0 && fa.c >= 2 && J % 2 == 0 && J % fa.c == 0 && J * fa.L == h && fa.L % 2 == 0 &&
            fa.cin[0] == 1 && fa.rin == J && (fa.ncd == 1 || (fa.ncd == 2 && fa.cin[1] == h))) {
            fp.src = A;
            fa.pro = PRO_CUNTWIST;
            fa.nreal = n;
            fa.cin[1] = h + 1;
            fp.t_aux = un.t_tab;
            fp.note += ", c2r untwist in the loads";
            cx.sp.ops.erase(cx.sp.ops.begin() + int64_t(at) - 1);
        }
        return true;
    }
    Op he = line_op(OP_HERM_EXPAND, A, B_S3);
    set_lines_rows(he.la, rows, h + 1, n);
    he.la.n = n;
    he.grid = grid_for(rows * n, he.block);
    cx.sp.ops.push_back(he);
    cx.need_scratch(B_S3, rows * n);
    if (!add_c2c_axis(cx, n, 1, rows, B_S3, B_S3, err)) return false;
    Op cr = line_op(OP_CPLX_TO_REAL, B_S3, B);
    cr.dst_real = 1;
    set_lines_rows(cr.la, rows, n, n);
    cr.la.n = n;
    cr.grid = grid_for(rows * n, cr.block);
    cx.sp.ops.push_back(cr);
    return true;
}

} // namespace

// ----------------------------------------------------------------------------- public helpers

int fixed_shape_id(const int *radices, int nst)
{
    struct Shape {
        int n;
        int r[kMaxStages];
    };
#define MIFFT_SHAPE_ROW(...) {int(sizeof((int[]){__VA_ARGS__}) / sizeof(int)), {__VA_ARGS__}},
    static const Shape table[] = {MIFFT_FIXED_SHAPES(MIFFT_SHAPE_ROW)};
#undef MIFFT_SHAPE_ROW
    const int count = int(sizeof(table) / sizeof(table[0]));
    for (int i = 0; i < count; ++i) {
        if (table[i].n != nst) continue;
        bool eq = true;
        for (int s = 0; s < nst; ++s) eq = eq && table[i].r[s] == radices[s];
        if (eq) return i;
    }
    return -1;
}

int mfma_shape_id(const int *radices, int nst)
{
    struct Shape {
        int n;
        int r[kMaxStages];
    };
#define MIFFT_SHAPE_ROW(...) {int(sizeof((int[]){__VA_ARGS__}) / sizeof(int)), {__VA_ARGS__}},
    static const Shape table[] = {MIFFT_MFMA_SHAPES(MIFFT_SHAPE_ROW)};
#undef MIFFT_SHAPE_ROW
    const int count = int(sizeof(table) / sizeof(table[0]));
    for (int i = 0; i < count; ++i) {
        if (table[i].n != nst) continue;
        bool eq = true;
        for (int s = 0; s < nst; ++s) eq = eq && table[i].r[s] == radices[s];
        if (eq) return i;
    }
    return -1;
}

std::vector<int> inner_radices16(int64_t L)
{
    // as many radix-16 stages as possible (the matrix-core stages), then the odd radices
    std::vector<int> r = base_radices(L);
    if (r.empty() || (r.size() == 1 && r[0] == 1)) return r;
    int64_t m = L;
    int a2 = 0;
    while (m % 2 == 0) {
        m /= 2;
        ++a2;
    }
    std::vector<int> out;
    for (int i = 0; i < a2 / 4; ++i) out.push_back(16);
    if (a2 % 4) out.push_back(1 << (a2 % 4));
    for (int x : r)
        if (x % 2 != 0) out.push_back(x);
    return out;
}

const char *op_name(int type)
{
    static const char *names[OP_NTYPES] = {"pass",       "chirp_pad",  "mul_conj",    "chirp_extract",
                                           "r2c_twist",  "c2r_untwist", "real_to_cplx", "half_copy",
                                           "herm_expand", "cplx_to_real", "dct2_pre",   "dct2_post",
                                           "dct3_pre",   "dct3_post",  "dct2_twpost", "dct3_preuntwist"};
    return (type >= 0 && type < OP_NTYPES) ? names[type] : "?";
}

std::string TableReq::key() const
{
    std::ostringstream o;
    o << int(kind) << ':' << N << ':' << e0 << ':' << step << ':' << count;
    if (kind == INNER)
        for (int s = 0; s < nst; ++s) o << ':' << st[s].r;
    return o.str();
}

bool is_smooth7(int64_t n)
{
    if (n < 1) return false;
    for (int p : {2, 3, 5, 7})
        while (n % p == 0) n /= p;
    return n == 1;
}

// Fewest-stage decomposition of a 7-smooth L using the composite radices 6, 10, 12, 14
// and 15 (prime-factor butterflies) besides 2..16: each composite absorbs two primes in
// one stage.  Ties keep the fewest composites.  Radices in descending order.
std::vector<int> composite_radices(int64_t L)
{
    int e[8] = {0};
    int64_t m = L;
    for (int p : {2, 3, 5, 7})
        while (m % p == 0) {
            m /= p;
            e[p]++;
        }
    if (m != 1 || L <= 1) return {};
    int best = 1 << 30, best_comp = 0, pick[5] = {0, 0, 0, 0, 0}; // 14, 15, 10, 12, 6
    for (int n14 = 0; n14 <= std::min(e[7], e[2]); ++n14)
        for (int n15 = 0; n15 <= std::min(e[5], e[3]); ++n15)
            for (int n10 = 0; n10 <= std::min(e[5] - n15, e[2] - n14); ++n10)
                for (int n12 = 0; n12 <= std::min(e[3] - n15, (e[2] - n14 - n10) / 2); ++n12)
                    for (int n6 = 0; n6 <= std::min(e[3] - n15 - n12, e[2] - n14 - n10 - 2 * n12); ++n6) {
                        const int r2 = e[2] - n14 - n10 - 2 * n12 - n6, r3 = e[3] - n15 - n12 - n6;
                        const int r5 = e[5] - n15 - n10, r7 = e[7] - n14;
                        const int comp = n14 + n15 + n10 + n12 + n6;
                        const int st = comp + r7 + r5 + (r3 + 1) / 2 + (r2 + 3) / 4;
                        if (st < best || (st == best && comp < best_comp)) {
                            best = st;
                            best_comp = comp;
                            pick[0] = n14, pick[1] = n15, pick[2] = n10, pick[3] = n12, pick[4] = n6;
                        }
                    }
    std::vector<int> r;
    const int comps[5] = {14, 15, 10, 12, 6};
    for (int i = 0; i < 5; ++i)
        for (int k = 0; k < pick[i]; ++k) r.push_back(comps[i]);
    const int r2 = e[2] - pick[0] - pick[2] - 2 * pick[3] - pick[4], r3 = e[3] - pick[1] - pick[3] - pick[4];
    const int r5 = e[5] - pick[1] - pick[2], r7 = e[7] - pick[0];
    if (r2 > 0) {
        const int s = (r2 + 3) / 4, base = r2 / s, extra = r2 % s;
        for (int i = 0; i < s; ++i) r.push_back(1 << (base + (i < extra ? 1 : 0)));
    }
    for (int i = 0; i < r3 / 2; ++i) r.push_back(9);
    if (r3 % 2) r.push_back(3);
    for (int i = 0; i < r5; ++i) r.push_back(5);
    for (int i = 0; i < r7; ++i) r.push_back(7);
    std::sort(r.rbegin(), r.rend());
    return r;
}

// Decomposition with the base radices only (powers of two spread over <= 16, 9/3, 5, 7).
std::vector<int> base_radices(int64_t L)
{
    std::vector<int> r;
    if (L <= 1) {
        r.push_back(1);
        return r;
    }
    int a[8] = {0};
    int64_t m = L;
    for (int p : {2, 3, 5, 7})
        while (m % p == 0) {
            m /= p;
            a[p]++;
        }
    if (m != 1) return {}; // not 7-smooth: no in-workgroup decomposition
    // powers of two: the fewest stages of at most 16, bits spread evenly
    if (a[2] > 0) {
        const int s = (a[2] + 3) / 4;
        const int base = a[2] / s, extra = a[2] % s;
        for (int i = 0; i < s; ++i) r.push_back(1 << (base + (i < extra ? 1 : 0)));
    }
    for (int i = 0; i < a[3] / 2; ++i) r.push_back(9);
    if (a[3] % 2) r.push_back(3);
    for (int i = 0; i < a[5]; ++i) r.push_back(5);
    for (int i = 0; i < a[7]; ++i) r.push_back(7);
    return r;
}

std::vector<int> inner_radices(int64_t L)
{
    // a specialised kernel keeps its sequence; otherwise fewer stages win
    std::vector<int> r = base_radices(L);
    if (r.empty() || fixed_shape_id(r.data(), int(r.size())) >= 0) return r;
    std::vector<int> c = composite_radices(L);
    return (!c.empty() && c.size() < r.size()) ? c : r;
}

std::vector<int64_t> pass_lengths(int64_t n, int64_t max_len)
{
    if (n <= max_len) return {n};
    std::vector<int64_t> f = prime_factors(n);
    std::sort(f.rbegin(), f.rend());
    for (int p = 2; p <= 8; ++p) {
        // longest-processing-time assignment of the prime factors to p groups
        std::vector<int64_t> g(p, 1);
        for (int64_t q : f) {
            auto it = std::min_element(g.begin(), g.end());
            *it *= q;
        }
        bool ok = true;
        for (int64_t x : g) ok = ok && x <= max_len;
        if (ok) {
            std::sort(g.rbegin(), g.rend());
            return g;
        }
    }
    return {};
}

std::string PlanSpec::describe() const
{
    static const char *bn[B_NBUF] = {"in", "out", "s0", "s1", "s2", "s3", "s4"};
    std::ostringstream o;
    o << "mifft plan rank=" << rank << " dims=";
    for (int a = 0; a < rank; ++a) o << (a ? "x" : "") << dims[a];
    static const char *kinds[5] = {"c2c", "r2c", "c2r", "dct2", "dct3"};
    o << " batch=" << batch << " kind=" << kinds[kind >= 0 && kind < 5 ? kind : 0]
      << " dir=" << (direction < 0 ? "fwd" : "inv") << " dtype=" << dtype << "\n";
    if (chunk > 0)
        o << "  chunks of " << chunk << " transforms (" << (batch + chunk - 1) / chunk << " chunks"
          << (batch % chunk ? ", the last of " + std::to_string(batch % chunk) : std::string()) << ")\n";
    auto list = [&](const std::vector<Op> &v) {
        for (size_t i = 0; i < v.size(); ++i) {
            const Op &op = v[i];
            o << "  op" << i << " " << op_name(op.type) << " " << bn[op.src] << "->" << bn[op.dst] << " ";
            if (op.type == OP_PASS)
                o << fmt_pass(op.pa) << " lp=" << op.pa.lp << " key=" << pass_key(*this, op.pa);
            else
                o << "lines=" << op.la.nlines << " n=" << op.la.n << " M=" << op.la.M;
            o << " grid=" << op.grid << " block=" << op.block;
            if (!op.note.empty()) o << " [" << op.note << "]";
            o << "\n";
        }
    };
    list(ops);
    if (!ops_inplace.empty()) {
        o << "  in place (in == out):\n";
        list(ops_inplace);
    }
    if (!tail_ops.empty()) {
        o << "  last chunk:\n";
        list(tail_ops);
    }
    if (!tail_ops_inplace.empty()) {
        o << "  last chunk in place:\n";
        list(tail_ops_inplace);
    }
    o << "  tables=" << tables.size() << " table_bytes=" << table_elems * (f64 ? 16 : 8);
    for (int b = B_S0; b < B_NBUF; ++b)
        if (scratch_elems[b]) o << " " << bn[b] << "_bytes=" << scratch_elems[b] * (f64 ? 16 : 8);
    o << "\n";
    return o.str();
}

namespace {
// The op lists (out of place, and in place for c2c) of `batch` transforms of the plan's
// shape, appended to the context's spec; tables and scratch sizes accumulate in it.
int plan_ops(Ctx &cx, int64_t batch, std::string &err)
{
    PlanSpec &sp = cx.sp;
    const int rank = sp.rank, kind = sp.kind, direction = sp.direction;
    const int64_t *dims = sp.dims;
    int64_t per = 1;
    for (int a = 0; a < rank; ++a) per *= dims[a];
    const int64_t n_last = dims[rank - 1];
    const int64_t h = n_last / 2 + 1;
    const int64_t half_per = per / n_last * h;
    bool ok = true;

    if (kind == 0) {
        // contiguous axis first (reads the input, writes the output), then the others in
        // place.  A second list serves in == out: there the first axis starts from the
        // output buffer, so a multi-pass chain routes its first pass through scratch.
        for (int variant = 0; variant < (sp.ragged ? 1 : 2) && ok; ++variant) {
            std::vector<Op> saved;
            if (variant == 1) saved.swap(sp.ops);
            for (int a = rank - 1; a >= 0 && ok; --a) {
                int64_t S = 1, O = batch;
                for (int b = a + 1; b < rank; ++b) S *= dims[b];
                for (int b = 0; b < a; ++b) O *= dims[b];
                const int src = (a == rank - 1 && variant == 0) ? B_IN : B_OUT;
                if (dims[a] == 1 && a != rank - 1) continue;
                ok = add_c2c_axis(cx, dims[a], S, O, src, B_OUT, err);
            }
            if (variant == 1) {
                // identical buffer use apart from in/out naming: the plain list is already safe
                bool same = saved.size() == sp.ops.size();
                for (size_t i = 0; same && i < saved.size(); ++i)
                    same = (saved[i].src == B_IN ? B_OUT : saved[i].src) == sp.ops[i].src &&
                           saved[i].dst == sp.ops[i].dst;
                if (!same) sp.ops_inplace.swap(sp.ops);
                sp.ops.swap(saved);
            }
        }
    } else if (kind >= 3) {
        // DCT-II / DCT-III through one n-point real transform (Makhoul's reordering).
        // Type 2 reorders the reals into `out`, takes their half spectrum with the r2c
        // rows plan into S4 and rotates it into `out`; type 3 runs those steps inverted.
        const int64_t n = dims[0];
        const int64_t hb = n / 2 + 1; // half-spectrum bins
        TableReq tw{};
        tw.kind = TableReq::RANGE;
        tw.N = 4 * n;
        tw.e0 = 0;
        tw.step = 1;
        tw.count = n;
        const int t_w = cx.table(tw);
        if (kind == 3) {
            Op pre = line_op(OP_DCT2_PRE, B_IN, B_OUT);
            pre.src_real = pre.dst_real = 1;
            set_lines_rows(pre.la, batch, n, n);
            pre.la.n = n;
            pre.grid = grid_for(batch * n, pre.block);
            pre.note = "dct2 n=" + std::to_string(n);
            const size_t ipre = cx.sp.ops.size();
            cx.sp.ops.push_back(pre);
            // the rotation rides with the twist in the last pass's stores in float32 (2^20-point
            // rows 0.835 -> 0.82 ms); in float64 its 8-byte scattered reals made that pass
            // slower than the separate twist-and-rotation op (0.91 -> 1.03 ms), which it keeps
            ok = add_r2c_rows(cx, n, batch, B_OUT, B_S4, err, !cx.sp.f64);
            const bool folded = ok && cx.sp.ops.back().type == OP_PASS && cx.sp.ops.back().pa.epi == EPI_RTWIST;
            if (ok && (folded || cx.sp.ops.back().type == OP_R2C_TWIST)) {
                // staged real transform: when its first pass is a specialised kernel whose
                // columns run within a line (then over the lines), that pass reads the
                // reordered samples straight from the input (PRO_DCT2) and the reordering
                // op goes
                Op &first = cx.sp.ops[ipre + 1];
                PassArgs &fa = first.pa;
                const int64_t h = n / 2;
                if (first.type == OP_PASS && first.src == B_OUT && fa.pro == PRO_PLAIN && fa.epi == EPI_PLAIN &&
                    fa.shape >= 0 && fa.mode == 0 && fa.tw_dim < 0 && !fa.conj_in && fa.cin[0] == 1 &&
                    (fa.ncd == 1 || (fa.ncd == 2 && fa.cin[1] == h)) && fa.csz[0] * fa.L == h &&
                    fa.rin == fa.csz[0] && std::getenv("MIFFT_DCT2_UNFUSED") == nullptr) {
                    first.src = B_IN;
                    fa.pro = PRO_DCT2;
                    fa.nreal = n;
                    first.note = "dct2 n=" + std::to_string(n) + ", reordering in the loads";
                    cx.sp.ops.erase(cx.sp.ops.begin() + int64_t(ipre));
                }
                if (folded) {
                    // the twist already rides in the last pass's stores: the rotation joins it
                    Op &last = cx.sp.ops.back();
                    last.dst = B_OUT;
                    last.dst_real = 1;
                    last.pa.epi = EPI_DTWIST;
                    last.pa.bm = n;
                    last.t_aux2 = t_w;
                    last.note += " with the DCT-II rotation";
                } else {
                    // its twist and the rotation become one pass over the n/2-point spectrum
                    // (no half spectrum written and read back)
                    Op tw = cx.sp.ops.back();
                    cx.sp.ops.pop_back();
                    Op tp = line_op(OP_DCT2_TWPOST, tw.src, B_OUT);
                    tp.dst_real = 1;
                    set_lines_rows(tp.la, batch, n / 2, n);
                    tp.la.n = n;
                    tp.t_tab = t_w;      // W_4n^k, k < n
                    tp.t_tab2 = tw.t_tab; // W_n^k, k <= n/2
                    tp.grid = grid_for(batch * (n / 4 + 1), tp.block);
                    cx.sp.ops.push_back(tp);
                }
            } else {
                cx.need_scratch(B_S4, hb * batch);
                Op post = line_op(OP_DCT2_POST, B_S4, B_OUT);
                post.dst_real = 1;
                set_lines_rows(post.la, batch, hb, n);
                post.la.n = n;
                post.t_tab = t_w;
                post.grid = grid_for(batch * n, post.block);
                cx.sp.ops.push_back(post);
            }
        } else {
            // rotate into a half spectrum in S2 (the c2r plan consumes its input in its
            // first op, before anything of its own touches S2), take its unnormalised
            // real inverse into S4, undo the reordering into `out`
            Op pre = line_op(OP_DCT3_PRE, B_IN, B_S2);
            pre.src_real = 1;
            set_lines_rows(pre.la, batch, n, hb);
            pre.la.n = n;
            pre.t_tab = t_w;
            pre.grid = grid_for(batch * hb, pre.block);
            pre.note = "dct3 n=" + std::to_string(n);
            cx.sp.ops.push_back(pre);
            const size_t c0 = cx.sp.ops.size();
            // DCT-III keeps the untwist as an op: it fuses with the rotation there, and the
            // last pass then takes the inverse reordering
            ok = add_c2r_rows(cx, n, batch, B_S2, B_S4, err, false);
            if (ok) {
                // the c2r steps run a forward transform of the conjugate and conjugate
                // the result (as an inverse plan's first and last ops do), without 1/n
                Op &f = cx.sp.ops[c0];
                if (f.type == OP_PASS) f.pa.conj_in = 1; else f.la.conj_in = 1;
                Op &l = cx.sp.ops.back();
                if (l.type == OP_PASS) l.pa.conj_out = 1; else l.la.conj_out = 1;
                if (cx.sp.ops[c0].type == OP_C2R_UNTWIST) {
                    // staged real inverse: the rotation and the untwist become one pass that
                    // reads the input reals and writes the z spectrum (no half spectrum
                    // written and read back)
                    const Op un = cx.sp.ops[c0];
                    Op pu = line_op(OP_DCT3_PREUNTWIST, B_IN, un.dst);
                    pu.src_real = 1;
                    set_lines_rows(pu.la, batch, n, n / 2);
                    pu.la.n = n;
                    pu.t_tab = t_w;        // W_4n^k, k < n
                    pu.t_tab2 = un.t_tab;  // W_n^k, k <= n/2
                    pu.grid = grid_for(batch * (n / 4 + 1), pu.block);
                    pu.note = "dct3 n=" + std::to_string(n);
                    cx.sp.ops.erase(cx.sp.ops.begin() + int64_t(c0) - 1, cx.sp.ops.begin() + int64_t(c0) + 1);
                    cx.sp.ops.insert(cx.sp.ops.begin() + int64_t(c0) - 1, pu);
                } else {
                    cx.need_scratch(B_S2, hb * batch); // the half spectrum the c2r plan reads
                }
            }
            // staged real inverse whose last pass is a specialised kernel with columns within
            // a line (then over the lines): that pass stores each point's two reals straight
            // to their natural positions in `out` (EPI_DCT3) and the reordering op goes
            bool fused = false;
            if (ok && cx.sp.ops[c0 - 1].type == OP_DCT3_PREUNTWIST) {
                Op &last = cx.sp.ops.back();
                PassArgs &la = last.pa;
                const int64_t hh = n / 2;
                if (last.type == OP_PASS && last.dst == B_S4 && la.epi == EPI_PLAIN && la.pro == PRO_PLAIN &&
                    la.shape >= 0 && la.mode == 0 && la.cout[0] == 1 &&
                    (la.ncd == 1 || (la.ncd == 2 && la.cout[1] == hh)) && la.csz[0] * la.L == hh &&
                    la.rout == la.csz[0] && std::getenv("MIFFT_DCT3_UNFUSED") == nullptr) {
                    last.dst = B_OUT;
                    last.dst_real = 1;
                    la.epi = EPI_DCT3;
                    la.nreal = n;
                    last.note = "dct3 n=" + std::to_string(n) + ", reordering in the stores";
                    fused = true;
                }
            }
            if (!fused) {
                cx.need_scratch(B_S4, n * batch); // n reals per line (complex units: room to spare)
                Op post = line_op(OP_DCT3_POST, B_S4, B_OUT);
                post.src_real = post.dst_real = 1;
                set_lines_rows(post.la, batch, n, n);
                post.la.n = n;
                post.grid = grid_for(batch * n, post.block);
                cx.sp.ops.push_back(post);
            }
        }
    } else if (kind == 1) {
        const int64_t rows = batch * (per / n_last);
        ok = add_r2c_rows(cx, n_last, rows, B_IN, B_OUT, err);
        int64_t hd[3];
        for (int a = 0; a < rank; ++a) hd[a] = dims[a];
        hd[rank - 1] = h;
        for (int a = rank - 2; a >= 0 && ok; --a) {
            int64_t S = 1, O = batch;
            for (int b = a + 1; b < rank; ++b) S *= hd[b];
            for (int b = 0; b < a; ++b) O *= hd[b];
            if (hd[a] == 1) continue;
            ok = add_c2c_axis(cx, hd[a], S, O, B_OUT, B_OUT, err);
        }
    } else {
        const int64_t rows = batch * (per / n_last);
        int64_t hd[3];
        for (int a = 0; a < rank; ++a) hd[a] = dims[a];
        hd[rank - 1] = h;
        // leading axes first, on the half spectrum: the input stays untouched, so the
        // first of them writes a staging copy (S4) and the rest work in place there
        int src = B_IN;
        for (int a = rank - 2; a >= 0 && ok; --a) {
            int64_t S = 1, O = batch;
            for (int b = a + 1; b < rank; ++b) S *= hd[b];
            for (int b = 0; b < a; ++b) O *= hd[b];
            if (hd[a] == 1) continue;
            ok = add_c2c_axis(cx, hd[a], S, O, src, B_S4, err);
            src = B_S4;
        }
        if (src == B_S4) cx.need_scratch(B_S4, half_per * batch);
        if (ok) ok = add_c2r_rows(cx, n_last, rows, src, B_OUT, err);
    }
    if (!ok) return kUnsupported;
    if (sp.ops.empty()) {
        err = "internal: empty plan";
        return kUnsupported;
    }
    // inverse: conjugate on the first load and the last store, scale once at the end
    if (direction == 1) {
        for (std::vector<Op> *list : {&sp.ops, &sp.ops_inplace}) {
            if (list->empty()) continue;
            Op &f = list->front();
            Op &l = list->back();
            if (f.type == OP_PASS) f.pa.conj_in = 1; else f.la.conj_in = 1;
            if (l.type == OP_PASS) {
                l.pa.conj_out = 1;
                l.pa.scale *= 1.0 / double(per);
            } else {
                l.la.conj_out = 1;
                l.la.scale *= 1.0 / double(per);
            }
        }
    }
    return kOK;
}

// Transforms per chunk when the batch runs in chunks (0: one chunk).  A plan of more
// than one op (its intermediates pass through the output or plan-owned scratch) runs
// its batch in chunks of about kChunkBytes of input (or the size the tuning table's
// chunk entry names), so that each intermediate is chunk-sized and still in the
// last-level cache (MALL) when the next op reads it, and the plan's scratch stays
// bounded.  MIFFT_CHUNK_BYTES overrides the size (0 disables chunking).
int64_t chunk_transforms(const PlanSpec &sp, int64_t batch, int64_t in_bytes_per_transform)
{
    if (sp.ragged || batch < 2 || sp.ops.size() < 2) return 0;
    int64_t target = kChunkBytes;
    Tune t;
    if (find_tune(chunk_key(sp), t) && t.b >= 0) target = t.b;
    if (const char *e = std::getenv("MIFFT_CHUNK_BYTES")) target = std::atoll(e);
    if (sp.chunk_target >= 0) target = sp.chunk_target;
    if (target <= 0) return 0;
    // as many chunks as the target size asks for, the transforms spread evenly over them
    const double total = double(batch) * double(in_bytes_per_transform);
    const int64_t nch = std::min<int64_t>(batch, int64_t(std::ceil(total / double(target))));
    if (nch < 2) return 0;
    return (batch + nch - 1) / nch;
}

} // namespace

int build_plan(int rank, const int64_t *dims, int64_t batch, int kind, int direction, int dtype,
               PlanSpec &sp, std::string &err)
{
    // MIFFT_GENERIC_ONLY=1 sends every pass to the runtime-radix kernel (for testing it
    // on shapes that normally have specialised kernels)
    const char *go = std::getenv("MIFFT_GENERIC_ONLY");
    const bool generic_only = sp.generic_only || (go && go[0] == '1'), ragged = sp.ragged;
    const int64_t chunk_target = sp.chunk_target;
    sp = PlanSpec();
    sp.generic_only = generic_only;
    sp.ragged = ragged;
    sp.chunk_target = chunk_target;
    if (rank < 1 || rank > 3 || !dims) {
        err = "rank must be 1, 2 or 3 and dims non-NULL";
        return kInvalid;
    }
    if (batch < 1) {
        err = "batch must be >= 1";
        return kInvalid;
    }
    for (int a = 0; a < rank; ++a)
        if (dims[a] < 1) {
            err = "every dim must be >= 1";
            return kInvalid;
        }
    if (kind < 0 || kind > 4) {
        err = "kind must be FFT_C2C, FFT_R2C, FFT_C2R, FFT_DCT2 or FFT_DCT3";
        return kInvalid;
    }
    if (kind >= 3 && (direction != -1 || rank != 1)) {
        err = "FFT_DCT2 / FFT_DCT3 are rank-1 transforms planned with FFT_FORWARD";
        return kInvalid;
    }
    if (direction != -1 && direction != 1) {
        err = "direction must be FFT_FORWARD (-1) or FFT_INVERSE (+1)";
        return kInvalid;
    }
    if (dtype < 0 || dtype > 3) {
        err = "dtype must be one of FFT_F32, FFT_F64, FFT_F32_BF16X2, FFT_F32_BF16X3";
        return kInvalid;
    }
    if (kind == 1 && direction != -1) {
        err = "R2C requires FFT_FORWARD";
        return kInvalid;
    }
    if (kind == 2 && direction != 1) {
        err = "C2R requires FFT_INVERSE";
        return kInvalid;
    }
    if (dtype >= 2 && (kind != 0 || rank != 1)) {
        err = "the split-BF16 forms support 1-D C2C only";
        return kUnsupported;
    }
    sp.rank = rank;
    for (int a = 0; a < rank; ++a) sp.dims[a] = dims[a];
    sp.batch = batch;
    sp.kind = kind;
    sp.direction = direction;
    sp.dtype = dtype;
    sp.f64 = dtype == 1;

    int64_t per = 1;
    for (int a = 0; a < rank; ++a) per *= dims[a];
    const int64_t n_last = dims[rank - 1];
    const int64_t h = n_last / 2 + 1;
    const int64_t half_per = per / n_last * h;
    const double lim = 4294967295.0; // 32-bit column/element indexing
    if (double(per) * double(batch) >= lim || double(half_per) * double(batch) >= lim) {
        err = "too many elements in one call (limit 2^32 - 1)";
        return kUnsupported;
    }
    Ctx cx(sp);
    int st = plan_ops(cx, batch, err);
    if (st != kOK) return st;
    sp.in_dist = kind == 2 ? half_per : per;   // elements of the input's type per transform
    sp.out_dist = kind == 1 ? half_per : per;
    sp.in_elems = sp.in_dist * batch;
    sp.out_elems = sp.out_dist * batch;
    const int64_t rb = sp.f64 ? 8 : 4; // bytes per real
    const int64_t chunk = chunk_transforms(sp, batch, sp.in_dist * (kind == 0 || kind == 2 ? 2 * rb : rb));
    if (chunk > 0) {
        // re-plan for a chunk, and for the remainder if the batch is not a multiple of it;
        // the scratch is sized for a chunk (tables are shared: their keys do not depend on
        // the batch)
        sp.ops.clear();
        sp.ops_inplace.clear();
        for (int b = 0; b < B_NBUF; ++b) sp.scratch_elems[b] = 0;
        cx.route_scratch = true;
        const int64_t tail = batch % chunk;
        if (tail > 0) {
            st = plan_ops(cx, tail, err);
            if (st != kOK) return st;
            sp.tail_ops.swap(sp.ops);
            sp.tail_ops_inplace.swap(sp.ops_inplace);
        }
        st = plan_ops(cx, chunk, err);
        if (st != kOK) return st;
        sp.chunk = chunk;
    }
    // a scratch buffer no op names (its last user retargeted, as a fused DCT-III store
    // is) holds no memory
    bool named[B_NBUF] = {};
    for (const std::vector<Op> *list : {&sp.ops, &sp.ops_inplace, &sp.tail_ops, &sp.tail_ops_inplace})
        for (const Op &op : *list) named[op.src] = named[op.dst] = true;
    for (int b = B_S0; b < B_NBUF; ++b)
        if (!named[b]) sp.scratch_elems[b] = 0;
    // every scratch buffer an op names is allocated
    for (const std::vector<Op> *list : {&sp.ops, &sp.ops_inplace, &sp.tail_ops, &sp.tail_ops_inplace})
        for (const Op &op : *list)
            for (int b : {op.src, op.dst})
                if (b >= B_S0 && sp.scratch_elems[b] <= 0) {
                    err = std::string("internal: op ") + op_name(op.type) + " uses scratch buffer " +
                          std::to_string(b - B_S0) + ", which the plan does not size";
                    return kInternal;
                }
    // streamed accesses: the input read by the first pass and the output written by the
    // last are touched once per call (MIFFT_NT=0 turns the hint off)
    const char *nte = std::getenv("MIFFT_NT");
    const bool nt = !(nte && nte[0] == '0');
    for (std::vector<Op> *list : {&sp.ops, &sp.ops_inplace, &sp.tail_ops, &sp.tail_ops_inplace})
        for (size_t i = 0; i < list->size(); ++i) {
            Op &op = (*list)[i];
            if (op.type != OP_PASS) continue;
            op.pa.nt_in = nt && op.src == B_IN;
            op.pa.nt_out = nt && op.dst == B_OUT && i + 1 == list->size();
        }
    return kOK;
}

} // namespace mifft

namespace mifft {

int build_many(int64_t count, const int64_t *lengths, int kind, int direction, int dtype, ManySpec &ms,
               std::string &err)
{
    ms = ManySpec();
    if (count < 1 || !lengths) {
        err = "count must be >= 1 and lengths non-NULL";
        return kInvalid;
    }
    if (kind != 0) {
        err = "ragged plans are complex-to-complex only";
        return kUnsupported;
    }
    if (dtype != 0 && dtype != 1) {
        err = "ragged plans take FFT_F32 or FFT_F64";
        return kUnsupported;
    }
    if (direction != -1 && direction != 1) {
        err = "direction must be FFT_FORWARD (-1) or FFT_INVERSE (+1)";
        return kInvalid;
    }
    ms.f64 = dtype == 1;
    ms.direction = direction;
    ms.dtype = dtype;
    std::map<int64_t, int> cls_of;
    std::map<std::string, int> table_ids;
    ms.xform_class.resize(size_t(count));
    for (int64_t t = 0; t < count; ++t) {
        const int64_t n = lengths[t];
        if (n < 1) {
            err = "every length must be >= 1";
            return kInvalid;
        }
        auto it = cls_of.find(n);
        if (it == cls_of.end()) {
            PlanSpec sp;
            sp.generic_only = true;
            sp.ragged = true;
            const int st = build_plan(1, &n, 1, 0, direction, dtype, sp, err);
            if (st != kOK) return st;
            ManySpec::Class c;
            c.n = n;
            c.first_op = int(ms.ops.size());
            c.nops = int(sp.ops.size());
            int64_t off = 0;
            for (int b = B_S0; b < B_NBUF; ++b) {
                c.sofs[b] = off;
                off += (sp.scratch_elems[b] + 63) / 64 * 64;
            }
            c.scratch = off;
            // tables: merge into the ragged plan's arena, deduplicated by key
            std::vector<int> remap(sp.tables.size());
            for (size_t i = 0; i < sp.tables.size(); ++i) {
                const std::string k = sp.tables[i].key();
                auto f = table_ids.find(k);
                if (f == table_ids.end()) {
                    TableReq tr = sp.tables[i];
                    tr.offset = ms.table_elems;
                    ms.table_elems += (tr.count + 31) / 32 * 32;
                    ms.tables.push_back(tr);
                    f = table_ids.emplace(k, int(ms.tables.size()) - 1).first;
                }
                remap[i] = f->second;
            }
            for (Op op : sp.ops) {
                for (int *id : {&op.t_itw, &op.t_lo, &op.t_hi, &op.t_aux, &op.t_aux2, &op.t_tab, &op.t_tab2})
                    if (*id >= 0) *id = remap[size_t(*id)];
                ms.ops.push_back(op);
            }
            ms.classes.push_back(c);
            it = cls_of.emplace(n, int(ms.classes.size()) - 1).first;
        }
        ms.xform_class[size_t(t)] = it->second;
        ms.classes[size_t(it->second)].count++;
    }
    return kOK;
}

std::string ManySpec::describe() const
{
    std::ostringstream o;
    int64_t total = 0;
    for (const Class &c : classes) total += c.count;
    o << "mifft ragged plan: " << total << " transforms, " << classes.size() << " distinct lengths, "
      << ops.size() << " ops, " << tables.size() << " tables, dir=" << (direction < 0 ? "fwd" : "inv")
      << " dtype=" << dtype << "\n";
    // per-length plans
    static const char *bn[B_NBUF] = {"in", "out", "s0", "s1", "s2", "s3", "s4"};
    {
        for (const Class &c : classes) {
            o << "  n=" << c.n << " count=" << c.count << " scratch=" << c.scratch << "\n";
            for (int k = 0; k < c.nops; ++k) {
                const Op &op = ops[size_t(c.first_op + k)];
                o << "    op" << k << " " << op_name(op.type) << " " << bn[op.src] << "->" << bn[op.dst] << " ";
                if (op.type == OP_PASS)
                    o << fmt_pass(op.pa) << " lp=" << op.pa.lp;
                else
                    o << "lines=" << op.la.nlines << " n=" << op.la.n << " M=" << op.la.M;
                o << "\n";
            }
        }
    }
    return o.str();
}

// Parts of one op of a ragged class: tiles of a pass, chunks of an element-wise op.
static int64_t op_parts(const Op &op)
{
    if (op.type == OP_PASS) return op.pa.ntiles;
    return (line_total(op.type, op.la) + kRagLineChunk - 1) / kRagLineChunk;
}

// Points one part of an op touches (the scheduler's cost unit).
static int64_t part_cost(const Op &op, int64_t part)
{
    if (op.type == OP_PASS) {
        const int64_t col0 = part * op.pa.c;
        return std::min<int64_t>(op.pa.c, op.pa.ncols - col0) * op.pa.L;
    }
    const int64_t total = line_total(op.type, op.la);
    return std::min<int64_t>(kRagLineChunk, total - part * kRagLineChunk);
}

int schedule_many(const ManySpec &ms, RaggedSchedule &rs, std::string &err)
{
    rs = RaggedSchedule();
    const size_t ncls = ms.classes.size();
    int64_t whole_parts = kRagWholeParts;
    int64_t xcd_group = kRagXcdGroup;
    Tune tw;
    if (find_tune("rag:schedule", tw)) {
        if (tw.w > 0) whole_parts = tw.w;
        if (tw.c > 0) xcd_group = tw.c;
    }
    std::vector<char> whole(ncls, 0);
    std::vector<int64_t> wcost(ncls, 0);
    size_t nph = 1;
    for (size_t c = 0; c < ncls; ++c) {
        const ManySpec::Class &cl = ms.classes[c];
        int64_t parts = 0;
        for (int o = 0; o < cl.nops; ++o) {
            const Op &op = ms.ops[size_t(cl.first_op + o)];
            const int64_t np = op_parts(op);
            parts += np;
            for (int64_t j = 0; j < np; ++j) wcost[c] += part_cost(op, j);
        }
        whole[c] = parts <= whole_parts;
        if (!whole[c]) nph = std::max(nph, size_t(cl.nops));
    }
    struct Item {
        RaggedSchedule::Block b;
        int64_t cost;
    };
    std::vector<std::vector<Item>> ph(nph);
    std::vector<int64_t> load(nph, 0);
    std::vector<uint32_t> wholes;
    const int64_t count = int64_t(ms.xform_class.size());
    for (int64_t t = 0; t < count; ++t) {
        const size_t c = size_t(ms.xform_class[size_t(t)]);
        const ManySpec::Class &cl = ms.classes[c];
        if (whole[c]) {
            wholes.push_back(uint32_t(t));
            ++rs.whole_transforms;
            continue;
        }
        ++rs.split_transforms;
        for (int o = 0; o < cl.nops; ++o) {
            const Op &op = ms.ops[size_t(cl.first_op + o)];
            const int64_t np = op_parts(op);
            for (int64_t j = 0; j < np; ++j) {
                const int64_t w = part_cost(op, j);
                ph[size_t(o)].push_back(Item{{uint32_t(t), uint32_t(o), uint32_t(j), 0u}, w});
                load[size_t(o)] += w;
            }
        }
    }
    std::stable_sort(wholes.begin(), wholes.end(), [&](uint32_t a, uint32_t b) {
        return wcost[size_t(ms.xform_class[a])] > wcost[size_t(ms.xform_class[b])];
    });
    for (uint32_t t : wholes) {
        const size_t k = size_t(std::min_element(load.begin(), load.end()) - load.begin());
        const int64_t w = wcost[size_t(ms.xform_class[t])];
        ph[k].push_back(Item{{t, 0u, 0u, 1u}, w});
        load[k] += w;
    }
    for (size_t k = 0; k < nph; ++k) {
        std::stable_sort(ph[k].begin(), ph[k].end(), [](const Item &a, const Item &b) { return a.cost > b.cost; });
        if (ph[k].empty()) continue;
        if (ph[k].size() > size_t(0x7fffffff)) {
            err = "too many blocks in one phase";
            return kUnsupported;
        }
        rs.phase_first.push_back(uint32_t(rs.blocks.size()));
        rs.phase_blocks.push_back(uint32_t(ph[k].size()));
        // The hardware deals a launch's workgroups round-robin over the XCDs.  Within
        // each window of kXcds x group positions, give every XCD a run of `group`
        // consecutive items: neighbouring parts of one op (which share cache lines at
        // their edges, all the more so at the unaligned offsets of a packed ragged
        // buffer) then meet in one L2, while the window keeps the cost order.
        const size_t nk = ph[k].size(), win = size_t(kXcds) * size_t(xcd_group);
        for (size_t w0 = 0; w0 < nk; w0 += win) {
            const uint32_t m = uint32_t(std::min(win, nk - w0));
            const uint32_t q = m / kXcds, rem = m % kXcds;
            for (uint32_t p = 0; p < m; ++p) {
                const uint32_t x = p % kXcds, sl = p / kXcds;
                rs.blocks.push_back(ph[k][w0 + x * q + std::min(x, rem) + sl].b);
            }
        }
    }
    // every part of every op of a split transform exactly once, in the phase of its
    // op; every whole transform exactly once
    std::vector<int64_t> seen(size_t(count), 0);
    for (size_t k = 0; k < rs.phase_first.size(); ++k)
        for (uint32_t i = 0; i < rs.phase_blocks[k]; ++i) {
            const RaggedSchedule::Block &b = rs.blocks[rs.phase_first[k] + i];
            if (b.t >= uint64_t(count) || (!b.whole && b.op != k)) {
                err = "internal: ragged schedule out of order";
                return kInternal;
            }
            seen[b.t] += b.whole ? -1 : 1;
        }
    for (int64_t t = 0; t < count; ++t) {
        const size_t c = size_t(ms.xform_class[size_t(t)]);
        int64_t want = -1;
        if (!whole[c]) {
            want = 0;
            const ManySpec::Class &cl = ms.classes[c];
            for (int o = 0; o < cl.nops; ++o) want += op_parts(ms.ops[size_t(cl.first_op + o)]);
        }
        if (seen[size_t(t)] != want) {
            err = "internal: ragged schedule misses a part";
            return kInternal;
        }
    }
    return kOK;
}

std::string RaggedSchedule::describe() const
{
    std::ostringstream o;
    o << "  schedule: whole=" << whole_transforms << " split=" << split_transforms << " phases=" << phase_first.size()
      << " blocks=";
    for (size_t k = 0; k < phase_blocks.size(); ++k) o << (k ? "+" : "") << phase_blocks[k];
    o << "\n";
    return o.str();
}

int tune_set(const char *entries, int replace)
{
    std::map<std::string, Tune> add;
    if (entries) parse_tune_items(entries, add);
    std::lock_guard<std::mutex> lock(tune_mutex());
    std::map<std::string, Tune> &tab = tune_table_locked();
    if (replace) tab.clear();
    for (const auto &kv : add) tab[kv.first] = kv.second;
    return kOK;
}

std::string tune_dump()
{
    std::lock_guard<std::mutex> lock(tune_mutex());
    std::ostringstream o;
    for (const auto &kv : tune_table_locked()) o << kv.first << "=" << format_tune(kv.second) << "\n";
    return o.str();
}

} // namespace mifft
