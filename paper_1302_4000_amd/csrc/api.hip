// C-ABI entry points (include/clusco.h): argument validation, workspace
// layout and the launch sequence.  Every argument error is caught here,
// before anything is enqueued.  Nothing on the per-call path allocates
// device memory or synchronises the host; the first batched call for a new
// shape uploads its plan (a small device table) once.
#include <dlfcn.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <list>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

using namespace clusco;

namespace {

struct BatchPlan {
    // key
    std::vector<int64_t> key;
    // device tables: ModelSet[nset] then Problem[nprob]
    void *dtab = nullptr;
    int32_t nset = 0, nprob = 0;
    int64_t total_models = 0, T = 0, n_wtiles = 0;
    size_t ws_total = 0, off_list = 0;
    Problem first{};          // any problem (for launches with one)
    int sched = SCHED_STAGED;  // tile schedule of the launches
    int emode = 0;             // kernel arithmetic (x4 when every problem is)
    int64_t T4 = 0;            // split-BF16: tiles of the four-product problems (they
                               // come first and take a launch of their own)
    // cached graph for the last buffers it was captured with
    hipGraphExec_t exec = nullptr;
    const void *g_coords = nullptr, *g_out = nullptr, *g_ws = nullptr;
    // used inside a graph the caller captured: its table address is baked
    // into that graph, so the plan is kept until the handle is destroyed
    bool pinned = false;
};

// Kernel configuration of one problem: what the tuning table chooses per
// (precision, N bucket, L bucket).
struct KernelCfg {
    int products = 3;               // split-BF16: MFMA products per K-block (3 or 4)
    int schedule = SCHED_STAGED;    // SCHED_STAGED or SCHED_PERSISTENT
    int band = 16;                  // tile rows per band of the tile order
    int frame = 1;                  // contract residuals in the reference frame
    int id = -1;                    // bucket index in the table (-1: not from the table)
    int source = 0;                 // 0 built-in default, 1 tuning table, 2 forced
};

struct TuneEntry {
    int mode, nb, lb;
    int call;       // 0: single calls; 1: ensembles inside batched calls
    KernelCfg cfg;
};

// Tuning table: bucket edges (ascending lower bounds; bucket i holds
// edges[i] <= x < edges[i+1], the last one open) and the chosen
// configuration per (precision, N bucket, L bucket).
struct TuneTable {
    std::vector<int64_t> n_edges, l_edges;
    std::vector<TuneEntry> entries;
    std::string path;
};

} // namespace

struct clusco_ctx {
    int device;
    double tol[NMODES];   // fix-up tolerance per precision (A); <= 0 disables
    std::string last_error;
    // stage timing (measurement only): 4 events per recorded call
    std::vector<hipEvent_t> events;
    int slots = 0, used = 0;
    // batched plans, most recent first
    std::list<BatchPlan> plans;
    hipStream_t capture = nullptr;
    // device address of this device's built-in scratch (no-alloc entry
    // point), looked up once per device when the handle is created
    void *scratch = nullptr;
    hipError_t scratch_err = hipSuccess;
    // kernel configurations: tuning table, an optional forced configuration,
    // and a generation count that changes with either (part of plan keys)
    std::string arch;
    TuneTable tune;
    bool forced = false;
    KernelCfg force;
    int64_t tune_gen = 0;
};

// Built-in workspace of clusco_crmsd_matrix_noalloc: every device that loads
// the library holds one copy until the process ends.  Host code never uses
// the array's name as an address (on the host it is only a stand-in for the
// symbol); it uses the device address hipGetSymbolAddress returns, kept per
// device in scratch_ptr.
static __device__ __align__(256) char scratch[CLUSCO_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES];
hipError_t scratch_status[MAX_DEVICES];
bool scratch_done[MAX_DEVICES];

// Device address of `scratch` on the current device `dev` (looked up once).
hipError_t scratch_setup(int dev, void **ptr)
{
    *ptr = nullptr;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_done[dev]) {
        void *p = nullptr;
        scratch_status[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        scratch_ptr[dev] = scratch_status[dev] == hipSuccess ? p : nullptr;
        scratch_done[dev] = true;
    }
    *ptr = scratch_ptr[dev];
    return scratch_status[dev];
}

} // namespace

namespace {

constexpr int64_t MAX_N = 1 << 20;   // fix-up entries hold 16-bit row blocks
constexpr size_t MAX_PLANS = 8;

clusco_status fail(clusco_handle h, clusco_status s, const char *msg)
{
    if (h) h->last_error = msg;
    return s;
}

clusco_status hip_fail(clusco_handle h, hipError_t e, const char *where)
{
    if (h) {
        h->last_error = where;
        h->last_error += ": ";
        h->last_error += hipGetErrorString(e);
    }
    return CLUSCO_ERR_HIP;
}

bool valid_precision(clusco_precision p)
{
    return p == CLUSCO_FP32 || p == CLUSCO_SPLIT_BF16 || p == CLUSCO_SPLIT_FP16 || p == CLUSCO_FP64 ||
           p == CLUSCO_SPLIT_BF16X4;
}

int mode_of(clusco_precision p)
{
    switch (p) {
    case CLUSCO_FP32: return MODE_FP32;
    case CLUSCO_SPLIT_BF16: return MODE_BF16;
    case CLUSCO_SPLIT_BF16X4: return MODE_BF16X4;
    case CLUSCO_SPLIT_FP16: return MODE_FP16;
    default: return MODE_FP64;
    }
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Makes the handle's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev)
    {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Error model of the contraction, the basis of the FP64 fix-up flag.
//
// Eq. 2 gives L s^2 = E_i + E_j - 2 S(H), S the signed sum of the singular
// values of H.  An error dH of the correlation moves S by at most about |dH|
// and hence the score s by d(L s^2) / (2 L s).  The correlation's error comes
// from the low-precision contraction of the vectors the MFMAs see (the
// centred models, or in the reference frame their residuals d from the
// reference), whose squared size is W = sum |d|^2 (W = E without the frame),
// plus the FP64 epilogue's own error, relative to S itself (of the size of
// the radii E).  Writing them as eps_W (W_i + W_j) / 2 and
// eps_E (E_i + E_j) / 2 bounds the score error by
//     err(s) <= (eps_W (W_i + W_j) + eps_E (E_i + E_j)) / (L s),
// which grows without bound as s -> 0: small scores need the fix-up.  eps_W
// has two measured parts:
//   accumulation  every MFMA step rounds the FP32 accumulators once, so an
//                 accumulator that grows steadily to about W carries about
//                 2^-24 W sqrt(steps / 3) of rounding (a random walk over
//                 the steps): steps = Lp/2 (FP32, 2 atoms per step),
//                 3 Lp/16 (split, 16 atoms per product, three products) or
//                 4 Lp/16 (split x4);
//   dropped term  split-BF16 x3 leaves out lo*lo' (|lo| <= 2^-9 |d|): per
//                 atom a product of about 2^-18 |d||d'| with a random sign,
//                 2^-18 W / sqrt(L) summed (split-FP16 x3 drops 2^-24 |d||d'|,
//                 which the accumulation part covers; x4 drops nothing).
// The coefficients are fitted to GPU measurements of max err s L / (W_i + W_j)
// with the fix-up off (FP64 oracle, L = 150, 300 and 500); EPS_MARGIN keeps
// every measured maximum at most 1 / EPS_MARGIN of the model's value.
// eps_E covers the epilogue's largest root (Newton steps stop below 1e-5
// relative change: the root is then good to about 1e-10) with a margin of two;
// the refined reciprocal square roots and FP64 rounding add about 1e-15.
constexpr double K_ACC = 0.70, K_DROP = 1.90, EPS_MARGIN = 1.5, EPS_ROOT = 2e-10;

double contraction_eps(int mode, int64_t L)
{
    if (mode == MODE_FP64) return 0.0;
    const double Lp = (double)round_up(L, kblock(mode));
    const double steps = mode == MODE_FP32     ? Lp / 2.0
                         : mode == MODE_BF16X4 ? Lp / 4.0
                                               : 3.0 * Lp / 16.0;
    const double acc = std::ldexp(1.0, -24) * std::sqrt(steps / 3.0);
    const double drop = mode == MODE_BF16 ? std::ldexp(1.0, -18) / std::sqrt((double)L) : 0.0;
    return EPS_MARGIN * (K_ACC * acc + K_DROP * drop);
}

// Flag a pair when its score bound exceeds half the tolerance, i.e. when
// s < F_i + F_j with the per-model flag weight F = fw W + fe E,
// fw = 2 eps_W / (L tol), fe = 2 eps_E / (L tol).  An unflagged pair's error
// is then at most tol / (2 EPS_MARGIN) by the measured maxima.  tol is the
// requested precision's; eps_W is the arithmetic's (split-BF16 with four
// products has its own).
struct FlagCoefs {
    double fw = 0.0, fe = 0.0;
    bool on = false;
};

FlagCoefs flag_coefs(clusco_handle h, int mode, int arith, int64_t L)
{
    FlagCoefs f;
    const double tol = h ? h->tol[mode] : 0.0;
    if (mode == MODE_FP64 || !(tol > 0.0)) return f;
    const double k = 2.0 / ((double)L * tol);
    f.fw = k * contraction_eps(arith, L);
    f.fe = k * EPS_ROOT;
    f.on = true;
    return f;
}

// ---------------------------------------------------------------- tuning

int bucket_of(const std::vector<int64_t> &edges, int64_t x)
{
    int b = 0;
    for (size_t i = 1; i < edges.size(); ++i)
        if (x >= edges[i]) b = (int)i;
    return b;
}

// Configuration for a problem of N models (an all-vs-all ensemble, or the
// all-vs-all size with as many pairs for a cross comparison) of L atoms; in a
// batched call (batched) the bucket's batched entry when the table has one,
// else its single-call entry.
KernelCfg config_for(clusco_handle h, int mode, int64_t N, int64_t L, bool batched = false)
{
    KernelCfg c;
    if (h->forced) {
        c = h->force;
        c.source = 2;
    } else if (!h->tune.n_edges.empty() && !h->tune.l_edges.empty()) {
        const int nb = bucket_of(h->tune.n_edges, N), lb = bucket_of(h->tune.l_edges, L);
        const int want = batched ? 1 : 0;
        const TuneEntry *own = nullptr, *single = nullptr;
        for (const TuneEntry &t : h->tune.entries) {
            if (t.mode != mode || t.nb != nb || t.lb != lb) continue;
            if (t.call == want) {
                own = &t;
                break;
            }
            if (t.call == 0 && !single) single = &t;
        }
        const TuneEntry *hit = own ? own : single;
        if (hit) {
            c = hit->cfg;
            c.id = nb * (int)h->tune.l_edges.size() + lb;
            c.source = 1;
        }
    }
    if (mode != MODE_BF16) c.products = mode == MODE_BF16X4 ? 4 : 3;
    // the persistent schedule serves problems without the reference frame
    if (mode == MODE_FP64 || c.schedule == SCHED_PERSISTENT) c.frame = 0;
    return c;
}

// The arithmetic a problem's contraction uses: split-BF16 with four
// products is the x4 mode.
int arith_mode(int mode, const KernelCfg &c)
{
    return mode == MODE_BF16 && c.products == 4 ? MODE_BF16X4 : mode;
}

// The set's share of configuration c: the reference frame (reference
// candidates: the first models of the set `own`, whose moments live in its
// workspace slot) and the flag coefficients.
void configure_set(const KernelCfg &c, const FlagCoefs &f, const ModelSet &own, ModelSet &s)
{
    s.frame = c.frame;
    s.ref_X = own.X;
    s.ref_N = own.N;
    s.ref_b = own.use_b;
    s.refinfo = own.refinfo;
    s.ref_own = &own == &s;
    s.fw = f.fw;
    s.fe = f.fe;
}

// The problem's share of configuration c.
void configure_problem(const KernelCfg &c, int arith, const FlagCoefs &f, Problem &p)
{
    p.x4 = arith == MODE_BF16X4;
    p.band = c.band;
    p.cfg = c.id;
    p.frame = c.frame;
    p.flag_coef = f.on ? 1.0 : -1.0;
}

// A minimal JSON reader for the tuning file (objects, arrays, strings,
// numbers, true / false / null; nesting depth at most 32).
struct JVal {
    enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
    double num = 0.0;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;
    const JVal *get(const char *k) const
    {
        for (const auto &kv : obj)
            if (kv.first == k) return &kv.second;
        return nullptr;
    }
};

struct JParser {
    const char *p, *end;
    std::string err;
    void skip()
    {
        while (p < end && (*p == ' ' || *p == '\n' || *p == '\t' || *p == '\r')) ++p;
    }
    bool fail_at(const char *what)
    {
        if (err.empty()) err = what;
        return false;
    }
    bool word(const char *w)
    {
        const size_t n = strlen(w);
        if ((size_t)(end - p) < n || strncmp(p, w, n) != 0) return fail_at("bad literal");
        p += n;
        return true;
    }
    bool string(std::string &out)
    {
        if (p >= end || *p != '"') return fail_at("expected a string");
        ++p;
        while (p < end && *p != '"') {
            if (*p == '\\') {
                if (++p >= end) break;
                const char c = *p;
                if (c == 'u') {
                    if (end - p < 5) return fail_at("bad escape");
                    p += 4;
                    out += '?';
                } else {
                    out += c == 'n' ? '\n' : c == 't' ? '\t' : c == 'r' ? '\r' : c == 'b' ? '\b' : c == 'f' ? '\f' : c;
                }
                ++p;
            } else {
                out += *p++;
            }
        }
        if (p >= end) return fail_at("unterminated string");
        ++p;
        return true;
    }
    bool value(JVal &v, int depth)
    {
        if (depth > 32) return fail_at("nesting too deep");
        skip();
        if (p >= end) return fail_at("unexpected end");
        const char c = *p;
        if (c == '{') {
            v.kind = JVal::OBJ;
            ++p;
            skip();
            if (p < end && *p == '}') { ++p; return true; }
            for (;;) {
                skip();
                std::string k;
                if (!string(k)) return false;
                skip();
                if (p >= end || *p != ':') return fail_at("expected ':'");
                ++p;
                JVal x;
                if (!value(x, depth + 1)) return false;
                v.obj.emplace_back(std::move(k), std::move(x));
                skip();
                if (p < end && *p == ',') { ++p; continue; }
                if (p < end && *p == '}') { ++p; return true; }
                return fail_at("expected ',' or '}'");
            }
        }
        if (c == '[') {
            v.kind = JVal::ARR;
            ++p;
            skip();
            if (p < end && *p == ']') { ++p; return true; }
            for (;;) {
                JVal x;
                if (!value(x, depth + 1)) return false;
                v.arr.push_back(std::move(x));
                skip();
                if (p < end && *p == ',') { ++p; continue; }
                if (p < end && *p == ']') { ++p; return true; }
                return fail_at("expected ',' or ']'");
            }
        }
        if (c == '"') {
            v.kind = JVal::STR;
            return string(v.str);
        }
        if (c == 't') { v.kind = JVal::BOOL; v.num = 1; return word("true"); }
        if (c == 'f') { v.kind = JVal::BOOL; return word("false"); }
        if (c == 'n') return word("null");
        char *q = nullptr;
        std::string tok(p, (size_t)std::min<ptrdiff_t>(end - p, 64));
        v.num = strtod(tok.c_str(), &q);
        if (q == tok.c_str()) return fail_at("bad number");
        v.kind = JVal::NUM;
        p += q - tok.c_str();
        return true;
    }
};

int mode_of_name(const std::string &s)
{
    if (s == "fp32") return MODE_FP32;
    if (s == "split_bf16") return MODE_BF16;
    if (s == "split_fp16") return MODE_FP16;
    if (s == "split_bf16x4") return MODE_BF16X4;
    return -1;
}

bool read_edges(const JVal *v, std::vector<int64_t> &out)
{
    if (!v || v->kind != JVal::ARR || v->arr.empty() || v->arr.size() > 64) return false;
    for (const JVal &x : v->arr) {
        if (x.kind != JVal::NUM || x.num < 0 || x.num > 1e12 || x.num != std::floor(x.num))
            return false;
        if (!out.empty() && (int64_t)x.num <= out.back()) return false;
        out.push_back((int64_t)x.num);
    }
    return true;
}

// Parses and checks a tuning file; on success *t holds it.  `arch` (may be
// empty: not known) must match the file's "arch".
clusco_status parse_tuning(const std::string &text, const std::string &arch, TuneTable *t,
                           std::string *err)
{
    JParser jp{text.data(), text.data() + text.size(), {}};
    JVal root;
    if (!jp.value(root, 0)) {
        *err = "tuning file: " + jp.err;
        return CLUSCO_ERR_INVALID_ARG;
    }
    if (root.kind != JVal::OBJ) {
        *err = "tuning file: not a JSON object";
        return CLUSCO_ERR_INVALID_ARG;
    }
    const JVal *a = root.get("arch");
    if (!a || a->kind != JVal::STR) {
        *err = "tuning file: no \"arch\"";
        return CLUSCO_ERR_INVALID_ARG;
    }
    if (!arch.empty() && a->str != arch) {
        *err = "tuning file is for " + a->str + ", the device is " + arch;
        return CLUSCO_ERR_UNSUPPORTED;
    }
    TuneTable out;
    if (!read_edges(root.get("n_edges"), out.n_edges) || !read_edges(root.get("l_edges"), out.l_edges)) {
        *err = "tuning file: n_edges / l_edges must be ascending non-negative integers";
        return CLUSCO_ERR_INVALID_ARG;
    }
    const JVal *es = root.get("entries");
    if (!es || es->kind != JVal::ARR) {
        *err = "tuning file: no \"entries\" array";
        return CLUSCO_ERR_INVALID_ARG;
    }
    for (const JVal &e : es->arr) {
        const JVal *pr = e.get("precision"), *nb = e.get("n_bucket"), *lb = e.get("l_bucket"),
                   *pd = e.get("products"), *sc = e.get("schedule"), *bd = e.get("band");
        TuneEntry t{};
        bool ok = e.kind == JVal::OBJ && pr && pr->kind == JVal::STR && nb && nb->kind == JVal::NUM &&
                  lb && lb->kind == JVal::NUM && pd && pd->kind == JVal::NUM && sc &&
                  sc->kind == JVal::STR && bd && bd->kind == JVal::NUM;
        if (ok) {
            t.mode = mode_of_name(pr->str);
            t.nb = (int)nb->num;
            t.lb = (int)lb->num;
            t.cfg.products = (int)pd->num;
            t.cfg.schedule = sc->str == "staged" ? SCHED_STAGED : sc->str == "persistent" ? SCHED_PERSISTENT : -1;
            t.cfg.band = (int)bd->num;
            const JVal *fr = e.get("frame");
            if (fr) t.cfg.frame = fr->kind == JVal::NUM && (fr->num == 0 || fr->num == 1) ? (int)fr->num : -1;
            const JVal *cl = e.get("call");
            t.call = 0;
            if (cl) t.call = cl->kind == JVal::STR && cl->str == "single" ? 0
                           : cl->kind == JVal::STR && cl->str == "batched" ? 1 : -1;
            ok = t.call >= 0 && t.cfg.frame >= 0 && t.mode >= 0 && nb->num == t.nb && lb->num == t.lb && t.nb >= 0 &&
                 t.nb < (int)out.n_edges.size() && t.lb >= 0 && t.lb < (int)out.l_edges.size() &&
                 (t.cfg.products == 3 || t.cfg.products == 4) && t.cfg.schedule >= 0 &&
                 bd->num == t.cfg.band && t.cfg.band >= 1 && t.cfg.band <= 256;
        }
        if (!ok) {
            *err = "tuning file: bad entry (needs precision, n_bucket, l_bucket, products 3|4, "
                   "schedule staged|persistent, band 1..256, optional frame 0|1, optional call "
                   "single|batched, buckets within the edges)";
            return CLUSCO_ERR_INVALID_ARG;
        }
        out.entries.push_back(t);
    }
    *t = std::move(out);
    return CLUSCO_OK;
}

clusco_status load_tuning_file(clusco_handle h, const std::string &path, std::string *err)
{
    FILE *f = fopen(path.c_str(), "rb");
    if (!f) {
        *err = "cannot open tuning file " + path;
        return CLUSCO_ERR_INVALID_ARG;
    }
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0 && text.size() < (16u << 20)) text.append(buf, n);
    fclose(f);
    TuneTable t;
    const clusco_status st = parse_tuning(text, h->arch, &t, err);
    if (st != CLUSCO_OK) return st;
    t.path = path;
    h->tune = std::move(t);
    ++h->tune_gen;
    return CLUSCO_OK;
}

// <directory of this library>/tuning/<arch>.json
std::string default_tuning_path(const std::string &arch)
{
    Dl_info info{};
    if (arch.empty() || !dladdr((void *)&default_tuning_path, &info) || !info.dli_fname) return "";
    std::string lib = info.dli_fname;
    const size_t slash = lib.rfind('/');
    const std::string dir = slash == std::string::npos ? "." : lib.substr(0, slash);
    return dir + "/tuning/" + arch + ".json";
}

void stage_mark(clusco_handle h, int k, hipStream_t s)
{
    if (h->used >= h->slots) return;
    (void)hipEventRecord(h->events[4 * h->used + k], s);
    if (k == 3) ++h->used;
}

// ---------------------------------------------------------------- layout

size_t take(size_t &o, size_t bytes)
{
    size_t r = o;
    o += (size_t)round_up((int64_t)bytes, 256);
    return r;
}

ModelSet make_set(int mode, int64_t X, int64_t N, int64_t L, int64_t model0, int use_b, size_t &o)
{
    ModelSet s{};
    s.X = X;
    s.N = N;
    s.Np = round_up(N > 0 ? N : 1, TILE);
    s.L = L;
    s.Lp = round_up(L, kblock(mode));
    s.KB = s.Lp / kblock(mode);
    s.model0 = model0;
    s.use_b = use_b;
    s.E = (int64_t)take(o, sizeof(double) * s.Np);
    s.cen = (int64_t)take(o, sizeof(double) * 3 * s.Np);
    s.E64 = (int64_t)take(o, sizeof(double) * s.Np);
    s.U = (int64_t)take(o, sizeof(double) * 9 * s.Np);
    s.PT = (int64_t)take(o, sizeof(double) * 9 * s.Np);
    s.F = (int64_t)take(o, sizeof(double) * s.Np);
    s.refinfo = (int64_t)take(o, sizeof(double) * REF_INFO);
    s.ops = (int64_t)take(o, op_bytes_per_model(mode, s.Lp) * s.Np);
    return s;
}

Problem make_problem(const ModelSet &A, const ModelSet &B, int sym, double coef)
{
    Problem p{};
    p.NA = A.N;
    p.NB = B.N;
    p.L = A.L;
    p.KB = A.KB;
    p.nbA = A.Np / TILE;
    p.nbB = B.Np / TILE;
    p.nrbA = A.Np / ROWBLK;
    p.nrbB = B.Np / ROWBLK;
    p.opsA = A.ops;
    p.opsB = B.ops;
    p.EA = A.E;
    p.EB = B.E;
    p.cenA = A.cen;
    p.cenB = B.cen;
    p.E64A = A.E64;
    p.E64B = B.E64;
    p.UA = A.U;
    p.PTB = B.PT;
    p.FA = A.F;
    p.FB = B.F;
    p.XA = A.X;
    p.XB = B.X;
    p.flag_coef = coef;
    p.sym = sym;
    p.x4 = 0;
    p.band = KernelCfg{}.band;
    p.cfg = -1;
    p.frame = A.frame;
    return p;
}

struct SingleLayout {
    ModelSet A, B;
    Problem p;
    size_t total, off_list;
    KernelCfg cfg;
    int emode;            // arithmetic of the contraction (x4 when chosen)
};

// Configuration of a single problem of N models (frame: whether the
// reference frame may be used; the backward never uses it).
void configure(clusco_handle h, int mode, int64_t N, bool frame, SingleLayout &s)
{
    if (h) s.cfg = config_for(h, mode, N, s.A.L);
    if (!frame) s.cfg.frame = 0;
    s.emode = arith_mode(mode, s.cfg);
    const FlagCoefs f = flag_coefs(h, mode, s.emode, s.A.L);
    // the reference is chosen among the first models of the first set, for
    // both sets
    configure_set(s.cfg, f, s.A, s.A);
    configure_set(s.cfg, f, s.A, s.B);
}

SingleLayout single_layout(clusco_handle h, int mode, int64_t N, int64_t L, bool frame = true)
{
    SingleLayout s{};
    size_t o = 256;
    s.A = make_set(mode, 0, N, L, 0, 0, o);
    s.B = s.A;
    configure(h, mode, N, frame, s);
    s.B = s.A;
    s.p = make_problem(s.A, s.A, 1, -1.0);
    configure_problem(s.cfg, s.emode, flag_coefs(h, mode, s.emode, L), s.p);
    s.off_list = take(o, sizeof(FixEntry) * problem_wtiles(s.p));
    s.total = o;
    return s;
}

// A cross comparison takes the configuration of the all-vs-all size with as
// many pairs.
SingleLayout cross_layout(clusco_handle h, int mode, int64_t Na, int64_t Nb, int64_t L,
                          bool frame = true)
{
    SingleLayout s{};
    size_t o = 256;
    s.A = make_set(mode, 0, Na, L, 0, 0, o);
    s.B = make_set(mode, 0, Nb, L, s.A.Np, 1, o);
    configure(h, mode, (int64_t)std::sqrt(2.0 * (double)Na * (double)Nb) + 1, frame, s);
    s.p = make_problem(s.A, s.B, 0, -1.0);
    configure_problem(s.cfg, s.emode, flag_coefs(h, mode, s.emode, L), s.p);
    s.off_list = take(o, sizeof(FixEntry) * problem_wtiles(s.p));
    s.total = o;
    return s;
}

// The backward recomputes each pair's correlation with the forward's
// contraction (FP32 MFMA for the FP32 and FP64 precisions) and stores one
// 12-float record per pair after the forward layout.
int bwd_mode(int mode) { return mode == MODE_FP64 ? MODE_FP32 : mode; }

struct BwdLayout {
    SingleLayout s;
    size_t off_wq, off_pa, off_pb, off_part, total;
};

size_t grad_planes_bytes(int64_t n, int64_t L)
{
    return sizeof(float) * 3 * (size_t)grad_partners_padded(n) * (size_t)grad_atoms_padded(L);
}

BwdLayout bwd_layout(clusco_handle h, int mode, int64_t NA, int64_t NB, int64_t L, bool cross)
{
    BwdLayout b{};
    b.s = cross ? cross_layout(h, bwd_mode(mode), NA, NB, L, false)
                : single_layout(h, bwd_mode(mode), NA, L, false);
    size_t o = b.s.total;
    const int64_t pairs = cross ? NA * NB : NA * (NA - 1) / 2;
    b.off_wq = take(o, sizeof(float) * 12 * (pairs > 0 ? pairs : 1));
    b.off_pa = take(o, grad_planes_bytes(NA, L));
    b.off_pb = cross ? take(o, grad_planes_bytes(NB, L)) : b.off_pa;
    size_t part = grad_partial_bytes(NA, cross ? NB : NA, L);
    if (cross) part = std::max(part, grad_partial_bytes(NB, NA, L));
    b.off_part = take(o, part > 0 ? part : 1);
    b.total = o;
    return b;
}

clusco_status enqueue_bwd(clusco_handle h, int mode, const float *XA, const float *XB,
                          char *ws, const BwdLayout &b, bool cross, const float *rmsd,
                          const float *gout, float *gradA, float *gradB, hipStream_t s)
{
    const bool timing = h->used < h->slots;
    const int m = bwd_mode(mode);
    PrepLaunch pl{};
    pl.XA = XA;
    pl.XB = XB;
    pl.ws = ws;
    pl.mode = m;
    pl.counters = (int *)ws;
    pl.set[0] = b.s.A;
    pl.set[1] = b.s.B;
    pl.nset = cross ? 2 : 1;
    pl.total = b.s.A.Np + (cross ? b.s.B.Np : 0);
    if (timing) stage_mark(h, 0, s);
    hipError_t e = launch_prep(pl, s);
    if (e != hipSuccess) return hip_fail(h, e, "prep launch");
    if (timing) stage_mark(h, 1, s);
    TileLaunch tl{};
    tl.ws = ws;
    tl.prob = b.s.p;
    tl.nprob = 1;
    tl.kind = cross ? TK_RECT : TK_SYM;
    tl.T = problem_tiles(b.s.p);
    tl.counters = (int *)ws;
    tl.list = (FixEntry *)(ws + b.s.off_list);
    tl.rmsd = rmsd;
    tl.gout = gout;
    tl.wq = (float *)(ws + b.off_wq);
    e = launch_tile(m, tl, s, OP_BWD);
    if (e != hipSuccess) return hip_fail(h, e, "backward pairs launch");
    if (timing) stage_mark(h, 2, s);
    const double *cenA = (const double *)(ws + b.s.A.cen);
    const double *cenB = (const double *)(ws + b.s.B.cen);
    const int64_t NA = b.s.p.NA, NB = b.s.p.NB, L = b.s.p.L, Lp = grad_atoms_padded(L);
    float *PA = (float *)(ws + b.off_pa), *PB = (float *)(ws + b.off_pb);
    e = launch_grad_planes(XA, cenA, PA, NA, L, s);
    if (e == hipSuccess && cross) e = launch_grad_planes(XB, cenB, PB, NB, L, s);
    if (e != hipSuccess) return hip_fail(h, e, "gradient planes launch");
    // the two sides run one after the other on the stream and share the partials
    auto side = [&](const float *XR, const double *cenR, const float *P, float *grad, int64_t NR,
                    int64_t NC, int kind) {
        const GradSplit sp = grad_split(NR, NC, L);
        const size_t nw = (size_t)sp.nsplit * (size_t)NR;
        double *part = (double *)(ws + b.off_part);
        GradLaunch gl{XR, cenR, (const float4 *)P, tl.wq, grad, part, part + 3 * L * nw, NR, NC, L, Lp, kind,
                      sp.nsplit, sp.bps, 0};
        return launch_grad(gl, s);
    };
    e = side(XA, cenA, cross ? PB : PA, gradA, NA, cross ? NB : NA, cross ? GK_CROSS_A : GK_SYM);
    if (e != hipSuccess) return hip_fail(h, e, "gradient launch");
    if (cross && gradB) {
        e = side(XB, cenB, PA, gradB, NB, NA, GK_CROSS_B);
        if (e != hipSuccess) return hip_fail(h, e, "gradient launch");
    }
    if (timing) stage_mark(h, 3, s);
    return CLUSCO_OK;
}

// Enqueue prep -> tile -> fix-up for the given sets / problems.
clusco_status enqueue(clusco_handle h, int mode, const float *XA, const float *XB, char *ws,
                      float *out, const SingleLayout *single, const BatchPlan *plan, int kind,
                      hipStream_t s, bool timing)
{
    int *counters = (int *)ws;
    PrepLaunch pl{};
    pl.XA = XA;
    pl.XB = XB;
    pl.ws = ws;
    pl.mode = mode;
    pl.counters = counters;
    TileLaunch tl{};
    tl.ws = ws;
    tl.out = out;
    tl.kind = kind;
    tl.counters = counters;
    FixupLaunch fl{};
    fl.XA = XA;
    fl.XB = XB;
    fl.ws = ws;
    fl.out = out;
    fl.counters = counters;
    fl.all = mode == MODE_FP64;
    double coef;
    if (single) {
        pl.set[0] = single->A;
        pl.set[1] = single->B;
        pl.nset = kind == TK_RECT ? 2 : 1;
        pl.total = single->A.Np + (kind == TK_RECT ? single->B.Np : 0);
        tl.prob = single->p;
        tl.nprob = 1;
        tl.T = problem_tiles(single->p);
        tl.list = (FixEntry *)(ws + single->off_list);
        fl.prob = single->p;
        fl.nprob = 1;
        fl.n_all = problem_wtiles(single->p);
        fl.list = tl.list;
        coef = single->p.flag_coef;
        tl.sched = single->cfg.schedule;
    } else {
        pl.table = (const ModelSet *)plan->dtab;
        pl.nset = plan->nset;
        pl.total = plan->total_models;
        const Problem *pt = (const Problem *)((const char *)plan->dtab +
                                              sizeof(ModelSet) * plan->nset);
        tl.table = pt;
        tl.nprob = plan->nprob;
        tl.T = plan->T;
        tl.list = (FixEntry *)(ws + plan->off_list);
        fl.table = pt;
        fl.nprob = plan->nprob;
        fl.n_all = plan->n_wtiles;
        fl.list = tl.list;
        coef = plan->first.flag_coef;
        tl.sched = plan->sched;
    }
    const int emode = single ? single->emode : plan->emode;
    if (timing) stage_mark(h, 0, s);
    hipError_t e = launch_prep(pl, s);
    if (e != hipSuccess) return hip_fail(h, e, "prep launch");
    if (timing) stage_mark(h, 1, s);
    if (mode != MODE_FP64) {
        if (plan && plan->T4 > 0 && plan->T4 < plan->T) {
            // a batch whose split-BF16 problems differ in their product
            // count: the four-product tiles, then the three-product ones
            TileLaunch t4 = tl;
            t4.T = plan->T4;
            t4.ctr = 1;
            e = launch_tile(MODE_BF16X4, t4, s);
            if (e == hipSuccess) {
                TileLaunch t3 = tl;
                t3.t0 = plan->T4;
                t3.T = plan->T - plan->T4;
                t3.ctr = 2;
                e = launch_tile(MODE_BF16, t3, s);
            }
        } else {
            tl.ctr = 1;
            e = launch_tile(emode, tl, s);
        }
        if (e != hipSuccess) return hip_fail(h, e, "tile launch");
    }
    if (timing) stage_mark(h, 2, s);
    if (mode == MODE_FP64 || coef > 0.0) {
        e = launch_fixup(fl, s);
        if (e != hipSuccess) return hip_fail(h, e, "fix-up launch");
    }
    if (timing) stage_mark(h, 3, s);
    return CLUSCO_OK;
}

// ---------------------------------------------------------------- batches

struct BatchInput {
    int32_t E;
    const int64_t *N, *L, *coff, *ooff;
};

std::vector<int64_t> batch_key(clusco_handle h, int mode, const BatchInput &b, bool with_offsets)
{
    std::vector<int64_t> k;
    k.reserve(4 * b.E + 4);
    k.push_back(mode);
    k.push_back(h->tune_gen);
    k.push_back(b.E);
    double tol = h->tol[mode];
    int64_t t;
    memcpy(&t, &tol, 8);
    k.push_back(t);
    for (int32_t e = 0; e < b.E; ++e) {
        k.push_back(b.N[e]);
        k.push_back(b.L[e]);
        if (with_offsets) {
            k.push_back(b.coff[e]);
            k.push_back(b.ooff[e]);
        }
    }
    return k;
}

// Host-side plan: sets by descending length, problems sorted by cost per tile
// (padded length, then size) so the persistent kernel starts the longest
// tiles first.  Returns the workspace size; fills tables when asked.
struct PlanKernel {
    int sched = SCHED_STAGED, emode = 0;
    int64_t T4 = 0;
};

size_t plan_layout(clusco_handle h, int mode, const BatchInput &b, std::vector<ModelSet> *sets,
                   std::vector<Problem> *probs, size_t *off_list, int64_t *T, int64_t *nw,
                   int64_t *total, PlanKernel *pk = nullptr)
{
    size_t o = 256;
    std::vector<ModelSet> S;
    std::vector<Problem> P;
    int64_t model0 = 0;
    // each problem takes its bucket's configuration; the launch takes the
    // schedule that most of the work (tiles x K-blocks x products) prefers
    // among those that keep every problem's own arithmetic: the persistent
    // schedule has no reference frame, so it is out when a problem uses the
    // frame (every ensemble's scores then equal those of its single call)
    std::vector<KernelCfg> cfg(b.E);
    double vote[2] = {0.0, 0.0};
    bool framed = false;
    for (int32_t e = 0; e < b.E; ++e) {
        if (b.N[e] < 2) continue;
        cfg[e] = config_for(h, mode, b.N[e], b.L[e], true);
        framed = framed || cfg[e].frame;
        const int64_t nb = round_up(b.N[e], TILE) / TILE;
        vote[cfg[e].schedule] += (double)tri_count(nb) *
            (double)round_up(b.L[e], kblock(mode)) * (double)cfg[e].products;
    }
    const int sched = !framed && vote[SCHED_PERSISTENT] > vote[SCHED_STAGED] ? SCHED_PERSISTENT
                                                                             : SCHED_STAGED;
    // sets (and so the prep's waves, which take the models in set order) go
    // longest model first: the longest models' chain of dependent loads sets
    // the prep's time, so they start before the short ones fill the GPU
    std::vector<int32_t> order;
    for (int32_t e = 0; e < b.E; ++e)
        if (b.N[e] >= 2) order.push_back(e);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return b.L[x] > b.L[y]; });
    int nx4 = 0;
    for (const int32_t e : order) {
        ModelSet s = make_set(mode, b.coff ? b.coff[e] : 0, b.N[e], b.L[e], model0, 0, o);
        model0 += s.Np;
        const KernelCfg c = cfg[e];
        const int am = arith_mode(mode, c);
        const FlagCoefs f = flag_coefs(h, mode, am, b.L[e]);
        configure_set(c, f, s, s);            // the reference is one of the ensemble's models
        S.push_back(s);
        Problem p = make_problem(s, s, 1, -1.0);
        configure_problem(c, am, f, p);
        p.out = b.ooff ? b.ooff[e] : 0;
        nx4 += p.x4;
        P.push_back(p);
    }
    // four-product problems first (a launch of their own when mixed), then
    // the most expensive tiles first
    std::stable_sort(P.begin(), P.end(), [](const Problem &x, const Problem &y) {
        if (x.x4 != y.x4) return x.x4 > y.x4;
        if (x.KB != y.KB) return x.KB > y.KB;
        return x.NA > y.NA;
    });
    int64_t T4 = 0;
    for (const Problem &p : P) T4 += p.x4 ? problem_tiles(p) : 0;
    if (pk) {
        pk->sched = sched;
        pk->emode = (nx4 > 0 && nx4 == (int)P.size()) ? MODE_BF16X4 : mode;
        pk->T4 = (nx4 > 0 && nx4 < (int)P.size()) ? T4 : 0;
    }
    int64_t t0 = 0, w0 = 0;
    for (Problem &p : P) {
        p.tile0 = t0;
        p.wtile0 = w0;
        t0 += problem_tiles(p);
        w0 += problem_wtiles(p);
    }
    size_t ol = take(o, sizeof(FixEntry) * (w0 > 0 ? w0 : 1));
    if (sets) *sets = S;
    if (probs) *probs = P;
    if (off_list) *off_list = ol;
    if (T) *T = t0;
    if (nw) *nw = w0;
    if (total) *total = model0;
    return o;
}

void free_plan(BatchPlan &p)
{
    if (p.exec) (void)hipGraphExecDestroy(p.exec);
    if (p.dtab) (void)hipFree(p.dtab);
    p.exec = nullptr;
    p.dtab = nullptr;
}

BatchPlan *find_plan(clusco_handle h, const std::vector<int64_t> &key)
{
    for (auto it = h->plans.begin(); it != h->plans.end(); ++it) {
        if (it->key == key) {
            h->plans.splice(h->plans.begin(), h->plans, it);
            return &h->plans.front();
        }
    }
    return nullptr;
}

// Builds and uploads a new plan (one hipMalloc and a blocking copy: never
// called while the caller's stream is being captured).  The least recently
// used unpinned plans beyond MAX_PLANS are freed.
clusco_status create_plan(clusco_handle h, int mode, const BatchInput &b,
                          std::vector<int64_t> key, BatchPlan **out)
{
    BatchPlan p;
    p.key = std::move(key);
    std::vector<ModelSet> sets;
    std::vector<Problem> probs;
    PlanKernel pk;
    p.ws_total = plan_layout(h, mode, b, &sets, &probs, &p.off_list, &p.T, &p.n_wtiles,
                             &p.total_models, &pk);
    p.sched = pk.sched;
    p.emode = pk.emode;
    p.T4 = pk.T4;
    p.nset = (int32_t)sets.size();
    p.nprob = (int32_t)probs.size();
    if (p.nprob > 0) {
        p.first = probs[0];
        const size_t bytes = sizeof(ModelSet) * sets.size() + sizeof(Problem) * probs.size();
        std::vector<char> host(bytes);
        memcpy(host.data(), sets.data(), sizeof(ModelSet) * sets.size());
        memcpy(host.data() + sizeof(ModelSet) * sets.size(), probs.data(),
               sizeof(Problem) * probs.size());
        hipError_t e = hipMalloc(&p.dtab, bytes);
        if (e == hipSuccess) e = hipMemcpy(p.dtab, host.data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            free_plan(p);
            return hip_fail(h, e, "upload batch plan");
        }
    }
    h->plans.push_front(std::move(p));
    size_t unpinned = 0;
    for (auto it = h->plans.begin(); it != h->plans.end();) {
        if (!it->pinned && ++unpinned > MAX_PLANS) {
            free_plan(*it);
            it = h->plans.erase(it);
        } else {
            ++it;
        }
    }
    *out = &h->plans.front();
    return CLUSCO_OK;
}

clusco_status check_batch(clusco_handle h, const BatchInput &b, bool need_offsets)
{
    if (b.E < 0) return fail(h, CLUSCO_ERR_INVALID_ARG, "E < 0");
    if (b.E == 0) return CLUSCO_OK;
    if (!b.N || !b.L || (need_offsets && (!b.coff || !b.ooff)))
        return fail(h, CLUSCO_ERR_INVALID_ARG, "null shape or offset array");
    for (int32_t e = 0; e < b.E; ++e) {
        if (b.N[e] < 0 || b.L[e] < 1) return fail(h, CLUSCO_ERR_INVALID_ARG, "need N >= 0, L >= 1");
        if (b.N[e] > MAX_N) return fail(h, CLUSCO_ERR_UNSUPPORTED, "N above 2^20");
        if (need_offsets && (b.coff[e] < 0 || b.ooff[e] < 0))
            return fail(h, CLUSCO_ERR_INVALID_ARG, "negative offset");
    }
    return CLUSCO_OK;
}

} // namespace

extern "C" {

const char *clusco_status_string(clusco_status s)
{
    switch (s) {
    case CLUSCO_OK: return "CLUSCO_OK";
    case CLUSCO_ERR_INVALID_ARG: return "CLUSCO_ERR_INVALID_ARG";
    case CLUSCO_ERR_WORKSPACE: return "CLUSCO_ERR_WORKSPACE";
    case CLUSCO_ERR_UNSUPPORTED: return "CLUSCO_ERR_UNSUPPORTED";
    case CLUSCO_ERR_HIP: return "CLUSCO_ERR_HIP";
    }
    return "CLUSCO_ERR_UNKNOWN";
}

clusco_status clusco_create(clusco_handle *h, int device)
{
    if (!h || device < 0) return CLUSCO_ERR_INVALID_ARG;
    clusco_ctx *c = new (std::nothrow) clusco_ctx;
    if (!c) return CLUSCO_ERR_INVALID_ARG;
    c->device = device;
    c->tol[MODE_FP32] = 1e-4;
    c->tol[MODE_BF16] = 5e-4;
    c->tol[MODE_BF16X4] = 5e-4;
    c->tol[MODE_FP16] = 1e-4;
    c->tol[MODE_FP64] = 1e-6;
    {
        DeviceGuard g(device);
        c->scratch_err = g.err != hipSuccess ? g.err : scratch_setup(device, &c->scratch);
        hipDeviceProp_t prop;
        if (g.err == hipSuccess && hipGetDeviceProperties(&prop, device) == hipSuccess) {
            c->arch = prop.gcnArchName;
            const size_t colon = c->arch.find(':');
            if (colon != std::string::npos) c->arch.resize(colon);
        }
    }
    // the tuning table: $CLUSCO_TUNING if set (empty: none), else the file
    // for this architecture next to the library; without one (or if it does
    // not parse) every problem takes the built-in default configuration
    const char *env = getenv("CLUSCO_TUNING");
    const std::string path = env ? std::string(env) : default_tuning_path(c->arch);
    if (!path.empty()) {
        std::string err;
        (void)load_tuning_file(c, path, &err);
    }
    *h = c;
    return CLUSCO_OK;
}

clusco_status clusco_load_tuning(clusco_handle h, const char *path)
{
    if (!h) return CLUSCO_ERR_INVALID_ARG;
    h->last_error.clear();
    if (!path) {
        h->tune = TuneTable{};
        ++h->tune_gen;
        return CLUSCO_OK;
    }
    std::string err;
    const clusco_status st = load_tuning_file(h, path, &err);
    return st == CLUSCO_OK ? st : fail(h, st, err.c_str());
}

static clusco_status get_config(clusco_handle h, int64_t N, int64_t L, clusco_precision p,
                                clusco_config *cfg, bool batched)
{
    if (!h || !cfg) return CLUSCO_ERR_INVALID_ARG;
    if (!valid_precision(p)) return fail(h, CLUSCO_ERR_UNSUPPORTED, "unknown precision");
    if (N < 0 || L < 1) return fail(h, CLUSCO_ERR_INVALID_ARG, "need N >= 0 and L >= 1");
    const KernelCfg c = config_for(h, mode_of(p), N, L, batched);
    cfg->products = c.products;
    cfg->schedule = c.schedule;
    cfg->band = c.band;
    cfg->frame = c.frame;
    cfg->source = c.source;
    cfg->bucket = c.id;
    return CLUSCO_OK;
}

clusco_status clusco_get_config(clusco_handle h, int64_t N, int64_t L, clusco_precision p,
                                clusco_config *cfg)
{
    return get_config(h, N, L, p, cfg, false);
}

clusco_status clusco_get_config_batched(clusco_handle h, int64_t N, int64_t L,
                                        clusco_precision p, clusco_config *cfg)
{
    return get_config(h, N, L, p, cfg, true);
}

clusco_status clusco_force_config(clusco_handle h, const clusco_config *cfg)
{
    if (!h) return CLUSCO_ERR_INVALID_ARG;
    h->last_error.clear();
    if (!cfg) {
        h->forced = false;
    } else {
        if ((cfg->products != 3 && cfg->products != 4) ||
            (cfg->schedule != CLUSCO_SCHED_STAGED && cfg->schedule != CLUSCO_SCHED_PERSISTENT) ||
            cfg->band < 1 || cfg->band > 256 || (cfg->frame != 0 && cfg->frame != 1))
            return fail(h, CLUSCO_ERR_INVALID_ARG,
                        "need products 3 or 4, a known schedule, band in 1..256, frame 0 or 1");
        h->forced = true;
        h->force = KernelCfg{};
        h->force.products = cfg->products;
        h->force.schedule = cfg->schedule;
        h->force.band = cfg->band;
        h->force.frame = cfg->frame;
    }
    ++h->tune_gen;
    return CLUSCO_OK;
}

const char *clusco_tuning_path(clusco_handle h)
{
    return h ? h->tune.path.c_str() : "";
}

void clusco_destroy(clusco_handle h)
{
    if (!h) return;
    {
        DeviceGuard g(h->device);
        for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
        for (BatchPlan &p : h->plans) free_plan(p);
        if (h->capture) (void)hipStreamDestroy(h->capture);
    }
    delete h;
}

const char *clusco_last_error(clusco_handle h) { return h ? h->last_error.c_str() : ""; }

clusco_status clusco_set_tolerance(clusco_handle h, clusco_precision p, double tol)
{
    if (!h) return CLUSCO_ERR_INVALID_ARG;
    if (!valid_precision(p)) return fail(h, CLUSCO_ERR_UNSUPPORTED, "unknown precision");
    h->tol[mode_of(p)] = tol;
    return CLUSCO_OK;
}

clusco_status clusco_flag_epsilon(clusco_handle h, clusco_precision p, int64_t L, double *eps)
{
    if (!h || !eps) return CLUSCO_ERR_INVALID_ARG;
    if (!valid_precision(p)) return fail(h, CLUSCO_ERR_UNSUPPORTED, "unknown precision");
    if (L < 1) return fail(h, CLUSCO_ERR_INVALID_ARG, "need L >= 1");
    *eps = contraction_eps(mode_of(p), L);
    return CLUSCO_OK;
}

size_t clusco_crmsd_workspace_size(clusco_handle h, int64_t N, int64_t L, clusco_precision p)
{
    if (!h || N < 0 || N > MAX_N || L < 1 || !valid_precision(p)) return 0;
    return single_layout(h, mode_of(p), N, L).total;
}

clusco_status clusco_crmsd_matrix(clusco_handle h, const float *coords, int64_t N, int64_t L,
                                  clusco_precision p, float *out, void *ws, size_t ws_bytes,
                                  void *stream)
{
    if (!h) return CLUSCO_ERR_INVALID_ARG;
    h->last_error.clear();
    if (!valid_precision(p)) return fail(h, CLUSCO_ERR_UNSUPPORTED, "unknown precision");
    if (N < 0 || L < 1) return fail(h, CLUSCO_ERR_INVALID_ARG, "need N >= 0 and L >= 1");
    if (N > MAX_N) return fail(h, CLUSCO_ERR_UNSUPPORTED, "N above 2^20");
    if (N < 2) return CLUSCO_OK;
    if (!coords || !out) return fail(h, CLUSCO_ERR_INVALID_ARG, "null coords or out");
    if (!aligned(coords, 4) || !aligned(out, 4))
        return fail(h, CLUSCO_ERR_INVALID_ARG, "coords and out must be 4-byte aligned");
    const int mode = mode_of(p);
    const SingleLayout s = single_layout(h, mode, N, L);
    if (!ws || ws_bytes < s.total) return fail(h, CLUSCO_ERR_WORKSPACE, "workspace too small");
    if (!aligned(ws, 256)) return fail(h, CLUSCO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
    return enqueue(h, mode, coords, coords, (char *)ws, out, &s, nullptr, TK_SYM,
                   (hipStream_t)stream, true);
}

clusco_status clusco_crmsd_matrix_noalloc(clusco_handle h, const float *coords, int64_t N,
                                          int64_t L, clusco_precision p, float *out, void *stream)
{
    if (!h) return CLUSCO_ERR_INVALID_ARG;
    h->last_error.clear();
    if (!valid_precision(p)) return fail(h, CLUSCO_ERR_UNSUPPORTED, "unknown precision");
    if (N < 0 || L < 1) return fail(h, CLUSCO_ERR_INVALID_ARG, "need N >= 0 and L >= 1");
    if (N > MAX_N) return fail(h, CLUSCO_ERR_UNSUPPORTED, "N above 2^20");
    if (N < 2) return CLUSCO_OK;
    if (!coords || !out) return fail(h, CLUSCO_ERR_INVALID_ARG, "null coords or out");
    if (!aligned(coords, 4) || !aligned(out, 4))
        return fail(h, CLUSCO_ERR_INVALID_ARG, "coords and out must be 4-byte aligned");
    const int mode = mode_of(p);
    const SingleLayout s = single_layout(h, mode, N, L);
    if (s.total > (size_t)CLUSCO_SCRATCH_BYTES)
        return fail(h, CLUSCO_ERR_UNSUPPORTED,
                    "workspace for these N, L exceeds the built-in scratch (CLUSCO_SCRATCH_BYTES); "
                    "use clusco_crmsd_matrix with a caller workspace");
    if (h->scratch_err != hipSuccess || !h->scratch)
        return hip_fail(h, h->scratch_err != hipSuccess ? h->scratch_err : hipErrorInvalidSymbol,
                        "built-in scratch address");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
    // the prep kernel zeroes the counters at the head of the scratch; nothing
    // else in it needs to start at zero
    return enqueue(h, mode, coords, coords, (char *)h->scratch, out, &s, nullptr, TK_SYM,
                   (hipStream_t)stream, true);
}

clusco_status clusco_fixup_count(clusco_handle h, const void *ws, int64_t *count, void *stream)
{
    if (!h || !ws || !count) return CLUSCO_ERR_INVALID_ARG;
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
    int v = 0;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(&v, ws, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "read fix-up counter");
    *count = v;
    return CLUSCO_OK;
}

clusco_status clusco_stage_timing(clusco_handle h, int max_calls)
{
    if (!h || max_calls < 0) return CLUSCO_ERR_INVALID_ARG;
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    h->events.clear();
    h->slots = h->used = 0;
    for (int k = 0; k < 4 * max_calls; ++k) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return hip_fail(h, err, "create timing events");
        h->events.push_back(e);
    }
    h->slots = max_calls;
    return CLUSCO_OK;
}

clusco_status clusco_stage_times(clusco_handle h, double ms[3], int *calls)
{
    if (!h || !ms || !calls) return CLUSCO_ERR_INVALID_ARG;
    ms[0] = ms[1] = ms[2] = 0.0;
    *calls = h->used;
    if (h->used == 0) return CLUSCO_OK;
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
    hipError_t err = hipEventSynchronize(h->events[4 * h->used - 1]);
    if (err != hipSuccess) return hip_fail(h, err, "wait for timing events");
    for (int c = 0; c < h->used; ++c) {
        for (int k = 0; k < 3; ++k) {
            float t = 0.0f;
            err = hipEventElapsedTime(&t, h->events[4 * c + k], h->events[4 * c + k + 1]);
            if (err != hipSuccess) return hip_fail(h, err, "read timing events");
            ms[k] += t;
        }
    }
    h->used = 0;
    return CLUSCO_OK;
}

// ------------------------------------------------------------- batched

size_t clusco_crmsd_batched_workspace_size(clusco_handle h, int32_t E, const int64_t *h_N,
                                           const int64_t *h_L, clusco_precision p)
{
    if (!h || !valid_precision(p)) return 0;
    BatchInput b{E, h_N, h_L, nullptr, nullptr};
    if (check_batch(h, b, false) != CLUSCO_OK) return 0;
    return plan_layout(h, mode_of(p), b, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
}

clusco_status clusco_crmsd_batched(clusco_handle h, int32_t E, const int64_t *h_N,
                                   const int64_t *h_L, const int64_t *h_coord_off,
                                   const int64_t *h_out_off, const float *coords,
                                   clusco_precision p, float *out, void *ws, size_t ws_bytes,
                                   void *stream)
{
    if (!h) return CLUSCO_ERR_INVALID_ARG;
    h->last_error.clear();
    if (!valid_precision(p)) return fail(h, CLUSCO_ERR_UNSUPPORTED, "unknown precision");
    BatchInput b{E, h_N, h_L, h_coord_off, h_out_off};
    clusco_status st = check_batch(h, b, true);
    if (st != CLUSCO_OK || E == 0) return st;
    bool work = false;
    for (int32_t e = 0; e < E; ++e) work |= h_N[e] >= 2;
    if (!work) return CLUSCO_OK;
    if (!coords || !out) return fail(h, CLUSCO_ERR_INVALID_ARG, "null coords or out");
    if (!aligned(coords, 4) || !aligned(out, 4))
        return fail(h, CLUSCO_ERR_INVALID_ARG, "coords and out must be 4-byte aligned");
    const int mode = mode_of(p);
    const size_t need =
        plan_layout(h, mode, b, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    if (!ws || ws_bytes < need) return fail(h, CLUSCO_ERR_WORKSPACE, "workspace too small");
    if (!aligned(ws, 256)) return fail(h, CLUSCO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");

    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
    hipStream_t s = (hipStream_t)stream;

    // Inside the caller's own graph capture nothing may allocate or copy
    // synchronously: the plan must already exist (an earlier call with the
    // same shapes), and it is pinned because the caller's graph keeps its
    // table address.  Otherwise launches are direct while stage timing
    // records, else the plan's own graph is replayed (captured first).
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cs);
    if (e != hipSuccess) return hip_fail(h, e, "query stream capture");
    std::vector<int64_t> key = batch_key(h, mode, b, true);
    BatchPlan *plan = find_plan(h, key);
    if (cs != hipStreamCaptureStatusNone) {
        if (!plan)
            return fail(h, CLUSCO_ERR_UNSUPPORTED,
                        "no cached plan for these shapes under graph capture: make one call "
                        "with the same shapes outside the capture first");
        plan->pinned = true;
        return enqueue(h, mode, coords, coords, (char *)ws, out, nullptr, plan, TK_BATCH, s,
                       false);
    }
    if (!plan) {
        st = create_plan(h, mode, b, std::move(key), &plan);
        if (st != CLUSCO_OK) return st;
    }
    const bool timing = h->used < h->slots;
    if (timing)
        return enqueue(h, mode, coords, coords, (char *)ws, out, nullptr, plan, TK_BATCH, s,
                       timing);

    if (!plan->exec || plan->g_coords != coords || plan->g_out != out || plan->g_ws != ws) {
        if (plan->exec) {
            (void)hipGraphExecDestroy(plan->exec);
            plan->exec = nullptr;
        }
        if (!h->capture) {
            e = hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(h, e, "create capture stream");
        }
        e = hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(h, e, "begin capture");
        st = enqueue(h, mode, coords, coords, (char *)ws, out, nullptr, plan, TK_BATCH,
                     h->capture, false);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(h->capture, &graph);
        if (st != CLUSCO_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return hip_fail(h, e, "end capture");
        e = hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            plan->exec = nullptr;
            return hip_fail(h, e, "instantiate graph");
        }
        plan->g_coords = coords;
        plan->g_out = out;
        plan->g_ws = ws;
    }
    e = hipGraphLaunch(plan->exec, s);
    if (e != hipSuccess) return hip_fail(h, e, "graph launch");
    return CLUSCO_OK;
}

// ------------------------------------------------------------------ cross

size_t clusco_crmsd_cross_workspace_size(clusco_handle h, int64_t Na, int64_t Nb, int64_t L,
                                         clusco_precision p)
{
    if (!h || Na < 0 || Nb < 0 || Na > MAX_N || Nb > MAX_N || L < 1 || !valid_precision(p))
        return 0;
    return cross_layout(h, mode_of(p), Na, Nb, L).total;
}

clusco_status clusco_crmsd_cross(clusco_handle h, const float *A, int64_t Na, const float *B,
                                 int64_t Nb, int64_t L, clusco_precision p, float *out,
                                 void *ws, size_t ws_bytes, void *stream)
{
    if (!h) return CLUSCO_ERR_INVALID_ARG;
    h->last_error.clear();
    if (!valid_precision(p)) return fail(h, CLUSCO_ERR_UNSUPPORTED, "unknown precision");
    if (Na < 0 || Nb < 0 || L < 1) return fail(h, CLUSCO_ERR_INVALID_ARG, "need Na, Nb >= 0, L >= 1");
    if (Na > MAX_N || Nb > MAX_N) return fail(h, CLUSCO_ERR_UNSUPPORTED, "set above 2^20 models");
    if (Na == 0 || Nb == 0) return CLUSCO_OK;
    if (!A || !B || !out) return fail(h, CLUSCO_ERR_INVALID_ARG, "null A, B or out");
    if (!aligned(A, 4) || !aligned(B, 4) || !aligned(out, 4))
        return fail(h, CLUSCO_ERR_INVALID_ARG, "A, B and out must be 4-byte aligned");
    const int mode = mode_of(p);
    const SingleLayout s = cross_layout(h, mode, Na, Nb, L);
    if (!ws || ws_bytes < s.total) return fail(h, CLUSCO_ERR_WORKSPACE, "workspace too small");
    if (!aligned(ws, 256)) return fail(h, CLUSCO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
    return enqueue(h, mode, A, B, (char *)ws, out, &s, nullptr, TK_RECT, (hipStream_t)stream,
                   true);
}

// --------------------------------------------------------------- backward

size_t clusco_crmsd_backward_workspace_size(clusco_handle h, int64_t N, int64_t L,
                                            clusco_precision p)
{
    if (!h || N < 0 || N > MAX_N || L < 1 || !valid_precision(p)) return 0;
    return bwd_layout(h, mode_of(p), N, N, L, false).total;
}

clusco_status clusco_crmsd_backward(clusco_handle h, const float *coords, int64_t N, int64_t L,
                                    const float *rmsd, const float *grad_out,
                                    clusco_precision p, float *grad_coords, void *ws,
                                    size_t ws_bytes, void *stream)
{
    if (!h) return CLUSCO_ERR_INVALID_ARG;
    h->last_error.clear();
    if (!valid_precision(p)) return fail(h, CLUSCO_ERR_UNSUPPORTED, "unknown precision");
    if (N < 0 || L < 1) return fail(h, CLUSCO_ERR_INVALID_ARG, "need N >= 0 and L >= 1");
    if (N > MAX_N) return fail(h, CLUSCO_ERR_UNSUPPORTED, "N above 2^20");
    if (N == 0) return CLUSCO_OK;
    if (!grad_coords || !aligned(grad_coords, 4))
        return fail(h, CLUSCO_ERR_INVALID_ARG, "grad_coords null or misaligned");
    hipStream_t s = (hipStream_t)stream;
    if (N == 1) {
        DeviceGuard g(h->device);
        if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
        hipError_t e = launch_zero(grad_coords, 3 * L, s);
        return e == hipSuccess ? CLUSCO_OK : hip_fail(h, e, "zero launch");
    }
    if (!coords || !rmsd || !grad_out)
        return fail(h, CLUSCO_ERR_INVALID_ARG, "null coords, rmsd or grad_out");
    if (!aligned(coords, 4) || !aligned(rmsd, 4) || !aligned(grad_out, 4))
        return fail(h, CLUSCO_ERR_INVALID_ARG, "inputs must be 4-byte aligned");
    const int mode = mode_of(p);
    const BwdLayout b = bwd_layout(h, mode, N, N, L, false);
    if (!ws || ws_bytes < b.total) return fail(h, CLUSCO_ERR_WORKSPACE, "workspace too small");
    if (!aligned(ws, 256)) return fail(h, CLUSCO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
    return enqueue_bwd(h, mode, coords, coords, (char *)ws, b, false, rmsd, grad_out, grad_coords,
                       nullptr, s);
}

size_t clusco_crmsd_cross_backward_workspace_size(clusco_handle h, int64_t Na, int64_t Nb,
                                                  int64_t L, clusco_precision p)
{
    if (!h || Na < 0 || Nb < 0 || Na > MAX_N || Nb > MAX_N || L < 1 || !valid_precision(p))
        return 0;
    return bwd_layout(h, mode_of(p), Na, Nb, L, true).total;
}

clusco_status clusco_crmsd_cross_backward(clusco_handle h, const float *A, int64_t Na,
                                          const float *B, int64_t Nb, int64_t L,
                                          const float *rmsd, const float *grad_out,
                                          clusco_precision p, float *grad_A, float *grad_B,
                                          void *ws, size_t ws_bytes, void *stream)
{
    if (!h) return CLUSCO_ERR_INVALID_ARG;
    h->last_error.clear();
    if (!valid_precision(p)) return fail(h, CLUSCO_ERR_UNSUPPORTED, "unknown precision");
    if (Na < 0 || Nb < 0 || L < 1) return fail(h, CLUSCO_ERR_INVALID_ARG, "need Na, Nb >= 0, L >= 1");
    if (Na > MAX_N || Nb > MAX_N) return fail(h, CLUSCO_ERR_UNSUPPORTED, "set above 2^20 models");
    if ((Na > 0 && !grad_A) || !aligned(grad_A, 4) || !aligned(grad_B, 4))
        return fail(h, CLUSCO_ERR_INVALID_ARG, "grad_A null or gradients misaligned");
    hipStream_t s = (hipStream_t)stream;
    if (Na == 0 || Nb == 0) {
        DeviceGuard g(h->device);
        if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
        hipError_t e = launch_zero(grad_A, 3 * L * Na, s);
        if (e == hipSuccess && grad_B) e = launch_zero(grad_B, 3 * L * Nb, s);
        return e == hipSuccess ? CLUSCO_OK : hip_fail(h, e, "zero launch");
    }
    if (!A || !B || !rmsd || !grad_out)
        return fail(h, CLUSCO_ERR_INVALID_ARG, "null A, B, rmsd or grad_out");
    if (!aligned(A, 4) || !aligned(B, 4) || !aligned(rmsd, 4) || !aligned(grad_out, 4))
        return fail(h, CLUSCO_ERR_INVALID_ARG, "inputs must be 4-byte aligned");
    const int mode = mode_of(p);
    const BwdLayout b = bwd_layout(h, mode, Na, Nb, L, true);
    if (!ws || ws_bytes < b.total) return fail(h, CLUSCO_ERR_WORKSPACE, "workspace too small");
    if (!aligned(ws, 256)) return fail(h, CLUSCO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
    return enqueue_bwd(h, mode, A, B, (char *)ws, b, true, rmsd, grad_out, grad_A, grad_B, s);
}

// -------------------------------------------------------------- threshold

namespace {

struct ThrLayout {
    SingleLayout s;
    size_t off_masks, total;
};

static ThrLayout thr_layout(clusco_handle h, int mode, int64_t N, int64_t L)
{
    ThrLayout t{};
    t.s = single_layout(h, mode, N, L);
    size_t o = t.s.total;
    t.off_masks = take(o, sizeof(uint32_t) * 32 * problem_wtiles(t.s.p));
    t.total = o;
    return t;
}

} // namespace

size_t clusco_crmsd_threshold_workspace_size(clusco_handle h, int64_t N, int64_t L,
                                             clusco_precision p)
{
    if (!h || N < 0 || N > MAX_N || L < 1 || !valid_precision(p)) return 0;
    return thr_layout(h, mode_of(p), N, L).total;
}

clusco_status clusco_crmsd_threshold(clusco_handle h, const float *coords, int64_t N, int64_t L,
                                     clusco_precision p, float cutoff, int32_t *out_i,
                                     int32_t *out_j, float *out_score, int64_t capacity,
                                     uint64_t *count, void *ws, size_t ws_bytes, void *stream)
{
    if (!h) return CLUSCO_ERR_INVALID_ARG;
    h->last_error.clear();
    if (!valid_precision(p)) return fail(h, CLUSCO_ERR_UNSUPPORTED, "unknown precision");
    if (N < 0 || L < 1 || capacity < 0 || !(cutoff == cutoff))
        return fail(h, CLUSCO_ERR_INVALID_ARG, "need N >= 0, L >= 1, capacity >= 0, cutoff not NaN");
    if (N > MAX_N) return fail(h, CLUSCO_ERR_UNSUPPORTED, "N above 2^20");
    if (!count || !aligned(count, 8)) return fail(h, CLUSCO_ERR_INVALID_ARG, "count null or misaligned");
    hipStream_t st = (hipStream_t)stream;
    if (N < 2) {
        DeviceGuard g(h->device);
        if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
        hipError_t e = launch_zero((float *)count, 2, st);
        return e == hipSuccess ? CLUSCO_OK : hip_fail(h, e, "zero launch");
    }
    if (!coords || !aligned(coords, 4)) return fail(h, CLUSCO_ERR_INVALID_ARG, "coords null or misaligned");
    if (capacity > 0 && (!out_i || !out_j || !out_score || !aligned(out_i, 4) ||
                         !aligned(out_j, 4) || !aligned(out_score, 4)))
        return fail(h, CLUSCO_ERR_INVALID_ARG, "output arrays null or misaligned");
    const int mode = mode_of(p);
    const ThrLayout t = thr_layout(h, mode, N, L);
    if (!ws || ws_bytes < t.total) return fail(h, CLUSCO_ERR_WORKSPACE, "workspace too small");
    if (!aligned(ws, 256)) return fail(h, CLUSCO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
    char *w = (char *)ws;
    Emit em{};
    em.cutoff = cutoff;
    em.i = out_i;
    em.j = out_j;
    em.score = out_score;
    em.capacity = capacity;
    em.count = (unsigned long long *)count;
    em.masks = (uint32_t *)(w + t.off_masks);

    stage_mark(h, 0, st);
    PrepLaunch pl{};
    pl.XA = pl.XB = coords;
    pl.ws = w;
    pl.mode = mode;
    pl.counters = (int *)w;
    pl.zero64 = em.count;
    pl.set[0] = pl.set[1] = t.s.A;
    pl.nset = 1;
    pl.total = t.s.A.Np;
    hipError_t e = launch_prep(pl, st);
    if (e != hipSuccess) return hip_fail(h, e, "prep launch");
    stage_mark(h, 1, st);
    FixupLaunch fl{};
    fl.XA = fl.XB = coords;
    fl.ws = w;
    fl.prob = t.s.p;
    fl.nprob = 1;
    fl.counters = (int *)w;
    fl.list = (FixEntry *)(w + t.s.off_list);
    fl.thr = 1;
    fl.emit = em;
    if (mode != MODE_FP64) {
        TileLaunch tl{};
        tl.ws = w;
        tl.prob = t.s.p;
        tl.nprob = 1;
        tl.kind = TK_SYM;
        tl.T = problem_tiles(t.s.p);
        tl.counters = (int *)w;
        tl.list = (FixEntry *)(w + t.s.off_list);
        tl.emit = em;
        e = launch_tile(t.s.emode, tl, st, OP_THR);
        if (e != hipSuccess) return hip_fail(h, e, "threshold tile launch");
        stage_mark(h, 2, st);
        if (t.s.p.flag_coef > 0.0) {
            e = launch_fixup(fl, st);
            if (e != hipSuccess) return hip_fail(h, e, "fix-up launch");
        }
    } else {
        stage_mark(h, 2, st);
        fl.all = 1;
        fl.n_all = problem_wtiles(t.s.p);
        e = launch_fixup(fl, st);
        if (e != hipSuccess) return hip_fail(h, e, "fp64 launch");
    }
    stage_mark(h, 3, st);
    return CLUSCO_OK;
}

// ---------------------------------------------------------------- dRMSD

namespace {

constexpr int64_t MAX_DIST_L = 4096;   // atom pairs are packed as two 16-bit indices

struct DistLayout {
    DistLaunch d;
    size_t total;
};

// Every non-FP64 mode accumulates the Gram products in FP32, one rounding per
// MFMA step: K/2 steps (FP32), 3K/16 (split) or 4K/16 (split x4).  For a pair
// of similar models the partial sums grow linearly to about E, so the
// rounding errors add up to about eps E with eps = 2^-24 sqrt(steps / 3).  A
// pair is flagged when eps (E_i + E_j) / (K score) could exceed tol / 2 (a
// margin of four on the first-order score error eps (E_i + E_j) / (2 K score)).
static double dist_flag_coef(clusco_handle h, int mode, int64_t K)
{
    const double tol = h->tol[mode];
    if (mode == MODE_FP64 || !(tol > 0.0) || K < 1) return -1.0;
    const double steps = mode == MODE_FP32     ? K / 2.0
                         : mode == MODE_BF16X4 ? K / 4.0
                                               : 3.0 * K / 16.0;
    const double eps = std::ldexp(1.0, -24) * std::sqrt(steps / 3.0);
    return 2.0 * eps / ((double)K * tol);
}

static DistLayout dist_layout(clusco_handle h, int mode, int64_t N, int64_t L)
{
    DistLayout r{};
    DistLaunch &d = r.d;
    d.N = N;
    d.Np = round_up(N > 0 ? N : 1, 256);   // whole 256-model tiles of operands
    d.L = L;
    d.K = L * (L - 1) / 2;
    d.Kp = round_up(d.K > 0 ? d.K : 1, 16);
    d.KB = d.Kp / kblock(mode == MODE_FP64 ? MODE_BF16 : mode);
    d.nref = N < 256 ? N : 256;
    d.nb = d.Np / 256;
    d.T = tri_count(d.nb);
    d.nrb = d.Np / ROWBLK;
    size_t o = 256;
    d.off_c = (int64_t)take(o, sizeof(double) * d.Kp);
    d.off_pq = (int64_t)take(o, sizeof(uint32_t) * d.Kp);
    d.off_E = (int64_t)take(o, sizeof(double) * d.Np);
    d.off_ops = mode == MODE_FP64 ? 0 : (int64_t)take(o, (size_t)4 * d.Np * d.Kp);
    const size_t off_list = take(o, sizeof(FixEntry) * tri_count(d.nrb));
    d.all = mode == MODE_FP64;
    d.flag_coef = h ? dist_flag_coef(h, mode, d.K) : -1.0;
    d.list = (FixEntry *)off_list;   // relative until the workspace is known
    r.total = o;
    return r;
}

} // namespace

size_t clusco_drmsd_workspace_size(clusco_handle h, int64_t N, int64_t L, clusco_precision p)
{
    if (!h || N < 0 || N > MAX_N || L < 1 || L > MAX_DIST_L || !valid_precision(p)) return 0;
    return dist_layout(h, mode_of(p), N, L).total;
}

clusco_status clusco_drmsd_matrix(clusco_handle h, const float *coords, int64_t N, int64_t L,
                                  clusco_precision p, float *out, void *ws, size_t ws_bytes,
                                  void *stream)
{
    if (!h) return CLUSCO_ERR_INVALID_ARG;
    h->last_error.clear();
    if (!valid_precision(p)) return fail(h, CLUSCO_ERR_UNSUPPORTED, "unknown precision");
    if (N < 0 || L < 1) return fail(h, CLUSCO_ERR_INVALID_ARG, "need N >= 0 and L >= 1");
    if (N > MAX_N) return fail(h, CLUSCO_ERR_UNSUPPORTED, "N above 2^20");
    if (L > MAX_DIST_L) return fail(h, CLUSCO_ERR_UNSUPPORTED, "L above 4096");
    if (N < 2) return CLUSCO_OK;
    if (!coords || !out) return fail(h, CLUSCO_ERR_INVALID_ARG, "null coords or out");
    if (!aligned(coords, 4) || !aligned(out, 4))
        return fail(h, CLUSCO_ERR_INVALID_ARG, "coords and out must be 4-byte aligned");
    const int mode = mode_of(p);
    DistLayout r = dist_layout(h, mode, N, L);
    if (!ws || ws_bytes < r.total) return fail(h, CLUSCO_ERR_WORKSPACE, "workspace too small");
    if (!aligned(ws, 256)) return fail(h, CLUSCO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
    hipStream_t st = (hipStream_t)stream;
    if (L == 1) {
        hipError_t e = launch_zero(out, N * (N - 1) / 2, st);
        return e == hipSuccess ? CLUSCO_OK : hip_fail(h, e, "zero launch");
    }
    DistLaunch &d = r.d;
    d.X = coords;
    d.ws = (char *)ws;
    d.out = out;
    d.counters = (int *)ws;
    d.list = (FixEntry *)((char *)ws + (size_t)d.list);
    stage_mark(h, 0, st);
    hipError_t e = launch_dist_prep(mode, d, st);
    if (e != hipSuccess) return hip_fail(h, e, "dRMSD prep launch");
    stage_mark(h, 1, st);
    if (mode != MODE_FP64) {
        e = launch_dist_tile(mode, d, st);
        if (e != hipSuccess) return hip_fail(h, e, "dRMSD tile launch");
    }
    stage_mark(h, 2, st);
    if (d.all || d.flag_coef > 0.0) {
        e = launch_dist_fixup(d, st);
        if (e != hipSuccess) return hip_fail(h, e, "dRMSD fix-up launch");
    }
    stage_mark(h, 3, st);
    return CLUSCO_OK;
}

// ----------------------------------------------------------------- CMO

namespace {

struct CmoLayout {
    CmoLaunch c;
    size_t total;
};

static CmoLayout cmo_layout(int64_t N, int64_t L)
{
    CmoLayout r{};
    CmoLaunch &c = r.c;
    c.N = N;
    c.Np = round_up(N > 0 ? N : 1, 256);
    c.L = L;
    c.K = L * (L - 1) / 2;
    c.Kp = round_up(c.K > 0 ? c.K : 1, 32);
    c.KB = c.Kp / 32;
    c.nb = c.Np / 256;
    c.T = tri_count(c.nb);
    size_t o = 256;
    c.off_pq = (int64_t)take(o, sizeof(uint32_t) * c.Kp);
    c.off_n = (int64_t)take(o, sizeof(int32_t) * c.Np);
    c.off_ops = (int64_t)take(o, (size_t)c.Np * c.Kp);
    r.total = o;
    return r;
}

} // namespace

size_t clusco_cmo_workspace_size(clusco_handle h, int64_t N, int64_t L)
{
    if (!h || N < 0 || N > MAX_N || L < 1 || L > MAX_DIST_L) return 0;
    return cmo_layout(N, L).total;
}

clusco_status clusco_cmo_matrix(clusco_handle h, const float *coords, int64_t N, int64_t L,
                                float cutoff, float *out, void *ws, size_t ws_bytes, void *stream)
{
    if (!h) return CLUSCO_ERR_INVALID_ARG;
    h->last_error.clear();
    if (N < 0 || L < 1) return fail(h, CLUSCO_ERR_INVALID_ARG, "need N >= 0 and L >= 1");
    if (!(cutoff >= 0.0f) || !std::isfinite(cutoff))
        return fail(h, CLUSCO_ERR_INVALID_ARG, "cutoff must be finite and >= 0");
    if (N > MAX_N) return fail(h, CLUSCO_ERR_UNSUPPORTED, "N above 2^20");
    if (L > MAX_DIST_L) return fail(h, CLUSCO_ERR_UNSUPPORTED, "L above 4096");
    if (N < 2) return CLUSCO_OK;
    if (!coords || !out) return fail(h, CLUSCO_ERR_INVALID_ARG, "null coords or out");
    if (!aligned(coords, 4) || !aligned(out, 4))
        return fail(h, CLUSCO_ERR_INVALID_ARG, "coords and out must be 4-byte aligned");
    CmoLayout r = cmo_layout(N, L);
    if (!ws || ws_bytes < r.total) return fail(h, CLUSCO_ERR_WORKSPACE, "workspace too small");
    if (!aligned(ws, 256)) return fail(h, CLUSCO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
    hipStream_t st = (hipStream_t)stream;
    if (L == 1) {
        hipError_t e = launch_zero(out, N * (N - 1) / 2, st);
        return e == hipSuccess ? CLUSCO_OK : hip_fail(h, e, "zero launch");
    }
    CmoLaunch &c = r.c;
    c.X = coords;
    c.ws = (char *)ws;
    c.out = out;
    c.cutoff = cutoff;
    stage_mark(h, 0, st);
    stage_mark(h, 1, st);
    hipError_t e = launch_cmo(c, st);
    if (e != hipSuccess) return hip_fail(h, e, "CMO launch");
    stage_mark(h, 2, st);
    stage_mark(h, 3, st);
    return CLUSCO_OK;
}

// ---------------------------------------------------------- clustering

size_t clusco_cluster_workspace_size(clusco_handle h, int64_t N, int32_t k)
{
    if (!h || N < 1 || N > MAX_N || k < 1 || k > N) return 0;
    return 256 + (size_t)round_up(8 * N, 256);
}

clusco_status clusco_kmedoids(clusco_handle h, const float *D, int64_t N, int32_t k,
                              const int32_t *h_init, int32_t max_iter, int32_t check_every,
                              int32_t *labels, int32_t *medoids, int64_t *sizes, double *mean_r,
                              int64_t *info, void *ws, size_t ws_bytes, void *stream)
{
    if (!h) return CLUSCO_ERR_INVALID_ARG;
    h->last_error.clear();
    if (N < 1 || k < 1 || k > N || max_iter < 0 || max_iter > 100000 || check_every < 0)
        return fail(h, CLUSCO_ERR_INVALID_ARG,
                    "need 1 <= k <= N, 0 <= max_iter <= 100000 and check_every >= 0");
    if (N > MAX_N) return fail(h, CLUSCO_ERR_UNSUPPORTED, "N above 2^20");
    if (!h_init) return fail(h, CLUSCO_ERR_INVALID_ARG, "null initial medoids");
    {
        std::vector<int32_t> v(h_init, h_init + k);
        std::sort(v.begin(), v.end());
        if (v.front() < 0 || v.back() >= N || std::adjacent_find(v.begin(), v.end()) != v.end())
            return fail(h, CLUSCO_ERR_INVALID_ARG, "initial medoids must be distinct models in [0, N)");
    }
    if ((N > 1 && !D) || !labels || !medoids || !sizes || !mean_r || !info)
        return fail(h, CLUSCO_ERR_INVALID_ARG, "null matrix or output");
    if (!aligned(D, 4) || !aligned(labels, 4) || !aligned(medoids, 4) || !aligned(sizes, 8) ||
        !aligned(mean_r, 8) || !aligned(info, 8))
        return fail(h, CLUSCO_ERR_INVALID_ARG, "misaligned matrix or output");
    const size_t need = clusco_cluster_workspace_size(h, N, k);
    if (!ws || ws_bytes < need) return fail(h, CLUSCO_ERR_WORKSPACE, "workspace too small");
    if (!aligned(ws, 256)) return fail(h, CLUSCO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    DeviceGuard g(h->device);
    if (g.err != hipSuccess) return hip_fail(h, g.err, "set device");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(medoids, h_init, sizeof(int32_t) * k, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(h, e, "copy initial medoids");
    ClusterLaunch a{};
    a.D = D;
    a.N = N;
    a.k = k;
    a.medoid = medoids;
    a.label = labels;
    a.state = (int *)ws;
    a.cost = (long long *)((char *)ws + 256);
    a.size = (long long *)sizes;
    a.mean_r = mean_r;
    a.info = (long long *)info;
    e = launch_cluster_begin(a, st);
    if (e != hipSuccess) return hip_fail(h, e, "clustering launch");
    if (check_every == 0) {
        e = launch_cluster_iters(a, max_iter, st);
        if (e != hipSuccess) return hip_fail(h, e, "clustering launch");
    } else {
        for (int32_t done = 0; done < max_iter;) {
            const int32_t n = std::min(check_every, max_iter - done);
            e = launch_cluster_iters(a, n, st);
            if (e != hipSuccess) return hip_fail(h, e, "clustering launch");
            done += n;
            int flag = 0;
            e = hipMemcpyAsync(&flag, a.state, sizeof(int), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) return hip_fail(h, e, "read convergence flag");
            if (flag) break;
        }
    }
    e = launch_cluster_end(a, st);
    return e == hipSuccess ? CLUSCO_OK : hip_fail(h, e, "clustering launch");
}

} // extern "C"
