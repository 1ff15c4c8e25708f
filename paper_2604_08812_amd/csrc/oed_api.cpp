// liboed C ABI: context, greedy loop and queries (declarations and contract in include/oed.h).
//
// The host enqueues the whole greedy loop without synchronising: the number
// of remaining candidates after k picks is known on the host, the identity of
// each pick stays on the device (active list, last pick, status word) and is
// read back once per call.  All device memory is allocated in oed_create.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/oed.h"
#include "oed_internal.h"

using namespace oed;

namespace {

const int NKC = OED_K_COUNT;

struct EvPair {
    hipEvent_t a, b;
};

}  // namespace

struct oed_ctx {
    // problem
    int N_s = 0, N_c = 0, N_t = 0, N_tp = 0;
    int kdtype = 0;
    int64_t ld = 0;
    double sigma2 = 0, half_noise = 0;
    int prec = OED_PREC_FP64;
    int rtype = R_F64, wtype = W_F64;
    int syrk_variant = SYRK_LDS;
    int fixed_variant = -1;  // oed_options.tile_size: the downdate kernel the tuner must keep (-1: free)
    int stl = STL_COL4;  // downdate super-tile order (see super_tile())
    int delay = 1;  // > 1: up to delay - 1 block columns held and subtracted with the next one
    double tuned_ms[MAX_DELAY] = {0};  // autotuner: estimated time per pick for delay 1..MAX_DELAY
    // left-looking: R keeps K off the diagonal; W slot k holds pick k's block column
    bool left = false;
    int max_budget = 0;
    bool diag_current = true;  // the diagonal blocks include every formed block column
    // right-looking, N_t <= REGS_MAX_NT: the diagonal blocks are kept current eagerly (the block
    // column kernel subtracts each new column from them in place, fuse_diag) and the downdate
    // skips them, so the gains never carry the held columns
    bool eager = false;
    int newest = -1;  // W slot of the block column the diagonal blocks do not include yet (the
                      // gain launch applies it; only where fuse_diag does not hold)
    void *C = nullptr;         // column partial sums (LEFT_SPLITS x N_c blocks, R's type)
    double *noise_h = nullptr; // per-sensor noise terms by local index (device), or null
    uint32_t flags = 0;
    std::string tune_cache;  // autotuner cache file ("" = in-process only)
    int fail_step = 0;       // test hook: the fail_step-th pick since creation / reset fails once
    hipStream_t stream = nullptr;
    int device = 0;
    std::vector<int> cmap;  // local -> original sensor index (ascending)
    std::vector<int> lmap;  // original -> local (-1 = not a candidate)
    // device memory
    void *R = nullptr, *W = nullptr, *W2 = nullptr;  // `delay` W slots (BF16: hi, lo parts)
    int64_t wslot = 0;                               // elements per W slot
    double *V = nullptr;
    double *Linv = nullptr, *gains = nullptr, *pick_gain = nullptr, *scratch_gain = nullptr,
           *scratch_pick = nullptr, *fcache = nullptr;
    int *act[2] = {nullptr, nullptr}, *picks = nullptr, *state = nullptr, *dcmap = nullptr;
    int64_t dev_bytes = 0;
    // host mirror of the selection
    int cur = 0;       // which act buffer is current
    int n_act = 0;     // remaining candidates
    int k = 0;         // picks made
    bool pending = false;  // the last pick's block column and downdate are not formed yet
    int nheld = 0;         // block columns formed but not yet subtracted from R (W slots 0 .. nheld-1)
    bool poisoned = false;
    // OED_FLAG_DEFER_PACK: block rows filled by oed_pack_rows; steps need all of them
    bool deferred = false;
    std::vector<char> row_packed;  // by local index
    int unpacked = 0;
    std::vector<int> h_picks;   // local indices
    std::vector<double> h_gains;
    std::vector<char> picked;  // by local index
    // profiling
    std::vector<EvPair> ev_pool;
    std::vector<std::pair<int, int>> ev_used;  // (kernel class, pool index)
    double prof_ms[NKC] = {0};
    int64_t prof_n[NKC] = {0};
    double syrk_flops = 0, syrk_bytes = 0;
    std::string err;
};

namespace {

// Text of the calling thread's last failed oed_create (oed_last_error(NULL)).
thread_local std::string g_create_err;

oed_status fail(oed_ctx *h, oed_status st, const std::string &msg)
{
    if (h) h->err = msg;
    return st;
}

#define HIPCHK(h, call)                                                                                     \
    do {                                                                                                    \
        hipError_t e_ = (call);                                                                             \
        if (e_ != hipSuccess)                                                                               \
            return fail(h, e_ == hipErrorOutOfMemory ? OED_E_OOM : OED_E_HIP,                              \
                        std::string(#call) + ": " + hipGetErrorString(e_));                                 \
    } while (0)

size_t relem(const oed_ctx *h) { return h->rtype == R_F64 ? 8 : 4; }

hipError_t dmalloc(oed_ctx *h, void **p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) h->dev_bytes += (int64_t)bytes;
    return e;
}

// Event bracketing of one kernel launch when profiling.
struct Prof {
    oed_ctx *h;
    int cls;
    int idx = -1;
    Prof(oed_ctx *h_, int c) : h(h_), cls(c)
    {
        if (!(h->flags & OED_FLAG_PROFILE)) return;
        idx = (int)h->ev_used.size();
        if (idx >= (int)h->ev_pool.size()) {
            EvPair p;
            if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) {
                idx = -1;
                return;
            }
            h->ev_pool.push_back(p);
        }
        h->ev_used.push_back({cls, idx});
        (void)hipEventRecord(h->ev_pool[idx].a, h->stream);
    }
    ~Prof()
    {
        if (idx >= 0) (void)hipEventRecord(h->ev_pool[idx].b, h->stream);
    }
};

// Called after a stream synchronisation: fold the recorded events into the totals.
void collect_profile(oed_ctx *h)
{
    for (auto &u : h->ev_used) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, h->ev_pool[u.second].a, h->ev_pool[u.second].b) == hipSuccess) {
            h->prof_ms[u.first] += ms;
            h->prof_n[u.first] += 1;
        }
    }
    h->ev_used.clear();
}

void free_all(oed_ctx *h)
{
    void *ptrs[] = {h->R, h->W, h->W2, h->V, h->C, h->noise_h, h->Linv, h->gains, h->pick_gain, h->scratch_gain, h->scratch_pick,
                    h->fcache, h->act[0], h->act[1], h->picks, h->state, h->dcmap};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (auto &e : h->ev_pool) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    h->ev_pool.clear();
}

// Forget all picks: fresh active list and state words (the working copy is untouched).
oed_status reset_state(oed_ctx *h)
{
    HIPCHK(h, launch_init_state(h->act[0], h->N_c, h->state, h->stream));
    h->cur = 0;
    h->n_act = h->N_c;
    h->k = 0;
    h->pending = false;
    h->nheld = 0;
    h->diag_current = true;
    h->newest = -1;
    h->poisoned = false;
    h->h_picks.clear();
    h->h_gains.clear();
    h->picked.assign(h->N_c, 0);
    return OED_OK;
}

oed_status load_R(oed_ctx *h, const void *K)
{
    {
        Prof pr(h, OED_K_PACK);
        HIPCHK(h, launch_pack(K, h->kdtype, h->ld, h->N_t, h->N_tp, h->dcmap, h->N_c, h->R, h->rtype, h->stream));
    }
    return reset_state(h);
}

// Steps need every candidate's block row in the working copy.
oed_status need_packed(oed_ctx *h)
{
    if (h->deferred && h->unpacked > 0)
        return fail(h, OED_E_STATE,
                    std::to_string(h->unpacked) + " candidate block rows not packed yet (oed_pack_rows)");
    return OED_OK;
}

// Descriptor of the handle's current state (see StepDesc).
StepDesc desc(const oed_ctx *h)
{
    StepDesc d{};
    d.R = h->R;
    d.W = h->W;
    d.W2 = h->W2;
    d.wslot = h->wslot;
    d.nheld = h->nheld;
    d.V = h->V;
    d.nw = 1;
    d.stl = h->stl;
    d.act_in = h->act[h->cur];
    d.act_out = h->act[h->cur ^ 1];
    d.gains = h->gains;
    d.Linv = h->Linv;
    d.fcache = h->fcache;
    d.state = h->state;
    d.picks = h->picks;
    d.pick_gain = h->pick_gain;
    d.half_noise = h->half_noise;
    d.noise_h = h->noise_h;
    d.n_act = h->n_act;
    d.N_t = h->N_t;
    d.N_tp = h->N_tp;
    d.step = h->k;
    d.forced = -1;
    d.item0 = 0;
    d.nitems = h->n_act;
    return d;
}

oed_status enqueue_syrk(oed_ctx *h, StepDesc d)
{
    d.nitems = syrk_items(h->syrk_variant, h->n_act, h->N_tp, h->stl);
    d.skipdiag = h->eager ? 1 : 0;
    {
        Prof pr(h, OED_K_SYRK);
        HIPCHK(h, launch_syrk(d, h->rtype, h->wtype, h->syrk_variant, h->stream));
    }
    const double n = (double)h->n_act * h->N_t;
    h->syrk_flops += d.nw * (double)h->N_t * n * (n + 1.0);
    h->syrk_bytes += (double)relem(h) * (n * (n + h->N_t) + d.nw * n * h->N_t);
    return OED_OK;
}

// Element size of W.
size_t welem(const oed_ctx *h) { return h->wtype == W_F64 ? 8 : h->wtype == W_F32 ? 4 : 2; }

constexpr int LEFT_SPLITS = 4;

// The block column kernel applies the new column to the diagonal blocks itself (single launches,
// N_tp <= 128) wherever they are kept current step by step: the eager right-looking path and the
// left-looking method.  The gain launch then factors them as they are.
bool fuse_diag(const oed_ctx *h) { return (h->eager || h->left) && h->N_tp <= 128; }

// Left-looking: form the block column of the last pick s (pick k-1) from K and the k-1 earlier
// block columns: the partial sums sum_h W_h,i W_h,s^T (column kernel, LEFT_SPLITS parts), then
// W_i = (K_is - sums) L_s^-T into W slot k-1.  The diagonal blocks get this column from the block
// column kernel (fuse_diag) or at the next gain launch.
oed_status advance_left(oed_ctx *h)
{
    if (!h->pending) return OED_OK;
    h->pending = false;
    if (h->n_act == 0) return OED_OK;
    const int hist = h->k - 1;
    const int64_t bs = (int64_t)h->N_tp * h->N_tp;
    StepDesc d = desc(h);
    d.nheld = 0;
    d.C = h->C;
    d.cstride = (int64_t)h->N_c * bs;
    d.nsplit = std::min(LEFT_SPLITS, hist);
    if (hist > 0) {
        d.nw = hist;
        d.nitems = (int64_t)d.nsplit * syrk_tile_rows(h->n_act, h->N_tp);
        {
            Prof pr(h, OED_K_SYRK);
            HIPCHK(h, launch_column(d, h->rtype, h->wtype, h->stream));
        }
        const double n = (double)h->n_act * h->N_t;
        h->syrk_flops += 2.0 * n * h->N_t * hist * h->N_t;
        h->syrk_bytes += (double)relem(h) * (n * hist * h->N_t + (double)hist * h->N_t * h->N_t + d.nsplit * n * h->N_t);
    }
    d.W = (char *)h->W + (size_t)(hist * h->wslot) * welem(h);  // output: slot k-1
    if (h->W2) d.W2 = (char *)h->W2 + (size_t)(hist * h->wslot) * 2;
    d.diag = fuse_diag(h) ? 1 : 0;  // the new column applied to the diagonal blocks there and then
    {
        Prof pr(h, OED_K_TRSM);
        HIPCHK(h, launch_trsm(d, h->rtype, h->wtype, h->stream));
    }
    h->diag_current = d.diag != 0;
    return OED_OK;
}

// Form the block column W of the last pick (Sec. III-D: the new block row of the factor) and
// subtract the outer products from R.  With delay p > 1 and `full` false, block columns are
// held (W slots 0 .. nheld-1; the gain and pick kernels correct for them exactly) until p of
// them are formed, then subtracted in one downdate of inner dimension p N_t: 1/p of the R
// traffic per pick.  `full` leaves R current.
oed_status advance(oed_ctx *h, bool full)
{
    if (h->left) return advance_left(h);
    if (h->pending) {
        h->pending = false;
        if (h->n_act == 0) {
            h->nheld = 0;
            return OED_OK;
        }
        StepDesc d = desc(h);
        d.diag = fuse_diag(h) ? 1 : 0;
        {
            Prof pr(h, OED_K_TRSM);
            if (h->nheld > 0) HIPCHK(h, launch_vcorr(d, h->wtype, h->stream));
            HIPCHK(h, launch_trsm(d, h->rtype, h->wtype, h->stream));
        }
        d.diag = 0;
        if (h->eager && !fuse_diag(h)) {
            h->newest = h->nheld;  // the next gain launch applies it to the diagonal blocks
            h->diag_current = false;
        }
        if (h->nheld + 1 < h->delay && !full) {
            ++h->nheld;
            return OED_OK;
        }
        d.nw = h->nheld + 1;
        h->nheld = 0;
        return enqueue_syrk(h, d);
    }
    if (full && h->nheld > 0) {
        StepDesc d = desc(h);
        d.nw = h->nheld;
        d.nheld = 0;
        h->nheld = 0;
        return enqueue_syrk(h, d);
    }
    return OED_OK;
}

// ---- autotuner (OED_FLAG_AUTOTUNE with delay 0)
//
// On the freshly packed working copy it times, per delay depth p = 1..MAX_DELAY, the kernels of
// one pick: the gains and the block column with h = 0 .. p-1 block columns held, the V
// correction for h > 0, and the downdate of p block columns with each downdate kernel in the first
// tile order (the per-wave kernel too at p = 1); the per-pick cost is
// t_syrk(p)/p + (1/p) sum_h (t_gain(h) + t_vcorr(h) + t_trsm(h)), taken at the
// first step's candidate count and at half of it (the leading half of the active list) and
// averaged; the choice is the least estimate (the shallowest depth on ties), after which the other
// tile orders of TUNE_ORDERS are timed at that depth and the fastest kept.  The W slots are
// zero while the downdates are timed, so R - 0 leaves R exactly as packed; the gains, L_s^-1 and
// W buffers it writes are overwritten by the first step.  Results are cached per (device,
// precision, N_tp, ceil(N_c / 32)) in the process and, with oed_options.tune_cache, in a text file
// keyed by the GPU's architecture name and compute-unit count instead of the device index; a
// matching line of the file takes precedence over the process's cache.

constexpr int TUNE_ORDERS[] = {STL_COL4, STL_COL8, STL_COL2, STL_ROW8};
constexpr int N_TUNE_ORDERS = sizeof(TUNE_ORDERS) / sizeof(TUNE_ORDERS[0]);

struct TuneKey {
    int dev, prec, ntp, nbucket;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(dev, prec, ntp, nbucket) < std::tie(o.dev, o.prec, o.ntp, o.nbucket);
    }
};
struct TuneVal {
    int delay, variant, stl;
    double ms[MAX_DELAY];
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

// The tune-cache line of a handle's shape on its GPU: "oedtune1 <arch> <CUs> <precision> <N_tp>
// <candidates/32>" followed by "<delay> <variant> <tile code> <ms per pick for delay 1..8>".
std::string tune_cache_key(const oed_ctx *h)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) {
        arch = prop.gcnArchName;
        cus = prop.multiProcessorCount;
    }
    for (char &c : arch)
        if (c == ' ') c = '_';
    return "oedtune1 " + arch + " " + std::to_string(cus) + " " + std::to_string(h->prec) + " " +
           std::to_string(h->N_tp) + " " + std::to_string((h->N_c + 31) / 32);
}

bool tune_cache_read(const oed_ctx *h, const std::string &key, TuneVal &v)
{
    FILE *f = std::fopen(h->tune_cache.c_str(), "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        std::string ln(line);
        if (ln.compare(0, key.size(), key) != 0 || ln.size() <= key.size() || ln[key.size()] != ' ') continue;
        TuneVal t{};
        const char *p = ln.c_str() + key.size();
        int used = 0;
        if (std::sscanf(p, " %d %d %d%n", &t.delay, &t.variant, &t.stl, &used) != 3) continue;
        p += used;
        bool ok = t.delay >= 1 && t.delay <= MAX_DELAY &&
                  (t.variant == SYRK_DIRECT || t.variant == SYRK_LDS ||
                   (t.variant == SYRK_BIG && h->wtype == W_BF16X3));
        for (int q = 0; q < MAX_DELAY && ok; ++q) {
            if (std::sscanf(p, " %lf%n", &t.ms[q], &used) != 1) ok = false;
            p += used;
        }
        ok = ok && std::find(TUNE_ORDERS, TUNE_ORDERS + N_TUNE_ORDERS, t.stl) != TUNE_ORDERS + N_TUNE_ORDERS;
        if (ok) {
            v = t;  // the last matching line wins
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void tune_cache_append(const oed_ctx *h, const std::string &key, const TuneVal &v)
{
    FILE *f = std::fopen(h->tune_cache.c_str(), "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d", key.c_str(), v.delay, v.variant, v.stl);
    for (int q = 0; q < MAX_DELAY; ++q) std::fprintf(f, " %.6g", v.ms[q]);
    std::fprintf(f, "\n");
    std::fclose(f);
}

void tune_apply(oed_ctx *h, const TuneVal &v)
{
    h->delay = v.delay;
    h->syrk_variant = v.variant;
    h->stl = v.stl;
    std::copy(v.ms, v.ms + MAX_DELAY, h->tuned_ms);
}

// Milliseconds of one call of f (the minimum over three rounds).
template <typename F>
hipError_t time_ms(oed_ctx *h, hipEvent_t a, hipEvent_t b, F f, double *out)
{
    double best = 1e300;
    for (int round = 0; round < 3; ++round) {
        hipError_t e = hipEventRecord(a, h->stream);
        if (e == hipSuccess) e = f();
        if (e == hipSuccess) e = hipEventRecord(b, h->stream);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e != hipSuccess) return e;
        best = std::min(best, (double)ms);
    }
    *out = best;
    return hipSuccess;
}

oed_status autotune(oed_ctx *h)
{
    const TuneKey key{h->device, h->prec, h->N_tp, (h->N_c + 31) / 32};
    // the cache file first (it outlives the process), then the process's own choices
    const std::string ckey = h->tune_cache.empty() ? std::string() : tune_cache_key(h);
    if (!ckey.empty()) {
        TuneVal v;
        if (tune_cache_read(h, ckey, v)) {
            tune_apply(h, v);
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune[key] = v;
            return OED_OK;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            tune_apply(h, it->second);
            if (!ckey.empty()) tune_cache_append(h, ckey, it->second);
            return OED_OK;
        }
    }
    const int64_t bs = (int64_t)h->N_tp * h->N_tp;
    const size_t we = h->wtype == W_F64 ? 8 : h->wtype == W_F32 ? 4 : 2;
    const size_t wbytes = (size_t)(MAX_DELAY * h->wslot) * we;
    hipEvent_t a = nullptr, b = nullptr;
    HIPCHK(h, hipEventCreate(&a));
    HIPCHK(h, hipEventCreate(&b));
    auto done = [&](oed_status st) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return st;
    };
    auto zero_w = [&]() -> hipError_t {
        hipError_t e = hipMemsetAsync(h->W, 0, wbytes, h->stream);
        if (e == hipSuccess && h->W2) e = hipMemsetAsync(h->W2, 0, wbytes, h->stream);
        return e;
    };
    hipError_t e = zero_w();
    if (e == hipSuccess) e = hipMemsetAsync(h->Linv, 0, sizeof(double) * bs, h->stream);
    // the per-pick estimates at the first step's size n and at n / 2, averaged: the run's later
    // steps work on fewer candidates, where each launch's fixed cost weighs more
    // downdate kernels tried: the 128 x 128 LDS tile, and for the BF16 split product the 256 x 256 one
    // (unless oed_options.tile_size fixed one of them)
    int variants[2] = {SYRK_LDS, SYRK_BIG};
    int nvar = h->wtype == W_BF16X3 ? 2 : 1;
    if (h->fixed_variant >= 0) {
        variants[0] = h->fixed_variant;
        nvar = 1;
    }
    double t_step[2][MAX_DELAY] = {{0}}, t_syrk[2][MAX_DELAY][N_TUNE_ORDERS][2] = {}, t_direct[2] = {1e300, 1e300};
    const int n_at[2] = {h->n_act, std::max(1, h->n_act / 2)};
    auto syrk_desc = [&](int p, int o, int z) {
        StepDesc d = desc(h);
        d.n_act = n_at[z];
        d.nheld = 0;
        d.nw = p;
        d.stl = TUNE_ORDERS[o];
        d.skipdiag = h->eager ? 1 : 0;
        return d;
    };
    // the downdate of p zero W slots (R - 0 leaves R as packed) in tile order o with kernel v
    auto time_syrk = [&](int p, int o, int v, int z, double *out) {
        StepDesc d = syrk_desc(p, o, z);
        d.nitems = syrk_items(variants[v], n_at[z], h->N_tp, d.stl);
        return time_ms(h, a, b, [&] { return launch_syrk(d, h->rtype, h->wtype, variants[v], h->stream); }, out);
    };
    for (int z = 0; z < 2 && e == hipSuccess; ++z) {
        for (int hh = 0; hh < MAX_DELAY && e == hipSuccess; ++hh) {
            StepDesc d = desc(h);
            d.n_act = n_at[z];
            d.nitems = n_at[z];
            d.nheld = hh;
            // eager diagonal: the block column kernel applies the new column to the diagonal blocks
            // and the gain launch factors them as they are (the W slots and L_s^-1 are zero, so R
            // stays exactly as packed)
            StepDesc dg = d;
            if (h->eager) {
                dg.nheld = 0;
                d.diag = fuse_diag(h) ? 1 : 0;
                if (!d.diag) {
                    dg.nheld = hh > 0 ? 1 : 0;
                    dg.wb = dg.nheld;
                }
            }
            double tg = 0, tt = 0;
            e = time_ms(h, a, b, [&] { return launch_gain(dg, h->rtype, h->wtype, h->stream); }, &tg);
            if (e == hipSuccess)
                e = time_ms(h, a, b, [&] {
                    hipError_t r = hh > 0 ? launch_vcorr(d, h->wtype, h->stream) : hipSuccess;
                    return r == hipSuccess ? launch_trsm(d, h->rtype, h->wtype, h->stream) : r;
                }, &tt);
            t_step[z][hh] = tg + tt;
        }
        if (e == hipSuccess) e = zero_w();
        // phase 1: every depth in the first tile order, every downdate kernel
        for (int p = 1; p <= MAX_DELAY && e == hipSuccess; ++p)
            for (int v = 0; v < nvar && e == hipSuccess; ++v) {
                e = time_syrk(p, 0, v, z, &t_syrk[z][p - 1][0][v]);
                if (e == hipSuccess && p == 1 && v == 0 && h->wtype != W_BF16X3 && h->fixed_variant < 0) {
                    StepDesc d = syrk_desc(p, 0, z);
                    d.nitems = syrk_tiles(n_at[z], h->N_tp, d.stl);
                    e = time_ms(h, a, b, [&] { return launch_syrk(d, h->rtype, h->wtype, SYRK_DIRECT, h->stream); },
                                &t_direct[z]);
                }
            }
    }
    if (e != hipSuccess) return done(fail(h, e == hipErrorOutOfMemory ? OED_E_OOM : OED_E_HIP,
                                          std::string("autotune: ") + hipGetErrorString(e)));
    TuneVal v{1, variants[0], TUNE_ORDERS[0], {0}};
    int best_v[MAX_DELAY] = {0};
    bool direct_at1 = false;
    double best = 1e300;
    auto estimate = [&](int p, double syrk0, double syrk1) {
        double sum = 0;
        for (int z = 0; z < 2; ++z) {
            double steps = 0;
            for (int hh = 0; hh < p; ++hh) steps += t_step[z][hh];
            sum += ((z ? syrk1 : syrk0) + steps) / p;
        }
        return 0.5 * sum;
    };
    for (int p = 1; p <= MAX_DELAY; ++p) {
        double tbest = 1e300;
        for (int vv = 0; vv < nvar; ++vv) {
            const double t = t_syrk[0][p - 1][0][vv] + t_syrk[1][p - 1][0][vv];
            if (t < tbest) {
                tbest = t;
                best_v[p - 1] = vv;
            }
        }
        const bool direct = p == 1 && t_direct[0] + t_direct[1] < tbest;
        if (p == 1) direct_at1 = direct;
        v.ms[p - 1] = direct ? estimate(p, t_direct[0], t_direct[1])
                             : estimate(p, t_syrk[0][p - 1][0][best_v[p - 1]], t_syrk[1][p - 1][0][best_v[p - 1]]);
        best = std::min(best, v.ms[p - 1]);
    }
    // the least estimate, the shallowest depth on ties (a margin towards shallower depths chose
    // delay 3 at 600 x 128 FP32, measured 1.5% slower than 4)
    for (int p = 1; p <= MAX_DELAY; ++p)
        if (v.ms[p - 1] <= best) {
            v.delay = p;
            v.variant = variants[best_v[p - 1]];
            if (p == 1 && direct_at1) v.variant = SYRK_DIRECT;
            break;
        }
    // phase 2: the other tile orders at the chosen depth and kernel
    if (v.variant != SYRK_DIRECT) {
        const int p = v.delay, vv = best_v[p - 1];
        double tbest = t_syrk[0][p - 1][0][vv] + t_syrk[1][p - 1][0][vv];
        for (int o = 1; o < N_TUNE_ORDERS && e == hipSuccess; ++o) {
            for (int z = 0; z < 2 && e == hipSuccess; ++z) e = time_syrk(p, o, vv, z, &t_syrk[z][p - 1][o][vv]);
            const double t = t_syrk[0][p - 1][o][vv] + t_syrk[1][p - 1][o][vv];
            // another order only when it is clearly faster (the timings of one launch scatter by
            // about 0.5%; at 600 x 128 the first order was the fastest over whole selections)
            if (e == hipSuccess && t < 0.99 * tbest) {
                tbest = t;
                v.stl = TUNE_ORDERS[o];
                v.ms[p - 1] = estimate(p, t_syrk[0][p - 1][o][vv], t_syrk[1][p - 1][o][vv]);
            }
        }
        if (e != hipSuccess) return done(fail(h, e == hipErrorOutOfMemory ? OED_E_OOM : OED_E_HIP,
                                              std::string("autotune: ") + hipGetErrorString(e)));
    }
    tune_apply(h, v);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = v;
    }
    if (!ckey.empty()) tune_cache_append(h, ckey, v);
    return done(OED_OK);
}

oed_status enqueue_gains(oed_ctx *h)
{
    StepDesc d = desc(h);
    d.scratch = h->scratch_gain;
    if (h->eager) {
        // the diagonal blocks include every column but the newest one: apply it and write back
        d.nheld = 0;
        if (!h->diag_current && h->newest >= 0) {
            d.W = (char *)h->W + (size_t)(h->newest * h->wslot) * welem(h);
            if (h->W2) d.W2 = (char *)h->W2 + (size_t)(h->newest * h->wslot) * 2;
            d.nheld = 1;
            d.wb = 1;
        }
        h->diag_current = true;
    } else if (h->left && !h->diag_current) {
        // apply the newest block column (slot k-1) to the diagonal blocks, in place
        d.W = (char *)h->W + (size_t)((h->k - 1) * h->wslot) * welem(h);
        if (h->W2) d.W2 = (char *)h->W2 + (size_t)((h->k - 1) * h->wslot) * 2;
        d.nheld = 1;
        d.wb = 1;
        h->diag_current = true;
    }
    Prof pr(h, OED_K_GAIN);
    HIPCHK(h, launch_gain(d, h->rtype, h->wtype, h->stream));
    return OED_OK;
}

oed_status enqueue_pick(oed_ctx *h, int forced_local)
{
    StepDesc d = desc(h);
    d.scratch = h->scratch_pick;
    if (h->eager) d.nheld = 0;  // the winner's diagonal block is current
    d.forced = forced_local;
    d.nitems = 1;
    {
        Prof pr(h, OED_K_PICK);
        HIPCHK(h, launch_pick(d, h->rtype, h->wtype, h->stream));
    }
    h->cur ^= 1;
    h->n_act -= 1;
    h->k += 1;
    h->pending = true;
    return OED_OK;
}

// Read back picks [k0, k) and the status word; reconcile the host mirror.
oed_status sync_picks(oed_ctx *h, int k0, oed_status *dev_status)
{
    const int n = h->k - k0;
    std::vector<int> idx(std::max(n, 1));
    std::vector<double> g(std::max(n, 1));
    int st[ST_WORDS];
    if (n > 0) {
        HIPCHK(h, hipMemcpyAsync(idx.data(), h->picks + k0, sizeof(int) * n, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(h, hipMemcpyAsync(g.data(), h->pick_gain + k0, sizeof(double) * n, hipMemcpyDeviceToHost, h->stream));
    }
    HIPCHK(h, hipMemcpyAsync(st, h->state, sizeof(st), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    collect_profile(h);
    *dev_status = (oed_status)st[ST_STATUS];
    const int made = std::min(n, std::max(0, st[ST_NPICKS] - k0));
    if (st[ST_STATUS] != 0) {
        // the device stopped after `made` picks; later kernels were no-ops
        h->k = k0 + made;
        h->n_act = h->N_c - h->k;
        h->pending = false;
        h->nheld = 0;
        h->poisoned = true;
    }
    for (int q = 0; q < made; ++q) {
        h->h_picks.push_back(idx[q]);
        h->h_gains.push_back(g[q]);
        if (idx[q] >= 0 && idx[q] < h->N_c) h->picked[idx[q]] = 1;
    }
    return OED_OK;
}

// The debug_fail_step hook: the fail_step-th pick since creation or the last reset fails once,
// on the host, before anything of it is enqueued.
oed_status step_hook(oed_ctx *h)
{
    if (h->fail_step > 0 && h->k + 1 == h->fail_step) {
        h->fail_step = 0;
        return fail(h, OED_E_HIP, "injected failure before pick " + std::to_string(h->k + 1) +
                                      " (oed_options.debug_fail_step)");
    }
    return OED_OK;
}

// A step failed before or while it was enqueued: wait for what was enqueued before it, hand back
// the picks it made (if the outputs are given), and stop the handle until oed_reset.  The first
// failure's status and text are kept.
oed_status stop_after_failure(oed_ctx *h, oed_status st, int k0, int32_t *idx_out, double *gain_out, int32_t *n_out)
{
    const std::string msg = h->err;
    // the failing step's pick was not enqueued: the mirror counts only launched picks
    oed_status dev = OED_OK;
    if (sync_picks(h, k0, &dev) == OED_OK && idx_out && gain_out) {
        const int made = (int)h->h_picks.size() - k0;
        for (int q = 0; q < made; ++q) {
            idx_out[q] = h->cmap[h->h_picks[k0 + q]];
            gain_out[q] = h->h_gains[k0 + q];
        }
        if (n_out) *n_out = made;
    }
    h->poisoned = true;
    h->pending = false;
    h->err = msg;
    return st;
}

}  // namespace

extern "C" {

void oed_options_init(oed_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->struct_size = sizeof(oed_options);
    opt->precision = OED_PREC_FP64;
}

const char *oed_status_string(int32_t s)
{
    switch (s) {
    case OED_OK: return "OED_OK";
    case OED_E_ARG: return "OED_E_ARG";
    case OED_E_NOT_SPD: return "OED_E_NOT_SPD";
    case OED_E_OOM: return "OED_E_OOM";
    case OED_E_HIP: return "OED_E_HIP";
    case OED_E_STATE: return "OED_E_STATE";
    case OED_E_UNSUPPORTED: return "OED_E_UNSUPPORTED";
    default: return "OED_E_UNKNOWN";
    }
}

const char *oed_last_error(const oed_ctx *h) { return h ? h->err.c_str() : g_create_err.c_str(); }

oed_status oed_create(oed_ctx **out, const void *K, int32_t dtype, int64_t ld, int32_t N_s, int32_t N_t,
                      double sigma2, void *stream, const oed_options *opt)
{
    g_create_err.clear();
    auto cfail = [](oed_status st, const std::string &msg) {
        g_create_err = msg;
        return st;
    };
    if (!out) return cfail(OED_E_ARG, "out is NULL");
    *out = nullptr;
    oed_options o;
    oed_options_init(&o);
    if (opt) {
        if (opt->struct_size != sizeof(oed_options)) return cfail(OED_E_ARG, "oed_options.struct_size mismatch");
        o = *opt;
    }
    const bool deferred = (o.flags & OED_FLAG_DEFER_PACK) != 0;
    if (deferred) {
        // no K: dtype and ld are not used
        if (K || (o.flags & OED_FLAG_AUTOTUNE)) return cfail(OED_E_ARG, "deferred packing takes no K and no autotuner");
        dtype = OED_F64;
        ld = (int64_t)N_s * N_t;
    }
    if ((!K && !deferred) || (dtype != OED_F64 && dtype != OED_F32) || N_s < 1 || N_t < 1 || N_t > 4096 ||
        ld < (int64_t)N_s * N_t || !(sigma2 > 0.0) || !std::isfinite(sigma2))
        return cfail(OED_E_ARG, "bad K, dtype, shape, leading dimension or sigma2");
    if (o.precision != OED_PREC_FP64 && o.precision != OED_PREC_MIXED_F32 && o.precision != OED_PREC_MIXED_BF16X3)
        return cfail(OED_E_ARG, "unknown precision");
    if (o.delay < 0 || o.delay > MAX_DELAY) return cfail(OED_E_ARG, "delay out of range");
    // held block columns need the register or blocked factorisations (they apply them on the fly)
    if (o.delay > 1 && N_t > BLK_MAX_NTP) return cfail(OED_E_UNSUPPORTED, "delay > 1 needs N_t <= 1024");
    if (o.method != OED_METHOD_RIGHT_LOOKING && o.method != OED_METHOD_LEFT_LOOKING && o.method != OED_METHOD_AUTO)
        return cfail(OED_E_ARG, "unknown method");
    if (o.max_budget < 0 || o.max_budget > N_s) return cfail(OED_E_ARG, "max_budget out of range");
    // left-looking needs the diagonal-block update of the register or blocked gain kernels
    if (o.method == OED_METHOD_LEFT_LOOKING && N_t > BLK_MAX_NTP)
        return cfail(OED_E_UNSUPPORTED, "the left-looking method serves N_t <= 1024");
    if (o.tile_order < OED_TILES_AUTO || o.tile_order > OED_TILES_COL2) return cfail(OED_E_ARG, "unknown tile order");
    if (o.max_device_bytes < 0 || o.debug_fail_step < 0) return cfail(OED_E_ARG, "negative limit or hook step");
    if (o.tile_size != 0 && o.tile_size != 128 && o.tile_size != 256) return cfail(OED_E_ARG, "tile_size: 0, 128 or 256");
    if (o.tile_size == 256 && (o.precision != OED_PREC_MIXED_BF16X3 || N_t > 128))
        return cfail(OED_E_UNSUPPORTED, "256 x 256 downdate tiles serve the BF16 split product with N_t <= 128");
    for (int r : o.reserved)
        if (r != 0) return cfail(OED_E_ARG, "reserved option fields must be 0");

    oed_ctx *h = new (std::nothrow) oed_ctx();
    if (!h) return cfail(OED_E_OOM, "host allocation of the handle failed");
    h->N_s = N_s;
    h->N_t = N_t;
    // the BF16 operands hold 32 inner indices per lane group of four
    h->N_tp = o.precision == OED_PREC_MIXED_BF16X3 ? (N_t + 31) / 32 * 32 : (N_t + 15) / 16 * 16;
    h->kdtype = dtype;
    h->ld = ld;
    h->sigma2 = sigma2;
    h->half_noise = 0.5 * N_t * std::log(sigma2);
    h->prec = o.precision;
    h->rtype = o.precision == OED_PREC_FP64 ? R_F64 : R_F32;
    h->wtype = o.precision == OED_PREC_FP64 ? W_F64 : o.precision == OED_PREC_MIXED_F32 ? W_F32 : W_BF16X3;
    h->flags = o.flags;
    h->fail_step = o.debug_fail_step;
    if (o.tune_cache) h->tune_cache = o.tune_cache;
    static const int stl_of[] = {STL_COL4, STL_ROW8, STL_COL8, STL_COL4, STL_COL2};
    h->stl = stl_of[o.tile_order];
    // downdate kernel: 128 x 128 tiles, or (BF16 split product) 256 x 256, which the autotuner weighs
    // against it; without the tuner 128 x 128 (faster at 600 x 128: 11.6 against 15.3 ms per launch at
    // delay 7)
    if (o.tile_size == 128) h->fixed_variant = SYRK_LDS;
    if (o.tile_size == 256) h->fixed_variant = SYRK_BIG;
    h->syrk_variant = o.tile_size == 256 ? SYRK_BIG : SYRK_LDS;
    // delay 0 (automatic): hold block columns whenever the register factorisations and the LDS
    // downdate serve the block size
    h->delay = o.delay == 0 ? (N_t <= REGS_MAX_NT ? DEFAULT_DELAY : 1) : o.delay;
    if (o.method == OED_METHOD_AUTO) {
        const int nc = o.candidates ? o.n_candidates : N_s;
        const int mb = o.max_budget > 0 ? std::min(o.max_budget, nc) : nc;
        o.method = (N_t <= BLK_MAX_NTP && 2 * mb <= nc) ? OED_METHOD_LEFT_LOOKING : OED_METHOD_RIGHT_LOOKING;
    }
    h->left = o.method == OED_METHOD_LEFT_LOOKING;
    if (h->left) h->delay = 1;
    h->eager = !h->left && N_t <= REGS_MAX_NT;
    // the autotuner chooses the depth and, unless one is given, the tile order
    const bool tune = !h->left && o.delay == 0 && (o.flags & OED_FLAG_AUTOTUNE) && N_t <= REGS_MAX_NT;
    const bool tune_tiles = tune && o.tile_order == OED_TILES_AUTO;
    h->stream = (hipStream_t)stream;
    h->lmap.assign(N_s, -1);
    if (o.candidates) {
        if (o.n_candidates < 1 || o.n_candidates > N_s) {
            delete h;
            return cfail(OED_E_ARG, "n_candidates out of range");
        }
        h->cmap.assign(o.candidates, o.candidates + o.n_candidates);
        std::sort(h->cmap.begin(), h->cmap.end());
        for (size_t q = 0; q < h->cmap.size(); ++q)
            if (h->cmap[q] < 0 || h->cmap[q] >= N_s || (q > 0 && h->cmap[q] == h->cmap[q - 1])) {
                delete h;
                return cfail(OED_E_ARG, "candidate out of range or repeated");
            }
    } else {
        h->cmap.resize(N_s);
        for (int q = 0; q < N_s; ++q) h->cmap[q] = q;
    }
    h->N_c = (int)h->cmap.size();
    std::vector<double> hloc;
    if (o.noise_half_logdet) {
        hloc.resize(h->N_c);
        for (int q = 0; q < h->N_c; ++q) {
            hloc[q] = o.noise_half_logdet[h->cmap[q]];
            if (!std::isfinite(hloc[q])) {
                delete h;
                return cfail(OED_E_ARG, "non-finite noise_half_logdet entry");
            }
        }
    }
    h->max_budget = (o.max_budget == 0 || o.max_budget > h->N_c) ? h->N_c : o.max_budget;
    for (int q = 0; q < h->N_c; ++q) h->lmap[h->cmap[q]] = q;

    // every device buffer of the handle, sized before anything is allocated
    const int64_t bs = (int64_t)h->N_tp * h->N_tp;
    const int64_t nblk = (int64_t)h->N_c * (h->N_c + 1) / 2;
    const size_t we = h->wtype == W_F64 ? 8 : h->wtype == W_F32 ? 4 : 2;
    h->wslot = h->N_c * bs;
    const int slots = h->left ? h->max_budget : tune ? MAX_DELAY : h->delay;
    const size_t sg = gain_scratch_doubles(h->N_t, h->N_tp, h->N_c), sp = pick_scratch_doubles(h->N_t, h->N_tp);
    struct Buf {
        void **ptr;
        size_t bytes;
    };
    const Buf bufs[] = {
        {&h->R, (size_t)(nblk * bs) * relem(h)},
        {&h->C, h->left ? (size_t)(LEFT_SPLITS * h->N_c * bs) * relem(h) : 0},
        {&h->W, (size_t)(slots * h->wslot) * we},
        {&h->W2, h->wtype == W_BF16X3 ? (size_t)(slots * h->wslot) * 2 : 0},
        {(void **)&h->V, slots > 1 ? sizeof(double) * bs * (slots - 1) : 0},
        {(void **)&h->Linv, sizeof(double) * bs},
        {(void **)&h->gains, sizeof(double) * h->N_c},
        {(void **)&h->pick_gain, sizeof(double) * h->N_c},
        {(void **)&h->act[0], sizeof(int) * h->N_c},
        {(void **)&h->act[1], sizeof(int) * h->N_c},
        {(void **)&h->picks, sizeof(int) * h->N_c},
        {(void **)&h->state, sizeof(int) * ST_WORDS},
        {(void **)&h->dcmap, sizeof(int) * h->N_c},
        {(void **)&h->scratch_gain, sizeof(double) * sg},
        {(void **)&h->scratch_pick, sizeof(double) * sp},
        {(void **)&h->fcache, h->N_t <= REGS_MAX_NT ? sizeof(double) * 256 * FCACHE_BLOCKS * h->N_c : 0},
        {(void **)&h->noise_h, hloc.empty() ? 0 : sizeof(double) * h->N_c},
    };
    int64_t need = 0;
    for (const Buf &b : bufs) need += (int64_t)b.bytes;
    if (o.max_device_bytes > 0 && need > o.max_device_bytes) {
        delete h;
        return cfail(OED_E_OOM, "the handle needs " + std::to_string(need) + " bytes of device memory, more than "
                                "max_device_bytes = " + std::to_string(o.max_device_bytes));
    }

    oed_status st = OED_OK;
    auto setup = [&]() -> oed_status {
        HIPCHK(h, hipGetDevice(&h->device));
        for (const Buf &b : bufs)
            if (b.bytes) HIPCHK(h, dmalloc(h, b.ptr, b.bytes));
        HIPCHK(h, hipMemcpyAsync(h->dcmap, h->cmap.data(), sizeof(int) * h->N_c, hipMemcpyHostToDevice, h->stream));
        if (!hloc.empty())
            HIPCHK(h, hipMemcpyAsync(h->noise_h, hloc.data(), sizeof(double) * h->N_c, hipMemcpyHostToDevice, h->stream));
        h->deferred = deferred;
        if (deferred) {
            h->row_packed.assign(h->N_c, 0);
            h->unpacked = h->N_c;
        }
        oed_status s2 = deferred ? reset_state(h) : load_R(h, K);
        if (s2 != OED_OK) return s2;
        HIPCHK(h, hipStreamSynchronize(h->stream));
        collect_profile(h);
        if (tune) {
            const int keep_stl = h->stl;
            s2 = autotune(h);
            if (!tune_tiles) h->stl = keep_stl;
            if (h->fixed_variant >= 0) h->syrk_variant = h->fixed_variant;
            return s2;
        }
        return OED_OK;
    };
    st = setup();
    if (st != OED_OK) {
        g_create_err = h->err;
        free_all(h);
        delete h;
        return st;
    }
    *out = h;
    return OED_OK;
}

oed_status oed_reset(oed_ctx *h, const void *K)
{
    if (!h) return OED_E_ARG;
    if (h->deferred) {
        if (K) return fail(h, OED_E_ARG, "deferred packing: reset with K = NULL and pack the rows again");
        h->row_packed.assign(h->N_c, 0);
        h->unpacked = h->N_c;
        oed_status st = reset_state(h);
        if (st != OED_OK) return st;
        HIPCHK(h, hipStreamSynchronize(h->stream));
        return OED_OK;
    }
    if (!K) return fail(h, OED_E_ARG, "K is NULL");
    oed_status st = load_R(h, K);
    if (st != OED_OK) return st;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    collect_profile(h);
    return OED_OK;
}

oed_status oed_pack_rows(oed_ctx *h, const void *K_rows, int32_t dtype, int64_t ld, int32_t sensor0,
                         int32_t n_sensors)
{
    if (!h) return OED_E_ARG;
    if (!h->deferred) return fail(h, OED_E_STATE, "handle was not created with OED_FLAG_DEFER_PACK");
    if (h->k > 0 || h->pending) return fail(h, OED_E_STATE, "picks made: reset the handle before packing");
    if (!K_rows || (dtype != OED_F64 && dtype != OED_F32) || sensor0 < 0 || n_sensors < 1 ||
        (int64_t)sensor0 + n_sensors > h->N_s || ld < ((int64_t)sensor0 + n_sensors) * h->N_t)
        return fail(h, OED_E_ARG, "bad panel");
    // candidates are ascending, so the panel's candidates are local indices i0 .. i1-1 and every
    // block (i, j <= i) lies in the panel's lower block triangle
    const int i0 = (int)(std::lower_bound(h->cmap.begin(), h->cmap.end(), sensor0) - h->cmap.begin());
    const int i1 = (int)(std::lower_bound(h->cmap.begin(), h->cmap.end(), sensor0 + n_sensors) - h->cmap.begin());
    if (i1 > i0) {
        {
            Prof pr(h, OED_K_PACK);
            HIPCHK(h, launch_pack_range(K_rows, dtype, ld, (int64_t)sensor0 * h->N_t, h->N_t, h->N_tp, h->dcmap,
                                        blk_index(i0, 0), blk_index(i1, 0) - blk_index(i0, 0), h->R, h->rtype,
                                        h->stream));
        }
        HIPCHK(h, hipStreamSynchronize(h->stream));
        collect_profile(h);
        for (int i = i0; i < i1; ++i)
            if (!h->row_packed[i]) {
                h->row_packed[i] = 1;
                --h->unpacked;
            }
    }
    return OED_OK;
}

oed_status oed_greedy(oed_ctx *h, int32_t budget, int32_t *idx_out, double *gain_out, int32_t *n_out)
{
    if (!h) return OED_E_ARG;
    if (n_out) *n_out = 0;
    if (need_packed(h) != OED_OK) return OED_E_STATE;
    if (h->poisoned) return fail(h, OED_E_STATE, "handle stopped after a non-positive-definite step; reset it");
    if (budget < 0 || budget > h->n_act) return fail(h, OED_E_ARG, "budget out of range");
    if (h->left && h->k + budget > h->max_budget) return fail(h, OED_E_ARG, "budget beyond max_budget");
    if (budget > 0 && (!idx_out || !gain_out)) return fail(h, OED_E_ARG, "NULL output array");
    const int k0 = h->k;
    for (int step = 0; step < budget; ++step) {
        oed_status st = step_hook(h);
        if (st == OED_OK) st = advance(h, false);
        if (st == OED_OK) st = enqueue_gains(h);
        if (st == OED_OK) st = enqueue_pick(h, -1);
        if (st != OED_OK) return stop_after_failure(h, st, k0, idx_out, gain_out, n_out);
    }
    oed_status dev = OED_OK;
    oed_status st = sync_picks(h, k0, &dev);
    if (st != OED_OK) return st;
    const int made = h->k - k0;
    for (int q = 0; q < made; ++q) {
        idx_out[q] = h->cmap[h->h_picks[k0 + q]];
        gain_out[q] = h->h_gains[k0 + q];
    }
    if (n_out) *n_out = made;
    if (dev == 2) return fail(h, OED_E_NOT_SPD, "every remaining candidate has a non-positive-definite Schur block");
    if (dev != 0) return fail(h, OED_E_STATE, "device reported status " + std::to_string((int)dev));
    return OED_OK;
}

oed_status oed_force(oed_ctx *h, int32_t idx, double *gain_out)
{
    if (!h) return OED_E_ARG;
    if (h->poisoned) return fail(h, OED_E_STATE, "handle stopped; reset it");
    if (need_packed(h) != OED_OK) return OED_E_STATE;
    if (idx < 0 || idx >= h->N_s || h->lmap[idx] < 0 || h->picked[h->lmap[idx]])
        return fail(h, OED_E_ARG, "index is not a remaining candidate");
    const int k0 = h->k;
    if (h->left && h->k >= h->max_budget) return fail(h, OED_E_ARG, "max_budget picks already made");
    oed_status st = step_hook(h);
    if (st != OED_OK) return stop_after_failure(h, st, k0, nullptr, nullptr, nullptr);
    st = advance(h, false);
    if (st == OED_OK && (h->left || h->eager) && !h->diag_current) st = enqueue_gains(h);
    if (st == OED_OK) st = enqueue_pick(h, h->lmap[idx]);
    if (st != OED_OK) return st;
    oed_status dev = OED_OK;
    st = sync_picks(h, k0, &dev);
    if (st != OED_OK) return st;
    if (dev == 2) return fail(h, OED_E_NOT_SPD, "Schur block of the forced sensor is not positive definite");
    if (dev != 0) return fail(h, OED_E_STATE, "device reported status " + std::to_string((int)dev));
    if (gain_out) *gain_out = h->h_gains.back();
    return OED_OK;
}

oed_status oed_scores(oed_ctx *h, double *out)
{
    if (!h || !out) return OED_E_ARG;
    if (h->poisoned) return fail(h, OED_E_STATE, "handle stopped; reset it");
    if (need_packed(h) != OED_OK) return OED_E_STATE;
    for (int q = 0; q < h->N_s; ++q) out[q] = -INFINITY;
    if (h->n_act == 0) return OED_OK;
    oed_status st = advance(h, false);
    if (st == OED_OK) st = enqueue_gains(h);
    if (st != OED_OK) return st;
    std::vector<double> g(h->n_act);
    std::vector<int> act(h->n_act);
    HIPCHK(h, hipMemcpyAsync(g.data(), h->gains, sizeof(double) * h->n_act, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(act.data(), h->act[h->cur], sizeof(int) * h->n_act, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    collect_profile(h);
    for (int p = 0; p < h->n_act; ++p) out[h->cmap[act[p]]] = g[p];
    return OED_OK;
}

oed_status oed_schur_block(oed_ctx *h, int32_t i, int32_t j, double *out)
{
    if (!h || !out) return OED_E_ARG;
    if (h->poisoned) return fail(h, OED_E_STATE, "handle stopped; reset it");
    if (need_packed(h) != OED_OK) return OED_E_STATE;
    if (i < 0 || j < 0 || i >= h->N_s || j >= h->N_s) return fail(h, OED_E_ARG, "index out of range");
    int li = h->lmap[i], lj = h->lmap[j];
    if (li < 0 || lj < 0 || h->picked[li] || h->picked[lj]) return fail(h, OED_E_ARG, "not a remaining candidate");
    oed_status st = advance(h, true);
    // bring the diagonal blocks up to date (the gains are recomputed as a side effect)
    if (st == OED_OK && (h->left || h->eager) && !h->diag_current) st = enqueue_gains(h);
    if (st != OED_OK) return st;
    const bool tr = li < lj;
    if (tr) std::swap(li, lj);
    // the block is formed on the device into the L_s^-1 buffer (N_tp^2 >= N_t^2 doubles), which no
    // step needs between here and the next pick: the last pick's block column is formed above
    const int nsub = (h->left && li != lj) ? h->k : 0;
    HIPCHK(h, launch_schur_block(h->R, h->rtype, h->W, h->W2, h->wtype, h->wslot, nsub, li, lj, tr ? 1 : 0, h->N_t,
                                 h->N_tp, h->Linv, h->stream));
    HIPCHK(h, hipMemcpyAsync(out, h->Linv, sizeof(double) * h->N_t * h->N_t, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    collect_profile(h);
    return OED_OK;
}

oed_status oed_picks(oed_ctx *h, int32_t *idx_out, double *gain_out, int32_t *n_out)
{
    if (!h || !n_out) return OED_E_ARG;
    *n_out = (int32_t)h->h_picks.size();
    for (size_t q = 0; q < h->h_picks.size(); ++q) {
        if (idx_out) idx_out[q] = h->cmap[h->h_picks[q]];
        if (gain_out) gain_out[q] = h->h_gains[q];
    }
    return OED_OK;
}

oed_status oed_get_profile(oed_ctx *h, oed_profile *out, int32_t reset)
{
    if (!h || !out) return OED_E_ARG;
    if (!(h->flags & OED_FLAG_PROFILE)) return fail(h, OED_E_STATE, "created without OED_FLAG_PROFILE");
    HIPCHK(h, hipStreamSynchronize(h->stream));
    collect_profile(h);
    for (int c = 0; c < NKC; ++c) {
        out->ms[c] = h->prof_ms[c];
        out->launches[c] = h->prof_n[c];
    }
    out->syrk_flops = h->syrk_flops;
    out->syrk_bytes = h->syrk_bytes;
    if (reset) {
        for (int c = 0; c < NKC; ++c) {
            h->prof_ms[c] = 0;
            h->prof_n[c] = 0;
        }
        h->syrk_flops = h->syrk_bytes = 0;
    }
    return OED_OK;
}

oed_status oed_get_config(const oed_ctx *h, int32_t *delay, int32_t *syrk_variant, int32_t *tile_order,
                          double *per_pick_ms)
{
    if (!h) return OED_E_ARG;
    if (syrk_variant && h->left) {
        *syrk_variant = -1;
        syrk_variant = nullptr;
    }
    if (delay) *delay = h->delay;
    if (syrk_variant) *syrk_variant = h->syrk_variant;
    if (tile_order)
        *tile_order = h->stl == STL_ROW8 ? OED_TILES_ROW8 : h->stl == STL_COL8 ? OED_TILES_COL8
                      : h->stl == STL_COL4 ? OED_TILES_COL4 : OED_TILES_COL2;
    if (per_pick_ms) std::copy(h->tuned_ms, h->tuned_ms + MAX_DELAY, per_pick_ms);
    return OED_OK;
}

oed_status oed_device_bytes(const oed_ctx *h, int64_t *bytes)
{
    if (!h || !bytes) return OED_E_ARG;
    *bytes = h->dev_bytes;
    return OED_OK;
}

oed_status oed_destroy(oed_ctx *h)
{
    if (!h) return OED_OK;
    (void)hipStreamSynchronize(h->stream);
    free_all(h);
    delete h;
    return OED_OK;
}

}  // extern "C"
