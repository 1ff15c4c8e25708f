// Batched selection over many independent designs (declarations and contract in include/oed.h).
//
// Each instance has its own working copy, W blocks, active lists and state words.  The
// schedule of the whole run is known on the host before anything executes (instance i runs
// budget_i steps; after its k-th pick N_c - k - 1 candidates remain), so all step descriptors
// are built once and uploaded once, and a run is a fixed sequence of batched launches:
//   init state (per instance), then for every step k:
//   gains (all instances with budget > k), pick (same), and, for the instances that pick again,
//   the block column W and the downdate (one launch per padded block size N_tp).
// That sequence is captured into a HIP graph on the first run and replayed afterwards.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/oed.h"
#include "oed_internal.h"

using namespace oed;

namespace {

struct Inst {
    int N_s = 0, N_t = 0, N_tp = 0, budget = 0, kdtype = 0;
    int64_t ld = 0;
    double sigma2 = 0, half_noise = 0;
    void *R = nullptr, *W = nullptr, *W2 = nullptr;  // `delay` W slots (BF16: hi, lo parts)
    int64_t wslot = 0;                               // elements per W slot
    double *V = nullptr;
    void *C = nullptr;  // left-looking column partial sums (LEFT_SPLITS x N_s blocks, R's type)
    double *Linv = nullptr, *gains = nullptr, *pick_gain = nullptr, *fcache = nullptr;
    int *act[2] = {nullptr, nullptr}, *cmap = nullptr, *picks = nullptr, *state = nullptr;
    size_t off_gain = 0, off_int = 0;  // offsets of this instance's results in the results block
    int branch = 0;                    // launch sequence (stream) the instance runs in
};

enum LaunchKind { L_INIT, L_GAIN, L_PICK, L_VCORR, L_TRSM, L_SYRK, L_COLUMN };

constexpr int LEFT_SPLITS = 4;

struct Launch {
    int kind = L_INIT;
    int inst = -1;       // L_INIT
    int64_t desc0 = 0;   // first descriptor
    int ndesc = 0;
    int64_t total = 0;   // work items
    int N_tp = 0;        // L_SYRK
    int nw = 1;          // L_SYRK
    int max_Nt = 0;      // L_PICK
    int branch = 0;      // launch sequence (stream) of the launch
};

Launch make_launch(int kind, int64_t desc0)
{
    Launch L;
    L.kind = kind;
    L.desc0 = desc0;
    return L;
}

}  // namespace

struct oed_batch {
    std::vector<Inst> in;
    int prec = OED_PREC_FP64, rtype = R_F64, wtype = W_F64;
    int delay = 2;
    int stl = STL_COL4;  // downdate tile order (see super_tile())
    bool left = false;  // left-looking: W slot k holds pick k's block column
    bool eval = false;  // design evaluation: pick k is candidate k, no gain scoring
    double tuned_ms[MAX_DELAY] = {0};  // autotuner: eager run time for delay 1..MAX_DELAY (default order)
    uint32_t flags = 0;
    hipStream_t stream = nullptr;  // the batch's own stream (graph capture and replay)
    hipStream_t caller = nullptr;  // the stream given at creation: K is complete in its order
    hipEvent_t ev_in = nullptr;    // recorded on `caller` before every pack
    // independent launch sequences: instances split into nbranch groups of about equal work, each
    // group's launches on a stream of its own (branch 0: `stream`), forked from and joined into
    // `stream`, so one group's latency-bound steps overlap another's downdates
    int nbranch = 1;
    std::vector<hipStream_t> bstream;  // branches 1 .. nbranch-1
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
    std::vector<void *> allocs;
    char *results = nullptr;  // [gains of all picks (double)][picks + state words (int)]
    size_t results_bytes = 0, n_gain = 0;
    StepDesc *d_descs = nullptr;
    std::vector<StepDesc> descs;
    std::vector<Launch> launches;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool ran = false;
    double last_ms = 0, syrk_flops = 0, syrk_bytes = 0;
    std::string err;
};

namespace {

oed_status bfail(oed_batch *b, oed_status st, const std::string &msg)
{
    if (b) b->err = msg;
    return st;
}

#define BCHK(b, call)                                                                                       \
    do {                                                                                                    \
        hipError_t e_ = (call);                                                                             \
        if (e_ != hipSuccess)                                                                               \
            return bfail(b, e_ == hipErrorOutOfMemory ? OED_E_OOM : OED_E_HIP,                             \
                         std::string(#call) + ": " + hipGetErrorString(e_));                                \
    } while (0)

hipError_t balloc(oed_batch *b, void **p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) b->allocs.push_back(*p);
    return e;
}

void bfree(oed_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (void *p : b->allocs) (void)hipFree(p);
    b->allocs.clear();
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    for (hipEvent_t e : b->ev_join)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t t : b->bstream)
        if (t) (void)hipStreamDestroy(t);
    if (b->stream) (void)hipStreamDestroy(b->stream);
}

oed_status check_instances(const oed_instance *inst, int32_t n)
{
    if (!inst || n < 1) return OED_E_ARG;
    for (int i = 0; i < n; ++i) {
        const oed_instance &x = inst[i];
        if (!x.K_dev || (x.dtype != OED_F64 && x.dtype != OED_F32) || x.N_s < 1 || x.N_t < 1 ||
            x.ld < (int64_t)x.N_s * x.N_t || !(x.sigma2 > 0.0) || !std::isfinite(x.sigma2) || x.budget < 1 ||
            x.budget > x.N_s)
            return OED_E_ARG;
        if (x.N_t > REGS_MAX_NT) return OED_E_UNSUPPORTED;
    }
    return OED_OK;
}

// Pack every working copy from inst[].K_dev on the batch stream, ordered after everything enqueued
// so far on the creation stream (where the caller wrote K), and wait for it.
oed_status pack_all(oed_batch *b, const oed_instance *inst)
{
    BCHK(b, hipEventRecord(b->ev_in, b->caller));
    BCHK(b, hipStreamWaitEvent(b->stream, b->ev_in, 0));
    for (size_t i = 0; i < b->in.size(); ++i) {
        const Inst &x = b->in[i];
        BCHK(b, launch_pack(inst[i].K_dev, x.kdtype, x.ld, x.N_t, x.N_tp, x.cmap, x.N_s, x.R, b->rtype, b->stream));
    }
    BCHK(b, hipStreamSynchronize(b->stream));
    b->ran = false;
    return OED_OK;
}

// Descriptor of instance x at step k, before (gains, pick) or after (block column, downdate)
// its k-th pick.  With delay p the block column of pick k goes to W slot k mod p; slots
// 0 .. (k mod p) - 1 hold the earlier ones, and after every p-th pick all p are subtracted in
// one downdate.
StepDesc inst_desc(const Inst &x, int k, bool after_pick, int delay, int stl = STL_COL4)
{
    StepDesc d{};
    d.stl = stl;
    d.R = x.R;
    d.W = x.W;
    d.W2 = x.W2;
    d.wslot = x.wslot;
    d.nheld = k % delay;
    d.V = x.V;
    d.nw = 1;
    d.act_in = x.act[(k + (after_pick ? 1 : 0)) & 1];
    d.act_out = x.act[(k + 1) & 1];
    d.gains = x.gains;
    d.Linv = x.Linv;
    d.fcache = x.fcache;
    d.state = x.state;
    d.picks = x.picks;
    d.pick_gain = x.pick_gain;
    d.half_noise = x.half_noise;
    d.n_act = x.N_s - k - (after_pick ? 1 : 0);
    d.N_t = x.N_t;
    d.N_tp = x.N_tp;
    d.step = k;
    d.forced = -1;
    return d;
}

// Left-looking descriptor of instance x at step k.  Before the pick (gains) the newest block
// column, slot k - 1, is applied to the diagonal blocks in place; after the pick the column kernel
// sums slots 0 .. k-1 and the block column of pick k goes to slot k.
StepDesc inst_desc_left(const oed_batch *b, const Inst &x, int k, bool after_pick)
{
    StepDesc d = inst_desc(x, k, after_pick, 1);
    const size_t we = b->wtype == W_F64 ? 8 : b->wtype == W_F32 ? 4 : 2;
    const int64_t bs = (int64_t)x.N_tp * x.N_tp;
    d.nheld = 0;
    if (!after_pick) {
        if (k >= 1) {
            d.W = (char *)x.W + (size_t)((k - 1) * x.wslot) * we;
            if (x.W2) d.W2 = (char *)x.W2 + (size_t)((k - 1) * x.wslot) * 2;
            d.nheld = 1;
            d.wb = 1;
        }
        return d;
    }
    d.C = x.C;
    d.cstride = (int64_t)x.N_s * bs;
    d.nsplit = std::min(LEFT_SPLITS, k);
    d.nw = k;
    return d;
}

// Output slot k of the block-column launch after pick k (left-looking).
void left_out_slot(const oed_batch *b, const Inst &x, int k, StepDesc &d)
{
    const size_t we = b->wtype == W_F64 ? 8 : b->wtype == W_F32 ? 4 : 2;
    d.W = (char *)x.W + (size_t)(k * x.wslot) * we;
    if (x.W2) d.W2 = (char *)x.W2 + (size_t)(k * x.wslot) * 2;
}

void build_branch_left(oed_batch *b, int br)
{
    const double e = b->rtype == R_F64 ? 8.0 : 4.0;
    int maxB = 0;
    for (size_t i = 0; i < b->in.size(); ++i) {
        if (b->in[i].branch != br) continue;
        maxB = std::max(maxB, b->in[i].budget);
        Launch L = make_launch(L_INIT, 0);
        L.inst = (int)i;
        b->launches.push_back(L);
    }
    auto mine = [&](const Inst &x) { return x.branch == br; };
    for (int k = 0; k < maxB; ++k) {
        Launch g = make_launch(L_GAIN, (int64_t)b->descs.size());
        for (const Inst &x : b->in)
            if (mine(x) && x.budget > k) {
                StepDesc d = inst_desc_left(b, x, k, false);
                d.item0 = g.total;
                d.nitems = d.n_act;
                g.total += d.nitems;
                b->descs.push_back(d);
                ++g.ndesc;
            }
        b->launches.push_back(g);
        Launch p = make_launch(L_PICK, (int64_t)b->descs.size());
        for (const Inst &x : b->in)
            if (mine(x) && x.budget > k) {
                StepDesc d = inst_desc_left(b, x, k, false);
                d.nheld = 0;
                d.wb = 0;
                d.item0 = p.total;
                d.nitems = 1;
                p.total += 1;
                p.max_Nt = std::max(p.max_Nt, x.N_t);
                b->descs.push_back(d);
                ++p.ndesc;
            }
        b->launches.push_back(p);
        // block column of pick k for the instances that pick again
        std::map<int, std::vector<const Inst *>> by_ntp;
        for (const Inst &x : b->in)
            if (mine(x) && x.budget > k + 1 && k >= 1) by_ntp[x.N_tp].push_back(&x);
        for (auto &kv : by_ntp) {
            Launch c = make_launch(L_COLUMN, (int64_t)b->descs.size());
            c.N_tp = kv.first;
            for (const Inst *x : kv.second) {
                StepDesc d = inst_desc_left(b, *x, k, true);
                d.item0 = c.total;
                d.nitems = (int64_t)d.nsplit * syrk_tile_rows(d.n_act, d.N_tp);
                c.total += d.nitems;
                b->descs.push_back(d);
                ++c.ndesc;
                const double n = (double)d.n_act * x->N_t;
                b->syrk_flops += 2.0 * n * x->N_t * k * x->N_t;
                b->syrk_bytes += e * (n * k * x->N_t + (double)k * x->N_t * x->N_t + d.nsplit * n * x->N_t);
            }
            b->launches.push_back(c);
        }
        Launch t = make_launch(L_TRSM, (int64_t)b->descs.size());
        for (const Inst &x : b->in)
            if (mine(x) && x.budget > k + 1) {
                StepDesc d = inst_desc_left(b, x, k, true);
                left_out_slot(b, x, k, d);
                d.item0 = t.total;
                d.nitems = d.n_act;
                t.total += d.nitems;
                b->descs.push_back(d);
                ++t.ndesc;
            }
        if (t.ndesc) b->launches.push_back(t);
    }
}

// The descriptors and launches of branch br (the instances with x.branch == br).
void build_branch(oed_batch *b, int br)
{
    const double e = b->rtype == R_F64 ? 8.0 : 4.0;
    int maxB = 0;
    for (size_t i = 0; i < b->in.size(); ++i) {
        if (b->in[i].branch != br) continue;
        maxB = std::max(maxB, b->in[i].budget);
        Launch L = make_launch(L_INIT, 0);
        L.inst = (int)i;
        b->launches.push_back(L);
    }
    auto mine = [&](const Inst &x) { return x.branch == br; };
    for (int k = 0; k < maxB; ++k) {
        // gains and pick of step k (design evaluation: no gains, the pick is candidate k)
        if (!b->eval) {
            Launch g = make_launch(L_GAIN, (int64_t)b->descs.size());
            for (const Inst &x : b->in)
                if (mine(x) && x.budget > k) {
                    StepDesc d = inst_desc(x, k, false, b->delay);
                    // eager diagonal: apply the newest block column (pick k - 1, slot (k - 1) mod
                    // delay) to the diagonal blocks and write them back; the rest are included
                    d.nheld = 0;
                    if (k >= 1) {
                        const size_t we = b->wtype == W_F64 ? 8 : b->wtype == W_F32 ? 4 : 2;
                        const int slot = (k - 1) % b->delay;
                        d.W = (char *)x.W + (size_t)(slot * x.wslot) * we;
                        if (x.W2) d.W2 = (char *)x.W2 + (size_t)(slot * x.wslot) * 2;
                        d.nheld = 1;
                        d.wb = 1;
                    }
                    d.item0 = g.total;
                    d.nitems = d.n_act;
                    g.total += d.nitems;
                    b->descs.push_back(d);
                    ++g.ndesc;
                }
            b->launches.push_back(g);
        }
        Launch p = make_launch(L_PICK, (int64_t)b->descs.size());
        for (const Inst &x : b->in)
            if (mine(x) && x.budget > k) {
                StepDesc d = inst_desc(x, k, false, b->delay);
                if (b->eval)
                    d.forced = k;  // no gain launches: the pick applies the held columns itself
                else
                    d.nheld = 0;   // the winner's diagonal block is current
                d.item0 = p.total;
                d.nitems = 1;
                p.total += 1;
                p.max_Nt = std::max(p.max_Nt, x.N_t);
                b->descs.push_back(d);
                ++p.ndesc;
            }
        b->launches.push_back(p);
        // block column and downdate for the instances that pick again; with delay p the
        // block column is held unless this is the p-th pick since the last downdate
        const bool hold = (k % b->delay) + 1 < b->delay;
        const bool corr = k % b->delay > 0;
        const int nw = k % b->delay + 1;
        if (corr) {
            Launch v = make_launch(L_VCORR, (int64_t)b->descs.size());
            for (const Inst &x : b->in)
                if (mine(x) && x.budget > k + 1) {
                    StepDesc d = inst_desc(x, k, true, b->delay);
                    d.item0 = v.total;
                    d.nitems = (int64_t)d.nheld * (x.N_tp / 16) * (x.N_tp / 16);
                    v.total += d.nitems;
                    b->descs.push_back(d);
                    ++v.ndesc;
                }
            if (v.ndesc) b->launches.push_back(v);
        }
        Launch t = make_launch(L_TRSM, (int64_t)b->descs.size());
        std::map<int, std::vector<const Inst *>> by_ntp;
        for (const Inst &x : b->in)
            if (mine(x) && x.budget > k + 1) {
                StepDesc d = inst_desc(x, k, true, b->delay);
                d.item0 = t.total;
                d.nitems = d.n_act;
                t.total += d.nitems;
                b->descs.push_back(d);
                ++t.ndesc;
                by_ntp[x.N_tp].push_back(&x);
                if (!hold) {
                    const double nr = (double)d.n_act * x.N_t;
                    b->syrk_flops += nw * (double)x.N_t * nr * (nr + 1.0);
                    b->syrk_bytes += e * (nr * (nr + x.N_t) + nw * nr * x.N_t);
                }
            }
        if (t.ndesc == 0) continue;
        b->launches.push_back(t);
        if (hold) continue;
        for (auto &kv : by_ntp) {
            Launch s = make_launch(L_SYRK, (int64_t)b->descs.size());
            s.N_tp = kv.first;
            s.nw = nw;
            for (const Inst *x : kv.second) {
                StepDesc d = inst_desc(*x, k, true, b->delay, b->stl);
                d.nw = s.nw;
                d.skipdiag = b->eval ? 0 : 1;  // kept current by the gain launches
                d.item0 = s.total;
                d.nitems = syrk_tiles(d.n_act, d.N_tp, b->stl);
                s.total += d.nitems;
                b->descs.push_back(d);
                ++s.ndesc;
            }
            b->launches.push_back(s);
        }
    }
}

// Build the descriptor array and the launch list of one run: branch after branch, each launch
// tagged with its branch.
void build_schedule(oed_batch *b)
{
    b->descs.clear();
    b->launches.clear();
    b->syrk_flops = b->syrk_bytes = 0;
    for (int br = 0; br < b->nbranch; ++br) {
        const size_t l0 = b->launches.size();
        if (b->left)
            build_branch_left(b, br);
        else
            build_branch(b, br);
        for (size_t l = l0; l < b->launches.size(); ++l) b->launches[l].branch = br;
    }
}

oed_status enqueue_run(oed_batch *b)
{
    // fork: every branch starts after what `stream` holds (the packs); join at the end
    if (b->nbranch > 1) {
        BCHK(b, hipEventRecord(b->ev_fork, b->stream));
        for (int br = 1; br < b->nbranch; ++br) BCHK(b, hipStreamWaitEvent(b->bstream[br - 1], b->ev_fork, 0));
    }
    for (const Launch &L : b->launches) {
        const StepDesc *d = b->d_descs + L.desc0;
        const hipStream_t stream = L.branch == 0 ? b->stream : b->bstream[L.branch - 1];
        switch (L.kind) {
        case L_INIT: {
            const Inst &x = b->in[L.inst];
            BCHK(b, launch_init_state(x.act[0], x.N_s, x.state, stream));
            break;
        }
        case L_GAIN: BCHK(b, launch_gain_batched(d, L.ndesc, L.total, b->rtype, b->wtype, stream)); break;
        case L_PICK: BCHK(b, launch_pick_batched(d, L.ndesc, L.max_Nt, b->rtype, b->wtype, stream)); break;
        case L_VCORR: BCHK(b, launch_vcorr_batched(d, L.ndesc, L.total, b->wtype, stream)); break;
        case L_COLUMN:
            BCHK(b, launch_column_batched(d, L.ndesc, L.total, L.N_tp, b->rtype, b->wtype, stream));
            break;
        case L_TRSM: BCHK(b, launch_trsm_batched(d, L.ndesc, L.total, b->rtype, b->wtype, stream)); break;
        case L_SYRK:
            BCHK(b, launch_syrk_batched(d, L.ndesc, L.total, L.N_tp, L.nw, b->rtype, b->wtype, SYRK_LDS, stream));
            break;
        }
    }
    if (b->nbranch > 1) {
        for (int br = 1; br < b->nbranch; ++br) {
            BCHK(b, hipEventRecord(b->ev_join[br - 1], b->bstream[br - 1]));
            BCHK(b, hipStreamWaitEvent(b->stream, b->ev_join[br - 1], 0));
        }
    }
    return OED_OK;
}

// Split the instances into b->nbranch groups of about equal work: largest first, each to the
// group with the least work so far (ties to the lowest group); work = the downdate flops of the
// whole selection, sum over the steps of N_t n^2 (n = remaining rows).
void assign_branches(oed_batch *b)
{
    const int n = (int)b->in.size();
    std::vector<double> cost(n, 0.0);
    for (int i = 0; i < n; ++i) {
        const Inst &x = b->in[i];
        for (int k = 0; k < x.budget; ++k) {
            const double r = (double)(x.N_s - k) * x.N_t;
            cost[i] += x.N_t * r * r;
        }
    }
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });
    std::vector<double> load(b->nbranch, 0.0);
    for (int i : order) {
        const int br = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        b->in[i].branch = br;
        load[br] += cost[i];
    }
}

// Autotuner (OED_BATCH_AUTOTUNE with no delay given): runs the whole selection once per delay
// depth p = 1..MAX_DELAY, eagerly, from freshly packed working copies, and keeps the fastest.
// All depths give the same picks up to rounding; W slots for MAX_DELAY are allocated.
oed_status autotune_batch(oed_batch *b, const oed_instance *inst, bool tiles, bool branches)
{
    auto timed_run = [&](double *out) -> oed_status {
        build_schedule(b);
        BCHK(b, hipMemcpy(b->d_descs, b->descs.data(), sizeof(StepDesc) * b->descs.size(), hipMemcpyHostToDevice));
        oed_status st = pack_all(b, inst);
        if (st != OED_OK) return st;
        BCHK(b, hipEventRecord(b->ev0, b->stream));
        st = enqueue_run(b);
        if (st != OED_OK) return st;
        BCHK(b, hipEventRecord(b->ev1, b->stream));
        BCHK(b, hipEventSynchronize(b->ev1));
        float ms = 0;
        BCHK(b, hipEventElapsedTime(&ms, b->ev0, b->ev1));
        *out = ms;
        return OED_OK;
    };
    double best = 1e300;
    int best_p = b->delay;
    for (int p = 1; p <= MAX_DELAY; ++p) {
        b->delay = p;
        oed_status st = timed_run(&b->tuned_ms[p - 1]);
        if (st != OED_OK) return st;
        if (b->tuned_ms[p - 1] < best) {
            best = b->tuned_ms[p - 1];
            best_p = p;
        }
    }
    b->delay = best_p;
    if (!tiles) return OED_OK;
    // the other tile orders at the chosen depth, each kept only when 1% faster (as the handle's tuner)
    const int orders[] = {STL_COL2, STL_COL8, STL_ROW8};
    int best_stl = b->stl;
    for (int o : orders) {
        b->stl = o;
        double ms = 0;
        oed_status st = timed_run(&ms);
        if (st != OED_OK) return st;
        if (ms < 0.99 * best) {
            best = ms;
            best_stl = o;
        }
    }
    b->stl = best_stl;
    if (!branches) return OED_OK;
    // 1 .. the most branches the streams were made for, at the chosen depth and order
    int best_br = b->nbranch;
    for (int nb = 1; nb <= (int)b->bstream.size() + 1; ++nb) {
        if (nb == b->nbranch) continue;
        const int keep = b->nbranch;
        b->nbranch = nb;
        assign_branches(b);
        double ms = 0;
        oed_status st = timed_run(&ms);
        if (st != OED_OK) return st;
        if (ms < best) {
            best = ms;
            best_br = nb;
        }
        b->nbranch = keep;
    }
    b->nbranch = best_br;
    assign_branches(b);
    return OED_OK;
}

}  // namespace

extern "C" {

// Batch creation; eval: design evaluation (pick k forced to candidate k, no gains, nothing
// packed: the caller sets every instance's candidate map and packs before each run).
static oed_status create_batch(oed_batch **out, const oed_instance *inst, int32_t n, int32_t precision,
                               void *stream, uint32_t flags, bool eval)
{
    if (!out) return OED_E_ARG;
    *out = nullptr;
    oed_status st = check_instances(inst, n);
    if (st != OED_OK) return st;
    if (precision != OED_PREC_FP64 && precision != OED_PREC_MIXED_F32 && precision != OED_PREC_MIXED_BF16X3)
        return OED_E_ARG;
    if (((flags >> 8) & 0xFu) > (unsigned)MAX_DELAY) return OED_E_ARG;
    const unsigned tiles = (flags >> 12) & 0xFu;
    if (tiles > OED_TILES_COL2) return OED_E_ARG;
    const unsigned branches = (flags >> 16) & 0xFu;
    if (branches > OED_BATCH_MAX_BRANCHES) return OED_E_ARG;
    oed_batch *b = new (std::nothrow) oed_batch();
    if (!b) return OED_E_OOM;
    b->prec = precision;
    b->rtype = precision == OED_PREC_FP64 ? R_F64 : R_F32;
    b->wtype = precision == OED_PREC_FP64 ? W_F64 : precision == OED_PREC_MIXED_F32 ? W_F32 : W_BF16X3;
    b->flags = flags;
    b->delay = (int)((flags >> 8) & 0xFu);
    b->left = (flags & OED_BATCH_LEFT_LOOKING) != 0;
    b->eval = eval;
    const bool tune = !b->left && b->delay == 0 && (flags & OED_BATCH_AUTOTUNE);
    static const int stl_of[] = {STL_COL4, STL_ROW8, STL_COL8, STL_COL4, STL_COL2};
    b->stl = stl_of[tiles];
    b->nbranch = std::min<int>(n, branches == 0 ? DEFAULT_BRANCHES : (int)branches);
    const bool tune_br = tune && !eval && branches == 0;
    if (b->delay == 0) b->delay = DEFAULT_DELAY;
    if (b->left) b->delay = 1;
    // W slots and held-column buffers for the deepest delay the batch may run with
    const int max_p = tune ? MAX_DELAY : b->delay;
    auto setup = [&]() -> oed_status {
        // the caller's K must be complete before the batch stream reads it
        b->caller = (hipStream_t)stream;
        BCHK(b, hipStreamSynchronize(b->caller));
        BCHK(b, hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
        BCHK(b, hipEventCreate(&b->ev0));
        BCHK(b, hipEventCreate(&b->ev1));
        BCHK(b, hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
        // streams and events for the most branches the batch may run with
        const int max_br = std::min<int>(n, tune_br ? OED_BATCH_MAX_BRANCHES : (int)b->nbranch);
        BCHK(b, hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
        b->bstream.assign(std::max(0, max_br - 1), nullptr);
        b->ev_join.assign(std::max(0, max_br - 1), nullptr);
        for (int q = 0; q + 1 < max_br; ++q) {
            BCHK(b, hipStreamCreateWithFlags(&b->bstream[q], hipStreamNonBlocking));
            BCHK(b, hipEventCreateWithFlags(&b->ev_join[q], hipEventDisableTiming));
        }
        const size_t er = b->rtype == R_F64 ? 8 : 4;
        size_t n_gain = 0, n_int = 0;
        b->in.resize(n);
        for (int i = 0; i < n; ++i) {
            Inst &x = b->in[i];
            const oed_instance &y = inst[i];
            x.N_s = y.N_s;
            x.N_t = y.N_t;
            x.N_tp = b->wtype == W_BF16X3 ? (y.N_t + 31) / 32 * 32 : (y.N_t + 15) / 16 * 16;
            x.budget = y.budget;
            x.kdtype = y.dtype;
            x.ld = y.ld;
            x.sigma2 = y.sigma2;
            x.half_noise = 0.5 * y.N_t * std::log(y.sigma2);
            const int64_t bs = (int64_t)x.N_tp * x.N_tp, nblk = (int64_t)x.N_s * (x.N_s + 1) / 2;
            BCHK(b, balloc(b, &x.R, (size_t)(nblk * bs) * er));
            x.wslot = x.N_s * bs;
            const int slots = b->left ? x.budget : max_p;
            if (b->wtype == W_BF16X3) {
                BCHK(b, balloc(b, &x.W, (size_t)(slots * x.wslot) * 2));
                BCHK(b, balloc(b, &x.W2, (size_t)(slots * x.wslot) * 2));
            } else {
                BCHK(b, balloc(b, &x.W, (size_t)(slots * x.wslot) * er));
            }
            if (max_p > 1) BCHK(b, balloc(b, (void **)&x.V, sizeof(double) * bs * (max_p - 1)));
            if (b->left) BCHK(b, balloc(b, &x.C, (size_t)(LEFT_SPLITS * x.N_s * bs) * er));
            BCHK(b, balloc(b, (void **)&x.Linv, sizeof(double) * bs));
            BCHK(b, balloc(b, (void **)&x.gains, sizeof(double) * x.N_s));
            if (!eval) BCHK(b, balloc(b, (void **)&x.fcache, sizeof(double) * 256 * FCACHE_BLOCKS * x.N_s));
            BCHK(b, balloc(b, (void **)&x.act[0], sizeof(int) * x.N_s));
            BCHK(b, balloc(b, (void **)&x.act[1], sizeof(int) * x.N_s));
            BCHK(b, balloc(b, (void **)&x.cmap, sizeof(int) * x.N_s));
            std::vector<int> id(x.N_s);
            for (int q = 0; q < x.N_s; ++q) id[q] = q;
            BCHK(b, hipMemcpy(x.cmap, id.data(), sizeof(int) * x.N_s, hipMemcpyHostToDevice));
            x.off_gain = n_gain;
            n_gain += x.budget;
            x.off_int = n_int;
            n_int += x.budget + ST_WORDS;
        }
        b->n_gain = n_gain;
        assign_branches(b);
        b->results_bytes = sizeof(double) * n_gain + sizeof(int) * n_int;
        BCHK(b, balloc(b, (void **)&b->results, b->results_bytes));
        int *ires = (int *)(b->results + sizeof(double) * n_gain);
        for (Inst &x : b->in) {
            x.pick_gain = (double *)b->results + x.off_gain;
            x.picks = ires + x.off_int;
            x.state = x.picks + x.budget;
        }
        // descriptor array sized for the longest schedule (every delay depth the tuner may try)
        size_t ndesc = 1;
        for (int p = tune ? 1 : b->delay; p <= max_p; ++p) {
            const int keep = b->delay, keep_br = b->nbranch;
            b->delay = p;
            for (int nb = 1; nb <= (int)b->bstream.size() + 1; ++nb) {
                b->nbranch = nb;
                assign_branches(b);
                build_schedule(b);
                ndesc = std::max(ndesc, b->descs.size());
            }
            b->delay = keep;
            b->nbranch = keep_br;
            assign_branches(b);
        }
        BCHK(b, balloc(b, (void **)&b->d_descs, sizeof(StepDesc) * ndesc));
        if (tune) {
            oed_status s2 = autotune_batch(b, inst, !eval && tiles == OED_TILES_AUTO, tune_br);
            if (s2 != OED_OK) return s2;
        }
        build_schedule(b);
        BCHK(b, hipMemcpy(b->d_descs, b->descs.data(), sizeof(StepDesc) * b->descs.size(), hipMemcpyHostToDevice));
        return eval ? OED_OK : pack_all(b, inst);
    };
    st = setup();
    if (st != OED_OK) {
        bfree(b);
        delete b;
        return st;
    }
    *out = b;
    return OED_OK;
}

oed_status oed_batch_create(oed_batch **out, const oed_instance *inst, int32_t n, int32_t precision, void *stream,
                            uint32_t flags)
{
    return create_batch(out, inst, n, precision, stream, flags, false);
}

oed_status oed_batch_get_config(const oed_batch *b, int32_t *delay, int32_t *tile_order, int32_t *branches,
                                double *per_run_ms)
{
    if (!b) return OED_E_ARG;
    if (delay) *delay = b->delay;
    if (branches) *branches = b->nbranch;
    if (tile_order)
        *tile_order = b->stl == STL_ROW8 ? OED_TILES_ROW8 : b->stl == STL_COL8 ? OED_TILES_COL8
                      : b->stl == STL_COL4 ? OED_TILES_COL4 : OED_TILES_COL2;
    if (per_run_ms) std::copy(b->tuned_ms, b->tuned_ms + MAX_DELAY, per_run_ms);
    return OED_OK;
}

oed_status oed_batch_reset(oed_batch *b, const oed_instance *inst, int32_t n)
{
    if (!b) return OED_E_ARG;
    if (n != (int32_t)b->in.size() || check_instances(inst, n) != OED_OK) return bfail(b, OED_E_ARG, "bad instances");
    for (int i = 0; i < n; ++i)
        if (inst[i].N_s != b->in[i].N_s || inst[i].N_t != b->in[i].N_t || inst[i].budget != b->in[i].budget ||
            inst[i].dtype != b->in[i].kdtype || inst[i].ld != b->in[i].ld)
            return bfail(b, OED_E_ARG, "instance shape differs from creation");
    return pack_all(b, inst);
}

oed_status oed_batch_run(oed_batch *b, int32_t *idx_out, double *gain_out, int32_t *n_out, int32_t *status_out)
{
    if (!b || !idx_out || !gain_out || !n_out || !status_out) return OED_E_ARG;
    if (b->ran) return bfail(b, OED_E_STATE, "batch already ran: reset it first");
    const bool graph = !(b->flags & OED_BATCH_NO_GRAPH);
    if (graph && !b->exec) {
        BCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
        oed_status st = enqueue_run(b);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(b->stream, &g);
        if (st != OED_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        BCHK(b, e);
        b->graph = g;
        BCHK(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    const bool prof = b->flags & OED_FLAG_PROFILE;
    if (prof) BCHK(b, hipEventRecord(b->ev0, b->stream));
    if (graph) {
        BCHK(b, hipGraphLaunch(b->exec, b->stream));
    } else {
        oed_status st = enqueue_run(b);
        if (st != OED_OK) return st;
    }
    if (prof) BCHK(b, hipEventRecord(b->ev1, b->stream));
    std::vector<char> h(b->results_bytes);
    BCHK(b, hipMemcpyAsync(h.data(), b->results, b->results_bytes, hipMemcpyDeviceToHost, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    b->ran = true;
    if (prof) {
        float ms = 0;
        BCHK(b, hipEventElapsedTime(&ms, b->ev0, b->ev1));
        b->last_ms = ms;
    }
    const double *hg = (const double *)h.data();
    const int *hi = (const int *)(h.data() + sizeof(double) * b->n_gain);
    size_t o = 0;
    oed_status worst = OED_OK;
    for (size_t i = 0; i < b->in.size(); ++i) {
        const Inst &x = b->in[i];
        const int *picks = hi + x.off_int, *state = picks + x.budget;
        const int made = std::max(0, std::min(x.budget, state[ST_NPICKS]));
        for (int q = 0; q < x.budget; ++q) {
            idx_out[o + q] = q < made ? picks[q] : -1;
            gain_out[o + q] = q < made ? hg[x.off_gain + q] : NAN;
        }
        n_out[i] = made;
        status_out[i] = state[ST_STATUS] == 0 ? OED_OK : state[ST_STATUS] == 2 ? OED_E_NOT_SPD : OED_E_STATE;
        if (status_out[i] != OED_OK) worst = OED_E_NOT_SPD;
        o += x.budget;
    }
    if (worst != OED_OK) return bfail(b, worst, "an instance stopped early; see status_out");
    return OED_OK;
}

oed_status oed_batch_stats(const oed_batch *b, double *run_ms, double *syrk_flops, double *syrk_bytes)
{
    if (!b) return OED_E_ARG;
    if (run_ms) *run_ms = b->last_ms;
    if (syrk_flops) *syrk_flops = b->syrk_flops;
    if (syrk_bytes) *syrk_bytes = b->syrk_bytes;
    return OED_OK;
}

oed_status oed_batch_destroy(oed_batch *b)
{
    if (!b) return OED_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    bfree(b);
    delete b;
    return OED_OK;
}

const char *oed_batch_last_error(const oed_batch *b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// Design evaluation: every design is one instance of an evaluation batch whose candidates are
// the design's sensors in the given order and whose k-th pick is forced to candidate k, so the
// pick kernel factors the Schur complement of s_k given s_0 .. s_{k-1} and records its term;
// the block-column and downdate launches are the selection's.  The batch (its memory, schedule
// and graph) is built once; a run fills the candidate maps, packs and replays it per chunk.

struct oed_eval {
    oed_batch *b = nullptr;
    std::vector<oed_instance> inst;  // nb copies of (K, N_t, B candidates, budget B)
    hipStream_t caller = nullptr;
    int N_s = 0, N_t = 0, B = 0, nb = 0;
    double last_ms = 0, syrk_flops = 0;
    int64_t executed = 0;
    std::string err;
};

namespace {

oed_status efail(oed_eval *e, oed_status st, const std::string &msg)
{
    if (e) e->err = msg;
    return st;
}

// Device bytes of one evaluation instance (working copy, W slots, V, L^-1 and small arrays).
size_t eval_inst_bytes(int B, int N_t, int precision, int delay)
{
    const bool bf = precision == OED_PREC_MIXED_BF16X3;
    const size_t er = precision == OED_PREC_FP64 ? 8 : 4, ew = bf ? 4 : er;
    const size_t N_tp = bf ? (N_t + 31) / 32 * 32 : (N_t + 15) / 16 * 16, bs = N_tp * N_tp;
    return (size_t)B * (B + 1) / 2 * bs * er + (size_t)delay * B * bs * ew + (size_t)delay * bs * 8 +
           (size_t)B * 64 + 4096;
}

}  // namespace

extern "C" {

oed_status oed_eval_create(oed_eval **out, const void *K_dev, int32_t dtype, int64_t ld, int32_t N_s, int32_t N_t,
                           double sigma2, int32_t B, int32_t max_batch, int32_t precision, void *stream,
                           uint32_t flags)
{
    if (!out) return OED_E_ARG;
    *out = nullptr;
    if (!K_dev || (dtype != OED_F64 && dtype != OED_F32) || N_s < 1 || N_t < 1 || ld < (int64_t)N_s * N_t ||
        !(sigma2 > 0.0) || !std::isfinite(sigma2) || B < 1 || B > N_s || max_batch < 0)
        return OED_E_ARG;
    if (precision != OED_PREC_FP64 && precision != OED_PREC_MIXED_F32 && precision != OED_PREC_MIXED_BF16X3)
        return OED_E_ARG;
    if (flags & ~(uint32_t)(OED_FLAG_PROFILE | OED_BATCH_NO_GRAPH | 0xF00u)) return OED_E_ARG;
    const int delay = (int)((flags >> 8) & 0xFu);
    if (delay > MAX_DELAY) return OED_E_ARG;
    if (N_t > REGS_MAX_NT) return OED_E_UNSUPPORTED;
    int nb = max_batch;
    if (nb == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return OED_E_HIP;
        const size_t per = eval_inst_bytes(B, N_t, precision, delay ? delay : DEFAULT_DELAY);
        nb = (int)std::max<size_t>(1, std::min<size_t>(64, fr / 2 / per));
    }
    oed_eval *e = new (std::nothrow) oed_eval();
    if (!e) return OED_E_OOM;
    e->N_s = N_s;
    e->N_t = N_t;
    e->B = B;
    e->nb = nb;
    e->caller = (hipStream_t)stream;
    oed_instance x{};
    x.K_dev = K_dev;
    x.dtype = dtype;
    x.N_s = B;
    x.N_t = N_t;
    x.budget = B;
    x.ld = ld;
    x.sigma2 = sigma2;
    e->inst.assign(nb, x);
    const oed_status st = create_batch(&e->b, e->inst.data(), nb, precision, stream, flags, true);
    if (st != OED_OK) {
        delete e;
        return st;
    }
    *out = e;
    return OED_OK;
}

oed_status oed_eval_run(oed_eval *e, const int32_t *designs, int32_t n, double *obj_out, double *terms_out)
{
    if (!e) return OED_E_ARG;
    if (n < 0 || (n > 0 && (!designs || !obj_out))) return efail(e, OED_E_ARG, "bad arguments");
    const int B = e->B, nb = e->nb;
    std::vector<char> seen(e->N_s);
    for (int64_t r = 0; r < n; ++r) {
        std::fill(seen.begin(), seen.end(), 0);
        for (int k = 0; k < B; ++k) {
            const int32_t s = designs[r * B + k];
            if (s < 0 || s >= e->N_s || seen[s])
                return efail(e, OED_E_ARG, "design " + std::to_string(r) + ": sensor out of range or repeated");
            seen[s] = 1;
        }
    }
    oed_batch *b = e->b;
    if (hipStreamSynchronize(e->caller) != hipSuccess) return efail(e, OED_E_HIP, "caller stream");
    std::vector<int32_t> idx((size_t)nb * B), made(nb), stat(nb);
    std::vector<double> g((size_t)nb * B);
    e->last_ms = 0;
    e->syrk_flops = 0;
    e->executed = 0;
    oed_status worst = OED_OK;
    for (int64_t c0 = 0; c0 < n; c0 += nb) {
        const int cnt = (int)std::min<int64_t>(nb, n - c0);
        // a short last chunk repeats its last design in the unused instances
        for (int i = 0; i < nb; ++i) {
            const int32_t *S = designs + (size_t)(c0 + std::min(i, cnt - 1)) * B;
            if (hipMemcpy(b->in[i].cmap, S, sizeof(int32_t) * B, hipMemcpyHostToDevice) != hipSuccess)
                return efail(e, OED_E_HIP, "candidate map upload");
        }
        oed_status st = pack_all(b, e->inst.data());
        if (st != OED_OK) return efail(e, st, b->err);
        st = oed_batch_run(b, idx.data(), g.data(), made.data(), stat.data());
        if (st != OED_OK && st != OED_E_NOT_SPD) return efail(e, st, b->err);
        e->last_ms += b->last_ms;
        e->syrk_flops += b->syrk_flops;
        e->executed += nb;
        for (int i = 0; i < cnt; ++i) {
            const size_t r = (size_t)(c0 + i);
            bool ok = stat[i] == OED_OK && made[i] == B;
            double sum = 0.0;
            for (int k = 0; k < B; ++k) {
                const bool have = k < made[i] && idx[(size_t)i * B + k] == k;
                ok = ok && have;
                const double t = have ? g[(size_t)i * B + k] : NAN;
                sum += t;
                if (terms_out) terms_out[r * B + k] = t;
            }
            obj_out[r] = ok ? sum : NAN;
            if (!ok) worst = OED_E_NOT_SPD;
        }
    }
    if (worst != OED_OK)
        return efail(e, worst, "a design has a Schur block that is not positive definite: its objective is NaN");
    return OED_OK;
}

oed_status oed_eval_stats(const oed_eval *e, double *run_ms, double *syrk_flops, int64_t *executed, int32_t *batch)
{
    if (!e) return OED_E_ARG;
    if (run_ms) *run_ms = e->last_ms;
    if (syrk_flops) *syrk_flops = e->syrk_flops;
    if (executed) *executed = e->executed;
    if (batch) *batch = e->nb;
    return OED_OK;
}

oed_status oed_eval_destroy(oed_eval *e)
{
    if (!e) return OED_OK;
    (void)oed_batch_destroy(e->b);
    delete e;
    return OED_OK;
}

const char *oed_eval_last_error(const oed_eval *e) { return e ? e->err.c_str() : "null evaluator"; }

}  // extern "C"
