// oed_greedy_noalloc: a whole greedy selection that allocates nothing (declaration and contract in
// include/oed.h).  The working copy R, the W slots, L_s^-1, the held-column corrections, the
// gains, the active lists and the state words live in one file-scope device array, `scratch`,
// of OED_NOALLOC_MAX_BYTES (the factor cache of the pick too); the kernels are those of oed_create / oed_greedy (right-looking,
// fixed delay depth, LDS downdate), launched in the same order, so the picks and gains are
// bitwise those of a handle created with the same precision and delay.
//
// In host code the name `scratch` is a host-side stand-in and must never reach a kernel or a
// copy: its device address is taken once per device with hipGetSymbolAddress (with that device
// current) and kept in g_scratch[device]; every use goes through that pointer.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "../../include/oed.h"
#include "oed_internal.h"

using namespace oed;

static __device__ __align__(256) double scratch[OED_NOALLOC_MAX_BYTES / sizeof(double)];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[MAX_DEVICES] = {nullptr};

oed_status report(char *err, int32_t err_len, oed_status st, const char *fmt, ...)
{
    if (err && err_len > 0) {
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(err, (size_t)err_len, fmt, ap);
        va_end(ap);
    }
    return st;
}

int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

// Byte offsets of the buffers inside the scratch array (each 256-byte aligned).
struct Layout {
    int64_t R, W, W2, V, Linv, gains, fcache, act0, act1, cmap, state, total;
};

Layout layout(int N, int N_tp, int prec, int delay)
{
    const int64_t bs = (int64_t)N_tp * N_tp;
    const int64_t re = prec == OED_PREC_FP64 ? 8 : 4;
    const int64_t we = prec == OED_PREC_FP64 ? 8 : prec == OED_PREC_MIXED_F32 ? 4 : 2;
    Layout L{};
    int64_t o = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = o;
        o += align256(bytes);
        return at;
    };
    L.R = take((int64_t)N * (N + 1) / 2 * bs * re);
    L.W = take(delay * (int64_t)N * bs * we);
    L.W2 = prec == OED_PREC_MIXED_BF16X3 ? take(delay * (int64_t)N * bs * 2) : -1;
    L.V = delay > 1 ? take((int64_t)(delay - 1) * bs * 8) : -1;
    L.Linv = take(bs * 8);
    L.gains = take((int64_t)N * 8);
    L.fcache = take((int64_t)N * FCACHE_BLOCKS * 256 * 8);
    L.act0 = take((int64_t)N * 4);
    L.act1 = take((int64_t)N * 4);
    L.cmap = take((int64_t)N * 4);
    L.state = take((int64_t)ST_WORDS * 4);
    L.total = o;
    return L;
}

}  // namespace

extern "C" {

OED_API oed_status oed_greedy_noalloc(const void *K_dev, int32_t dtype, int64_t ld, int32_t N_s, int32_t N_t,
                                      double sigma2, int32_t precision, int32_t delay, int32_t budget, void *stream,
                                      int32_t *idx_dev, double *gain_dev, int32_t *status_dev, char *err,
                                      int32_t err_len)
{
    if (err && err_len > 0) err[0] = 0;
    if (!K_dev || (dtype != OED_F64 && dtype != OED_F32) || N_s < 1 || N_t < 1 || ld < (int64_t)N_s * N_t ||
        !(sigma2 > 0.0) || !std::isfinite(sigma2))
        return report(err, err_len, OED_E_ARG, "bad K, dtype, shape, leading dimension or sigma2");
    if (precision != OED_PREC_FP64 && precision != OED_PREC_MIXED_F32 && precision != OED_PREC_MIXED_BF16X3)
        return report(err, err_len, OED_E_ARG, "unknown precision %d", (int)precision);
    if (N_t > REGS_MAX_NT)
        return report(err, err_len, OED_E_UNSUPPORTED, "N_t = %d: the no-allocation selection serves N_t <= %d",
                      (int)N_t, REGS_MAX_NT);
    if (delay == 0) delay = DEFAULT_DELAY;
    if (delay < 1 || delay > MAX_DELAY) return report(err, err_len, OED_E_ARG, "delay %d out of range", (int)delay);
    if (budget < 0 || budget > N_s) return report(err, err_len, OED_E_ARG, "budget %d out of range", (int)budget);
    if (!status_dev || (budget > 0 && (!idx_dev || !gain_dev)))
        return report(err, err_len, OED_E_ARG, "NULL output array");
    const int N_tp = precision == OED_PREC_MIXED_BF16X3 ? (N_t + 31) / 32 * 32 : (N_t + 15) / 16 * 16;
    const Layout L = layout(N_s, N_tp, precision, delay);
    if (L.total > (int64_t)OED_NOALLOC_MAX_BYTES)
        return report(err, err_len, OED_E_UNSUPPORTED,
                      "N_s = %d, N_t = %d at this precision and delay %d needs %lld bytes of scratch; the "
                      "no-allocation selection has %lld",
                      (int)N_s, (int)N_t, (int)delay, (long long)L.total, (long long)OED_NOALLOC_MAX_BYTES);

    // the device address of `scratch` on the current device, taken once per device
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return report(err, err_len, OED_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return report(err, err_len, OED_E_UNSUPPORTED, "device %d", dev);
    char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch[dev]) {
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return report(err, err_len, OED_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            g_scratch[dev] = p;
        }
        base = (char *)g_scratch[dev];
    }

    const hipStream_t s = (hipStream_t)stream;
    const int rtype = precision == OED_PREC_FP64 ? R_F64 : R_F32;
    const int wtype = precision == OED_PREC_FP64 ? W_F64 : precision == OED_PREC_MIXED_F32 ? W_F32 : W_BF16X3;
    int *act[2] = {(int *)(base + L.act0), (int *)(base + L.act1)};
    int *state = (int *)(base + L.state);
    int *cmap = (int *)(base + L.cmap);

#define NA_CHK(call)                                                                                       \
    do {                                                                                                   \
        hipError_t e_ = (call);                                                                            \
        if (e_ != hipSuccess) return report(err, err_len, OED_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

    // every buffer that is read before it is written starts here: the identity candidate map, the
    // active list, the state words (all by kernels) and R (packed in full, padding included)
    NA_CHK(launch_init_state(cmap, N_s, state, s));
    NA_CHK(launch_init_state(act[0], N_s, state, s));
    NA_CHK(launch_pack(K_dev, dtype, ld, N_t, N_tp, cmap, N_s, base + L.R, rtype, s));

    StepDesc d{};
    d.R = base + L.R;
    d.W = base + L.W;
    d.W2 = L.W2 >= 0 ? base + L.W2 : nullptr;
    d.wslot = (int64_t)N_s * N_tp * N_tp;
    d.V = L.V >= 0 ? (double *)(base + L.V) : nullptr;
    d.gains = (double *)(base + L.gains);
    d.Linv = (double *)(base + L.Linv);
    d.fcache = (double *)(base + L.fcache);
    d.state = state;
    d.picks = idx_dev;       // all sensors are candidates: local index = sensor index
    d.pick_gain = gain_dev;
    d.half_noise = 0.5 * N_t * std::log(sigma2);
    d.N_t = N_t;
    d.N_tp = N_tp;
    d.forced = -1;
    d.stl = STL_COL4;  // the handle's default tile order

    // the greedy loop of oed_greedy: the block column of pick k and, every `delay` picks, the
    // downdate of the held columns are enqueued at the start of step k + 1
    int cur = 0, n_act = N_s, nheld = 0;
    bool pending = false;
    for (int k = 0; k < budget; ++k) {
        d.act_in = act[cur];
        d.act_out = act[cur ^ 1];
        d.n_act = n_act;
        d.nitems = n_act;
        d.nw = 1;
        d.nheld = nheld;
        d.step = k;
        if (pending) {
            if (nheld > 0) NA_CHK(launch_vcorr(d, wtype, s));
            // as the handle: the block column kernel also applies the new column to the diagonal
            // blocks, so the gain launch factors them as they are
            StepDesc t = d;
            t.diag = 1;
            NA_CHK(launch_trsm(t, rtype, wtype, s));
            if (nheld + 1 < delay) {
                ++nheld;
            } else {
                StepDesc u = d;
                u.nw = nheld + 1;
                u.nitems = syrk_tiles(n_act, N_tp, u.stl);
                u.skipdiag = 1;
                NA_CHK(launch_syrk(u, rtype, wtype, SYRK_LDS, s));
                nheld = 0;
            }
            d.nheld = nheld;
        }
        // the pick finds the winner's diagonal block current too
        StepDesc g = d;
        g.nitems = n_act;
        g.nheld = 0;
        NA_CHK(launch_gain(g, rtype, wtype, s));
        StepDesc pk = d;
        pk.nitems = 1;
        pk.nheld = 0;
        NA_CHK(launch_pick(pk, rtype, wtype, s));
        cur ^= 1;
        --n_act;
        pending = true;
    }
    // status word and pick count (ST_STATUS, ST_NPICKS are the first two state words)
    NA_CHK(hipMemcpyAsync(status_dev, state, 2 * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
#undef NA_CHK
    return OED_OK;
}

}  // extern "C"
