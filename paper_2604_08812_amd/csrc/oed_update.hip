// The Schur-complement downdate of one greedy step, R -= W W^T on the lower triangle of the
// remaining rows (Sec. III-D), on MFMA.  (The block column W is formed in oed_blockcol.hip, the
// left-looking method's column products in oed_column.hip.)
#include "oed_device.h"

namespace oed {

// ---------------------------------------------------------------------------------------------
// Downdate R_IJ -= W_I W_J^T over 128 x 128 tiles of the remaining rows, lower triangle only.
// Four waves per tile, each a 64 x 64 quarter = 4 x 4 MFMA 16x16 blocks.  Tiles are handed
// out XCD by XCD (work-group id mod 8 is the XCD) in contiguous chunks, so the row panel of
// W that neighbouring tiles share stays in that XCD's L2.
template <typename T>
__device__ void syrk_direct_body(const StepDesc &d, int64_t tile)
{
    typedef typename V4<T>::type vec;
    if (d.state[ST_STATUS] != 0) return;
    T *__restrict__ R = (T *)d.R;
    const T *__restrict__ W = (const T *)d.W;
    const int *__restrict__ act = d.act_in;
    const int n_act = d.n_act, N_tp = d.N_tp;
    int64_t P, Q;
    if (!super_tile(tile, syrk_tile_rows(d.n_act, d.N_tp), d.stl, P, Q)) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wr = wave >> 1, wc = wave & 1;
    const int alane = a_lane<T>(lane);
    const int nb = N_tp >> 4;
    const int rows = n_act * N_tp;
    const int64_t bs = (int64_t)N_tp * N_tp;

    int ia[4], ta[4], ja[4], tc[4];
    bool vr[4], vc[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int r = (int)P * 128 + wr * 64 + 16 * b;
        vr[b] = r < rows;
        ia[b] = vr[b] ? act[r / N_tp] : 0;
        ta[b] = (r % N_tp) >> 4;
        const int c = (int)Q * 128 + wc * 64 + 16 * b;
        vc[b] = c < rows;
        ja[b] = vc[b] ? act[c / N_tp] : 0;
        tc[b] = (c % N_tp) >> 4;
    }
    bool any = false;
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c) any |= vr[b] && vc[c] && ia[b] >= ja[c] && !(d.skipdiag && ia[b] == ja[c]);
    if (!any) return;

    vec acc[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (vr[b] && vc[c] && ia[b] >= ja[c] && !(d.skipdiag && ia[b] == ja[c]))
                acc[b][c] = ld4(R + blk_index(ia[b], ja[c]) * bs + ((ta[b] * nb + tc[c]) << 8) + lane * 4);
            else
                acc[b][c] = vec{0, 0, 0, 0};
        }
    for (int q = 0; q < nb; ++q) {
        vec a[4], w[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            a[b] = vr[b] ? ld4(W + (int64_t)ia[b] * bs + ((ta[b] * nb + q) << 8) + alane * 4) : vec{0, 0, 0, 0};
            w[b] = vc[b] ? ld4(W + (int64_t)ja[b] * bs + ((tc[b] * nb + q) << 8) + lane * 4) : vec{0, 0, 0, 0};
        }
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[b][c] = mfma16(-a[b][s4], w[c][s4], acc[b][c]);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (vr[b] && vc[c] && ia[b] >= ja[c] && !(d.skipdiag && ia[b] == ja[c]))
                st4(R + blk_index(ia[b], ja[c]) * bs + ((ta[b] * nb + tc[c]) << 8) + lane * 4, acc[b][c]);
}

// ---------------------------------------------------------------------------------------------
// Addresses shared by the LDS-staged downdates.  The work-group's tile (P, Q) covers rows
// 128P.. and columns 128Q..; wave w stages sub-block rows w and w + 4 of both W panels and
// owns output quarter (w / 2, w % 2) = 4 x 4 blocks of 16 x 16.  Every global load is
// unconditional: rows past the last active block read a valid (clamped) address and the
// blocks that would use them are never stored, so a wait for one batch of loads never has
// to wait for another issued later.  The active-list lookups are wave-uniform (scalar).
// All fields are wave-uniform (scalar registers); lane offsets are added at each access.
struct TileMap {
    int64_t wA[2], wB[2];  // element offsets of the wave's staged W sub-blocks (slice 0)
    int64_t rblk[16];      // element offsets of the wave's output blocks in R
    bool ok[16];           // output block is in the lower triangle of active rows
    bool any;
};

__device__ __forceinline__ void tile_map_n(const StepDesc &d, const int N_tp, int64_t P, int64_t Q, int wave,
                                           TileMap &m)
{
    const int NB = N_tp / 16;
    const int *__restrict__ act = d.act_in;
    const int rows = d.n_act * N_tp, last = d.n_act - 1;
    const int64_t bs = (int64_t)N_tp * N_tp;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int sb = wave + 4 * h;
        const int r = (int)P * 128 + 16 * sb, c = (int)Q * 128 + 16 * sb;
        const int ia = uniform_at(act, min(r / N_tp, last)), ja = uniform_at(act, min(c / N_tp, last));
        m.wA[h] = (int64_t)ia * bs + (int64_t)((r % N_tp) >> 4) * (NB * 256);
        m.wB[h] = (int64_t)ja * bs + (int64_t)((c % N_tp) >> 4) * (NB * 256);
    }
    m.any = false;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int r = (int)P * 128 + (wave >> 1) * 64 + 16 * b;
        const int ia = uniform_at(act, min(r / N_tp, last)), ta = (r % N_tp) >> 4;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int cc = (int)Q * 128 + (wave & 1) * 64 + 16 * c;
            const int ja = uniform_at(act, min(cc / N_tp, last)), tc = (cc % N_tp) >> 4;
            const bool o = r < rows && cc < rows && ia >= ja && !(d.skipdiag && ia == ja);
            m.ok[4 * b + c] = o;
            m.any |= o;
            m.rblk[4 * b + c] = o ? blk_index(ia, ja) * bs + ((ta * NB + tc) << 8) : 0;
        }
    }
}

template <int N_tp>
__device__ __forceinline__ void tile_map(const StepDesc &d, int64_t P, int64_t Q, int wave, TileMap &m)
{
    tile_map_n(d, N_tp, P, Q, wave, m);
}

// ---------------------------------------------------------------------------------------------
// Downdate, LDS-staged and software-pipelined variant for N_tp = 16*NB <= 128.
// Per 16-wide slice q of the inner index, the work-group stages the 128 x 16 A panel (tile
// rows) and B panel (tile columns) of W into LDS once (double-buffered, one barrier per
// slice) and every wave reads its operands from there; the next slice's global loads are in
// flight while the current slice's MFMAs run.  The product W_I W_J^T accumulates from zero
// and is subtracted from R at the end, which reads the R tile in the epilogue: with p W slots
// per launch the tile's MFMA work is p times longer than its R traffic, and without a register
// copy of the tile the FP32 kernel fits three work-groups per CU, whose MFMAs cover each
// other's epilogues (streaming R into registers during the last slot measured slower there).
template <typename T, int NB, int KS>
__device__ void syrk_lds_body(const StepDesc &d, int64_t tile)
{
    // KS consecutive 16-wide inner slices are staged per barrier (NB % KS == 0)
    typedef typename V4<T>::type vec;
    constexpr int N_tp = 16 * NB;
    constexpr int NST = NB / KS;              // stages per W block
    constexpr bool FLAT = sizeof(T) == 4;     // FP32: the slice's MFMAs without a branch
    __shared__ vec lds[2][2][KS][8 * 64];      // [buffer][A/B][slice][sub-block * 64 + lane]
    if (d.state[ST_STATUS] != 0) return;
    int64_t P, Q;
    if (!super_tile(tile, syrk_tile_rows(d.n_act, d.N_tp), d.stl, P, Q)) return;
    T *__restrict__ R = (T *)d.R;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), wr = wave >> 1, wc = wave & 1;
    const int alane = a_lane<T>(lane);
    TileMap m;
    tile_map<N_tp>(d, P, Q, wave, m);
    T *Rl = R + lane * 4;  // this lane's element of an output block
    // W slot `slot`, at this lane's element of a staged sub-block
    const T *W0 = (const T *)d.W + lane * 4;
    const int64_t wslot = d.wslot;
    auto wblk = [&](int slot) -> const T * { return W0 + slot * wslot; };

    vec acc[16];
#pragma unroll
    for (int f = 0; f < 16; ++f) acc[f] = vec{0, 0, 0, 0};
    vec sa[KS][2], sbv[KS][2];
    auto stage = [&](const T *src) {
#pragma unroll
        for (int k = 0; k < KS; ++k)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                sa[k][h] = ld4(src + (k << 8) + m.wA[h]);
                sbv[k][h] = ld4(src + (k << 8) + m.wB[h]);
            }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int k = 0; k < KS; ++k)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                lds[buf][0][k][(wave + 4 * h) * 64 + lane] = sa[k][h];
                lds[buf][1][k][(wave + 4 * h) * 64 + lane] = sbv[k][h];
            }
    };
    stage(wblk(0));
    put(0);
    __syncthreads();

    // The NST stages of one W block (cur); the stage after its last one is the first of nxt
    // (null: none).  par: LDS buffer of its first stage.
    auto pass = [&](const T *cur, const T *nxt, int par) {
#pragma unroll
        for (int q = 0; q < NST; ++q) {
            const int buf = par ^ (q & 1);
            const bool more = q + 1 < NST || nxt;
            if (more) stage(q + 1 < NST ? cur + (((q + 1) * KS) << 8) : nxt);
            // FP32: the MFMAs run unconditionally (a wave with no output block in the triangle
            // computes products it never stores), so that each slice is one basic block and the
            // scheduling barrier keeps the next slice's loads ahead of them instead of sunk below
            // (2.4% faster at 600 x 128).  FP64 keeps the branch: there the same form spills.
            if constexpr (FLAT) __builtin_amdgcn_sched_barrier(0);
            if (FLAT || m.any) {
                // row block by row block: the first sixteen MFMAs need only w and a[0], and the
                // compiler runs the last row blocks of a slice after the barrier, under the next
                // slice's LDS reads (3% faster in FP32 than taking each k-step over all sixteen blocks
                // in turn; per output block the MFMAs keep their order, so the bits are the same)
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    vec a[4], w[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) w[c] = lds[buf][1][k][(wc * 4 + c) * 64 + lane];
#pragma unroll
                    for (int b = 0; b < 4; ++b) a[b] = lds[buf][0][k][(wr * 4 + b) * 64 + alane];
#pragma unroll
                    for (int b = 0; b < 4; ++b)
#pragma unroll
                        for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                            for (int c = 0; c < 4; ++c) acc[4 * b + c] = mfma16(a[b][s4], w[c][s4], acc[4 * b + c]);
                }
            }
            if (more) put(buf ^ 1);
            __syncthreads();
        }
    };
    const int nw = d.nw;
    for (int slot = 0; slot + 1 < nw; ++slot) pass(wblk(slot), wblk(slot + 1), (slot * NST) & 1);
    pass(wblk(nw - 1), nullptr, ((nw - 1) * NST) & 1);

    if (!m.any) return;
    // the tile's loads in flight together, all 16 in FP32, four at a time in FP64 (registers);
    // blocks outside the triangle read a valid address and are not stored
    constexpr int GR = sizeof(T) == 4 ? 16 : 4;
#pragma unroll
    for (int f0 = 0; f0 < 16; f0 += GR) {
        vec rt[GR];
#pragma unroll
        for (int f = 0; f < GR; ++f) rt[f] = ld4_stream(Rl + m.rblk[f0 + f]);
#pragma unroll
        for (int f = 0; f < GR; ++f)
            if (m.ok[f0 + f]) st4_stream(Rl + m.rblk[f0 + f], rt[f] - acc[f0 + f]);
    }
}

// ---------------------------------------------------------------------------------------------
// Downdate for N_tp = 16 nb > 128 (runtime block size): the LDS-staged, double-buffered tile of
// syrk_lds_body with a run-time slice loop; R is read in the epilogue, as there (the K extent of
// N_tp > 128 is long against the tile's R traffic, and the kernel then fits four work-groups
// per CU, which cover each other's epilogues).
constexpr int RT_MIN_NB = 9;

template <typename T>
__device__ void syrk_lds_rt_body(const StepDesc &d, int64_t tile)
{
    typedef typename V4<T>::type vec;
    __shared__ vec lds[2][2][8 * 64];  // [buffer][A/B][sub-block * 64 + lane]
    if (d.state[ST_STATUS] != 0) return;
    int64_t P, Q;
    if (!super_tile(tile, syrk_tile_rows(d.n_act, d.N_tp), d.stl, P, Q)) return;
    const int nb = d.N_tp >> 4;
    T *__restrict__ R = (T *)d.R;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), wr = wave >> 1, wc = wave & 1;
    const int alane = a_lane<T>(lane);
    TileMap m;
    tile_map_n(d, d.N_tp, P, Q, wave, m);
    T *Rl = R + lane * 4;
    const T *W0 = (const T *)d.W + lane * 4;
    const int64_t wslot = d.wslot;

    vec acc[16];
#pragma unroll
    for (int f = 0; f < 16; ++f) acc[f] = vec{0, 0, 0, 0};
    vec sa[2], sbv[2];
    auto stage = [&](const T *src) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            sa[h] = ld4(src + m.wA[h]);
            sbv[h] = ld4(src + m.wB[h]);
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            lds[buf][0][(wave + 4 * h) * 64 + lane] = sa[h];
            lds[buf][1][(wave + 4 * h) * 64 + lane] = sbv[h];
        }
    };
    // row block by row block, as in syrk_lds_body
    auto mma = [&](int buf) {
        if (!m.any) return;
        vec a[4], w[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) w[c] = lds[buf][1][(wc * 4 + c) * 64 + lane];
#pragma unroll
        for (int b = 0; b < 4; ++b) a[b] = lds[buf][0][(wr * 4 + b) * 64 + alane];
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[4 * b + c] = mfma16(a[b][s4], w[c][s4], acc[4 * b + c]);
    };
    stage(W0);
    put(0);
    __syncthreads();
    int buf = 0;
    const int nw = d.nw;
    for (int slot = 0; slot < nw; ++slot) {
        const T *cur = W0 + slot * wslot;
        const bool last = slot + 1 == nw;
        // slice q of a staged sub-block row sits 256 q elements after its slice 0
        for (int q = 0; q < nb; ++q) {
            const bool more = q + 1 < nb || !last;
            if (more) stage(q + 1 < nb ? cur + ((q + 1) << 8) : cur + wslot);
            mma(buf);
            if (more) put(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }

    if (!m.any) return;
    // the tile's loads four at a time (more would cost the fourth work-group per CU in FP32)
    constexpr int GR = 4;
#pragma unroll
    for (int f0 = 0; f0 < 16; f0 += GR) {
        vec rt[GR];
#pragma unroll
        for (int f = 0; f < GR; ++f) rt[f] = ld4_stream(Rl + m.rblk[f0 + f]);
#pragma unroll
        for (int f = 0; f < GR; ++f)
            if (m.ok[f0 + f]) st4_stream(Rl + m.rblk[f0 + f], rt[f] - acc[f0 + f]);
    }
}

// ---------------------------------------------------------------------------------------------
// Downdate with W split into BF16 hi + lo parts (N_tp = 32 * NB32): R_IJ -= hi_I hi_J^T +
// hi_I lo_J^T + lo_I hi_J^T on the 16x16x32 BF16 MFMA with FP32 accumulation.  Per 32-wide
// inner slice the work-group stages the hi and lo parts of both W panels in LDS (double
// buffered); otherwise as syrk_lds_body.
template <int NB32>
__device__ void syrk_bf16_body(const StepDesc &d, int64_t tile)
{
    constexpr int N_tp = 32 * NB32;
    constexpr int PER = (16 + NB32 - 1) / NB32;  // R blocks fetched per slice of the last W block
    __shared__ u32x4 lds[2][4][8 * 64];          // [buffer][A hi, A lo, B hi, B lo][sub-block * 64 + lane]
    if (d.state[ST_STATUS] != 0) return;
    int64_t P, Q;
    if (!super_tile(tile, syrk_tile_rows(d.n_act, d.N_tp), d.stl, P, Q)) return;
    float *__restrict__ R = (float *)d.R;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), wr = wave >> 1, wc = wave & 1;
    TileMap m;
    tile_map<N_tp>(d, P, Q, wave, m);  // W offsets in BF16 elements: a 16 x 32 tile is 512
    float *Rl = R + lane * 4;
    typedef const unsigned short *bp;
    const bp Wh0 = (bp)d.W + lane * 8, Wl0 = (bp)d.W2 + lane * 8;
    const int64_t wslot = d.wslot;
    auto whi = [&](int slot) -> bp { return Wh0 + slot * wslot; };
    auto wlo = [&](int slot) -> bp { return Wl0 + slot * wslot; };

    floatx4 rt[16], acc[16];
#pragma unroll
    for (int f = 0; f < 16; ++f) acc[f] = floatx4{0, 0, 0, 0};
    u32x4 st[2][4];  // [h][A hi, A lo, B hi, B lo]
    auto stage = [&](bp hi, bp lo) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            st[h][0] = *reinterpret_cast<const u32x4 *>(hi + m.wA[h]);
            st[h][1] = *reinterpret_cast<const u32x4 *>(lo + m.wA[h]);
            st[h][2] = *reinterpret_cast<const u32x4 *>(hi + m.wB[h]);
            st[h][3] = *reinterpret_cast<const u32x4 *>(lo + m.wB[h]);
        }
    };
    stage(whi(0), wlo(0));
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k = 0; k < 4; ++k) lds[0][k][(wave + 4 * h) * 64 + lane] = st[h][k];
    __syncthreads();

    // as in syrk_lds_body, per 32-wide slice
    auto pass = [&](auto pref, bp chi, bp clo, bp nhi, bp nlo, int par) {
        constexpr bool PREF = decltype(pref)::value;
#pragma unroll
        for (int q = 0; q < NB32; ++q) {
            const int buf = par ^ (q & 1);
            const bool more = q + 1 < NB32 || nhi;
            if (more) {
                if (q + 1 < NB32)
                    stage(chi + ((q + 1) << 9), clo + ((q + 1) << 9));
                else
                    stage(nhi, nlo);
            }
            if (PREF) {
#pragma unroll
                for (int f = q * PER; f < (q + 1) * PER && f < 16; ++f) rt[f] = ld4_stream(Rl + m.rblk[f]);
            }
            // as in the FP32 downdate: the MFMAs without a branch, the loads kept ahead of them
            __builtin_amdgcn_sched_barrier(0);
            {
                u32x4 wh[4], wl[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    wh[c] = lds[buf][2][(wc * 4 + c) * 64 + lane];
                    wl[c] = lds[buf][3][(wc * 4 + c) * 64 + lane];
                }
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const u32x4 ah = lds[buf][0][(wr * 4 + b) * 64 + lane];
                    const u32x4 al = lds[buf][1][(wr * 4 + b) * 64 + lane];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        acc[4 * b + c] = mfma_bf16(ah, wh[c], acc[4 * b + c]);
                        acc[4 * b + c] = mfma_bf16(ah, wl[c], acc[4 * b + c]);
                        acc[4 * b + c] = mfma_bf16(al, wh[c], acc[4 * b + c]);
                    }
                }
            }
            if (more) {
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int k = 0; k < 4; ++k) lds[buf ^ 1][k][(wave + 4 * h) * 64 + lane] = st[h][k];
            }
            __syncthreads();
        }
    };
    const int nw = d.nw;
    for (int slot = 0; slot + 1 < nw; ++slot)
        pass(BoolC<false>(), whi(slot), wlo(slot), whi(slot + 1), wlo(slot + 1), (slot * NB32) & 1);
    pass(BoolC<true>(), whi(nw - 1), wlo(nw - 1), nullptr, nullptr, ((nw - 1) * NB32) & 1);

    if (!m.any) return;
#pragma unroll
    for (int f = 0; f < 16; ++f)
        if (m.ok[f]) st4_stream(Rl + m.rblk[f], rt[f] - acc[f]);
}

// ---------------------------------------------------------------------------------------------
// The BF16 split-product downdate for N_tp = 32 nb32 > 128 (run-time block size): the staging and
// products of syrk_bf16_body with a run-time slice loop.  Half of the tile's sixteen R blocks are
// loaded two slices before the end, so that the last slices' MFMAs cover their latency, the other
// half with the epilogue's stores of the first (all sixteen early spill: the kernel keeps two
// work-groups per CU, which its 64 KB of LDS allow, only within 256 registers).
__device__ void syrk_bf16_rt_body(const StepDesc &d, int64_t tile)
{
    __shared__ u32x4 lds[2][4][8 * 64];  // [buffer][A hi, A lo, B hi, B lo][sub-block * 64 + lane]
    if (d.state[ST_STATUS] != 0) return;
    int64_t P, Q;
    if (!super_tile(tile, syrk_tile_rows(d.n_act, d.N_tp), d.stl, P, Q)) return;
    const int nb32 = d.N_tp >> 5;
    float *__restrict__ R = (float *)d.R;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), wr = wave >> 1, wc = wave & 1;
    TileMap m;
    tile_map_n(d, d.N_tp, P, Q, wave, m);  // W offsets in BF16 elements: a 16 x 32 tile is 512
    float *Rl = R + lane * 4;
    typedef const unsigned short *bp;
    const bp Wh0 = (bp)d.W + lane * 8, Wl0 = (bp)d.W2 + lane * 8;
    const int64_t wslot = d.wslot;

    floatx4 acc[16];
#pragma unroll
    for (int f = 0; f < 16; ++f) acc[f] = floatx4{0, 0, 0, 0};
    u32x4 st[2][4];  // [h][A hi, A lo, B hi, B lo]
    auto stage = [&](bp hi, bp lo) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            st[h][0] = *reinterpret_cast<const u32x4 *>(hi + m.wA[h]);
            st[h][1] = *reinterpret_cast<const u32x4 *>(lo + m.wA[h]);
            st[h][2] = *reinterpret_cast<const u32x4 *>(hi + m.wB[h]);
            st[h][3] = *reinterpret_cast<const u32x4 *>(lo + m.wB[h]);
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int k = 0; k < 4; ++k) lds[buf][k][(wave + 4 * h) * 64 + lane] = st[h][k];
    };
    // the MFMAs run without a branch (a wave with no output block computes products it never
    // stores), so that the scheduling barrier keeps the next slice's loads ahead of them
    auto mma = [&](int buf) {
        u32x4 wh[4], wl[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            wh[c] = lds[buf][2][(wc * 4 + c) * 64 + lane];
            wl[c] = lds[buf][3][(wc * 4 + c) * 64 + lane];
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const u32x4 ah = lds[buf][0][(wr * 4 + b) * 64 + lane];
            const u32x4 al = lds[buf][1][(wr * 4 + b) * 64 + lane];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                acc[4 * b + c] = mfma_bf16(ah, wh[c], acc[4 * b + c]);
                acc[4 * b + c] = mfma_bf16(ah, wl[c], acc[4 * b + c]);
                acc[4 * b + c] = mfma_bf16(al, wh[c], acc[4 * b + c]);
            }
        }
    };
    floatx4 rt[8];
    stage(Wh0, Wl0);
    put(0);
    __syncthreads();
    int buf = 0;
    const int nw = d.nw;
    for (int slot = 0; slot < nw; ++slot) {
        const bp chi = Wh0 + slot * wslot, clo = Wl0 + slot * wslot;
        const bool last = slot + 1 == nw;
        // 32-wide slice q of a staged sub-block row sits 512 q elements after its slice 0
        for (int q = 0; q < nb32; ++q) {
            const bool more = q + 1 < nb32 || !last;
            if (more) {
                if (q + 1 < nb32)
                    stage(chi + ((q + 1) << 9), clo + ((q + 1) << 9));
                else
                    stage(chi + wslot, clo + wslot);
            }
            // blocks outside the triangle read a valid address and are not stored
            if (last && q == nb32 - 2) {
#pragma unroll
                for (int f = 0; f < 8; ++f) rt[f] = ld4_stream(Rl + m.rblk[f]);
            }
            __builtin_amdgcn_sched_barrier(0);
            mma(buf);
            if (more) put(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }

    if (!m.any) return;
    floatx4 r2[8];
#pragma unroll
    for (int f = 0; f < 8; ++f) r2[f] = ld4_stream(Rl + m.rblk[8 + f]);
#pragma unroll
    for (int f = 0; f < 8; ++f)
        if (m.ok[f]) st4_stream(Rl + m.rblk[f], rt[f] - acc[f]);
#pragma unroll
    for (int f = 0; f < 8; ++f)
        if (m.ok[8 + f]) st4_stream(Rl + m.rblk[8 + f], r2[f] - acc[8 + f]);
}

// ---------------------------------------------------------------------------------------------
// The BF16 split-product downdate over 256 x 256 tiles (SYRK_BIG): eight waves, wave w computes
// rows 64 (w / 2) .. + 63 of the tile against columns 128 (w % 2) .. + 127, 4 x 8 blocks of 16 x 16.
// Per 32-wide inner slice the work-group stages the 256-row A and B panels, hi and lo parts, in LDS
// (double buffered, 128 KB of dynamic LDS: one work-group per CU, two waves per SIMD).  Against the
// 128 x 128 tile of syrk_bf16_body every staged operand feeds twice the MFMAs, which halves the W
// traffic from L2 and the LDS reads per flop (that kernel reads about as many LDS bytes as its
// MFMAs can consume).  Tiles run in the super-tile order of d.stl over 256-row tiles.
constexpr int BIG_TILE = 256;
constexpr size_t BIG_LDS_BYTES = 2 * 4 * 16 * 64 * sizeof(u32x4);

template <int NB32>
__device__ void syrk_bf16_big_body(const StepDesc &d, int64_t tile, u32x4 *lds)
{
    constexpr int N_tp = 32 * NB32, NB = N_tp / 16;
    constexpr int64_t bs = (int64_t)N_tp * N_tp;
    if (d.state[ST_STATUS] != 0) return;
    const int rows = d.n_act * N_tp, last = d.n_act - 1;
    int64_t P, Q;
    if (!super_tile(tile, (rows + BIG_TILE - 1) / BIG_TILE, d.stl, P, Q)) return;
    const int *__restrict__ act = d.act_in;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), wr = wave >> 1, wc = wave & 1;
    // the wave stages sub-block rows `wave` and `wave + 8` of both panels (slice 0 offsets)
    int64_t wA[2], wB[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int sb = wave + 8 * h;
        const int r = (int)P * BIG_TILE + 16 * sb, c = (int)Q * BIG_TILE + 16 * sb;
        const int ia = uniform_at(act, min(r / N_tp, last)), ja = uniform_at(act, min(c / N_tp, last));
        wA[h] = ia * bs + (int64_t)((r % N_tp) >> 4) * (NB * 256);
        wB[h] = ja * bs + (int64_t)((c % N_tp) >> 4) * (NB * 256);
    }
    typedef const unsigned short *bp;
    const bp Wh0 = (bp)d.W + lane * 8, Wl0 = (bp)d.W2 + lane * 8;
    const int64_t wslot = d.wslot;
    auto L = [&](int buf, int part, int sb) -> u32x4 * { return lds + ((((buf << 2) + part) << 4) + sb) * 64; };

    floatx4 acc[4][8];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[b][c] = floatx4{0, 0, 0, 0};
    u32x4 st[2][4];  // [h][A hi, A lo, B hi, B lo]
    auto stage = [&](bp hi, bp lo) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            st[h][0] = *reinterpret_cast<const u32x4 *>(hi + wA[h]);
            st[h][1] = *reinterpret_cast<const u32x4 *>(lo + wA[h]);
            st[h][2] = *reinterpret_cast<const u32x4 *>(hi + wB[h]);
            st[h][3] = *reinterpret_cast<const u32x4 *>(lo + wB[h]);
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int k = 0; k < 4; ++k) L(buf, k, wave + 8 * h)[lane] = st[h][k];
    };
    stage(Wh0, Wl0);
    put(0);
    __syncthreads();

    const int nw = d.nw;
    int buf = 0;
    for (int slot = 0; slot < nw; ++slot) {
        const bp chi = Wh0 + slot * wslot, clo = Wl0 + slot * wslot;
#pragma unroll
        for (int q = 0; q < NB32; ++q) {
            const bool more = q + 1 < NB32 || slot + 1 < nw;
            if (more) {
                if (q + 1 < NB32)
                    stage(chi + ((q + 1) << 9), clo + ((q + 1) << 9));
                else
                    stage(chi + wslot, clo + wslot);
            }
            // the slice's MFMAs without a branch, the next slice's loads kept ahead of them
            __builtin_amdgcn_sched_barrier(0);
            {
                u32x4 ah[4], al[4];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    ah[b] = L(buf, 0, wr * 4 + b)[lane];
                    al[b] = L(buf, 1, wr * 4 + b)[lane];
                }
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const u32x4 bh = L(buf, 2, wc * 8 + c)[lane];
                    const u32x4 bl = L(buf, 3, wc * 8 + c)[lane];
                    // the three products of a block pair four MFMAs apart
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[b][c] = mfma_bf16(ah[b], bh, acc[b][c]);
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[b][c] = mfma_bf16(ah[b], bl, acc[b][c]);
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[b][c] = mfma_bf16(al[b], bh, acc[b][c]);
                }
            }
            if (more) put(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }

    // epilogue: R -= acc on the wave's blocks in the lower triangle, eight loads in flight at a time
    float *__restrict__ Rl = (float *)d.R + lane * 4;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int r = (int)P * BIG_TILE + wr * 64 + 16 * b;
        const int ia = uniform_at(act, min(r / N_tp, last)), ta = (r % N_tp) >> 4;
        int64_t off[8];
        bool ok[8];
        bool any = false;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int cc = (int)Q * BIG_TILE + wc * 128 + 16 * c;
            const int ja = uniform_at(act, min(cc / N_tp, last)), tc = (cc % N_tp) >> 4;
            ok[c] = r < rows && cc < rows && ia >= ja && !(d.skipdiag && ia == ja);
            off[c] = ok[c] ? blk_index(ia, ja) * bs + ((ta * NB + tc) << 8) : 0;
            any |= ok[c];
        }
        if (!any) continue;
        floatx4 rt[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) rt[c] = ld4_stream(Rl + off[c]);
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (ok[c]) st4_stream(Rl + off[c], rt[c] - acc[b][c]);
    }
}

// ---------------------------------------------------------------------------------------------
// Kernels: single instance (descriptor by value) and batched (descriptor array).

template <typename T>
__global__ void __launch_bounds__(256) syrk_direct_kernel(StepDesc d, int64_t per_xcd)
{
    const int64_t tile = xcd_item(blockIdx.x, per_xcd);
    if (tile >= d.nitems) return;
    syrk_direct_body<T>(d, tile);
}

template <typename T>
__global__ void __launch_bounds__(256) syrk_direct_batched(const StepDesc *__restrict__ ds, int n, int64_t total,
                                                           int64_t per_xcd)
{
    const int64_t item = xcd_item(blockIdx.x, per_xcd);
    if (item >= total) return;
    const int i = find_instance(ds, n, item);
    if (i < 0) return;
    const StepDesc d = ds[i];
    syrk_direct_body<T>(d, item - d.item0);
}

template <typename T>
__global__ void __launch_bounds__(256, (sizeof(T) == 4 ? 3 : 2)) syrk_lds_rt_kernel(StepDesc d, int64_t per_xcd)
{
    const int64_t tile = xcd_item(blockIdx.x, per_xcd);
    if (tile >= d.nitems) return;
    syrk_lds_rt_body<T>(d, tile);
}

template <typename T, int NB, int KS>
__global__ void __launch_bounds__(256, (sizeof(T) == 4 ? 3 : 2)) syrk_lds_kernel(StepDesc d, int64_t per_xcd)
{
    const int64_t tile = xcd_item(blockIdx.x, per_xcd);
    if (tile >= d.nitems) return;
    syrk_lds_body<T, NB, KS>(d, tile);
}

template <typename T, int NB, int KS>
__global__ void __launch_bounds__(256, 2) syrk_lds_batched(const StepDesc *__restrict__ ds, int n, int64_t total,
                                                           int64_t per_xcd)
{
    const int64_t item = xcd_item(blockIdx.x, per_xcd);
    if (item >= total) return;
    const int i = find_instance(ds, n, item);
    if (i < 0) return;
    const StepDesc d = ds[i];
    syrk_lds_body<T, NB, KS>(d, item - d.item0);
}

template <int NB32>
__global__ void __launch_bounds__(256, 2) syrk_bf16_kernel(StepDesc d, int64_t per_xcd)
{
    const int64_t tile = xcd_item(blockIdx.x, per_xcd);
    if (tile >= d.nitems) return;
    syrk_bf16_body<NB32>(d, tile);
}

template <int NB32>
__global__ void __launch_bounds__(256, 2) syrk_bf16_batched(const StepDesc *__restrict__ ds, int n, int64_t total,
                                                            int64_t per_xcd)
{
    const int64_t item = xcd_item(blockIdx.x, per_xcd);
    if (item >= total) return;
    const int i = find_instance(ds, n, item);
    if (i < 0) return;
    const StepDesc d = ds[i];
    syrk_bf16_body<NB32>(d, item - d.item0);
}

__global__ void __launch_bounds__(256, 2) syrk_bf16_rt_kernel(StepDesc d, int64_t per_xcd)
{
    const int64_t tile = xcd_item(blockIdx.x, per_xcd);
    if (tile >= d.nitems) return;
    syrk_bf16_rt_body(d, tile);
}

template <int NB32>
__global__ void __launch_bounds__(512, 1) syrk_bf16_big_kernel(StepDesc d, int64_t per_xcd)
{
    extern __shared__ u32x4 big_lds[];
    const int64_t tile = xcd_item(blockIdx.x, per_xcd);
    if (tile >= d.nitems) return;
    syrk_bf16_big_body<NB32>(d, tile, big_lds);
}

template <int NB32>
__global__ void __launch_bounds__(512, 1) syrk_bf16_big_batched(const StepDesc *__restrict__ ds, int n, int64_t total,
                                                                int64_t per_xcd)
{
    extern __shared__ u32x4 big_lds[];
    const int64_t item = xcd_item(blockIdx.x, per_xcd);
    if (item >= total) return;
    const int i = find_instance(ds, n, item);
    if (i < 0) return;
    const StepDesc d = ds[i];
    syrk_bf16_big_body<NB32>(d, item - d.item0, big_lds);
}

// ---------------------------------------------------------------------------------------------
// Launchers.

// Single (descs == nullptr: d by value) or batched downdate launch over `total` tiles.
// nw > 1 (held W applied with the new one) needs the LDS variant.
template <typename T>
static hipError_t launch_syrk_t(const StepDesc *descs, const StepDesc &d, int n, int64_t total, int N_tp, int nw,
                                int variant, hipStream_t s)
{
    if (N_tp < 16 || N_tp % 16 != 0 || nw < 1 || nw > MAX_DELAY) return hipErrorInvalidValue;
    const int nb = N_tp / 16;
    const int64_t per_xcd = (total + 7) / 8;
    const dim3 grid((unsigned)(per_xcd * 8)), block(256);
    if (variant == SYRK_LDS && nb <= 8) {
        switch (nb) {
// One 16-wide slice per barrier (two, KS = 2, measured 5% slower for FP32 at 600 x 128)
#define OED_SYRK_CASE(NBV)                                                                                    \
    case NBV: {                                                                                               \
        constexpr int KSV = 1;                                                                                \
        if (descs)                                                                                            \
            hipLaunchKernelGGL((syrk_lds_batched<T, NBV, KSV>), grid, block, 0, s, descs, n, total, per_xcd); \
        else                                                                                                  \
            hipLaunchKernelGGL((syrk_lds_kernel<T, NBV, KSV>), grid, block, 0, s, d, per_xcd);                \
        break;                                                                                                \
    }
            OED_SYRK_CASE(1)
            OED_SYRK_CASE(2)
            OED_SYRK_CASE(3)
            OED_SYRK_CASE(4)
            OED_SYRK_CASE(5)
            OED_SYRK_CASE(6)
            OED_SYRK_CASE(7)
            OED_SYRK_CASE(8)
#undef OED_SYRK_CASE
        }
        return hipGetLastError();
    }
    // single instances only: batches hold N_t <= 128
    if (variant == SYRK_LDS && nb >= RT_MIN_NB && !descs) {
        hipLaunchKernelGGL(syrk_lds_rt_kernel<T>, grid, block, 0, s, d, per_xcd);
        return hipGetLastError();
    }
    if (nw != 1) return hipErrorInvalidValue;
    if (descs)
        hipLaunchKernelGGL(syrk_direct_batched<T>, grid, block, 0, s, descs, n, total, per_xcd);
    else
        hipLaunchKernelGGL(syrk_direct_kernel<T>, grid, block, 0, s, d, per_xcd);
    return hipGetLastError();
}

// BF16 split-product downdate (single or batched).
template <typename K>
static void allow_big_lds(K kernel)
{
    (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)BIG_LDS_BYTES);
}

static hipError_t launch_syrk_bf16(const StepDesc *descs, const StepDesc &d, int n, int64_t total, int N_tp, int nw,
                                   int variant, hipStream_t s)
{
    if (N_tp < 32 || N_tp % 32 != 0 || nw < 1 || nw > MAX_DELAY) return hipErrorInvalidValue;
    const int64_t per_xcd = (total + 7) / 8;
    if (N_tp > 128) {
        // single instances with 128 x 128 tiles only: batches hold N_t <= 128
        if (descs || variant != SYRK_LDS) return hipErrorInvalidValue;
        hipLaunchKernelGGL(syrk_bf16_rt_kernel, dim3((unsigned)(per_xcd * 8)), dim3(256), 0, s, d, per_xcd);
        return hipGetLastError();
    }
    if (variant == SYRK_BIG) {
        const dim3 grid((unsigned)(per_xcd * 8)), block(512);
        switch (N_tp / 32) {
#define OED_BF16_BIG_CASE(V)                                                                                       \
    case V:                                                                                                        \
        if (descs) {                                                                                               \
            allow_big_lds(syrk_bf16_big_batched<V>);                                                               \
            hipLaunchKernelGGL((syrk_bf16_big_batched<V>), grid, block, BIG_LDS_BYTES, s, descs, n, total, per_xcd); \
        } else {                                                                                                   \
            allow_big_lds(syrk_bf16_big_kernel<V>);                                                                \
            hipLaunchKernelGGL((syrk_bf16_big_kernel<V>), grid, block, BIG_LDS_BYTES, s, d, per_xcd);              \
        }                                                                                                          \
        break;
            OED_BF16_BIG_CASE(1)
            OED_BF16_BIG_CASE(2)
            OED_BF16_BIG_CASE(3)
            OED_BF16_BIG_CASE(4)
#undef OED_BF16_BIG_CASE
        }
        return hipGetLastError();
    }
    const dim3 grid((unsigned)(per_xcd * 8)), block(256);
    switch (N_tp / 32) {
#define OED_BF16_CASE(V)                                                                                     \
    case V:                                                                                                  \
        if (descs)                                                                                           \
            hipLaunchKernelGGL((syrk_bf16_batched<V>), grid, block, 0, s, descs, n, total, per_xcd);         \
        else                                                                                                 \
            hipLaunchKernelGGL((syrk_bf16_kernel<V>), grid, block, 0, s, d, per_xcd);                        \
        break;
        OED_BF16_CASE(1)
        OED_BF16_CASE(2)
        OED_BF16_CASE(3)
        OED_BF16_CASE(4)
#undef OED_BF16_CASE
    }
    return hipGetLastError();
}

hipError_t launch_syrk(const StepDesc &d, int rtype, int wtype, int variant, hipStream_t s)
{
    if (d.n_act <= 0 || d.nitems <= 0) return hipSuccess;
    if (d.nw > 1 && d.wslot <= 0) return hipErrorInvalidValue;
    if (rtype == R_F32 && wtype == W_BF16X3) return launch_syrk_bf16(nullptr, d, 1, d.nitems, d.N_tp, d.nw, variant, s);
    if (rtype == R_F64 && wtype == W_F64) return launch_syrk_t<double>(nullptr, d, 1, d.nitems, d.N_tp, d.nw, variant, s);
    if (rtype == R_F32 && wtype == W_F32) return launch_syrk_t<float>(nullptr, d, 1, d.nitems, d.N_tp, d.nw, variant, s);
    return hipErrorInvalidValue;
}

hipError_t launch_syrk_batched(const StepDesc *descs, int n, int64_t total, int N_tp, int nw, int rtype, int wtype,
                               int variant, hipStream_t s)
{
    if (n <= 0 || total <= 0) return hipSuccess;
    StepDesc none{};
    if (rtype == R_F32 && wtype == W_BF16X3) return launch_syrk_bf16(descs, none, n, total, N_tp, nw, variant, s);
    if (rtype == R_F64 && wtype == W_F64) return launch_syrk_t<double>(descs, none, n, total, N_tp, nw, variant, s);
    if (rtype == R_F32 && wtype == W_F32) return launch_syrk_t<float>(descs, none, n, total, N_tp, nw, variant, s);
    return hipErrorInvalidValue;
}

}  // namespace oed
