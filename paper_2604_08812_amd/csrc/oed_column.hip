// The left-looking method's column products (the order of Algorithm 1, Sec. III-D): for the new pick
// s and every remaining candidate i, the split-K partial sums of sum_h W_h,i W_h,s^T over the stored
// block columns, from which the block column kernel forms C_i = K_is - sum_h W_h,i W_h,s^T.
#include "oed_device.h"

namespace oed {

// ---------------------------------------------------------------------------------------------
// Left-looking block column (the order of Algorithm 1): for the new pick s and every remaining
// candidate i, the partial sums sum_{h in split} W_h,i W_h,s^T over the stored W slots, on MFMA
// with the operands staged in LDS as in the downdate; one work-group per (split, 128-row tile).
// The 128 x N_tp output tile is the rows of the remaining candidates against the N_tp rows of
// s; wave w computes rows 32w .. 32w + 31 against all N_tp columns (no idle MFMAs for N_tp < 128).
// Partial q goes to d.C + q cstride in candidate i's block, transposed: sub-block (c, tb) holds pick
// rows 16c .. 16c + 15 against candidate rows 16tb .. 16tb + 15 in the accumulator order, so the
// block column kernel reads the four pick rows of its lanes with one vector load.  (The pick's rows
// are the MFMA's A operand: the same products in the same order as the untransposed product.)
template <typename T, int NB>
__device__ void column_body(const StepDesc &d, int64_t item)
{
    typedef typename V4<T>::type vec;
    constexpr int N_tp = 16 * NB;
    __shared__ vec lds[2][2][8 * 64];
    if (d.state[ST_STATUS] != 0 || d.nsplit <= 0) return;
    const int64_t rows_t = syrk_tile_rows(d.n_act, N_tp);
    const int split = (int)(item / rows_t);
    const int64_t P = item % rows_t;
    if (split >= d.nsplit) return;
    const int h0 = (int)((int64_t)split * d.nw / d.nsplit), h1 = (int)((int64_t)(split + 1) * d.nw / d.nsplit);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int alane = a_lane<T>(lane);
    const int *__restrict__ act = d.act_in;
    const int rows = d.n_act * N_tp, last = d.n_act - 1;
    const int s = uniform_at(d.state, ST_LAST);
    const int64_t bs = (int64_t)N_tp * N_tp;
    // staged operands: rows of the tile (A) and the rows of s (B; sub-blocks past N_tp clamped)
    int64_t wA[2], wB[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int sb = wave + 4 * h;
        const int r = (int)P * 128 + 16 * sb;
        wA[h] = (int64_t)uniform_at(act, min(r / N_tp, last)) * bs + (int64_t)((r % N_tp) >> 4) * (NB * 256);
        wB[h] = (int64_t)s * bs + (int64_t)(sb < NB ? sb : 0) * (NB * 256);
    }
    int64_t off[2];
    bool ok[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int r = (int)P * 128 + wave * 32 + 16 * b;
        ok[b] = r < rows;
        off[b] = (int64_t)uniform_at(act, min(r / N_tp, last)) * bs + (((r % N_tp) >> 4) << 8);
    }
    const bool any = ok[0];
    const T *W0 = (const T *)d.W + lane * 4;
    const int64_t wslot = d.wslot;
    vec acc[2][NB];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[b][c] = vec{0, 0, 0, 0};
    vec sa[2], sbv[2];
    {
        const T *w0 = W0 + h0 * wslot;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            sa[h] = ld4(w0 + wA[h]);
            sbv[h] = ld4(w0 + wB[h]);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            lds[0][0][(wave + 4 * h) * 64 + lane] = sa[h];
            lds[0][1][(wave + 4 * h) * 64 + lane] = sbv[h];
        }
    }
    __syncthreads();
    int par = 0;
    for (int slot = h0; slot < h1; ++slot) {
        const T *cur = W0 + slot * wslot;
        const T *nxt = slot + 1 < h1 ? cur + wslot : nullptr;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int buf = par ^ (q & 1);
            const bool more = q + 1 < NB || nxt;
            if (more) {
                const T *src = q + 1 < NB ? cur + ((q + 1) << 8) : nxt;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    sa[h] = ld4(src + wA[h]);
                    sbv[h] = ld4(src + wB[h]);
                }
            }
            // FP32: the MFMAs without a branch, the loads kept ahead of them (as in the downdate)
            if constexpr (sizeof(T) == 4) __builtin_amdgcn_sched_barrier(0);
            if (sizeof(T) == 4 || any) {
                // the pick's rows are the A operand (the FP64 MFMA reads its rows at the permuted
                // lane): the output lands transposed, pick row u, candidate row t (see above)
                vec a[2], w[NB];
#pragma unroll
                for (int b = 0; b < 2; ++b) a[b] = lds[buf][0][(2 * wave + b) * 64 + lane];
#pragma unroll
                for (int c = 0; c < NB; ++c) w[c] = lds[buf][1][c * 64 + alane];
                if constexpr (sizeof(T) == 4) {
                    // FP32: pick row block by pick row block (the first MFMAs need a and w[0] only;
                    // per output block the MFMAs keep their order, as in the downdate): 5.8% faster
                    // at 600 x 128 than each k-step over all blocks in turn, which FP64 keeps (1.3%
                    // slower there this way)
#pragma unroll
                    for (int c = 0; c < NB; ++c)
#pragma unroll
                        for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                            for (int b = 0; b < 2; ++b) acc[b][c] = mfma16(w[c][s4], a[b][s4], acc[b][c]);
                } else {
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                        for (int b = 0; b < 2; ++b)
#pragma unroll
                            for (int c = 0; c < NB; ++c) acc[b][c] = mfma16(w[c][s4], a[b][s4], acc[b][c]);
                }
            }
            if (more) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    lds[buf ^ 1][0][(wave + 4 * h) * 64 + lane] = sa[h];
                    lds[buf ^ 1][1][(wave + 4 * h) * 64 + lane] = sbv[h];
                }
            }
            __syncthreads();
        }
        par ^= NB & 1;
    }
    T *Cq = (T *)d.C + split * d.cstride + lane * 4;
#pragma unroll
    for (int b = 0; b < 2; ++b)
        if (ok[b]) {
#pragma unroll
            for (int c = 0; c < NB; ++c) st4(Cq + off[b] + ((c * NB) << 8), acc[b][c]);
        }
}

// Left-looking block column for N_tp = 16 nb > 128: as column_body, with a run-time slice
// loop and the N_tp columns of the pick taken in chunks of 128 (eight sub-blocks), the chunk
// being the fastest index of the work item (split, row tile, chunk), so that the work-groups of
// one row tile run together and share its rows of W in L2.
template <typename T>
__device__ void column_rt_body(const StepDesc &d, int64_t item)
{
    typedef typename V4<T>::type vec;
    __shared__ vec lds[2][2][8 * 64];
    if (d.state[ST_STATUS] != 0 || d.nsplit <= 0) return;
    const int N_tp = d.N_tp, nb = N_tp >> 4, nchunk = (nb + 7) >> 3;
    const int64_t rows_t = syrk_tile_rows(d.n_act, N_tp);
    const int64_t per_split = rows_t * nchunk;
    const int split = (int)(item / per_split);
    const int64_t rem = item - split * per_split;
    const int64_t P = rem / nchunk;
    const int cc = (int)(rem - P * nchunk);
    if (split >= d.nsplit) return;
    const int h0 = (int)((int64_t)split * d.nw / d.nsplit), h1 = (int)((int64_t)(split + 1) * d.nw / d.nsplit);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int alane = a_lane<T>(lane);
    const int *__restrict__ act = d.act_in;
    const int rows = d.n_act * N_tp, last = d.n_act - 1;
    const int s = uniform_at(d.state, ST_LAST);
    const int64_t bs = (int64_t)N_tp * N_tp;
    const int ncol = min(8, nb - 8 * cc);
    // staged operands: rows of the tile (A) and the chunk's rows of s (B; past nb clamped)
    int64_t wA[2], wB[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int sb = wave + 4 * h;
        const int r = (int)P * 128 + 16 * sb;
        wA[h] = (int64_t)uniform_at(act, min(r / N_tp, last)) * bs + (int64_t)((r % N_tp) >> 4) * (nb * 256);
        const int sbB = 8 * cc + sb;
        wB[h] = (int64_t)s * bs + (int64_t)(sbB < nb ? sbB : 0) * (nb * 256);
    }
    int64_t off[2];
    bool ok[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int r = (int)P * 128 + wave * 32 + 16 * b;
        ok[b] = r < rows;
        off[b] = (int64_t)uniform_at(act, min(r / N_tp, last)) * bs + ((8 * cc * nb + ((r % N_tp) >> 4)) << 8);
    }
    const bool any = ok[0];
    const T *W0 = (const T *)d.W + lane * 4;
    const int64_t wslot = d.wslot;
    vec acc[2][8];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[b][c] = vec{0, 0, 0, 0};
    vec sa[2], sbv[2];
    auto stage = [&](const T *src) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            sa[h] = ld4(src + wA[h]);
            sbv[h] = ld4(src + wB[h]);
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            lds[buf][0][(wave + 4 * h) * 64 + lane] = sa[h];
            lds[buf][1][(wave + 4 * h) * 64 + lane] = sbv[h];
        }
    };
    stage(W0 + h0 * wslot);
    put(0);
    __syncthreads();
    int buf = 0;
    for (int slot = h0; slot < h1; ++slot) {
        const T *cur = W0 + slot * wslot;
        for (int q = 0; q < nb; ++q) {
            const bool more = q + 1 < nb || slot + 1 < h1;
            if (more) stage(q + 1 < nb ? cur + ((q + 1) << 8) : cur + wslot);
            if (any) {
                vec a[2], w[8];
#pragma unroll
                for (int b = 0; b < 2; ++b) a[b] = lds[buf][0][(2 * wave + b) * 64 + lane];
#pragma unroll
                for (int c = 0; c < 8; ++c) w[c] = lds[buf][1][c * 64 + alane];
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int c = 0; c < 8; ++c) acc[b][c] = mfma16(w[c][s4], a[b][s4], acc[b][c]);
            }
            if (more) put(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }
    T *Cq = (T *)d.C + split * d.cstride + lane * 4;
#pragma unroll
    for (int b = 0; b < 2; ++b)
        if (ok[b]) {
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (c < ncol) st4(Cq + off[b] + ((c * nb) << 8), acc[b][c]);
        }
}

// The same with W in BF16 hi + lo parts (32-wide slices; hi hi^T + hi lo^T + lo hi^T on the
// 16x16x32 BF16 MFMA, FP32 accumulation).
template <int NB32>
__device__ void column_bf16_body(const StepDesc &d, int64_t item)
{
    constexpr int N_tp = 32 * NB32, NB = 2 * NB32;
    __shared__ u32x4 lds[2][4][8 * 64];  // [buffer][A hi, A lo, B hi, B lo][sub-block * 64 + lane]
    if (d.state[ST_STATUS] != 0 || d.nsplit <= 0) return;
    const int64_t rows_t = syrk_tile_rows(d.n_act, N_tp);
    const int split = (int)(item / rows_t);
    const int64_t P = item % rows_t;
    if (split >= d.nsplit) return;
    const int h0 = (int)((int64_t)split * d.nw / d.nsplit), h1 = (int)((int64_t)(split + 1) * d.nw / d.nsplit);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int *__restrict__ act = d.act_in;
    const int rows = d.n_act * N_tp, last = d.n_act - 1;
    const int s = uniform_at(d.state, ST_LAST);
    const int64_t bs = (int64_t)N_tp * N_tp;
    int64_t wA[2], wB[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int sb = wave + 4 * h;
        const int r = (int)P * 128 + 16 * sb;
        wA[h] = (int64_t)uniform_at(act, min(r / N_tp, last)) * bs + (int64_t)((r % N_tp) >> 4) * (NB * 256);
        wB[h] = (int64_t)s * bs + (int64_t)(sb < NB ? sb : 0) * (NB * 256);
    }
    int64_t off[2];
    bool ok[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int r = (int)P * 128 + wave * 32 + 16 * b;
        ok[b] = r < rows;
        off[b] = (int64_t)uniform_at(act, min(r / N_tp, last)) * bs + (((r % N_tp) >> 4) << 8);
    }
    const bool any = ok[0];
    typedef const unsigned short *bp;
    const bp Wh0 = (bp)d.W + lane * 8, Wl0 = (bp)d.W2 + lane * 8;
    const int64_t wslot = d.wslot;
    floatx4 acc[2][NB];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[b][c] = floatx4{0, 0, 0, 0};
    u32x4 st[2][4];
    auto stage = [&](bp hi, bp lo) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            st[h][0] = *reinterpret_cast<const u32x4 *>(hi + wA[h]);
            st[h][1] = *reinterpret_cast<const u32x4 *>(lo + wA[h]);
            st[h][2] = *reinterpret_cast<const u32x4 *>(hi + wB[h]);
            st[h][3] = *reinterpret_cast<const u32x4 *>(lo + wB[h]);
        }
    };
    stage(Wh0 + h0 * wslot, Wl0 + h0 * wslot);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k = 0; k < 4; ++k) lds[0][k][(wave + 4 * h) * 64 + lane] = st[h][k];
    __syncthreads();
    int par = 0;
    for (int slot = h0; slot < h1; ++slot) {
        const bp chi = Wh0 + slot * wslot, clo = Wl0 + slot * wslot;
        const bool nxt = slot + 1 < h1;
#pragma unroll
        for (int q = 0; q < NB32; ++q) {
            const int buf = par ^ (q & 1);
            const bool more = q + 1 < NB32 || nxt;
            if (more) {
                if (q + 1 < NB32)
                    stage(chi + ((q + 1) << 9), clo + ((q + 1) << 9));
                else
                    stage(chi + wslot, clo + wslot);
            }
            if (any) {
                u32x4 ah[2], al[2];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    ah[b] = lds[buf][0][(2 * wave + b) * 64 + lane];
                    al[b] = lds[buf][1][(2 * wave + b) * 64 + lane];
                }
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    const u32x4 wh = lds[buf][2][c * 64 + lane], wl = lds[buf][3][c * 64 + lane];
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        // transposed output (pick rows first): hi hi^T, hi lo^T, lo hi^T of the
                        // candidate's rows against the pick's, in that order
                        acc[b][c] = mfma_bf16(wh, ah[b], acc[b][c]);
                        acc[b][c] = mfma_bf16(wl, ah[b], acc[b][c]);
                        acc[b][c] = mfma_bf16(wh, al[b], acc[b][c]);
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
        par ^= NB32 & 1;
    }
    float *Cq = (float *)d.C + split * d.cstride + lane * 4;
#pragma unroll
    for (int b = 0; b < 2; ++b)
        if (ok[b]) {
#pragma unroll
            for (int c = 0; c < NB; ++c) st4(Cq + off[b] + ((c * NB) << 8), acc[b][c]);
        }
}

// The BF16 hi + lo form for N_tp = 32 nb32 > 128: the work items and output chunks of
// column_rt_body, the staging and products of column_bf16_body, with a run-time slice loop.
__device__ void column_bf16_rt_body(const StepDesc &d, int64_t item)
{
    __shared__ u32x4 lds[2][4][8 * 64];  // [buffer][A hi, A lo, B hi, B lo][sub-block * 64 + lane]
    if (d.state[ST_STATUS] != 0 || d.nsplit <= 0) return;
    const int N_tp = d.N_tp, nb = N_tp >> 4, nb32 = N_tp >> 5, nchunk = (nb + 7) >> 3;
    const int64_t rows_t = syrk_tile_rows(d.n_act, N_tp);
    const int64_t per_split = rows_t * nchunk;
    const int split = (int)(item / per_split);
    const int64_t rem = item - split * per_split;
    const int64_t P = rem / nchunk;
    const int cc = (int)(rem - P * nchunk);
    if (split >= d.nsplit) return;
    const int h0 = (int)((int64_t)split * d.nw / d.nsplit), h1 = (int)((int64_t)(split + 1) * d.nw / d.nsplit);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int *__restrict__ act = d.act_in;
    const int rows = d.n_act * N_tp, last = d.n_act - 1;
    const int s = uniform_at(d.state, ST_LAST);
    const int64_t bs = (int64_t)N_tp * N_tp;
    const int ncol = min(8, nb - 8 * cc);
    // staged operands (BF16 elements; a 16-row sub-block row spans nb * 256 of them): rows of the
    // tile (A) and the chunk's rows of s (B; past nb clamped)
    int64_t wA[2], wB[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int sb = wave + 4 * h;
        const int r = (int)P * 128 + 16 * sb;
        wA[h] = (int64_t)uniform_at(act, min(r / N_tp, last)) * bs + (int64_t)((r % N_tp) >> 4) * (nb * 256);
        const int sbB = 8 * cc + sb;
        wB[h] = (int64_t)s * bs + (int64_t)(sbB < nb ? sbB : 0) * (nb * 256);
    }
    int64_t off[2];
    bool ok[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int r = (int)P * 128 + wave * 32 + 16 * b;
        ok[b] = r < rows;
        off[b] = (int64_t)uniform_at(act, min(r / N_tp, last)) * bs + ((8 * cc * nb + ((r % N_tp) >> 4)) << 8);
    }
    const bool any = ok[0];
    typedef const unsigned short *bp;
    const bp Wh0 = (bp)d.W + lane * 8, Wl0 = (bp)d.W2 + lane * 8;
    const int64_t wslot = d.wslot;
    floatx4 acc[2][8];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[b][c] = floatx4{0, 0, 0, 0};
    u32x4 st[2][4];
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
            for (int k = 0; k < 4; ++k) lds[buf][k][(wave + 4 * h) * 64 + lane] = st[h][k];
    };
    stage(Wh0 + h0 * wslot, Wl0 + h0 * wslot);
    put(0);
    __syncthreads();
    int buf = 0;
    for (int slot = h0; slot < h1; ++slot) {
        const bp chi = Wh0 + slot * wslot, clo = Wl0 + slot * wslot;
        for (int q = 0; q < nb32; ++q) {
            const bool more = q + 1 < nb32 || slot + 1 < h1;
            if (more) {
                if (q + 1 < nb32)
                    stage(chi + ((q + 1) << 9), clo + ((q + 1) << 9));
                else
                    stage(chi + wslot, clo + wslot);
            }
            if (any) {
                u32x4 ah[2], al[2];
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    ah[b] = lds[buf][0][(2 * wave + b) * 64 + lane];
                    al[b] = lds[buf][1][(2 * wave + b) * 64 + lane];
                }
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const u32x4 wh = lds[buf][2][c * 64 + lane], wl = lds[buf][3][c * 64 + lane];
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        acc[b][c] = mfma_bf16(wh, ah[b], acc[b][c]);
                        acc[b][c] = mfma_bf16(wl, ah[b], acc[b][c]);
                        acc[b][c] = mfma_bf16(wh, al[b], acc[b][c]);
                    }
                }
            }
            if (more) put(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }
    float *Cq = (float *)d.C + split * d.cstride + lane * 4;
#pragma unroll
    for (int b = 0; b < 2; ++b)
        if (ok[b]) {
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (c < ncol) st4(Cq + off[b] + ((c * nb) << 8), acc[b][c]);
        }
}

// ---------------------------------------------------------------------------------------------
// Kernels: single instance (descriptor by value) and batched (descriptor array).

template <typename T, int NB>
__global__ void __launch_bounds__(256, 2) column_kernel(StepDesc d, int64_t per_xcd)
{
    const int64_t item = xcd_item(blockIdx.x, per_xcd);
    if (item >= d.nitems) return;
    column_body<T, NB>(d, item);
}

// d.nitems here counts (split, row tile, column chunk) items
template <typename T>
__global__ void __launch_bounds__(256, (sizeof(T) == 4 ? 4 : 2)) column_rt_kernel(StepDesc d, int64_t per_xcd)
{
    const int64_t item = xcd_item(blockIdx.x, per_xcd);
    if (item >= d.nitems) return;
    column_rt_body<T>(d, item);
}

// d.nitems here counts (split, row tile, column chunk) items
__global__ void __launch_bounds__(256, 2) column_bf16_rt_kernel(StepDesc d, int64_t per_xcd)
{
    const int64_t item = xcd_item(blockIdx.x, per_xcd);
    if (item >= d.nitems) return;
    column_bf16_rt_body(d, item);
}

template <int NB32>
__global__ void __launch_bounds__(256, 2) column_bf16_kernel(StepDesc d, int64_t per_xcd)
{
    const int64_t item = xcd_item(blockIdx.x, per_xcd);
    if (item >= d.nitems) return;
    column_bf16_body<NB32>(d, item);
}

template <typename T, int NB>
__global__ void __launch_bounds__(256, 2) column_batched(const StepDesc *__restrict__ ds, int n, int64_t total,
                                                         int64_t per_xcd)
{
    const int64_t item = xcd_item(blockIdx.x, per_xcd);
    if (item >= total) return;
    const int i = find_instance(ds, n, item);
    if (i < 0) return;
    const StepDesc d = ds[i];
    column_body<T, NB>(d, item - d.item0);
}

template <int NB32>
__global__ void __launch_bounds__(256, 2) column_bf16_batched(const StepDesc *__restrict__ ds, int n, int64_t total,
                                                              int64_t per_xcd)
{
    const int64_t item = xcd_item(blockIdx.x, per_xcd);
    if (item >= total) return;
    const int i = find_instance(ds, n, item);
    if (i < 0) return;
    const StepDesc d = ds[i];
    column_bf16_body<NB32>(d, item - d.item0);
}

// ---------------------------------------------------------------------------------------------
// Launchers.

template <typename T>
static hipError_t launch_column_t(const StepDesc &d, hipStream_t s)
{
    const int64_t per_xcd = (d.nitems + 7) / 8;
    const dim3 grid((unsigned)(per_xcd * 8)), block(256);
    switch (d.N_tp / 16) {
#define OED_COL_CASE(NBV)                                                                      \
    case NBV: hipLaunchKernelGGL((column_kernel<T, NBV>), grid, block, 0, s, d, per_xcd); break;
        OED_COL_CASE(1)
        OED_COL_CASE(2)
        OED_COL_CASE(3)
        OED_COL_CASE(4)
        OED_COL_CASE(5)
        OED_COL_CASE(6)
        OED_COL_CASE(7)
        OED_COL_CASE(8)
#undef OED_COL_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_column(const StepDesc &d, int rtype, int wtype, hipStream_t s)
{
    if (d.n_act <= 0 || d.nsplit <= 0 || d.nitems <= 0) return hipSuccess;
    if (d.N_tp % 16 != 0 || d.nw < d.nsplit || !d.C) return hipErrorInvalidValue;
    if (d.N_tp > 128) {
        if (wtype == W_BF16X3 && (d.N_tp % 32 != 0 || !d.W2)) return hipErrorInvalidValue;
        // one item per (split, row tile, 128-column chunk of the pick)
        StepDesc e = d;
        e.nitems = d.nitems * ((d.N_tp / 16 + 7) / 8);
        const int64_t per_xcd = (e.nitems + 7) / 8;
        const dim3 grid((unsigned)(per_xcd * 8)), block(256);
        if (wtype == W_BF16X3)
            hipLaunchKernelGGL(column_bf16_rt_kernel, grid, block, 0, s, e, per_xcd);
        else if (rtype == R_F64)
            hipLaunchKernelGGL(column_rt_kernel<double>, grid, block, 0, s, e, per_xcd);
        else
            hipLaunchKernelGGL(column_rt_kernel<float>, grid, block, 0, s, e, per_xcd);
        return hipGetLastError();
    }
    if (wtype == W_BF16X3) {
        if (d.N_tp % 32 != 0 || !d.W2) return hipErrorInvalidValue;
        const int64_t per_xcd = (d.nitems + 7) / 8;
        const dim3 grid((unsigned)(per_xcd * 8)), block(256);
        switch (d.N_tp / 32) {
        case 1: hipLaunchKernelGGL((column_bf16_kernel<1>), grid, block, 0, s, d, per_xcd); break;
        case 2: hipLaunchKernelGGL((column_bf16_kernel<2>), grid, block, 0, s, d, per_xcd); break;
        case 3: hipLaunchKernelGGL((column_bf16_kernel<3>), grid, block, 0, s, d, per_xcd); break;
        case 4: hipLaunchKernelGGL((column_bf16_kernel<4>), grid, block, 0, s, d, per_xcd); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    return rtype == R_F64 ? launch_column_t<double>(d, s) : launch_column_t<float>(d, s);
}

hipError_t launch_column_batched(const StepDesc *descs, int n, int64_t total, int N_tp, int rtype, int wtype,
                                 hipStream_t s)
{
    if (n <= 0 || total <= 0) return hipSuccess;
    if (N_tp % 16 != 0 || N_tp > 128) return hipErrorInvalidValue;
    const int64_t per_xcd = (total + 7) / 8;
    const dim3 grid((unsigned)(per_xcd * 8)), block(256);
    if (wtype == W_BF16X3) {
        switch (N_tp / 32) {
        case 1: hipLaunchKernelGGL((column_bf16_batched<1>), grid, block, 0, s, descs, n, total, per_xcd); break;
        case 2: hipLaunchKernelGGL((column_bf16_batched<2>), grid, block, 0, s, descs, n, total, per_xcd); break;
        case 3: hipLaunchKernelGGL((column_bf16_batched<3>), grid, block, 0, s, descs, n, total, per_xcd); break;
        case 4: hipLaunchKernelGGL((column_bf16_batched<4>), grid, block, 0, s, descs, n, total, per_xcd); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (N_tp / 16) {
#define OED_COLB_CASE(NBV)                                                                                         \
    case NBV:                                                                                                      \
        if (rtype == R_F64)                                                                                        \
            hipLaunchKernelGGL((column_batched<double, NBV>), grid, block, 0, s, descs, n, total, per_xcd);        \
        else                                                                                                       \
            hipLaunchKernelGGL((column_batched<float, NBV>), grid, block, 0, s, descs, n, total, per_xcd);         \
        break;
        OED_COLB_CASE(1)
        OED_COLB_CASE(2)
        OED_COLB_CASE(3)
        OED_COLB_CASE(4)
        OED_COLB_CASE(5)
        OED_COLB_CASE(6)
        OED_COLB_CASE(7)
        OED_COLB_CASE(8)
#undef OED_COLB_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace oed
