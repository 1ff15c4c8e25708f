// The block column of one greedy step: W = R[:, s] L_s^-T for every remaining row, the new block
// row of the factor in Algorithm 1 (Sec. III-D), with the corrections for block columns that the
// delayed downdate still holds back (V_h = L_s^-1 P_h,s), and the Schur-block query.
#include <type_traits>

#include "oed_device.h"

namespace oed {

// W_i = C_i L_s^-T computed as W_i^T = L_s^-1 C_i^T on FP64 MFMA (16x16x4): the accumulator of
// output sub-block (k-block kc, t-block tb) is then already in W's operand order.
template <typename TW>
__device__ __forceinline__ void store_w(TW *W, int64_t off, doublex4 a)
{
    typename V4<TW>::type v;
    v[0] = (TW)a[0];
    v[1] = (TW)a[1];
    v[2] = (TW)a[2];
    v[3] = (TW)a[3];
    st4(W + off, v);
}

// W in BF16 hi/lo parts: the accumulator of sub-block (tb, kc) holds rows 16tb + l%16 and
// inner indices 16kc + 4g + r; in the 16 x 32 BF16 operand order those four values are
// consecutive (lane ((k%32)/8)*16 + l%16, elements k%8), so each part is one 8-byte store.
// hi = bf16(w), lo = bf16(w - hi) with the residual taken in FP64.
__device__ __forceinline__ void store_w_bf16(unsigned short *Wh, unsigned short *Wl, int tb, int kc, int nb32, int lane,
                                             doublex4 a)
{
    const int g = lane >> 4, l16 = lane & 15;
    const int64_t off = ((int64_t)(tb * nb32 + (kc >> 1)) << 9) + ((((((kc & 1) << 1) + (g >> 1)) << 4) + l16) << 3) +
                        4 * (g & 1);
    u16x4 hi, lo;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const unsigned short h = f2bf((float)a[r]);
        hi[r] = h;
        lo[r] = f2bf((float)(a[r] - (double)bf2f(h)));
    }
    *reinterpret_cast<u16x4 *>(Wh + off) = hi;
    *reinterpret_cast<u16x4 *>(Wl + off) = lo;
}

// Four consecutive inner indices k = 16q + 4g .. 16q + 4g + 3 of row t = 16 tb + l % 16 of a W
// block, as doubles (lane l = 16 g + l % 16): one vector load in the FP32 / FP64 operand order,
// hi + lo of two 8-byte loads in the BF16 16 x 32 order.
template <typename TW>
__device__ __forceinline__ void w_row4(const TW *Wb, const TW *, int tb, int q, int nb, int lane, double (&v)[4])
{
    const typename V4<TW>::type x = ld4(Wb + ((int64_t)(tb * nb + q) << 8) + lane * 4);
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = (double)x[r];
}
template <>
__device__ __forceinline__ void w_row4<unsigned short>(const unsigned short *Wh, const unsigned short *Wl, int tb, int q,
                                                       int nb, int lane, double (&v)[4])
{
    const int g = lane >> 4, l16 = lane & 15;
    const int64_t off = ((int64_t)(tb * (nb >> 1) + (q >> 1)) << 9) +
                        (((((q & 1) << 1) + (g >> 1)) << 4) + l16) * 8 + 4 * (g & 1);
    const u16x4 h = *reinterpret_cast<const u16x4 *>(Wh + off), l = *reinterpret_cast<const u16x4 *>(Wl + off);
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = (double)bf2f(h[r]) + (double)bf2f(l[r]);
}

// One element (t, k) of a W block as a double.
template <typename TW>
__device__ __forceinline__ double w_elem(const TW *Wb, const TW *, int t, int k, int nb)
{
    return (double)Wb[((int64_t)((t >> 4) * nb + (k >> 4)) << 8) + ((((k & 15) >> 2) << 4) + (t & 15)) * 4 + (k & 3)];
}
template <>
__device__ __forceinline__ double w_elem<unsigned short>(const unsigned short *Wh, const unsigned short *Wl, int t, int k,
                                                         int nb)
{
    const int64_t o = ((int64_t)((t >> 4) * (nb >> 1) + (k >> 5)) << 9) + ((((k & 31) >> 3) << 4) + (t & 15)) * 8 + (k & 7);
    return (double)bf2f(Wh[o]) + (double)bf2f(Wl[o]);
}

// Correction of a delayed downdate: with the W of earlier picks held back (P_h), the block
// column of the new pick s is W_i = (R_is - sum_h P_h,i P_h,s^T) L_s^-T
// = R_is L_s^-T - sum_h P_h,i V_h^T with V_h = L_s^-1 P_h,s.  One wave per 16 x 16 sub-block of
// one V_h: V_h^T = P_h,s^T L_s^-T accumulated on FP64 MFMA lands in the accumulator order, which
// is V's operand order (the order of L_s^-1).
template <typename TW>
__device__ void vcorr_body(const StepDesc &d, int item)
{
    if (d.state[ST_STATUS] != 0) return;
    const int nb = d.N_tp >> 4;
    const int hp = item / (nb * nb);
    if (hp >= d.nheld) return;
    item -= hp * nb * nb;
    const int kb = item / nb, ab = item % nb;  // V^T sub-block (kb, ab) = V sub-block (ab, kb)
    const int lane = threadIdx.x & 63, g = lane >> 4, al = a_lane<double>(lane) & 15;
    const int s = uniform_at(d.state, ST_LAST);
    const int64_t bs = (int64_t)d.N_tp * d.N_tp;
    const TW *Ps = (const TW *)d.W + hp * d.wslot + s * bs;
    const TW *Ps2 = d.W2 ? (const TW *)d.W2 + hp * d.wslot + s * bs : nullptr;
    const int nbr = (d.N_t + 15) >> 4;  // rows of P_s past N_t are zero
    doublex4 acc{0.0, 0.0, 0.0, 0.0};
    for (int mq = 0; mq < nbr; ++mq) {
        const doublex4 b = ld4(d.Linv + ((ab * nb + mq) << 8) + lane * 4);
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
            acc = mfma16(w_elem<TW>(Ps, Ps2, 16 * mq + 4 * g + s4, 16 * kb + al, nb), b[s4], acc);
    }
    if constexpr (sizeof(TW) == 8) {
        st4(d.V + hp * bs + ((ab * nb + kb) << 8) + lane * 4, acc);
    } else {
        // the mixed paths apply V_h on the FP32 MFMA: keep it rounded to FP32 (the block column
        // kernel reads half the bytes and converts nothing)
        floatx4 v;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = (float)acc[r];
        st4((float *)d.V + hp * bs + ((ab * nb + kb) << 8) + lane * 4, v);
    }
}

template <typename TR, typename TW>
__device__ void trsm_body(const StepDesc &d, int p)
{
    if (d.state[ST_STATUS] != 0 || p >= d.n_act) return;
    const TR *__restrict__ R = (const TR *)d.R;
    TW *__restrict__ W = (TW *)d.W;
    const double *__restrict__ Linv = d.Linv;
    const int N_tp = d.N_tp;
    const int i = d.act_in[p], s = d.state[ST_LAST];
    const int nb = N_tp >> 4;
    const int64_t bs = (int64_t)N_tp * N_tp;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, l16 = lane & 15;
    const int alane = a_lane<double>(lane);
    const bool below = i > s;
    const TR *Cb = R + blk_index(below ? i : s, below ? s : i) * bs;
    TW *Wi = W + d.nheld * d.wslot + (int64_t)i * bs;             // slot nheld
    TW *Wi2 = (TW *)d.W2 + d.nheld * d.wslot + (int64_t)i * bs;
    for (int tb = wave; tb < nb; tb += 4) {
        for (int kg = 0; kg < nb; kg += 8) {
            const int kend = min(nb, kg + 8);
            doublex4 acc[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) acc[c] = doublex4{0.0, 0.0, 0.0, 0.0};
            // - sum_h P_h,i V_h^T first (held block columns; inner index over the held pick's
            // block, V_h in L_s^-1's order).  Mixed paths: on the FP32 MFMA (P is FP32, or BF16
            // hi + lo, exact in FP32; V_h rounded to FP32), the precision in which the downdate
            // would have subtracted them, then carried on in FP64.
            const int nbr = (d.N_t + 15) >> 4;
            if constexpr (sizeof(TR) == 4) {
                floatx4 hacc[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) hacc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
                for (int hp = 0; hp < d.nheld; ++hp) {
                    const TW *Pi = (const TW *)d.W + hp * d.wslot + (int64_t)i * bs;
                    const TW *Pi2 = d.W2 ? (const TW *)d.W2 + hp * d.wslot + (int64_t)i * bs : nullptr;
                    const float *Vh = (const float *)d.V + hp * bs;
                    for (int q = 0; q < nbr; ++q) {
                        double v[4];
                        w_row4<TW>(Pi, Pi2, tb, q, nb, lane, v);
                        float b[4];
#pragma unroll
                        for (int s4 = 0; s4 < 4; ++s4) b[s4] = (float)-v[s4];
#pragma unroll
                        for (int c = 0; c < 8; ++c) {
                            const int kc = kg + c;
                            if (kc < kend) {
                                // the FP32 MFMA takes its A operand in the natural lane order
                                const floatx4 a = ld4(Vh + ((kc * nb + q) << 8) + lane * 4);
#pragma unroll
                                for (int s4 = 0; s4 < 4; ++s4) hacc[c] = mfma16(a[s4], b[s4], hacc[c]);
                            }
                        }
                    }
                }
#pragma unroll
                for (int c = 0; c < 8; ++c)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[c][r] = (double)hacc[c][r];
            } else {
                for (int hp = 0; hp < d.nheld; ++hp) {
                    const TW *Pi = (const TW *)d.W + hp * d.wslot + (int64_t)i * bs;
                    const TW *Pi2 = d.W2 ? (const TW *)d.W2 + hp * d.wslot + (int64_t)i * bs : nullptr;
                    const double *Vh = d.V + hp * bs;
                    for (int q = 0; q < nbr; ++q) {
                        double b[4];
                        w_row4<TW>(Pi, Pi2, tb, q, nb, lane, b);
#pragma unroll
                        for (int s4 = 0; s4 < 4; ++s4) b[s4] = -b[s4];
#pragma unroll
                        for (int c = 0; c < 8; ++c) {
                            const int kc = kg + c;
                            if (kc < kend) {
                                const doublex4 a = ld4(Vh + ((kc * nb + q) << 8) + alane * 4);
#pragma unroll
                                for (int s4 = 0; s4 < 4; ++s4) acc[c] = mfma16(a[s4], b[s4], acc[c]);
                            }
                        }
                    }
                }
            }
            for (int q = 0; q < kend; ++q) {
                double b[4];
                if (below) {
                    const int t = 16 * tb + l16;
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) b[s4] = (double)Cb[acc_off(t, 16 * q + 4 * g + s4, nb)];
                } else {
                    const typename V4<TR>::type v = ld4(Cb + acc_off(16 * q + 4 * g, 16 * tb + l16, nb));
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) b[s4] = (double)v[s4];
                }
                // left-looking: C_i = K_is - sum_h W_h,i W_h,s^T, the sum in nsplit partials
                for (int sp = 0; sp < d.nsplit; ++sp) {
                    // transposed sub-block (q, tb): the lane's four pick rows in one vector
                    const TR *Cp = (const TR *)d.C + sp * d.cstride + (int64_t)i * bs;
                    const typename V4<TR>::type v = ld4(Cp + ((q * nb + tb) << 8) + lane * 4);
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) b[s4] -= (double)v[s4];
                }
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int kc = kg + c;
                    if (kc >= q && kc < kend) {
                        const doublex4 a = ld4(Linv + ((kc * nb + q) << 8) + alane * 4);
#pragma unroll
                        for (int s4 = 0; s4 < 4; ++s4) acc[c] = mfma16(a[s4], b[s4], acc[c]);
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int kc = kg + c;
                if (kc < kend) {
                    if constexpr (sizeof(TW) == 2)
                        store_w_bf16(Wi, Wi2, tb, kc, nb >> 1, lane, acc[c]);
                    else
                        store_w(Wi, ((int64_t)(tb * nb + kc) << 8) + lane * 4, acc[c]);
                }
            }
        }
    }
}

constexpr int TRSM_MAX_SPLITS = 4;  // left-looking partial sums the kernel reads (LEFT_SPLITS)

// A row block of a held W (P_h,i), four consecutive inner indices per lane, as loaded: FP32 or
// FP64 one vector, BF16 the hi and lo parts (w_row4 without the conversion, so that the load can
// be issued a slice ahead and waited for only where it is used).
template <typename TW>
struct PRaw {
    typename V4<TW>::type x;
    __device__ __forceinline__ void load(const TW *Wb, const TW *, int tb, int q, int nb, int lane)
    {
        x = ld4(Wb + ((int64_t)(tb * nb + q) << 8) + lane * 4);
    }
    __device__ __forceinline__ double get(int r) const { return (double)x[r]; }
};
template <>
struct PRaw<unsigned short> {
    u16x4 h, l;
    __device__ __forceinline__ void load(const unsigned short *Wh, const unsigned short *Wl, int tb, int q, int nb,
                                         int lane)
    {
        const int g = lane >> 4, l16 = lane & 15;
        const int64_t off = ((int64_t)(tb * (nb >> 1) + (q >> 1)) << 9) +
                            (((((q & 1) << 1) + (g >> 1)) << 4) + l16) * 8 + 4 * (g & 1);
        h = *reinterpret_cast<const u16x4 *>(Wh + off);
        l = *reinterpret_cast<const u16x4 *>(Wl + off);
    }
    __device__ __forceinline__ double get(int r) const { return (double)bf2f(h[r]) + (double)bf2f(l[r]); }
};

// D_ii -= W_i W_i^T on candidate i's own diagonal block: the update the gain kernel makes when it
// applies the newest block column (HeldProd over the nbr inner blocks, then
// R = (TR)((double)R - (double)q)), made here from the W_i the work-group has just formed.  The
// rounded W_i (as stored) is staged in LDS, wave w takes the lower blocks (C, I), I <= C < nbr,
// numbered w, w + NB, ..., and forms each as q^T = P_C P_I^T: the same products in the same order
// as the gain kernel's q = P_I P_C^T (the MFMA's operands swapped, each product commutes), which
// lands in R's storage order, so the block is read and written with vector accesses.  FP64 stages
// the inner blocks four at a time (64 KB of LDS).
template <typename TR, typename TW, int NB>
struct DiagStage {
    static constexpr int KH = sizeof(TW) == 8 ? (NB < 4 ? NB : 4) : NB;  // inner blocks per stage
};

template <typename TR, typename TW, int NB>
__device__ __forceinline__ void diag_update(TR *__restrict__ Rd, const doublex4 (&acc)[NB], int nbr, int tb,
                                            int lane, char *lds)
{
    using VR = typename V4<TR>::type;
    constexpr int KH = DiagStage<TR, TW, NB>::KH;
    constexpr int PERW = (NB * (NB + 1) / 2 + NB - 1) / NB;
    const int nblk = nbr * (nbr + 1) / 2;
    const int al = a_lane<double>(lane);
    // the blocks of this wave and their current values, loaded first (their latency is covered
    // by the staging and the products); a slot past the last block reads block 0 and is not stored
    int bc[PERW], bi[PERW];
    VR rv[PERW];
#pragma unroll
    for (int u = 0; u < PERW; ++u) {
        const int b = tb + u * NB;
        const int bb = b < nblk ? b : 0;
        bc[u] = (int)tri_row(bb);
        bi[u] = bb - bc[u] * (bc[u] + 1) / 2;
        rv[u] = ld4(Rd + ((bc[u] * NB + bi[u]) << 8) + lane * 4);
    }
    typedef typename std::conditional<sizeof(TW) == 8, doublex4, floatx4>::type QV;
    QV q[PERW];
#pragma unroll
    for (int k0 = 0; k0 < NB; k0 += KH) {
        __syncthreads();  // the LDS is free (the slices of the block column, or the previous stage)
        // the wave's row block tb of W_i, rounded as stored, inner blocks k0 .. k0 + KH - 1
        if constexpr (sizeof(TW) == 2) {
            unsigned short *Lh = (unsigned short *)lds, *Ll = Lh + NB * NB * 256;
#pragma unroll
            for (int c = 0; c < NB; ++c) store_w_bf16(Lh, Ll, tb, c, NB >> 1, lane, acc[c]);
        } else {
            TW *L = (TW *)lds;
#pragma unroll
            for (int c = 0; c < KH; ++c)
                if (k0 + c < NB) store_w(L, ((int64_t)(tb * KH + c) << 8) + lane * 4, acc[k0 + c]);
        }
        __syncthreads();
        if (k0 == 0) {
            // the products start here, after the wave's W_i went to LDS (fewer live registers)
#pragma unroll
            for (int u = 0; u < PERW; ++u) q[u] = QV{0, 0, 0, 0};
        }
#pragma unroll
        for (int u = 0; u < PERW; ++u) {
            if (tb + u * NB >= nblk) break;
            const int C = bc[u], I = bi[u];
            if constexpr (sizeof(TW) == 2) {
                const unsigned short *Lh = (const unsigned short *)lds, *Ll = Lh + NB * NB * 256;
                constexpr int N32 = NB / 2;
                const int n32 = (nbr + 1) >> 1;
#pragma unroll
                for (int kc = 0; kc < (N32 > 0 ? N32 : 1); ++kc)
                    if (kc < n32) {
                        const int oc = ((C * N32 + kc) << 9) + lane * 8, oi = ((I * N32 + kc) << 9) + lane * 8;
                        const u32x4 ch = *reinterpret_cast<const u32x4 *>(Lh + oc);
                        const u32x4 cl = *reinterpret_cast<const u32x4 *>(Ll + oc);
                        const u32x4 ih = *reinterpret_cast<const u32x4 *>(Lh + oi);
                        const u32x4 il = *reinterpret_cast<const u32x4 *>(Ll + oi);
                        // hi_I hi_C + hi_I lo_C + lo_I hi_C, in that order
                        q[u] = mfma_bf16(ch, ih, q[u]);
                        q[u] = mfma_bf16(cl, ih, q[u]);
                        q[u] = mfma_bf16(ch, il, q[u]);
                    }
            } else {
                const TW *L = (const TW *)lds;
#pragma unroll
                for (int c = 0; c < KH; ++c)
                    if (k0 + c < nbr) {
                        // FP64: the A operand's rows at the permuted lane, as everywhere
                        const typename V4<TW>::type a =
                            ld4(L + ((C * KH + c) << 8) + (sizeof(TW) == 8 ? al : lane) * 4);
                        const typename V4<TW>::type b = ld4(L + ((I * KH + c) << 8) + lane * 4);
#pragma unroll
                        for (int s4 = 0; s4 < 4; ++s4) q[u] = mfma16(a[s4], b[s4], q[u]);
                    }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < PERW; ++u) {
        if (tb + u * NB >= nblk) break;
        VR v;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = (TR)((double)rv[u][r] - (double)q[u][r]);
        st4(Rd + ((bc[u] * NB + bi[u]) << 8) + lane * 4, v);
    }
}

// The block column for N_tp = 16 NB <= 128 (single launches): one work-group of NB waves per
// remaining row i, wave w computing sub-block row tb = w of W_i (all NB sub-blocks of it).  The
// operands every wave needs -- V_h of the held columns and L_s^-1 -- pass through LDS one
// 16-column slice at a time, double-buffered: while the waves multiply slice j, the next slice is
// on its way from L2, and so are the wave's own rows of P_h,i (or of R_is and the left-looking
// partial sums) for it.  Slices: (h, q) for every held column h and 16-column block q of P_h,i,
// then q = 0 .. NB-1 of L_s^-1 (only the sub-blocks c >= q of its lower triangle).  Every
// accumulator sees the products of trsm_body in the same order, so W is bitwise the same.  With
// d.diag the work-group then applies W_i to candidate i's diagonal block (diag_update).
template <typename TR, typename TW, int NB, bool LEFT>
__device__ void trsm_nb_body(const StepDesc &d, int p)
{
    if (d.state[ST_STATUS] != 0 || p >= d.n_act) return;
    constexpr int MS = LEFT ? TRSM_MAX_SPLITS : 0;  // partial sums read (left-looking only)
    using VE = typename std::conditional<sizeof(TR) == 4, float, double>::type;  // V's element
    constexpr int nb = NB;
    constexpr int NT = 64 * NB;                 // threads
    constexpr int64_t bs = 256 * NB * NB;
    // the slice buffers (2 x NB sub-blocks of 256 doubles), and after the slices the staged W_i of
    // the diagonal update (NB^2 sub-blocks of FP32 / BF16 hi + lo, or NB x 4 of FP64)
    constexpr int SLICE_D = 2 * NB * 256;                                             // doubles
    constexpr int STAGE_D = sizeof(TW) == 8 ? NB * DiagStage<TR, TW, NB>::KH * 256 : NB * NB * 128;
    __shared__ __align__(16) double lds_all[SLICE_D > STAGE_D ? SLICE_D : STAGE_D];
    double(*sbuf)[NB * 256] = reinterpret_cast<double(*)[NB * 256]>(lds_all);
    const TR *__restrict__ R = (const TR *)d.R;
    const int i = d.act_in[p], s = d.state[ST_LAST];
    const int lane = threadIdx.x & 63, g = lane >> 4, l16 = lane & 15;
    const int tb = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int alane = a_lane<double>(lane);
    const bool below = i > s;
    const TR *Cb = R + blk_index(below ? i : s, below ? s : i) * bs;
    const int nbr = (d.N_t + 15) >> 4;          // rows of P past N_t are zero
    // left-looking runs hold no block column back; the FP32 variant has its held-slice loop compiled
    // out (that spills less there; for the BF16 variant keeping it does)
    const int nheld = (LEFT && sizeof(TW) == 4) ? 0 : d.nheld, nsplit = min(d.nsplit, MS);
    const int nhs = nheld * nbr;                // held slices
    const int nsl = nhs + NB;                   // all slices
    const int t = 16 * tb + l16;

    // the shared operand of slice j in 16-byte chunks: chunk ch of a slice whose sub-blocks
    // c0 .. NB-1 are staged lands at LDS byte c0 * 256 * eb + 16 ch (eb: element bytes)
    u32x4 stg[2];
    auto fetch_shared = [&](int j) {
        const bool held = j < nhs;
        const int q = held ? j % nbr : j - nhs;
        const int c0 = held ? 0 : q, eb = held ? (int)sizeof(VE) : 8, cpb = 16 * eb;
        const char *src = held ? (const char *)((const VE *)d.V + (j / nbr) * bs + (q << 8))
                               : (const char *)(d.Linv + (q << 8));
        const int nch = (NB - c0) * cpb;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int ch = (int)threadIdx.x + r * NT;
            if (ch < nch) {
                const int c = c0 + ch / cpb, off = ch % cpb;
                stg[r] = *reinterpret_cast<const u32x4 *>(src + ((int64_t)c * nb << 8) * eb + off * 16);
            }
        }
    };
    auto store_shared = [&](int j, int buf) {
        const bool held = j < nhs;
        const int c0 = held ? 0 : j - nhs, eb = held ? (int)sizeof(VE) : 8, cpb = 16 * eb;
        const int nch = (NB - c0) * cpb;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int ch = (int)threadIdx.x + r * NT;
            if (ch < nch) *reinterpret_cast<u32x4 *>((char *)sbuf[buf] + c0 * 256 * eb + ch * 16) = stg[r];
        }
    };
    // the wave's own operand of slice j, as loaded: row block tb of P_h,i (held slices), or of
    // R_is and of the left-looking partial sums (slices of L_s^-1)
    PRaw<TW> pr;
    TR cr[1 + MS][4];
    auto fetch_own = [&](int j) {
        if (j < nhs) {
            const int hp = j / nbr, q = j % nbr;
            const TW *Pi = (const TW *)d.W + hp * d.wslot + (int64_t)i * bs;
            const TW *Pi2 = d.W2 ? (const TW *)d.W2 + hp * d.wslot + (int64_t)i * bs : nullptr;
            pr.load(Pi, Pi2, tb, q, nb, lane);
        } else {
            const int q = j - nhs;
            if (below) {
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) cr[0][s4] = Cb[acc_off(t, 16 * q + 4 * g + s4, nb)];
            } else {
                const typename V4<TR>::type v = ld4(Cb + acc_off(16 * q + 4 * g, t, nb));
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) cr[0][s4] = v[s4];
            }
#pragma unroll
            for (int sp = 0; sp < MS; ++sp)
                if (sp < nsplit) {
                    // transposed sub-block (q, tb): the lane's four pick rows in one vector
                    const TR *Cp = (const TR *)d.C + sp * d.cstride + (int64_t)i * bs;
                    const typename V4<TR>::type v = ld4(Cp + ((q * nb + tb) << 8) + lane * 4);
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) cr[1 + sp][s4] = v[s4];
                }
        }
    };
    // after the multiplications of slice j: the next slice into the other buffer
    auto advance = [&](int j) {
        if (j + 1 < nsl) {
            store_shared(j + 1, (j + 1) & 1);
            __syncthreads();
        }
    };

    fetch_shared(0);
    fetch_own(0);
    store_shared(0, 0);
    __syncthreads();

    doublex4 acc[NB];
    if constexpr (sizeof(TR) == 4) {
        // - sum_h P_h,i V_h^T on the FP32 MFMA (P is FP32, or BF16 hi + lo, exact in FP32; V_h
        // rounded to FP32) -- the precision the downdate itself would have subtracted these
        // columns in -- accumulated apart and carried on in FP64
        floatx4 hacc[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) hacc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
        for (int j = 0; j < nhs; ++j) {
            float b[4];
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) b[s4] = (float)-pr.get(s4);
            fetch_shared(j + 1);
            fetch_own(j + 1);
            const float *Vs = (const float *)sbuf[j & 1];
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                // the FP32 MFMA takes its A operand in the natural lane order
                const floatx4 a = ld4(Vs + (c << 8) + lane * 4);
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) hacc[c] = mfma16(a[s4], b[s4], hacc[c]);
            }
            advance(j);
        }
#pragma unroll
        for (int c = 0; c < NB; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[c][r] = (double)hacc[c][r];
    } else {
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[c] = doublex4{0.0, 0.0, 0.0, 0.0};
        for (int j = 0; j < nhs; ++j) {
            double b[4];
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) b[s4] = -pr.get(s4);
            fetch_shared(j + 1);
            fetch_own(j + 1);
            const double *Vs = sbuf[j & 1];
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const doublex4 a = ld4(Vs + (c << 8) + alane * 4);
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) acc[c] = mfma16(a[s4], b[s4], acc[c]);
            }
            advance(j);
        }
    }
    // + C_i L_s^-T, C_i = R_is (right-looking) or K_is - sum_h W_h,i W_h,s^T (left-looking, the sum
    // in nsplit partials)
    for (int q = 0; q < NB; ++q) {
        const int j = nhs + q;
        double b[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            b[s4] = (double)cr[0][s4];
#pragma unroll
            for (int sp = 0; sp < MS; ++sp)
                if (sp < nsplit) b[s4] -= (double)cr[1 + sp][s4];
        }
        if (j + 1 < nsl) {
            fetch_shared(j + 1);
            fetch_own(j + 1);
        }
        const double *Ls = sbuf[j & 1];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            if (c >= q) {
                const doublex4 a = ld4(Ls + (c << 8) + alane * 4);
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) acc[c] = mfma16(a[s4], b[s4], acc[c]);
            }
        }
        advance(j);
    }
    TW *Wi = (TW *)d.W + nheld * d.wslot + (int64_t)i * bs;  // slot nheld
    TW *Wi2 = (TW *)d.W2 + nheld * d.wslot + (int64_t)i * bs;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        if constexpr (sizeof(TW) == 2)
            store_w_bf16(Wi, Wi2, tb, c, nb >> 1, lane, acc[c]);
        else
            store_w(Wi, ((int64_t)(tb * nb + c) << 8) + lane * 4, acc[c]);
    }
    if (d.diag) diag_update<TR, TW, NB>((TR *)d.R + blk_index(i, i) * bs, acc, nbr, tb, lane, (char *)lds_all);
}

// ---------------------------------------------------------------------------------------------
// Kernels: single instance (descriptor by value) and batched (descriptor array).

template <typename TR, typename TW>
__global__ void __launch_bounds__(256) trsm_kernel(StepDesc d)
{
    trsm_body<TR, TW>(d, blockIdx.x);
}

template <typename TR, typename TW, int NB, bool LEFT>
__global__ void __launch_bounds__(64 * NB, (LEFT && sizeof(TR) == 8) ? 2 : 4) trsm_nb_kernel(StepDesc d)
{
    trsm_nb_body<TR, TW, NB, LEFT>(d, blockIdx.x);
}

template <typename TR, typename TW>
__global__ void __launch_bounds__(256) trsm_batched(const StepDesc *__restrict__ ds, int n)
{
    const int i = find_instance(ds, n, blockIdx.x);
    if (i < 0) return;
    const StepDesc d = ds[i];
    trsm_body<TR, TW>(d, (int)(blockIdx.x - d.item0));
}

template <typename TW>
__global__ void __launch_bounds__(64) vcorr_kernel(StepDesc d)
{
    vcorr_body<TW>(d, blockIdx.x);
}

template <typename TW>
__global__ void __launch_bounds__(64) vcorr_batched(const StepDesc *__restrict__ ds, int n)
{
    const int i = find_instance(ds, n, blockIdx.x);
    if (i < 0) return;
    const StepDesc d = ds[i];
    vcorr_body<TW>(d, (int)(blockIdx.x - d.item0));
}

// ---------------------------------------------------------------------------------------------
// Query: block (li, lj) of the current Schur complement, unpadded FP64 row-major N_t x N_t, from
// R's stored lower block (li >= lj; with tr the transpose is returned, on the diagonal the lower
// triangle is mirrored) minus sum_k W_k,li W_k,lj^T over the nsub W slots that R does not include
// (left-looking: every formed block column; right-looking: none).  One thread per element.
template <typename TR, typename TW>
__global__ void __launch_bounds__(256) schur_block_kernel(const TR *__restrict__ R, const TW *__restrict__ W,
                                                          const TW *__restrict__ W2, int64_t wslot, int nsub, int li,
                                                          int lj, int tr, int N_t, int N_tp, double *__restrict__ out)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N_t * N_t) return;
    const int a = e / N_t, b = e - a * N_t;      // element (a, b) of the returned block
    const int t = tr ? b : a, u = tr ? a : b;    // element (t, u) of stored block (li, lj)
    const int nb = N_tp >> 4;
    const int64_t bs = (int64_t)N_tp * N_tp;
    const TR *Rb = R + blk_index(li, lj) * bs;
    // a diagonal block is current on its lower triangle only
    const int o = (li == lj && u > t) ? acc_off(u, t, nb) : acc_off(t, u, nb);
    double v = (double)Rb[o];
    for (int k = 0; k < nsub; ++k) {
        const TW *Wi = W + k * wslot + (int64_t)li * bs, *Wj = W + k * wslot + (int64_t)lj * bs;
        const TW *Wi2 = W2 ? W2 + k * wslot + (int64_t)li * bs : nullptr;
        const TW *Wj2 = W2 ? W2 + k * wslot + (int64_t)lj * bs : nullptr;
        double acc = 0.0;
        for (int m = 0; m < N_t; ++m) acc += w_elem<TW>(Wi, Wi2, t, m, nb) * w_elem<TW>(Wj, Wj2, u, m, nb);
        v -= acc;
    }
    out[e] = v;
}

hipError_t launch_schur_block(const void *R, int rtype, const void *W, const void *W2, int wtype, int64_t wslot,
                              int nsub, int li, int lj, int tr, int N_t, int N_tp, double *out, hipStream_t s)
{
    const dim3 grid((unsigned)((N_t * N_t + 255) / 256)), block(256);
#define OED_SCHUR(TR, TW)                                                                                       \
    hipLaunchKernelGGL((schur_block_kernel<TR, TW>), grid, block, 0, s, (const TR *)R, (const TW *)W,              \
                       (const TW *)W2, wslot, nsub, li, lj, tr, N_t, N_tp, out)
    if (rtype == R_F64 && wtype == W_F64)
        OED_SCHUR(double, double);
    else if (rtype == R_F32 && wtype == W_F32)
        OED_SCHUR(float, float);
    else if (rtype == R_F32 && wtype == W_BF16X3)
        OED_SCHUR(float, unsigned short);
    else
        return hipErrorInvalidValue;
#undef OED_SCHUR
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Launchers.

template <typename TR, typename TW>
static hipError_t launch_trsm_t(const StepDesc *descs, const StepDesc &d, int n, int64_t total, hipStream_t s)
{
    // the in-place diagonal update exists in the single-launch kernel only
    if (d.diag && (descs || d.N_tp > 128)) return hipErrorInvalidValue;
    if (!descs && d.N_tp <= 128) {
        if (d.nsplit > TRSM_MAX_SPLITS) return hipErrorInvalidValue;
        const dim3 grid((unsigned)total), block(d.N_tp * 4);
        switch (d.N_tp / 16) {
#define OED_TRSM_CASE(NBV)                                                                        \
    case NBV:                                                                                     \
        if (d.nsplit > 0)                                                                         \
            hipLaunchKernelGGL((trsm_nb_kernel<TR, TW, NBV, true>), grid, block, 0, s, d);        \
        else                                                                                      \
            hipLaunchKernelGGL((trsm_nb_kernel<TR, TW, NBV, false>), grid, block, 0, s, d);       \
        break;
            OED_TRSM_CASE(1)
            OED_TRSM_CASE(2)
            OED_TRSM_CASE(3)
            OED_TRSM_CASE(4)
            OED_TRSM_CASE(5)
            OED_TRSM_CASE(6)
            OED_TRSM_CASE(7)
            OED_TRSM_CASE(8)
#undef OED_TRSM_CASE
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (descs)
        hipLaunchKernelGGL((trsm_batched<TR, TW>), dim3((unsigned)total), dim3(256), 0, s, descs, n);
    else
        hipLaunchKernelGGL((trsm_kernel<TR, TW>), dim3((unsigned)total), dim3(256), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_trsm(const StepDesc &d, int rtype, int wtype, hipStream_t s)
{
    if (d.n_act <= 0) return hipSuccess;
    if (rtype == R_F64 && wtype == W_F64) return launch_trsm_t<double, double>(nullptr, d, 1, d.n_act, s);
    if (rtype == R_F32 && wtype == W_F32) return launch_trsm_t<float, float>(nullptr, d, 1, d.n_act, s);
    if (rtype == R_F32 && wtype == W_BF16X3) return launch_trsm_t<float, unsigned short>(nullptr, d, 1, d.n_act, s);
    return hipErrorInvalidValue;
}

hipError_t launch_trsm_batched(const StepDesc *descs, int n, int64_t total, int rtype, int wtype, hipStream_t s)
{
    if (n <= 0 || total <= 0) return hipSuccess;
    StepDesc none{};
    if (rtype == R_F64 && wtype == W_F64) return launch_trsm_t<double, double>(descs, none, n, total, s);
    if (rtype == R_F32 && wtype == W_F32) return launch_trsm_t<float, float>(descs, none, n, total, s);
    if (rtype == R_F32 && wtype == W_BF16X3) return launch_trsm_t<float, unsigned short>(descs, none, n, total, s);
    return hipErrorInvalidValue;
}

template <typename TW>
static hipError_t launch_vcorr_t(const StepDesc *descs, const StepDesc &d, int n, int64_t total, hipStream_t s)
{
    if (descs)
        hipLaunchKernelGGL((vcorr_batched<TW>), dim3((unsigned)total), dim3(64), 0, s, descs, n);
    else
        hipLaunchKernelGGL((vcorr_kernel<TW>), dim3((unsigned)total), dim3(64), 0, s, d);
    return hipGetLastError();
}

// One work-group per 16 x 16 sub-block of each V_h (single: d.nitems ignored, nheld (N_tp / 16)^2 groups).
hipError_t launch_vcorr(const StepDesc &d, int wtype, hipStream_t s)
{
    if (d.nheld < 1 || d.nheld >= MAX_DELAY || !d.V) return hipErrorInvalidValue;
    const int64_t total = (int64_t)d.nheld * (d.N_tp / 16) * (d.N_tp / 16);
    if (wtype == W_F64) return launch_vcorr_t<double>(nullptr, d, 1, total, s);
    if (wtype == W_F32) return launch_vcorr_t<float>(nullptr, d, 1, total, s);
    if (wtype == W_BF16X3) return launch_vcorr_t<unsigned short>(nullptr, d, 1, total, s);
    return hipErrorInvalidValue;
}

hipError_t launch_vcorr_batched(const StepDesc *descs, int n, int64_t total, int wtype, hipStream_t s)
{
    if (n <= 0 || total <= 0) return hipSuccess;
    StepDesc none{};
    if (wtype == W_F64) return launch_vcorr_t<double>(descs, none, n, total, s);
    if (wtype == W_F32) return launch_vcorr_t<float>(descs, none, n, total, s);
    if (wtype == W_BF16X3) return launch_vcorr_t<unsigned short>(descs, none, n, total, s);
    return hipErrorInvalidValue;
}

}  // namespace oed
