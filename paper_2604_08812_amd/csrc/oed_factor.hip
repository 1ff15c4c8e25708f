// FP64 factorisation kernels of one greedy step: the gains of all remaining candidates (a
// Cholesky of every diagonal block R_jj, i.e. of every matrix M_j of Algorithm 1, Sec. III-D),
// and the pick (argmax with lowest-index ties, active-list update, factor of the winner and
// its inverse).  Blocked factorisations on the FP64 MFMA serve N_t <= REGS_MAX_NT (register
// resident) and N_tp <= BLK_MAX_NTP (global scratch); element-wise LDS or global-scratch kernels
// serve larger blocks.
#include <algorithm>

#include "oed_device.h"

namespace oed {

// ---------------------------------------------------------------------------------------------
// FP64 factorisation helpers (whole work-group; A is a packed lower triangle).

// Load the real N_t x N_t lower part of a diagonal block of R (accumulator order) into A.
template <typename TR>
__device__ void load_diag_block(const TR *__restrict__ Rb, int N_t, int N_tp, double *A)
{
    const int nb = N_tp >> 4;
    const int n2 = N_tp * N_tp;
    for (int o = threadIdx.x; o < n2; o += blockDim.x) {
        const int sb = o >> 8, w = o & 255, lane = w >> 2, reg = w & 3;
        const int t = (sb / nb) * 16 + ((lane >> 4) << 2) + reg;
        const int u = (sb % nb) * 16 + (lane & 15);
        if (t < N_t && u <= t) A[tri(t) + u] = (double)Rb[o];
    }
}

// Right-looking Cholesky in place (A -> L).  Returns sum_t ln L_tt in every thread,
// or -inf as soon as a pivot is not > 0 or not finite.  blockDim.x must be 256.
__device__ double chol_packed(double *A, int n)
{
    double logsum = 0.0;
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
    for (int j = 0; j < n; ++j) {
        __syncthreads();
        const int jj = tri(j) + j;
        const double d = A[jj];
        if (!(d > 0.0) || !isfinite(d)) return -INFINITY;
        const double l = sqrt(d);
        logsum += log(l);
        for (int t = j + 1 + (int)threadIdx.x; t < n; t += blockDim.x) A[tri(t) + j] /= l;
        __syncthreads();
        if (threadIdx.x == 0) A[jj] = l;
        for (int t = j + 1 + tr; t < n; t += 16) {
            double *At = A + tri(t);
            const double ltj = At[j];
            for (int u = j + 1 + tc; u <= t; u += 16) At[u] -= ltj * A[tri(u) + j];
        }
    }
    __syncthreads();
    return logsum;
}

// X = L^-1 for the packed lower factor L (both packed lower, n x n).
__device__ void tri_inverse(const double *L, double *X, int n)
{
    const int m = tri(n);
    for (int o = threadIdx.x; o < m; o += blockDim.x) X[o] = 0.0;
    __syncthreads();
    for (int t = threadIdx.x; t < n; t += blockDim.x) X[tri(t) + t] = 1.0;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        const double ljj = L[tri(j) + j];
        double *Xj = X + tri(j);
        for (int c = threadIdx.x; c <= j; c += blockDim.x) Xj[c] /= ljj;
        __syncthreads();
        const int w = j + 1, total = (n - j - 1) * w;
        for (int f = threadIdx.x; f < total; f += blockDim.x) {
            const int i = j + 1 + f / w, c = f - (f / w) * w;
            X[tri(i) + c] -= L[tri(i) + j] * Xj[c];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------------
// Register-resident FP64 factorisations for N_t <= 128 (work-group of 256 threads).
//
// Product P_I P_J^T of sub-block rows I and J of one candidate's held W block (the W of an
// earlier pick that R does not include yet), over its first nk 16-wide inner blocks (the rest
// is padding, zero), in the 16x16 accumulator order of R: element (4g + r, l % 16) of lane l,
// register r.  Same operand orders and MFMA types as the downdate.
template <typename TW>
struct HeldProd;
template <>
struct HeldProd<double> {
    __device__ static __forceinline__ doublex4 run(const double *P, const double *, int I, int J, int nb, int nk,
                                                   int lane)
    {
        const int al = a_lane<double>(lane);
        doublex4 acc{0.0, 0.0, 0.0, 0.0};
        for (int kc = 0; kc < nk; ++kc) {
            const doublex4 a = ld4(P + ((I * nb + kc) << 8) + al * 4);
            const doublex4 b = ld4(P + ((J * nb + kc) << 8) + lane * 4);
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) acc = mfma16(a[s4], b[s4], acc);
        }
        return acc;
    }
};
template <>
struct HeldProd<float> {
    __device__ static __forceinline__ floatx4 run(const float *P, const float *, int I, int J, int nb, int nk,
                                                  int lane)
    {
        floatx4 acc{0.f, 0.f, 0.f, 0.f};
        for (int kc = 0; kc < nk; ++kc) {
            const floatx4 a = ld4(P + ((I * nb + kc) << 8) + lane * 4);
            const floatx4 b = ld4(P + ((J * nb + kc) << 8) + lane * 4);
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) acc = mfma16(a[s4], b[s4], acc);
        }
        return acc;
    }
};
template <>
struct HeldProd<unsigned short> {
    // BF16 hi (P) and lo (P2) parts, 16 x 32 sub-blocks: hi hi^T + hi lo^T + lo hi^T
    __device__ static __forceinline__ floatx4 run(const unsigned short *P, const unsigned short *P2, int I, int J,
                                                  int nb, int nk, int lane)
    {
        const int nb32 = nb >> 1;
        floatx4 acc{0.f, 0.f, 0.f, 0.f};
        for (int kc = 0; kc < (nk + 1) >> 1; ++kc) {
            const int64_t oa = ((int64_t)(I * nb32 + kc) << 9) + lane * 8, ob = ((int64_t)(J * nb32 + kc) << 9) + lane * 8;
            const u32x4 ah = *reinterpret_cast<const u32x4 *>(P + oa), al = *reinterpret_cast<const u32x4 *>(P2 + oa);
            const u32x4 bh = *reinterpret_cast<const u32x4 *>(P + ob), bl = *reinterpret_cast<const u32x4 *>(P2 + ob);
            acc = mfma_bf16(ah, bh, acc);
            acc = mfma_bf16(ah, bl, acc);
            acc = mfma_bf16(al, bh, acc);
        }
        return acc;
    }
};

// ---------------------------------------------------------------------------------------------
// Blocked register Cholesky on FP64 MFMA for N_t <= 128 (gains and picks).  Upper form:
// A = U^T U, block by block, with A held as its upper 16x16 blocks (I, C), I <= C, in the
// accumulator order (lane l, g = l/16 holds elements (4g + r, l % 16), r = 0..3).  Wave w
// owns block columns C in {w, 7 - w}.  Step p:
//   (a) the owner of column p factors A_pp = U_pp^T U_pp inside one wave and publishes
//       Y = U_pp^-1 through LDS (one barrier);
//   (b) every owner of a column C > p forms U_pC = U_pp^-T A_pC on the MFMA (the B operand is
//       the register block itself) and publishes it (one barrier);
//   (c) every owner updates its blocks A_IC -= U_pI^T U_pC, p < I <= C (MFMA).
// In this form every product takes its B operand in the accumulator order and its A operand
// from an accumulator-order block read at the permuted lane a_lane() (see mfma16 / a_lane),
// so no operand is ever transposed.  The stored lower blocks of R are read transposed.

// In-wave factorisation of one 16x16 diagonal block M (accumulator order) by symmetric
// elimination, carrying X = L_u^-1 along (M = L_u D L_u^T, L_u unit lower): then
// U^-T = D^-1/2 X and Y = U^-1 has Y[a][b] = X[b][a] / sqrt(d_b).  Writes Y in the accumulator
// order to ylds (256 doubles) and the pivots d_j to piv[0..15] (LDS, lane 0).  Returns false,
// uniformly over the wave, at a pivot that is not > 0 or not finite.
__device__ __forceinline__ bool chol16_inv(doublex4 M, double *ylds, double *piv)
{
    const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    doublex4 X;
#pragma unroll
    for (int r = 0; r < 4; ++r) X[r] = (4 * g + r == c) ? 1.0 : 0.0;
    // a run-time loop keeps the code small (it is instantiated once per block column)
#pragma unroll 1
    for (int j = 0; j < 16; ++j) {
        const int jg = j >> 2, jr = j & 3;
        // the pivot and row j of the eliminated block (row j: lanes of group jg, register jr);
        // column j of the lane's own rows 4g + r sits in lane 16 g + j by symmetry
        const double mj = M[jr], xj = X[jr];
        const int src = jg * 16 + j;  // wave-uniform
        const double d = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(mj), src),
                                          __builtin_amdgcn_readlane(__double2loint(mj), src));
        if (!(d > 0.0) || !isfinite(d)) return false;
        if (lane == 0) piv[j] = d;
        // 1/d from the hardware reciprocal and two Newton steps (within an ulp or two)
        double inv = __builtin_amdgcn_rcp(d);
        inv = fma(inv, fma(-d, inv, 1.0), inv);
        inv = fma(inv, fma(-d, inv, 1.0), inv);
        const double mjc = c > j ? __shfl(mj, jg * 16 + c) : 0.0;
        const double xjc = __shfl(xj, jg * 16 + c);
        double mja[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) mja[r] = __shfl(M[r], g * 16 + j);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double m = 4 * g + r > j ? mja[r] * inv : 0.0;
            M[r] = fma(-m, mjc, M[r]);
            X[r] = fma(-m, xjc, X[r]);
        }
    }
    // the pivots went to LDS from lane 0; the wave's LDS accesses complete in order
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int x = 4 * g + r;
        ylds[((((c >> 2) << 4) + x) << 2) + (c & 3)] = X[r] / sqrt(piv[x]);
    }
    return true;
}

// The register blocks of one wave: block column C0 = w (<= 3) keeps blocks I = 0..3 (those
// with I <= C0 are used), block column C1 = 7 - w (>= 4) keeps blocks I = 0..7.  ub() maps
// (h, I) to them; with h and I compile-time constants the selection is static.
struct UBlocks {
    doublex4 c0[4], c1[8];
};
__device__ __forceinline__ doublex4 &ub(UBlocks &A, int h, int I) { return h ? A.c1[I & 7] : A.c0[I & 3]; }

// Load the candidate's current Schur block as upper blocks: block (I, C) of the upper form is
// the transpose of the stored lower block (C, I); with held W blocks (slots 0 .. nheld-1 at
// candidate offset pofs) their products P_I P_C^T are subtracted, and with d.wb the corrected
// block is written back (left-looking).
template <typename TR, typename TW>
__device__ __forceinline__ void load_upper(UBlocks &A, const TR *__restrict__ Rb, int nbr, int nb, const StepDesc &d,
                                           int64_t pofs)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
    // element (4g + r, c) of upper (I, C) = element (c, 4g + r) of lower (C, I)
    const int tofs = ((((c >> 2) << 4) + 4 * g) << 2) + (c & 3);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int C = h ? 7 - w : w;
#pragma unroll
        for (int I = 0; I < (h ? 8 : 4); ++I) {
            if (C < nbr && I <= C) {
                const TR *blk = Rb + ((C * nb + I) << 8) + tofs;
#pragma unroll
                for (int r = 0; r < 4; ++r) ub(A, h, I)[r] = (double)blk[4 * r];
            } else {
                ub(A, h, I) = doublex4{0.0, 0.0, 0.0, 0.0};
            }
        }
    }
    for (int hp = 0; hp < d.nheld; ++hp) {
        const TW *P = (const TW *)d.W + hp * d.wslot + pofs;
        const TW *P2 = d.W2 ? (const TW *)d.W2 + hp * d.wslot + pofs : nullptr;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int C = h ? 7 - w : w;
#pragma unroll
            for (int I = 0; I < (h ? 8 : 4); ++I)
                if (C < nbr && I <= C) {
                    const auto q = HeldProd<TW>::run(P, P2, I, C, nb, nbr, lane);
#pragma unroll
                    for (int r = 0; r < 4; ++r) ub(A, h, I)[r] -= (double)q[r];
                }
        }
    }
    if (d.wb && d.nheld > 0) {
        // the corrected blocks as stored: the factorisation below takes the rounded value too,
        // as it would after the block column kernel's in-place update (trsm with d.diag)
        TR *Rw = const_cast<TR *>(Rb);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int C = h ? 7 - w : w;
#pragma unroll
            for (int I = 0; I < (h ? 8 : 4); ++I)
                if (C < nbr && I <= C) {
                    TR *blk = Rw + ((C * nb + I) << 8) + tofs;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const TR v = (TR)ub(A, h, I)[r];
                        blk[4 * r] = v;
                        ub(A, h, I)[r] = (double)v;
                    }
                }
        }
    }
}

// Step p of the blocked factorisation (p is a compile-time constant, so that every register
// block is addressed statically).  Returns false (uniformly) at a failed pivot.
template <int p>
__device__ __forceinline__ bool chol_mfma_step(UBlocks &A, int nbr, double *piv, doublex4 (*Ls)[8][64], int *sfail,
                                               doublex4 (*Ysave)[64], doublex4 (*Usave)[64])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int al = a_lane<double>(lane);
    const int C0 = w, C1 = 7 - w;
    constexpr int buf = p & 1, hp = p < 4 ? 0 : 1;  // column p is a C0 column iff p <= 3
    // (a) the owner of block column p
    if ((hp ? C1 : C0) == p) {
        const bool ok = chol16_inv(ub(A, hp, p), (double *)Ls[buf][p], piv + 16 * p);
        if (lane == 0) sfail[buf] = ok ? 0 : 1;
    }
    __syncthreads();
    if (sfail[buf]) return false;
    if (Ysave && (hp ? C1 : C0) == p) Ysave[p][lane] = Ls[buf][p][lane];
    // (b) U_pC = U_pp^-T A_pC for the owned columns C > p
    const doublex4 y = Ls[buf][p][al];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int C = h ? C1 : C0;
        if ((h || p < 4) && C > p && C < nbr) {
            doublex4 acc{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) acc = mfma16(y[s4], ub(A, h, p)[s4], acc);
            ub(A, h, p) = acc;
            Ls[buf][C][lane] = acc;
            // U_pC is final: kept for the pick as soon as it is formed, so the factor cache's stores
            // spread over the factorisation instead of trailing it
            if (Usave) Usave[C * (C - 1) / 2 + p][lane] = acc;
        }
    }
    __syncthreads();
    // (c) A_IC -= U_pI^T U_pC for p < I <= C
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int C = h ? C1 : C0;
        if ((h || p < 4) && C > p && C < nbr) {
#pragma unroll
            for (int I = p + 1; I < (h ? 8 : 4); ++I)
                if (I <= C) {
                    const doublex4 u = Ls[buf][I][al];
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) ub(A, h, I) = mfma16(-u[s4], ub(A, h, p)[s4], ub(A, h, I));
                }
        }
    }
    return true;
}

// The blocked factorisation of the register blocks A (loaded by load_upper); pivots d_j go to
// piv[0 .. 16 nbr), with Ysave (8 blocks) U_pp^-1 of every diagonal block is kept and with Usave
// (block (I, C) at C (C - 1) / 2 + I) every off-diagonal block U_IC, I < C.  On return A holds the
// off-diagonal blocks of U.  Returns false (uniformly) at a pivot that is not > 0 or not finite.
__device__ __forceinline__ bool chol_mfma_regs(UBlocks &A, int nbr, double *piv, doublex4 (*Ysave)[64],
                                               doublex4 (*Usave)[64])
{
    __shared__ doublex4 Ls[2][8][64];  // [step parity][block column][lane]
    __shared__ int sfail[2];
    if (!chol_mfma_step<0>(A, nbr, piv, Ls, sfail, Ysave, Usave)) return false;
    if (nbr > 1 && !chol_mfma_step<1>(A, nbr, piv, Ls, sfail, Ysave, Usave)) return false;
    if (nbr > 2 && !chol_mfma_step<2>(A, nbr, piv, Ls, sfail, Ysave, Usave)) return false;
    if (nbr > 3 && !chol_mfma_step<3>(A, nbr, piv, Ls, sfail, Ysave, Usave)) return false;
    if (nbr > 4 && !chol_mfma_step<4>(A, nbr, piv, Ls, sfail, Ysave, Usave)) return false;
    if (nbr > 5 && !chol_mfma_step<5>(A, nbr, piv, Ls, sfail, Ysave, Usave)) return false;
    if (nbr > 6 && !chol_mfma_step<6>(A, nbr, piv, Ls, sfail, Ysave, Usave)) return false;
    if (nbr > 7 && !chol_mfma_step<7>(A, nbr, piv, Ls, sfail, Ysave, Usave)) return false;
    return true;
}

// Blocks of a candidate's factor kept by the gain kernel for the pick (FCACHE_BLOCKS of 256
// doubles, lane-major doublex4 per block): slot p < 8 holds U_pp^-1, slot 8 + C (C - 1) / 2 + I
// holds the off-diagonal block U_IC, I < C.  Only blocks with C < ceil(N_t / 16) are written.
constexpr int FCACHE_UO = 8;

// The gain kernel's factorisation: the pivots, and with fc (the candidate's factor-cache slots,
// global memory) U_pp^-1 and the off-diagonal blocks of U for the pick.
template <typename TR, typename TW>
__device__ __forceinline__ bool chol_mfma(const TR *__restrict__ Rb, int N_t, int nb, double *piv, const StepDesc &d,
                                          int64_t pofs, doublex4 (*fc)[64])
{
    const int nbr = (N_t + 15) >> 4;
    UBlocks A;
    load_upper<TR, TW>(A, Rb, nbr, nb, d, pofs);
    return chol_mfma_regs(A, nbr, piv, fc, fc ? fc + FCACHE_UO : nullptr);
}


// The inverse Z = L^-1 = U^-T of a factor held in LDS (Y: U_pp^-1, Uo: U_rp at p (p - 1) / 2 + r), by
// block columns in registers (wave w: columns w and 7 - w), Z_qq = (U_qq^-1)^T and down the column
// Z_pq = -(U_pp^-1)^T sum_{r = q}^{p-1} U_rp^T Z_rq, written to Linv in the operand order.  Blocks of
// Linv outside the factored part: zero above the diagonal, identity on the padding.
__device__ __forceinline__ void inv_from_lds(const doublex4 (*Y)[64], const doublex4 (*Uo)[64], int N_t, int N_tp,
                                             double *__restrict__ Linv)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c = lane & 15;
    const int al = a_lane<double>(lane);
    const int nbr = (N_t + 15) >> 4, nb = N_tp >> 4;
    // element (4g + r, c) of a block's transpose sits at tofs + 4r of the block (accumulator order)
    const int tofs = ((((c >> 2) << 4) + 4 * g) << 2) + (c & 3);
    // Z column q0 = w keeps blocks P = 0..7 (those with P >= q0 used), q1 = 7 - w blocks P = 4..7
    doublex4 z0[8], z1[4];
    auto zb = [&](int h, int P) -> doublex4 & { return h ? z1[(P - 4) & 3] : z0[P & 7]; };
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = h ? 7 - w : w;
        if (q >= nbr) continue;
        // Z_qq = (U_qq^-1)^T: the transpose of Y_q, read through LDS
        const double *Yq = (const double *)Y[q];
        doublex4 t;
#pragma unroll
        for (int r = 0; r < 4; ++r) t[r] = Yq[tofs + 4 * r];
#pragma unroll
        for (int P = (h ? 4 : 0); P < 8; ++P)
            if (P == q) zb(h, P) = t;
#pragma unroll
        for (int P = (h ? 4 : 0); P < 8; ++P) {
            if (P <= q || P >= nbr) continue;
            doublex4 acc{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int r = (h ? 4 : 0); r < 8; ++r) {
                if (r < q || r >= P) continue;
                const doublex4 u = Uo[P * (P - 1) / 2 + r][al];
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) acc = mfma16(u[s4], zb(h, r)[s4], acc);
            }
            const doublex4 y = Y[P][al];
            doublex4 z{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) z = mfma16(-y[s4], acc[s4], z);
            zb(h, P) = z;
        }
        // Z_Pq to Linv: element (16P + 4g + r, 16q + c) in the operand order
#pragma unroll
        for (int P = (h ? 4 : 0); P < 8; ++P) {
            if (P < q || P >= nbr) continue;
            double *dst = Linv + ((P * nb + q) << 8) + tofs;
#pragma unroll
            for (int r = 0; r < 4; ++r) dst[4 * r] = zb(h, P)[r];
        }
    }
    for (int o = tid; o < N_tp * N_tp; o += blockDim.x) {
        const int sb = o >> 8, ww = o & 255, ln = ww >> 2, reg = ww & 3;
        const int I = sb / nb, J = sb % nb;
        if (I >= nbr || J >= nbr || J > I) {
            const int k = I * 16 + (ln & 15), kp = J * 16 + ((ln >> 4) << 2) + reg;
            Linv[o] = k == kp ? 1.0 : 0.0;
        }
    }
}

// The pick's factor and inverse for N_t <= 128: the register factorisation above (keeping every
// U_pp^-1), the off-diagonal blocks of U published to LDS, then the inverse (inv_from_lds).
template <typename TR, typename TW>
__device__ __forceinline__ bool chol_inv_mfma(const TR *__restrict__ Rb, int N_t, int N_tp, double *piv,
                                              const StepDesc &d, int64_t pofs, double *__restrict__ Linv,
                                              doublex4 (*Y)[64], doublex4 (*Uo)[64])
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nbr = (N_t + 15) >> 4, nb = N_tp >> 4;
    {
        UBlocks A;
        load_upper<TR, TW>(A, Rb, nbr, nb, d, pofs);
        if (!chol_mfma_regs(A, nbr, piv, Y, nullptr)) return false;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int C = h ? 7 - w : w;
#pragma unroll
            for (int I = 0; I < (h ? 8 : 4); ++I)
                if (I < C && C < nbr) Uo[C * (C - 1) / 2 + I][lane] = ub(A, h, I);
        }
    }
    (void)tid;
    __syncthreads();
    inv_from_lds(Y, Uo, N_t, N_tp, Linv);
    return true;
}

// 1/2 sum_{j < n} ln piv[j] (n <= 256), the same value in every thread (fixed reduction order).
__device__ __forceinline__ double half_sum_log(const double *piv, int n, double *red)
{
    const int tid = threadIdx.x, lane = tid & 63;
    double v = tid < n ? log(piv[tid]) : 0.0;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[tid >> 6] = v;
    __syncthreads();
    const double t = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return 0.5 * t;
}


// Argmax of the gains (exact ties -> lowest position, NaN -> -inf) or the position of a forced
// sensor.  Returns the position (same in all threads) or -1 after setting the status word.
__device__ __forceinline__ int select_winner(const int *__restrict__ act_in, int n_act, const double *__restrict__ gains,
                             int forced, int *state, double *gain_out)
{
    __shared__ double red_g[4];
    __shared__ int red_p[4];
    const int tid = threadIdx.x;
    double bg = -INFINITY;
    int bp = 0x7fffffff;
    if (forced < 0) {
        for (int p = tid; p < n_act; p += blockDim.x) {
            double v = gains[p];
            if (isnan(v)) v = -INFINITY;
            if (v > bg || (v == bg && p < bp)) {
                bg = v;
                bp = p;
            }
        }
    } else {
        for (int p = tid; p < n_act; p += blockDim.x)
            if (act_in[p] == forced) {
                bg = 0.0;
                bp = p;
            }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double og = __shfl_xor(bg, off);
        const int op = __shfl_xor(bp, off);
        if (og > bg || (og == bg && op < bp)) {
            bg = og;
            bp = op;
        }
    }
    if ((tid & 63) == 0) {
        red_g[tid >> 6] = bg;
        red_p[tid >> 6] = bp;
    }
    __syncthreads();
    double gsel = red_g[0];
    int q = red_p[0];
    for (int w = 1; w < 4; ++w)
        if (red_g[w] > gsel || (red_g[w] == gsel && red_p[w] < q)) {
            gsel = red_g[w];
            q = red_p[w];
        }
    __syncthreads();
    if (q < 0 || q >= n_act) {  // forced index not among the remaining candidates
        if (tid == 0) state[ST_STATUS] = 1;
        return -1;
    }
    if (forced < 0 && gsel == -INFINITY) {
        if (tid == 0) state[ST_STATUS] = 2;
        return -1;
    }
    *gain_out = gsel;
    return q;
}

// ---------------------------------------------------------------------------------------------
// Kernel bodies (one work-group; early exits are uniform across it).

template <typename TR, typename TW>
__device__ void gain_regs_body(const StepDesc &d, int p)
{
    __shared__ double piv[128];
    __shared__ double red[4];
    if (d.state[ST_STATUS] != 0 || p >= d.n_act) return;
    const int i = uniform_at(d.act_in, p);
    const int64_t bs = (int64_t)d.N_tp * d.N_tp;
    doublex4(*fc)[64] = d.fcache ? (doublex4(*)[64])(d.fcache + (int64_t)i * (FCACHE_BLOCKS * 256)) : nullptr;
    const bool ok = chol_mfma<TR, TW>((const TR *)d.R + blk_index(i, i) * bs, d.N_t, d.N_tp >> 4, piv, d, i * bs, fc);
    if (!ok) {
        if (threadIdx.x == 0) d.gains[p] = -INFINITY;
        return;
    }
    const double ls = half_sum_log(piv, d.N_t, red);
    if (threadIdx.x == 0) d.gains[p] = ls - (d.noise_h ? d.noise_h[i] : d.half_noise);
}

template <typename TR, typename TW>
__device__ void pick_regs_body(const StepDesc &d)
{
    __shared__ double piv[128];
    __shared__ double red[4];
    __shared__ doublex4 Y[8][64];    // U_pp^-1
    __shared__ doublex4 Uo[28][64];  // U_rp, r < p, at p (p - 1) / 2 + r
    if (d.state[ST_STATUS] != 0) return;
    const int tid = threadIdx.x;
    double g = 0.0;
    const int pos = select_winner(d.act_in, d.n_act, d.gains, d.forced, d.state, &g);
    if (pos < 0) return;
    const int s = d.act_in[pos];
    for (int p = tid; p < d.n_act - 1; p += blockDim.x) d.act_out[p] = d.act_in[p < pos ? p : p + 1];
    if (d.fcache && d.forced < 0) {
        // the gain kernel of this step factored the winner's block: its U_pp^-1 and off-diagonal
        // blocks of U are in the factor cache, and only the inverse is left to form
        const int nbr = (d.N_t + 15) >> 4;
        const doublex4 *fc = (const doublex4 *)(d.fcache + (int64_t)s * (FCACHE_BLOCKS * 256));
        for (int o = tid; o < 36 * 64; o += blockDim.x) {
            const int blk = o >> 6, ln = o & 63;
            const bool used = blk < FCACHE_UO ? blk < nbr : (blk - FCACHE_UO) < nbr * (nbr - 1) / 2;
            if (!used) continue;
            const doublex4 v = fc[o];
            if (blk < FCACHE_UO)
                Y[blk][ln] = v;
            else
                Uo[blk - FCACHE_UO][ln] = v;
        }
        __syncthreads();
        inv_from_lds(Y, Uo, d.N_t, d.N_tp, d.Linv);
        if (tid == 0) {
            d.picks[d.step] = s;
            d.pick_gain[d.step] = g;
            d.state[ST_NPICKS] = d.step + 1;
            d.state[ST_LAST] = s;
        }
        return;
    }
    const int64_t bs = (int64_t)d.N_tp * d.N_tp;
    const bool ok = chol_inv_mfma<TR, TW>((const TR *)d.R + blk_index(s, s) * bs, d.N_t, d.N_tp, piv, d, s * bs,
                                          d.Linv, Y, Uo);
    if (!ok) {
        if (tid == 0) d.state[ST_STATUS] = 2;
        return;
    }
    const double ls = half_sum_log(piv, d.N_t, red);
    if (tid == 0) {
        d.picks[d.step] = s;
        d.pick_gain[d.step] = d.forced < 0 ? g : ls - (d.noise_h ? d.noise_h[s] : d.half_noise);
        d.state[ST_NPICKS] = d.step + 1;
        d.state[ST_LAST] = s;
    }
}

template <typename TR>
__device__ void gain_lds_body(const StepDesc &d, int p, double *lds)
{
    if (d.state[ST_STATUS] != 0 || p >= d.n_act) return;
    double *A = d.scratch ? d.scratch + (int64_t)p * tri(d.N_t) : lds;
    const int i = uniform_at(d.act_in, p);
    load_diag_block((const TR *)d.R + blk_index(i, i) * (int64_t)d.N_tp * d.N_tp, d.N_t, d.N_tp, A);
    const double ls = chol_packed(A, d.N_t);
    if (threadIdx.x == 0) d.gains[p] = (ls == -INFINITY) ? -INFINITY : ls - (d.noise_h ? d.noise_h[i] : d.half_noise);
}

template <typename TR>
__device__ void pick_lds_body(const StepDesc &d, double *lds)
{
    if (d.state[ST_STATUS] != 0) return;
    const int tid = threadIdx.x;
    double g = 0.0;
    const int pos = select_winner(d.act_in, d.n_act, d.gains, d.forced, d.state, &g);
    if (pos < 0) return;
    const int s = d.act_in[pos];
    for (int p = tid; p < d.n_act - 1; p += blockDim.x) d.act_out[p] = d.act_in[p < pos ? p : p + 1];
    double *A = d.scratch ? d.scratch : lds;
    double *X = A + tri(d.N_t);
    const int N_t = d.N_t, N_tp = d.N_tp;
    load_diag_block((const TR *)d.R + blk_index(s, s) * (int64_t)N_tp * N_tp, N_t, N_tp, A);
    const double ls = chol_packed(A, N_t);
    if (ls == -INFINITY) {
        if (tid == 0) d.state[ST_STATUS] = 2;
        return;
    }
    if (tid == 0) {
        d.picks[d.step] = s;
        d.pick_gain[d.step] = d.forced < 0 ? g : ls - (d.noise_h ? d.noise_h[s] : d.half_noise);
        d.state[ST_NPICKS] = d.step + 1;
        d.state[ST_LAST] = s;
    }
    tri_inverse(A, X, N_t);
    const int nb = N_tp >> 4;
    for (int o = tid; o < N_tp * N_tp; o += blockDim.x) {
        const int sb = o >> 8, w = o & 255, lane = w >> 2, reg = w & 3;
        const int k = (sb / nb) * 16 + (lane & 15);
        const int kp = (sb % nb) * 16 + ((lane >> 4) << 2) + reg;
        double v;
        if (k < N_t && kp < N_t)
            v = kp <= k ? X[tri(k) + kp] : 0.0;
        else
            v = (k == kp) ? 1.0 : 0.0;
        d.Linv[o] = v;
    }
}

// ---------------------------------------------------------------------------------------------
// Blocked factorisation in global scratch for 128 < N_t <= 16 BLK_MAX_NB (one work-group per
// block; the block is too large for registers or LDS).  The same upper form as chol_mfma: the
// upper 16x16 blocks (I, C), I <= C < nbr, in FP64 accumulator order, block (I, C) at
// S + 256 (C (C + 1) / 2 + I).  Step p: wave p % 4 factors A_pp in-wave (chol16_inv) and
// publishes U_pp^-1; the row blocks U_pC = U_pp^-T A_pC are formed and published through LDS;
// the trailing blocks A_IC -= U_pI^T U_pC are updated in place.  Traffic per block: about
// nbr^3 / 3 block reads and writes (13 MB at N_t = 420), against nbr^3 16^3 / 6 element
// reads and writes for an unblocked factorisation.

__device__ __forceinline__ int64_t ublk(int I, int C) { return ((int64_t)C * (C + 1) / 2 + I) << 8; }

// Copy the candidate's diagonal block of R (lower blocks, TR) into S as upper FP64 blocks.
// With held W blocks (slots 0 .. d.nheld-1 at candidate offset pofs: FP64, FP32 or BF16 hi + lo
// parts) their products P_I P_C^T are subtracted, and with d.wb the corrected block is written
// back to R (left-looking: the newest block column applied to the diagonal block in place).
template <typename TR, typename TW>
__device__ void load_upper_global(const TR *__restrict__ Rb, int nb, int nbr, double *__restrict__ S,
                                  const StepDesc &d, int64_t pofs)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
    const int tofs = ((((c >> 2) << 4) + 4 * g) << 2) + (c & 3);
    for (int C = w; C < nbr; C += 4)
        for (int I = 0; I <= C; ++I) {
            const TR *blk = Rb + ((C * nb + I) << 8) + tofs;
            doublex4 v;
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = (double)blk[4 * r];
            for (int hp = 0; hp < d.nheld; ++hp) {
                const TW *Pw = (const TW *)d.W + hp * d.wslot + pofs;
                const TW *Pw2 = d.W2 ? (const TW *)d.W2 + hp * d.wslot + pofs : nullptr;
                const auto q = HeldProd<TW>::run(Pw, Pw2, I, C, nb, nbr, lane);
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] -= (double)q[r];
            }
            if (d.wb && d.nheld > 0) {
                TR *wblk = const_cast<TR *>(blk);
#pragma unroll
                for (int r = 0; r < 4; ++r) wblk[4 * r] = (TR)v[r];
            }
            st4(S + ublk(I, C) + lane * 4, v);
        }
}

// The factorisation of the upper blocks in S (whole work-group).  Ub: LDS, (nbr + 1) x 64
// doublex4 (row blocks of the step, then U_pp^-1).  With Yg, U_pp^-1 of every diagonal block is
// also kept there (block p at Yg + 256 p).  Pivots to piv (16 nbr).  Returns false (uniformly) at
// a pivot that is not > 0 or not finite.
__device__ bool chol_blocked(double *__restrict__ S, int nbr, double *piv, double *__restrict__ Yg,
                             doublex4 *Ub, int *sfail)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int al = a_lane<double>(lane);
    doublex4 *Yl = Ub + nbr * 64;
    for (int p = 0; p < nbr; ++p) {
        if (w == (p & 3)) {
            const bool ok = chol16_inv(ld4(S + ublk(p, p) + lane * 4), (double *)Yl, piv + 16 * p);
            if (lane == 0) *sfail = ok ? 0 : 1;
        }
        __syncthreads();
        if (*sfail) return false;
        const doublex4 y = Yl[al];
        if (Yg && w == 0) st4(Yg + ((int64_t)p << 8) + lane * 4, Yl[lane]);
        for (int C = p + 1 + w; C < nbr; C += 4) {
            const doublex4 a = ld4(S + ublk(p, C) + lane * 4);
            doublex4 acc{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) acc = mfma16(y[s4], a[s4], acc);
            st4(S + ublk(p, C) + lane * 4, acc);
            Ub[C * 64 + lane] = acc;
        }
        __syncthreads();
        for (int C = p + 1 + w; C < nbr; C += 4) {
            const doublex4 b = Ub[C * 64 + lane];
            for (int I = p + 1; I <= C; ++I) {
                const doublex4 u = Ub[I * 64 + al];
                doublex4 acc = ld4(S + ublk(I, C) + lane * 4);
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) acc = mfma16(-u[s4], b[s4], acc);
                st4(S + ublk(I, C) + lane * 4, acc);
            }
        }
        // the next step's owner reads its updated diagonal block, and Ub is rewritten
        __syncthreads();
    }
    return true;
}

// 1/2 sum_{j < n} ln piv[j] for any n (whole work-group, fixed reduction order).
__device__ double half_sum_log_any(const double *piv, int n, double *red)
{
    const int tid = threadIdx.x, lane = tid & 63;
    double v = 0.0;
    for (int t = tid; t < n; t += blockDim.x) v += log(piv[t]);
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[tid >> 6] = v;
    __syncthreads();
    const double t = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return 0.5 * t;
}

constexpr int BLK_MAX_NB = BLK_MAX_NTP / 16;

// Dynamic LDS of the blocked kernels: Ub ((nbr + 1) blocks) and the pivots.
__host__ __device__ inline size_t blocked_lds_bytes(int nbr)
{
    return (size_t)(nbr + 1) * 64 * sizeof(doublex4) + (size_t)16 * nbr * sizeof(double);
}

template <typename TR, typename TW>
__device__ void gain_blocked_body(const StepDesc &d, int p, unsigned char *dyn)
{
    __shared__ double red[4];
    __shared__ int sfail;
    if (d.state[ST_STATUS] != 0 || p >= d.n_act) return;
    const int nbr = d.N_tp >> 4;
    doublex4 *Ub = (doublex4 *)dyn;
    double *piv = (double *)(Ub + (nbr + 1) * 64);
    const int64_t nblk = (int64_t)nbr * (nbr + 1) / 2;
    double *S = d.scratch + p * (nblk << 8);
    const int i = uniform_at(d.act_in, p);
    const int64_t bs = (int64_t)d.N_tp * d.N_tp;
    load_upper_global<TR, TW>((const TR *)d.R + blk_index(i, i) * bs, nbr, nbr, S, d, i * bs);
    __syncthreads();
    if (!chol_blocked(S, nbr, piv, nullptr, Ub, &sfail)) {
        if (threadIdx.x == 0) d.gains[p] = -INFINITY;
        return;
    }
    const double ls = half_sum_log_any(piv, d.N_t, red);
    if (threadIdx.x == 0) d.gains[p] = ls - (d.noise_h ? d.noise_h[i] : d.half_noise);
}

// Pick: the winner's factorisation as in the gain kernel, then Z = L^-1 = U^-T by block
// columns q (wave q % 4, no barriers): Z_qq = (U_qq^-1)^T and, down the column,
// Z_pq = -(U_pp^-1)^T sum_{r = q}^{p-1} U_rp^T Z_rq; Z is written to Linv in the operand order.
// Scratch: S (nblk blocks), U_pp^-1 (nbr blocks), Z (nblk lower blocks, (p, q) at p(p+1)/2 + q).
template <typename TR, typename TW>
__device__ void pick_blocked_body(const StepDesc &d, unsigned char *dyn)
{
    __shared__ double red[4];
    __shared__ int sfail;
    if (d.state[ST_STATUS] != 0) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c = lane & 15;
    const int al = a_lane<double>(lane);
    double g_sel = 0.0;
    const int pos = select_winner(d.act_in, d.n_act, d.gains, d.forced, d.state, &g_sel);
    if (pos < 0) return;
    const int s = d.act_in[pos];
    for (int q = tid; q < d.n_act - 1; q += blockDim.x) d.act_out[q] = d.act_in[q < pos ? q : q + 1];
    const int nbr = d.N_tp >> 4;
    doublex4 *Ub = (doublex4 *)dyn;
    double *piv = (double *)(Ub + (nbr + 1) * 64);
    const int64_t nblk = (int64_t)nbr * (nbr + 1) / 2;
    double *S = d.scratch, *Yg = S + (nblk << 8), *Z = Yg + ((int64_t)nbr << 8);
    const int64_t bs = (int64_t)d.N_tp * d.N_tp;
    load_upper_global<TR, TW>((const TR *)d.R + blk_index(s, s) * bs, nbr, nbr, S, d, s * bs);
    __syncthreads();
    if (!chol_blocked(S, nbr, piv, Yg, Ub, &sfail)) {
        if (tid == 0) d.state[ST_STATUS] = 2;
        return;
    }
    const double ls = half_sum_log_any(piv, d.N_t, red);
    if (tid == 0) {
        d.picks[d.step] = s;
        d.pick_gain[d.step] = d.forced < 0 ? g_sel : ls - (d.noise_h ? d.noise_h[s] : d.half_noise);
        d.state[ST_NPICKS] = d.step + 1;
        d.state[ST_LAST] = s;
    }
    // element (4g + r, c) of a block's transpose sits at tofs + 4r of the block
    const int tofs = ((((c >> 2) << 4) + 4 * g) << 2) + (c & 3);
    auto zblk = [](int P, int Q) -> int64_t { return ((int64_t)P * (P + 1) / 2 + Q) << 8; };
    for (int q = w; q < nbr; q += 4) {
        doublex4 zqq;
#pragma unroll
        for (int r = 0; r < 4; ++r) zqq[r] = Yg[((int64_t)q << 8) + tofs + 4 * r];
        st4(Z + zblk(q, q) + lane * 4, zqq);
        for (int P = q + 1; P < nbr; ++P) {
            doublex4 t{0.0, 0.0, 0.0, 0.0};
            for (int r = q; r < P; ++r) {
                const doublex4 u = ld4(S + ublk(r, P) + al * 4);
                const doublex4 z = ld4(Z + zblk(r, q) + lane * 4);
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) t = mfma16(u[s4], z[s4], t);
            }
            const doublex4 y = ld4(Yg + ((int64_t)P << 8) + al * 4);
            doublex4 zpq{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) zpq = mfma16(-y[s4], t[s4], zpq);
            st4(Z + zblk(P, q) + lane * 4, zpq);
        }
    }
    __syncthreads();
    // Linv: lower blocks (P, Q) from Z, the operand order; blocks above the diagonal are zero
    const int nb = nbr;
    for (int b = w; b < nbr * nbr; b += 4) {
        const int P = b / nbr, Q = b - P * nbr;
        doublex4 v{0.0, 0.0, 0.0, 0.0};
        if (Q <= P) v = ld4(Z + zblk(P, Q) + lane * 4);
        // element (16P + 4g + r, 16Q + c) of L^-1 -> operand position (t, k)
        double *dst = d.Linv + ((int64_t)(P * nb + Q) << 8) + tofs;
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[4 * r] = v[r];
    }
}

// ---------------------------------------------------------------------------------------------
// Kernels: single instance (descriptor by value) and batched (descriptor array).

template <typename TR, typename TW>
__global__ void __launch_bounds__(256, 3) gain_regs_kernel(StepDesc d)
{
    gain_regs_body<TR, TW>(d, blockIdx.x);
}

template <typename TR, typename TW>
__global__ void __launch_bounds__(256, 3) gain_regs_batched(const StepDesc *__restrict__ ds, int n)
{
    const int i = find_instance(ds, n, blockIdx.x);
    if (i < 0) return;
    const StepDesc d = ds[i];
    gain_regs_body<TR, TW>(d, (int)(blockIdx.x - d.item0));
}

// One work-group per pick: 512 registers per lane hold the block and its inverse.
template <typename TR, typename TW>
__global__ void __launch_bounds__(256, 1) pick_regs_kernel(StepDesc d)
{
    pick_regs_body<TR, TW>(d);
}

template <typename TR, typename TW>
__global__ void __launch_bounds__(256, 1) pick_regs_batched(const StepDesc *__restrict__ ds, int n)
{
    const int i = find_instance(ds, n, blockIdx.x);
    if (i < 0) return;
    const StepDesc d = ds[i];
    pick_regs_body<TR, TW>(d);
}

template <typename TR, typename TW>
__global__ void __launch_bounds__(256) gain_blocked_kernel(StepDesc d)
{
    extern __shared__ double dyn[];
    gain_blocked_body<TR, TW>(d, blockIdx.x, (unsigned char *)dyn);
}

template <typename TR, typename TW>
__global__ void __launch_bounds__(256) pick_blocked_kernel(StepDesc d)
{
    extern __shared__ double dyn[];
    pick_blocked_body<TR, TW>(d, (unsigned char *)dyn);
}

template <typename TR>
__global__ void __launch_bounds__(256) gain_lds_kernel(StepDesc d)
{
    extern __shared__ double dyn[];
    gain_lds_body<TR>(d, blockIdx.x, dyn);
}

template <typename TR>
__global__ void __launch_bounds__(256) pick_lds_kernel(StepDesc d)
{
    extern __shared__ double dyn[];
    pick_lds_body<TR>(d, dyn);
}

// ---------------------------------------------------------------------------------------------
// Launchers.

static int g_max_lds = -1;
static int max_lds()
{
    if (g_max_lds < 0) {
        int dev = 0, v = 65536;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess)
            g_max_lds = v;
        else
            g_max_lds = 65536;
    }
    return g_max_lds;
}

size_t gain_scratch_doubles(int N_t, int N_tp, int N_c)
{
    if (N_t <= REGS_MAX_NT) return 0;
    const size_t nbr = N_tp / 16;
    if (nbr <= (size_t)BLK_MAX_NB) return nbr * (nbr + 1) / 2 * 256 * N_c;
    return gain_lds_bytes(N_t) ? 0 : (size_t)N_t * (N_t + 1) / 2 * N_c;
}

size_t pick_scratch_doubles(int N_t, int N_tp)
{
    if (N_t <= REGS_MAX_NT) return 0;
    const size_t nbr = N_tp / 16;
    if (nbr <= (size_t)BLK_MAX_NB) return (nbr * (nbr + 1) + nbr) * 256;
    return pick_lds_bytes(N_t) ? 0 : (size_t)N_t * (N_t + 1);
}

size_t gain_lds_bytes(int N_t)
{
    const size_t b = sizeof(double) * (size_t)N_t * (N_t + 1) / 2;
    return b <= (size_t)max_lds() ? b : 0;
}
size_t pick_lds_bytes(int N_t)
{
    const size_t b = 2 * sizeof(double) * (size_t)N_t * (N_t + 1) / 2;
    return b <= (size_t)max_lds() - 256 ? b : 0;
}

template <typename K>
static void allow_lds(K kernel, size_t bytes)
{
    if (bytes > 65536) (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// The LDS factorisation kernels (N_t > REGS_MAX_NT) take no held W.
template <typename TR, typename TW>
static hipError_t launch_gain_t(const StepDesc &d, hipStream_t s)
{
    if (d.n_act <= 0) return hipSuccess;
    if (d.N_t <= REGS_MAX_NT) {
        hipLaunchKernelGGL((gain_regs_kernel<TR, TW>), dim3(d.n_act), dim3(256), 0, s, d);
    } else if (d.N_tp <= 16 * BLK_MAX_NB) {
        if (!d.scratch) return hipErrorInvalidValue;
        const size_t lds = blocked_lds_bytes(d.N_tp >> 4);
        allow_lds(gain_blocked_kernel<TR, TW>, lds);
        hipLaunchKernelGGL((gain_blocked_kernel<TR, TW>), dim3(d.n_act), dim3(256), lds, s, d);
    } else {
        if (d.nheld) return hipErrorInvalidValue;
        const size_t lds = d.scratch ? 0 : gain_lds_bytes(d.N_t);
        allow_lds(gain_lds_kernel<TR>, lds);
        hipLaunchKernelGGL(gain_lds_kernel<TR>, dim3(d.n_act), dim3(256), lds, s, d);
    }
    return hipGetLastError();
}

template <typename TR, typename TW>
static hipError_t launch_pick_t(const StepDesc &d, hipStream_t s)
{
    if (d.N_t <= REGS_MAX_NT) {
        hipLaunchKernelGGL((pick_regs_kernel<TR, TW>), dim3(1), dim3(256), 0, s, d);
    } else if (d.N_tp <= 16 * BLK_MAX_NB) {
        // held block columns: as in the gain kernel
        if (!d.scratch) return hipErrorInvalidValue;
        const size_t lds = blocked_lds_bytes(d.N_tp >> 4);
        allow_lds(pick_blocked_kernel<TR, TW>, lds);
        hipLaunchKernelGGL((pick_blocked_kernel<TR, TW>), dim3(1), dim3(256), lds, s, d);
    } else {
        if (d.nheld) return hipErrorInvalidValue;
        const size_t lds = d.scratch ? 0 : pick_lds_bytes(d.N_t);
        allow_lds(pick_lds_kernel<TR>, lds);
        hipLaunchKernelGGL(pick_lds_kernel<TR>, dim3(1), dim3(256), lds, s, d);
    }
    return hipGetLastError();
}

hipError_t launch_gain(const StepDesc &d, int rtype, int wtype, hipStream_t s)
{
    if (rtype == R_F64 && wtype == W_F64) return launch_gain_t<double, double>(d, s);
    if (rtype == R_F32 && wtype == W_F32) return launch_gain_t<float, float>(d, s);
    if (rtype == R_F32 && wtype == W_BF16X3) return launch_gain_t<float, unsigned short>(d, s);
    return hipErrorInvalidValue;
}

hipError_t launch_pick(const StepDesc &d, int rtype, int wtype, hipStream_t s)
{
    if (rtype == R_F64 && wtype == W_F64) return launch_pick_t<double, double>(d, s);
    if (rtype == R_F32 && wtype == W_F32) return launch_pick_t<float, float>(d, s);
    if (rtype == R_F32 && wtype == W_BF16X3) return launch_pick_t<float, unsigned short>(d, s);
    return hipErrorInvalidValue;
}

template <typename TR, typename TW>
static void gain_batched_t(const StepDesc *descs, int n, int64_t total, hipStream_t s)
{
    hipLaunchKernelGGL((gain_regs_batched<TR, TW>), dim3((unsigned)total), dim3(256), 0, s, descs, n);
}

hipError_t launch_gain_batched(const StepDesc *descs, int n, int64_t total, int rtype, int wtype, hipStream_t s)
{
    if (n <= 0 || total <= 0) return hipSuccess;
    if (rtype == R_F64 && wtype == W_F64)
        gain_batched_t<double, double>(descs, n, total, s);
    else if (rtype == R_F32 && wtype == W_F32)
        gain_batched_t<float, float>(descs, n, total, s);
    else if (rtype == R_F32 && wtype == W_BF16X3)
        gain_batched_t<float, unsigned short>(descs, n, total, s);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename TR, typename TW>
static void pick_batched_t(const StepDesc *descs, int n, size_t, hipStream_t s)
{
    hipLaunchKernelGGL((pick_regs_batched<TR, TW>), dim3(n), dim3(256), 0, s, descs, n);
}

hipError_t launch_pick_batched(const StepDesc *descs, int n, int max_Nt, int rtype, int wtype, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * (size_t)max_Nt * (max_Nt + 1) / 2;
    if (rtype == R_F64 && wtype == W_F64)
        pick_batched_t<double, double>(descs, n, lds, s);
    else if (rtype == R_F32 && wtype == W_F32)
        pick_batched_t<float, float>(descs, n, lds, s);
    else if (rtype == R_F32 && wtype == W_BF16X3)
        pick_batched_t<float, unsigned short>(descs, n, lds, s);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace oed
