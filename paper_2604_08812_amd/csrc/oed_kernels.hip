// HIP kernels (gfx950) of the greedy D-optimal sensor selection.
//
// One greedy step (Sec. III-D; paper's left-looking Algorithm 1 reordered into
// the equivalent right-looking block update, same Schur blocks):
//   gain_kernel  : for every remaining candidate j, an FP64 Cholesky of the
//                  diagonal block R_jj (= M_j of Algorithm 1) and its gain
//                  1/2 logdet(sigma^-2 R_jj) = sum ln L_tt - (N_t/2) ln sigma^2.
//   pick_kernel  : argmax of the gains (exact ties -> lowest index; NaN counts
//                  as -inf), removal of the winner s from the active list, FP64
//                  Cholesky L_s of R_ss and its inverse L_s^-1.
//   trsm_kernel  : W_i = C_i L_s^-T for every remaining i, C_i the (i, s) block
//                  of R (the new block row of the factor in Algorithm 1), on
//                  FP64 MFMA, stored in the element type of the downdate.
//   syrk_kernel  : R_IJ -= W_I W_J^T on the lower triangle of the remaining
//                  rows (the Schur-complement update that turns K_ss into M_s).
// See oed_internal.h for the storage layouts.
#include "oed_internal.h"

#include <math.h>

namespace oed {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T>
struct V4;
template <>
struct V4<float> {
    typedef floatx4 type;
};
template <>
struct V4<double> {
    typedef doublex4 type;
};

__device__ __forceinline__ floatx4 mfma16(float a, float b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 mfma16(double a, double b, doublex4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Lane whose stored operand row the A operand of `lane` must carry.  The FP32 16x16x4 MFMA
// returns output row m of a 16x16 block at lane 16*(m/4) + n, register m%4; the FP64 one at
// lane 16*(m%4) + n, register m/4.  Feeding the FP64 A operand the rows in the order
// pi(r) = 4*(r%4) + r/4 (an involution) makes both land in the same accumulator storage order.
template <typename T>
__device__ __forceinline__ int a_lane(int lane)
{
    return lane;
}
template <>
__device__ __forceinline__ int a_lane<double>(int lane)
{
    return (lane & 48) | ((lane & 3) << 2) | ((lane & 15) >> 2);
}

template <typename T>
__device__ __forceinline__ typename V4<T>::type ld4(const T *p)
{
    return *reinterpret_cast<const typename V4<T>::type *>(p);
}
template <typename T>
__device__ __forceinline__ void st4(T *p, typename V4<T>::type v)
{
    *reinterpret_cast<typename V4<T>::type *>(p) = v;
}

// Row of the packed lower triangle: element (t, u), u <= t, at tri(t) + u.
__device__ __forceinline__ int tri(int t) { return t * (t + 1) / 2; }

// Largest i with i(i+1)/2 <= b.
__device__ __forceinline__ int64_t tri_row(int64_t b)
{
    int64_t i = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= b) ++i;
    while (i * (i + 1) / 2 > b) --i;
    return i;
}

// ---------------------------------------------------------------------------------------------
// Pack the candidate part of K's lower triangle into R (padded, packed, accumulator order).
// One thread per (block, sub-block, lane): it writes the lane's 4 elements with one vector store.
template <typename TK, typename TR>
__global__ void __launch_bounds__(256) pack_kernel(const TK *__restrict__ K, int64_t ld, int N_t, int N_tp,
                                                   const int *__restrict__ cmap, int64_t nblocks,
                                                   TR *__restrict__ R)
{
    const int nb = N_tp >> 4;
    const int64_t per_block = (int64_t)nb * nb * 64;
    const int64_t total = nblocks * per_block;
    const int64_t bs = (int64_t)N_tp * N_tp;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = e / per_block;
        const int rem = (int)(e - b * per_block);
        const int sb = rem >> 6, lane = rem & 63;
        const int64_t i = tri_row(b), j = b - i * (i + 1) / 2;
        const int tb = sb / nb, ub = sb - tb * nb;
        const int u = ub * 16 + (lane & 15);
        const int t0 = tb * 16 + ((lane >> 4) << 2);
        const int64_t ci = cmap[i], cj = cmap[j];
        typename V4<TR>::type v;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int t = t0 + r;
            double x;
            if (t < N_t && u < N_t) {
                int64_t row, col;
                if (i != j) {
                    row = ci * N_t + t;
                    col = cj * N_t + u;
                } else {
                    row = ci * N_t + (t >= u ? t : u);
                    col = ci * N_t + (t >= u ? u : t);
                }
                x = (double)K[row * ld + col];
            } else {
                x = (i == j && t == u) ? 1.0 : 0.0;
            }
            v[r] = (TR)x;
        }
        st4(R + b * bs + ((int64_t)sb << 8) + lane * 4, v);
    }
}

__global__ void init_state_kernel(int *act, int n, int *state)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) act[p] = p;
    if (p < ST_WORDS) state[p] = 0;
}

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
// Gains of all remaining candidates: one work-group per candidate.
template <typename TR>
__global__ void __launch_bounds__(256) gain_kernel(const TR *__restrict__ R, const int *__restrict__ act,
                                                   int n_act, int N_t, int N_tp, double half_noise,
                                                   double *__restrict__ gains, const int *__restrict__ state,
                                                   double *scratch)
{
    extern __shared__ double lds[];
    if (state[ST_STATUS] != 0) return;
    const int p = blockIdx.x;
    if (p >= n_act) return;
    double *A = scratch ? scratch + (int64_t)p * tri(N_t) : lds;
    const int i = act[p];
    const int64_t bs = (int64_t)N_tp * N_tp;
    load_diag_block(R + blk_index(i, i) * bs, N_t, N_tp, A);
    const double ls = chol_packed(A, N_t);
    if (threadIdx.x == 0) gains[p] = (ls == -INFINITY) ? -INFINITY : ls - half_noise;
}

// ---------------------------------------------------------------------------------------------
// Pick: argmax (or a forced index), active-list update, FP64 factor of the winner and its inverse.
template <typename TR>
__global__ void __launch_bounds__(256) pick_kernel(const TR *__restrict__ R, const int *__restrict__ act_in,
                                                   int *__restrict__ act_out, int n_act,
                                                   const double *__restrict__ gains, int N_t, int N_tp,
                                                   double half_noise, int step, int forced, int *picks,
                                                   double *pick_gain, int *state, double *__restrict__ Linv,
                                                   double *scratch)
{
    extern __shared__ double lds[];
    __shared__ double red_g[4];
    __shared__ int red_p[4];
    __shared__ int s_pos;
    __shared__ double s_gain;
    if (state[ST_STATUS] != 0) return;
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
    if (tid == 0) {
        double g = red_g[0];
        int q = red_p[0];
        for (int w = 1; w < 4; ++w)
            if (red_g[w] > g || (red_g[w] == g && red_p[w] < q)) {
                g = red_g[w];
                q = red_p[w];
            }
        s_pos = q;
        s_gain = g;
    }
    __syncthreads();
    const int pos = s_pos;
    if (pos < 0 || pos >= n_act) {  // forced index not among the remaining candidates
        if (tid == 0) state[ST_STATUS] = 1;
        return;
    }
    if (forced < 0 && s_gain == -INFINITY) {
        if (tid == 0) state[ST_STATUS] = 2;
        return;
    }
    const int s = act_in[pos];
    for (int p = tid; p < n_act - 1; p += blockDim.x) act_out[p] = act_in[p < pos ? p : p + 1];

    double *A = scratch ? scratch : lds;
    double *X = A + tri(N_t);
    const int64_t bs = (int64_t)N_tp * N_tp;
    load_diag_block(R + blk_index(s, s) * bs, N_t, N_tp, A);
    const double ls = chol_packed(A, N_t);
    if (ls == -INFINITY) {
        if (tid == 0) state[ST_STATUS] = 2;
        return;
    }
    if (tid == 0) {
        picks[step] = s;
        pick_gain[step] = forced < 0 ? s_gain : ls - half_noise;
        state[ST_NPICKS] = step + 1;
        state[ST_LAST] = s;
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
        Linv[o] = v;
    }
}

// ---------------------------------------------------------------------------------------------
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

template <typename TR, typename TW>
__global__ void __launch_bounds__(256) trsm_kernel(const TR *__restrict__ R, const int *__restrict__ act, int n_act,
                                                   const int *__restrict__ state, const double *__restrict__ Linv,
                                                   int N_tp, TW *__restrict__ W)
{
    if (state[ST_STATUS] != 0) return;
    const int p = blockIdx.x;
    if (p >= n_act) return;
    const int i = act[p], s = state[ST_LAST];
    const int nb = N_tp >> 4;
    const int64_t bs = (int64_t)N_tp * N_tp;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, l16 = lane & 15;
    const int alane = a_lane<double>(lane);
    const bool below = i > s;
    const TR *Cb = R + blk_index(below ? i : s, below ? s : i) * bs;
    TW *Wi = W + (int64_t)i * bs;
    for (int tb = wave; tb < nb; tb += 4) {
        for (int kg = 0; kg < nb; kg += 8) {
            const int kend = min(nb, kg + 8);
            doublex4 acc[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) acc[c] = doublex4{0.0, 0.0, 0.0, 0.0};
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
                if (kc < kend) store_w(Wi, ((int64_t)(tb * nb + kc) << 8) + lane * 4, acc[c]);
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------
// Downdate R_IJ -= W_I W_J^T over 128 x 128 tiles of the remaining rows, lower triangle only.
// Four waves per tile, each a 64 x 64 quarter = 4 x 4 MFMA 16x16 blocks.  Tiles are handed
// out XCD by XCD (work-group id mod 8 is the XCD) in contiguous chunks, so the row panel of
// W that neighbouring tiles share stays in that XCD's L2.
template <typename T>
__global__ void __launch_bounds__(256) syrk_kernel(T *__restrict__ R, const T *__restrict__ W,
                                                   const int *__restrict__ act, int n_act, int N_tp,
                                                   int64_t ntiles, int64_t per_xcd, const int *__restrict__ state)
{
    typedef typename V4<T>::type vec;
    if (state[ST_STATUS] != 0) return;
    const int64_t wg = blockIdx.x;
    const int64_t tile = (wg & 7) * per_xcd + (wg >> 3);
    if (tile >= ntiles) return;
    const int64_t P = tri_row(tile), Q = tile - P * (P + 1) / 2;
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
        for (int c = 0; c < 4; ++c) any |= vr[b] && vc[c] && ia[b] >= ja[c];
    if (!any) return;

    vec acc[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (vr[b] && vc[c] && ia[b] >= ja[c])
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
            if (vr[b] && vc[c] && ia[b] >= ja[c])
                st4(R + blk_index(ia[b], ja[c]) * bs + ((ta[b] * nb + tc[c]) << 8) + lane * 4, acc[b][c]);
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

hipError_t launch_pack(const void *K, int kdtype, int64_t ld, int N_t, int N_tp, const int *cmap, int N_c,
                       void *R, int rtype, hipStream_t s)
{
    const int64_t nblocks = (int64_t)N_c * (N_c + 1) / 2;
    const int64_t threads = nblocks * (N_tp / 16) * (N_tp / 16) * 64;
    const int64_t grid = std::min<int64_t>((threads + 255) / 256, 1 << 20);
    if (kdtype == 0 && rtype == R_F64)
        hipLaunchKernelGGL((pack_kernel<double, double>), dim3(grid), dim3(256), 0, s, (const double *)K, ld, N_t, N_tp,
                           cmap, nblocks, (double *)R);
    else if (kdtype == 0 && rtype == R_F32)
        hipLaunchKernelGGL((pack_kernel<double, float>), dim3(grid), dim3(256), 0, s, (const double *)K, ld, N_t, N_tp,
                           cmap, nblocks, (float *)R);
    else if (kdtype == 1 && rtype == R_F64)
        hipLaunchKernelGGL((pack_kernel<float, double>), dim3(grid), dim3(256), 0, s, (const float *)K, ld, N_t, N_tp,
                           cmap, nblocks, (double *)R);
    else
        hipLaunchKernelGGL((pack_kernel<float, float>), dim3(grid), dim3(256), 0, s, (const float *)K, ld, N_t, N_tp,
                           cmap, nblocks, (float *)R);
    return hipGetLastError();
}

hipError_t launch_init_state(int *act, int n, double *pick_gain, int *picks, int *state, hipStream_t s)
{
    (void)pick_gain;
    (void)picks;
    const int threads = std::max(n, (int)ST_WORDS);
    hipLaunchKernelGGL(init_state_kernel, dim3((threads + 255) / 256), dim3(256), 0, s, act, n, state);
    return hipGetLastError();
}

hipError_t launch_gain(const void *R, int rtype, const int *act, int n_act, int N_t, int N_tp, double half_noise,
                       double *gains, const int *state, double *scratch, hipStream_t s)
{
    if (n_act <= 0) return hipSuccess;
    const size_t lds = scratch ? 0 : gain_lds_bytes(N_t);
    if (rtype == R_F64) {
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)gain_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(gain_kernel<double>, dim3(n_act), dim3(256), lds, s, (const double *)R, act, n_act, N_t,
                           N_tp, half_noise, gains, state, scratch);
    } else {
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)gain_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(gain_kernel<float>, dim3(n_act), dim3(256), lds, s, (const float *)R, act, n_act, N_t,
                           N_tp, half_noise, gains, state, scratch);
    }
    return hipGetLastError();
}

hipError_t launch_pick(const void *R, int rtype, const int *act_in, int *act_out, int n_act, const double *gains,
                       int N_t, int N_tp, double half_noise, int step, int forced, int *picks, double *pick_gain,
                       int *state, double *Linv, double *scratch, hipStream_t s)
{
    const size_t lds = scratch ? 0 : pick_lds_bytes(N_t);
    if (rtype == R_F64) {
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)pick_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(pick_kernel<double>, dim3(1), dim3(256), lds, s, (const double *)R, act_in, act_out, n_act,
                           gains, N_t, N_tp, half_noise, step, forced, picks, pick_gain, state, Linv, scratch);
    } else {
        if (lds > 65536)
            (void)hipFuncSetAttribute((const void *)pick_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(pick_kernel<float>, dim3(1), dim3(256), lds, s, (const float *)R, act_in, act_out, n_act,
                           gains, N_t, N_tp, half_noise, step, forced, picks, pick_gain, state, Linv, scratch);
    }
    return hipGetLastError();
}

hipError_t launch_trsm(const void *R, int rtype, const int *act, int n_act, const int *state, const double *Linv,
                       int N_tp, void *W, int wtype, hipStream_t s)
{
    if (n_act <= 0) return hipSuccess;
    if (rtype == R_F64 && wtype == W_F64)
        hipLaunchKernelGGL((trsm_kernel<double, double>), dim3(n_act), dim3(256), 0, s, (const double *)R, act, n_act,
                           state, Linv, N_tp, (double *)W);
    else if (rtype == R_F32 && wtype == W_F32)
        hipLaunchKernelGGL((trsm_kernel<float, float>), dim3(n_act), dim3(256), 0, s, (const float *)R, act, n_act,
                           state, Linv, N_tp, (float *)W);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_syrk(void *R, int rtype, const void *W, int wtype, const int *act, int n_act, int N_tp,
                       const int *state, hipStream_t s)
{
    if (n_act <= 0) return hipSuccess;
    const int64_t rows = (int64_t)n_act * N_tp;
    const int64_t T = (rows + 127) / 128;
    const int64_t ntiles = T * (T + 1) / 2;
    const int64_t per_xcd = (ntiles + 7) / 8;
    const int64_t grid = per_xcd * 8;
    if (rtype == R_F64 && wtype == W_F64)
        hipLaunchKernelGGL(syrk_kernel<double>, dim3(grid), dim3(256), 0, s, (double *)R, (const double *)W, act, n_act,
                           N_tp, ntiles, per_xcd, state);
    else if (rtype == R_F32 && wtype == W_F32)
        hipLaunchKernelGGL(syrk_kernel<float>, dim3(grid), dim3(256), 0, s, (float *)R, (const float *)W, act, n_act,
                           N_tp, ntiles, per_xcd, state);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace oed
