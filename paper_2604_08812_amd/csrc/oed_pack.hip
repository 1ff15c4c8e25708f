// Packing of the caller's K into the working copy R, and per-selection state reset.
#include <algorithm>

#include "oed_device.h"

namespace oed {

// ---------------------------------------------------------------------------------------------
// Pack the candidate part of K's lower triangle into R (padded, packed, accumulator order).
// Candidate i is sensor cmap[i]; the map need not be increasing (blocks above K's diagonal are
// read as the transpose of the block below it).
// One thread per (block, sub-block, lane): it writes the lane's 4 elements with one vector store.
// Blocks b0 .. b0 + nblocks - 1 of R are packed; K's row r is read at K + (r - row0) ld.
template <typename TK, typename TR>
__global__ void __launch_bounds__(256) pack_kernel(const TK *__restrict__ K, int64_t ld, int64_t row0, int N_t,
                                                   int N_tp, const int *__restrict__ cmap, int64_t b0,
                                                   int64_t nblocks, TR *__restrict__ R)
{
    const int nb = N_tp >> 4;
    const int64_t per_block = (int64_t)nb * nb * 64;
    const int64_t total = nblocks * per_block;
    const int64_t bs = (int64_t)N_tp * N_tp;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = b0 + e / per_block;
        const int rem = (int)(e - (b - b0) * per_block);
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
                if (ci > cj) {
                    row = ci * N_t + t;
                    col = cj * N_t + u;
                } else if (ci < cj) {  // block (ci, cj) lies above K's diagonal: its transpose
                    row = cj * N_t + u;
                    col = ci * N_t + t;
                } else {
                    row = ci * N_t + (t >= u ? t : u);
                    col = ci * N_t + (t >= u ? u : t);
                }
                x = (double)K[(row - row0) * ld + col];
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

hipError_t launch_pack_range(const void *K, int kdtype, int64_t ld, int64_t row0, int N_t, int N_tp,
                             const int *cmap, int64_t b0, int64_t nblocks, void *R, int rtype, hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    const int64_t threads = nblocks * (N_tp / 16) * (N_tp / 16) * 64;
    const int64_t grid = std::min<int64_t>((threads + 255) / 256, 1 << 20);
#define OED_PACK(TK, TR)                                                                                         \
    hipLaunchKernelGGL((pack_kernel<TK, TR>), dim3(grid), dim3(256), 0, s, (const TK *)K, ld, row0, N_t, N_tp, cmap, \
                       b0, nblocks, (TR *)R)
    if (kdtype == 0 && rtype == R_F64)
        OED_PACK(double, double);
    else if (kdtype == 0 && rtype == R_F32)
        OED_PACK(double, float);
    else if (kdtype == 1 && rtype == R_F64)
        OED_PACK(float, double);
    else
        OED_PACK(float, float);
#undef OED_PACK
    return hipGetLastError();
}

hipError_t launch_pack(const void *K, int kdtype, int64_t ld, int N_t, int N_tp, const int *cmap, int N_c,
                       void *R, int rtype, hipStream_t s)
{
    return launch_pack_range(K, kdtype, ld, 0, N_t, N_tp, cmap, 0, (int64_t)N_c * (N_c + 1) / 2, R, rtype, s);
}

hipError_t launch_init_state(int *act, int n, int *state, hipStream_t s)
{
    const int threads = std::max(n, (int)ST_WORDS);
    hipLaunchKernelGGL(init_state_kernel, dim3((threads + 255) / 256), dim3(256), 0, s, act, n, state);
    return hipGetLastError();
}

}  // namespace oed
