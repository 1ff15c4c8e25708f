// Internal declarations of liboed: storage layouts and kernel launchers.
//
// Storage of the working copy R (the Schur complement of the candidate part of
// K; its diagonal blocks are the matrices M_s of Algorithm 1, Sec. III-D):
//  * Sensor blocks are padded from N_t to N_tp = ceil(N_t/16)*16 rows; a padded
//    diagonal block carries 1 on the padded diagonal and 0 elsewhere, padded
//    off-diagonal entries are 0.  Padding leaves every log-determinant and every
//    Schur complement of the real part unchanged and is never modified by the
//    downdate (its rows of W are exactly zero).
//  * Only blocks (i, j) with i >= j (local candidate indices) are stored, packed
//    by block row: block (i, j) starts at element (i(i+1)/2 + j) * N_tp^2.
//  * Inside a block, 16x16 sub-blocks are stored contiguously (256 elements),
//    sub-blocks in row-major order.  Inside a sub-block the order is the MFMA
//    16x16 accumulator order: element (t, u) sits at lane ((t%16)/4)*16 + u%16,
//    register t%4, offset lane*4 + register.  A wave loads or stores one
//    sub-block with one 4-element vector access per lane.
//  * Only the lower triangle of a diagonal block is kept current: where a sensor
//    block straddles two 128-row tiles of the downdate, its strict upper part is
//    in a tile above the diagonal, which is never visited.  Readers of diagonal
//    blocks use the lower triangle only.
// Storage of W (one N_tp x N_tp block per candidate, row t = observation,
// column k = inner index) and of L_s^-1: 16x16 sub-blocks in row-major order,
// inside a sub-block the MFMA operand order: element (t, k) at lane
// ((k%16)/4)*16 + t%16, register k%4.  Lane l then holds the four consecutive
// inner indices 4*(l/16) .. 4*(l/16)+3 of row l%16, which is what four
// consecutive 16x16x4 MFMA steps consume when the inner index of step s for
// lane group g is 16q + 4g + s.
// The BF16 hi/lo parts of W use a 16x32 sub-block (rows x inner) in the operand
// order of the 16x16x32 BF16 MFMA: element (t, k) at lane ((k%32)/8)*16 + t%16,
// register k%8.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace oed {

enum RType { R_F64 = 0, R_F32 = 1 };
enum WType { W_F64 = 0, W_F32 = 1, W_BF16X3 = 2 };

__host__ __device__ inline int64_t blk_index(int64_t i, int64_t j) { return i * (i + 1) / 2 + j; }

__host__ __device__ inline int acc_off(int t, int u, int nb)
{
    return (((t >> 4) * nb + (u >> 4)) << 8) + (((((t & 15) >> 2) << 4) + (u & 15)) << 2) + (t & 3);
}

__host__ __device__ inline int opd_off(int t, int k, int nb)
{
    return (((t >> 4) * nb + (k >> 4)) << 8) + (((((k & 15) >> 2) << 4) + (t & 15)) << 2) + (k & 3);
}

// BF16 operand order: nb32 = N_tp/32 (N_tp must be a multiple of 32).
__host__ __device__ inline int opd16_off(int t, int k, int nb32)
{
    return (((t >> 4) * nb32 + (k >> 5)) << 9) + (((((k & 31) >> 3) << 4) + (t & 15)) << 3) + (k & 7);
}

// Device state words (int32) shared by the kernels of one context.
enum StateWord { ST_STATUS = 0, ST_NPICKS = 1, ST_LAST = 2, ST_WORDS = 16 };

struct Launch {
    hipStream_t stream;
};

hipError_t launch_pack(const void *K, int kdtype, int64_t ld, int N_t, int N_tp, const int *cmap, int N_c,
                       void *R, int rtype, hipStream_t s);
hipError_t launch_init_state(int *act, int n, double *pick_gain, int *picks, int *state, hipStream_t s);
hipError_t launch_gain(const void *R, int rtype, const int *act, int n_act, int N_t, int N_tp, double half_noise,
                       double *gains, const int *state, double *scratch, hipStream_t s);
hipError_t launch_pick(const void *R, int rtype, const int *act_in, int *act_out, int n_act, const double *gains,
                       int N_t, int N_tp, double half_noise, int step, int forced, int *picks, double *pick_gain,
                       int *state, double *Linv, double *scratch, hipStream_t s);
hipError_t launch_trsm(const void *R, int rtype, const int *act, int n_act, const int *state, const double *Linv,
                       int N_tp, void *W, int wtype, hipStream_t s);
hipError_t launch_syrk(void *R, int rtype, const void *W, int wtype, const int *act, int n_act, int N_tp,
                       const int *state, hipStream_t s);
hipError_t launch_gather_block(const void *R, int rtype, int i, int j, int N_tp, double *out, hipStream_t s);

// Bytes of dynamic LDS the FP64 factorisation kernels need (0 = use global scratch).
size_t gain_lds_bytes(int N_t);
size_t pick_lds_bytes(int N_t);

}  // namespace oed
