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

// One instance at one phase of one greedy step: everything a kernel needs to know.  Single
// launches pass it by value; batched launches pass a device array sorted by item0, and every
// work-group finds its instance by binary search.
// Largest downdate delay depth: up to MAX_DELAY - 1 block columns held back; DEFAULT_DELAY is the
// depth taken when none is given and the autotuner is not asked for.
constexpr int MAX_DELAY = 8;  // OED_MAX_DELAY of the C ABI
constexpr int DEFAULT_DELAY = 4;
// Concurrent launch sequences of a batch when none is given (OED_BATCH_BRANCHES).
constexpr int DEFAULT_BRANCHES = 4;

struct StepDesc {
    void *R;               // working copy (element type by precision)
    void *W;               // W slots (element type by precision; BF16X3: the hi parts): slot h at
                           // W + h * wslot elements; held block columns in slots 0 .. nheld-1, the
                           // block column of the last pick goes to slot nheld
    void *W2;              // BF16X3: the lo parts (same layout), else unused
    int64_t wslot;         // elements per W slot (N_c N_tp^2)
    double *V;             // L_s^-1 P_h,s of the last pick s for every held h (operand order, N_tp^2 each;
                           // FP64, stored as FP32 in the mixed paths, which apply it on the FP32 MFMA)
    int nheld;             // number of held W (gain, pick, vcorr, trsm)
    int wb;                // gain: write the corrected diagonal blocks back to R (left-looking)
    int nsplit;            // left-looking: column partial sums in C (column kernel: splits of the
                           // W slots; trsm: C_i = R_is - sum of the nsplit partials), 0 = none
    void *C;               // left-looking column partial sums: split q at C + q cstride elements,
                           // candidate i's block at + i N_tp^2, R's type, transposed: sub-block
                           // (c, t) holds pick rows 16c.. against candidate rows 16t.. (accumulator order)
    int64_t cstride;
    const int *act_in;     // remaining candidates (gain, pick: before the pick; trsm, syrk: after it)
    int *act_out;          // pick: remaining candidates after the pick
    double *gains;         // gains by position in act_in
    double *Linv;          // L_s^-1 of the last pick, operand order
    int *state;            // ST_* words of the instance
    int *picks;            // local index of every pick
    double *pick_gain;     // gain of every pick
    double *scratch;       // global scratch of the LDS factorisation kernels (N_t > REGS_MAX_NT)
    double *fcache;        // N_t <= REGS_MAX_NT: per candidate (local index) FCACHE_BLOCKS blocks of 256
                           // doubles, the factor the gain kernel found, for the pick of the same step;
                           // null: the pick factors the winner itself
    double half_noise;     // (N_t / 2) ln sigma^2 (isotropic noise)
    const double *noise_h; // per-sensor noise term h_j by local candidate index, or null: half_noise
    int n_act;             // number of entries of act_in
    int N_t, N_tp;         // real and padded block size
    int step;              // pick: index of this pick
    int forced;            // pick: forced local index, or -1 for the argmax
    int nw;                // syrk: W slots 0 .. nw-1 applied (inner dimension nw N_tp)
    int stl;               // syrk: super-tile code of the tile order (see super_tile(); 0 = 8 x 8)
    int skipdiag;          // syrk: leave the diagonal blocks alone (kept current by the gain or
                           // block column kernel)
    int diag;              // trsm (N_tp <= 128, single launches): also subtract the new block column
                           // from every remaining diagonal block, D_ii -= W_i W_i^T, in place
    int64_t item0;         // batched launches: first work item of this instance
    int64_t nitems;        // work items of this instance (gain, trsm: n_act; pick: 1; syrk: tiles)
};

// Work items (tile slots) of the downdate over n remaining candidates: 128 x 128 tiles of the
// lower triangle, grouped in b x b super-tiles of b^2 slots each, b = 2^(stl & 7) (8 for 0; see
// super_tile()).
__host__ __device__ inline int64_t syrk_tile_rows(int n_act, int N_tp) { return ((int64_t)n_act * N_tp + 127) / 128; }
__host__ __device__ inline int64_t syrk_tiles(int n_act, int N_tp, int stl)
{
    const int lb = (stl & 7) ? (stl & 7) : 3;
    const int64_t b = (int64_t)1 << lb;
    const int64_t ST = (syrk_tile_rows(n_act, N_tp) + b - 1) / b;
    return b * b * (ST * (ST + 1) / 2);
}
// The same over 256 x 256 tiles (SYRK_BIG).
__host__ __device__ inline int64_t syrk_tiles_big(int n_act, int N_tp, int stl)
{
    const int lb = (stl & 7) ? (stl & 7) : 3;
    const int64_t b = (int64_t)1 << lb;
    const int64_t T = ((int64_t)n_act * N_tp + 255) / 256;
    const int64_t ST = (T + b - 1) / b;
    return b * b * (ST * (ST + 1) / 2);
}
// Work items of a downdate launch of the given variant.
__host__ __device__ inline int64_t syrk_items(int variant, int n_act, int N_tp, int stl)
{
    return variant == 2 ? syrk_tiles_big(n_act, N_tp, stl) : syrk_tiles(n_act, N_tp, stl);
}
// Super-tile codes (StepDesc::stl): edge 2^(code & 7) tiles, code & 8 = row-major inside.
constexpr int STL_ROW8 = 8 | 3;  // 8 x 8, row-major: the order of the first downdate kernels
constexpr int STL_COL4 = 2;      // 4 x 4, down the columns
constexpr int STL_COL8 = 3;      // 8 x 8, down the columns
constexpr int STL_COL2 = 1;      // 2 x 2, down the columns

hipError_t launch_pack(const void *K, int kdtype, int64_t ld, int N_t, int N_tp, const int *cmap, int N_c,
                       void *R, int rtype, hipStream_t s);
// Blocks b0 .. b0 + nblocks - 1 of R only, K's row r read at K + (r - row0) ld: the block rows of
// consecutive candidates from a panel of K's rows.
hipError_t launch_pack_range(const void *K, int kdtype, int64_t ld, int64_t row0, int N_t, int N_tp,
                             const int *cmap, int64_t b0, int64_t nblocks, void *R, int rtype, hipStream_t s);
hipError_t launch_init_state(int *act, int n, int *state, hipStream_t s);

// Single-instance launches (d.item0 = 0, d.nitems = work items).
// Delayed downdate: while W slots 0 .. nheld-1 hold the block columns P_h of earlier picks that
// R does not include yet, the gain and pick kernels factor R_jj - sum_h P_h,j P_h,j^T,
// launch_vcorr forms V_h = L_s^-1 P_h,s for the new pick s, and the block-column kernel writes
// W_i = R_is L_s^-T - sum_h P_h,i V_h^T to slot nheld.
hipError_t launch_gain(const StepDesc &d, int rtype, int wtype, hipStream_t s);
hipError_t launch_pick(const StepDesc &d, int rtype, int wtype, hipStream_t s);
hipError_t launch_vcorr(const StepDesc &d, int wtype, hipStream_t s);
hipError_t launch_trsm(const StepDesc &d, int rtype, int wtype, hipStream_t s);
// Left-looking block column (Algorithm 1's order): partial sums of sum_h W_h,i W_h,s^T over the
// d.nw W slots, split in d.nsplit parts (d.nitems = nsplit * row tiles), for every remaining i.
hipError_t launch_column(const StepDesc &d, int rtype, int wtype, hipStream_t s);
// Batched: one common N_tp per launch; each descriptor's nitems = nsplit * its row tiles.
hipError_t launch_column_batched(const StepDesc *descs, int n, int64_t total, int N_tp, int rtype, int wtype,
                                 hipStream_t s);
// Downdate kernels: SYRK_DIRECT streams W operands from global memory per wave (any N_tp);
// SYRK_LDS stages them through LDS with a software pipeline (a run-time slice loop for
// N_tp > 128).  W_BF16X3 always runs the BF16 split-product kernel (N_tp a multiple of 32; above
// 128 single instances with SYRK_LDS only).
// SYRK_BIG: 256 x 256 tiles, eight waves (the BF16 split product only; its work items are
// syrk_tiles_big()).
enum SyrkVariant { SYRK_DIRECT = 0, SYRK_LDS = 1, SYRK_BIG = 2, SYRK_NVARIANTS = 3 };
hipError_t launch_syrk(const StepDesc &d, int rtype, int wtype, int variant, hipStream_t s);

// Block (li, lj), li >= lj, of the current Schur complement into out (device, N_t x N_t FP64
// row-major; tr: its transpose), subtracting the nsub W slots R does not include.
hipError_t launch_schur_block(const void *R, int rtype, const void *W, const void *W2, int wtype, int64_t wslot,
                              int nsub, int li, int lj, int tr, int N_t, int N_tp, double *out, hipStream_t s);

// Batched launches over n instances (descs: device array sorted by item0, total work items).
// The register factorisation kernels serve all of them (max_Nt <= REGS_MAX_NT); a batched
// downdate launch needs one common N_tp.
hipError_t launch_gain_batched(const StepDesc *descs, int n, int64_t total, int rtype, int wtype, hipStream_t s);
hipError_t launch_pick_batched(const StepDesc *descs, int n, int max_Nt, int rtype, int wtype, hipStream_t s);
hipError_t launch_vcorr_batched(const StepDesc *descs, int n, int64_t total, int wtype, hipStream_t s);
hipError_t launch_trsm_batched(const StepDesc *descs, int n, int64_t total, int rtype, int wtype, hipStream_t s);
// nw: W blocks every instance of the launch applies (its descriptors' nw)
hipError_t launch_syrk_batched(const StepDesc *descs, int n, int64_t total, int N_tp, int nw, int rtype, int wtype,
                               int variant, hipStream_t s);

// Largest N_t handled by the register-resident factorisation kernels; beyond it the
// LDS / global-scratch kernels run.
constexpr int REGS_MAX_NT = 128;
// Blocks of 16 x 16 doubles the factor cache keeps per candidate: U_pp^-1 for the 8 diagonal
// blocks and the 28 off-diagonal blocks of U (N_t <= REGS_MAX_NT).
constexpr int FCACHE_BLOCKS = 36;
// Largest padded block size of the blocked global-scratch factorisation kernels (and of the
// left-looking method beyond REGS_MAX_NT); larger blocks fall back to element-wise kernels.
constexpr int BLK_MAX_NTP = 1024;

// Global scratch (doubles) the factorisation kernels of a block size need: the gain kernel for
// N_c candidates and the pick kernel (0: none).
size_t gain_scratch_doubles(int N_t, int N_tp, int N_c);
size_t pick_scratch_doubles(int N_t, int N_tp);

// Bytes of dynamic LDS the LDS factorisation kernels need (0 = use global scratch).
size_t gain_lds_bytes(int N_t);
size_t pick_lds_bytes(int N_t);

}  // namespace oed
