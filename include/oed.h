/*
 * oed.h -- C ABI of liboed: greedy D-optimal sensor selection on one MI355X.
 *
 * The problem (paper, Sec. III-A to III-D): K is the dense data-space matrix
 * K = Gamma_noise + F Gamma_prior F^* of a linear-Gaussian inverse problem,
 * with one N_t x N_t block per candidate sensor (sensor i owns rows and
 * columns i*N_t .. i*N_t+N_t-1).  With isotropic noise sigma^2 I, greedy
 * D-optimal selection adds, at every step, the remaining candidate j with the
 * largest information gain
 *     g_j = 1/2 logdet(sigma^-2 S_j),
 * where S_j is the N_t x N_t Schur complement of K_jj given the sensors
 * already selected (the matrix M_s of Algorithm 1, Sec. III-D).  Exact ties go
 * to the lowest sensor index.  The sum of the first k gains is
 * 1/2 logdet(sigma^-2 K_AA) for the selected set A (Sec. III-C objective).
 *
 * The library keeps the Schur complement R of the candidate part of K in HBM
 * and, per step, (a) factors every remaining diagonal block in FP64 and takes
 * the argmax of the gains, (b) forms W = R[:, s] L_s^-T for the winner s, and
 * (c) downdates R -= W W^T on its lower triangle.
 *
 * Conventions shared by all calls:
 *  - Device pointers are HIP device memory of the current device; host
 *    pointers are ordinary host memory.  The library never frees caller memory.
 *  - K is row-major with leading dimension ld >= N_s*N_t elements, FP64 or
 *    FP32; only its lower triangle (column <= row) is read, and only during
 *    oed_create / oed_reset (the library keeps its own packed working copy).
 *  - Sensor indices are 0-based indices into K's block rows.
 *  - All work is enqueued on the stream given to oed_create (a hipStream_t;
 *    NULL = the default stream).  Calls that return host results synchronise
 *    that stream before returning.
 *  - Every call returns an oed_status; no call aborts or throws.  The text of
 *    the last error of a handle is available from oed_last_error().
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef OED_H
#define OED_H

#include <stdint.h>

#ifndef OED_API
#define OED_API __attribute__((visibility("default")))
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oed_ctx oed_ctx;

typedef enum oed_status {
    OED_OK = 0,
    OED_E_ARG = 1,         /* invalid argument (sizes, sigma2 <= 0 or NaN, NULL, index) */
    OED_E_NOT_SPD = 2,     /* every remaining candidate has a non-positive-definite Schur block */
    OED_E_OOM = 3,         /* device or host allocation failed */
    OED_E_HIP = 4,         /* a HIP runtime call failed */
    OED_E_STATE = 5,       /* the handle cannot do this now (e.g. after OED_E_NOT_SPD) */
    OED_E_UNSUPPORTED = 6  /* a valid request this build does not handle */
} oed_status;

typedef enum oed_dtype { OED_F64 = 0, OED_F32 = 1 } oed_dtype;

/*
 * Arithmetic of the working copy R and of the downdate R -= W W^T.
 *  FP64         : R, W and the downdate in FP64 (FP64 MFMA).
 *  MIXED_F32    : R and W stored in FP32, downdate on FP32 MFMA with FP32
 *                 accumulation.  Diagonal-block Cholesky factorisations, gains,
 *                 the winner's factor and the solve forming W run in FP64.
 *  MIXED_BF16X3 : like MIXED_F32, but W is split into BF16 hi + lo parts
 *                 (hi = bf16(w), lo = bf16(w - hi)) and the product is
 *                 hi*hi + hi*lo + lo*hi on BF16 MFMA with FP32 accumulation
 *                 (relative error of each product term about 2^-16).  Blocks
 *                 are padded to a multiple of 32 rows instead of 16.
 * The paper keeps K in FP64 and runs the whole candidate loop in FP32 (Sec. IV);
 * MIXED_F32 keeps the precision-critical factorisations in FP64 instead.
 */
typedef enum oed_precision {
    OED_PREC_FP64 = 0,
    OED_PREC_MIXED_F32 = 1,
    OED_PREC_MIXED_BF16X3 = 2
} oed_precision;

/* oed_options.flags */
/* Deepest downdate delay (oed_options.delay, OED_BATCH_DELAY). */
#define OED_MAX_DELAY 8

#define OED_FLAG_PROFILE 0x1u /* time every kernel with HIP events (see oed_get_profile) */
#define OED_FLAG_AUTOTUNE 0x4u /* with delay 0: choose the delay depth and the downdate kernel by
                                  timing one step's kernels on the packed working copy (see
                                  oed_get_config); the choice is cached per device, precision,
                                  block size and candidate count for the life of the process */
#define OED_FLAG_DEFER_PACK 0x8u /* create without K (K_dev must be NULL; dtype and ld are ignored):
                                    the working copy is filled block row by block row with
                                    oed_pack_rows before the first step, so that K never has to
                                    be resident in full beside it (600 sensors x 420 observations,
                                    the paper's shape: the FP32 working copy takes 135 GB, a full
                                    FP32 K another 254 GB).  Not with OED_FLAG_AUTOTUNE. */

typedef struct oed_options {
    uint32_t struct_size;       /* sizeof(oed_options); set by oed_options_init */
    int32_t precision;          /* oed_precision, default OED_PREC_FP64 */
    uint32_t flags;             /* OED_FLAG_* */
    const int32_t *candidates;  /* host array of candidate sensors (the set C of Sec. III-A);
                                   NULL = all N_s sensors.  Copied during oed_create. */
    int32_t n_candidates;       /* length of candidates */
    int32_t delay;              /* downdate delay depth p, 1..OED_MAX_DELAY: hold up to p - 1
                                   picks' block columns W and subtract them together with the next
                                   one (the gain, pick and block-column steps correct for the held
                                   ones exactly; same picks, 1/p of the R traffic per pick).
                                   1 = subtract every pick's W W^T at the next step; 0 = automatic
                                   (with OED_FLAG_AUTOTUNE the autotuner's choice, else 4, for
                                   N_t <= 128; 1 otherwise).  With 128 < N_t <= 1024 a depth p > 1
                                   is taken as given (the gain and pick kernels then apply the held
                                   columns themselves); p > 1 with N_t > 1024: OED_E_UNSUPPORTED */
    int32_t method;             /* OED_METHOD_RIGHT_LOOKING (default), _LEFT_LOOKING or _AUTO */
    int32_t max_budget;         /* left-looking: most picks the handle will make (the W history
                                   is allocated for them); 0 = all candidates */
    const double *noise_half_logdet; /* host array, one per sensor (length N_s): h_j = 1/2 logdet of
                                   sensor j's noise covariance block, for noise independent between
                                   sensors (the computable objective of Sec. III-C with a
                                   block-diagonal noise covariance; K must include that noise).  A
                                   candidate then scores 1/2 logdet S_j - h_j.  NULL = isotropic
                                   noise sigma2: h_j = (N_t/2) ln sigma2.  Copied during oed_create;
                                   non-finite entries: OED_E_ARG. */
    const char *tune_cache;     /* path of a text file the autotuner (OED_FLAG_AUTOTUNE) reads its
                                   choice from and appends a newly tuned one to, keyed by the GPU's
                                   name, precision, block size, candidate count / 32 and method;
                                   NULL = keep choices in the process only.  An unreadable or
                                   unwritable file is ignored (the tuner then times as usual). */
    int64_t max_device_bytes;   /* 0 = no limit; else oed_create returns OED_E_OOM, before any
                                   allocation or other HIP call, when the handle would hold more
                                   device memory than this (oed_last_error(NULL) gives the bytes) */
    int32_t tile_order;         /* downdate tile order, OED_TILES_*: 0 = automatic (the autotuner's
                                   choice with OED_FLAG_AUTOTUNE, else OED_TILES_COL4) */
    int32_t debug_fail_step;    /* test hook for the error paths: k >= 1 makes the k-th pick after
                                   creation (or the last reset) fail once with OED_E_HIP on the
                                   host, before anything of that step is enqueued; 0 = off */
    int32_t tile_size;          /* downdate work-group tile: 128 (128 x 128, four waves), 256 (256 x 256,
                                   eight waves; MIXED_BF16X3 with N_t <= 128 only, else
                                   OED_E_UNSUPPORTED) or 0 =
                                   automatic (the autotuner's choice with OED_FLAG_AUTOTUNE, else
                                   128) */
    int32_t reserved[1];        /* must be 0 */
} oed_options;

/*
 * oed_options.tile_order: the order in which the downdate's 128 x 128 tiles of the lower
 * triangle are handed out (one contiguous share per XCD).  Tiles are grouped in b x b
 * super-tiles swept band by band; COL orders run down each super-tile's columns, so the tiles
 * sharing a column panel of W are consecutive and the band's b row panels stay in the XCD's L2;
 * ROW8 runs along the rows of 8 x 8 super-tiles.  The order changes only speed, never results.
 */
#define OED_TILES_AUTO 0
#define OED_TILES_ROW8 1
#define OED_TILES_COL8 2
#define OED_TILES_COL4 3
#define OED_TILES_COL2 4

/*
 * oed_options.method.
 *  RIGHT_LOOKING : R is the Schur complement of all remaining candidates; every pick subtracts
 *                  its block column's outer product from all of R (the downdate).
 *  LEFT_LOOKING  : the order of Algorithm 1 (Sec. III-D): R keeps K off the diagonal; every
 *                  pick forms only its own block column, K_is - sum over the earlier picks'
 *                  block columns (W history), and updates the diagonal blocks.  About 1/3 of
 *                  the flops of RIGHT_LOOKING at 600 x 128, budget 175.  Every precision
 *                  for N_t <= 1024 (else OED_E_UNSUPPORTED); the delay option does not
 *                  apply.
 */
#define OED_METHOD_RIGHT_LOOKING 0
#define OED_METHOD_LEFT_LOOKING 1
/* AUTO: left-looking when it needs fewer flops, i.e. for max_budget <= N_c / 2 (per pick k the
   column costs 2 k N_t^3 per remaining candidate against (N_c - k) N_t^3 for the downdate), and
   N_t <= 1024; else right-looking. */
#define OED_METHOD_AUTO 2

/* Fill *opt with the defaults (FP64, no flags, all sensors). */
OED_API void oed_options_init(oed_options *opt);

/*
 * Create a selection context for K (device memory, dtype OED_F64 or OED_F32,
 * leading dimension ld) with N_s sensors of N_t observations each and noise
 * variance sigma2 > 0.  The candidate part of K's lower triangle is copied into
 * a packed working copy R (half of the dense size; FP64 or FP32 by precision).
 * K is not referenced after this call returns.  All device memory the greedy
 * loop needs is allocated here; later calls allocate nothing on the device.
 * stream: a hipStream_t (NULL = default stream).  opt: NULL = defaults.
 * On success *out is a new handle; on failure *out is NULL.
 */
OED_API oed_status oed_create(oed_ctx **out, const void *K_dev, int32_t dtype, int64_t ld, int32_t N_s,
                      int32_t N_t, double sigma2, void *stream, const oed_options *opt);

/*
 * Reload the working copy from K_dev (same dtype, ld and shape as at creation)
 * and forget all picks.  Allocates nothing.  For a handle created with
 * OED_FLAG_DEFER_PACK, K_dev must be NULL: the picks are forgotten and every
 * block row must be packed again with oed_pack_rows.
 */
OED_API oed_status oed_reset(oed_ctx *h, const void *K_dev);

/*
 * Pack the block rows of sensors sensor0 .. sensor0 + n_sensors - 1 into the
 * working copy of a handle created with OED_FLAG_DEFER_PACK (Sec. III-F keeps
 * K out of device memory and fetches its blocks as needed; here the caller
 * forms K panel by panel and frees each panel after this call).  K_rows
 * (device, dtype OED_F64 or OED_F32, row-major, leading dimension ld) holds
 * rows sensor0*N_t .. (sensor0 + n_sensors)*N_t - 1 of K, row r at
 * K_rows + (r - sensor0*N_t)*ld, with at least the columns
 * 0 .. (sensor0 + n_sensors)*N_t - 1 (ld >= that width); only column <= row is
 * read.  Sensors that are not candidates are skipped; packing a row twice
 * overwrites it.  Only before the first pick (after creation or a reset).
 * The greedy, force, scores and Schur-block calls return OED_E_STATE until
 * every candidate's block row has been packed.  Synchronises the handle's
 * stream before returning, so the caller may free K_rows afterwards.
 */
OED_API oed_status oed_pack_rows(oed_ctx *h, const void *K_rows, int32_t dtype, int64_t ld, int32_t sensor0,
                                 int32_t n_sensors);

/*
 * Run `budget` more greedy steps (Sec. III-D): each step scores all remaining
 * candidates, picks the best and conditions on it.  idx_out[k] (host,
 * length budget) receives the sensor index of the k-th new pick, gain_out[k]
 * (host, length budget) its gain in nats.  *n_out = picks actually made.
 * 0 <= budget <= number of remaining candidates, else OED_E_ARG.
 * Returns OED_E_NOT_SPD, with the picks made before it, when every remaining
 * candidate has a non-positive-definite Schur block; the handle then only
 * accepts oed_reset / oed_destroy / queries.  One host synchronisation per call.
 */
OED_API oed_status oed_greedy(oed_ctx *h, int32_t budget, int32_t *idx_out, double *gain_out,
                      int32_t *n_out);

/*
 * Force the next pick to be sensor idx (a remaining candidate) instead of the
 * argmax: used to resume from a saved selection or to replay another
 * trajectory.  *gain_out (host, may be NULL) receives its gain.
 */
OED_API oed_status oed_force(oed_ctx *h, int32_t idx, double *gain_out);

/*
 * Gains of all candidates at the current step, as the next greedy step would
 * score them.  gains_out: host, length N_s; -inf for sensors that are picked
 * or not candidates (and for non-positive-definite Schur blocks).
 */
OED_API oed_status oed_scores(oed_ctx *h, double *gains_out);

/*
 * Block (i, j) of the current Schur complement of the remaining candidates
 * (both i and j remaining candidates), in FP64, unpadded, row-major N_t x N_t
 * into host memory out.  Any order of i, j is accepted (R is symmetric).  The
 * block is formed on the device (left-looking: the stored K block minus the
 * formed block columns' products) and copied to the host; a diagnostic query,
 * not part of the greedy loop.
 */
OED_API oed_status oed_schur_block(oed_ctx *h, int32_t i, int32_t j, double *out);

/* All picks so far (host arrays of capacity >= N_s); *n_out = count. */
OED_API oed_status oed_picks(oed_ctx *h, int32_t *idx_out, double *gain_out, int32_t *n_out);

/* Kernel classes reported by oed_get_profile. */
enum { OED_K_GAIN = 0, OED_K_PICK = 1, OED_K_TRSM = 2, OED_K_SYRK = 3, OED_K_PACK = 4, OED_K_COUNT = 5 };

typedef struct oed_profile {
    double ms[OED_K_COUNT];        /* summed kernel time, from HIP events on the context stream */
    int64_t launches[OED_K_COUNT];
    double syrk_flops;             /* algorithmic flops of all downdates: sum N_t * n (n + 1),
                                      n = remaining rows (remaining sensors * N_t) */
    double syrk_bytes;             /* algorithmic HBM bytes: sum e * (n (n + N_t) + n N_t),
                                      e = bytes per element of R (lower blocks read and
                                      written once, W read once) */
} oed_profile;

/* Read (and with reset != 0 clear) the accumulated profile.  Needs OED_FLAG_PROFILE. */
OED_API oed_status oed_get_profile(oed_ctx *h, oed_profile *out, int32_t reset);

/*
 * Batched selection: many independent designs of uneven sizes (candidate counts, N_t, sigma2,
 * budgets) selected together.  Every step's work for all instances still running is issued
 * as one launch per kernel (gains, pick, block column, downdate per block size), and the whole
 * schedule of all steps is captured once into a HIP graph, so oed_batch_run is one graph
 * launch plus one copy of the results.  Same precisions and conventions as the single-design
 * calls; every instance needs 1 <= N_t <= 128.
 */
typedef struct oed_instance {
    const void *K_dev;  /* device, row-major, lower triangle read (during create / reset only) */
    int32_t dtype;      /* OED_F64 or OED_F32 */
    int32_t N_s, N_t;   /* sensors and observations per sensor */
    int32_t budget;     /* picks, 1 <= budget <= N_s */
    int64_t ld;         /* leading dimension of K, >= N_s * N_t */
    double sigma2;      /* noise variance, > 0 */
} oed_instance;

typedef struct oed_batch oed_batch;

/* Don't capture the schedule into a HIP graph: enqueue the launches on every run. */
#define OED_BATCH_NO_GRAPH 0x2u
/* Downdate delay depth p in 1..OED_MAX_DELAY (see oed_options.delay); without it the depth is 4,
   or the autotuner's choice with OED_BATCH_AUTOTUNE. */
#define OED_BATCH_DELAY(p) ((uint32_t)(p) << 8)
/* Without OED_BATCH_DELAY: run the whole selection once per delay depth during creation and
   keep the fastest (see oed_batch_get_config). */
#define OED_BATCH_AUTOTUNE 0x10u
/* Downdate tile order o (OED_TILES_*, see oed_options.tile_order); without it OED_TILES_COL4, or
   the autotuner's choice with OED_BATCH_AUTOTUNE. */
#define OED_BATCH_TILES(o) ((uint32_t)(o) << 12)
/* Run the instances as g independent launch sequences (1 <= g <= OED_BATCH_MAX_BRANCHES): the
   instances are split into g groups of about equal downdate work, each group's launches go to a
   stream of its own, forked from and joined into the batch's stream (captured as parallel
   branches of the one graph), so one group's latency-bound steps overlap another's downdates.
   Without it: 4 (at most the number of instances), or with OED_BATCH_AUTOTUNE the tuner's choice.
   Results do not depend on g. */
#define OED_BATCH_MAX_BRANCHES 4
#define OED_BATCH_BRANCHES(g) ((uint32_t)(g) << 16)
/* Left-looking method for every instance (see OED_METHOD_LEFT_LOOKING; no delay, no autotuner). */
#define OED_BATCH_LEFT_LOOKING 0x20u

/*
 * Create a batch over inst[0..n): validates every instance, allocates all device memory,
 * packs every working copy and builds the launch schedule.  flags: OED_FLAG_PROFILE (time
 * each run with HIP events), OED_BATCH_NO_GRAPH, OED_BATCH_DELAY(p), OED_BATCH_TILES(o),
 * OED_BATCH_AUTOTUNE, OED_BATCH_LEFT_LOOKING.  On failure
 * *out is NULL.
 */
OED_API oed_status oed_batch_create(oed_batch **out, const oed_instance *inst, int32_t n, int32_t precision,
                                    void *stream, uint32_t flags);

/*
 * Run every instance's greedy selection from its start.  Outputs (host):
 * idx_out / gain_out: picks of instance i at offset sum_{j<i} budget_j, length budget_i;
 * n_out[i]: picks made; status_out[i]: OED_OK, or OED_E_NOT_SPD if instance i stopped early.
 * A second run without oed_batch_reset selects on the already conditioned working copies and
 * is rejected (OED_E_STATE).
 */
OED_API oed_status oed_batch_run(oed_batch *b, int32_t *idx_out, double *gain_out, int32_t *n_out,
                                 int32_t *status_out);

/* Reload every working copy from inst[] (same shapes, dtypes and leading dimensions as at
 * creation, else OED_E_ARG); allocates nothing.  The packing is ordered after all work enqueued
 * so far on the stream given at creation (where the caller may still be writing K), and the call
 * returns once it is done, so K may be changed or freed afterwards. */
OED_API oed_status oed_batch_reset(oed_batch *b, const oed_instance *inst, int32_t n);

/* Milliseconds of the last run (HIP events around it; needs OED_FLAG_PROFILE), and the
 * algorithmic downdate flops and bytes of one run (definitions as in oed_profile). */
OED_API oed_status oed_batch_stats(const oed_batch *b, double *run_ms, double *syrk_flops, double *syrk_bytes);

/* The delay depth, the downdate tile order (OED_TILES_*) and the number of launch sequences the
   batch runs with, and with OED_BATCH_AUTOTUNE the autotuner's run time for depths
   1..OED_MAX_DELAY in the default tile order and one sequence (OED_MAX_DELAY doubles, host); the
   tuner then tries the other orders and sequence counts at the chosen depth.  Any output pointer
   may be NULL. */
OED_API oed_status oed_batch_get_config(const oed_batch *b, int32_t *delay, int32_t *tile_order, int32_t *branches,
                                        double *per_run_ms);
OED_API oed_status oed_batch_destroy(oed_batch *b);
OED_API const char *oed_batch_last_error(const oed_batch *b);

/* ---------------------------------------------------------------------------------------------
 * Design evaluation: the objective of given sensor sets, as in the comparison of the greedy
 * design with random and uniformly spaced ones (Sec. IV-E, Fig. 5).  For a design
 * S = (s_0, ..., s_{B-1}) of distinct sensors and isotropic noise (Sec. III-C),
 *     f(S) = 1/2 logdet(sigma^-2 K_SS) = sum_k t_k,  t_k = 1/2 logdet(S_k) - (N_t/2) ln sigma^2,
 * where S_k is the Schur complement of K's block s_k given s_0 .. s_{k-1} (chain rule of the
 * determinant, the recursion of Algorithm 1, Sec. III-D).  t_k is the gain the greedy would
 * credit s_k after conditioning on s_0 .. s_{k-1}, so the greedy design in its pick order
 * reproduces the greedy gains term by term.  f(S) does not depend on the order; the terms do.
 * Each design runs as a selection whose k-th pick is forced to s_k (a blocked right-looking
 * Cholesky of K_SS with the pick, block-column and downdate kernels; no gain scoring), and up
 * to `batch` designs run together in one batched launch sequence (a HIP graph unless
 * OED_BATCH_NO_GRAPH).
 */
typedef struct oed_eval oed_eval;

/*
 * Evaluator of designs of B sensors (1 <= B <= N_s) over K (device, dtype OED_F64 or OED_F32,
 * row-major, ld >= N_s*N_t, lower triangle read; it must stay valid and unchanged for the life
 * of the evaluator, since every run packs from it).  N_t <= 128.  max_batch: designs per batched
 * launch sequence; 0 = as many as fit in half the free device memory, at most 64.  precision:
 * oed_precision (downdate type; the block factorisations are FP64).  flags: OED_FLAG_PROFILE,
 * OED_BATCH_NO_GRAPH, OED_BATCH_DELAY(p); anything else is OED_E_ARG.  Allocates all device
 * memory of the evaluator.  On failure *out is NULL.
 */
OED_API oed_status oed_eval_create(oed_eval **out, const void *K_dev, int32_t dtype, int64_t ld, int32_t N_s,
                                   int32_t N_t, double sigma2, int32_t B, int32_t max_batch, int32_t precision,
                                   void *stream, uint32_t flags);

/*
 * Evaluate n designs: designs (host) holds design r at designs[r*B .. r*B+B), each entry a
 * sensor in [0, N_s), no sensor twice in a design (else OED_E_ARG and nothing runs).  Outputs
 * (host): obj_out[r] = f(S_r); terms_out (may be NULL) [r*B + k] = t_k of design r.  A design
 * whose Schur block is not positive definite gets obj NaN (terms NaN from that block on), the
 * others are still evaluated, and the call returns OED_E_NOT_SPD.  Designs run in chunks of the
 * evaluator's batch size; a short last chunk costs a full one.  Synchronises the creation stream
 * first, then runs on the evaluator's own stream and returns when the results are on the host.
 */
OED_API oed_status oed_eval_run(oed_eval *e, const int32_t *designs, int32_t n, double *obj_out,
                                double *terms_out);

/* Of the last oed_eval_run: *run_ms, milliseconds of its launch sequences (HIP events; needs
 * OED_FLAG_PROFILE, else 0); *syrk_flops, algorithmic downdate flops executed (definition as in
 * oed_profile, all executed instances); *executed, instances executed (n rounded up to chunks);
 * *batch, designs per chunk.  Any output pointer may be NULL. */
OED_API oed_status oed_eval_stats(const oed_eval *e, double *run_ms, double *syrk_flops, int64_t *executed,
                                  int32_t *batch);
OED_API oed_status oed_eval_destroy(oed_eval *e);
OED_API const char *oed_eval_last_error(const oed_eval *e);

/* ---------------------------------------------------------------------------------------------
 * A whole greedy selection that allocates nothing, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * It runs the kernels of oed_create + oed_greedy (right-looking, LDS downdate, delay depth
 * `delay`, all N_s sensors candidates, isotropic noise) in the same order, so its picks and
 * gains equal, bit for bit, those of a handle created with the same precision and delay and
 * run for the same budget.  Every workspace (working copy R, W slots, L_s^-1, held-column
 * corrections, gains, active lists, state words) lives in one static device array of
 * OED_NOALLOC_MAX_BYTES that the library holds on each GPU it runs on until the process ends;
 * the call makes no hipMalloc / hipFree and no allocating library call.
 *
 * Arguments: K_dev, dtype, ld, N_s, N_t, sigma2 as for oed_create (device K, row-major, lower
 * triangle read); precision: oed_precision; delay: 1..OED_MAX_DELAY (0 = 4); 0 <= budget <= N_s.
 * Outputs (device memory of the current device, caller-owned): idx_dev[k] (int32, length
 * budget) the k-th pick's sensor index, gain_dev[k] (FP64, length budget) its gain;
 * status_dev[0] (int32) 0 = all picks made, 2 = every remaining candidate had a
 * non-positive-definite Schur block (picks after that are not written), status_dev[1] = picks
 * made.  err (host, may be NULL): err_len bytes receiving the text of a failure.
 *
 * Everything is enqueued on `stream` (hipStream_t, NULL = default) and the call returns without
 * synchronising; the outputs are valid once the stream reaches that point.  Rejected before
 * anything runs: invalid arguments (OED_E_ARG), N_t > 128 or a problem whose workspaces exceed
 * OED_NOALLOC_MAX_BYTES (OED_E_UNSUPPORTED; the message gives the bytes needed:
 * the sum of N_s (N_s + 1)/2 N_tp^2 e_R (R), delay N_s N_tp^2 e_W (W; BF16: twice),
 * 8 (delay - 1) N_tp^2 (if delay > 1), 8 N_tp^2, 8 N_s, 73,728 N_s (the factor cache of the
 * pick), three times 4 N_s and 64 bytes, each
 * rounded up to a multiple of 256; N_tp = N_t rounded up to a multiple of 16, of 32 for
 * MIXED_BF16X3; e_R = 8 for FP64, else 4; e_W = 8, 4 or 2 by precision).
 * All calls on one GPU share its one array, which keeps the last call's contents (every buffer
 * is re-initialised by kernels before it is read): two calls that overlap in time on the same
 * GPU (different streams or threads) race and give undefined results.
 */
#define OED_NOALLOC_MAX_BYTES (64ull << 20)
OED_API oed_status oed_greedy_noalloc(const void *K_dev, int32_t dtype, int64_t ld, int32_t N_s, int32_t N_t,
                                      double sigma2, int32_t precision, int32_t delay, int32_t budget, void *stream,
                                      int32_t *idx_dev, double *gain_dev, int32_t *status_dev, char *err,
                                      int32_t err_len);

/* Bytes of device memory the handle holds. */
OED_API oed_status oed_device_bytes(const oed_ctx *h, int64_t *bytes);

/*
 * The configuration the handle runs with: *delay (1..OED_MAX_DELAY), *syrk_variant (0: per-wave
 * global operands, 1: LDS-staged 128 x 128 tiles, 2: LDS-staged 256 x 256 tiles, -1: left-looking,
 * no downdate), *tile_order (OED_TILES_*: the
 * downdate's tile order, chosen by the autotuner unless given), and, if per_pick_ms is not NULL,
 * the autotuner's estimate of the time per pick for delay depths 1..OED_MAX_DELAY (OED_MAX_DELAY
 * doubles, host; 0 where not measured, all 0 without OED_FLAG_AUTOTUNE).  Any output pointer may
 * be NULL.
 */
OED_API oed_status oed_get_config(const oed_ctx *h, int32_t *delay, int32_t *syrk_variant, int32_t *tile_order,
                                  double *per_pick_ms);

/* Destroy the handle and free its device memory.  NULL is accepted. */
OED_API oed_status oed_destroy(oed_ctx *h);

/* Text of the handle's last error ("" if none).  For NULL: the text of the last failed
 * oed_create on the calling thread ("" if none). */
OED_API const char *oed_last_error(const oed_ctx *h);

/* Name of a status code. */
OED_API const char *oed_status_string(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* OED_H */
