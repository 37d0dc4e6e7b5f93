/*
 * mlmc_expv: multilevel Monte Carlo action of the matrix exponential on MI355X (gfx950).
 *
 * Computes x = exp(beta A) u for a general sparse n x n matrix A (CSR) and one or more
 * right-hand sides u, by the multilevel Monte Carlo method of Acebron, Herrero &
 * Monteiro (arXiv:1904.12754):
 *   - A is split as A = D - T (section 2.1): r_i = sum_{j != i} |a_ij| is the jump rate
 *     of row i, d_i = a_ii + r_i its diagonal weight, sigma_ij = [a_ij < 0] the sign of a
 *     jump i -> j;
 *   - x_i is the expectation of a multiplicative functional of a continuous-time Markov
 *     chain started at i, with exponential holding times of rate r and jump law
 *     |a_ij| / r_i (section 3, the integral form of the backward equation), sampled on
 *     N = 2^l steps of length dt_l = beta / 2^l with the Strang-split weights
 *     (section 2.1, the single-entry representation);
 *   - levels l0..L are combined by the telescoping estimator (section 2.2); level l > l0
 *     draws P_l - P_{l-1} from one path (the coupling of Algorithm 2);
 *   - sample sizes are either given (fixed schedule) or chosen by Algorithm 1.
 *
 * All entry points return an int status (MLMC_OK = 0). On failure a thread-local detail
 * string is available from mlmc_last_error(). Nothing here allocates on behalf of the
 * caller: A (host or device memory) and the plan options are read and copied, u and x are
 * caller owned device buffers. A plan owns its device tables until mlmc_expv_destroy.
 *
 * Streams: every call that takes `stream` (a hipStream_t, or NULL for the default
 * stream) orders its device work on that stream. Fixed-schedule runs are asynchronous
 * except that filling `stats` waits for the stream once; adaptive runs (Algorithm 1)
 * wait for the stream once per driver iteration. A plan is not re-entrant: calls on one
 * plan must not overlap. Distinct plans may run concurrently.
 *
 * Random numbers: walks draw from Philox4x32-10 (Salmon et al., SC'11) keyed by the
 * 64-bit seed, with counter (index, walk, row, level<<26 | instance<<14 | stream):
 * stream 0 gives the per-step holding-time tests (step n reads word n%4 of block n/4),
 * stream 1 the jumps (the walk's j-th jump reads block j: slot, alias coin, next holding
 * time). Results are therefore a pure function of (A, u, beta, levels, walks, seed,
 * instance), independent of launch shape and of how walk ranges are split. Every reduction
 * (per-lane compensated sums, wave and chunk sums, the level combine) runs in a fixed order
 * and the counters are integers, so results are bitwise reproducible from run to run: there
 * is no faster non-deterministic mode to select. The paths themselves are returned by
 * mlmc_expv_trace.
 */
#ifndef MLMC_EXPV_H
#define MLMC_EXPV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------- */
#define MLMC_OK 0
#define MLMC_ERR_INVALID_ARG 1     /* a null pointer, a size or an option out of range     */
#define MLMC_ERR_INVALID_MATRIX 2  /* CSR not well formed: row_ptr not monotone, column out
                                      of range, repeated column in a row, non-finite value */
#define MLMC_ERR_OUT_OF_MEMORY 3   /* a device or host allocation failed                    */
#define MLMC_ERR_HIP 4             /* a HIP runtime call failed                             */
#define MLMC_ERR_NONFINITE 5       /* some samples overflowed (count in stats->nonfinite);
                                      the result is still written                           */
#define MLMC_ERR_NOT_CONVERGED 6   /* Algorithm 1 hit its level or walk cap before reaching
                                      eps; the best estimate is still written               */
#define MLMC_ERR_UNSUPPORTED 7     /* a valid request the library does not serve            */
#define MLMC_ERR_RNG_OVERFLOW 8    /* a Philox counter word would wrap: a walk index reaches
                                      2^32, or a walk's expected number of jumps
                                      (beta * max_i r_i) reaches 2^31 (its jump index is a
                                      32-bit counter word)                                  */

/* ---- element types and precision --------------------------------------------------- */
#define MLMC_DTYPE_F32 0
#define MLMC_DTYPE_F64 1

/* Weights along a path (the exponents of the Strang factors and the sample Y):
 * FP64, or FP32 with compensated (Kahan) FP32 per-lane sums.
 * Path decisions (holding times, jump choice) are FP64/integer in both modes, so both
 * modes follow identical paths. Per-row and cross-level combination is always FP64. */
#define MLMC_PRECISION_FP64 0
#define MLMC_PRECISION_FP32 1

#define MLMC_MAX_LEVELS 40

typedef struct mlmc_plan mlmc_plan_t;

/* Where the arrays of a matrix live. */
#define MLMC_MEMORY_HOST 0
#define MLMC_MEMORY_DEVICE 1

/* A general sparse matrix in CSR form, in host memory or in device memory of the current
 * device (`memory`; a zero-initialised struct means host). Columns within a row need not be
 * sorted but must not repeat. A missing diagonal entry means a_ii = 0; explicit zeros
 * are ignored. n < 2^31, number of off-diagonal nonzeros < 2^32. The plan reads the arrays
 * once, while it is built (device arrays are copied to the host on the plan's stream, which
 * the call waits for: the plan is built on the host, section 2.1's split and the alias
 * tables), and keeps no pointer to them. */
typedef struct {
    int64_t n;
    const int64_t *row_ptr;   /* n + 1 entries, row_ptr[0] = 0 */
    const int32_t *col_idx;   /* row_ptr[n] entries */
    const void *values;       /* row_ptr[n] entries of values_dtype */
    int32_t values_dtype;     /* MLMC_DTYPE_F32 or MLMC_DTYPE_F64 */
    int32_t memory;           /* MLMC_MEMORY_HOST or MLMC_MEMORY_DEVICE */
} mlmc_csr_t;

/* Options fixed when a plan is built. */
typedef struct {
    double beta;              /* the scalar in exp(beta A) (time, or inverse temperature); > 0 */
    int32_t precision;        /* MLMC_PRECISION_FP64 or MLMC_PRECISION_FP32 */
    int32_t l0;               /* coarsest level; < 0 selects the rule of section 4,
                                 l0 = max(0, ceil(log2(2 beta max_i r_i))) */
    const int64_t *rows;      /* host array of the requested rows (estimates x_i for these i
                                 only), or NULL for all n rows */
    int64_t n_rows;           /* entries in rows (ignored when rows is NULL) */
} mlmc_plan_opts_t;

/* Read-only facts about a plan. */
typedef struct {
    int64_t n, n_rows, n_slots;   /* rows of A, requested rows, off-diagonal nonzeros */
    int32_t l0, precision;
    double beta, r_max, d_min, d_max;
    int64_t device_bytes;         /* device memory the plan holds */
    double jump_probability;      /* mean over the requested rows of 1 - exp(-beta r_i): the
                                     share of walks that leave their start row */
    int32_t screened;             /* 1 when jump_probability < 1/4: the walk kernels with
                                     several right-hand sides then first draw the steps of
                                     each walk at its start row and run in full only the
                                     walks that jump (same paths and samples) */
    int32_t pad;
} mlmc_plan_info_t;

/* Options of one run. */
typedef struct {
    uint64_t seed;            /* Philox key */
    int32_t instance;         /* 0..4095, selects an independent family of streams */
    int32_t num_levels;       /* fixed schedule: levels l0 .. l0 + num_levels - 1 */
    const int64_t *walks;     /* fixed schedule: walks per requested row at each level
                                 (host array of num_levels entries, each in [1, 2^32)) */
    double eps;               /* > 0 selects Algorithm 1 with target RMSE eps (the fixed
                                 schedule fields are then ignored) */
    int64_t pilot_walks;      /* Algorithm 1: walks per row per level of the pilot run;
                                 0 selects max(2, ceil(2^18 / (rows x right-hand sides))),
                                 at least 2^18 samples per pilot level (functional and
                                 forward runs: total walks per level; 0 selects 2^18) */
    int32_t max_levels;       /* Algorithm 1: cap on the number of levels */
    int64_t max_walks;        /* Algorithm 1: cap on walks per row per level (0 = 2^32 - 1) */
} mlmc_run_opts_t;

/* Statistics of one run (host struct, filled when non-NULL). Level q holds level l0 + q.
 * Level moments are averaged over requested rows and right-hand sides. */
typedef struct {
    int32_t l0, num_levels, converged, driver_iterations;
    int64_t walks[MLMC_MAX_LEVELS];          /* M_l per row */
    int64_t jumps[MLMC_MAX_LEVELS];          /* total jumps taken at the level */
    double level_mean_rms[MLMC_MAX_LEVELS];  /* sqrt(mean m_{l,i}^2 - level_var / M_l): the
                                                root mean square of the level term, less the
                                                sampling noise of the M_l-walk means */
    double level_var[MLMC_MAX_LEVELS];       /* mean V_{l,i}: per-walk sample variance, unbiased
                                                (M/(M-1) times mean square less squared mean) */
    double level_cost[MLMC_MAX_LEVELS];      /* cost model N_l + 4 * jumps per walk */
    int64_t steps;                           /* sum over walks of N_l */
    int64_t total_jumps;
    int64_t nonfinite;                       /* samples that were not finite */
    double est_variance;                     /* sum_l level_var / M_l */
    double est_bias;                         /* Algorithm 1's extrapolated bias (0 if fixed) */
    double kernel_ms;                        /* device time from the first walk launch to the
                                                last (includes reductions and, in adaptive
                                                runs, host round trips between iterations) */
    double walk_kernel_ms;                   /* sum of the walk-kernel durations alone, timed
                                                with a pair of events around each launch */
    int64_t walk_launches;                   /* walk-kernel launches in the run */
} mlmc_stats_t;

/* Build a plan: validate A, split A = D - T, build the alias tables of the jump law and
 * the per-level step thresholds, and upload them. `stream` orders the uploads.
 * Returns INVALID_ARG for beta <= 0 or a coarsest level so coarse that some row would
 * jump in every step with certainty at 32-bit resolution (r_i dt_l0 > 22), INVALID_MATRIX
 * for a malformed CSR, HIP_ERROR if device arrays cannot be read, and RNG_OVERFLOW when
 * beta * max_i r_i >= 2^31. */
int mlmc_expv_plan(mlmc_plan_t **out, const mlmc_csr_t *A, const mlmc_plan_opts_t *opts,
                   void *stream);

int mlmc_expv_plan_info(const mlmc_plan_t *plan, mlmc_plan_info_t *info);

/* Estimate x = exp(beta A) u at the plan's requested rows.
 *   u: DEVICE, n x nrhs row major, u_dtype MLMC_DTYPE_F32 or MLMC_DTYPE_F64.
 *   x: DEVICE, n_rows x nrhs row major FP64, overwritten.
 * Fixed schedule (opts->eps <= 0): levels l0 .. l0 + num_levels - 1 with walks[q] walks
 * per row at level l0 + q. Adaptive (opts->eps > 0): Algorithm 1 of the paper, with
 * Giles' optimal sample sizes and a bias test of weak order 2 (section 4). */
int mlmc_expv_run(mlmc_plan_t *plan, const void *u, int32_t nrhs, int32_t u_dtype,
                  const mlmc_run_opts_t *opts, double *x, mlmc_stats_t *stats, void *stream);

/* Algorithm 2's accumulators for one level: for walks walk0 .. walk0 + walks - 1 of every
 * requested row, sum1 = sum Y and sum2 = sum Y^2 per (row, rhs), where Y = u_j (eta_fine -
 * eta_coarse) at levels above l0 and Y = u_j eta_fine at l0 (j the final state).
 *   sum1, sum2: DEVICE, n_rows x nrhs FP64, overwritten.
 *   jumps: HOST, nullable; receives the jump count (waits for the stream).
 *   hash_sums: DEVICE, nullable, n_rows entries; receives per requested row the sum
 *     (mod 2^64) of the path hashes of its walks, the hash of mlmc_expv_trace. Asking for
 *     it selects a kernel variant that also hashes; the walks are the same. */
int mlmc_expv_level_sums(mlmc_plan_t *plan, const void *u, int32_t nrhs, int32_t u_dtype,
                         uint64_t seed, int32_t instance, int32_t level, uint32_t walk0,
                         uint32_t walks, double *sum1, double *sum2, int64_t *jumps,
                         uint64_t *hash_sums, void *stream);

/* mlmc_expv_level_sums without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Arguments, outputs and results are those of mlmc_expv_level_sums; the differences:
 *   - the per-(row, chunk) partial sums of a launch live in a fixed 32 MiB device array of
 *     the library (one per device, held until the process ends) instead of a plan-owned
 *     buffer grown with hipMalloc; any walk count is accepted: the walks are split into
 *     consecutive launches whose partials fit in the array (a launch with one chunk per row
 *     writes the sums directly and uses none of it);
 *   - the level's tables must exist already: the plan builds level l0 at creation, and any
 *     earlier call at a level (run, level sums, trace) builds that level; otherwise
 *     MLMC_ERR_INVALID_ARG and nothing is launched;
 *   - counters and hash_sums are cleared by a kernel (no memset node), and no timing events
 *     are recorded, so the call can be captured into a graph when jumps is NULL (asking for
 *     jumps waits for the stream).
 * The array is shared by every call on a device and keeps the last call's contents; calls
 * that overlap on one device (on different streams, or on different plans) race on it and
 * must be serialised by the caller, as must calls on one plan. */
int mlmc_expv_level_sums_noalloc(mlmc_plan_t *plan, const void *u, int32_t nrhs,
                                 int32_t u_dtype, uint64_t seed, int32_t instance,
                                 int32_t level, uint32_t walk0, uint32_t walks, double *sum1,
                                 double *sum2, int64_t *jumps, uint64_t *hash_sums,
                                 void *stream);

/* Individual walks at one level, for inspection: walk walks[q] from row rows[q]
 * (rows[q] is a row index of A, not an index into the requested rows).
 * All arrays DEVICE, count entries: final state, sign (+1/-1), jump count, a 64-bit
 * FNV-1a hash of the (state, step) pair of every jump (offset 14695981039346656037,
 * prime 1099511628211; per jump hash ^= state, *= prime, ^= 1-based step, *= prime),
 * and the natural logs of |eta_fine| and |eta_coarse| (the latter is meaningful for
 * level > 0). Path decisions are identical in both precisions; the logs are computed in
 * the plan's precision. */
int mlmc_expv_trace(mlmc_plan_t *plan, uint64_t seed, int32_t instance, int32_t level,
                    int64_t count, const int64_t *rows, const uint32_t *walks,
                    int64_t *final_state, int32_t *sign, int64_t *jumps, uint64_t *hash,
                    double *log_eta_fine, double *log_eta_coarse, void *stream);

/* Algorithm 3 (section 5): the solution of x' = A x + F, x(0) = u, with F constant in time,
 *   x(beta) = exp(beta A) u + int_0^beta exp(sA) F ds,
 * where each walk also carries the composite Simpson sum of the source term over its grid
 * times (weights 1, 4, 2, ..., 4, 1 times dt/3; F read at the path's state at each grid
 * time; the coarse functional uses the coarse rule on the even points, so the levels still
 * telescope). One right-hand side; F: DEVICE, n entries of u_dtype; the plan's l0 must be
 * >= 1. Otherwise as mlmc_expv_run and mlmc_expv_level_sums (whose sums then hold the
 * combined samples). */
int mlmc_expv_run_source(mlmc_plan_t *plan, const void *u, const void *F, int32_t u_dtype,
                         const mlmc_run_opts_t *opts, double *x, mlmc_stats_t *stats,
                         void *stream);

int mlmc_expv_level_sums_source(mlmc_plan_t *plan, const void *u, const void *F,
                                int32_t u_dtype, uint64_t seed, int32_t instance, int32_t level,
                                uint32_t walk0, uint32_t walks, double *sum1, double *sum2,
                                int64_t *jumps, uint64_t *hash_sums, void *stream);

/* Scalar functional (w, exp(beta A) u) by walks from random start rows (the full-vector
 * representation of section 2.1, summed against w). Walk m starts at row l with probability
 * |u_l| / U (U = sum of |u_l| in row order; the start row is drawn from an alias table over
 * rows, built like the slot tables, with the words of the Philox block (0, m, 0, stream 2))
 * and runs as walk m of row l on the plan's tables; its sample is
 *   U sign(u_l) w_j eta_fine                  at l0,
 *   U sign(u_l) w_j (eta_fine - eta_coarse)   above l0        (j the final state).
 * The plan must be built on A^T (the transposed generator); for a symmetric A, such as a
 * network's adjacency matrix, the plan of A serves, and u = w = 1 gives the total
 * communicability (1, exp(beta A) 1). u, w: DEVICE, n entries of dtype. The walks use the
 * plain jump law (a proposal set on the plan is not used here).
 * mlmc_expv_functional: fixed schedule (opts->walks[q] = total walks at level l0 + q) or
 *   Algorithm 1 on the scalar's variance (opts->eps > 0; pilot_walks total walks per level).
 *   result, variance: HOST (variance nullable: the estimator's variance). stats: per level
 *   the total walks, jumps, |level mean|, per-walk variance of U * sample, cost.
 * mlmc_expv_functional_level_sums: walks walk0 .. walk0 + walks - 1 of one level; HOST
 *   outputs: the sums of sign(u_l) w_j (eta_f - eta_c) (without U) and of their squares,
 *   jumps and the sum (mod 2^64) of the path hashes (nullable), and U (nullable).
 * Both wait for the stream. */
int mlmc_expv_functional(mlmc_plan_t *plan, const void *u, const void *w, int32_t dtype,
                         const mlmc_run_opts_t *opts, double *result, double *variance,
                         mlmc_stats_t *stats, void *stream);

int mlmc_expv_functional_level_sums(mlmc_plan_t *plan, const void *u, const void *w,
                                    int32_t dtype, uint64_t seed, int32_t instance,
                                    int32_t level, uint32_t walk0, uint32_t walks, double *sum1,
                                    double *sum2, int64_t *jumps, uint64_t *hash_sum, double *U,
                                    void *stream);

/* The full vector x = exp(beta A) u by the same walks (the forward representation of
 * section 2.1): walk m (start row l drawn from |u_l| / U as above, run on the plan of A^T)
 * deposits its sample sign(u_l) eta_fine (l0) or sign(u_l) (eta_fine - eta_coarse) (above
 * l0) at its final state j, so that the level term of x_j is U sum1[j] / M. At a finite
 * level this estimates (u, S^N e_j) with S the Strang step of A^T's own splitting; all
 * levels converge to exp(beta A) u. The deposits are FP64 atomic additions, so the sums
 * carry rounding that depends on the order of the walks' ends (they are not bit-reproducible
 * between runs; the paths are). u: DEVICE, n entries of dtype.
 * mlmc_expv_forward_level_sums: walks walk0 .. walk0 + walks - 1 of one level. sum1, sum2:
 *   DEVICE, n doubles each, overwritten with the per-state sums of the deposits (without U)
 *   and of their squares. HOST outputs (nullable): jumps, the sum (mod 2^64) of the path
 *   hashes, U.
 * mlmc_expv_forward: fixed schedule (opts->walks[q] = total walks at level l0 + q) or
 *   Algorithm 1 (opts->eps > 0, pilot_walks total walks per level) on the mean over the
 *   entries of the per-entry variance, with the bias test on the root-mean-square level
 *   terms, as for the backward full vector. x: DEVICE, n doubles; variance: DEVICE, n doubles
 *   or null (the per-entry variance of the estimate). stats (nullable): per level the total
 *   walks, jumps, root mean square of the level term over the entries, mean over the entries
 *   of the per-walk variance of U times the deposit, cost.
 * Both wait for the stream. */
int mlmc_expv_forward(mlmc_plan_t *plan, const void *u, int32_t dtype, const mlmc_run_opts_t *opts,
                      double *x, double *variance, mlmc_stats_t *stats, void *stream);

int mlmc_expv_forward_level_sums(mlmc_plan_t *plan, const void *u, int32_t dtype, uint64_t seed,
                                 int32_t instance, int32_t level, uint32_t walk0, uint32_t walks,
                                 double *sum1, double *sum2, int64_t *jumps, uint64_t *hash_sum,
                                 double *U, void *stream);

void mlmc_expv_destroy(mlmc_plan_t *plan);

/* ---- batched runs ------------------------------------------------------------------
 * Many plans (different matrices, right-hand sides or times) with fixed level schedules
 * in a few launches: every (instance, level) is split into items of whole walks of one
 * row, so instances of very different sizes share the chip without a launch per instance.
 * The items run either on a grid of one wave per item (the dispatcher hands them out in
 * order as waves end, so the waves in flight hold neighbouring rows and none idles before
 * the end) or on a resident grid whose waves take the items of a phase (a range of
 * consecutive items) in a fixed interleaved order (wave w takes items w, w + waves, ...).
 * Plans with an active proposal are rejected. The sequence (reset, walk phases,
 * per-row sums, per-instance FP64 combine of the levels, section 2.2) is captured once in a
 * hipGraph at creation and replayed by mlmc_expv_batch_launch. Instance b draws the
 * random streams of instance number b (the `instance` of a single run), so its estimate
 * follows the same paths as mlmc_expv_run(plans[b], ..., instance = b) with the same seed
 * and schedule. */
typedef struct mlmc_batch mlmc_batch_t;

typedef struct {
    int32_t count;                    /* instances, 1..4096 */
    mlmc_plan_t *const *plans;        /* count plans, all of one precision; a plan may appear
                                         in only one live batch at a time */
    const void *const *u;             /* count DEVICE pointers, n_b x nrhs_b row major */
    const int32_t *nrhs;              /* count entries in [1, 256] */
    int32_t u_dtype;                  /* one element type for every u */
    double *const *x;                 /* count DEVICE outputs, n_rows_b x nrhs_b FP64 */
    int32_t num_levels;               /* levels l0_b .. l0_b + num_levels - 1 of each plan */
    const int64_t *walks;             /* HOST, count x num_levels walks per row (row major) */
    int32_t autotune;                 /* 1: time candidate launch shapes (walks per item 1024,
                                         4096 and the size rule's choice x a grid of one wave
                                         per item or a resident grid of 16, 20 or 32 waves
                                         per CU) on every 8th instance at full sample sizes
                                         and keep the fastest; the choice is cached per class
                                         of batch for the process.
                                         0: walks per item from the total walk count
                                         (64 .. 4096) and the grid of waves_per_cu. */
    int32_t waves_per_cu;             /* without autotune: 0 = a grid of one wave per item
                                         (two walk launches, the coarsest levels then the
                                         rest); 1..64 = a resident grid of that many waves
                                         per CU taking the items of a phase round robin */
} mlmc_batch_desc_t;

#define MLMC_BATCH_TUNE_MAX 12   /* autotuner candidates reported in mlmc_batch_info_t */

typedef struct {
    int32_t count, segments, walks_per_item;
    int32_t waves_per_cu;             /* resident waves per CU of the walk grid, 0 for a grid
                                         of one wave per item */
    int32_t graph_nodes;
    int32_t phases;                   /* walk launches in the graph (phases of consecutive
                                         items) */
    int64_t items;                    /* (row, walk chunk) items per launch */
    int64_t device_bytes;
    int32_t tune_count;               /* candidates the autotuner timed (0 when the choice
                                         came from the cache or autotune was off) */
    int32_t tune_walks_per_item[MLMC_BATCH_TUNE_MAX];
    int32_t tune_waves_per_cu[MLMC_BATCH_TUNE_MAX];   /* 0: one wave per item */
    int32_t pad;
    double tune_ms[MLMC_BATCH_TUNE_MAX];  /* their times on the instance subset (ms) */
} mlmc_batch_info_t;

/* Validate, upload the levels' tables, optionally autotune, lay out the work, and capture
 * and instantiate the graph. The pointers in `desc` (u, x) are baked into the graph: they
 * must stay valid for the life of the batch. Waits for `stream`. */
int mlmc_expv_batch_create(mlmc_batch_t **out, const mlmc_batch_desc_t *desc, void *stream);

/* Replay the graph with Philox key `seed` on `stream` (asynchronous). Overwrites every x. */
int mlmc_expv_batch_launch(mlmc_batch_t *batch, uint64_t seed, void *stream);

/* Statistics of the last launch, one struct per instance (HOST array of count). Waits for
 * `stream`. kernel_ms and walk_kernel_ms are both the device time of the whole graph (its walk
 * phases and the short per-row sum and combine kernels after them); walk_launches is the
 * number of walk phases the graph launches. */
int mlmc_expv_batch_stats(mlmc_batch_t *batch, mlmc_stats_t *per_instance, void *stream);

int mlmc_expv_batch_info(const mlmc_batch_t *batch, mlmc_batch_info_t *info);

void mlmc_expv_batch_destroy(mlmc_batch_t *batch);

/* ---- learned proposal (importance sampling of the jump law) ------------------------
 * The walks may draw their jumps from a law q instead of the jump law p_s = |a_ks| / r_k of
 * section 3, with the path's functional multiplied by p/q of every jump taken. Any q with
 * the support of p leaves each level's expectation, and so the estimator of section 2.2,
 * unchanged; a q close to |Y| p lowers the variance. q is a small network of row features:
 *   features of row k (16): max(log p_s, -20) and clip(log((|xhat(col_s)| + delta) /
 *     (|xhat_k| + delta)), -8, 8) for slots s = 0..5, r_k dt, d_k dt, |xhat_k| / max|xhat|,
 *     (l - l0) / 8   (xhat: a pilot estimate of x, delta = 1e-6 max|xhat|; slot features
 *     are 0 past the row's slots)
 *   16 -> 64 (ReLU) -> 64 (ReLU) -> 7;  q_s = alpha softmax(z)_s + (1 - alpha) p_s over
 *     the row's slots, z_s = feature s + feature 6 + s + output s (a log-ratio prior whose
 *     softmax is p_s (|xhat(col_s)| + delta) normalised, plus the network's correction),
 *     alpha = 0.9 sigmoid(output 6)
 * Rows with more than 6 off-diagonal entries keep q = p. The defensive mixture bounds the
 * ratio p/q by 10. Tables are built on the device (BF16 matrix-core inference, FP32
 * accumulation), one alias table per level. Walks of levels with tables use them while the
 * proposal is enabled; runs, level sums and traces all follow it. Path decisions under a
 * proposal are integer (alias thresholds) as without one. */
#define MLMC_PROPOSAL_PARAMS 5703   /* W1 16x64, b1 64, W2 64x64, b2 64, W3 64x7, b3 7 (row
                                       major, in this order; W maps inputs to outputs) */

/* Set the proposal of levels l0 .. l0 + num_levels - 1 and enable it.
 *   params: HOST, MLMC_PROPOSAL_PARAMS floats, copied; NULL selects the identity proposal
 *     (the plain tables with ratio 1: walks and results are those without a proposal).
 *   xhat: DEVICE, n FP64, copied; NULL means zeros.
 * Levels at or above l0 + num_levels walk with the plain law. */
int mlmc_expv_proposal_set(mlmc_plan_t *plan, const float *params, const double *xhat,
                           int32_t num_levels, void *stream);

/* Switch a set proposal off (0) or on again (1). */
int mlmc_expv_proposal_enable(mlmc_plan_t *plan, int32_t on);

/* Export the proposal tables of one level (rebuilding them from the parameters).
 * All arrays DEVICE, n_slots entries in the plan's slot order (rows in order, the row's
 * off-diagonal entries in CSR order): alias threshold (the own slot is kept iff the coin
 * word is below it), alias slot index within the row, ratio p/q and q (FP32). */
int mlmc_expv_proposal_tables(mlmc_plan_t *plan, int32_t level, uint32_t *thr,
                              int32_t *alias_slot, float *ratio, float *q, void *stream);

/* Training loss and its gradient for given parameters, in FP32 on the device:
 *   L = ( - sum_b w_b log q_{slot_b}(row_b) + shrink sum_b w_b sum_s c_{b,s}^2 ) / sum_b w_b
 * (the cross-entropy method, whose minimiser over all laws is q ~ |Y| p, plus a shrinkage of
 * the network's corrections c = outputs 0..5 over the row's slots towards the prior).
 * Transitions with slot -1, or a slot past the row's entries, contribute nothing.
 *   params: HOST; xhat: DEVICE n FP64 or NULL; rows, slots, weights: HOST, count entries
 *   (rows in [0, n), slots in [-1, 6), weights finite >= 0); grad: HOST
 *   MLMC_PROPOSAL_PARAMS floats; loss: HOST. Waits for the stream. */
int mlmc_expv_proposal_loss_grad(mlmc_plan_t *plan, const float *params, const double *xhat,
                                 int32_t level, int32_t count, const int64_t *rows,
                                 const int32_t *slots, const float *weights, double shrink,
                                 float *grad, double *loss, void *stream);

typedef struct {
    uint64_t seed;              /* Philox key of the pilot and capture walks (instances 4095
                                   and 4094, kept apart from runs that use other instances) */
    const float *init_params;   /* HOST, MLMC_PROPOSAL_PARAMS floats */
    int64_t pilot_walks;        /* level-l0 walks per row of the pilot estimate xhat */
    int32_t capture_walks;      /* level-l0 walks per sampled row whose jumps are recorded
                                   (the first 8 jumps out of rows with <= 6 entries) */
    int32_t sample_stride;      /* rows 0, stride, 2 stride, ... are sampled */
    int32_t steps;              /* Adam steps */
    int32_t batch;              /* transitions per step, <= 2^20 */
    double lr;                  /* Adam step size (beta1 0.9, beta2 0.999, eps 1e-8) */
    double shrink;              /* weight of the shrinkage term of the loss, >= 0 */
    int32_t num_levels;         /* levels that get tables, as in mlmc_expv_proposal_set */
    int32_t judge_walks;        /* 0 or 2..65536: level-l0 walks per row of the variance
                                   judge (instance 4093); 0 skips it */
} mlmc_train_opts_t;

typedef struct {
    int64_t transitions;        /* recorded transitions with a nonzero weight */
    int64_t held_out;           /* of these, held out for validation (every 8th, <= 65536) */
    int32_t steps, n_losses;
    int32_t best_step, pad;     /* Adam steps of the kept parameters (0: the initial ones) */
    double train_ms;            /* device time of the whole call */
    double first_loss, last_loss;            /* minibatch losses */
    double first_val_loss, best_val_loss;    /* held-out losses */
    double judge_var_plain;     /* variance judge: mean per-walk variance at l0 under the */
    double judge_var_learned;   /*   plain law and under the trained proposal */
    int32_t accepted, pad2;     /* 1: the proposal is enabled (judge skipped, or it won) */
    double losses[64];          /* the last n_losses minibatch losses, every 16 steps */
} mlmc_train_stats_t;

/* Train the proposal and set it (as mlmc_expv_proposal_set with the trained parameters and
 * the pilot estimate): pilot estimate of x from plain level-l0 walks, capture of their
 * jumps with |Y| weights, minibatch Adam on the loss of mlmc_expv_proposal_loss_grad over
 * all but every 8th transition, and early stopping: the held-out loss is evaluated every 16
 * steps and the parameters with the lowest one (the initial parameters included) are kept.
 * Then, if judge_walks > 0, fresh level-l0 walks measure the per-walk variance under the
 * plain law and under the proposal, and the proposal is left enabled only if it is lower
 * (otherwise it is set but disabled, and runs use the plain law).
 * Needs a plan over all rows and an FP32 right-hand side (u: DEVICE, n entries).
 * params_out: HOST, nullable. Waits for the stream. */
int mlmc_expv_proposal_train(mlmc_plan_t *plan, const void *u, int32_t u_dtype,
                             const mlmc_train_opts_t *opts, float *params_out,
                             mlmc_train_stats_t *stats, void *stream);

/* Algorithm 1 with the proposal of level l0 learned inside the run (a project addition;
 * each level's expectation, and so the estimator of section 2.2, is unchanged).
 *   1. The run's plain pilot: M0 walks per row on l0 .. l0 + 4 (as mlmc_expv_run).
 *   2. Training on its estimate xhat = sum of the pilot's level means, as
 *      mlmc_expv_proposal_train does after its own pilot: capture, Adam with early
 *      stopping, tables. train->pilot_walks and train->judge_walks are not read;
 *      train->num_levels must be 1.
 *   3. The variance judge: M0 level-l0 walks under the proposal, with the pilot's walk
 *      indices. They replace the plain pilot's level-l0 walks if their mean per-walk
 *      variance is lower; otherwise they are dropped and the run keeps the plain law.
 *   4. The rest of Algorithm 1, as mlmc_expv_run.
 * The proposal stays set, and enabled iff it won. Needs nrhs = 1, u FP32 (DEVICE, n
 * entries), a plan over all rows and opts->eps > 0.
 * stats: walks[0] counts the walks of the estimate; steps and jumps count every walk run,
 * the dropped ones included. train_stats (nullable): as mlmc_expv_proposal_train's, with
 * train_ms the device time from the end of the pilot to the variance judge's decision.
 * params_out: HOST, nullable. Waits for the stream. */
int mlmc_expv_run_learned(mlmc_plan_t *plan, const void *u, int32_t u_dtype,
                          const mlmc_run_opts_t *opts, const mlmc_train_opts_t *train,
                          float *params_out, double *x, mlmc_stats_t *stats,
                          mlmc_train_stats_t *train_stats, void *stream);

const char *mlmc_status_string(int status);
const char *mlmc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MLMC_EXPV_H */
