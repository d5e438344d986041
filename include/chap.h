/*
 * chap.h - C ABI of the MI355X (gfx950) tabu-search best-shift library.
 *
 * The library implements the GPU tabu-search hot path of the CHAP MIP primal
 * heuristic (section 3.1 "GPU Tabu Search" of the paper): for every variable
 * an exact best shift (Eq. 1; flip for binaries, Algorithm 1 "Best Shift via
 * Sort-Scan-Argmax" for all others), the global best admissible move under a
 * tabu list with aspiration, and the sparse residual update.
 *
 * Conventions shared by every call
 *   - Every function except the destroy calls, chap_last_error and the
 *     accessors returns int: CHAP_OK (0) on success, a negative CHAP_E* code
 *     on failure. chap_last_error() returns the message of the last failure on
 *     the calling thread. A failed call leaves every handle unchanged.
 *   - Handles are not thread-safe: one thread (and one HIP stream) at a time
 *     per handle.
 *   - Problem form (section 3.1, problem statement):
 *         min c^T x  s.t.  A x (<=, >=, =) b,  l <= x <= u,  x_j integer
 *     for is_int[j] = 1. Rows are normalised to '<=' (section 3.1 "Memory
 *     Considerations", second remark): a 'L' row stays, a 'G' row is negated,
 *     an 'E' row becomes the consecutive pair (row, negated row). The
 *     normalised rows are numbered 0..m'-1 in that order; index m' is the
 *     objective cutoff row c^T x <= cutoff (section 3.2), inactive until a
 *     feasible point is known.
 *   - A normalised row i is violated iff its residual r_i = a_i^T x - b_i
 *     exceeds the feasibility tolerance eps (residual storage: section 3.1
 *     "Memory Considerations", first remark). The breakpoint of row i on
 *     variable j is t = xbar_j + (eps - r_i) / a_ij, rounded down when
 *     a_ij > 0 and up when a_ij < 0 for an integer variable (Algorithm 1,
 *     phase 1).
 *   - Arithmetic is IEEE FP64 (no contraction, correctly rounded division).
 *     Scores are sums of +-w_i and +-w_i/2; with integer-valued weights they
 *     are exact, so results do not depend on summation order.
 */
#ifndef CHAP_H
#define CHAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CHAP_OK = 0,
  CHAP_EINVAL = -1,   /* invalid argument or inconsistent problem data */
  CHAP_ENOMEM = -2,   /* host or device allocation failed */
  CHAP_EHIP = -3,     /* a HIP runtime call failed */
  CHAP_ESTATE = -4,   /* call not valid in the handle's current state */
  CHAP_ENOTBUILT = -5 /* no usable gfx950 device */
};

typedef struct chap_problem chap_problem;
typedef struct chap_run chap_run;

typedef struct {
  double feas_tol;      /* eps; default 1e-6 */
  int32_t graph_iters;  /* tabu iterations recorded per HIP graph; 0 = 64 */
  int32_t short_max;    /* normalised entries up to which a column is scored
                           by one lane (1..8); 0 = 8 */
  int32_t chunk_min;    /* entries above which an integer column with at most
                           64 values is split over workgroups; 0 = 4096 */
  int32_t chunk_len;    /* nonzeros per workgroup chunk for those columns;
                           0 = 4096 */
  int32_t row_stage;    /* 1 (default, also 0): on all-integer instances whose
                           row activities fit int32, score short and packed
                           columns with at most 64 values from per-entry
                           records made by workgroups that each gather rows
                           from one eighth of the rows (the same results,
                           fewer HBM bytes); -1: never */
  int32_t rescore_cap;  /* affected rescoring of chap_tabu_run walks: 0
                           (default) scores every column every iteration;
                           > 0 (at most 4096): after a move that changes
                           no weight, no incumbent and no cutoff residual,
                           only the columns sharing a row with the moved
                           column (and the moved column) are scored again
                           when they are at most rescore_cap columns, every
                           other score being unchanged (section 3.1 "Memory
                           Considerations", first paragraph); otherwise the
                           iteration scores every column. Same trajectory as
                           0. Disables row_stage (the staged pass leaves the
                           long columns' scores to the move selection).
                           chap_batch_run and chap_learned_run walks score
                           every column. */
} chap_options;

/* One trace record per tabu iteration (48 bytes, host order). */
typedef struct {
  int64_t iter;  /* iteration index k */
  int32_t var;   /* moved variable, -1 when the step reweighted */
  int32_t kind;  /* 0 move, 1 move allowed by aspiration, 2 reweight */
  double x_old;  /* value before the move (0 for a reweight) */
  double x_new;  /* value after the move (0 for a reweight) */
  double score;  /* best-shift score s_j of the move (0 for a reweight) */
  int64_t viol;  /* violated normalised rows after the step (cutoff row
                    counted when active) */
  double obj;    /* c^T x after the step */
} chap_trace_record;

/* Fills *opt with the defaults. */
void chap_options_default(chap_options *opt);

/*
 * chap_problem_create - validate, normalise and upload one MIP.
 *
 * Defined by the problem statement of section 3.1 and the normalisation of
 * section 3.1 "Memory Considerations".
 *   n, m           variables and original rows (>= 0).
 *   csr_*          host CSR of A: csr_row_ptr (m+1, int64, [0]=0, non-
 *                  decreasing), csr_col (nnz, int32 in [0,n)), csr_val (nnz).
 *   csc_*          host CSC of the same A: csc_col_ptr (n+1), csc_row (nnz,
 *                  int32 in [0,m)), csc_val (nnz). CSR and CSC must hold the
 *                  same entries (any order within a row or column); no
 *                  (row, col) pair may repeat; stored zeros are dropped.
 *   sense          m chars 'L', 'G' or 'E'.     rhs   m finite values.
 *   lb, ub         n bounds; -inf/+inf allowed (HUGE_VAL). Integer bounds
 *                  are rounded inward; lb must not exceed ub afterwards.
 *   is_int         n flags (0/1). A [0,1] integer variable is binary.
 *   obj            n finite objective coefficients.
 *   opt            NULL for the defaults.
 * All host arrays are copied; the caller may free them on return. The
 * residual of every row is accumulated in the order of csr_col within the row.
 * Limits: nnz < 2^31 and every column shorter than 2^31 entries.
 * Errors: CHAP_EINVAL (with a message naming the first offending entry),
 * CHAP_ENOMEM, CHAP_EHIP, CHAP_ENOTBUILT. On error *out is left unchanged.
 */
int chap_problem_create(chap_problem **out, int32_t n, int32_t m, const int64_t *csr_row_ptr,
                        const int32_t *csr_col, const double *csr_val, const int64_t *csc_col_ptr,
                        const int32_t *csc_row, const double *csc_val, const char *sense,
                        const double *rhs, const double *lb, const double *ub, const uint8_t *is_int,
                        const double *obj, const chap_options *opt);

void chap_problem_destroy(chap_problem *p);

/* m' (normalised rows, excluding the cutoff row whose index is m'). */
int32_t chap_problem_num_norm_rows(const chap_problem *p);

/* For each normalised row: its original row and sign (+1 or -1). Host
 * arrays of m' entries. */
int chap_problem_norm_row_map(const chap_problem *p, int32_t *orig_row, int8_t *sign);

/*
 * chap_best_shift - one exact best-shift pass over all variables.
 *
 * Computes the residuals of every normalised row from scratch at d_x, then
 * for every variable j the best shift of Eq. (1): the flip for a binary
 * variable; otherwise the smallest candidate position (bounds and row
 * breakpoints inside [l_j, u_j], the incumbent excluded) that maximises the
 * score s_j of section 3.1 "Scoring Functions", as Algorithm 1 returns it.
 * When no candidate scores above zero the result is (xbar_j, 0) (Algorithm 1
 * explanation, phase 4).
 *   d_x        device, n doubles: the incumbent (inside the bounds, integral
 *              on integer variables; otherwise the result is unspecified).
 *   d_w        device, m'+1 floats: row weights in normalised order, the last
 *              one for the cutoff row. Must be finite and >= 0.
 *   cutoff_rhs the cutoff row c^T x <= cutoff_rhs is active iff finite.
 *   d_shift    device, n doubles, out: xhat_j.
 *   d_score    device, n doubles, out: s_j (> 0, or 0 when no improvement).
 *   hip_stream hipStream_t to run on (NULL = the null stream).
 * Asynchronous: returns once the work is queued. The pass kernels are
 * captured into a HIP graph on the first call and replayed by later calls.
 * The problem's internal buffers are reused by every call, so calls on one
 * problem must not overlap (queue them on one stream). Errors: CHAP_EINVAL,
 * CHAP_EHIP.
 */
int chap_best_shift(chap_problem *p, const double *d_x, const float *d_w, double cutoff_rhs,
                    double *d_shift, double *d_score, void *hip_stream);

/*
 * chap_best_shift_noalloc - chap_best_shift for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, and
 * harnesses that forbid hipMalloc. Same arguments, results and errors as
 * chap_best_shift (results bit for bit equal); it calls no hipMalloc, hipFree
 * or allocating routine, creates no graph, stream or event, and launches the
 * pass kernels one by one on hip_stream. Every per-call buffer comes from one
 * scratch array of chap_best_shift_noalloc_max_bytes() (64 MiB) per GPU,
 * held by the library until the process ends and shared by every call on
 * that GPU: calls that overlap on one GPU (any problem, any stream) race and
 * must be serialised by the caller. The problem's device must be current.
 * CHAP_EINVAL when the problem needs more scratch than that (the message
 * says how much; about 25 bytes per variable, 24 per row and 8 per entry of
 * the staged narrow columns), or on the checks of chap_best_shift.
 */
int chap_best_shift_noalloc(chap_problem *p, const double *d_x, const float *d_w, double cutoff_rhs,
                            double *d_shift, double *d_score, void *hip_stream);
size_t chap_best_shift_noalloc_max_bytes(void);

/*
 * chap_jump_values - the jump value of every variable: the value that
 * minimises the weighted violation of the variable's constraints with every
 * other variable held at d_x (the jump value of Feasibility Jump, which
 * section 3.1 "Best Shift Moves" recalls as the move its line sweep
 * generalises).
 * For variable j, V_j(t) is the sum, over j's normalised rows in ascending
 * order (an equality row: the row, then its negation) and then the cutoff
 * row when active and c_j != 0, of w_i max(0, r_i + a_ij (t - xbar_j)), each
 * term added to the sum in that order. The jump value minimises V_j over the
 * domain (integers for integer variables) without xbar_j; ties go to the
 * value closest to xbar_j, then to the smaller one. An integer variable with
 * at most 64 values tries every value; any other variable the kinks of V_j
 * (xbar_j - r_i / a_ij, for integers the integers on either side), its
 * finite bounds and, for integers, xbar_j +- 1. The score is V_j(xbar_j) -
 * V_j(t*) (may be negative); with no value to try the result is (xbar_j, 0).
 *   d_x, d_w, cutoff_rhs, hip_stream  as chap_best_shift.
 *   d_jump     device, n doubles, out: t*_j (original order).
 *   d_score    device, n doubles, out: the jump score.
 * Asynchronous. Columns with more than 4096 entries add per-chunk partial
 * sums (exact on integer data; within rounding of the stored-order sum
 * otherwise). Uses the buffers of chap_best_shift: calls of either function
 * on one problem must not overlap. Errors: CHAP_EINVAL, CHAP_ENOMEM,
 * CHAP_EHIP.
 */
int chap_jump_values(chap_problem *p, const double *d_x, const float *d_w, double cutoff_rhs,
                     double *d_jump, double *d_score, void *hip_stream);

/* Duration of the jump kernels (after the residual and weight set-up) of the
 * most recent chap_jump_values call on this problem (HIP events on that
 * call's stream); waits for that call. *ms = 0 before the first call. */
int chap_jump_values_ms(chap_problem *p, double *ms);

/*
 * chap_best_shift_pass_ms - duration of the best-shift kernels (the pass
 * after the residual and weight set-up) of the most recent chap_best_shift
 * call on this problem, measured with HIP events recorded on that call's
 * stream. Waits for that call to finish. *ms = 0 before the first call.
 * Errors: CHAP_EINVAL, CHAP_EHIP.
 */
int chap_best_shift_pass_ms(chap_problem *p, double *ms);

/*
 * chap_tabu_run - one tabu walk of `iters` iterations (section 3.1).
 *
 * Start point: seed = 0 -> x_j = clamp(0, l_j, u_j); otherwise an integer
 * variable with finite bounds starts at l_j + (h mod (u_j - l_j + 1)) with h
 * the (j+1)-th output of SplitMix64 seeded with `seed`; continuous and
 * unbounded variables start at clamp(0, l_j, u_j). Weights start at 1.
 * Every iteration: if no normalised row is violated the point is an
 * incumbent (objective cutoff c^T x <= f_best - delta, section 3.2; delta = 1
 * when the objective is integral on integer variables, else
 * 1e-4 max(1, |f_best|)); then every variable's best shift is computed; the
 * move is the highest positive score (lowest index on ties) among variables
 * not tabu, except that the overall best may be taken while tabu when its
 * move leaves no violated row (aspiration); a moved variable stays tabu for
 * `tenure` iterations; when no move is admissible, the weight of every
 * violated normalised row (cutoff included) grows by 1.
 *   iters >= 0, tenure >= 0, iters + tenure < 2^31.
 *   x0         optional host start point (n doubles, caller's order) replacing
 *              the seed rule: inside the bounds and integral on integer
 *              variables (CHAP_EINVAL otherwise); NULL to use the seed rule.
 *   hip_stream work is ordered after what is queued on this stream.
 * Synchronous: on return *out holds the trace and the final state.
 * Errors: CHAP_EINVAL, CHAP_ENOMEM, CHAP_EHIP.
 */
int chap_tabu_run(chap_problem *p, int64_t iters, int32_t tenure, uint64_t seed, const double *x0,
                  chap_run **out, void *hip_stream);

/*
 * chap_batch_run - many independent tabu walks advanced together (section
 * 3.1 "Parallel Tabu Search Instances": each walk has its own point, tabu
 * list and weights).
 *
 * Walk w runs on problem probs[walk_prob[w]] from the start point
 * walk_x0[w] when walk_x0 and walk_x0[w] are not NULL (n host doubles, the
 * rules of chap_tabu_run's x0), else from the start point of seed
 * walk_seed[w] (the rule of chap_tabu_run). All walks run `iters`
 * iterations with the same tenure. Every iteration is one launch per kernel
 * over all walks (the blocks of each launch are divided among the walks by
 * their work), several iterations are recorded in one HIP graph. Walk w's
 * result is identical to chap_tabu_run(probs[walk_prob[w]], iters, tenure,
 * walk_seed[w], walk_x0 ? walk_x0[w] : NULL, ...).
 *   probs      nprob problem handles (same device); a problem may serve any
 *              number of walks.
 *   walk_prob  nwalks indices into probs.    walk_seed  nwalks seeds.
 *   out        host array of nwalks run handles, filled on success (each
 *              released with chap_run_destroy).
 * Synchronous. Errors: CHAP_EINVAL, CHAP_ENOMEM, CHAP_EHIP.
 */
int chap_batch_run(chap_problem *const *probs, int32_t nprob, const int32_t *walk_prob,
                   const uint64_t *walk_seed, const double *const *walk_x0, int32_t nwalks, int64_t iters,
                   int32_t tenure, chap_run **out, void *hip_stream);

/*
 * chap_autotune - picks the kernel routing thresholds and graph size for an
 * instance by measurement (the paper fixes its length classes for H100,
 * section 3.1 "Kernel Specialization"; here they are tuned per instance).
 *
 * For each candidate option set the problem is re-planned from a host copy
 * of p's input arrays and walk_iters tabu iterations are timed (start seed 0,
 * tenure 10, after a short warm-up). Results never depend on the options
 * (same trajectories), only speed does.
 *   cands, ncand  candidate sets (feas_tol is ignored: p's is kept); ncand = 0
 *                 uses a built-in grid of 8 over short_max {4, 8},
 *                 chunk_min = chunk_len {2048, 4096}, graph_iters {32, 64}
 *   walk_iters    1 .. 2^20 timed iterations per candidate
 *   best          the fastest candidate (pass it to chap_problem_create)
 *   ms_per_iter   optional, one entry per candidate (8 for the grid)
 * Synchronous; uses the current device. CHAP_EINVAL on bad arguments.
 */
/*
 * chap_batch_restarts - chap_batch_run with diversity-driven restarts
 * (section 3.1 "Parallel Tabu Search Instances": the paper measures the
 * diversity of an instance against the other active ones by the Hamming
 * distance over the discrete variables, d(x, y) = #{i in I : x_i != y_i},
 * and restarts instances that come too close to others).
 * The walks run in segments of restart_every iterations. At the end of each
 * segment but the last, walk w restarts when a walk w' < w on the same
 * problem lies at distance < min_distance (all distances taken at the points
 * before any restart of that boundary). A restart keeps the walk's
 * iteration count, best feasible point and cutoff row (a restart point that
 * is feasible under the cutoff becomes the new incumbent) and starts again
 * from the start point of seed walk_seed[w] + c * 0x9E3779B97F4A7C15 (mod
 * 2^64; c = 1, 2, ... counts the walk's restarts) with unit weights and an
 * empty tabu list. Between segments the host reads the distances (one
 * kernel over every pair of walks on a problem) and re-initialises the
 * restarted walks; each segment is the batched graph of chap_batch_run.
 *   restart_every  > 0.    min_distance  >= 0 (0: no restarts).
 * Other arguments as chap_batch_run (no start points). Walk w's iterations
 * at which it restarted: chap_run_restarts. chap_run_best_infeasible is not
 * recorded for a walk that restarted (CHAP_EINVAL). Synchronous. Errors:
 * CHAP_EINVAL, CHAP_ENOMEM, CHAP_EHIP.
 */
int chap_batch_restarts(chap_problem *const *probs, int32_t nprob, const int32_t *walk_prob,
                        const uint64_t *walk_seed, int32_t nwalks, int64_t iters, int32_t tenure,
                        int64_t restart_every, int64_t min_distance, chap_run **out, void *hip_stream);

/* The iterations at which a walk of chap_batch_restarts restarted (*count of
 * them, ascending; owned by the run). Zero for other runs. */
int chap_run_restarts(const chap_run *r, const int64_t **iters, int64_t *count);

int chap_autotune(const chap_problem *p, const chap_options *cands, int32_t ncand, int64_t walk_iters,
                  chap_options *best, double *ms_per_iter);

/* Trace of a run: *records points into the run (valid until
 * chap_run_destroy), *count = iters. */
int chap_run_trace(const chap_run *r, const chap_trace_record **records, int64_t *count);

/*
 * Final state of a run, copied into caller host arrays (any pointer may be
 * NULL to skip it): x (n), resid (m'+1, normalised order, cutoff last; 0 for
 * an inactive cutoff), w (m'+1), best_x (n, only written when a feasible
 * point was found). *best_obj = +inf and *cutoff_rhs = +inf when none was.
 */
int chap_run_state(const chap_run *r, double *x, double *resid, float *w, double *best_obj,
                   double *best_x, double *cutoff_rhs);

/*
 * chap_run_best_infeasible - the best infeasible point the walk visited (the
 * pool keeps partial solutions besides feasible ones, section 3.2 and
 * Fig. 1): among its start point and the point after each iteration, those
 * violating at least one normalised row of the problem (the cutoff row not
 * counted), the first with the fewest such rows.
 *   x         optional host array of n doubles (caller's order), filled when
 *             such a point exists.
 *   violated  its violated normalised rows (0 when none exists).
 *   iter      the iteration after which it was reached; -1 for the start
 *             point, -2 when every visited point was feasible.
 * Errors: CHAP_EINVAL, CHAP_EHIP.
 */
int chap_run_best_infeasible(const chap_run *r, double *x, int64_t *violated, int64_t *iter);

/* GPU time of the run's iteration graphs in milliseconds (HIP events); for
 * a batch, the time of the whole batch. */
double chap_run_elapsed_ms(const chap_run *r);

/* Iterations of a chap_tabu_run walk that scored only the columns affected
 * by the previous move (problems created with rescore_cap > 0; section 3.1
 * "Memory Considerations", first paragraph); 0 for other runs. Errors:
 * CHAP_EINVAL (null argument). */
int chap_run_rescored(const chap_run *r, int64_t *iters);

void chap_run_destroy(chap_run *r);

/* Message of the last failed call on this thread ("" if none). */
const char *chap_last_error(void);

/*
 * Candidate-proposal network.
 *
 * The paper scores every variable exactly in every iteration (section 3.1,
 * "Scoring Functions"). The learned proposal is an addition beside that
 * method: a small network ranks the variables, only its top-ranked ones get
 * the exact FP64 best shift of Eq. 1 / Algorithm 1, and a periodic full pass
 * is both the fallback and the judge, so every move taken is still an exact
 * best shift. The network maps 16 inputs to one output through two hidden
 * layers of 64 ReLU units:
 *     y = W3 relu(W2 relu(W1 x + b1) + b2) + b3.
 * Products take bfloat16 operands (inputs, weights and hidden activations
 * rounded to nearest even) and accumulate in FP32 on the matrix cores;
 * parameters and biases are FP32. Training minimises the mean squared error
 * with Adam (beta1 0.9, beta2 0.999, epsilon 1e-8) on FP32 master parameters,
 * whose bfloat16 copy the forward pass uses.
 *
 * Parameters, flat FP32 order (CHAP_MODEL_NPARAM values): W1[64][16] (row =
 * hidden unit), b1[64], W2[64][64], b2[64], W3[64], b3.
 * Feature rows: 16 bfloat16 values per sample (uint16_t bit patterns), row
 * major, in the input order listed under chap_learned_run.
 */
#define CHAP_MODEL_NPARAM 5313

typedef struct chap_model chap_model;

/* New network on the current device with He-uniform weights: weight p of a
 * layer with fan-in k is (2u - 1) sqrt(6/k), u = (splitmix64(seed, p) >> 11)
 * 2^-53 (SplitMix64 as for start points), rounded to FP32; biases 0. */
int chap_model_create(chap_model **out, uint64_t seed);
void chap_model_destroy(chap_model *m);

/* Copies the FP32 parameters to / from a host array of CHAP_MODEL_NPARAM
 * floats. set rejects non-finite values (CHAP_EINVAL) and resets Adam. Both
 * synchronise the device. */
int chap_model_get_params(const chap_model *m, float *params);
int chap_model_set_params(chap_model *m, const float *params);

/* Network outputs for n feature rows: d_feat (device, n x 16 bfloat16),
 * d_out (device, n floats). Asynchronous on hip_stream. */
int chap_model_forward(chap_model *m, const uint16_t *d_feat, int64_t n, float *d_out,
                       void *hip_stream);

/* Gradient of L = (1/n) sum_i (y_i - target_i)^2 with respect to the flat
 * parameters: d_feat (device, n x 16), d_target (device, n floats), d_grad
 * (device, CHAP_MODEL_NPARAM floats). Sums are taken in a fixed order, so
 * the result is reproducible bit for bit. Asynchronous on hip_stream. */
int chap_model_grad(chap_model *m, const uint16_t *d_feat, const float *d_target, int64_t n,
                    float *d_grad, void *hip_stream);

/* `steps` Adam steps with learning rate lr on minibatches of `batch` pairs
 * drawn from the npairs rows of (d_feat, d_target): sample i of step k is row
 * splitmix64(seed, k * batch + i) mod npairs. Asynchronous on hip_stream. */
int chap_model_train(chap_model *m, const uint16_t *d_feat, const float *d_target, int64_t npairs,
                     int32_t steps, int32_t batch, float lr, uint64_t seed, void *hip_stream);

/*
 * Learned tabu walk.
 *
 * Iterations run in blocks of full_every. The first iteration of a block is
 * a full evaluation, identical to an iteration of chap_tabu_run (exact best
 * shift of every column, selection under tabu/aspiration, move or reweight);
 * it also judges the network (was its move in the network's current
 * proposal set?), optionally trains the network on that evaluation, and
 * refreshes the stored inputs. Each further iteration is a proposal
 * iteration: the network scores every proposable column, the topk best
 * (ties: lowest internal index) get the exact best shift of Eq. 1 /
 * Algorithm 1, and the move is chosen among them with the same tabu and
 * aspiration rules (aspiration needs the move to leave no violated row). A
 * proposal iteration without an admissible move makes no move and no
 * reweight (a stall); the rest of its block does nothing and the next
 * iteration is a full evaluation. Every move taken is an exact best shift.
 *
 * Trace kinds: 0/1/2 as chap_tabu_run for full evaluations; 8 (move) and
 * 9 (move by aspiration) for proposal iterations; 3 for a stall.
 *
 * Proposable columns: binaries and integer columns with finite bounds and at
 * most 64 values, at any length; other columns when their breakpoints fit
 * one workgroup (normalised entries + 2 bounds + cutoff entry <= 4096).
 * Longer general columns are scored only by the full evaluations.
 * topk and train_pairs are at most 8192.
 *
 * Network inputs of column j (index: meaning), each computed in FP64 and
 * rounded once to bfloat16:
 *   0 weighted violated share: sum of w_i over violated normalised rows of j
 *     / sum of w_i over all normalised rows of j (cutoff row excluded; 0 if
 *     none)            1 log2(1 + stored entries of j)
 *   2 c_j / max|c| (0 if c = 0)
 *   3 s_last_j / sum_i w_i, clamped to [-4, 4] (0 if no rows), s_last = the
 *     exact score at the last full evaluation
 *   4 1 if binary   5 1 if integer and not binary   6 1 if continuous
 *   7 (x_j - l_j)/(u_j - l_j); 0.5 with an infinite bound; 0 if l_j = u_j
 *   8 log2(1 + min(u_j - l_j, 2^20)); 20 with an infinite bound
 *   9 violated normalised rows of j / normalised rows of j (0 if none)
 *  10 sum over violated rows of |a_ij| min(r_i, 1000) / (1000 sum_i |a_ij|)
 *  11 sign(xhat_last_j - x_j), xhat_last = best shift at the last full
 *     evaluation
 *  12 min(k - last_move_j, 1024) / 1024 (never moved: last_move = -1024)
 *  13 min(k - k_last_full, 64) / 64
 *  14 V / m' (violated normalised rows, cutoff included when active)
 *  15 log2(1 + moves of j)
 * Inputs 0, 3, 9, 10 are refreshed at full evaluations only; 7, 11, 12, 15
 * follow the column's own moves at once.
 *
 * Training (train_steps > 0): at each full evaluation, the T = train_pairs
 * columns with the largest exact scores and T proposable columns drawn with
 * SplitMix64 (train_seed, index evals * 2T + i) form 2T pairs whose target
 * is max(s_j, 0) / max_i s_i (0 when no score is positive); train_steps Adam
 * steps are taken on them with learning rate lr. With log_pairs > 0 the
 * pairs of every full evaluation are also kept (until log_pairs pairs).
 */
typedef struct {
  int32_t topk;        /* columns given the exact best shift per proposal
                          iteration; default 1024 */
  int32_t full_every;  /* iterations per block; 1 = every iteration full
                          (the chap_tabu_run trajectory); default 64 */
  int32_t train_steps; /* Adam steps per full evaluation; default 0 */
  int32_t train_pairs; /* T; default 1024 */
  float lr;            /* Adam learning rate; default 1e-3 */
  int32_t log_sets;    /* 1: keep every proposal set in the run */
  int64_t log_pairs;   /* capacity of the pair log (pairs); default 0 */
  uint64_t train_seed; /* seed of the random training pairs; default 0 */
  int32_t refresh_every; /* proposal iterations per proposal set: the
                            network scores every column and a new set is
                            chosen at the first proposal iteration of a
                            block and every refresh_every proposal
                            iterations after it; the iterations between
                            evaluate the same set exactly at their own
                            point. Default 1 (a new set every iteration) */
} chap_learned_options;

void chap_learned_options_default(chap_learned_options *opt);

/* One learned walk with model m (same device as p; trained in place when
 * train_steps > 0). Start point, seed, tenure and iters as chap_tabu_run;
 * opt may be NULL for the defaults. Synchronous; *out as chap_tabu_run.
 * CHAP_EINVAL on invalid options (topk, full_every, train_pairs,
 * refresh_every <= 0, lr <= 0, train_steps < 0). */
int chap_learned_run(chap_problem *p, chap_model *m, const chap_learned_options *opt,
                     int64_t iters, int32_t tenure, uint64_t seed, const double *x0,
                     chap_run **out, void *hip_stream);

/* Counters of a learned run: full evaluations, evaluations whose move was
 * in the network's proposal set, stalls. Zero for other runs. */
int chap_run_learned_stats(const chap_run *r, int64_t *evals, int64_t *hits, int64_t *stalls);

/* Proposal sets of a learned run with log_sets: iteration k's set is
 * sets[offsets[k] .. offsets[k+1]) (original column indices, ascending
 * internal order); full evaluations have empty ranges. *iters = 0 without
 * the log. Pointers valid until chap_run_destroy. */
int chap_run_proposals(const chap_run *r, const int32_t **sets, const int64_t **offsets,
                       int64_t *iters);

/* Logged training pairs (count x 16 bfloat16 inputs, count targets). */
int chap_run_pairs(const chap_run *r, const uint16_t **feat, const float **target, int64_t *count);

/* Network inputs of every column at a given state, as defined above:
 * d_x (n), d_w (m'+1, cutoff weight last), cutoff_rhs (+inf: inactive),
 * d_s_last and d_xhat_last (n, FP64), d_last_move and d_moves (n, int32),
 * iteration k and k_last_full <= k; all device arrays in original order.
 * Writes d_out (device, n x 16 bfloat16 bits, original order); rows of
 * columns that are never proposed are zero. Synchronous. */
int chap_features(chap_problem *p, const double *d_x, const float *d_w, double cutoff_rhs,
                  const double *d_s_last, const double *d_xhat_last, const int32_t *d_last_move,
                  const int32_t *d_moves, int64_t k, int64_t k_last_full, uint16_t *d_out,
                  void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* CHAP_H */
