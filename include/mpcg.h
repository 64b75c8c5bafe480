/*
 * mpcg.h -- C ABI of the MI355X (gfx950) mixed-precision conjugate-gradient
 * library.
 *
 * Method: conjugate gradients for Ax = b with A sparse symmetric positive
 * definite (paper section 3, updates of x, r, p and the alpha/beta formulas),
 * where each iteration's SpMV, inner products and vector updates run in a
 * precision chosen per iteration by a policy (section 4.2 assigns precisions to
 * the matrix-vector product and the inner products; here the controlled triple is
 * {SpMV, dot, axpy}).  alpha, beta, the residual replacement and the convergence
 * test are fp64.  Policies: fixed, the tabular Q-learning policy of section 4.1
 * (greedy inference as Algorithm 2, epsilon-greedy training as Algorithm 1), and
 * an MLP policy.
 *
 * Conventions for every entry point:
 *   - Return value: MPCG_OK (0) or a negative error code; a solve returns its
 *     convergence status through mpcg_result.status.  No C++ exception crosses
 *     this boundary.  mpcg_last_error() gives a message for the calling thread.
 *   - "device pointer": memory allocated on the GPU the library runs on (e.g. a
 *     torch tensor's data_ptr()).  "host pointer": ordinary CPU memory.
 *   - Handles are not thread-safe.  All work of a matrix handle is enqueued on
 *     the stream given at creation, in order; entry points that return host data
 *     synchronise that stream before returning.
 *   - The library never frees caller memory; handles own what they allocate.
 *   - Formats: MPCG_FP16 = 0, MPCG_BF16 = 1, MPCG_FP32 = 2, MPCG_FP64 = 3,
 *     MPCG_Q52 = 4 (Table 1's quarter precision: 1 sign, 5 exponent, 2 fraction
 *     bits; matrix storage of the SpMV only), and MPCG_TF32 = 5 (section 5's
 *     format set: 1 sign, 8 exponent, 10 fraction bits, i.e. fp32's range with
 *     fp16's significand; gfx950 has no tf32 storage or arithmetic, so values
 *     are rounded to it and held in fp32 containers, at fp32's bytes and time).
 *     An action is a = 16*f_spmv + 4*f_dot + f_axpy: 0..63 for the four
 *     arithmetic formats (the joint table's and the network's action set),
 *     64..79 for q52 SpMV storage with f_dot, f_axpy in 0..3 (fixed policies),
 *     and 128..252 = 128 + 25*d_spmv + 5*d_dot + d_axpy over the digits
 *     0..3 (the four formats) and 4 (tf32) when a slot is tf32.
 *   - Vector "tier": vectors of an iteration whose axpy format is fp64 are stored
 *     as double, otherwise as float (tier64 = 1 / 0).
 */
#ifndef MPCG_H
#define MPCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPCG_OK 0
#define MPCG_ERR_INVALID (-1)     /* bad argument (NULL, size, enum)            */
#define MPCG_ERR_CSR (-2)         /* malformed CSR input                        */
#define MPCG_ERR_DEVICE (-3)      /* HIP runtime error                          */
#define MPCG_ERR_NOMEM (-4)       /* device or host allocation failed           */

/* mpcg_result.status */
#define MPCG_CONVERGED 0          /* true fp64 relative residual <= tol          */
#define MPCG_MAXIT 1              /* iteration budget exhausted                  */
#define MPCG_CONVERGED_FALLBACK 2 /* converged after the fp64 fallback restart   */
#define MPCG_BREAKDOWN 3          /* breakdown (nu <= 0 or non-finite scalars)   */

#define MPCG_FP16 0
#define MPCG_BF16 1
#define MPCG_FP32 2
#define MPCG_FP64 3
#define MPCG_Q52 4
#define MPCG_TF32 5

#define MPCG_MEM_HOST 0
#define MPCG_MEM_DEVICE 1

#define MPCG_POLICY_FIXED 0       /* one action every iteration                  */
#define MPCG_POLICY_QTABLE 1      /* greedy over a Q-table (Algorithm 2)         */
#define MPCG_POLICY_QTABLE_TRAIN 2/* epsilon-greedy + Q-learning (Algorithm 1)   */
#define MPCG_POLICY_MLP 3         /* greedy over MLP logits                      */

/* history flag bits (per iteration) */
#define MPCG_FLAG_REPLACED 1
#define MPCG_FLAG_EXPLORED 2
#define MPCG_FLAG_FALLBACK 4
#define MPCG_FLAG_SWITCH 8

#define MPCG_MLP_IN 16
#define MPCG_MLP_HIDDEN 128
#define MPCG_N_ACTIONS 64

typedef struct mpcg_matrix mpcg_matrix;
typedef struct mpcg_policy mpcg_policy;

/*
 * Policy description (section 4.1).  State s = (j*b_it + i)*2 + stag with the
 * iteration bin i = min(k / ceil(t_bin/b_it), b_it-1), the residual bin
 * j = #{ t : rho <= T_t } over the b_res-1 decreasing thresholds T_t that the
 * library derives from b_res and eps_min (mpcg_residual_thresholds), and
 * stag = [k >= w_stag and rho_k >= rho_{k-w_stag}].  Reward (section 4.1):
 * w1*min(-log10 rho', -log10 eps_min) - w2*(c[f_s]+c[f_d]+c[f_a]) + w3 on
 * convergence; a breakdown ends the episode with -w2*cost - w3.  Q update:
 * Q += lr*(R + gamma*max Q(s',.) - Q) (terminal: without the max term).
 */
typedef struct {
    int32_t kind;              /* MPCG_POLICY_*                                  */
    int32_t fixed_action;      /* used by MPCG_POLICY_FIXED (0..79, 128..252)    */
    int32_t t_bin;             /* iteration-bin horizon (1000)                   */
    int32_t b_it;              /* iteration bins (5)                             */
    int32_t b_res;             /* residual bins (10), in [1, 17]                 */
    int32_t w_stag;            /* stagnation window (10)                         */
    double lr, gamma;          /* Q-learning rate and discount (0.1, 0.9)        */
    double w1, w2, w3;         /* reward weights (1.0, 0.1, 10.0)                */
    double eps_min;            /* residual floor of the accuracy term and of the
                                  residual bins (1e-16); must be a power of ten
                                  10^-E (the double nearest to it), 1 <= E <= 300 */
    double cost[4];            /* c(fp16), c(bf16), c(fp32), c(fp64); a q52 SpMV
                                  is charged c(fp16)                             */
    uint64_t seed;             /* exploration draws                              */
    int32_t replace_period;    /* R seen by the MLP features                     */
    int32_t decision_period;   /* D: the policy acts at iterations k = 0 mod D
                                  (and at a start or restart) and its action
                                  holds in between; a decision's reward charges
                                  the cost of every iteration it ran and its
                                  Q update (and rollout) happens when it ends.
                                  0 or 1: every iteration (section 4.1)        */
    int32_t per_op;            /* 1: one Q-table per operation (section 4.1's
                                  Q_j for SpMV, dot, update), Q_j(s, p) at
                                  table row s, column 4 j + p; the greedy action
                                  takes each table's argmax, exploration draws
                                  per operation, and every Q_j is updated with
                                  the shared reward.  2: tables for the SpMV and
                                  the dot only, the updates fixed in fp64
                                  (section 4.2 keeps the residual update in full
                                  precision).  0: one joint table over the 64
                                  actions                                        */
    int32_t nfmt;              /* formats per operation table: 4 (0 reads as 4),
                                  or 5 with tf32 as digit 4 (section 5's set
                                  {fp16, bf16, tf32, fp32, fp64}); Q_j(s, d) at
                                  column nfmt*j + d; 5 needs per_op 1 or 2 for
                                  the table policies                           */
    double cost_tf32;          /* c(tf32) (section 5: 0.8 in C1, 0.5 in C2)     */
} mpcg_policy_desc;

typedef struct {
    int32_t replace_period;    /* R: true-residual replacement every R iterations
                                  (0: only when the recursive residual <= tol)  */
    int32_t fallback;          /* 1: restart as fp64 CG on breakdown/stagnation */
    int32_t chunk;             /* iterations enqueued between done-flag polls
                                  (0: library default)                          */
    int32_t profile;           /* 1: time every kernel launch of the solve with
                                  HIP events on the handle's stream (see
                                  mpcg_get_profile); adds event overhead        */
    int32_t spmv_rows;         /* rows per SpMV workgroup: 512, 1024 or 2048
                                  (0: chosen from n); results do not depend
                                  on it                                          */
    int32_t index16;           /* 0: the SpMV reads 16-bit column deltas
                                  (col - row) when every one fits, which
                                  mpcg_create_csr detects; -1: always the
                                  32-bit indices; results do not depend on it */
    int32_t precond;           /* 0: no preconditioner (M = I); 1: Jacobi,
                                  M = diag(A) kept as the fp32 of 1 / a_ii
                                  (section 3's z = M^-1 r, section 4.2's fixed
                                  fp32 preconditioner).  z = rd_fa(m r) at the
                                  update format, sigma = r.z at the dot format,
                                  p = z + beta p; rho stays ||r|| / ||b||; at a
                                  replacement sigma = r64.(M^-1 r64) in fp64,
                                  and the direction restarts (p = z) when the
                                  true residual exceeds twice the recursive one.
                                  Not for batched solves.                       */
    int32_t stop_rule;         /* 0: converged when the true fp64 relres is <= tol
                                  at a replacement (a recursive rho <= tol
                                  triggers one); 1: section 5's termination, the
                                  recursive rho < tol after at least 10
                                  iterations, no true-residual check (the result
                                  still reports the final x's true relres)     */
    int32_t rho_fp64;          /* 0: rho_k = sqrt(r.r)/||b|| with r.r at the dot
                                  format (it is also sigma'); 1: rho_k from an
                                  fp64 r.r of the stored recursive residual
                                  (section 1 keeps residual computations in
                                  fp64), sigma' still at the dot format.
                                  Not for batched solves.                       */
    int32_t emulate;           /* 0: the hardware reading (matrix stored in the
                                  SpMV format, operands rounded, low-precision
                                  vectors in fp32 containers); 1: the paper's
                                  emulation reading of fl_p(op) (section 4):
                                  every operation computes in fp64 and rounds
                                  its result to its format (each q_i of the
                                  SpMV, the total of a dot, each updated
                                  element), all vectors in fp64.  Not for q52
                                  actions or batched solves.                    */
    int32_t vec16;             /* 1: 16-bit vector storage: while the update
                                  format is bf16, r, p and x_lo are held in bf16
                                  containers (q stays fp32), so a start,
                                  replacement or tier change rounds r and p to
                                  bf16 instead of fp32; the updates themselves
                                  are unchanged.  Not with precond, rho_fp64,
                                  emulate or batched solves.                    */
    int32_t variant;           /* 0: the CG iteration of section 3 (three
                                  launches per iteration); 1: single-reduction
                                  CG (Chronopoulos and Gear, 1989): one SpMV
                                  w = A r followed by both inner products,
                                  gamma = r.r and delta = r.w, s = A p carried
                                  by a recurrence, two launches per iteration;
                                  2: pipelined CG (Ghysels and Vanroose, 2014):
                                  w = A r and z = A s carried by recurrences
                                  too, so the iteration's SpMV q = A w does
                                  not wait for its inner products; two
                                  launches per iteration, six vector updates.
                                  In exact arithmetic both give the iterates
                                  of variant 0.  A replacement also recomputes
                                  s = A p (and w = A r, z = A s).  Fixed
                                  policies with actions 0..79 only; not with
                                  fallback, precond, stop_rule, rho_fp64,
                                  emulate, vec16, profile or batched solves.
                                  Low-precision arithmetic makes the
                                  recurrences drift faster than section 3's
                                  iteration (variant 2 most); breakdown then
                                  ends the solve with status MPCG_BREAKDOWN.  */
} mpcg_solve_opts;

/* Per-kernel timing of the last solve made with opts.profile = 1.  One CG
 * iteration ("slot") is three launches: KA = SpMV with the fused nu = p.q
 * partial; KB = scalar step (alpha) + x/r update with the sigma' = r.r
 * partial; KX = scalar step (beta, policy) + direction update.  Policies that
 * write shared state or evaluate an MLP add two one-block step kernels (KS).
 * Times are sums of event-bracketed launch durations in ms. */
typedef struct {
    int32_t n_iter_slots;      /* slots whose KA ran a CG iteration              */
    int32_t n_resid_slots;     /* slots whose KA ran an fp64 residual            */
    int32_t n_idle_slots;      /* slots enqueued after the solve had finished    */
    int32_t reserved;
    double ka_iter_ms;         /* KA over iteration slots                        */
    double kb_iter_ms;         /* KB over iteration slots                        */
    double kx_iter_ms;         /* KX over iteration slots                        */
    double ks_iter_ms;         /* step kernels over iteration slots              */
    double resid_ms;           /* all launches of residual slots                 */
    double idle_ms;            /* all launches of idle slots                     */
} mpcg_profile;

typedef struct {
    int32_t status;            /* MPCG_CONVERGED ... MPCG_BREAKDOWN              */
    int32_t iters;             /* iterations performed                           */
    int32_t n_replace;         /* true-residual replacements                     */
    int32_t fallback_at;       /* iteration of the fp64 fallback, -1 if none     */
    double relres_true;        /* ||b - A x||_2 / ||b||_2 in fp64, final x       */
    double cost_sum;           /* sum over iterations of the policy's op costs   */
    double time_ms;            /* device time from first enqueue to done         */
    int32_t slots;             /* kernel slots enqueued (diagnostic)             */
    int32_t spmv_rows;         /* kernel configuration used: rows per SpMV
                                  workgroup (512, 1024 or 2048)                  */
    int32_t index16;           /* kernel configuration used: 1 if the SpMV read
                                  16-bit column deltas                           */
    int32_t reserved;
} mpcg_result;

/* ---------------------------------------------------------------- matrices */

/*
 * Copies a CSR matrix (row_ptr int32[n+1], col int32[nnz], val double[nnz]) to
 * the device and builds the fp32, bf16 and fp16 shadows (fp16 with an exact
 * power-of-two scale per row that puts the row's largest magnitude in
 * (2^14, 2^15]; Table 1 ranges).  mem_kind says where the three arrays live
 * (MPCG_MEM_HOST or MPCG_MEM_DEVICE).  stream: a hipStream_t (NULL: the null
 * stream) on which this handle's work runs.  Validation: 1 <= n, nnz < 2^31,
 * row_ptr[0] = 0, row_ptr[n] = nnz, row_ptr non-decreasing, 0 <= col < n,
 * columns strictly increasing within a row, values finite, every row has a
 * positive diagonal entry.  Device arrays are copied to the host for this
 * check first, so both kinds are validated the same way.  Error: MPCG_ERR_CSR
 * with a message naming the first bad row.
 */
int mpcg_create_csr(int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col,
                    const double *val, int mem_kind, void *stream, mpcg_matrix **out);

/* Frees the handle and everything it owns.  NULL is a no-op. */
int mpcg_destroy(mpcg_matrix *A);

typedef struct {
    int64_t n, nnz;
    int32_t index16;           /* 1: 16-bit column deltas are stored (every
                                  |col - row| <= 32767)                          */
    int32_t reserved;
} mpcg_matrix_info;

/* Sizes and storage choices of a matrix handle (host struct). */
int mpcg_get_info(mpcg_matrix *A, mpcg_matrix_info *info);

/* Copies the shadows to host arrays: float[nnz], uint16 bf16 bits[nnz],
 * uint16 fp16 bits[nnz] (row-scaled values), int8 row exponents[n]. */
int mpcg_get_shadows(mpcg_matrix *A, float *f32, uint16_t *bf16, uint16_t *f16, int8_t *rexp);
/* Copies the Jacobi preconditioner, float[n]: the fp64 reciprocal of each
 * diagonal entry rounded to fp32 (0 for a row without one). */
int mpcg_get_precond(mpcg_matrix *A, float *minv);
/* Copies the q52 shadow (Table 1's quarter precision, round to nearest even
 * from fp64, after the same exact per-row power-of-two scale as fp16) to a
 * host uint8 array[nnz] of its bit patterns. */
int mpcg_get_shadow_q52(mpcg_matrix *A, uint8_t *q52);
/* Action code of a format triple (the encoding above): f_spmv one of the six
 * formats, f_dot and f_axpy one of fp16, bf16, fp32, fp64, tf32 (the four
 * arithmetic formats with a q52 SpMV).  Returns the code (>= 0) or
 * MPCG_ERR_INVALID. */
int mpcg_action(int f_spmv, int f_dot, int f_axpy);
/* The formats of an action code; MPCG_ERR_INVALID for a code outside 0..79,
 * 128..252. */
int mpcg_action_formats(int action, int32_t *f_spmv, int32_t *f_dot, int32_t *f_axpy);
/* Copies the tf32 shadow (round to nearest even from fp64 to 11 significant
 * bits in fp32's exponent range, no row scale) to a host float array[nnz]. */
int mpcg_get_shadow_tf32(mpcg_matrix *A, float *tf32);

/* ---------------------------------------------------------------- policies */

/*
 * Residual-bin thresholds of section 4.1 (the residual bin j_k with
 * delta = -log10(eps_min) / b_res): out[j-1] = T_j, the double nearest to
 * 10^(-delta j) = 10^(-E j / b_res) for j = 1 .. b_res-1, where eps_min is the
 * double nearest to 10^-E.  Computed exactly on the host (big-integer
 * comparisons against the neighbouring doubles' midpoints), so
 * j_k = #{ j : rho_k <= T_j } equals the floor formula away from the real
 * boundaries and is decided identically everywhere.  out: host double[b_res-1].
 * Errors: MPCG_ERR_INVALID if b_res is outside [1, 17] or eps_min is not such a
 * power of ten.  Pure host code: needs no GPU.
 */
int mpcg_residual_thresholds(int32_t b_res, double eps_min, double *out);

/* Creates a policy; Q-table (n_states x 64, zero) and rollout log live on the
 * device.  The residual-bin thresholds are derived from b_res and eps_min as by
 * mpcg_residual_thresholds.  Errors: MPCG_ERR_INVALID for a bad kind, action,
 * bin parameter or eps_min. */
int mpcg_policy_create(const mpcg_policy_desc *desc, mpcg_policy **out);
/* Waits for the solves on the streams of the matrices the policy is set on,
 * and detaches it from them (they fall back to their default fixed fp64
 * policy). */
int mpcg_policy_destroy(mpcg_policy *P);
/* Host double[n_states*64] in/out, n_states = b_res*b_it*2. */
int mpcg_policy_set_qtable(mpcg_policy *P, const double *q);
int mpcg_policy_get_qtable(mpcg_policy *P, double *q);
/* Episode index and exploration rate used by the next training solves. */
int mpcg_policy_set_episode(mpcg_policy *P, int64_t episode, double epsilon);
/* MLP weights, host float arrays: W1[128][16], b1[128], W2[128][128], b2[128],
 * W3[64][128], b3[64].  Weights are used as given (bf16-representable values
 * are expected; the decision path computes in fp32). */
int mpcg_policy_set_mlp(mpcg_policy *P, const float *W1, const float *b1, const float *W2,
                        const float *b2, const float *W3, const float *b3);
/* Rollout log of (features, action, reward, done, next features) per decision,
 * capacity entries on the device; 0 disables.  Appends across solves. */
int mpcg_policy_rollouts_enable(mpcg_policy *P, int32_t capacity);
int mpcg_policy_rollouts_count(mpcg_policy *P, int32_t *n);
int mpcg_policy_get_rollouts(mpcg_policy *P, float *feat, float *next_feat, int32_t *act,
                             float *rew, uint8_t *done, int32_t cap, int32_t *n_out);
int mpcg_policy_rollouts_reset(mpcg_policy *P);
/*
 * Evaluates the policy's greedy decision on m given states, on the device:
 * k[m] iteration, rho[m] relative residual, stag[m] flag, and for MLP policies
 * feat[m][16] features (may be NULL otherwise).  Writes state[m] and action[m]
 * (host arrays).  Used to check that decisions are bit-exact for identical states.
 */
int mpcg_policy_decide(mpcg_policy *P, int32_t m, const int64_t *k, const double *rho,
                       const int32_t *stag, const float *feat, int32_t *state, int32_t *action);

/* Attaches a policy (not owned; must outlive the solves).  NULL: fixed fp64.
 * The policy's table and log calls wait for the streams of the matrices it is
 * attached to; mpcg_destroy of a matrix detaches it. */
int mpcg_set_policy(mpcg_matrix *A, mpcg_policy *P);
int mpcg_set_options(mpcg_matrix *A, const mpcg_solve_opts *opts);

/* ---------------------------------------------------------------- solves */

/*
 * Solves A x = b.  b (double[n]) and x (double[n]) are device pointers; x is
 * read as the initial guess and overwritten with the result.  Stops when the
 * true fp64 relative residual is <= tol (checked at each replacement), after
 * maxit iterations, or on breakdown.  Runs on the handle's stream with no host
 * synchronisation inside an iteration; returns after the solve is complete.
 * res (host) receives the summary.  tol > 0 and maxit >= 0 are required.
 */
int mpcg_solve(mpcg_matrix *A, const double *b, double *x, double tol, int32_t maxit,
               mpcg_result *res);

/* ---------------------------------------------------------------- batched
 * Many independent systems, either in one persistent launch (each workgroup
 * takes whole systems from a queue) or in lockstep (each iteration's three
 * kernels cover every running system).  Each system runs the solve of
 * section 3 with the policy
 * attached to that system (fixed, Q-table or MLP; not training policies or
 * rollout logs, whose state is shared), its own options (replacement period,
 * fallback) and its own tol / maxit.  Every system's result -- iterations,
 * history, x -- is bit-identical to mpcg_solve on that system alone, for every
 * configuration.
 */
typedef struct {
    int32_t workgroups;        /* persistent workgroups (0: autotuned)          */
    int32_t spmv_rows;         /* rows per SpMV group, 512/1024/2048 (0: autotuned) */
    int32_t order;             /* 0: largest systems (nnz) first; 1: as given   */
    int32_t autotune_iters;    /* iterations per system in each autotuning trial
                                  (0: 16)                                        */
    int32_t split_rows;        /* systems with more rows than this run through
                                  the full-device path (mpcg_solve) after the
                                  persistent launch; 0: autotuned, -1: none    */
    int32_t strategy;          /* 1: one persistent launch (workgroups take
                                  whole systems); 2: lockstep -- three launches
                                  per iteration over the row groups and blocks
                                  of all running systems; 0: autotuned          */
} mpcg_batch_opts;

typedef struct {
    double time_ms;            /* device time of the batched launch             */
    double tune_ms;            /* device time of the autotuning trials          */
    int32_t workgroups;        /* configuration used                            */
    int32_t spmv_rows;
    int32_t tuned;             /* 0: given, 1: autotuned now, 2: autotuner cache */
    int32_t split_rows;        /* -1: every system in the persistent launch     */
    int32_t n_split;           /* systems solved through the full-device path   */
    int32_t strategy;          /* strategy used (1 or 2)                        */
    double persistent_ms;      /* device time of the persistent launch          */
    double split_ms;           /* device time of the full-device solves         */
} mpcg_batch_info;

/*
 * Solves A[i] x[i] = b[i] for i < nsys.  A[i] are distinct handles on one
 * device; b[i], x[i] are device double[n_i] (x[i]: initial guess in, solution
 * out); tol[i], maxit[i] host arrays as in mpcg_solve; res[i] (host) receives
 * each system's summary (time_ms: the whole batch).  Runs on A[0]'s stream
 * after synchronising every A[i]'s stream.  The autotuner (options 0) times
 * short trials of candidate configurations (workgroups, SpMV group rows, size
 * split) on copies of x0 and remembers the choice for the batch shape (count,
 * total rows, total nonzeros).  info (host, may be NULL) receives the
 * configuration and times.
 */
int mpcg_solve_batched(int32_t nsys, mpcg_matrix *const *A, const double *const *b, double *const *x,
                       const double *tol, const int32_t *maxit, const mpcg_batch_opts *opts,
                       mpcg_result *res, mpcg_batch_info *info);

/* ---------------------------------------------------------------- training
 * Tabular Q-learning over many systems (section 4.1, Algorithm 1): episodes run
 * one after the other, each a full solve from x0 = 0 (section 4.2's start) with
 * the epsilon-greedy training policy P, which updates its device Q-table (and
 * logs rollouts if enabled) inside the solve.  Episode j (0-based, in the order
 * below) has the number e = first_episode + j, which seeds its exploration
 * draws, and epsilon_e = eps_start + (eps_end - eps_start) (e - 1) / (E_total - 1)
 * (E_total = 1: eps_start), a linear schedule from eps_start to eps_end.
 */
typedef struct {
    int32_t episodes;          /* E >= 1 episodes per system                     */
    int32_t maxit;             /* iteration budget of an episode (T_max)         */
    double tol;                /* convergence threshold of an episode (> 0)      */
    double eps_start, eps_end; /* epsilon schedule, both in [0, 1]               */
    int32_t order;             /* 0: all episodes of system 0, then system 1 ...
                                  1: sweeps: episode 1 of every system, then 2 ... */
    int32_t first_episode;     /* number of the first episode (>= 1)             */
    int32_t total_episodes;    /* E_total of the schedule (0: first_episode - 1 +
                                  m * episodes, i.e. this call's last episode)   */
    int32_t reserved;
} mpcg_train_desc;

typedef struct {
    int32_t system;            /* index into A[]                                  */
    int32_t episode;           /* episode number e                                */
    double epsilon;            /* epsilon_e                                       */
    mpcg_result res;           /* the episode's solve                             */
} mpcg_episode_result;

/*
 * Trains P (kind MPCG_POLICY_QTABLE_TRAIN) on m systems: A[i] with device
 * right-hand side b[i] and device solution buffer x[i] (double[n_i], zeroed by
 * the call before each episode of system i).  Each system keeps its own solve
 * options (replacement period, fallback); its attached policy is restored
 * afterwards.  out (host, may be NULL) receives m * episodes records in episode
 * order.  Errors as mpcg_solve; invalid descriptors give MPCG_ERR_INVALID.
 */
int mpcg_train_qlearning(mpcg_policy *P, int32_t m, mpcg_matrix *const *A, const double *const *b,
                         double *const *x, const mpcg_train_desc *desc, mpcg_episode_result *out);

/* ---------------------------------------------------------------- MLP trainer
 * The MLP policy's network (16 features -> 128 -> 128 -> 64 action values,
 * GELU) trained by fitted Q-iteration, the function-approximation form of the
 * Q-learning update of section 4.1: per epoch the targets
 *   y_t = r_t + gamma (1 - done_t) max_a Q_frozen(s_{t+1}, a)
 * come from the weights frozen at the epoch's start; each batch then takes one
 * Adam step (fp32 master weights) on mean 1/2 (Q(s_t, a_t) - y_t)^2.  The
 * products run on bfloat16 matrix cores with fp32 accumulation.  Parameters
 * are float[26944] in the order W1[128][16] | b1[128] | W2[128][128] | b2[128]
 * | W3[64][128] | b3[64] (W[out][in], row-major).  Data arrays are device
 * pointers: feat, next float[n][16], act int32[n] (0..63), rew float[n],
 * done uint8[n].
 */
typedef struct mpcg_mlp mpcg_mlp;

typedef struct {
    int32_t batch;             /* samples per Adam step, a multiple of 64       */
    int32_t epochs;            /* passes over the floor(n / batch) batches, in
                                  the order given                                */
    double lr, beta1, beta2, eps;   /* Adam (1e-3, 0.9, 0.999, 1e-8)            */
    double gamma;              /* discount of the targets (section 4.1: 0.9)    */
} mpcg_mlp_train_desc;

/* Creates a network with the given initial parameters (host array), its Adam
 * state zeroed; runs on `stream` (hipStream_t, NULL: default stream). */
int mpcg_mlp_create(const float *params, void *stream, mpcg_mlp **out);
int mpcg_mlp_destroy(mpcg_mlp *net);
/* Replaces the parameters (host array) and zeroes the Adam state. */
int mpcg_mlp_set_params(mpcg_mlp *net, const float *params);
/* Copies the fp32 master parameters to host memory. */
int mpcg_mlp_get_params(mpcg_mlp *net, float *params_out);
/* logits[n][64] (device) = the training forward pass (bfloat16 matrix cores)
 * of feat[n][16] (device) with the current weights. */
int mpcg_mlp_forward(mpcg_mlp *net, const float *feat, int32_t n, float *logits);
/* Gradient of the loss over one batch of B samples (B a multiple of 64;
 * device feat, act, target float[B]) for the current weights, no update: grad
 * (host float[26944]) and *loss (host). */
int mpcg_mlp_grad(mpcg_mlp *net, const float *feat, const int32_t *act, const float *target, int32_t B,
                  float *grad, float *loss);
/* Trains on n rollouts; epoch_loss (host float[epochs], may be NULL) receives
 * each epoch's mean batch loss. */
int mpcg_mlp_train(mpcg_mlp *net, const float *feat, const float *next, const int32_t *act, const float *rew,
                   const uint8_t *done, int32_t n, const mpcg_mlp_train_desc *desc, float *epoch_loss);
/* Gives P (kind MPCG_POLICY_MLP) the network's weights for the decision path:
 * weights rounded to bfloat16, biases fp32. */
int mpcg_policy_set_mlp_from(mpcg_policy *P, mpcg_mlp *net);

/*
 * History of the last solve, host arrays (any may be NULL):
 *   rho[cap]     relative residual rho_k, k = 0..iters (the true one where replaced)
 *   act[cap]     action of iteration k, k = 0..iters-1
 *   flags[cap]   MPCG_FLAG_* of iteration k
 *   rep_k[rep_cap], rep_rho[rep_cap]  iteration and true relres of each replacement
 * n_hist (host int32, may be NULL) receives iters+1.
 */
int mpcg_get_history(mpcg_matrix *A, double *rho, uint8_t *act, uint8_t *flags, int32_t cap,
                     int32_t *rep_k, double *rep_rho, int32_t rep_cap, int32_t *n_hist);

/* ---------------------------------------------------------------- single ops
 * The hot-path kernels one at a time, on the handle's stream (device pointers).
 * p, q, u, v, y are float[n] (tier64 = 0) or double[n] (tier64 = 1).
 */
/* q = SpMV_f(A, p): row fma chain in CSR order, accumulated in fp32 (f != 3) or
 * fp64 (f = 3), output rounded to the tier; f = MPCG_Q52 reads the q52 shadow,
 * f = MPCG_TF32 the tf32 shadow. */
int mpcg_op_spmv(mpcg_matrix *A, int fmt, int tier64, const void *p, void *q);
/* *out (host) = dot_f(u, v): operands rounded to f, products in the accumulation
 * format, pairwise sum over the zero-padded power-of-two length; f is one of
 * the four arithmetic formats or MPCG_TF32 (fp32 accumulation). */
int mpcg_op_dot(mpcg_matrix *A, int fmt, int tier64, const void *u, const void *v, double *out);
/*
 * mpcg_op_dot without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same kernels and result as mpcg_op_dot, but the block
 * partials live in one static device array of the library (512 KiB per device,
 * held until the process ends) and the result is written to out, a device
 * double; nothing is synchronised: the result is ready when the handle's
 * stream reaches it.  Limit: n <= 65536 * 2048 = 134,217,728 elements, else
 * MPCG_ERR_INVALID before any launch.  Every call on one device shares that
 * array, so calls that overlap on one device (several streams, several host
 * threads) race and must be serialised by the caller.
 */
int mpcg_op_dot_noalloc(mpcg_matrix *A, int fmt, int tier64, const void *u, const void *v, double *out);
/* y = rd_f(fma(alpha, u, y)) (tier of f; MPCG_TF32: fp32 containers) */
int mpcg_op_axpy(mpcg_matrix *A, int fmt, double alpha, const void *u, void *y);
/* r (double[n], device) = b - A x in fp64 */
int mpcg_op_residual(mpcg_matrix *A, const double *b, const double *x, double *r);

/*
 * Measurement of the SpMV's random-access floor for this matrix: a flat pass
 * over its CSR entries that streams the int32 column indices and bf16 values
 * (coalesced) and gathers p[col] for every entry, eight independent gathers in
 * flight per thread, with no row structure and no output.  An SpMV over the
 * same columns cannot gather faster.  p: device float[n].  Launched
 * 2 + repeats times on the handle's stream; *us_per_launch (host) receives the
 * mean of the last `repeats` launches (HIP events).
 */
int mpcg_gather_floor(mpcg_matrix *A, const float *p, int32_t repeats, double *us_per_launch);

/* Copies the per-kernel timing of the last profiled solve (zeros otherwise). */
int mpcg_get_profile(mpcg_matrix *A, mpcg_profile *out);

const char *mpcg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MPCG_H */
