/*
 * mpcg_oracle.c -- CPU oracle for the mixed-precision conjugate-gradient hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU library shares no
 * code, header, table or constant with it.
 *
 * Plain, slow, single-threaded C.  fp64 is native double; fp32 arithmetic is
 * native float with fmaf (C99: one rounding); fp16 and bf16 occur only as
 * roundings of fp32/fp64 values (orc_rd), never as arithmetic formats, because
 * every fp16/bf16 operation of the method accumulates in fp32.
 *
 * What is computed (paper: section 3, eqs. for x, r, p, alpha, beta; section 4.2
 * for the four precision-controlled operations; section 4.1 for the MDP;
 * Algorithms 1 and 2 for the training and inference loops).  The paper leaves the
 * following open, and this oracle fixes them (each reading is listed, with its
 * reason, in the design notes of the repository):
 *
 *   formats   f in {0 fp16, 1 bf16, 2 fp32, 3 fp64}   (Table 1 parameters)
 *   acc(f)    fp32 for f <= 2, fp64 for f = 3
 *   tier(f)   storage of the vectors r, p, q, x_lo: fp64 if f = 3 else fp32
 *   action    a = 16 f_s + 4 f_d + f_a : precisions of SpMV, dot, axpy
 *
 *   SpMV_f    q_i = rd_tier( 2^{e_i} * acc ), acc = fma chain over the row in CSR
 *             order in acc(f) of (A_f[k], p[col[k]] read in acc(f)); A_f is the
 *             fp64 matrix rounded to f; for fp16 each row is first scaled by the
 *             exact power of two 2^{-e_i} that puts its largest magnitude in
 *             (2^14, 2^15]  (e_i = 0 for every other format)
 *   dot_f     sum over i of rd_acc( rd_f(u_i) * rd_f(v_i) ), the sum taken in
 *             acc(f) as a pairwise (recursive halving) sum over the vector
 *             zero-padded to the next power of two; ORDER_SEQ instead takes the
 *             fma chain in ascending i
 *   axpy_f    y_i = rd_f( fma_acc( rd_acc(alpha), u_i, y_i ) ), kept in tier(f)
 *   residual  r64_i = b_i - (fma chain in fp64 of row i of A times x_hi)
 *
 *   Iteration (unpreconditioned, M = I; reliable-update mixed CG):
 *     bnorm = sqrt(dot64(b,b)); x_hi = x0; x_lo = 0
 *     r64 = residual(x_hi); sigma = dot64(r64,r64); rho_0 = sqrt(sigma)/bnorm
 *     stop if rho_0 <= tol
 *     a_0 = policy(state(0, rho_0, 0)); r = rd_tier(a_0)(r64); p = r
 *     loop over k:
 *       q = SpMV_fs(p); nu = dot_fd(p,q)
 *       breakdown if not (nu > 0 and finite) or alpha = sigma/nu not finite
 *       x_lo = axpy_fa(alpha, p, x_lo); r = axpy_fa(-alpha, q, r)
 *       sigma' = dot_fd(r,r); k += 1; rho' = sqrt(sigma')/bnorm
 *       replacement when (R > 0 and k mod R == 0) or rho' <= tol or sigma' not
 *       finite:  x_hi += x_lo; x_lo = 0; r64 = residual(x_hi);
 *                sigma64 = dot64(r64,r64); rho_true = sqrt(sigma64)/bnorm
 *                converged if rho_true <= tol; breakdown if it is not finite;
 *                otherwise r = rd_tier(r64), sigma' = sigma64, rho' = rho_true;
 *                stagnation if rho_true >= the value two replacements earlier
 *       stag = k >= W and rho' >= rho_{k-W};  s' = state(k, rho', stag)
 *       training: Q update of (s, a) toward R + gamma max Q(s', .)
 *       stop at k = maxit
 *       beta = sigma'/sigma (breakdown if not finite); p = axpy_fa(beta, p, r)
 *       sigma = sigma'; a' = policy(s'); if tier changes:
 *         x_hi += x_lo; x_lo = 0; r, p rounded to the new tier
 *     fallback (optional): on breakdown or stagnation, once per solve, fold x_lo
 *     into x_hi and restart as plain fp64 CG (fixed action 63) from x_hi.
 *
 *   emulate (the paper's reading of fl_p(op)): every operation computes in
 *   fp64 and rounds its result to its format (SpMV: each q_i; dots: the
 *   total; updates and the preconditioner solve: each element); r, p, q and
 *   x_lo are fp64 vectors, so there is no tier switch.
 *
 *   vec16: with f_a = bf16 the vectors r, p and x_lo are held in bf16
 *   containers (16-bit vector storage); the updates already round them to
 *   bf16, so the only change is at a start, replacement or tier switch, where
 *   r and p are rounded to bf16 instead of fp32.  q stays fp32.
 *
 *   rho_fp64 (section 1 keeps residual computations in fp64): rho' =
 *   sqrt(dot64(r,r))/bnorm of the recursive r, while sigma' (beta's
 *   numerator) stays dot_fd(r,r).
 *
 *   Preconditioned variant (section 3 with M != I; Jacobi M = diag(A), its
 *   inverse kept in fp32): z = rd_fa(m * r) in acc(f_a); sigma = r^T z at f_d
 *   (rho still from r^T r); at a start or replacement sigma = r64^T (m r64)
 *   in fp64; p_0 = z_0; p = axpy_fa(beta, p, z); breakdown also when
 *   sigma' <= 0.  A replacement restarts the direction (p = z, beta = 0): the
 *   preconditioned recursion converges within a few iterations, far below the
 *   true residual of a low-precision matrix, and keeping p across that gap
 *   makes beta blow up; restarted, the solve is an fp64-residual iterative
 *   refinement around low-precision PCG.
 *
 *   Folding x_hi += x_lo is elementwise and skips an element whose sum is not
 *   finite, so a blown-up low-precision increment never destroys x_hi.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define F16 0
#define BF16 1
#define F32 2
#define F64 3
#define Q52 4   /* Table 1's quarter precision: 5 exponent bits, t = 3 (the printed
                   t is garbled; u = 2^-3 = 0.125 as printed fixes it); used
                   only as the SpMV's matrix storage */
#define TF32 5  /* tf32, in section 5's format set but not in Table 1: fp32's
                   exponent range (e_min -126, e_max 127) with fp16's 11-bit
                   significand; values are held in fp32 containers */
#define NFMT 6

/* Table 1: significand bits t (with the implicit bit), e_min, e_max. */
static const int FMT_T[NFMT] = {11, 8, 24, 53, 3, 11};
static const int FMT_EMIN[NFMT] = {-14, -126, -126, -1022, -14, -126};
static const int FMT_EMAX[NFMT] = {15, 127, 127, 1023, 15, 127};

/* Actions.  0..63: 16 f_s + 4 f_d + f_a over {fp16, bf16, fp32, fp64};
 * 64..79: a q52 SpMV with 4 f_d + f_a; 128..252: 128 + 25 d_s + 5 d_d + d_a
 * over the digits {0: fp16, 1: bf16, 2: fp32, 3: fp64, 4: tf32} (an action
 * without a tf32 digit keeps its 0..63 code). */
static int dig_fmt(int d) { return d == 4 ? TF32 : d; }
static int fmt_dig(int f) { return f == TF32 ? 4 : f; }
static int act_fs(int a) { return a < 64 ? (a >> 4) & 3 : a < 80 ? Q52 : dig_fmt((a - 128) / 25); }
static int act_fd(int a) { return a < 80 ? (a >> 2) & 3 : dig_fmt(((a - 128) / 5) % 5); }
static int act_fa(int a) { return a < 80 ? a & 3 : dig_fmt((a - 128) % 5); }
static int act_compose(int ds, int dd, int da)
{
    if (ds == 4 || dd == 4 || da == 4) return 128 + 25 * ds + 5 * dd + da;
    return 16 * ds + 4 * dd + da;
}
int orc_act_decode(int a, int *fs, int *fd, int *fa)
{
    *fs = act_fs(a); *fd = act_fd(a); *fa = act_fa(a);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Rounding (section 4: fl_p(x) = x(1+delta), |delta| <= u_p; Table 1).      */
/* Round-to-nearest-even of the fp64 value x to format f, gradual underflow,  */
/* overflow to infinity, NaN and infinities passed through.                  */
/* ------------------------------------------------------------------------ */
double orc_rd(double x, int f)
{
    if (f == F64 || !isfinite(x) || x == 0.0)
        return x;
    int e2;
    (void)frexp(x, &e2);              /* |x| = m 2^e2, 0.5 <= m < 1 */
    int E = e2 - 1;                   /* floor(log2 |x|) */
    if (E < FMT_EMIN[f])
        E = FMT_EMIN[f];              /* subnormal range: fixed quantum */
    double quantum = ldexp(1.0, E - (FMT_T[f] - 1));
    double y = nearbyint(x / quantum) * quantum;   /* exact scaling, RNE */
    double xmax = ldexp(2.0 - ldexp(1.0, 1 - FMT_T[f]), FMT_EMAX[f]);
    if (fabs(y) > xmax)
        return copysign(INFINITY, x);
    return y;
}

void orc_rd_array(const double *x, double *y, int64_t n, int f)
{
    for (int64_t i = 0; i < n; ++i)
        y[i] = orc_rd(x[i], f);
}

/* Vector containers ("tiers"): 0 fp32, 1 fp64, 2 bf16 (vec16: updates in
 * bf16 keep r, p and x_lo in 16-bit containers; q stays fp32). */
static double rd_tier(double x, int tier) { return tier == 1 ? x : orc_rd(x, tier == 2 ? BF16 : F32); }
static int tier_of(int f, int vec16) { return f == F64 ? 1 : (vec16 && f == BF16) ? 2 : 0; }

/* fp16 row exponent: e with max|a| * 2^-e in (2^14, 2^15], clamped to int8. */
int orc_row_exp(const double *v, int64_t len)
{
    double mx = 0.0;
    for (int64_t k = 0; k < len; ++k)
        if (fabs(v[k]) > mx)
            mx = fabs(v[k]);
    if (!(mx > 0.0) || !isfinite(mx))
        return 0;
    int e2;
    double m = frexp(mx, &e2);          /* mx = m 2^e2 */
    int c = (m == 0.5) ? e2 - 1 : e2;   /* ceil(log2 mx) */
    int e = c - 15;
    if (e < -128) e = -128;
    if (e > 127) e = 127;
    return e;
}

/* ------------------------------------------------------------------------ */
/* Matrix with its low-precision shadows.                                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    const int32_t *row_ptr;
    const int32_t *col;
    const double *val;       /* fp64 */
    double *sh[NFMT];        /* sh[f][k]: value used by SpMV_f (fp16 and q52 scaled) */
    int32_t *e;              /* row exponents of the fp16 and q52 shadows */
} orc_mat;

static void mat_build(orc_mat *A, int64_t n, const int32_t *rp, const int32_t *ci, const double *v)
{
    int64_t nnz = rp[n];
    A->n = n; A->row_ptr = rp; A->col = ci; A->val = v;
    for (int f = 0; f < NFMT; ++f)
        A->sh[f] = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    A->e = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        int64_t s = rp[i], t = rp[i + 1];
        int e = orc_row_exp(v + s, t - s);
        A->e[i] = e;
        for (int64_t k = s; k < t; ++k) {
            A->sh[F64][k] = v[k];
            A->sh[F32][k] = orc_rd(v[k], F32);
            A->sh[BF16][k] = orc_rd(v[k], BF16);
            A->sh[F16][k] = orc_rd(ldexp(v[k], -e), F16);
            /* q52 shares the fp16 exponent range, so the same row scale keeps
               the row's largest magnitude below its x_max */
            A->sh[Q52][k] = orc_rd(ldexp(v[k], -e), Q52);
            A->sh[TF32][k] = orc_rd(v[k], TF32);    /* fp32's range: no scale */
        }
    }
}

static void mat_free(orc_mat *A)
{
    for (int f = 0; f < NFMT; ++f) free(A->sh[f]);
    free(A->e);
}

/* Shadows as stored by a conforming implementation (for parity of setup). */
void orc_shadows(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                 double *out_f32, double *out_bf16, double *out_f16, int32_t *out_e)
{
    orc_mat A;
    mat_build(&A, n, rp, ci, v);
    int64_t nnz = rp[n];
    memcpy(out_f32, A.sh[F32], sizeof(double) * (size_t)nnz);
    memcpy(out_bf16, A.sh[BF16], sizeof(double) * (size_t)nnz);
    memcpy(out_f16, A.sh[F16], sizeof(double) * (size_t)nnz);
    memcpy(out_e, A.e, sizeof(int32_t) * (size_t)n);
    mat_free(&A);
}

/* The tf32 shadow. */
void orc_shadow_tf32(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, double *out_tf32)
{
    orc_mat A;
    mat_build(&A, n, rp, ci, v);
    memcpy(out_tf32, A.sh[TF32], sizeof(double) * (size_t)rp[n]);
    mat_free(&A);
}

/* The q52 shadow (row-scaled values) and the row exponents. */
void orc_shadow_q52(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                    double *out_q52, int32_t *out_e)
{
    orc_mat A;
    mat_build(&A, n, rp, ci, v);
    memcpy(out_q52, A.sh[Q52], sizeof(double) * (size_t)rp[n]);
    memcpy(out_e, A.e, sizeof(int32_t) * (size_t)n);
    mat_free(&A);
}

/* SpMV at format fs; p holds values of tier `tier64`; q written in tier `tier64`. */
static void mat_spmv(const orc_mat *A, int fs, int tier64, const double *p, double *q)
{
    const double *a = A->sh[fs];
    for (int64_t i = 0; i < A->n; ++i) {
        int64_t s = A->row_ptr[i], t = A->row_ptr[i + 1];
        double row;
        if (fs == F64) {
            double acc = 0.0;
            for (int64_t k = s; k < t; ++k)
                acc = fma(a[k], p[A->col[k]], acc);
            row = acc;
        } else {
            float acc = 0.0f;
            for (int64_t k = s; k < t; ++k)
                acc = fmaf((float)a[k], (float)p[A->col[k]], acc);
            row = (double)acc;
        }
        if (fs == F16 || fs == Q52)
            row = ldexp(row, A->e[i]);
        q[i] = rd_tier(row, tier64);
    }
}

void orc_spmv(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
              int fs, int tier64, const double *p, double *q)
{
    orc_mat A;
    mat_build(&A, n, rp, ci, v);
    mat_spmv(&A, fs, tier64, p, q);
    mat_free(&A);
}

/* r64 = b - A x in fp64, the row product as an fma chain in CSR order. */
static void mat_residual(const orc_mat *A, const double *b, const double *x, double *r)
{
    for (int64_t i = 0; i < A->n; ++i) {
        double acc = 0.0;
        for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k)
            acc = fma(A->val[k], x[A->col[k]], acc);
        r[i] = b[i] - acc;
    }
}

void orc_residual(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                  const double *b, const double *x, double *r)
{
    orc_mat A;
    A.n = n; A.row_ptr = rp; A.col = ci; A.val = v;
    mat_residual(&A, b, x, r);
}

/* ------------------------------------------------------------------------ */
/* Inner products.                                                           */
/* ------------------------------------------------------------------------ */
#define ORDER_PAIRWISE 0
#define ORDER_SEQ 1

static double pw_sum(const double *leaf, int64_t lo, int64_t len, int64_t n, int acc32)
{
    if (lo >= n)
        return 0.0;                    /* all-padding subtree: +0 */
    if (len == 1)
        return leaf[lo];
    int64_t h = len / 2;
    double a = pw_sum(leaf, lo, h, n, acc32);
    double b = pw_sum(leaf, lo + h, h, n, acc32);
    return acc32 ? (double)((float)a + (float)b) : a + b;
}

static int64_t next_pow2(int64_t n)
{
    int64_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

double orc_dot(int64_t n, const double *u, const double *v, int fd, int order)
{
    int acc32 = fd != F64;
    if (order == ORDER_SEQ) {
        if (!acc32) {
            double acc = 0.0;
            for (int64_t i = 0; i < n; ++i) acc = fma(u[i], v[i], acc);
            return acc;
        }
        float acc = 0.0f;
        for (int64_t i = 0; i < n; ++i)
            acc = fmaf((float)orc_rd(u[i], fd), (float)orc_rd(v[i], fd), acc);
        return (double)acc;
    }
    double *leaf = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        if (acc32)
            leaf[i] = (double)((float)orc_rd(u[i], fd) * (float)orc_rd(v[i], fd));
        else
            leaf[i] = u[i] * v[i];
    }
    double s = pw_sum(leaf, 0, next_pow2(n), n, acc32);
    free(leaf);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Vector updates.                                                           */
/* ------------------------------------------------------------------------ */
/* y = rd_f(fma_acc(rd_acc(alpha), u, y)) */
void orc_axpy(int64_t n, double alpha, const double *u, double *y, int fa)
{
    if (fa == F64) {
        for (int64_t i = 0; i < n; ++i) y[i] = fma(alpha, u[i], y[i]);
        return;
    }
    float a32 = (float)alpha;
    for (int64_t i = 0; i < n; ++i)
        y[i] = orc_rd((double)fmaf(a32, (float)u[i], (float)y[i]), fa);
}

/* p = rd_f(fma_acc(rd_acc(beta), p, r)) */
static void xpay(int64_t n, double beta, const double *r, double *p, int fa)
{
    if (fa == F64) {
        for (int64_t i = 0; i < n; ++i) p[i] = fma(beta, p[i], r[i]);
        return;
    }
    float b32 = (float)beta;
    for (int64_t i = 0; i < n; ++i)
        p[i] = orc_rd((double)fmaf(b32, (float)p[i], (float)r[i]), fa);
}

void orc_xpay(int64_t n, double beta, const double *r, double *p, int fa) { xpay(n, beta, r, p, fa); }

static void fold(int64_t n, double *xhi, double *xlo)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = xhi[i] + xlo[i];
        if (isfinite(s)) xhi[i] = s;
        xlo[i] = 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Decimal logarithm for the reward (section 4.1, accuracy term).            */
/* ln x = e ln2 + 2 atanh(s), s = (m-1)/(m+1), m in [sqrt(1/2), sqrt(2)),      */
/* atanh(s) = s sum_j s^{2j}/(2j+1) (Taylor series, |s| < 0.172, 12 terms),    */
/* evaluated by Horner with fma.  Every step is an IEEE basic operation.     */
/* ------------------------------------------------------------------------ */
double orc_log10(double x)
{
    const double LN2 = 0.693147180559945309417232121458176568;
    const double LOG10E = 0.434294481903251827651128918916605082;
    const double SQRT_HALF = 0.707106781186547524400844362104849039;
    if (!(x > 0.0) || !isfinite(x))
        return NAN;
    int e;
    double m = frexp(x, &e);            /* x = m 2^e, m in [0.5, 1) */
    if (m < SQRT_HALF) {
        m = m * 2.0;
        e = e - 1;
    }
    double s = (m - 1.0) / (m + 1.0);
    double s2 = s * s;
    double h = 1.0 / 23.0;
    for (int j = 10; j >= 0; --j)
        h = fma(h, s2, 1.0 / (double)(2 * j + 1));
    double ln = fma((double)e, LN2, 2.0 * s * h);
    return ln * LOG10E;
}

/* ------------------------------------------------------------------------ */
/* Counter-based uniform draws: the SplitMix64 output function (Steele, Lea   */
/* and Flood, OOPSLA 2014) chained over (seed, episode, iteration, stream).  */
/* ------------------------------------------------------------------------ */
static uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t orc_mix64(uint64_t z) { return mix64(z); }

double orc_uniform(uint64_t seed, uint64_t episode, uint64_t k, uint64_t stream)
{
    uint64_t h = mix64(seed);
    h = mix64(h ^ episode);
    h = mix64(h ^ k);
    h = mix64(h ^ stream);
    return (double)(h >> 11) * 0x1.0p-53;
}

/* ------------------------------------------------------------------------ */
/* Policy: state, decision, reward, Q-learning (section 4.1, Algorithms 1-2). */
/* ------------------------------------------------------------------------ */
#define POL_FIXED 0
#define POL_QTABLE 1
#define POL_QTRAIN 2
#define POL_MLP 3

#define N_ACT 64
#define MLP_IN 16
#define MLP_H 128

typedef struct {
    int32_t kind;
    int32_t fixed_action;
    int32_t t_bin, b_it, b_res, w_stag;
    double res_edges[16];    /* b_res - 1 thresholds, decreasing */
    double *q;               /* [n_states][64] */
    double lr, gamma, w1, w2, w3, eps_min;
    double cost[4];          /* c(fp16), c(bf16), c(fp32), c(fp64) */
    double epsilon;
    uint64_t seed;
    int64_t episode;
    /* MLP policy: fp32 weights (bf16-representable) */
    const float *w1m, *b1m, *w2m, *b2m, *w3m, *b3m;
    int32_t replace_period;  /* R, used by the MLP features */
    int32_t decision_period; /* D: the policy acts every D iterations (0, 1: every one) */
    int32_t per_op;          /* 1: one Q-table per operation (section 4.1) in row[4 j + p];
                                2: tables for SpMV and dot only, updates in fp64
                                (section 4.2: the residual update in full precision) */
    int32_t nfmt;            /* formats per operation table: 4, or 5 with tf32
                                (digit 4; per-operation tables only) */
    double cost_tf32;        /* c(tf32) */
} orc_policy;

int orc_n_states(const orc_policy *pol) { return pol->b_res * pol->b_it * 2; }

int orc_state(const orc_policy *pol, int64_t k, double rho, int stag)
{
    int64_t width = (pol->t_bin + pol->b_it - 1) / pol->b_it;
    int64_t i = k / width;
    if (i > pol->b_it - 1) i = pol->b_it - 1;
    int j = 0;
    for (int t = 0; t < pol->b_res - 1; ++t)
        if (rho <= pol->res_edges[t]) j++;
    return (int)((j * pol->b_it + i) * 2 + (stag ? 1 : 0));
}

static int argmax_row(const double *row)
{
    int best = 0;
    for (int a = 1; a < N_ACT; ++a)
        if (row[a] > row[best]) best = a;
    return best;
}

static double max_row(const double *row) { return row[argmax_row(row)]; }

/* Separate Q-tables per operation (section 4.1: Q_j over states x precisions,
 * j = SpMV, dot, update), held in one table row per state: Q_j(s, d) =
 * q[s][S j + d] with S = nfmt formats per table and d the format digit.  The
 * greedy action takes each operation's argmax (lowest digit among ties). */
static int n_fmt(const orc_policy *pol) { return pol->nfmt == 5 ? 5 : 4; }

static int argmax_n(const double *t, int S)
{
    int best = 0;
    for (int p = 1; p < S; ++p)
        if (t[p] > t[best]) best = p;
    return best;
}

static int greedy_row(const orc_policy *pol, const double *row)
{
    if (!pol->per_op) return argmax_row(row);
    const int S = n_fmt(pol);
    return act_compose(argmax_n(row, S), argmax_n(row + S, S), pol->per_op == 2 ? F64 : argmax_n(row + 2 * S, S));
}

/* Q update of the decision (s, a) toward reward R, bootstrapped from state
 * s_next (s_next < 0: terminal).  With one table per operation each Q_j is
 * updated toward R + gamma max_p Q_j(s', p) (the paper's per-table update). */
static void q_learn(orc_policy *pol, int s, int a, double R, int s_next)
{
    if (!pol->per_op) {
        double t = s_next < 0 ? R : R + pol->gamma * max_row(&pol->q[s_next * N_ACT]);
        double *qsa = &pol->q[s * N_ACT + a];
        *qsa = *qsa + pol->lr * (t - *qsa);
        return;
    }
    const int S = n_fmt(pol);
    const int dj[3] = {fmt_dig(act_fs(a)), fmt_dig(act_fd(a)), fmt_dig(act_fa(a))};
    for (int j = 0; j < (pol->per_op == 2 ? 2 : 3); ++j) {
        double t = R;
        if (s_next >= 0) {
            const double *nx = &pol->q[s_next * N_ACT + S * j];
            t = R + pol->gamma * nx[argmax_n(nx, S)];
        }
        double *qsa = &pol->q[s * N_ACT + S * j + dj[j]];
        *qsa = *qsa + pol->lr * (t - *qsa);
    }
}

/* Cost of an action: c(f_s) + c(f_d) + c(f_a).  The cost settings give no
 * value for q52 (actions 64..79); it is charged as fp16. */
static double cost_fmt(const orc_policy *pol, int f)
{
    return f == TF32 ? pol->cost_tf32 : f == Q52 ? pol->cost[F16] : pol->cost[f];
}

static double cost_of(const orc_policy *pol, int a)
{
    return (cost_fmt(pol, act_fs(a)) + cost_fmt(pol, act_fd(a))) + cost_fmt(pol, act_fa(a));
}

/* Reward of one decision (section 4.1) whose action ran n_it iterations: the
 * accuracy term at the residual rho' after them, the cost of the n_it
 * iterations, the convergence bonus.  n_it = 1 is the paper's per-iteration
 * reward. */
static double reward(const orc_policy *pol, int a, double rho, int converged, int64_t n_it)
{
    double accterm = (rho <= pol->eps_min) ? -orc_log10(pol->eps_min) : -orc_log10(rho);
    double r = pol->w1 * accterm - pol->w2 * (cost_of(pol, a) * (double)n_it);
    if (converged) r = r + pol->w3;
    return r;
}

double orc_reward(const orc_policy *pol, int a, double rho, int terminal)
{
    return reward(pol, a, rho, terminal, 1);
}


/* GELU, erf form, with erf from Abramowitz & Stegun 7.1.28 (rational, only + x /). */
static float gelu(float x)
{
    const float a1 = 0.0705230784f, a2 = 0.0422820123f, a3 = 0.0092705272f;
    const float a4 = 0.0001520143f, a5 = 0.0002765672f, a6 = 0.0000430638f;
    float z = x * 0.70710678118654752f;
    float t = fabsf(z);
    float poly = fmaf(fmaf(fmaf(fmaf(fmaf(a6, t, a5), t, a4), t, a3), t, a2), t, a1);
    float d = fmaf(poly, t, 1.0f);
    float d2 = d * d, d4 = d2 * d2, d8 = d4 * d4, d16 = d8 * d8;
    float erfv = 1.0f - 1.0f / d16;
    if (z < 0.0f) erfv = -erfv;
    return 0.5f * x * (1.0f + erfv);
}

float orc_gelu(float x) { return gelu(x); }

static float rd_bf16f(float x) { return (float)orc_rd((double)x, BF16); }

/* MLP logits, decision path: fp32 fma chains in ascending input index. */
void orc_mlp_logits(const orc_policy *pol, const float *feat, float *logits)
{
    float x[MLP_IN], h1[MLP_H], h2[MLP_H];
    for (int i = 0; i < MLP_IN; ++i) x[i] = rd_bf16f(feat[i]);
    for (int j = 0; j < MLP_H; ++j) {
        float acc = 0.0f;
        for (int i = 0; i < MLP_IN; ++i) acc = fmaf(pol->w1m[j * MLP_IN + i], x[i], acc);
        h1[j] = rd_bf16f(gelu(acc + pol->b1m[j]));
    }
    for (int j = 0; j < MLP_H; ++j) {
        float acc = 0.0f;
        for (int i = 0; i < MLP_H; ++i) acc = fmaf(pol->w2m[j * MLP_H + i], h1[i], acc);
        h2[j] = rd_bf16f(gelu(acc + pol->b2m[j]));
    }
    for (int j = 0; j < N_ACT; ++j) {
        float acc = 0.0f;
        for (int i = 0; i < MLP_H; ++i) acc = fmaf(pol->w3m[j * MLP_H + i], h2[i], acc);
        logits[j] = acc + pol->b3m[j];
    }
}

static int argmax_f(const float *v, int n)
{
    int best = 0;
    for (int a = 1; a < n; ++a)
        if (v[a] > v[best]) best = a;
    return best;
}

/*
 * MLP features (16, fp32) of the state at iteration k: decimal logs of the last
 * eight relative residuals (index clamped at 0), the last one-step change, k over
 * the iteration-bin horizon, the stagnation flag, the decimal log of the last
 * true relative residual, the position inside the replacement period, and the
 * three formats of the previous action divided by 3.
 */
static double lg_clamped(const orc_policy *pol, double r)
{
    return (r <= pol->eps_min) ? orc_log10(pol->eps_min) : orc_log10(r);
}

void orc_mlp_features(const orc_policy *pol, int64_t k, const double *hist_rho, int stag,
                      double last_true, int prev_action, float *f)
{
    double lg[8];
    for (int i = 0; i < 8; ++i) {
        int64_t idx = k - i;
        if (idx < 0) idx = 0;
        lg[i] = lg_clamped(pol, hist_rho[idx]);
    }
    for (int i = 0; i < 8; ++i) f[i] = (float)lg[i];
    f[8] = (float)(lg[0] - lg[1]);
    f[9] = (float)((double)k / (double)pol->t_bin);
    f[10] = stag ? 1.0f : 0.0f;
    f[11] = (float)lg_clamped(pol, last_true);
    int R = pol->replace_period > 0 ? pol->replace_period : 1;
    f[12] = (float)((double)(k % R) / (double)R);
    f[13] = (float)((double)((prev_action >> 4) & 3) / 3.0);
    f[14] = (float)((double)((prev_action >> 2) & 3) / 3.0);
    f[15] = (float)((double)(prev_action & 3) / 3.0);
}

/* ------------------------------------------------------------------------ */
/* The solver.                                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    double tol;
    int32_t maxit;
    int32_t replace_period;   /* R; 0 = replace only on the rho' <= tol trigger */
    int32_t fallback;
    int32_t dot_order;
    int32_t precond;          /* 0: M = I; 1: Jacobi, M = diag(A) */
    int32_t stop_rule;        /* 0: true fp64 relres <= tol at a replacement;
                                 1: the paper's, recursive rho < tol with k >= 10 */
    int32_t rho_fp64;         /* 1: rho' from dot64(r, r) of the recursive r
                                 (residual computations in fp64, section 1);
                                 sigma' stays dot_fd */
    int32_t emulate;          /* 1: the paper's emulation reading: every
                                 operation computes in fp64 and rounds its
                                 result to its format; vectors in fp64 */
    int32_t vec16;            /* 1: with bf16 updates, r, p and x_lo live in
                                 bf16 containers: a start, replacement or tier
                                 switch rounds r and p to bf16 (not fp32) */
} orc_params;

typedef struct {
    int32_t status;           /* 0 conv, 1 maxit, 2 conv after fallback, 3 breakdown */
    int32_t iters;
    int32_t n_replace;
    int32_t fallback_at;      /* k at fallback, -1 if none */
    double relres_true;
    double cost_sum;
} orc_result;

#define FL_REPLACED 1
#define FL_EXPLORED 2
#define FL_FALLBACK 4
#define FL_SWITCH 8

typedef struct {
    double *hist_rho;          /* [maxit+1] */
    uint8_t *hist_act;         /* [maxit] */
    uint8_t *hist_flag;        /* [maxit] */
    int32_t *rep_k;            /* [rep_cap] */
    double *rep_rho;           /* [rep_cap] */
    int32_t rep_cap;
    int32_t roll_cap;          /* rollout log capacity (0: no log) */
    float *roll_feat;          /* [roll_cap][16] features of s_k */
    float *roll_next;          /* [roll_cap][16] features of s_{k+1} */
    int32_t *roll_act;         /* [roll_cap] */
    float *roll_rew;           /* [roll_cap] */
    uint8_t *roll_done;        /* [roll_cap] */
    int32_t roll_n;            /* out: entries written */
    int32_t dump_cap;          /* iterations whose alpha, beta, p, r are dumped */
    double *hist_alpha;        /* [dump_cap] or NULL */
    double *hist_beta;         /* [dump_cap] or NULL */
    double *dump_p;            /* [dump_cap][n] direction used by iteration k, or NULL */
    double *dump_r;            /* [dump_cap][n] residual r at the start of iteration k, or NULL */
    double *dump_s;            /* single-reduction and pipelined CG: [dump_cap][n] s
                                  (the recurrence for A p) used by iteration k, or NULL */
    double *dump_w;            /* pipelined CG: [dump_cap][n] w (for A r) at the start
                                  of iteration k, or NULL */
    double *dump_z;            /* pipelined CG: [dump_cap][n] z (for A s) used by
                                  iteration k, or NULL */
} orc_hist;

/* Stagnation flag of the state (a reading: the paper's state has no such
 * component; the flag is set when the residual has not decreased over the
 * last W iterations): stag_k = [k >= W and rho_k >= rho_{k-W}], on the history
 * rho_0 .. rho_k. */
int orc_stag(const double *hist_rho, int64_t k, int W)
{
    return (k >= W) && (hist_rho[k] >= hist_rho[k - W]);
}

/* Stagnation of the true residual, the fallback trigger (a reading: the
 * paper only says runs stop on numerical instabilities): at the m-th
 * replacement since the last (re)start, m >= 3, the true relative residual
 * has not decreased over the last two replacement periods,
 * rho_true(m) >= rho_true(m-2).  last3 holds rho_true(m-2), rho_true(m-1),
 * rho_true(m) in that order. */
int orc_stagnated(int m, const double last3[3])
{
    return m >= 3 && last3[2] >= last3[0];
}

static int decide(const orc_policy *pol, int kind, const float *feat, int s, int64_t k, int *explored)
{
    *explored = 0;
    switch (kind) {
    case POL_FIXED:
        return pol->fixed_action;
    case POL_QTABLE:
        return greedy_row(pol, &pol->q[s * N_ACT]);
    case POL_QTRAIN: {
        if (pol->per_op) {       /* an epsilon-greedy draw per operation, streams 2 .. 7 */
            const double *row = &pol->q[s * N_ACT];
            const int S = n_fmt(pol);
            int d[3];
            for (int j = 0; j < 3; ++j) {
                if (j == 2 && pol->per_op == 2) {     /* updates fixed in fp64 */
                    d[j] = F64;
                    break;
                }
                double u0 = orc_uniform(pol->seed, (uint64_t)pol->episode, (uint64_t)k, (uint64_t)(2 + 2 * j));
                if (u0 < pol->epsilon) {
                    double u1 = orc_uniform(pol->seed, (uint64_t)pol->episode, (uint64_t)k, (uint64_t)(3 + 2 * j));
                    d[j] = (int)(u1 * (double)S);
                    *explored = 1;
                } else {
                    d[j] = argmax_n(row + S * j, S);
                }
            }
            return act_compose(d[0], d[1], d[2]);
        }
        double u0 = orc_uniform(pol->seed, (uint64_t)pol->episode, (uint64_t)k, 0);
        if (u0 < pol->epsilon) {
            double u1 = orc_uniform(pol->seed, (uint64_t)pol->episode, (uint64_t)k, 1);
            *explored = 1;
            return (int)(u1 * 64.0);
        }
        return argmax_row(&pol->q[s * N_ACT]);
    }
    case POL_MLP: {
        float logits[N_ACT];
        orc_mlp_logits(pol, feat, logits);
        return argmax_f(logits, N_ACT);
    }
    }
    return 63;
}

static void roll_log(orc_hist *h, const float *f, const float *fn, int a, double rew, int done)
{
    if (h->roll_cap <= 0 || h->roll_n >= h->roll_cap) return;
    int i = h->roll_n++;
    memcpy(&h->roll_feat[(int64_t)i * MLP_IN], f, sizeof(float) * MLP_IN);
    memcpy(&h->roll_next[(int64_t)i * MLP_IN], fn, sizeof(float) * MLP_IN);
    h->roll_act[i] = a;
    h->roll_rew[i] = (float)rew;
    h->roll_done[i] = (uint8_t)done;
}

/* Jacobi preconditioner (section 3: z = M^-1 r with M approximating A; section
 * 4.2: M is kept in fixed fp32).  M = diag(A), stored as its inverse
 * m_i = rd_fp32(1 / a_ii) (the fp64 quotient rounded to fp32); a row without
 * a diagonal entry gets m_i = 0. */
static float *jacobi_inverse(int64_t n, const int32_t *rp, const int32_t *ci, const double *v)
{
    float *m = malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        m[i] = 0.0f;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] == i) m[i] = (float)(1.0 / v[k]);
    }
    return m;
}

/* The preconditioner solve z = M^-1 r at the precision of the vector updates
 * (the paper's p2 slot is taken by f_a): the product m_i r_i in acc(f_a),
 * rounded to f_a. */
static void precond_apply(int64_t n, const float *m, const double *r, double *z, int fa)
{
    for (int64_t i = 0; i < n; ++i)
        z[i] = fa == F64 ? (double)m[i] * r[i] : orc_rd((double)(m[i] * (float)r[i]), fa);
}

/* The paper's emulation reading (section 4's fl_p(op), and its low-precision
 * emulation): an operation at format p computes in fp64 and rounds its result
 * to p.  The SpMV rounds each q_i (fp64 row fma chain, no row scale), a dot
 * rounds the fp64 pairwise total, an update rounds each fp64 fma, the
 * preconditioner solve rounds each m_i r_i.  The vectors stay in fp64. */
static void spmv_emul(const orc_mat *A, int fs, const double *p, double *q)
{
    mat_spmv(A, F64, 1, p, q);
    for (int64_t i = 0; i < A->n; ++i) q[i] = orc_rd(q[i], fs);
}

static double dot_emul(int64_t n, const double *u, const double *v, int fd, int order)
{
    return orc_rd(orc_dot(n, u, v, F64, order), fd);
}

static void axpy_emul(int64_t n, double alpha, const double *u, double *y, int fa)
{
    for (int64_t i = 0; i < n; ++i) y[i] = orc_rd(fma(alpha, u[i], y[i]), fa);
}

static void xpay_emul(int64_t n, double beta, const double *r, double *p, int fa)
{
    for (int64_t i = 0; i < n; ++i) p[i] = orc_rd(fma(beta, p[i], r[i]), fa);
}

static void precond_emul(int64_t n, const float *m, const double *r, double *z, int fa)
{
    for (int64_t i = 0; i < n; ++i) z[i] = orc_rd((double)m[i] * r[i], fa);
}

/* r64^T M^-1 r64 in fp64 (a start, restart or replacement). */
static double precond_dot64(int64_t n, const float *m, const double *r64, double *work, int order)
{
    for (int64_t i = 0; i < n; ++i) work[i] = (double)m[i] * r64[i];
    return orc_dot(n, r64, work, F64, order);
}

void orc_jacobi_inverse(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, float *out)
{
    float *m = jacobi_inverse(n, rp, ci, v);
    memcpy(out, m, sizeof(float) * (size_t)n);
    free(m);
}

int orc_cg(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
           const double *b, const double *x0, double *x_out,
           const orc_params *prm, orc_policy *pol, orc_result *res, orc_hist *h)
{
    orc_mat A;
    mat_build(&A, n, rp, ci, v);
    size_t bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *xhi = malloc(bytes), *xlo = malloc(bytes), *r = malloc(bytes);
    double *p = malloc(bytes), *q = malloc(bytes), *r64 = malloc(bytes), *z = malloc(bytes);
    const int pc = prm->precond;
    const int emul = prm->emulate;
    float *minv = pc ? jacobi_inverse(n, rp, ci, v) : NULL;
    double *hist_rho = h->hist_rho;
    const int W = pol->w_stag;
    const int R = prm->replace_period;

    memset(res, 0, sizeof(*res));
    res->fallback_at = -1;
    h->roll_n = 0;

    int64_t k = 0;
    int kind = pol->kind;          /* policy in force: FIXED 63 after fallback */
    int fell_back = 0, nrep = 0, nrep_since = 0, status = -1;
    double rep_hist[3] = {0.0, 0.0, 0.0};
    double sigma = 0.0, last_true = 0.0;
    int a = 63, s = 0, tier = 1, prev_a = 63, explored = 0;
    float feat[MLP_IN], feat_next[MLP_IN];
    /* decision period (a reading; 1 is the paper's per-iteration decision):
       the action chosen at iteration k_dec holds until the next multiple of D */
    const int64_t D = pol->decision_period > 1 ? pol->decision_period : 1;
    int64_t k_dec = 0;

    double bnorm = sqrt(orc_dot(n, b, b, F64, prm->dot_order));
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x_out[i] = 0.0;
        hist_rho[0] = 0.0;
        res->status = 0;
        goto out;
    }
    for (int64_t i = 0; i < n; ++i) { xhi[i] = x0[i]; xlo[i] = 0.0; }

    int restart = 1;
    for (;;) {
        if (restart) {            /* start, or restart after fallback */
            restart = 0;
            fold(n, xhi, xlo);
            mat_residual(&A, b, xhi, r64);
            double s64 = orc_dot(n, r64, r64, F64, prm->dot_order);
            double rt = sqrt(s64) / bnorm;
            hist_rho[k] = rt;
            last_true = rt;
            nrep_since = 0;
            if (rt <= prm->tol) { status = fell_back ? 2 : 0; break; }
            if (!isfinite(rt)) { status = 3; break; }
            sigma = pc ? precond_dot64(n, minv, r64, z, prm->dot_order) : s64;
            int stag = orc_stag(hist_rho, k, W);
            s = orc_state(pol, k, rt, stag);
            orc_mlp_features(pol, k, hist_rho, stag, last_true, prev_a, feat);
            a = fell_back ? 63 : decide(pol, kind, feat, s, k, &explored);
            if (fell_back) explored = 0;
            k_dec = k;
            tier = emul ? 1 : tier_of(act_fa(a), prm->vec16);
            for (int64_t i = 0; i < n; ++i) { r[i] = rd_tier(r64[i], tier); p[i] = r[i]; }
            if (pc) {                                           /* p_0 = z_0 */
                if (emul) precond_emul(n, minv, r, p, act_fa(a));
                else precond_apply(n, minv, r, p, act_fa(a));
            }
        }
        if (k >= prm->maxit) { status = 1; break; }

        const int fs = act_fs(a), fd = act_fd(a), fa = act_fa(a);
        const int policy_active = !fell_back;
        const int training = policy_active && kind == POL_QTRAIN;
        h->hist_act[k] = (uint8_t)a;
        h->hist_flag[k] = explored ? FL_EXPLORED : 0;
        res->cost_sum += cost_of(pol, a);

        if (k < h->dump_cap && h->dump_p) memcpy(&h->dump_p[k * n], p, bytes);
        if (k < h->dump_cap && h->dump_r) memcpy(&h->dump_r[k * n], r, bytes);
        if (emul) spmv_emul(&A, fs, p, q);
        else mat_spmv(&A, fs, tier == 1, p, q);
        double nu = emul ? dot_emul(n, p, q, fd, prm->dot_order) : orc_dot(n, p, q, fd, prm->dot_order);
        double alpha = sigma / nu;
        if (k < h->dump_cap && h->hist_alpha) h->hist_alpha[k] = alpha;
        int broke = !(nu > 0.0 && isfinite(nu)) || !isfinite(alpha);
        int converged = 0, stagnated = 0, dir_restart = 0;
        double sig_new = 0.0, rho_new = 0.0, beta = 0.0;
        int64_t kk = k;
        if (!broke) {
            if (emul) {
                axpy_emul(n, alpha, p, xlo, fa);
                axpy_emul(n, -alpha, q, r, fa);
            } else {
                orc_axpy(n, alpha, p, xlo, fa);
                orc_axpy(n, -alpha, q, r, fa);
            }
            double sig_rr = prm->rho_fp64 ? orc_dot(n, r, r, F64, prm->dot_order)
                            : emul ? dot_emul(n, r, r, fd, prm->dot_order) : orc_dot(n, r, r, fd, prm->dot_order);
            sig_new = !prm->rho_fp64 ? sig_rr
                      : emul ? dot_emul(n, r, r, fd, prm->dot_order) : orc_dot(n, r, r, fd, prm->dot_order);
            if (pc) {                                             /* sigma' = r^T z */
                if (emul) {
                    precond_emul(n, minv, r, z, fa);
                    sig_new = dot_emul(n, r, z, fd, prm->dot_order);
                } else {
                    precond_apply(n, minv, r, z, fa);
                    sig_new = orc_dot(n, r, z, fd, prm->dot_order);
                }
            }
            k += 1;
            rho_new = sqrt(sig_rr) / bnorm;
            /* section 5's termination: the recursive residual below tol after
               at least 10 iterations, with no true-residual check */
            const int paper_stop = prm->stop_rule == 1 && rho_new < prm->tol && k >= 10 && isfinite(sig_rr) &&
                                   isfinite(sig_new);
            if (paper_stop) {
                converged = 1;
            } else if ((R > 0 && k % R == 0) || (prm->stop_rule == 0 && rho_new <= prm->tol) || !isfinite(sig_rr) ||
                       !isfinite(sig_new)) {
                const double rho_rec = rho_new;
                fold(n, xhi, xlo);
                mat_residual(&A, b, xhi, r64);
                double s64 = orc_dot(n, r64, r64, F64, prm->dot_order);
                double rt = sqrt(s64) / bnorm;
                if (nrep < h->rep_cap) { h->rep_k[nrep] = (int32_t)k; h->rep_rho[nrep] = rt; }
                nrep++;
                h->hist_flag[kk] |= FL_REPLACED;
                last_true = rt;
                rho_new = rt;
                if (rt <= prm->tol) {
                    converged = 1;
                } else if (!isfinite(rt)) {
                    broke = 1;
                } else {
                    for (int64_t i = 0; i < n; ++i) r[i] = rd_tier(r64[i], tier);
                    sig_new = pc ? precond_dot64(n, minv, r64, z, prm->dot_order) : s64;
                    /* with M, a replacement that more than doubles the
                       residual restarts the direction: p = z */
                    dir_restart = pc && !(rt <= 2.0 * rho_rec);
                    rep_hist[0] = rep_hist[1]; rep_hist[1] = rep_hist[2]; rep_hist[2] = rt;
                    nrep_since++;
                    if (orc_stagnated(nrep_since, rep_hist)) stagnated = 1;
                }
            }
            hist_rho[k] = rho_new;
            if (!broke && !converged) {
                beta = dir_restart ? 0.0 : sig_new / sigma;
                /* with M: r^T M^-1 r > 0 for r != 0 */
                if (!isfinite(beta) || (pc && !(sig_new > 0.0))) broke = 1;
            }
        }

        int stag = 0, s_next = s;
        if (!broke) {
            stag = orc_stag(hist_rho, k, W);
            s_next = orc_state(pol, k, rho_new, stag);
            if (policy_active)
                orc_mlp_features(pol, k, hist_rho, stag, last_true, a, feat_next);
        } else if (policy_active) {
            memcpy(feat_next, feat, sizeof(feat));
        }

        /* iterations run under the current decision, the failed one included */
        const int64_t n_it = (k > kk ? k : k + 1) - k_dec;
        if (converged) {
            double rw = reward(pol, a, rho_new, 1, n_it);
            if (training) q_learn(pol, s, a, rw, -1);
            if (policy_active) roll_log(h, feat, feat_next, a, rw, 1);
            status = fell_back ? 2 : 0;
            break;
        }
        if (broke || (stagnated && prm->fallback && !fell_back)) {
            double rw = -pol->w2 * (cost_of(pol, a) * (double)n_it) - pol->w3;
            if (training) q_learn(pol, s, a, rw, -1);
            if (policy_active) roll_log(h, feat, feat_next, a, rw, 1);
            if (!prm->fallback || fell_back) { status = 3; break; }
            fell_back = 1;
            res->fallback_at = (int32_t)k;
            h->hist_flag[kk] |= FL_FALLBACK;
            kind = POL_FIXED;
            restart = 1;
            prev_a = a;
            continue;
        }
        /* a decision ends at a multiple of D, and when the budget cuts it */
        const int dec_end = (k % D == 0) || k >= prm->maxit;
        if (dec_end) {
            double rw = reward(pol, a, rho_new, 0, n_it);
            if (training) q_learn(pol, s, a, rw, s_next);
            if (policy_active) roll_log(h, feat, feat_next, a, rw, 0);
        }
        if (k >= prm->maxit) { status = 1; break; }

        if (kk < h->dump_cap && h->hist_beta) h->hist_beta[kk] = beta;
        if (pc) {                                                 /* p = z + beta p */
            if (emul) precond_emul(n, minv, r, z, fa);
            else precond_apply(n, minv, r, z, fa);
            if (dir_restart) memcpy(p, z, bytes);
            else if (emul) xpay_emul(n, beta, z, p, fa);
            else xpay(n, beta, z, p, fa);
        } else if (emul) {
            xpay_emul(n, beta, r, p, fa);
        } else {
            xpay(n, beta, r, p, fa);
        }
        sigma = sig_new;
        prev_a = a;
        if (dec_end) {
            s = s_next;
            memcpy(feat, feat_next, sizeof(feat));
            a = fell_back ? 63 : decide(pol, kind, feat, s, k, &explored);
            if (fell_back) explored = 0;
            k_dec = k;
        } else {
            explored = 0;                  /* the action holds */
        }
        int nt = emul ? 1 : tier_of(act_fa(a), prm->vec16);
        if (nt != tier) {
            fold(n, xhi, xlo);
            for (int64_t i = 0; i < n; ++i) { r[i] = rd_tier(r[i], nt); p[i] = rd_tier(p[i], nt); }
            tier = nt;
            h->hist_flag[kk] |= FL_SWITCH;
        }
    }

    fold(n, xhi, xlo);
    for (int64_t i = 0; i < n; ++i) x_out[i] = xhi[i];
    if ((status == 0 || status == 2) && prm->stop_rule == 0) {
        res->relres_true = last_true;
    } else {
        mat_residual(&A, b, xhi, r64);
        res->relres_true = sqrt(orc_dot(n, r64, r64, F64, prm->dot_order)) / bnorm;
    }
    res->status = status;
    res->iters = (int32_t)k;
    res->n_replace = nrep;
out:
    free(xhi); free(xlo); free(r); free(p); free(q); free(r64); free(z);
    free(minv);
    mat_free(&A);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Single-reduction CG (Chronopoulos and Gear, 1989).                        */
/* ------------------------------------------------------------------------ */
/* The CG iteration of section 3 rearranged so that both inner products of an
 * iteration are taken together, right after its one SpMV: with w = A r,
 *   gamma_k = r_k.r_k,  delta_k = r_k.w_k,
 *   beta_k  = gamma_k / gamma_{k-1}            (beta_0 = 0),
 *   alpha_k = gamma_k / (delta_k - beta_k gamma_k / alpha_{k-1})
 *                                              (alpha_0 = gamma_0 / delta_0),
 *   p_k = r_k + beta_k p_{k-1},  s_k = w_k + beta_k s_{k-1}   (s_k = A p_k),
 *   x_{k+1} = x_k + alpha_k p_k,  r_{k+1} = r_k - alpha_k s_k.
 * In exact arithmetic the iterates are those of section 3's CG.
 *
 * Precision (a fixed action, as in section 4.2's operation list): the SpMV
 * w = A r at f_s, both inner products at f_d, the four vector updates at f_a
 * (each element rounded to f_a, vectors held in fp32 or, for f_a = fp64, fp64
 * containers), alpha and beta in fp64, x = x_hi (fp64) + x_lo (f_a) as in the
 * main solver.  True-residual replacement (every R iterations, and when the
 * recursive rho_k = sqrt(gamma_k) / ||b|| is <= tol) folds x_lo into x_hi,
 * sets r = rd(b - A x_hi) and, before the next update, recomputes s = A p at
 * f_s (the replacement of the recurrences' vectors by their true values used
 * for pipelined CG by Cools et al., 2018).  Stops when the true fp64 relres
 * is <= tol at a replacement, after maxit iterations, or when
 * delta_k - beta_k gamma_k / alpha_{k-1} is not positive or a scalar is not
 * finite (breakdown).  No fallback and no policy: cost_sum is 0.
 * History: rho_k is the true relres at the start and at replacements, the
 * recursive one otherwise; act[k] is the action; FL_REPLACED marks the
 * iteration that ended at a replacement. */
int orc_cg_sr(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
              const double *b, const double *x0, double *x_out, int action,
              const orc_params *prm, orc_result *res, orc_hist *h)
{
    memset(res, 0, sizeof(*res));
    res->fallback_at = -1;
    h->roll_n = 0;
    if (action < 0 || action >= 80) return -1;           /* the 4-format set and q52 SpMV */
    orc_mat A;
    mat_build(&A, n, rp, ci, v);
    size_t bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *xhi = malloc(bytes), *xlo = malloc(bytes), *r = malloc(bytes), *w = malloc(bytes);
    double *p = malloc(bytes), *sv = malloc(bytes), *r64 = malloc(bytes);
    const int fs = act_fs(action), fd = act_fd(action), fa = act_fa(action);
    const int tier = fa == F64 ? 1 : 0;
    const int R = prm->replace_period;
    const int order = prm->dot_order;
    double *hist_rho = h->hist_rho;
    int64_t k = 0;
    int nrep = 0, status = -1;
    double gamma_old = 0.0, alpha_old = 0.0, last_true = 0.0;

    double bnorm = sqrt(orc_dot(n, b, b, F64, order));
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x_out[i] = 0.0;
        hist_rho[0] = 0.0;
        res->status = 0;
        goto out;
    }
    for (int64_t i = 0; i < n; ++i) { xhi[i] = x0[i]; xlo[i] = 0.0; }

    /* start: the true residual; the first pass then takes beta = 0 */
    mat_residual(&A, b, xhi, r64);
    last_true = sqrt(orc_dot(n, r64, r64, F64, order)) / bnorm;
    hist_rho[0] = last_true;
    if (last_true <= prm->tol) { status = 0; goto done; }
    if (!isfinite(last_true)) { status = 3; goto done; }
    if (prm->maxit <= 0) { status = 1; goto done; }
    for (int64_t i = 0; i < n; ++i) r[i] = rd_tier(r64[i], tier);
    int first = 1, sync = 1;     /* sync: the pass after a start or replacement */

    for (;;) {
        mat_spmv(&A, fs, tier, r, w);
        if (sync && !first) mat_spmv(&A, fs, tier, p, sv);   /* s = A p again */
        const double gamma = orc_dot(n, r, r, fd, order);
        const double delta = orc_dot(n, r, w, fd, order);
        int replace = 0;
        if (!sync) {
            const double rho = sqrt(gamma) / bnorm;
            hist_rho[k] = rho;
            if (rho <= prm->tol) replace = 1;                 /* check it */
            else if (k >= prm->maxit) { status = 1; break; }
        }
        if (!replace) {
            sync = 0;
            const double beta = first ? 0.0 : gamma / gamma_old;
            const double den = first ? delta : delta - beta * gamma / alpha_old;
            const double alpha = gamma / den;
            if (!(den > 0.0) || !isfinite(alpha) || !isfinite(beta) || !isfinite(gamma)) { status = 3; break; }
            if (k < h->dump_cap && h->hist_alpha) h->hist_alpha[k] = alpha;
            if (k < h->dump_cap && h->hist_beta) h->hist_beta[k] = beta;
            if (first) {
                memcpy(p, r, bytes);
                memcpy(sv, w, bytes);
            } else {
                xpay(n, beta, r, p, fa);
                xpay(n, beta, w, sv, fa);
            }
            if (k < h->dump_cap && h->dump_p) memcpy(&h->dump_p[k * n], p, bytes);
            if (k < h->dump_cap && h->dump_r) memcpy(&h->dump_r[k * n], r, bytes);
            if (k < h->dump_cap && h->dump_s) memcpy(&h->dump_s[k * n], sv, bytes);
            orc_axpy(n, alpha, p, xlo, fa);
            orc_axpy(n, -alpha, sv, r, fa);
            h->hist_act[k] = (uint8_t)action;
            h->hist_flag[k] = 0;
            gamma_old = gamma;
            alpha_old = alpha;
            first = 0;
            k += 1;
            replace = R > 0 && k % R == 0;
        }
        if (replace) {
            fold(n, xhi, xlo);
            mat_residual(&A, b, xhi, r64);
            const double rt = sqrt(orc_dot(n, r64, r64, F64, order)) / bnorm;
            if (nrep < h->rep_cap) { h->rep_k[nrep] = (int32_t)k; h->rep_rho[nrep] = rt; }
            nrep++;
            if (k > 0) h->hist_flag[k - 1] |= FL_REPLACED;
            hist_rho[k] = rt;
            last_true = rt;
            if (rt <= prm->tol) { status = 0; break; }
            if (!isfinite(rt)) { status = 3; break; }
            if (k >= prm->maxit) { status = 1; break; }
            for (int64_t i = 0; i < n; ++i) r[i] = rd_tier(r64[i], tier);
            sync = 1;
        }
    }
done:
    fold(n, xhi, xlo);
    for (int64_t i = 0; i < n; ++i) x_out[i] = xhi[i];
    if (status == 0) {
        res->relres_true = last_true;
    } else {
        mat_residual(&A, b, xhi, r64);
        res->relres_true = sqrt(orc_dot(n, r64, r64, F64, order)) / bnorm;
    }
    res->status = status;
    res->iters = (int32_t)k;
    res->n_replace = nrep;
out:
    free(xhi); free(xlo); free(r); free(w); free(p); free(sv); free(r64);
    mat_free(&A);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Pipelined CG (Ghysels and Vanroose, 2014).                                */
/* ------------------------------------------------------------------------ */
/* The single-reduction iteration with w = A r also carried by a recurrence,
 * so that the SpMV of an iteration, q = A w, does not depend on its inner
 * products gamma = r.r and delta = w.r (which can then overlap it):
 *   beta, alpha as in the single-reduction iteration,
 *   z = q + beta z (z = A s),  s = w + beta s (s = A p),  p = r + beta p,
 *   x += alpha p,  r -= alpha s,  w -= alpha z.
 * In exact arithmetic the iterates are those of section 3's CG.  Formats as
 * in orc_cg_sr: the SpMV at f_s, both inner products at f_d, the six updates
 * at f_a, alpha and beta in fp64, x = x_hi + x_lo.  A start computes
 * r = rd(b - A x), then w = A r; the first step copies z = q, s = w, p = r.
 * A replacement (every R iterations, and when the recursive rho_k is <= tol)
 * folds x_lo, sets r = rd(b - A x_hi), then w = A r and s = A p, then z = A s
 * (all at f_s), the residual replacement of Cools et al. (2018) for this
 * iteration.  Stops, breakdown, histories and cost_sum as in orc_cg_sr. */
int orc_cg_pipe(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                const double *b, const double *x0, double *x_out, int action,
                const orc_params *prm, orc_result *res, orc_hist *h)
{
    memset(res, 0, sizeof(*res));
    res->fallback_at = -1;
    h->roll_n = 0;
    if (action < 0 || action >= 80) return -1;
    orc_mat A;
    mat_build(&A, n, rp, ci, v);
    size_t bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *xhi = malloc(bytes), *xlo = malloc(bytes), *r = malloc(bytes), *w = malloc(bytes);
    double *p = malloc(bytes), *sv = malloc(bytes), *z = malloc(bytes), *q = malloc(bytes);
    double *r64 = malloc(bytes);
    const int fs = act_fs(action), fd = act_fd(action), fa = act_fa(action);
    const int tier = fa == F64 ? 1 : 0;
    const int R = prm->replace_period;
    const int order = prm->dot_order;
    double *hist_rho = h->hist_rho;
    int64_t k = 0;
    int nrep = 0, status = -1;
    double gamma_old = 0.0, alpha_old = 0.0, last_true = 0.0;

    double bnorm = sqrt(orc_dot(n, b, b, F64, order));
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x_out[i] = 0.0;
        hist_rho[0] = 0.0;
        res->status = 0;
        goto out;
    }
    for (int64_t i = 0; i < n; ++i) { xhi[i] = x0[i]; xlo[i] = 0.0; }

    mat_residual(&A, b, xhi, r64);
    last_true = sqrt(orc_dot(n, r64, r64, F64, order)) / bnorm;
    hist_rho[0] = last_true;
    if (last_true <= prm->tol) { status = 0; goto done; }
    if (!isfinite(last_true)) { status = 3; goto done; }
    if (prm->maxit <= 0) { status = 1; goto done; }
    for (int64_t i = 0; i < n; ++i) r[i] = rd_tier(r64[i], tier);
    mat_spmv(&A, fs, tier, r, w);                          /* w = A r */
    int first = 1, sync = 1;   /* sync: the first pass after a start or replacement */

    for (;;) {
        const double gamma = orc_dot(n, r, r, fd, order);
        const double delta = orc_dot(n, w, r, fd, order);
        mat_spmv(&A, fs, tier, w, q);                      /* q = A w */
        if (sync && !first) mat_spmv(&A, fs, tier, sv, z); /* z = A s again */
        int replace = 0;
        if (!sync) {
            const double rho = sqrt(gamma) / bnorm;
            hist_rho[k] = rho;
            if (rho <= prm->tol) replace = 1;
            else if (k >= prm->maxit) { status = 1; break; }
        }
        if (!replace) {
            sync = 0;
            const double beta = first ? 0.0 : gamma / gamma_old;
            const double den = first ? delta : delta - beta * gamma / alpha_old;
            const double alpha = gamma / den;
            if (!(den > 0.0) || !isfinite(alpha) || !isfinite(beta) || !isfinite(gamma)) { status = 3; break; }
            if (k < h->dump_cap && h->hist_alpha) h->hist_alpha[k] = alpha;
            if (k < h->dump_cap && h->hist_beta) h->hist_beta[k] = beta;
            if (k < h->dump_cap && h->dump_w) memcpy(&h->dump_w[k * n], w, bytes);
            if (first) {
                memcpy(z, q, bytes);
                memcpy(sv, w, bytes);
                memcpy(p, r, bytes);
            } else {
                xpay(n, beta, q, z, fa);
                xpay(n, beta, w, sv, fa);
                xpay(n, beta, r, p, fa);
            }
            if (k < h->dump_cap && h->dump_p) memcpy(&h->dump_p[k * n], p, bytes);
            if (k < h->dump_cap && h->dump_r) memcpy(&h->dump_r[k * n], r, bytes);
            if (k < h->dump_cap && h->dump_s) memcpy(&h->dump_s[k * n], sv, bytes);
            if (k < h->dump_cap && h->dump_z) memcpy(&h->dump_z[k * n], z, bytes);
            orc_axpy(n, alpha, p, xlo, fa);
            orc_axpy(n, -alpha, sv, r, fa);
            orc_axpy(n, -alpha, z, w, fa);
            h->hist_act[k] = (uint8_t)action;
            h->hist_flag[k] = 0;
            gamma_old = gamma;
            alpha_old = alpha;
            first = 0;
            k += 1;
            replace = R > 0 && k % R == 0;
        }
        if (replace) {
            fold(n, xhi, xlo);
            mat_residual(&A, b, xhi, r64);
            const double rt = sqrt(orc_dot(n, r64, r64, F64, order)) / bnorm;
            if (nrep < h->rep_cap) { h->rep_k[nrep] = (int32_t)k; h->rep_rho[nrep] = rt; }
            nrep++;
            if (k > 0) h->hist_flag[k - 1] |= FL_REPLACED;
            hist_rho[k] = rt;
            last_true = rt;
            if (rt <= prm->tol) { status = 0; break; }
            if (!isfinite(rt)) { status = 3; break; }
            if (k >= prm->maxit) { status = 1; break; }
            for (int64_t i = 0; i < n; ++i) r[i] = rd_tier(r64[i], tier);
            mat_spmv(&A, fs, tier, r, w);                  /* w = A r */
            mat_spmv(&A, fs, tier, p, sv);                 /* s = A p */
            sync = 1;
        }
    }
done:
    fold(n, xhi, xlo);
    for (int64_t i = 0; i < n; ++i) x_out[i] = xhi[i];
    if (status == 0) {
        res->relres_true = last_true;
    } else {
        mat_residual(&A, b, xhi, r64);
        res->relres_true = sqrt(orc_dot(n, r64, r64, F64, order)) / bnorm;
    }
    res->status = status;
    res->iters = (int32_t)k;
    res->n_replace = nrep;
out:
    free(xhi); free(xlo); free(r); free(w); free(p); free(sv); free(z); free(q); free(r64);
    mat_free(&A);
    return 0;
}

/* Plain fp64 CG in native double (no emulation): the CPU speed baseline. */
int orc_cg_plain(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                 const double *b, double *x, double tol, int32_t maxit, int32_t *iters_out,
                 double *relres_out)
{
    size_t bytes = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *r = malloc(bytes), *p = malloc(bytes), *q = malloc(bytes);
    double bb = 0.0;
    for (int64_t i = 0; i < n; ++i) bb += b[i] * b[i];
    double bnorm = sqrt(bb);
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t kk = rp[i]; kk < rp[i + 1]; ++kk) acc += v[kk] * x[ci[kk]];
        r[i] = b[i] - acc;
        p[i] = r[i];
    }
    double sigma = 0.0;
    for (int64_t i = 0; i < n; ++i) sigma += r[i] * r[i];
    int32_t k = 0;
    while (k < maxit && sqrt(sigma) / bnorm > tol) {
        for (int64_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int64_t kk = rp[i]; kk < rp[i + 1]; ++kk) acc += v[kk] * p[ci[kk]];
            q[i] = acc;
        }
        double nu = 0.0;
        for (int64_t i = 0; i < n; ++i) nu += p[i] * q[i];
        double alpha = sigma / nu;
        double sn = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
            sn += r[i] * r[i];
        }
        double beta = sn / sigma;
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        sigma = sn;
        k++;
    }
    *iters_out = k;
    *relres_out = sqrt(sigma) / bnorm;
    free(r); free(p); free(q);
    return 0;
}
