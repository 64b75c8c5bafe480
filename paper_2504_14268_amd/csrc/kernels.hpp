// kernels.hpp -- device data layout shared by the solver kernels and the host engine.
#pragma once
#include "dev.hpp"

namespace mpcg {

constexpr int kMaxEdges = 16;
constexpr int kRPT = 2;                          // rows per thread in KA
constexpr int kKaRows = kRPT * kRowsPerBlock;    // rows per KA workgroup
constexpr int kMlpIn = 16, kMlpH = 128, kNAct = 64;
constexpr int kQbestMax = 256;                   // states whose greedy action travels with the policy
constexpr int kNoAllocPartials = 65536;          // block partials of the allocation-free dot (512 KiB)

// Matrix in HBM: CSR int32 indices, fp64 values and three shadows.  Value and
// index arrays are padded to a multiple of 8 entries (+8) so the SpMV can read
// aligned 8-entry groups without bounds checks.
struct Mat {
  int n, nnz;
  const int *rp, *ci;
  const int16_t *dc;          // col - row as int16 when every row fits, else NULL
  const uint32_t *pbf, *ph;   // with dc: bf16 / fp16 value | delta << 16 per entry
  const double *v64;
  const float *v32;
  const uint16_t *vbf, *vh;   // bf16 bits, fp16 bits (row-scaled)
  const uint8_t *v8;          // q52 bits (row-scaled like fp16)
  const float *vtf;           // tf32 values (fp32 containers)
  const int8_t *rexp;         // row exponents of the fp16 and q52 shadows
  const float *minv;          // Jacobi preconditioner: fp32 of 1 / a_ii (0 without a diagonal)
};

// Solver vectors.  r, p, q, x_lo exist in a float and a double container; the
// tier of the current iteration's axpy format says which one is live.
struct Vecs {
  const double *b;
  double *xout;   // caller's x: initial guess in, solution out
  double *xhi;    // fp64 accumulator of the solution
  float *r32, *q32, *xlo32;
  double *r64, *q64, *xlo64;
  float *p32;     // direction
  double *p64;
  uint16_t *r16, *p16, *x16;   // bf16 containers of r, p, x_lo (16-bit vector storage)
};

struct Hist {
  double *rho;     // [cap_it + 1]
  uint8_t *act;    // [cap_it]
  uint8_t *flag;   // [cap_it]
  int32_t *rep_k;  // [cap_rep]
  double *rep_rho; // [cap_rep]
  int cap_it, cap_rep;
};

enum { POL_FIXED = 0, POL_QTABLE = 1, POL_QTRAIN = 2, POL_MLP = 3 };

struct PolicyDev {
  int32_t kind, fixed_action, t_bin, b_it, b_res, w_stag;
  double edges[kMaxEdges];
  double *q;
  double lr, gamma, w1, w2, w3, eps_min;
  double cost[6];                // c(f) by format code: fp16, bf16, fp32, fp64, q52 (= fp16), tf32
  double epsilon;
  uint64_t seed;
  int64_t episode;
  const float *W1, *b1, *W2, *b2, *W3, *b3;
  int32_t replace_period;
  int32_t decision_period;       // the policy acts every decision_period iterations (<= 1: every one)
  int32_t per_op;                // 1: one Q-table per operation, Q_j(s, d) = q[s][nfmt j + d]
  int32_t nfmt;                  // formats per operation table: 4, or 5 (digit 4: tf32)
  int32_t roll_cap;
  float *roll_feat, *roll_next;
  int32_t *roll_act;
  float *roll_rew;
  uint8_t *roll_done;
  int32_t *roll_n;
  int32_t n_qbest;               // greedy table: qbest[s] = argmax_a q[s][a] for s < n_qbest (else 0 states)
  uint8_t qbest[kQbestMax];
};

// Phase of the next KA (mode), what KB executes (b_op), and the pending
// elementwise operation (k3op) that KB (after a start or a replacement) or KX
// (after an iteration) applies.
enum { M_INIT = 0, M_ITER = 1, M_REPLACE = 2, M_FINAL = 3, M_DONE = 4 };
enum { K3_NONE = 0, K3_XPAY = 1, K3_COPY = 2, K3_FOLD = 3 };
enum { B_NONE = 0, B_AXPY = 1, B_EXEC = 2 };
enum { FL_REPLACED = 1, FL_EXPLORED = 2, FL_FALLBACK = 4, FL_SWITCH = 8 };

// Device-resident solver state.  Every workgroup of a kernel holds the same
// copy in LDS; workgroup 0 commits it to the other half of the double buffer.
struct Ctl {
  int32_t mode, k3op, k3switch, tier;
  int32_t tier_old, action, k, maxit;
  int32_t status, fell_back, fallback_at, nrep;
  int32_t nrep_since, s, explored, prev_action;
  int32_t R, fallback_enabled, k3_fa, zero_solution;
  int32_t bnorm_ready, pend_sigma, b_op, step_done;
  int32_t fold_done, precond;     // precond: 1 = Jacobi-preconditioned iteration
  int32_t dir_restart, k_dec;     // 1: the next direction update restarts (p = z);
                                  // k_dec: iteration of the current decision
  int32_t stop_rule, rho64;       // stop_rule 1: stop when the recursive rho < tol with k >= 10;
                                  // rho64 1: rho from an fp64 r.r, sigma' at the dot format
  int32_t emul, vec16;            // emul 1: the paper's emulation reading (fp64 operations,
                                  // results rounded to their formats, fp64 vectors); vec16 1:
                                  // bf16 updates keep r, p, x_lo in bf16 containers (tier 2)
  double tol, bnorm, sigma, sig_new, alpha, beta, rho_new, last_true, cost_sum, relres_true;
  double rep_hist[3];
  float feat[kMlpIn];
  float feat_next[kMlpIn];
};

struct KArgs {
  Mat A;
  Vecs v;
  Ctl *ctl;            // ctl[0]: read by KA and KB, written by KX; ctl[1]: written by KB, read by KX
  int slow;            // 1: the scalar steps run in one-block kernels (KS)
  int full;            // 1: KB runs the full replicated step, the end-of-iteration step runs in KS
  const float *net;    // network weights (W1|b1|W2|b2|W3|b3) for KS to stage in LDS, or NULL
  const PolicyDev *pol;
  Hist h;
  double *part0;       // partials of b.b (start)
  double *part1;       // KA partials (nu or ||r64||^2), one per KA workgroup
  double *part2;       // KB partials (sigma' = r.r), one per 2048-element block
  double *part1b;      // with a preconditioner: KA's partials of r64.(M^-1 r64)
  double *part2b;      // with a preconditioner: KB's partials of r.z
  int P1;              // KA row groups (grows rows each)
  int grows;           // rows per KA group: 512, 1024 or 2048
  int P2;              // 2048-element vector blocks
  int G1;              // KA workgroups launched (P1 rounded up to 8)
  int precond;         // 1: launch the preconditioned KB / KX variants (Ctl.precond set too)
  int rho64;           // 1: launch the KB variant with rho in fp64 (Ctl.rho64 set too)
  int vec16;           // 1: launch the KA/KB/KX variants with the bf16 vector tier
  int ext;             // 1: launch the variants with tf32 and the emulation reading
  int8_t *slot_log;    // optional: KA records the mode of each slot (profiling)
  int slot;            // index of this slot (with slot_log)
};

// Single-reduction CG (Chronopoulos and Gear) and pipelined CG (Ghysels and
// Vanroose): two launches per iteration.  KS1 (row groups, like KA) runs the
// iteration's SpMV (w = A_fs r, or q = A_fs w when pipelined) with the
// partials of gamma = r.r and delta = r.w, or an fp64 residual; KS2 (vector
// blocks, like KB) runs the replicated scalar step and the vector updates.
// Phases of a slot (PC_W: the pipelined iteration's w = A r and s = A p after
// a start or replacement):
enum { SR_START = 0, SR_ITER = 1, SR_SYNC = 2, SR_RESID = 3, SR_FINAL = 4, SR_DONE = 5, PC_W = 6 };

struct SrCtl {
  int32_t mode, k, maxit, R;
  int32_t status, nrep, first, tier;   // first: the next update takes beta = 0 (p = r, s = w)
  int32_t action, fs, fd, fa;
  int32_t zero_solution;
  int32_t pipe;     // 1: pipelined CG
  int32_t sync;     // pipelined: the next iteration is the first after a start or replacement
  int32_t pad_;
  double tol, bnorm, gamma_old, alpha_old, rho_new, last_true, relres_true, pad2_;
};

struct SrArgs {
  Mat A;
  Vecs v;            // r, p, x_lo in the container of the update format; q holds w = A r
  float *s32;        // s, the recurrence for A p
  double *s64;
  float *w32, *z32;  // pipelined: w (for A r) and z (for A s) by recurrence; q holds A w
  double *w64, *z64;
  SrCtl *ctl;        // [2]: slot j's KS1 and KS2 read ctl[j & 1], KS2's workgroup 0 writes ctl[(j + 1) & 1]
  Hist h;
  double *pg, *pd;   // KS1 partials: gamma (or ||r64||^2) and delta (or ||b||^2), one per row group
  int P1, grows, G1, P2;
  int par;           // slot parity
  int tier;          // 1: the update format is fp64 (fp64 containers)
  int pipe;          // 1: the pipelined iteration's kernels
};

// One system of a batched solve: its kernel arguments (its own control block,
// policy, vectors, histories) and its slot budget.
struct BatchSys {
  KArgs a;
  int32_t max_slots;
  int32_t pad_[3];
};

// Entry of a lockstep table: a system and one of its row groups (KA) or vector
// blocks (KB, KX).
struct SysBlk {
  int32_t sys, idx;
};

}  // namespace mpcg
