// kernels.hpp -- device data layout shared by the solver kernels and the host engine.
#pragma once
#include "dev.hpp"

namespace mpcg {

constexpr int kMaxEdges = 16;
constexpr int kMlpIn = 16, kMlpH = 128, kNAct = 64;

// Matrix in HBM: CSR int32 indices, fp64 values and three shadows.  Value and
// index arrays are padded to a multiple of 8 entries (+8) so the SpMV can read
// aligned 8-entry groups without bounds checks.
struct Mat {
  int n, nnz;
  const int *rp, *ci;
  const double *v64;
  const float *v32;
  const uint16_t *vbf, *vh;   // bf16 bits, fp16 bits (row-scaled)
  const int8_t *rexp;         // fp16 row exponents
};

// Solver vectors.  r, p, q, x_lo exist in a float and a double container; the
// tier of the current iteration's axpy format says which one is live.
struct Vecs {
  const double *b;
  double *xout;   // caller's x: initial guess in, solution out
  double *xhi;    // fp64 accumulator of the solution
  float *r32, *p32, *q32, *xlo32;
  double *r64, *p64, *q64, *xlo64;
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
  double cost[4];
  double epsilon;
  uint64_t seed;
  int64_t episode;
  const float *W1, *b1, *W2, *b2, *W3, *b3;
  int32_t replace_period;
  int32_t roll_cap;
  float *roll_feat, *roll_next;
  int32_t *roll_act;
  float *roll_rew;
  uint8_t *roll_done;
  int32_t *roll_n;
};

// What the next kernel of each slot position does.
enum { M_INIT = 0, M_ITER = 1, M_REPLACE = 2, M_FINAL = 3, M_DONE = 4 };
enum { K2_NONE = 0, K2_AXPY = 1 };
enum { K3_NONE = 0, K3_XPAY = 1, K3_COPY = 2, K3_FOLD = 3 };
enum { FL_REPLACED = 1, FL_EXPLORED = 2, FL_FALLBACK = 4, FL_SWITCH = 8 };

// Device-resident solver state, written only by "last blocks" (one thread).
struct Ctl {
  int32_t mode, k2op, k3op, k3switch;
  int32_t tier, tier_old, action, k;
  int32_t maxit, status, fell_back, fallback_at;
  int32_t nrep, nrep_since, s, explored;
  int32_t prev_action, R, fallback_enabled, k3_fa;
  int32_t zero_solution, bnorm_ready, pad1, pad2;
  double tol, bnorm, sigma, sig_new, alpha, beta, rho_new, last_true, cost_sum, relres_true;
  double rep_hist[3];
  float feat[kMlpIn];
  float feat_next[kMlpIn];
};

struct KArgs {
  Mat A;
  Vecs v;
  Ctl *ctl;
  const PolicyDev *pol;
  Hist h;
  double *part0;       // partials of b.b (start)
  double *part1;       // K1 partials (nu or ||r64||^2), one per 2048-row group
  double *part2;       // K2 partials (sigma'), one per 2048-element block
  int P2;              // 2048-element groups = K1 groups = vector blocks
  int G1;              // K1 workgroups launched (P2 rounded up to 8)
  int8_t *slot_log;    // optional: K1 records the mode of each slot (profiling)
  int slot;            // index of this slot (with slot_log)
};

}  // namespace mpcg
