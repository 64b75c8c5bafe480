// api.hip -- host engine and C ABI (include/mpcg.h).
//
// The engine keeps every vector, the control blocks and the histories on the
// device.  A solve enqueues a start kernel, then iteration slots (KA, KB; with
// one-block step kernels between them for policies that need them) in chunks;
// after each chunk it copies the 4-byte mode word to pinned memory and checks
// the previous chunk's word, so the GPU always has a chunk queued and the host
// never waits inside an iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <new>
#include <numeric>
#include <set>
#include <string>
#include <vector>

#include "launch.hpp"
#include "mlp.hpp"
#include "mpcg.h"

using namespace mpcg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(e_ == hipErrorOutOfMemory ? MPCG_ERR_NOMEM : MPCG_ERR_DEVICE,            \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                      \
  } while (0)

template <typename T>
hipError_t dmalloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void **)p, count * sizeof(T));
}

template <typename T>
void dfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

int round_up(int x, int m) { return (x + m - 1) / m * m; }

// ---------------------------------------------------------------------------
// Residual-bin thresholds (section 4.1, the residual bin j_k): with
// delta = -log10(eps_min) / b_res, the bin boundaries are 10^(-delta j),
// j = 1 .. b_res-1.  eps_min must be a power of ten, 10^-E (the double nearest
// to it), so each boundary is 10^(-E j / b_res) exactly, and T_j is the double
// nearest to that real number.  The comparisons below are exact: a dyadic
// number M 2^F (M > 0 odd or even integer, F integer) lies below 10^(-N/D)
// iff M^D 10^N < 2^(-F D), compared as big integers.  10^(-N/D) is never a
// double's midpoint (it is not dyadic), so "nearest" has no ties.
// ---------------------------------------------------------------------------
struct Big {
  std::vector<uint32_t> w;   // little-endian base-2^32 digits, no leading zeros
  explicit Big(uint64_t v = 0) {
    while (v) { w.push_back((uint32_t)v); v >>= 32; }
  }
  void mul_small(uint32_t m) {
    uint64_t carry = 0;
    for (uint32_t &d : w) {
      const uint64_t t = (uint64_t)d * m + carry;
      d = (uint32_t)t;
      carry = t >> 32;
    }
    if (carry) w.push_back((uint32_t)carry);
  }
  static Big mul(const Big &a, const Big &b) {
    Big r;
    if (a.w.empty() || b.w.empty()) return r;
    r.w.assign(a.w.size() + b.w.size(), 0);
    for (size_t i = 0; i < a.w.size(); ++i) {
      uint64_t carry = 0;
      for (size_t j = 0; j < b.w.size(); ++j) {
        const uint64_t t = (uint64_t)a.w[i] * b.w[j] + r.w[i + j] + carry;
        r.w[i + j] = (uint32_t)t;
        carry = t >> 32;
      }
      size_t k = i + b.w.size();
      while (carry) {
        const uint64_t t = (uint64_t)r.w[k] + carry;
        r.w[k++] = (uint32_t)t;
        carry = t >> 32;
      }
    }
    while (!r.w.empty() && r.w.back() == 0) r.w.pop_back();
    return r;
  }
  static Big pow2(int64_t e) {   // 2^e, e >= 0
    Big r;
    r.w.assign((size_t)(e / 32) + 1, 0);
    r.w.back() = 1u << (e % 32);
    return r;
  }
  static int cmp(const Big &a, const Big &b) {
    if (a.w.size() != b.w.size()) return a.w.size() < b.w.size() ? -1 : 1;
    for (size_t i = a.w.size(); i-- > 0;)
      if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
    return 0;
  }
};

// sign of (M 2^F) - 10^(-N/D) for M >= 1, N >= 0, D >= 1
int cmp_dyadic_pow10(uint64_t M, int64_t F, int64_t N, int64_t D) {
  Big lhs(1);
  const Big m(M);
  for (int64_t i = 0; i < D; ++i) lhs = Big::mul(lhs, m);   // M^D
  for (int64_t i = 0; i < N; ++i) lhs.mul_small(10);          // M^D 10^N
  const int64_t s = F * D;                                    // compare with 2^(-s)
  if (s >= 0) {
    // M^D 10^N 2^s >= 1 > 10^0 unless everything is 1
    Big l2 = Big::mul(lhs, Big::pow2(s));
    return Big::cmp(l2, Big(1));
  }
  return Big::cmp(lhs, Big::pow2(-s));
}

// sign of x - 10^(-N/D) for a positive finite double x
int cmp_double_pow10(double x, int64_t N, int64_t D) {
  int e;
  const double fr = std::frexp(x, &e);                        // x = fr 2^e, fr in [0.5, 1)
  const uint64_t M = (uint64_t)std::ldexp(fr, 53);           // exact
  return cmp_dyadic_pow10(M, (int64_t)e - 53, N, D);
}

// sign of midpoint(x, nextafter(x, +inf)) - 10^(-N/D), x > 0 finite normal or subnormal
int cmp_mid_pow10(double x, int64_t N, int64_t D) {
  // The next double up is x + ulp(x) with ulp(x) = 2^F the spacing of x's
  // binade (also when it starts the next binade), so the midpoint is
  // (2 Mx + 1) 2^(F-1) with x = Mx 2^F.
  int e;
  const double fr = std::frexp(x, &e);
  uint64_t Mx = (uint64_t)std::ldexp(fr, 53);
  int64_t F = (int64_t)e - 53;
  if (x < std::ldexp(1.0, -1022)) {   // subnormal: spacing 2^-1074
    Mx = (uint64_t)std::ldexp(x, 1074);
    F = -1074;
  }
  return cmp_dyadic_pow10(2 * Mx + 1, F - 1, N, D);
}

// Power-of-ten exponent E with eps_min == (double)10^-E, or -1.
int pow10_exponent(double eps_min) {
  if (!(eps_min > 0.0 && eps_min < 1.0) || !std::isfinite(eps_min)) return -1;
  const int E = (int)std::lround(-std::log10(eps_min));
  if (E < 1 || E > 300) return -1;
  char buf[16];
  std::snprintf(buf, sizeof(buf), "1e-%d", E);
  return std::strtod(buf, nullptr) == eps_min ? E : -1;   // strtod rounds correctly
}

// T_j, j = 1 .. b_res-1: the double nearest to 10^(-E j / b_res).
int residual_thresholds(int b_res, double eps_min, double *out) {
  if (b_res < 1 || b_res > kMaxEdges + 1) return fail(MPCG_ERR_INVALID, "b_res must be in [1, 17]");
  const int E = pow10_exponent(eps_min);
  if (E < 0) return fail(MPCG_ERR_INVALID, "eps_min must be a power of ten 10^-E, 1 <= E <= 300");
  for (int j = 1; j < b_res; ++j) {
    const int64_t g = std::gcd((int64_t)E * j, (int64_t)b_res);
    const int64_t N = (int64_t)E * j / g, D = (int64_t)b_res / g;
    double c = (double)std::pow(10.0L, -(long double)N / (long double)D);
    // walk to the nearest double: the midpoint above c must lie above the
    // target and the midpoint below c below it
    for (int guard = 0; guard < 64 && cmp_mid_pow10(c, N, D) < 0; ++guard) c = std::nextafter(c, INFINITY);
    for (int guard = 0; guard < 64 && cmp_mid_pow10(std::nextafter(c, 0.0), N, D) > 0; ++guard)
      c = std::nextafter(c, 0.0);
    if (!(cmp_mid_pow10(c, N, D) > 0 && cmp_mid_pow10(std::nextafter(c, 0.0), N, D) < 0))
      return fail(MPCG_ERR_INVALID, "residual threshold search did not settle");
    out[j - 1] = c;
  }
  for (int j = b_res; j <= kMaxEdges; ++j) out[j - 1] = 0.0;
  return MPCG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
struct mpcg_policy {
  mpcg_policy_desc desc{};
  std::set<mpcg_matrix *> users;   // matrices whose mpcg_set_policy attached this policy
  double edges[kMaxEdges] = {};   // residual-bin thresholds derived from b_res, eps_min
  int n_states = 0;
  double *d_q = nullptr;
  std::vector<uint8_t> qbest;   // greedy action per state of the table last set from the host
  float *d_mlp = nullptr;   // W1 | b1 | W2 | b2 | W3 | b3
  bool has_mlp = false;
  int32_t roll_cap = 0;
  float *d_rf = nullptr, *d_rn = nullptr, *d_rr = nullptr;
  int32_t *d_ra = nullptr, *d_rcount = nullptr;
  uint8_t *d_rd = nullptr;
  int64_t episode = 0;
  double epsilon = 0.0;

  PolicyDev device_struct() const {
    PolicyDev p{};
    p.kind = desc.kind;
    p.fixed_action = desc.fixed_action;
    p.t_bin = desc.t_bin;
    p.b_it = desc.b_it;
    p.b_res = desc.b_res;
    p.w_stag = desc.w_stag;
    for (int i = 0; i < kMaxEdges; ++i) p.edges[i] = edges[i];
    p.q = d_q;
    p.lr = desc.lr;
    p.gamma = desc.gamma;
    p.w1 = desc.w1;
    p.w2 = desc.w2;
    p.w3 = desc.w3;
    p.eps_min = desc.eps_min;
    for (int i = 0; i < 4; ++i) p.cost[i] = desc.cost[i];
    p.cost[FP8] = desc.cost[MPCG_FP16];   // a q52 SpMV is charged as fp16
    p.cost[TF32] = desc.cost_tf32;
    p.epsilon = epsilon;
    p.seed = desc.seed;
    p.episode = episode;
    if (has_mlp) {
      p.W1 = d_mlp;
      p.b1 = p.W1 + kMlpH * kMlpIn;
      p.W2 = p.b1 + kMlpH;
      p.b2 = p.W2 + kMlpH * kMlpH;
      p.W3 = p.b2 + kMlpH;
      p.b3 = p.W3 + kNAct * kMlpH;
    }
    p.n_qbest = 0;
    if (desc.kind == MPCG_POLICY_QTABLE && n_states <= kQbestMax && (int)qbest.size() == n_states) {
      p.n_qbest = n_states;
      for (int s = 0; s < n_states; ++s) p.qbest[s] = qbest[s];
    }
    p.replace_period = desc.replace_period;
    p.decision_period = desc.decision_period;
    p.per_op = desc.per_op;
    p.nfmt = desc.nfmt == 5 ? 5 : 4;
    p.roll_cap = roll_cap;
    p.roll_feat = d_rf;
    p.roll_next = d_rn;
    p.roll_act = d_ra;
    p.roll_rew = d_rr;
    p.roll_done = d_rd;
    p.roll_n = d_rcount;
    return p;
  }

  void release() {
    dfree(d_q);
    dfree(d_mlp);
    dfree(d_rf);
    dfree(d_rn);
    dfree(d_rr);
    dfree(d_ra);
    dfree(d_rcount);
    dfree(d_rd);
  }
};


struct mpcg_matrix {
  int n = 0, nnz = 0, nnz_pad = 0;
  hipStream_t stream = nullptr;
  int *d_rp = nullptr, *d_ci = nullptr;
  int16_t *d_dc = nullptr;     // 16-bit column deltas, when every row fits
  uint32_t *d_pbf = nullptr, *d_ph = nullptr;   // with d_dc: interleaved 16-bit value | delta
  double *d_v64 = nullptr;
  float *d_v32 = nullptr;
  uint16_t *d_vbf = nullptr, *d_vh = nullptr;
  uint8_t *d_v8 = nullptr;     // q52 shadow (row-scaled like fp16)
  float *d_vtf = nullptr;      // tf32 shadow (fp32 containers)
  int8_t *d_rexp = nullptr;
  // workspace
  double *d_xhi = nullptr;
  float *d_r32 = nullptr, *d_q32 = nullptr, *d_xlo32 = nullptr, *d_p32 = nullptr;
  uint16_t *d_r16 = nullptr, *d_p16 = nullptr, *d_x16 = nullptr;   // bf16 containers (vec16)
  double *d_r64 = nullptr, *d_q64 = nullptr, *d_xlo64 = nullptr, *d_p64 = nullptr;
  double *d_part0 = nullptr, *d_part1 = nullptr, *d_part2 = nullptr, *d_scalar = nullptr;
  double *d_part1b = nullptr, *d_part2b = nullptr;   // preconditioned: r.(M^-1 r) partials
  float *d_minv = nullptr;     // Jacobi preconditioner: fp32 of 1 / a_ii
  float *d_s32 = nullptr;      // single-reduction CG: s, the recurrence for A p
  double *d_s64 = nullptr;
  float *d_w32 = nullptr, *d_z32 = nullptr;    // pipelined CG: w (A r) and z (A s)
  double *d_w64 = nullptr, *d_z64 = nullptr;
  SrCtl *d_sr = nullptr;       // single-reduction CG: [2] control blocks
  SrCtl *h_sr = nullptr;       // pinned [3]: the start state and the state after each chunk
  Ctl *d_ctl = nullptr;        // [2]
  Ctl *h_ctl = nullptr;        // pinned
  Ctl *h_poll = nullptr;       // pinned [2]: the control block after each chunk
  PolicyDev *d_pol = nullptr;
  PolicyDev *h_pol = nullptr;  // pinned staging
  // history
  int cap_it = -1, cap_rep = 0;
  double *d_hrho = nullptr, *d_reprho = nullptr;
  uint8_t *d_hact = nullptr, *d_hflag = nullptr;
  int32_t *d_repk = nullptr;
  int last_iters = -1, last_nrep = 0;
  // profiling
  int8_t *d_slotlog = nullptr;
  int slot_cap = 0;
  std::vector<hipEvent_t> pev;
  std::vector<float> ta, tb, tx, ts;
  mpcg_profile prof{};
  // policy
  mpcg_policy *pol = nullptr;
  mpcg_policy *defpol = nullptr;
  mpcg_solve_opts opts{50, 0, 32, 0, 0, 0, 0, 0, 0, 0, 0, 0};   // replace_period .. vec16, variant
  hipEvent_t ev_start = nullptr, ev_end = nullptr, ev_chunk[2] = {nullptr, nullptr};
  int P2 = 0;

  Mat mat() const {
    Mat m;
    m.n = n;
    m.nnz = nnz;
    m.rp = d_rp;
    m.ci = d_ci;
    m.dc = d_dc;
    m.pbf = d_pbf;
    m.ph = d_ph;
    m.v64 = d_v64;
    m.v32 = d_v32;
    m.vbf = d_vbf;
    m.vh = d_vh;
    m.v8 = d_v8;
    m.vtf = d_vtf;
    m.rexp = d_rexp;
    m.minv = d_minv;
    return m;
  }

  void release() {
    dfree(d_rp); dfree(d_ci); dfree(d_dc); dfree(d_pbf); dfree(d_ph); dfree(d_v64); dfree(d_v32); dfree(d_vbf); dfree(d_vh); dfree(d_v8); dfree(d_vtf); dfree(d_rexp);
    dfree(d_xhi); dfree(d_r32); dfree(d_p32); dfree(d_q32); dfree(d_xlo32);
    dfree(d_r16); dfree(d_p16); dfree(d_x16);
    dfree(d_r64); dfree(d_p64); dfree(d_q64); dfree(d_xlo64);
    dfree(d_part0); dfree(d_part1); dfree(d_part2); dfree(d_scalar); dfree(d_ctl); dfree(d_pol);
    dfree(d_part1b); dfree(d_part2b); dfree(d_minv);
    dfree(d_s32); dfree(d_s64); dfree(d_sr);
    dfree(d_w32); dfree(d_z32); dfree(d_w64); dfree(d_z64);
    if (h_sr) (void)hipHostFree(h_sr);
    h_sr = nullptr;
    dfree(d_hrho); dfree(d_reprho); dfree(d_hact); dfree(d_hflag); dfree(d_repk); dfree(d_slotlog);
    for (hipEvent_t e : pev) (void)hipEventDestroy(e);
    pev.clear();
    if (h_ctl) (void)hipHostFree(h_ctl);
    if (h_poll) (void)hipHostFree(h_poll);
    if (h_pol) (void)hipHostFree(h_pol);
    h_ctl = nullptr; h_poll = nullptr; h_pol = nullptr;
    for (hipEvent_t *e : {&ev_start, &ev_end, &ev_chunk[0], &ev_chunk[1]})
      if (*e) { (void)hipEventDestroy(*e); *e = nullptr; }
    if (defpol) { defpol->release(); delete defpol; defpol = nullptr; }
  }
};

// Waits for the work on the streams of the matrices a policy is attached to
// (a policy's tables and logs are written by their solves).
static int sync_users(mpcg_policy *P) {
  for (mpcg_matrix *A : P->users) {
    const hipError_t e = hipStreamSynchronize(A->stream);
    if (e != hipSuccess) return fail(MPCG_ERR_DEVICE, std::string("policy sync: ") + hipGetErrorString(e));
  }
  return MPCG_OK;
}

static void default_desc(mpcg_policy_desc *d) {
  std::memset(d, 0, sizeof(*d));
  d->kind = MPCG_POLICY_FIXED;
  d->fixed_action = 63;
  d->t_bin = 1000;
  d->b_it = 5;
  d->b_res = 10;
  d->w_stag = 10;
  d->lr = 0.1;
  d->gamma = 0.9;
  d->w1 = 1.0;
  d->w2 = 0.1;
  d->w3 = 10.0;
  d->eps_min = 1e-16;
  const double c1[4] = {0.8, 0.6, 1.0, 2.0};
  for (int i = 0; i < 4; ++i) d->cost[i] = c1[i];
  d->cost_tf32 = 0.8;
  d->nfmt = 4;
  d->replace_period = 50;
}

static int policy_alloc(mpcg_policy *P) {
  int rc = residual_thresholds(P->desc.b_res, P->desc.eps_min, P->edges);
  if (rc) return rc;
  P->n_states = P->desc.b_res * P->desc.b_it * 2;
  HIP_TRY(dmalloc(&P->d_q, (size_t)P->n_states * kNAct));
  HIP_TRY(hipMemset(P->d_q, 0, sizeof(double) * (size_t)P->n_states * kNAct));
  P->qbest.assign((size_t)P->n_states, 0);   // all-zero table: action 0 everywhere
  HIP_TRY(dmalloc(&P->d_rcount, 1));
  HIP_TRY(hipMemset(P->d_rcount, 0, sizeof(int32_t)));
  return MPCG_OK;
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
static int ensure_ws(mpcg_matrix *A) {
  if (A->d_xhi) return MPCG_OK;
  const size_t n = (size_t)A->n;
  HIP_TRY(dmalloc(&A->d_xhi, n));
  HIP_TRY(dmalloc(&A->d_r32, n)); HIP_TRY(dmalloc(&A->d_p32, n));
  HIP_TRY(dmalloc(&A->d_q32, n)); HIP_TRY(dmalloc(&A->d_xlo32, n));
  HIP_TRY(dmalloc(&A->d_r64, n)); HIP_TRY(dmalloc(&A->d_p64, n));
  HIP_TRY(dmalloc(&A->d_q64, n)); HIP_TRY(dmalloc(&A->d_xlo64, n));
  HIP_TRY(dmalloc(&A->d_r16, n)); HIP_TRY(dmalloc(&A->d_p16, n)); HIP_TRY(dmalloc(&A->d_x16, n));
  return MPCG_OK;
}

static int ensure_hist(mpcg_matrix *A, int maxit) {
  if (A->cap_it >= maxit) return MPCG_OK;
  dfree(A->d_hrho); dfree(A->d_hact); dfree(A->d_hflag); dfree(A->d_repk); dfree(A->d_reprho);
  const int cap = std::max(maxit, 16);
  HIP_TRY(dmalloc(&A->d_hrho, (size_t)cap + 1));
  HIP_TRY(dmalloc(&A->d_hact, (size_t)cap));
  HIP_TRY(dmalloc(&A->d_hflag, (size_t)cap));
  HIP_TRY(dmalloc(&A->d_repk, (size_t)cap + 1));
  HIP_TRY(dmalloc(&A->d_reprho, (size_t)cap + 1));
  A->cap_it = cap;
  A->cap_rep = cap + 1;
  dfree(A->d_slotlog);
  A->slot_cap = 2 * cap + 16;
  HIP_TRY(dmalloc(&A->d_slotlog, (size_t)A->slot_cap));
  return MPCG_OK;
}

// Kernel durations of each slot of a completed chunk (a start and a stop event
// per launch): KA, KB, KX and, for policies with one-block steps, the two step
// kernels.
// Launch durations of a chunk's slots: KA, [step before KB], KB, [step before
// KX], KX, in launch order.
static int collect_chunk(mpcg_matrix *A, int pool_idx, int chunk, int per_slot, bool step_b, bool step_x,
                         int64_t first, int m) {
  for (int s = 0; s < m; ++s) {
    hipEvent_t *e = &A->pev[((size_t)pool_idx * chunk + s) * per_slot];
    float t[5] = {0, 0, 0, 0, 0};
    for (int j = 0; 2 * j + 1 < per_slot; ++j) HIP_TRY(hipEventElapsedTime(&t[j], e[2 * j], e[2 * j + 1]));
    int j = 0;
    A->ta[first + s] = t[j++];
    A->ts[first + s] = 0.0f;
    if (step_b) A->ts[first + s] += t[j++];
    A->tb[first + s] = t[j++];
    if (step_x) A->ts[first + s] += t[j++];
    A->tx[first + s] = t[j++];
  }
  return MPCG_OK;
}

// Rows per SpMV workgroup: the largest group size that still gives about four
// workgroups per compute unit (256 CUs), at least 512.
static int spmv_group_rows(int n, int requested) {
  if (requested == 512 || requested == 1024 || requested == 2048) return requested;
  for (int g = 2048; g > 512; g >>= 1)
    if ((n + g - 1) / g >= 1024) return g;
  return 512;
}

static KArgs make_args(mpcg_matrix *A, const double *b, double *x) {
  KArgs a{};
  a.A = A->mat();
  a.v.b = b;
  a.v.xout = x;
  a.v.xhi = A->d_xhi;
  a.v.r32 = A->d_r32; a.v.q32 = A->d_q32; a.v.xlo32 = A->d_xlo32;
  a.v.r64 = A->d_r64; a.v.q64 = A->d_q64; a.v.xlo64 = A->d_xlo64;
  a.v.p32 = A->d_p32;
  a.v.p64 = A->d_p64;
  a.v.r16 = A->d_r16; a.v.p16 = A->d_p16; a.v.x16 = A->d_x16;
  a.ctl = A->d_ctl;
  a.pol = A->d_pol;
  a.h.rho = A->d_hrho;
  a.h.act = A->d_hact;
  a.h.flag = A->d_hflag;
  a.h.rep_k = A->d_repk;
  a.h.rep_rho = A->d_reprho;
  a.h.cap_it = A->cap_it;
  a.h.cap_rep = A->cap_rep;
  a.part0 = A->d_part0;
  a.part1 = A->d_part1;
  a.part2 = A->d_part2;
  a.part1b = A->d_part1b;
  a.part2b = A->d_part2b;
  a.precond = A->opts.precond;
  a.rho64 = A->opts.rho_fp64;
  a.vec16 = A->opts.vec16;
  if (A->opts.index16 < 0) {   // 32-bit indices requested
    a.A.dc = nullptr;
    a.A.pbf = nullptr;
    a.A.ph = nullptr;
  }
  a.grows = spmv_group_rows(A->n, A->opts.spmv_rows);
  a.P1 = (A->n + a.grows - 1) / a.grows;
  a.G1 = round_up(a.P1, 8);
  a.P2 = A->P2;
  return a;
}

// Chunk sizes follow the predicted end of the solve: from the last two polls,
// the recursive residual's decay per iteration gives the iterations still
// needed; once they fit in the chunk already in flight, the next chunks
// shrink (to no fewer than 4 slots), so few idle slots run after the stop.
struct ChunkPlan {
  int chunk;
  double tol;
  int poll_k[2] = {-1, -1};   // last two polled (iteration, residual), newest first
  double poll_rho[2] = {0.0, 0.0};
  int in_flight = 0;          // slots of the newest enqueued chunk
  int next() const {
    if (poll_k[1] < 0 || poll_k[0] <= poll_k[1] || !(poll_rho[0] > 0.0) || !(poll_rho[1] > poll_rho[0]) ||
        !std::isfinite(poll_rho[1]) || !(tol > 0.0))
      return chunk;
    if (poll_rho[0] <= tol) return std::min(chunk, 4);
    const double rate = std::log(poll_rho[0] / poll_rho[1]) / (double)(poll_k[0] - poll_k[1]);   // < 0
    const double need = std::log(tol / poll_rho[0]) / rate - (double)in_flight + 4.0;
    if (!(need < (double)chunk)) return chunk;
    return std::max(std::min(chunk, 4), (int)std::ceil(need));
  }
  void observe(int k, double rho) {
    poll_k[1] = poll_k[0];
    poll_rho[1] = poll_rho[0];
    poll_k[0] = k;
    poll_rho[0] = rho;
  }
};

// Single-reduction CG (opts.variant = 1) and pipelined CG (variant 2): one
// slot is KS1 (the iteration's SpMV with the partials of r.r and r.w, or an
// fp64 residual, or the pipelined sync SpMVs) and KS2 (scalar step and the
// vector updates); the device decides each slot's phase, the host only
// enqueues chunks of slots and polls the control block between them.
static int solve_sr(mpcg_matrix *A, mpcg_policy *P, const double *b, double *x, double tol, int32_t maxit,
                    mpcg_result *res) {
  hipStream_t st = A->stream;
  const size_t n = (size_t)A->n;
  if (!A->d_sr) {
    HIP_TRY(dmalloc(&A->d_s32, n));
    HIP_TRY(dmalloc(&A->d_s64, n));
    HIP_TRY(dmalloc(&A->d_sr, 2));
    HIP_TRY(hipHostMalloc((void **)&A->h_sr, 3 * sizeof(SrCtl), hipHostMallocDefault));
  }
  const bool pipe = A->opts.variant == 2;
  if (pipe && !A->d_w32) {
    HIP_TRY(dmalloc(&A->d_w32, n));
    HIP_TRY(dmalloc(&A->d_z32, n));
    HIP_TRY(dmalloc(&A->d_w64, n));
    HIP_TRY(dmalloc(&A->d_z64, n));
  }
  const int act = P->desc.fixed_action;
  SrCtl &c = A->h_sr[2];
  std::memset(&c, 0, sizeof(SrCtl));
  c.mode = SR_START;
  c.maxit = maxit;
  c.R = A->opts.replace_period;
  c.status = -1;
  c.first = 1;
  c.action = act;
  c.fs = act_fs(act);
  c.fd = act_fd(act);
  c.fa = act_fa(act);
  c.tier = c.fa == FP64 ? 1 : 0;
  c.pipe = pipe ? 1 : 0;
  c.tol = tol;
  HIP_TRY(hipMemcpyAsync(A->d_sr, &c, sizeof(SrCtl), hipMemcpyHostToDevice, st));

  const KArgs k = make_args(A, b, x);
  SrArgs a{};
  a.A = k.A;
  a.v = k.v;
  a.s32 = A->d_s32;
  a.s64 = A->d_s64;
  a.ctl = A->d_sr;
  a.h = k.h;
  a.pg = A->d_part1;
  a.pd = A->d_part1b;
  a.P1 = k.P1;
  a.grows = k.grows;
  a.G1 = k.G1;
  a.P2 = k.P2;
  a.tier = c.tier;
  a.pipe = c.pipe;
  a.w32 = A->d_w32;
  a.z32 = A->d_z32;
  a.w64 = A->d_w64;
  a.z64 = A->d_z64;

  const int chunk = A->opts.chunk > 0 ? A->opts.chunk : 32;
  // a start, one slot per iteration, up to two more per replacement (three
  // when pipelined: the sync phase), a final check
  const int64_t max_slots = (pipe ? 4 : 3) * (int64_t)maxit + 16;
  int64_t slots = 0;
  int ci = 0;
  ChunkPlan plan{chunk, tol};
  HIP_TRY(hipEventRecord(A->ev_start, st));
  while (slots < max_slots) {
    const int m = (int)std::min<int64_t>(plan.next(), max_slots - slots);
    plan.in_flight = m;
    const int idx = ci & 1;
    for (int j = 0; j < m; ++j) {
      a.par = (int)((slots + j) & 1);
      launch_sr_slot(a, st);
    }
    HIP_TRY(hipGetLastError());
    slots += m;
    // the state after the chunk's last slot
    HIP_TRY(hipMemcpyAsync(&A->h_sr[idx], A->d_sr + (slots & 1), sizeof(SrCtl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(A->ev_chunk[idx], st));
    if (ci > 0) {
      const int pidx = (ci - 1) & 1;
      HIP_TRY(hipEventSynchronize(A->ev_chunk[pidx]));
      const SrCtl &pc = A->h_sr[pidx];
      if (pc.mode == SR_DONE) break;
      plan.observe(pc.k, pc.rho_new);
    }
    ci++;
  }
  HIP_TRY(hipEventRecord(A->ev_end, st));
  HIP_TRY(hipStreamSynchronize(st));
  SrCtl &f = A->h_sr[2];
  HIP_TRY(hipMemcpy(&f, A->d_sr + (slots & 1), sizeof(SrCtl), hipMemcpyDeviceToHost));
  if (f.mode != SR_DONE)
    return fail(MPCG_ERR_DEVICE, "single-reduction / pipelined solver did not reach a final state");
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, A->ev_start, A->ev_end));
  std::memset(res, 0, sizeof(*res));
  res->status = f.status;
  res->iters = f.k;
  res->n_replace = f.nrep;
  res->fallback_at = -1;
  res->relres_true = f.relres_true;
  res->cost_sum = 0.0;
  res->time_ms = ms;
  res->slots = (int32_t)slots;
  res->spmv_rows = a.grows;
  res->index16 = a.A.dc ? 1 : 0;
  A->last_iters = f.k;
  A->last_nrep = f.nrep;
  std::memset(&A->prof, 0, sizeof(A->prof));
  return MPCG_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *mpcg_last_error(void) { return g_err.c_str(); }

int mpcg_residual_thresholds(int32_t b_res, double eps_min, double *out) {
  if (!out) return fail(MPCG_ERR_INVALID, "out is NULL");
  double t[kMaxEdges];
  const int rc = residual_thresholds(b_res, eps_min, t);
  if (rc) return rc;
  for (int j = 0; j + 1 < b_res; ++j) out[j] = t[j];
  return MPCG_OK;
}

static int validate_csr(int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, const double *v) {
  if (rp[0] != 0) return fail(MPCG_ERR_CSR, "row_ptr[0] != 0");
  if ((int64_t)rp[n] != nnz) return fail(MPCG_ERR_CSR, "row_ptr[n] != nnz");
  for (int64_t i = 0; i < n; ++i) {
    const int32_t s = rp[i], t = rp[i + 1];
    if (t < s) return fail(MPCG_ERR_CSR, "row_ptr decreases at row " + std::to_string(i));
    bool diag = false;
    for (int32_t k = s; k < t; ++k) {
      if (ci[k] < 0 || ci[k] >= n) return fail(MPCG_ERR_CSR, "column out of range in row " + std::to_string(i));
      if (k > s && ci[k] <= ci[k - 1])
        return fail(MPCG_ERR_CSR, "columns not strictly increasing in row " + std::to_string(i));
      if (!std::isfinite(v[k])) return fail(MPCG_ERR_CSR, "non-finite value in row " + std::to_string(i));
      if (ci[k] == i) {
        if (!(v[k] > 0.0)) return fail(MPCG_ERR_CSR, "non-positive diagonal in row " + std::to_string(i));
        diag = true;
      }
    }
    if (!diag) return fail(MPCG_ERR_CSR, "missing diagonal in row " + std::to_string(i));
  }
  return MPCG_OK;
}

int mpcg_create_csr(int64_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col, const double *val,
                    int mem_kind, void *stream, mpcg_matrix **out) {
  if (!out) return fail(MPCG_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!row_ptr || !col || !val) return fail(MPCG_ERR_INVALID, "NULL CSR array");
  if (n < 1 || nnz < 1 || n >= (int64_t)1 << 31 || nnz >= ((int64_t)1 << 31) - 64)
    return fail(MPCG_ERR_INVALID, "n and nnz must be in [1, 2^31)");
  if (mem_kind != MPCG_MEM_HOST && mem_kind != MPCG_MEM_DEVICE) return fail(MPCG_ERR_INVALID, "bad mem_kind");
  std::vector<int32_t> hrp, hci;
  std::vector<double> hv;
  const int32_t *rp = row_ptr, *ci = col;
  const double *v = val;
  if (mem_kind == MPCG_MEM_DEVICE) {
    hrp.resize(n + 1);
    hci.resize(nnz);
    hv.resize(nnz);
    HIP_TRY(hipMemcpy(hrp.data(), row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hci.data(), col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hv.data(), val, sizeof(double) * nnz, hipMemcpyDeviceToHost));
    rp = hrp.data();
    ci = hci.data();
    v = hv.data();
  }
  int rc = validate_csr(n, nnz, rp, ci, v);
  if (rc) return rc;

  mpcg_matrix *A = new (std::nothrow) mpcg_matrix();
  if (!A) return fail(MPCG_ERR_NOMEM, "host allocation failed");
  auto bail = [&](int code) {
    A->release();
    delete A;
    return code;
  };
#define TRY_A(expr)                                                                             \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return bail(fail(e_ == hipErrorOutOfMemory ? MPCG_ERR_NOMEM : MPCG_ERR_DEVICE,            \
                       std::string(#expr) + ": " + hipGetErrorString(e_)));                     \
  } while (0)
  A->n = (int)n;
  A->nnz = (int)nnz;
  A->nnz_pad = round_up((int)nnz, 8) + 8;
  A->stream = (hipStream_t)stream;
  A->P2 = (A->n + kVecBlock - 1) / kVecBlock;
  if ((A->n + kKaRows - 1) / kKaRows > 64 * kVecBlock)
    return bail(fail(MPCG_ERR_INVALID, "n too large for the partial reduction"));
  const size_t np = (size_t)A->nnz_pad;
  TRY_A(dmalloc(&A->d_rp, (size_t)n + 1));
  TRY_A(dmalloc(&A->d_ci, np));
  TRY_A(dmalloc(&A->d_v64, np));
  TRY_A(dmalloc(&A->d_v32, np));
  TRY_A(dmalloc(&A->d_vbf, np));
  TRY_A(dmalloc(&A->d_vh, np));
  TRY_A(dmalloc(&A->d_v8, np));
  TRY_A(dmalloc(&A->d_vtf, np));
  TRY_A(dmalloc(&A->d_rexp, (size_t)n));
  TRY_A(dmalloc(&A->d_minv, (size_t)n));
  TRY_A(hipMemsetAsync(A->d_ci, 0, sizeof(int) * np, A->stream));
  TRY_A(hipMemsetAsync(A->d_v64, 0, sizeof(double) * np, A->stream));
  TRY_A(hipMemsetAsync(A->d_v32, 0, sizeof(float) * np, A->stream));
  TRY_A(hipMemsetAsync(A->d_vbf, 0, sizeof(uint16_t) * np, A->stream));
  TRY_A(hipMemsetAsync(A->d_vh, 0, sizeof(uint16_t) * np, A->stream));
  TRY_A(hipMemsetAsync(A->d_v8, 0, np, A->stream));
  TRY_A(hipMemsetAsync(A->d_vtf, 0, sizeof(float) * np, A->stream));
  const hipMemcpyKind kind = mem_kind == MPCG_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  TRY_A(hipMemcpyAsync(A->d_rp, row_ptr, sizeof(int32_t) * (n + 1), kind, A->stream));
  TRY_A(hipMemcpyAsync(A->d_ci, col, sizeof(int32_t) * nnz, kind, A->stream));
  TRY_A(hipMemcpyAsync(A->d_v64, val, sizeof(double) * nnz, kind, A->stream));
  launch_shadows(A->n, A->d_rp, A->d_ci, A->d_v64, A->d_v32, A->d_vbf, A->d_vh, A->d_v8, A->d_vtf, A->d_rexp,
                 A->d_minv, A->stream);
  TRY_A(hipGetLastError());
  TRY_A(dmalloc(&A->d_part0, (size_t)A->P2 + 64));
  TRY_A(dmalloc(&A->d_part1, (size_t)(A->n + kKaRows - 1) / kKaRows + 64));
  TRY_A(dmalloc(&A->d_part2, (size_t)A->P2 + 64));
  TRY_A(dmalloc(&A->d_part1b, (size_t)(A->n + kKaRows - 1) / kKaRows + 64));
  TRY_A(dmalloc(&A->d_part2b, (size_t)A->P2 + 64));
  TRY_A(dmalloc(&A->d_scalar, 8));
  // 16-bit column deltas (col - row) when every one fits: the SpMV then reads
  // 2 bytes of index per entry instead of 4 (same columns, same order)
  TRY_A(dmalloc(&A->d_dc, np));
  TRY_A(hipMemsetAsync(A->d_dc, 0, sizeof(int16_t) * np, A->stream));
  TRY_A(hipMemsetAsync(A->d_scalar, 0, sizeof(double), A->stream));
  launch_dcol(A->n, A->d_rp, A->d_ci, A->d_dc, (int *)A->d_scalar, A->stream);
  TRY_A(hipGetLastError());
  {
    int bad = 0;
    TRY_A(hipMemcpyAsync(&bad, A->d_scalar, sizeof(int), hipMemcpyDeviceToHost, A->stream));
    TRY_A(hipStreamSynchronize(A->stream));
    if (bad) dfree(A->d_dc);
  }
  if (A->d_dc) {
    TRY_A(dmalloc(&A->d_pbf, np));
    TRY_A(dmalloc(&A->d_ph, np));
    launch_pack16((int)np, A->d_vbf, A->d_dc, A->d_pbf, A->stream);
    launch_pack16((int)np, A->d_vh, A->d_dc, A->d_ph, A->stream);
    TRY_A(hipGetLastError());
  }
  TRY_A(dmalloc(&A->d_ctl, 2));
  TRY_A(dmalloc(&A->d_pol, 1));
  TRY_A(hipHostMalloc((void **)&A->h_ctl, sizeof(Ctl), hipHostMallocDefault));
  TRY_A(hipHostMalloc((void **)&A->h_poll, 2 * sizeof(Ctl), hipHostMallocDefault));
  TRY_A(hipHostMalloc((void **)&A->h_pol, sizeof(PolicyDev), hipHostMallocDefault));
  TRY_A(hipEventCreate(&A->ev_start));
  TRY_A(hipEventCreate(&A->ev_end));
  TRY_A(hipEventCreateWithFlags(&A->ev_chunk[0], hipEventDisableTiming));
  TRY_A(hipEventCreateWithFlags(&A->ev_chunk[1], hipEventDisableTiming));
  A->defpol = new (std::nothrow) mpcg_policy();
  if (!A->defpol) return bail(fail(MPCG_ERR_NOMEM, "host allocation failed"));
  default_desc(&A->defpol->desc);
  rc = policy_alloc(A->defpol);
  if (rc) return bail(rc);
  TRY_A(hipStreamSynchronize(A->stream));
#undef TRY_A
  *out = A;
  return MPCG_OK;
}

int mpcg_destroy(mpcg_matrix *A) {
  if (!A) return MPCG_OK;
  if (A->stream) (void)hipStreamSynchronize(A->stream);
  if (A->pol) A->pol->users.erase(A);
  A->release();
  delete A;
  return MPCG_OK;
}

int mpcg_get_info(mpcg_matrix *A, mpcg_matrix_info *info) {
  if (!A || !info) return fail(MPCG_ERR_INVALID, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->n = A->n;
  info->nnz = A->nnz;
  info->index16 = A->d_dc ? 1 : 0;
  return MPCG_OK;
}

int mpcg_get_precond(mpcg_matrix *A, float *minv) {
  if (!A || !minv) return fail(MPCG_ERR_INVALID, "NULL argument");
  HIP_TRY(hipStreamSynchronize(A->stream));
  HIP_TRY(hipMemcpy(minv, A->d_minv, sizeof(float) * (size_t)A->n, hipMemcpyDeviceToHost));
  return MPCG_OK;
}

int mpcg_get_shadow_q52(mpcg_matrix *A, uint8_t *q52) {
  if (!A || !q52) return fail(MPCG_ERR_INVALID, "NULL argument");
  HIP_TRY(hipStreamSynchronize(A->stream));
  HIP_TRY(hipMemcpy(q52, A->d_v8, (size_t)A->nnz, hipMemcpyDeviceToHost));
  return MPCG_OK;
}

int mpcg_action(int f_spmv, int f_dot, int f_axpy) {
  auto dig = [](int f) { return f == MPCG_TF32 ? 4 : (f >= 0 && f <= 3 ? f : -1); };
  const int dd = dig(f_dot), da = dig(f_axpy);
  if (dd < 0 || da < 0) return fail(MPCG_ERR_INVALID, "f_dot and f_axpy must be fp16, bf16, fp32, fp64 or tf32");
  if (f_spmv == MPCG_Q52) {
    if (dd == 4 || da == 4) return fail(MPCG_ERR_INVALID, "a q52 SpMV takes the four arithmetic formats");
    return 64 + 4 * dd + da;
  }
  const int ds = dig(f_spmv);
  if (ds < 0) return fail(MPCG_ERR_INVALID, "bad f_spmv");
  return act_compose(ds, dd, da);
}

int mpcg_action_formats(int action, int32_t *f_spmv, int32_t *f_dot, int32_t *f_axpy) {
  if (!f_spmv || !f_dot || !f_axpy) return fail(MPCG_ERR_INVALID, "NULL argument");
  if (!act_valid(action)) return fail(MPCG_ERR_INVALID, "bad action code");
  *f_spmv = act_fs(action);
  *f_dot = act_fd(action);
  *f_axpy = act_fa(action);
  return MPCG_OK;
}

int mpcg_get_shadow_tf32(mpcg_matrix *A, float *tf32) {
  if (!A || !tf32) return fail(MPCG_ERR_INVALID, "NULL argument");
  HIP_TRY(hipStreamSynchronize(A->stream));
  HIP_TRY(hipMemcpy(tf32, A->d_vtf, sizeof(float) * (size_t)A->nnz, hipMemcpyDeviceToHost));
  return MPCG_OK;
}

int mpcg_get_shadows(mpcg_matrix *A, float *f32, uint16_t *bf16, uint16_t *f16, int8_t *rexp) {
  if (!A) return fail(MPCG_ERR_INVALID, "A is NULL");
  HIP_TRY(hipStreamSynchronize(A->stream));
  if (f32) HIP_TRY(hipMemcpy(f32, A->d_v32, sizeof(float) * A->nnz, hipMemcpyDeviceToHost));
  if (bf16) HIP_TRY(hipMemcpy(bf16, A->d_vbf, sizeof(uint16_t) * A->nnz, hipMemcpyDeviceToHost));
  if (f16) HIP_TRY(hipMemcpy(f16, A->d_vh, sizeof(uint16_t) * A->nnz, hipMemcpyDeviceToHost));
  if (rexp) HIP_TRY(hipMemcpy(rexp, A->d_rexp, A->n, hipMemcpyDeviceToHost));
  return MPCG_OK;
}

// ---------------------------------------------------------------- policies
int mpcg_policy_create(const mpcg_policy_desc *desc, mpcg_policy **out) {
  if (!desc || !out) return fail(MPCG_ERR_INVALID, "NULL argument");
  *out = nullptr;
  if (desc->kind < 0 || desc->kind > 3) return fail(MPCG_ERR_INVALID, "bad policy kind");
  if (!act_valid(desc->fixed_action)) return fail(MPCG_ERR_INVALID, "bad fixed_action (0..79 or 128..252)");
  if (desc->nfmt != 0 && desc->nfmt != 4 && desc->nfmt != 5) return fail(MPCG_ERR_INVALID, "nfmt must be 4 or 5");
  if (desc->nfmt == 5 && desc->per_op == 0 &&
      (desc->kind == MPCG_POLICY_QTABLE || desc->kind == MPCG_POLICY_QTABLE_TRAIN))
    return fail(MPCG_ERR_INVALID, "tf32 in the format set (nfmt 5) needs one table per operation (per_op 1 or 2)");
  if (!(desc->cost_tf32 >= 0.0) || !std::isfinite(desc->cost_tf32)) return fail(MPCG_ERR_INVALID, "bad cost_tf32");
  if (desc->b_it < 1 || desc->b_res < 1 || desc->b_res > kMaxEdges + 1 || desc->t_bin < 1 || desc->w_stag < 1)
    return fail(MPCG_ERR_INVALID, "bad bin parameters");
  if (desc->decision_period < 0) return fail(MPCG_ERR_INVALID, "negative decision_period");
  if (desc->per_op < 0 || desc->per_op > 2) return fail(MPCG_ERR_INVALID, "per_op must be 0, 1 or 2");
  mpcg_policy *P = new (std::nothrow) mpcg_policy();
  if (!P) return fail(MPCG_ERR_NOMEM, "host allocation failed");
  P->desc = *desc;
  int rc = policy_alloc(P);
  if (rc) {
    P->release();
    delete P;
    return rc;
  }
  *out = P;
  return MPCG_OK;
}

int mpcg_policy_destroy(mpcg_policy *P) {
  if (!P) return MPCG_OK;
  (void)sync_users(P);
  for (mpcg_matrix *A : P->users) A->pol = nullptr;   // back to the matrix's default policy
  P->users.clear();
  P->release();
  delete P;
  return MPCG_OK;
}

int mpcg_policy_set_qtable(mpcg_policy *P, const double *q) {
  if (!P || !q) return fail(MPCG_ERR_INVALID, "NULL argument");
  HIP_TRY(hipMemcpy(P->d_q, q, sizeof(double) * (size_t)P->n_states * kNAct, hipMemcpyHostToDevice));
  // the greedy action per state, by the device's rule (first strict maximum;
  // per operation with one table per operation)
  auto first_max = [](const double *row, int len) {
    int best = 0;
    double bv = row[0];
    for (int a = 1; a < len; ++a)
      if (row[a] > bv) { best = a; bv = row[a]; }
    return best;
  };
  P->qbest.resize((size_t)P->n_states);
  for (int s = 0; s < P->n_states; ++s) {
    const double *row = q + (size_t)s * kNAct;
    const int S = P->desc.nfmt == 5 ? 5 : 4;
    const int best = P->desc.per_op
                         ? act_compose(first_max(row, S), first_max(row + S, S),
                                       P->desc.per_op == 2 ? MPCG_FP64 : first_max(row + 2 * S, S))
                         : first_max(row, kNAct);
    P->qbest[s] = (uint8_t)best;
  }
  return MPCG_OK;
}

int mpcg_policy_get_qtable(mpcg_policy *P, double *q) {
  if (!P || !q) return fail(MPCG_ERR_INVALID, "NULL argument");
  {
    const int rc = sync_users(P);
    if (rc) return rc;
  }
  HIP_TRY(hipMemcpy(q, P->d_q, sizeof(double) * (size_t)P->n_states * kNAct, hipMemcpyDeviceToHost));
  return MPCG_OK;
}

int mpcg_policy_set_episode(mpcg_policy *P, int64_t episode, double epsilon) {
  if (!P) return fail(MPCG_ERR_INVALID, "P is NULL");
  if (!(epsilon >= 0.0 && epsilon <= 1.0)) return fail(MPCG_ERR_INVALID, "epsilon must be in [0, 1]");
  P->episode = episode;
  P->epsilon = epsilon;
  return MPCG_OK;
}

int mpcg_policy_set_mlp(mpcg_policy *P, const float *W1, const float *b1, const float *W2, const float *b2,
                        const float *W3, const float *b3) {
  if (!P || !W1 || !b1 || !W2 || !b2 || !W3 || !b3) return fail(MPCG_ERR_INVALID, "NULL argument");
  if (!P->d_mlp) HIP_TRY(dmalloc(&P->d_mlp, (size_t)kMlpParams));
  std::vector<float> h(kMlpParams);
  float *w = h.data();
  std::memcpy(w, W1, sizeof(float) * kMlpH * kMlpIn); w += kMlpH * kMlpIn;
  std::memcpy(w, b1, sizeof(float) * kMlpH); w += kMlpH;
  std::memcpy(w, W2, sizeof(float) * kMlpH * kMlpH); w += kMlpH * kMlpH;
  std::memcpy(w, b2, sizeof(float) * kMlpH); w += kMlpH;
  std::memcpy(w, W3, sizeof(float) * kNAct * kMlpH); w += kNAct * kMlpH;
  std::memcpy(w, b3, sizeof(float) * kNAct);
  HIP_TRY(hipMemcpy(P->d_mlp, h.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
  P->has_mlp = true;
  return MPCG_OK;
}

int mpcg_policy_rollouts_enable(mpcg_policy *P, int32_t capacity) {
  if (!P || capacity < 0) return fail(MPCG_ERR_INVALID, "bad argument");
  {
    const int rc = sync_users(P);
    if (rc) return rc;
  }
  dfree(P->d_rf); dfree(P->d_rn); dfree(P->d_rr); dfree(P->d_ra); dfree(P->d_rd);
  P->roll_cap = 0;
  if (capacity > 0) {
    HIP_TRY(dmalloc(&P->d_rf, (size_t)capacity * kMlpIn));
    HIP_TRY(dmalloc(&P->d_rn, (size_t)capacity * kMlpIn));
    HIP_TRY(dmalloc(&P->d_rr, (size_t)capacity));
    HIP_TRY(dmalloc(&P->d_ra, (size_t)capacity));
    HIP_TRY(dmalloc(&P->d_rd, (size_t)capacity));
    P->roll_cap = capacity;
  }
  HIP_TRY(hipMemset(P->d_rcount, 0, sizeof(int32_t)));
  return MPCG_OK;
}

int mpcg_policy_rollouts_count(mpcg_policy *P, int32_t *n) {
  if (!P || !n) return fail(MPCG_ERR_INVALID, "NULL argument");
  {
    const int rc = sync_users(P);
    if (rc) return rc;
  }
  HIP_TRY(hipMemcpy(n, P->d_rcount, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (*n > P->roll_cap) *n = P->roll_cap;
  return MPCG_OK;
}

int mpcg_policy_rollouts_reset(mpcg_policy *P) {
  if (!P) return fail(MPCG_ERR_INVALID, "P is NULL");
  {
    const int rc = sync_users(P);
    if (rc) return rc;
  }
  HIP_TRY(hipMemset(P->d_rcount, 0, sizeof(int32_t)));
  return MPCG_OK;
}

int mpcg_policy_get_rollouts(mpcg_policy *P, float *feat, float *next_feat, int32_t *act, float *rew,
                             uint8_t *done, int32_t cap, int32_t *n_out) {
  if (!P) return fail(MPCG_ERR_INVALID, "P is NULL");
  int32_t n = 0;
  int rc = mpcg_policy_rollouts_count(P, &n);
  if (rc) return rc;
  n = std::min(n, cap);
  if (n > 0) {
    if (feat) HIP_TRY(hipMemcpy(feat, P->d_rf, sizeof(float) * n * kMlpIn, hipMemcpyDeviceToHost));
    if (next_feat) HIP_TRY(hipMemcpy(next_feat, P->d_rn, sizeof(float) * n * kMlpIn, hipMemcpyDeviceToHost));
    if (act) HIP_TRY(hipMemcpy(act, P->d_ra, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    if (rew) HIP_TRY(hipMemcpy(rew, P->d_rr, sizeof(float) * n, hipMemcpyDeviceToHost));
    if (done) HIP_TRY(hipMemcpy(done, P->d_rd, n, hipMemcpyDeviceToHost));
  }
  if (n_out) *n_out = n;
  return MPCG_OK;
}

int mpcg_policy_decide(mpcg_policy *P, int32_t m, const int64_t *k, const double *rho, const int32_t *stag,
                       const float *feat, int32_t *state, int32_t *action) {
  if (!P || m < 0 || (m > 0 && (!k || !rho || !stag || !state || !action)))
    return fail(MPCG_ERR_INVALID, "bad argument");
  if (P->desc.kind == MPCG_POLICY_MLP && (!feat || !P->has_mlp))
    return fail(MPCG_ERR_INVALID, "MLP policy needs weights and features");
  if (m == 0) return MPCG_OK;
  PolicyDev *dP = nullptr;
  int64_t *dk = nullptr;
  double *drho = nullptr;
  int32_t *dst = nullptr, *ds = nullptr, *da = nullptr;
  float *df = nullptr;
  int rc = MPCG_OK;
  PolicyDev hp = P->device_struct();
  hipError_t e = dmalloc(&dP, 1);
  if (e == hipSuccess) e = dmalloc(&dk, m);
  if (e == hipSuccess) e = dmalloc(&drho, m);
  if (e == hipSuccess) e = dmalloc(&dst, m);
  if (e == hipSuccess) e = dmalloc(&ds, m);
  if (e == hipSuccess) e = dmalloc(&da, m);
  if (e == hipSuccess && feat) e = dmalloc(&df, (size_t)m * kMlpIn);
  if (e == hipSuccess) e = hipMemcpy(dP, &hp, sizeof(hp), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dk, k, sizeof(int64_t) * m, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(drho, rho, sizeof(double) * m, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dst, stag, sizeof(int32_t) * m, hipMemcpyHostToDevice);
  if (e == hipSuccess && feat) e = hipMemcpy(df, feat, sizeof(float) * m * kMlpIn, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    launch_policy_decide(dP, m, dk, drho, dst, df, ds, da, nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(state, ds, sizeof(int32_t) * m, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(action, da, sizeof(int32_t) * m, hipMemcpyDeviceToHost);
  if (e != hipSuccess) rc = fail(MPCG_ERR_DEVICE, std::string("policy_decide: ") + hipGetErrorString(e));
  dfree(dP); dfree(dk); dfree(drho); dfree(dst); dfree(ds); dfree(da); dfree(df);
  return rc;
}

int mpcg_set_policy(mpcg_matrix *A, mpcg_policy *P) {
  if (!A) return fail(MPCG_ERR_INVALID, "A is NULL");
  if (P && P->desc.kind == MPCG_POLICY_MLP && !P->has_mlp) return fail(MPCG_ERR_INVALID, "MLP policy has no weights");
  if (A->pol) A->pol->users.erase(A);
  A->pol = P;
  if (P) P->users.insert(A);
  return MPCG_OK;
}

int mpcg_set_options(mpcg_matrix *A, const mpcg_solve_opts *o) {
  if (!A || !o) return fail(MPCG_ERR_INVALID, "NULL argument");
  if (o->replace_period < 0 || o->chunk < 0) return fail(MPCG_ERR_INVALID, "negative option");
  if (o->spmv_rows != 0 && o->spmv_rows != 512 && o->spmv_rows != 1024 && o->spmv_rows != 2048)
    return fail(MPCG_ERR_INVALID, "spmv_rows must be 0, 512, 1024 or 2048");
  if (o->index16 != 0 && o->index16 != -1) return fail(MPCG_ERR_INVALID, "index16 must be 0 or -1");
  if (o->precond != 0 && o->precond != 1) return fail(MPCG_ERR_INVALID, "precond must be 0 or 1");
  if (o->stop_rule != 0 && o->stop_rule != 1) return fail(MPCG_ERR_INVALID, "stop_rule must be 0 or 1");
  if (o->rho_fp64 != 0 && o->rho_fp64 != 1) return fail(MPCG_ERR_INVALID, "rho_fp64 must be 0 or 1");
  if (o->emulate != 0 && o->emulate != 1) return fail(MPCG_ERR_INVALID, "emulate must be 0 or 1");
  if (o->vec16 != 0 && o->vec16 != 1) return fail(MPCG_ERR_INVALID, "vec16 must be 0 or 1");
  if (o->vec16 && (o->precond || o->rho_fp64 || o->emulate))
    return fail(MPCG_ERR_INVALID, "vec16 runs without the preconditioner, fp64 rho and the emulation reading");
  if (o->variant < 0 || o->variant > 2) return fail(MPCG_ERR_INVALID, "variant must be 0, 1 or 2");
  if (o->variant != 0 &&
      (o->fallback || o->precond || o->stop_rule || o->rho_fp64 || o->emulate || o->vec16 || o->profile))
    return fail(MPCG_ERR_INVALID,
                "the single-reduction and pipelined variants run without fallback, precond, stop_rule, "
                "rho_fp64, emulate, vec16 and profile");
  A->opts = *o;
  return MPCG_OK;
}

// ---------------------------------------------------------------- solve
// Policy descriptor and initial control block of a solve (start: fp64 action,
// residual of x0), staged through the handle's pinned buffers.
static int upload_start(mpcg_matrix *A, mpcg_policy *P, double tol, int32_t maxit, hipStream_t st) {
  *A->h_pol = P->device_struct();
  HIP_TRY(hipMemcpyAsync(A->d_pol, A->h_pol, sizeof(PolicyDev), hipMemcpyHostToDevice, st));
  Ctl &c = *A->h_ctl;
  std::memset(&c, 0, sizeof(Ctl));
  c.mode = M_INIT;
  c.tier = 1;
  c.action = 63;
  c.maxit = maxit;
  c.status = -1;
  c.fallback_at = -1;
  c.prev_action = 63;
  c.R = A->opts.replace_period;
  c.fallback_enabled = A->opts.fallback ? 1 : 0;
  c.precond = A->opts.precond;
  c.stop_rule = A->opts.stop_rule;
  c.rho64 = A->opts.rho_fp64;
  c.emul = A->opts.emulate;
  c.vec16 = A->opts.vec16;
  c.tol = tol;
  HIP_TRY(hipMemcpyAsync(A->d_ctl, A->h_ctl, sizeof(Ctl), hipMemcpyHostToDevice, st));
  return MPCG_OK;
}

static void fill_result(const Ctl &r, mpcg_result *res) {
  std::memset(res, 0, sizeof(*res));
  res->status = r.status;
  res->iters = r.k;
  res->n_replace = r.nrep;
  res->fallback_at = r.fell_back ? r.fallback_at : -1;
  res->relres_true = r.relres_true;
  res->cost_sum = r.cost_sum;
}

int mpcg_solve(mpcg_matrix *A, const double *b, double *x, double tol, int32_t maxit, mpcg_result *res) {
  if (!A || !b || !x || !res) return fail(MPCG_ERR_INVALID, "NULL argument");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(MPCG_ERR_INVALID, "tol must be positive and finite");
  if (maxit < 0 || maxit > (1 << 29)) return fail(MPCG_ERR_INVALID, "maxit out of range");
  int rc = ensure_ws(A);
  if (rc) return rc;
  rc = ensure_hist(A, maxit);
  if (rc) return rc;
  mpcg_policy *P = A->pol ? A->pol : A->defpol;
  if (P->desc.kind == MPCG_POLICY_MLP && !P->has_mlp) return fail(MPCG_ERR_INVALID, "MLP policy has no weights");
  if (A->opts.emulate && P->desc.kind == MPCG_POLICY_FIXED && act_fs(P->desc.fixed_action) == FP8)
    return fail(MPCG_ERR_INVALID, "the emulation reading has no q52 SpMV (Table 1's q52 is storage only here)");
  if (A->opts.variant != 0 && (P->desc.kind != MPCG_POLICY_FIXED || P->desc.fixed_action >= 80))
    return fail(MPCG_ERR_INVALID, "the single-reduction and pipelined variants take a fixed policy with an action 0..79");
  if (A->opts.variant != 0 && P->roll_cap > 0)
    return fail(MPCG_ERR_INVALID, "the single-reduction and pipelined variants log no rollouts");
  hipStream_t st = A->stream;
  HIP_TRY(hipStreamSynchronize(st));   // staging buffers below are reused
  if (A->opts.variant != 0) return solve_sr(A, P, b, x, tol, maxit, res);

  rc = upload_start(A, P, tol, maxit, st);
  if (rc) return rc;

  KArgs a = make_args(A, b, x);
  // the kernels with tf32 and the emulation reading, when the options or the
  // policy can use them
  a.ext = (A->opts.emulate || (P->desc.kind == MPCG_POLICY_FIXED && P->desc.fixed_action >= 128) ||
           P->desc.nfmt == 5) ? 1 : 0;
  // Q-learning writes the table during the solve: one-block steps.  The
  // network and rollout logging only read shared state: every KB workgroup
  // runs the full step (workgroup 0 writing the logs), and the per-iteration
  // decision runs once, in the one-block step kernel before KX.
  a.slow = P->desc.kind == MPCG_POLICY_QTABLE_TRAIN ? 1 : 0;
  a.full = !a.slow && (P->desc.kind == MPCG_POLICY_MLP || P->roll_cap > 0) ? 1 : 0;
  const bool step_x = a.slow || a.full;
  a.net = (P->desc.kind == MPCG_POLICY_MLP && P->has_mlp) ? P->d_mlp : nullptr;
  const int per_slot = 6 + (a.slow ? 2 : 0) + (step_x ? 2 : 0);   // a start and a stop event per launch
  const int chunk = A->opts.chunk > 0 ? A->opts.chunk : 32;
  const bool prof = A->opts.profile != 0;
  std::memset(&A->prof, 0, sizeof(A->prof));
  if (prof) {
    a.slot_log = A->d_slotlog;
    const size_t need = (size_t)2 * chunk * per_slot;
    while (A->pev.size() < need) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e));
      A->pev.push_back(e);
    }
    A->ta.assign(A->slot_cap, 0.0f);
    A->tb.assign(A->slot_cap, 0.0f);
    A->tx.assign(A->slot_cap, 0.0f);
    A->ts.assign(A->slot_cap, 0.0f);
  }
  HIP_TRY(hipEventRecord(A->ev_start, st));
  launch_start(a, st);
  HIP_TRY(hipGetLastError());
  const int64_t max_slots = 2 * (int64_t)maxit + 16;
  int64_t slots = 0;
  int ci = 0;
  bool done = false;
  int64_t chunk_first[2] = {0, 0};
  int chunk_m[2] = {0, 0};
  bool pending[2] = {false, false};
  ChunkPlan plan{chunk, tol};
  while (slots < max_slots) {
    const int m = (int)std::min<int64_t>(plan.next(), max_slots - slots);
    plan.in_flight = m;
    const int idx = ci & 1;
    chunk_first[idx] = slots;
    chunk_m[idx] = m;
    for (int s = 0; s < m; ++s) {
      if (prof) {
        hipEvent_t *e = &A->pev[((size_t)idx * chunk + s) * per_slot];
        a.slot = (int)(slots + s);
        launch_ka(a, st, e[0], e[1]);
        int ei = 2;
        if (a.slow) {
          launch_step_b(a, st, e[ei], e[ei + 1]);
          ei += 2;
        }
        launch_kb(a, st, e[ei], e[ei + 1]);
        ei += 2;
        if (step_x) {
          launch_step_x(a, st, e[ei], e[ei + 1]);
          ei += 2;
        }
        launch_kx(a, st, e[ei], e[ei + 1]);
      } else {
        launch_slot(a, st);
      }
    }
    HIP_TRY(hipGetLastError());
    slots += m;
    pending[idx] = true;
    HIP_TRY(hipMemcpyAsync(&A->h_poll[idx], A->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(A->ev_chunk[idx], st));
    if (ci > 0) {
      const int pidx = (ci - 1) & 1;
      HIP_TRY(hipEventSynchronize(A->ev_chunk[pidx]));
      if (prof && pending[pidx]) {
        int rc2 = collect_chunk(A, pidx, chunk, per_slot, a.slow, step_x, chunk_first[pidx], chunk_m[pidx]);
        if (rc2) return rc2;
      }
      pending[pidx] = false;
      const Ctl &pc = A->h_poll[pidx];
      if (pc.mode == M_DONE) {
        done = true;
        break;
      }
      plan.observe(pc.k, pc.rho_new);
    }
    ci++;
  }
  HIP_TRY(hipStreamSynchronize(st));
  if (prof) {
    for (int i = 0; i < 2; ++i)
      if (pending[i]) {
        int rc2 = collect_chunk(A, i, chunk, per_slot, a.slow, step_x, chunk_first[i], chunk_m[i]);
        if (rc2) return rc2;
      }
  }
  if (!done) {
    HIP_TRY(hipMemcpy(&A->h_poll[0], A->d_ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    if (A->h_poll[0].mode != M_DONE) return fail(MPCG_ERR_DEVICE, "solver did not reach a final state");
  }
  a.slot_log = nullptr;
  launch_finish(a, st);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(A->ev_end, st));
  // The finishing KB leaves the final state in ctl[1].
  HIP_TRY(hipMemcpyAsync(A->h_ctl, A->d_ctl + 1, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, A->ev_start, A->ev_end));
  const Ctl &r = *A->h_ctl;
  fill_result(r, res);
  res->time_ms = ms;
  res->slots = (int32_t)slots;
  res->spmv_rows = a.grows;
  res->index16 = a.A.dc ? 1 : 0;
  A->last_iters = r.k;
  A->last_nrep = r.nrep;
  if (prof) {
    std::vector<int8_t> modes((size_t)slots);
    HIP_TRY(hipMemcpy(modes.data(), A->d_slotlog, (size_t)slots, hipMemcpyDeviceToHost));
    mpcg_profile &pr = A->prof;
    for (int64_t s = 0; s < slots; ++s) {
      const double all = (double)A->ta[s] + A->tb[s] + A->tx[s] + A->ts[s];
      if (modes[s] == M_ITER) {
        pr.n_iter_slots++;
        pr.ka_iter_ms += A->ta[s];
        pr.kb_iter_ms += A->tb[s];
        pr.kx_iter_ms += A->tx[s];
        pr.ks_iter_ms += A->ts[s];
      } else if (modes[s] == M_DONE) {
        pr.n_idle_slots++;
        pr.idle_ms += all;
      } else {
        pr.n_resid_slots++;
        pr.resid_ms += all;
      }
    }
  }
  return MPCG_OK;
}

// ---------------------------------------------------------------- batched
namespace {

struct BatchCfg {
  int workgroups, spmv_rows, split_rows;   // split_rows < 0: no split
  int lockstep;                            // 1: lockstep kernels instead of the persistent launch
};

// Autotuner memory: the configuration chosen for a batch shape.
struct BatchKey {
  int nsys;
  int64_t sum_n, sum_nnz;
  bool operator<(const BatchKey &o) const {
    return std::tie(nsys, sum_n, sum_nnz) < std::tie(o.nsys, o.sum_n, o.sum_nnz);
  }
};
std::map<BatchKey, BatchCfg> g_batch_tuned;
std::mutex g_batch_mu;

}  // namespace

// One batched launch over the prepared systems with configuration cfg; x[i]
// receives the solutions (the caller's buffers or the autotuner's copies).
static int batch_run(int nsys, mpcg_matrix *const *A, const double *const *b, double *const *x, const double *tol,
                     const int32_t *maxit, const std::vector<mpcg_policy *> &pols, const std::vector<int32_t> &order,
                     const BatchCfg &cfg, hipStream_t st, float *ms_out) {
  std::vector<BatchSys> hs((size_t)nsys);
  for (int32_t i : order) {
    int rc = upload_start(A[i], pols[i], tol[i], maxit[i], st);
    if (rc) return rc;
    KArgs a = make_args(A[i], b[i], x[i]);
    a.grows = cfg.spmv_rows;
    a.P1 = (A[i]->n + a.grows - 1) / a.grows;
    a.G1 = round_up(a.P1, 8);
    hs[i].a = a;
    hs[i].max_slots = 2 * maxit[i] + 16;
  }
  BatchSys *d_sys = nullptr;
  int32_t *d_order = nullptr, *d_queue = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = MPCG_OK;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    dfree(d_sys);
    dfree(d_order);
    dfree(d_queue);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  hipError_t e = dmalloc(&d_sys, (size_t)nsys);
  if (e == hipSuccess) e = dmalloc(&d_order, (size_t)nsys);
  if (e == hipSuccess) e = dmalloc(&d_queue, 1);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipMemcpyAsync(d_sys, hs.data(), sizeof(BatchSys) * nsys, hipMemcpyHostToDevice, st);
  const int nq = (int)order.size();
  if (e == hipSuccess) e = hipMemcpyAsync(d_order, order.data(), sizeof(int32_t) * nq, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(d_queue, 0, sizeof(int32_t), st);
  if (e == hipSuccess) {
    launch_batched(d_sys, d_order, nq, d_queue, cfg.workgroups, st, e0, e1);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess && ms_out) e = hipEventElapsedTime(ms_out, e0, e1);
  if (e != hipSuccess)
    rc = fail(e == hipErrorOutOfMemory ? MPCG_ERR_NOMEM : MPCG_ERR_DEVICE,
              std::string("batched launch: ") + hipGetErrorString(e));
  cleanup();
  return rc;
}

// Lockstep strategy: each iteration is three launches over the row groups /
// vector blocks of every system still running.  The host enqueues chunks of
// iterations, gathers the systems' modes after each chunk and, one chunk
// behind, rebuilds the tables without the finished systems (double-buffered,
// so a table is rewritten only after the chunk that read it has completed).
static int batch_lockstep(int nsys, mpcg_matrix *const *A, const double *const *b, double *const *x,
                          const double *tol, const int32_t *maxit, const std::vector<mpcg_policy *> &pols,
                          const std::vector<int32_t> &order, const BatchCfg &cfg, hipStream_t st, float *ms_out) {
  std::vector<BatchSys> hs((size_t)nsys);
  int slow = 0, max_slots = 16;
  for (int32_t i : order) {
    int rc = upload_start(A[i], pols[i], tol[i], maxit[i], st);
    if (rc) return rc;
    KArgs a = make_args(A[i], b[i], x[i]);
    a.grows = cfg.spmv_rows;
    a.P1 = (A[i]->n + a.grows - 1) / a.grows;
    a.G1 = round_up(a.P1, 8);
    hs[i].a = a;
    hs[i].max_slots = 2 * maxit[i] + 16;
    max_slots = std::max(max_slots, hs[i].max_slots);
    if (pols[i]->desc.kind == MPCG_POLICY_MLP) slow = 1;
  }
  size_t cap_ka = 0, cap_vb = 0;
  for (int32_t i : order) {
    cap_ka += (size_t)hs[i].a.P1;
    cap_vb += (size_t)hs[i].a.P2;
  }
  const size_t nq = order.size();
  BatchSys *d_sys = nullptr;
  SysBlk *d_ka[2] = {nullptr, nullptr}, *d_vb[2] = {nullptr, nullptr};
  int32_t *d_act[2] = {nullptr, nullptr}, *d_modes = nullptr, *h_modes = nullptr;
  SysBlk *h_tab = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr, ev[2] = {nullptr, nullptr};
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    dfree(d_sys);
    for (int j = 0; j < 2; ++j) { dfree(d_ka[j]); dfree(d_vb[j]); dfree(d_act[j]); }
    dfree(d_modes);
    if (h_modes) (void)hipHostFree(h_modes);
    if (h_tab) (void)hipHostFree(h_tab);
    for (hipEvent_t *p : {&e0, &e1, &ev[0], &ev[1]})
      if (*p) (void)hipEventDestroy(*p);
  };
#define LS_TRY(expr)                                                                              \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) {                                                                       \
      cleanup();                                                                                  \
      return fail(e_ == hipErrorOutOfMemory ? MPCG_ERR_NOMEM : MPCG_ERR_DEVICE,                   \
                  std::string("lockstep: ") + #expr + ": " + hipGetErrorString(e_));             \
    }                                                                                             \
  } while (0)
  LS_TRY(dmalloc(&d_sys, (size_t)nsys));
  for (int j = 0; j < 2; ++j) {
    LS_TRY(dmalloc(&d_ka[j], cap_ka));
    LS_TRY(dmalloc(&d_vb[j], cap_vb));
    LS_TRY(dmalloc(&d_act[j], nq));
  }
  LS_TRY(dmalloc(&d_modes, nq));
  // pinned staging: modes of the two chunks in flight, and the tables of the
  // two buffers (ka, vb, act each)
  LS_TRY(hipHostMalloc((void **)&h_modes, sizeof(int32_t) * 2 * nq, hipHostMallocDefault));
  const size_t tab_words = cap_ka + cap_vb + (nq + 1) / 2 + 1;
  LS_TRY(hipHostMalloc((void **)&h_tab, sizeof(SysBlk) * 2 * tab_words, hipHostMallocDefault));
  LS_TRY(hipEventCreate(&e0));
  LS_TRY(hipEventCreate(&e1));
  LS_TRY(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  LS_TRY(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  LS_TRY(hipMemcpyAsync(d_sys, hs.data(), sizeof(BatchSys) * nsys, hipMemcpyHostToDevice, st));
  int nka[2] = {0, 0}, nvb[2] = {0, 0}, nact[2] = {0, 0};
  std::vector<int32_t> act_list[2];
  // writes the tables of `active` into buffer j (pinned staging, then device)
  auto build = [&](int j, const std::vector<int32_t> &active) -> hipError_t {
    SysBlk *ka = h_tab + (size_t)j * tab_words, *vb = ka + cap_ka;
    int32_t *ac = (int32_t *)(vb + cap_vb);
    int a1 = 0, a2 = 0;
    for (int32_t s : active) {
      for (int g = 0; g < hs[s].a.P1; ++g) ka[a1++] = SysBlk{s, g};
      for (int q = 0; q < hs[s].a.P2; ++q) vb[a2++] = SysBlk{s, q};
    }
    for (size_t t = 0; t < active.size(); ++t) ac[t] = active[t];
    nka[j] = a1;
    nvb[j] = a2;
    nact[j] = (int)active.size();
    act_list[j] = active;
    hipError_t e = hipSuccess;
    if (a1) e = hipMemcpyAsync(d_ka[j], ka, sizeof(SysBlk) * a1, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && a2) e = hipMemcpyAsync(d_vb[j], vb, sizeof(SysBlk) * a2, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && nact[j])
      e = hipMemcpyAsync(d_act[j], ac, sizeof(int32_t) * nact[j], hipMemcpyHostToDevice, st);
    return e;
  };
  std::vector<int32_t> all(order.begin(), order.end());
  LS_TRY(build(0, all));
  LS_TRY(build(1, all));
  LS_TRY(hipEventRecord(e0, st));
  launch_lock_start(d_sys, d_vb[0], nvb[0], st);
  LS_TRY(hipGetLastError());
  const int chunk = 16;
  int64_t slots = 0;
  int ci = 0;
  bool done = false;
  while (slots < max_slots && !done) {
    const int j = ci & 1;
    const int m = (int)std::min<int64_t>(chunk, max_slots - slots);
    for (int s = 0; s < m; ++s)
      launch_lock_slot(d_sys, d_ka[j], nka[j], d_vb[j], nvb[j], d_act[j], nact[j], slow, st);
    launch_lock_modes(d_sys, d_act[j], nact[j], d_modes, st);
    LS_TRY(hipGetLastError());
    if (nact[j]) LS_TRY(hipMemcpyAsync(h_modes + (size_t)j * nq, d_modes, sizeof(int32_t) * nact[j],
                                       hipMemcpyDeviceToHost, st));
    LS_TRY(hipEventRecord(ev[j], st));
    slots += m;
    // one chunk behind: the modes after chunk ci-1 give the active set of chunk ci+1
    if (ci > 0) {
      const int pj = (ci - 1) & 1;
      LS_TRY(hipEventSynchronize(ev[pj]));
      std::vector<int32_t> next;
      for (int t = 0; t < nact[pj]; ++t)
        if (h_modes[(size_t)pj * nq + t] != M_DONE) next.push_back(act_list[pj][t]);
      if (next.empty()) {
        done = true;
        break;
      }
      LS_TRY(build(pj, next));   // buffer pj is next used by chunk ci+1
    }
    ci++;
  }
  LS_TRY(hipStreamSynchronize(st));
  // the final state of every system: fold and x; a final true residual after a
  // budget stop or a breakdown
  LS_TRY(build(0, all));
  launch_lock_finish(d_sys, d_ka[0], nka[0], d_vb[0], nvb[0], d_act[0], nact[0], slow, st);
  LS_TRY(hipGetLastError());
  LS_TRY(hipEventRecord(e1, st));
  LS_TRY(hipStreamSynchronize(st));
  if (ms_out) LS_TRY(hipEventElapsedTime(ms_out, e0, e1));
#undef LS_TRY
  cleanup();
  return MPCG_OK;
}

// The whole batch under cfg: systems above the split through mpcg_solve (one
// after the other, after the persistent launch), the others in the launch.
// res may be NULL (trials).  Device times of both parts in ms_p / ms_s.
static int batch_all(int nsys, mpcg_matrix *const *A, const double *const *b, double *const *x, const double *tol,
                     const int32_t *maxit, const std::vector<mpcg_policy *> &pols, const std::vector<int32_t> &order,
                     const BatchCfg &cfg, hipStream_t st, mpcg_result *res, float *ms_p, float *ms_s, int *n_split) {
  std::vector<int32_t> small_order, large;
  for (int32_t i : order) {
    if (cfg.split_rows >= 0 && A[i]->n > cfg.split_rows) large.push_back(i);
    else small_order.push_back(i);
  }
  *ms_p = 0.0f;
  *ms_s = 0.0f;
  *n_split = (int)large.size();
  if (!small_order.empty()) {
    // the persistent kernel (or the lockstep kernels) over small_order
    int rc = cfg.lockstep ? batch_lockstep(nsys, A, b, x, tol, maxit, pols, small_order, cfg, st, ms_p)
                          : batch_run(nsys, A, b, x, tol, maxit, pols, small_order, cfg, st, ms_p);
    if (rc) return rc;
  }
  for (int32_t i : large) {
    mpcg_matrix *M = A[i];
    mpcg_policy *saved = M->pol;
    M->pol = pols[i];
    mpcg_result r;
    const int rc = mpcg_solve(M, b[i], x[i], tol[i], maxit[i], &r);
    M->pol = saved;
    if (rc) return rc;
    *ms_s += (float)r.time_ms;
    if (res) res[i] = r;
  }
  return MPCG_OK;
}

int mpcg_solve_batched(int32_t nsys, mpcg_matrix *const *A, const double *const *b, double *const *x,
                       const double *tol, const int32_t *maxit, const mpcg_batch_opts *opts, mpcg_result *res,
                       mpcg_batch_info *info) {
  if (nsys < 0 || (nsys > 0 && (!A || !b || !x || !tol || !maxit || !res)))
    return fail(MPCG_ERR_INVALID, "NULL or negative argument");
  mpcg_batch_opts o{0, 0, 0, 0, 0, 0};
  if (opts) o = *opts;
  if (o.workgroups < 0 || (o.spmv_rows != 0 && o.spmv_rows != 512 && o.spmv_rows != 1024 && o.spmv_rows != 2048) ||
      (o.order != 0 && o.order != 1) || o.autotune_iters < 0 || o.split_rows < -1 || o.strategy < 0 ||
      o.strategy > 2)
    return fail(MPCG_ERR_INVALID, "bad batch options");
  if (info) std::memset(info, 0, sizeof(*info));
  if (nsys == 0) return MPCG_OK;
  std::vector<mpcg_policy *> pols((size_t)nsys);
  int64_t sum_n = 0, sum_nnz = 0;
  for (int i = 0; i < nsys; ++i) {
    if (!A[i] || !b[i] || !x[i]) return fail(MPCG_ERR_INVALID, "NULL system");
    if (!(tol[i] > 0.0) || !std::isfinite(tol[i])) return fail(MPCG_ERR_INVALID, "tol must be positive and finite");
    if (maxit[i] < 0 || maxit[i] > (1 << 29)) return fail(MPCG_ERR_INVALID, "maxit out of range");
    if (A[i]->opts.precond) return fail(MPCG_ERR_INVALID, "batched solves are not preconditioned (precond = 0)");
    if (A[i]->opts.rho_fp64) return fail(MPCG_ERR_INVALID, "batched solves take rho at the dot format (rho_fp64 = 0)");
    if (A[i]->opts.emulate) return fail(MPCG_ERR_INVALID, "batched solves run the hardware reading (emulate = 0)");
    if (A[i]->opts.vec16) return fail(MPCG_ERR_INVALID, "batched solves keep fp32 vector containers (vec16 = 0)");
    if (A[i]->opts.variant) return fail(MPCG_ERR_INVALID, "batched solves run section 3's iteration (variant = 0)");
    mpcg_policy *P = A[i]->pol ? A[i]->pol : A[i]->defpol;
    if (P->desc.kind == MPCG_POLICY_QTABLE_TRAIN || P->roll_cap > 0)
      return fail(MPCG_ERR_INVALID, "training policies and rollout logs are not batched (shared state)");
    if (P->desc.kind == MPCG_POLICY_MLP && !P->has_mlp) return fail(MPCG_ERR_INVALID, "MLP policy has no weights");
    if (P->desc.fixed_action >= 128 || P->desc.nfmt == 5)
      return fail(MPCG_ERR_INVALID, "batched solves take the four arithmetic formats and q52 (no tf32)");
    pols[i] = P;
    int rc = ensure_ws(A[i]);
    if (rc) return rc;
    rc = ensure_hist(A[i], maxit[i]);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(A[i]->stream));
    sum_n += A[i]->n;
    sum_nnz += A[i]->nnz;
  }
  {
    std::vector<mpcg_matrix *> u(A, A + nsys);
    std::sort(u.begin(), u.end());
    if (std::adjacent_find(u.begin(), u.end()) != u.end())
      return fail(MPCG_ERR_INVALID, "a matrix handle appears twice in the batch");
  }
  hipStream_t st = A[0]->stream;
  std::vector<int32_t> order((size_t)nsys);
  for (int i = 0; i < nsys; ++i) order[i] = i;
  if (o.order == 0)
    std::stable_sort(order.begin(), order.end(), [&](int32_t p, int32_t q) { return A[p]->nnz > A[q]->nnz; });

  // strategy 1: persistent launch; 2: lockstep kernels (workgroups and split
  // do not apply); 0: the autotuner chooses.
  BatchCfg cfg{o.workgroups, o.spmv_rows, o.split_rows, o.strategy == 2 ? 1 : 0};
  if (o.strategy == 2) {
    cfg.workgroups = 1;
    cfg.split_rows = -1;
  }
  int tuned = 0;
  double tune_ms = 0.0;
  if (o.strategy == 0 || cfg.workgroups == 0 || cfg.spmv_rows == 0 || cfg.split_rows == 0) {
    const BatchKey key{nsys, sum_n, sum_nnz};
    bool have = false;
    {
      std::lock_guard<std::mutex> lk(g_batch_mu);
      auto it = g_batch_tuned.find(key);
      if (it != g_batch_tuned.end()) {
        if (o.strategy == 0) cfg = it->second;
        if (cfg.workgroups == 0) cfg.workgroups = it->second.workgroups;
        if (cfg.spmv_rows == 0) cfg.spmv_rows = it->second.spmv_rows;
        if (cfg.split_rows == 0) cfg.split_rows = it->second.split_rows;
        have = true;
        tuned = 2;
      }
    }
    if (!have) {
      // Timed trials of a few iterations per system on copies of x0; every
      // candidate gives the same results, only the time differs.
      std::vector<int> wgs, rows, splits;
      if (cfg.workgroups) wgs = {cfg.workgroups};
      else wgs = {256, 512};
      if (cfg.spmv_rows) rows = {cfg.spmv_rows};
      else rows = {512, 2048};
      if (cfg.split_rows) splits = {cfg.split_rows};
      else splits = {-1, 100000, 30000, 10000};
      std::vector<double *> xt((size_t)nsys, nullptr);
      std::vector<int32_t> mt((size_t)nsys);
      const int ti = o.autotune_iters > 0 ? o.autotune_iters : 16;
      int rc = MPCG_OK;
      for (int i = 0; i < nsys && rc == MPCG_OK; ++i) {
        hipError_t e = dmalloc(&xt[i], (size_t)A[i]->n);
        if (e == hipSuccess)
          e = hipMemcpyAsync(xt[i], x[i], sizeof(double) * A[i]->n, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) rc = fail(MPCG_ERR_NOMEM, "autotuner scratch");
        mt[i] = std::min(maxit[i], ti);
      }
      std::vector<BatchCfg> cands;
      if (o.strategy != 2)
        for (int w : wgs)
          for (int r : rows)
            for (int sp : splits) cands.push_back(BatchCfg{w, r, sp, 0});
      if (o.strategy != 1)
        for (int r : rows) cands.push_back(BatchCfg{1, r, -1, 1});
      BatchCfg best{0, 0, 0, 0};
      float best_ms = 0.0f;
      for (const BatchCfg &cand : cands) {
        if (rc) break;
        float mp = 0.0f, ms_ = 0.0f;
        int ns = 0;
        rc = batch_all(nsys, A, b, xt.data(), tol, mt.data(), pols, order, cand, st, nullptr, &mp, &ms_, &ns);
        const float t = mp + ms_;
        tune_ms += t;
        if (!rc && (best.workgroups == 0 || t < best_ms)) {
          best = cand;
          best_ms = t;
        }
        // the trial overwrote x: restore the copies of x0 for the next one
        for (int i = 0; i < nsys && !rc; ++i)
          if (hipMemcpyAsync(xt[i], x[i], sizeof(double) * A[i]->n, hipMemcpyDeviceToDevice, st) != hipSuccess)
            rc = fail(MPCG_ERR_DEVICE, "autotuner copy");
      }
      (void)hipStreamSynchronize(st);
      for (double *p : xt) dfree(p);
      if (rc) return rc;
      cfg = best;
      tuned = 1;
      std::lock_guard<std::mutex> lk(g_batch_mu);
      g_batch_tuned[key] = best;
    }
  }
  float ms_p = 0.0f, ms_s = 0.0f;
  int n_split = 0;
  int rc = batch_all(nsys, A, b, x, tol, maxit, pols, order, cfg, st, res, &ms_p, &ms_s, &n_split);
  if (rc) return rc;
  const float ms = ms_p + ms_s;
  for (int i = 0; i < nsys; ++i) {
    if (cfg.split_rows >= 0 && A[i]->n > cfg.split_rows) {
      res[i].time_ms = ms;
      continue;
    }
    Ctl r;
    HIP_TRY(hipMemcpy(&r, A[i]->d_ctl + 1, sizeof(Ctl), hipMemcpyDeviceToHost));
    if (r.status < 0) return fail(MPCG_ERR_DEVICE, "batched solve did not reach a final state");
    fill_result(r, &res[i]);
    res[i].time_ms = ms;
    res[i].spmv_rows = cfg.spmv_rows;
    res[i].index16 = (A[i]->d_dc && A[i]->opts.index16 >= 0) ? 1 : 0;
    A[i]->last_iters = r.k;
    A[i]->last_nrep = r.nrep;
  }
  if (info) {
    info->time_ms = ms;
    info->tune_ms = tune_ms;
    info->workgroups = cfg.workgroups;
    info->spmv_rows = cfg.spmv_rows;
    info->tuned = tuned;
    info->split_rows = cfg.split_rows;
    info->n_split = n_split;
    info->persistent_ms = ms_p;
    info->split_ms = ms_s;
    info->strategy = cfg.lockstep ? 2 : 1;
  }
  return MPCG_OK;
}

// ---------------------------------------------------------------- training
int mpcg_train_qlearning(mpcg_policy *P, int32_t m, mpcg_matrix *const *A, const double *const *b,
                         double *const *x, const mpcg_train_desc *d, mpcg_episode_result *out) {
  if (!P || !A || !b || !x || !d || m < 0) return fail(MPCG_ERR_INVALID, "NULL or negative argument");
  if (P->desc.kind != MPCG_POLICY_QTABLE_TRAIN) return fail(MPCG_ERR_INVALID, "policy is not a training policy");
  if (d->episodes < 1 || d->maxit < 0 || !(d->tol > 0.0) || !std::isfinite(d->tol) || d->first_episode < 1 ||
      !(d->eps_start >= 0.0 && d->eps_start <= 1.0) || !(d->eps_end >= 0.0 && d->eps_end <= 1.0) ||
      (d->order != 0 && d->order != 1) || d->total_episodes < 0)
    return fail(MPCG_ERR_INVALID, "bad training descriptor");
  for (int i = 0; i < m; ++i)
    if (!A[i] || !b[i] || !x[i]) return fail(MPCG_ERR_INVALID, "NULL system");
  const int64_t total = d->total_episodes > 0 ? d->total_episodes
                                              : (int64_t)d->first_episode - 1 + (int64_t)m * d->episodes;
  const int64_t njobs = (int64_t)m * d->episodes;
  for (int64_t j = 0; j < njobs; ++j) {
    const int sys = d->order == 0 ? (int)(j / d->episodes) : (int)(j % m);
    const int64_t e = d->first_episode + j;
    const double eps = total > 1 ? d->eps_start + (d->eps_end - d->eps_start) * (double)(e - 1) / (double)(total - 1)
                                 : d->eps_start;
    mpcg_matrix *M = A[sys];
    P->episode = e;
    P->epsilon = std::min(1.0, std::max(0.0, eps));
    mpcg_policy *saved = M->pol;
    M->pol = P;
    HIP_TRY(hipMemsetAsync(x[sys], 0, sizeof(double) * (size_t)M->n, M->stream));
    mpcg_result r;
    const int rc = mpcg_solve(M, b[sys], x[sys], d->tol, d->maxit, &r);
    M->pol = saved;
    if (rc) return rc;
    if (out) {
      out[j].system = sys;
      out[j].episode = (int32_t)e;
      out[j].epsilon = P->epsilon;
      out[j].res = r;
    }
  }
  return MPCG_OK;
}

// ---------------------------------------------------------------- MLP trainer
struct mpcg_mlp {
  hipStream_t stream = nullptr;
  float *d_master = nullptr, *d_m = nullptr, *d_v = nullptr;
  uint16_t *d_wb = nullptr;     // bf16 copies: current and frozen
  float *d_bias = nullptr;      // biases: current and frozen
  MlpWeights cur{}, frozen{};
  float *d_part = nullptr, *d_ploss = nullptr;
  int part_cap = 0;             // workgroups the partial buffers hold
  float *d_target = nullptr, *d_ymax = nullptr;
  int64_t tcap = 0;
  float *d_grad = nullptr, *d_loss = nullptr;
  int64_t loss_cap = 0;
  int64_t steps = 0;            // Adam steps taken

  void release() {
    dfree(d_master); dfree(d_m); dfree(d_v); dfree(d_wb); dfree(d_bias);
    dfree(d_part); dfree(d_ploss); dfree(d_target); dfree(d_ymax); dfree(d_grad); dfree(d_loss);
  }
};

static void mlp_views(mpcg_mlp *N) {
  const int nw = kMlpH * kMlpIn + kMlpH * kMlpH + kNAct * kMlpH + kMlpH * kMlpH + kNAct * kMlpH;
  auto carve = [&](uint16_t *base, float *bias, MlpWeights &w) {
    w.w1b = base;
    w.w2b = w.w1b + kMlpH * kMlpIn;
    w.w3b = w.w2b + kMlpH * kMlpH;
    w.w2t = w.w3b + kNAct * kMlpH;
    w.w3t = w.w2t + kMlpH * kMlpH;
    w.b1 = bias;
    w.b2 = w.b1 + kMlpH;
    w.b3 = w.b2 + kMlpH;
  };
  carve(N->d_wb, N->d_bias, N->cur);
  carve(N->d_wb + nw, N->d_bias + 2 * kMlpH + kNAct, N->frozen);
}

static int mlp_ensure_part(mpcg_mlp *N, int nwg) {
  if (N->part_cap >= nwg) return MPCG_OK;
  dfree(N->d_part);
  dfree(N->d_ploss);
  HIP_TRY(dmalloc(&N->d_part, (size_t)nwg * kMlpParams));
  HIP_TRY(dmalloc(&N->d_ploss, (size_t)nwg));
  N->part_cap = nwg;
  return MPCG_OK;
}

int mpcg_mlp_create(const float *params, void *stream, mpcg_mlp **out) {
  if (!params || !out) return fail(MPCG_ERR_INVALID, "NULL argument");
  *out = nullptr;
  mpcg_mlp *N = new (std::nothrow) mpcg_mlp();
  if (!N) return fail(MPCG_ERR_NOMEM, "host allocation failed");
  N->stream = (hipStream_t)stream;
  const int nw = kMlpH * kMlpIn + kMlpH * kMlpH + kNAct * kMlpH + kMlpH * kMlpH + kNAct * kMlpH;
  hipError_t e = dmalloc(&N->d_master, (size_t)kMlpParams);
  if (e == hipSuccess) e = dmalloc(&N->d_m, (size_t)kMlpParams);
  if (e == hipSuccess) e = dmalloc(&N->d_v, (size_t)kMlpParams);
  if (e == hipSuccess) e = dmalloc(&N->d_wb, (size_t)2 * nw);
  if (e == hipSuccess) e = dmalloc(&N->d_bias, (size_t)2 * (2 * kMlpH + kNAct));
  if (e == hipSuccess) e = dmalloc(&N->d_grad, (size_t)kMlpParams);
  if (e != hipSuccess) {
    N->release();
    delete N;
    return fail(MPCG_ERR_NOMEM, "MLP allocation failed");
  }
  mlp_views(N);
  *out = N;
  const int rc = mpcg_mlp_set_params(N, params);
  if (rc) {
    N->release();
    delete N;
    *out = nullptr;
  }
  return rc;
}

int mpcg_mlp_destroy(mpcg_mlp *N) {
  if (!N) return MPCG_OK;
  (void)hipStreamSynchronize(N->stream);
  N->release();
  delete N;
  return MPCG_OK;
}

int mpcg_mlp_set_params(mpcg_mlp *N, const float *params) {
  if (!N || !params) return fail(MPCG_ERR_INVALID, "NULL argument");
  for (int p = 0; p < kMlpParams; ++p)
    if (!std::isfinite(params[p])) return fail(MPCG_ERR_INVALID, "non-finite parameter");
  HIP_TRY(hipMemcpyAsync(N->d_master, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice, N->stream));
  HIP_TRY(hipMemsetAsync(N->d_m, 0, sizeof(float) * kMlpParams, N->stream));
  HIP_TRY(hipMemsetAsync(N->d_v, 0, sizeof(float) * kMlpParams, N->stream));
  launch_mlp_copies(N->cur, N->d_master, N->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(N->stream));
  N->steps = 0;
  return MPCG_OK;
}

int mpcg_mlp_get_params(mpcg_mlp *N, float *params) {
  if (!N || !params) return fail(MPCG_ERR_INVALID, "NULL argument");
  HIP_TRY(hipStreamSynchronize(N->stream));
  HIP_TRY(hipMemcpy(params, N->d_master, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
  return MPCG_OK;
}

int mpcg_mlp_forward(mpcg_mlp *N, const float *feat, int32_t n, float *logits) {
  if (!N || n < 0 || (n > 0 && (!feat || !logits))) return fail(MPCG_ERR_INVALID, "bad argument");
  launch_mlp_forward(N->cur, feat, n, logits, nullptr, nullptr, 0.0f, nullptr, nullptr, N->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(N->stream));
  return MPCG_OK;
}

int mpcg_mlp_grad(mpcg_mlp *N, const float *feat, const int32_t *act, const float *target, int32_t B, float *grad,
                  float *loss) {
  if (!N || !feat || !act || !target || !grad || B <= 0 || B % 64) return fail(MPCG_ERR_INVALID, "bad argument");
  int rc = mlp_ensure_part(N, B / 64);
  if (rc) return rc;
  if (!N->d_loss) {
    HIP_TRY(dmalloc(&N->d_loss, 1));
    N->loss_cap = 1;
  }
  launch_mlp_grad(N->cur, feat, act, target, 0, B, N->d_part, N->d_ploss, N->stream);
  launch_mlp_update(MlpState{N->d_master, N->d_m, N->d_v, N->cur}, N->d_part, N->d_ploss, B / 64, 0, 0, 0.f, 0.f, 0.f,
                    0.f, N->d_grad, N->d_loss, N->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(grad, N->d_grad, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, N->stream));
  float l = 0.0f;
  HIP_TRY(hipMemcpyAsync(&l, N->d_loss, sizeof(float), hipMemcpyDeviceToHost, N->stream));
  HIP_TRY(hipStreamSynchronize(N->stream));
  if (loss) *loss = l;
  return MPCG_OK;
}

int mpcg_mlp_train(mpcg_mlp *N, const float *feat, const float *next, const int32_t *act, const float *rew,
                   const uint8_t *done, int32_t n, const mpcg_mlp_train_desc *d, float *epoch_loss) {
  if (!N || !d || n < 0 || (n > 0 && (!feat || !next || !act || !rew || !done)))
    return fail(MPCG_ERR_INVALID, "bad argument");
  if (d->batch <= 0 || d->batch % 64 || d->epochs < 0 || !(d->lr > 0.0) || !(d->beta1 >= 0.0 && d->beta1 < 1.0) ||
      !(d->beta2 >= 0.0 && d->beta2 < 1.0) || !(d->eps > 0.0) || !(d->gamma >= 0.0 && d->gamma <= 1.0))
    return fail(MPCG_ERR_INVALID, "bad training descriptor");
  const int nb = n / d->batch;   // whole batches, in order
  int rc = mlp_ensure_part(N, d->batch / 64);
  if (rc) return rc;
  if (N->tcap < n) {
    dfree(N->d_target);
    dfree(N->d_ymax);
    HIP_TRY(dmalloc(&N->d_target, (size_t)std::max(n, 1)));
    HIP_TRY(dmalloc(&N->d_ymax, (size_t)std::max(n, 1)));
    N->tcap = n;
  }
  const int64_t nsteps = (int64_t)nb * d->epochs;
  if (N->loss_cap < nsteps) {
    dfree(N->d_loss);
    HIP_TRY(dmalloc(&N->d_loss, (size_t)std::max<int64_t>(nsteps, 1)));
    N->loss_cap = std::max<int64_t>(nsteps, 1);
  }
  const MlpState st{N->d_master, N->d_m, N->d_v, N->cur};
  int64_t k = 0;
  for (int ep = 0; ep < d->epochs; ++ep) {
    launch_mlp_copies(N->frozen, N->d_master, N->stream);   // weights frozen for this epoch's targets
    launch_mlp_forward(N->frozen, next, n, nullptr, rew, done, (float)d->gamma, N->d_target, N->d_ymax, N->stream);
    for (int j = 0; j < nb; ++j, ++k) {
      launch_mlp_grad(N->cur, feat, act, N->d_target, j * d->batch, d->batch, N->d_part, N->d_ploss, N->stream);
      N->steps++;
      launch_mlp_update(st, N->d_part, N->d_ploss, d->batch / 64, 1, (int)N->steps, (float)d->lr, (float)d->beta1,
                        (float)d->beta2, (float)d->eps, nullptr, N->d_loss + k, N->stream);
    }
    HIP_TRY(hipGetLastError());
  }
  std::vector<float> losses((size_t)std::max<int64_t>(nsteps, 1));
  if (nsteps > 0)
    HIP_TRY(hipMemcpyAsync(losses.data(), N->d_loss, sizeof(float) * nsteps, hipMemcpyDeviceToHost, N->stream));
  HIP_TRY(hipStreamSynchronize(N->stream));
  if (epoch_loss)
    for (int ep = 0; ep < d->epochs; ++ep) {
      double s = 0.0;
      for (int j = 0; j < nb; ++j) s += losses[(size_t)ep * nb + j];
      epoch_loss[ep] = nb ? (float)(s / nb) : 0.0f;
    }
  return MPCG_OK;
}

// Round-to-nearest-even to bfloat16 of an fp32 value (inf/nan kept).
static float host_bf16(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) != 0x7f800000u) {
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
  }
  float y;
  std::memcpy(&y, &u, 4);
  return y;
}

int mpcg_policy_set_mlp_from(mpcg_policy *P, mpcg_mlp *N) {
  if (!P || !N) return fail(MPCG_ERR_INVALID, "NULL argument");
  std::vector<float> p(kMlpParams);
  int rc = mpcg_mlp_get_params(N, p.data());
  if (rc) return rc;
  const int o1 = kMlpH * kMlpIn, o2 = o1 + kMlpH, o3 = o2 + kMlpH * kMlpH, o4 = o3 + kMlpH, o5 = o4 + kNAct * kMlpH;
  for (int i = 0; i < kMlpParams; ++i)
    if (i < o1 || (i >= o2 && i < o3) || (i >= o4 && i < o5)) p[i] = host_bf16(p[i]);
  const float *w = p.data();
  return mpcg_policy_set_mlp(P, w, w + o1, w + o2, w + o3, w + o4, w + o5);
}

int mpcg_get_profile(mpcg_matrix *A, mpcg_profile *out) {
  if (!A || !out) return fail(MPCG_ERR_INVALID, "NULL argument");
  *out = A->prof;
  return MPCG_OK;
}

int mpcg_get_history(mpcg_matrix *A, double *rho, uint8_t *act, uint8_t *flags, int32_t cap, int32_t *rep_k,
                     double *rep_rho, int32_t rep_cap, int32_t *n_hist) {
  if (!A) return fail(MPCG_ERR_INVALID, "A is NULL");
  if (A->last_iters < 0) return fail(MPCG_ERR_INVALID, "no solve yet");
  HIP_TRY(hipStreamSynchronize(A->stream));
  const int k = A->last_iters;
  if (rho) HIP_TRY(hipMemcpy(rho, A->d_hrho, sizeof(double) * std::min(k + 1, cap), hipMemcpyDeviceToHost));
  if (act && k > 0) HIP_TRY(hipMemcpy(act, A->d_hact, std::min(k, cap), hipMemcpyDeviceToHost));
  if (flags && k > 0) HIP_TRY(hipMemcpy(flags, A->d_hflag, std::min(k, cap), hipMemcpyDeviceToHost));
  const int nr = std::min(std::min(A->last_nrep, A->cap_rep), rep_cap);
  if (rep_k && nr > 0) HIP_TRY(hipMemcpy(rep_k, A->d_repk, sizeof(int32_t) * nr, hipMemcpyDeviceToHost));
  if (rep_rho && nr > 0) HIP_TRY(hipMemcpy(rep_rho, A->d_reprho, sizeof(double) * nr, hipMemcpyDeviceToHost));
  if (n_hist) *n_hist = k + 1;
  return MPCG_OK;
}

// ---------------------------------------------------------------- single ops
int mpcg_op_spmv(mpcg_matrix *A, int fmt, int tier64, const void *p, void *q) {
  if (!A || !p || !q || fmt < 0 || fmt > 5 || (tier64 != 0 && tier64 != 1))
    return fail(MPCG_ERR_INVALID, "bad argument");
  launch_op_spmv(A->mat(), fmt, tier64, p, q, A->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(A->stream));
  return MPCG_OK;
}

int mpcg_op_residual(mpcg_matrix *A, const double *b, const double *x, double *r) {
  if (!A || !b || !x || !r) return fail(MPCG_ERR_INVALID, "bad argument");
  launch_op_residual(A->mat(), b, x, r, A->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(A->stream));
  return MPCG_OK;
}

int mpcg_op_dot(mpcg_matrix *A, int fmt, int tier64, const void *u, const void *v, double *out) {
  if (!A || !u || !v || !out || fmt < 0 || fmt > 5 || fmt == MPCG_Q52 || (tier64 != 0 && tier64 != 1))
    return fail(MPCG_ERR_INVALID, "bad argument");
  launch_op_dot(A->n, fmt, tier64, u, v, A->d_part2, A->P2, A->d_scalar, A->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(out, A->d_scalar, sizeof(double), hipMemcpyDeviceToHost, A->stream));
  HIP_TRY(hipStreamSynchronize(A->stream));
  return MPCG_OK;
}

int mpcg_op_dot_noalloc(mpcg_matrix *A, int fmt, int tier64, const void *u, const void *v, double *out) {
  if (!A || !u || !v || !out || fmt < 0 || fmt > 5 || fmt == MPCG_Q52 || (tier64 != 0 && tier64 != 1))
    return fail(MPCG_ERR_INVALID, "bad argument");
  if ((int64_t)(A->n + kVecBlock - 1) / kVecBlock > kNoAllocPartials)
    return fail(MPCG_ERR_INVALID, "n exceeds the allocation-free dot's limit of " +
                                      std::to_string((int64_t)kNoAllocPartials * kVecBlock) + " elements");
  HIP_TRY(launch_op_dot_noalloc(A->n, fmt, tier64, u, v, out, A->stream));
  return MPCG_OK;
}

int mpcg_gather_floor(mpcg_matrix *A, const float *p, int32_t repeats, double *us_per_launch) {
  if (!A || !p || !us_per_launch || repeats < 1) return fail(MPCG_ERR_INVALID, "bad argument");
  int rc = ensure_ws(A);
  if (rc) return rc;
  const Mat m = A->mat();
  float *sink = A->d_q32;   // written only for a NaN sum
  launch_gather_floor(m, p, sink, A->stream);
  launch_gather_floor(m, p, sink, A->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(A->ev_start, A->stream));
  for (int i = 0; i < repeats; ++i) launch_gather_floor(m, p, sink, A->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(A->ev_end, A->stream));
  HIP_TRY(hipEventSynchronize(A->ev_end));
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, A->ev_start, A->ev_end));
  *us_per_launch = (double)ms * 1e3 / repeats;
  return MPCG_OK;
}

int mpcg_op_axpy(mpcg_matrix *A, int fmt, double alpha, const void *u, void *y) {
  if (!A || !u || !y || fmt < 0 || fmt > 5 || fmt == MPCG_Q52) return fail(MPCG_ERR_INVALID, "bad argument");
  launch_op_axpy(A->n, fmt, alpha, u, y, A->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(A->stream));
  return MPCG_OK;
}

}  // extern "C"
