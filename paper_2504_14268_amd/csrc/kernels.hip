// kernels.hip -- gfx950 kernels of the mixed-precision CG iteration.
//
// One CG iteration is one "slot" of four launches on one stream:
//   K1  SpMV q = A_fs p in the LDS-staged CSR form, fused partial of nu = p.q
//       (or, in the other modes: the fp64 residual b - A x_hi of a start,
//       restart, replacement or final check, fused with its squared norm);
//   K2  every block reduces K1's partials to nu and alpha = sigma/nu itself,
//       then x_lo += alpha p, r -= alpha q and the partial of sigma' = r.r;
//   KS  one block: the final reductions and the scalar step -- alpha, beta, rho,
//       convergence and replacement tests, the policy's state, reward, Q update
//       and next action; the only writer of the control block;
//   K3  p = r + beta p (or fold x_lo into x_hi, or p = r after a start), with
//       the conversion of r and p when the next action changes the tier.
// No kernel communicates between its own workgroups: kernel boundaries order
// every hand-off, so no workgroup pays a device-wide cache write-back.  The host
// only enqueues slots.
#include "kernels.hpp"
#include "launch.hpp"

namespace mpcg {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float fma_acc(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_acc(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename A, typename V>
__device__ __forceinline__ A to_acc(V v) { return (A)v; }   // float<-double: RNE; double<-float: exact

// y = rd_fa(fma_acc(rd_acc(alpha), u, y)) in the tier of fa
template <int FA>
__device__ __forceinline__ typename TierT<FA == FP64>::type axpy1(double alpha,
                                                                 typename TierT<FA == FP64>::type u,
                                                                 typename TierT<FA == FP64>::type y) {
  if constexpr (FA == FP64) return __builtin_fma(alpha, u, y);
  else return rd_from_f32<FA>(__builtin_fmaf((float)alpha, u, y));
}

template <typename V>
__device__ __forceinline__ void load8(const V *__restrict__ p, V (&v)[8]) {
  if constexpr (sizeof(V) == 4) {
    const float4 a = *(const float4 *)p, b = *(const float4 *)(p + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double2 d = *(const double2 *)(p + 2 * j);
      v[2 * j] = d.x; v[2 * j + 1] = d.y;
    }
  }
}

template <typename V>
__device__ __forceinline__ void store8(V *__restrict__ p, const V (&v)[8]) {
  if constexpr (sizeof(V) == 4) {
    *(float4 *)p = make_float4(v[0], v[1], v[2], v[3]);
    *(float4 *)(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) *(double2 *)(p + 2 * j) = make_double2(v[2 * j], v[2 * j + 1]);
  }
}

// 8 matrix values at aligned position c, widened to the accumulation type.
template <int FS>
__device__ __forceinline__ void load_vals8(const Mat &A, int c, typename AccT<FS>::type (&v)[8]) {
  if constexpr (FS == FP64) {
    load8(A.v64 + c, v);
  } else if constexpr (FS == FP32) {
    load8(A.v32 + c, v);
  } else {
    const uint4 w = *(const uint4 *)((FS == BF16 ? A.vbf : A.vh) + c);
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint16_t lo = (uint16_t)(ws[j] & 0xffffu), hi = (uint16_t)(ws[j] >> 16);
      if constexpr (FS == BF16) {
        v[2 * j] = bf16_bits_to_f32(lo); v[2 * j + 1] = bf16_bits_to_f32(hi);
      } else {
        v[2 * j] = f16_bits_to_f32(lo); v[2 * j + 1] = f16_bits_to_f32(hi);
      }
    }
  }
}

// LDS capacity (entries) of one staging window per 256 rows: 8 KiB of values
// (accumulation type) and their column indices.
template <typename Acc> struct Cap { static constexpr int value = 8192 / sizeof(Acc); };
constexpr int kRPT = 2;                                  // rows per thread in K1
constexpr int kLdsDoubles = kRPT * 2 * 8192 / 8;

template <typename A>
__device__ __forceinline__ void lds_store8(A *p, const A (&v)[8]) {
  if constexpr (sizeof(A) == 4) {
    *(float4 *)p = make_float4(v[0], v[1], v[2], v[3]);
    *(float4 *)(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) *(double2 *)(p + 2 * j) = make_double2(v[2 * j], v[2 * j + 1]);
  }
}

// Row accumulators of RPT*kRowsPerBlock consecutive rows starting at r0: thread
// t owns rows r0 + t + j*kRowsPerBlock (j < RPT) and runs each row's fma chain
// in CSR order.  The rows' values and column indices are staged through LDS in
// windows that start at 8-aligned positions (aligned 8-entry groups, vector
// loads and vector LDS stores).  x is gathered in the row loop: lane t reads
// the k-th column of its own row, so on banded and stencil matrices a
// wavefront's gathers fall on neighbouring addresses.  Gathers are issued eight
// at a time ahead of their fma chain.
template <int FS, int RPT, typename V>
__device__ __forceinline__ void spmv_rows(const Mat &A, const V *__restrict__ x, int r0, int nrows,
                                          void *lds_raw, typename AccT<FS>::type (&acc)[RPT]) {
  using Acc = typename AccT<FS>::type;
  constexpr int CAP = Cap<Acc>::value * RPT;
  Acc *lv = (Acc *)lds_raw;
  int *lc = (int *)(lv + CAP);
  const int tid = threadIdx.x;
  const int ks = A.rp[r0], ke = A.rp[r0 + nrows];
  int my_s[RPT], my_e[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int lr = tid + j * kRowsPerBlock;
    my_s[j] = 0;
    my_e[j] = 0;
    if (lr < nrows) {
      my_s[j] = A.rp[r0 + lr];
      my_e[j] = A.rp[r0 + lr + 1];
    }
    acc[j] = (Acc)0;
  }
  for (int wb = ks & ~7; wb < ke; wb += CAP) {
    const int we = min(wb + CAP, ke);
    for (int c = wb + tid * 8; c < we; c += kBlock * 8) {
      Acc v[8];
      load_vals8<FS>(A, c, v);
      lds_store8(lv + (c - wb), v);
      *(int4 *)(lc + (c - wb)) = *(const int4 *)(A.ci + c);
      *(int4 *)(lc + (c - wb) + 4) = *(const int4 *)(A.ci + c + 4);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int lo = max(my_s[j], wb), hi = min(my_e[j], we);
      for (int kk = lo; kk < hi; kk += 8) {
        const int cnt = hi - kk;
        Acc xv[8], vv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (u < cnt) {
            vv[u] = lv[kk - wb + u];
            xv[u] = to_acc<Acc>(x[lc[kk - wb + u]]);
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (u < cnt) acc[j] = fma_acc(vv[u], xv[u], acc[j]);
      }
    }
    __syncthreads();
  }
}

// Sums of RPT 256-row subtrees at once (one LDS round): each thread holds one
// leaf per subtree.
template <int RPT, typename A>
__device__ __forceinline__ void block_tree_multi(const A (&leaf)[RPT], double (&out)[RPT]) {
  __shared__ A ws[RPT][kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const A v = wave_tree(leaf[j]);
    if (lane == 0) ws[j][wave] = v;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < RPT; ++j) out[j] = (double)((ws[j][0] + ws[j][1]) + (ws[j][2] + ws[j][3]));
  __syncthreads();
}

// q_i = rd_tier(2^{e_i} acc) (e_i = 0 unless fp16)
template <int FS, typename V>
__device__ __forceinline__ V spmv_out(const Mat &A, int i, typename AccT<FS>::type acc) {
  if constexpr (FS == FP16) {
    const double s = ldexp((double)acc, (int)A.rexp[i]);
    return (V)s;
  } else {
    return (V)acc;
  }
}

template <int FD, typename V>
__device__ __forceinline__ double dot_leaf_block(V u, V v, bool valid) {
  using A = typename AccT<FD>::type;
  A l = valid ? dot_leaf<FD>(u, v) : (A)0;
  return (double)block_tree(l);
}

template <int FD, int RPT, typename V>
__device__ __forceinline__ void dot_leaf_multi(const V (&u)[RPT], const V (&v)[RPT], const bool (&valid)[RPT],
                                               double (&out)[RPT]) {
  using A = typename AccT<FD>::type;
  A l[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) l[j] = valid[j] ? dot_leaf<FD>(u[j], v[j]) : (A)0;
  block_tree_multi<RPT>(l, out);
}

template <int RPT, typename V>
__device__ __forceinline__ void dot_leaf_multi_rt(int fd, const V (&u)[RPT], const V (&v)[RPT],
                                                  const bool (&valid)[RPT], double (&out)[RPT]) {
  switch (fd) {
  case FP16: dot_leaf_multi<FP16, RPT>(u, v, valid, out); break;
  case BF16: dot_leaf_multi<BF16, RPT>(u, v, valid, out); break;
  case FP32: dot_leaf_multi<FP32, RPT>(u, v, valid, out); break;
  default: dot_leaf_multi<FP64, RPT>(u, v, valid, out); break;
  }
}

template <typename V>
__device__ __forceinline__ double dot_leaf_block_rt(int fd, V u, V v, bool valid) {
  switch (fd) {
  case FP16: return dot_leaf_block<FP16>(u, v, valid);
  case BF16: return dot_leaf_block<BF16>(u, v, valid);
  case FP32: return dot_leaf_block<FP32>(u, v, valid);
  default: return dot_leaf_block<FP64>(u, v, valid);
  }
}

// Pairwise total of P partials, identical in every thread of the block; per
// wavefront without a barrier when P is small enough (block-uniform choice).
template <typename A>
__device__ __forceinline__ double partials_total(const double *part, int P) {
  if (P <= kWaveReduceMax) return (double)wave_reduce_partials<A>(part, P);
  return (double)reduce_partials<A>(part, P);
}

__device__ __forceinline__ double reduce_partials_rt(int fd, const double *part, int P) {
  return fd == FP64 ? partials_total<double>(part, P) : partials_total<float>(part, P);
}

// Sum of eight consecutive sibling subtrees in the accumulation format of fd.
__device__ __forceinline__ double tree8_rt(int fd, const double (&s)[8]) {
  if (fd == FP64) return tree8(s);
  float f[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) f[j] = (float)s[j];
  return (double)tree8(f);
}

// XCD-aware order: consecutive workgroups land on different XCDs, so XCD x gets
// the contiguous range of groups [x*per, (x+1)*per) (its gathers share its L2).
__device__ __forceinline__ int xcd_group(int G) {
  const int per = G >> 3;
  const int b = blockIdx.x;
  return (b & 7) * per + (b >> 3);
}

// ---------------------------------------------------------------------------
// policy (section 4.1): state, decision, reward, Q update, features, MLP
// ---------------------------------------------------------------------------
__device__ int policy_state(const PolicyDev *P, int k, double rho, int stag) {
  const int width = (P->t_bin + P->b_it - 1) / P->b_it;
  int i = k / width;
  if (i > P->b_it - 1) i = P->b_it - 1;
  int j = 0;
  for (int t = 0; t < P->b_res - 1; ++t)
    if (rho <= P->edges[t]) j++;
  return (j * P->b_it + i) * 2 + (stag ? 1 : 0);
}

__device__ int q_argmax(const double *row) {
  int best = 0;
  double bv = row[0];
  for (int a = 1; a < kNAct; ++a)
    if (row[a] > bv) { best = a; bv = row[a]; }
  return best;
}

__device__ double policy_cost(const PolicyDev *P, int a) {
  return (P->cost[(a >> 4) & 3] + P->cost[(a >> 2) & 3]) + P->cost[a & 3];
}

__device__ double policy_reward(const PolicyDev *P, int a, double rho, bool conv) {
  const double accterm = (rho <= P->eps_min) ? -log10_policy(P->eps_min) : -log10_policy(rho);
  double r = P->w1 * accterm - P->w2 * policy_cost(P, a);
  if (conv) r = r + P->w3;
  return r;
}

__device__ void q_update(const PolicyDev *P, int s, int a, double target) {
  double *q = &P->q[s * kNAct + a];
  *q = *q + P->lr * (target - *q);
}

__device__ double lg_clamped(const PolicyDev *P, double r) {
  return (r <= P->eps_min) ? log10_policy(P->eps_min) : log10_policy(r);
}

__device__ void mlp_features(const PolicyDev *P, int k, const double *hr, int stag, double last_true,
                             int prev, float *f) {
  double lg[8];
  for (int i = 0; i < 8; ++i) {
    int idx = k - i;
    if (idx < 0) idx = 0;
    lg[i] = lg_clamped(P, hr[idx]);
  }
  for (int i = 0; i < 8; ++i) f[i] = (float)lg[i];
  f[8] = (float)(lg[0] - lg[1]);
  f[9] = (float)((double)k / (double)P->t_bin);
  f[10] = stag ? 1.0f : 0.0f;
  f[11] = (float)lg_clamped(P, last_true);
  const int R = P->replace_period > 0 ? P->replace_period : 1;
  f[12] = (float)((double)(k % R) / (double)R);
  f[13] = (float)((double)((prev >> 4) & 3) / 3.0);
  f[14] = (float)((double)((prev >> 2) & 3) / 3.0);
  f[15] = (float)((double)(prev & 3) / 3.0);
}

__device__ void roll_log(const PolicyDev *P, const float *f, const float *fn, int a, double rw, int done) {
  if (P->roll_cap <= 0) return;
  const int i = *P->roll_n;
  if (i >= P->roll_cap) return;
  *P->roll_n = i + 1;
  for (int j = 0; j < kMlpIn; ++j) {
    P->roll_feat[(size_t)i * kMlpIn + j] = f[j];
    P->roll_next[(size_t)i * kMlpIn + j] = fn[j];
  }
  P->roll_act[i] = a;
  P->roll_rew[i] = (float)rw;
  P->roll_done[i] = (uint8_t)done;
}

__device__ int decide_scalar(const PolicyDev *P, int s, int k, int *explored) {
  *explored = 0;
  switch (P->kind) {
  case POL_FIXED: return P->fixed_action;
  case POL_QTABLE: return q_argmax(&P->q[s * kNAct]);
  case POL_QTRAIN: {
    const double u0 = counter_uniform(P->seed, (uint64_t)P->episode, (uint64_t)k, 0);
    if (u0 < P->epsilon) {
      const double u1 = counter_uniform(P->seed, (uint64_t)P->episode, (uint64_t)k, 1);
      *explored = 1;
      return (int)(u1 * 64.0);
    }
    return q_argmax(&P->q[s * kNAct]);
  }
  }
  return 63;
}

// MLP logits by one block: x = bf16(feat); h1 = bf16(gelu(W1 x + b1));
// h2 = bf16(gelu(W2 h1 + b2)); y = W3 h2 + b3.  Each output is one thread's fp32
// fma chain over its inputs in ascending order.
__device__ void mlp_logits_block(const PolicyDev *P, const float *feat, float *logits) {
  __shared__ float x[kMlpIn], h1[kMlpH], h2[kMlpH];
  const int t = threadIdx.x;
  if (t < kMlpIn) x[t] = rd_bf16_from_f32(feat[t]);
  __syncthreads();
  if (t < kMlpH) {
    float acc = 0.0f;
    for (int i = 0; i < kMlpIn; ++i) acc = __builtin_fmaf(P->W1[t * kMlpIn + i], x[i], acc);
    h1[t] = rd_bf16_from_f32(gelu_as(acc + P->b1[t]));
  }
  __syncthreads();
  if (t < kMlpH) {
    float acc = 0.0f;
    for (int i = 0; i < kMlpH; ++i) acc = __builtin_fmaf(P->W2[t * kMlpH + i], h1[i], acc);
    h2[t] = rd_bf16_from_f32(gelu_as(acc + P->b2[t]));
  }
  __syncthreads();
  if (t < kNAct) {
    float acc = 0.0f;
    for (int i = 0; i < kMlpH; ++i) acc = __builtin_fmaf(P->W3[t * kMlpH + i], h2[i], acc);
    logits[t] = acc + P->b3[t];
  }
  __syncthreads();
}

__device__ int argmax64f(const float *v) {
  int best = 0;
  for (int a = 1; a < kNAct; ++a)
    if (v[a] > v[best]) best = a;
  return best;
}

// ---------------------------------------------------------------------------
// scalar step (KS): the control block and the policy description live in LDS
// for the duration of the step.
// ---------------------------------------------------------------------------
struct Sx {
  Ctl *ctl;
  const PolicyDev *pol;
  Hist h;
};
__device__ void set_done(Ctl *c) {
  c->mode = M_DONE;
  c->k2op = K2_NONE;
  c->k3op = K3_NONE;
}

// Install the next action.  After a start/restart r is in the fp64 container
// and K3 copies it into the new tier; otherwise K3 applies p = r + beta p in the
// old tier and converts r, p if the tier changes.
__device__ void apply_decision(const Sx &a, int na, int ex, bool from_init) {
  Ctl *c = a.ctl;
  const int k = c->k;
  if (from_init && k >= c->maxit) {
    c->status = 1;
    set_done(c);
    return;
  }
  const int nt = ((na & 3) == FP64) ? 1 : 0;
  if (from_init) {
    c->k3op = K3_COPY;
    c->k3switch = 0;
    c->tier_old = 1;
  } else {
    c->k3op = K3_XPAY;
    c->k3switch = (nt != c->tier);
    c->tier_old = c->tier;
    if (c->k3switch) a.h.flag[k - 1] |= FL_SWITCH;
  }
  c->tier = nt;
  c->action = na;
  c->explored = ex;
  c->k2op = K2_NONE;
  a.h.act[k] = (uint8_t)na;
  a.h.flag[k] = ex ? FL_EXPLORED : 0;
  c->cost_sum += policy_cost(a.pol, na);
  c->mode = M_ITER;
}

// Start / restart: rho_0 from the fp64 residual, first action.  Returns 1 when
// the decision needs the block's MLP forward (features left in s_feat).
__device__ int init_t0(const Sx &a, double s64, float *s_feat) {
  Ctl *c = a.ctl;
  const PolicyDev *P = a.pol;
  const int k = c->k;
  const double rt = sqrt(s64) / c->bnorm;
  a.h.rho[k] = rt;
  c->last_true = rt;
  c->nrep_since = 0;
  if (rt <= c->tol) {
    c->status = c->fell_back ? 2 : 0;
    c->relres_true = rt;
    set_done(c);
    return 0;
  }
  if (!isfinite(rt)) {
    c->status = 3;
    c->relres_true = rt;
    set_done(c);
    return 0;
  }
  c->sigma = s64;
  const int stag = (k >= P->w_stag) && (rt >= a.h.rho[k - P->w_stag]);
  const int s = policy_state(P, k, rt, stag);
  c->s = s;
  if (P->kind == POL_MLP || P->roll_cap > 0) mlp_features(P, k, a.h.rho, stag, rt, c->prev_action, c->feat);
  if (c->fell_back) {
    apply_decision(a, 63, 0, true);
    return 0;
  }
  if (P->kind == POL_MLP) {
    for (int i = 0; i < kMlpIn; ++i) s_feat[i] = c->feat[i];
    return 1;
  }
  int ex = 0;
  const int na = decide_scalar(P, s, k, &ex);
  apply_decision(a, na, ex, true);
  return 0;
}

// End of an iteration (or of a failed one): history, beta, training update,
// rollout, convergence / breakdown / fallback / budget, next action.
__device__ int finish_t0(const Sx &a, bool completed, bool broke, bool converged, bool stagnated,
                         float *s_feat) {
  Ctl *c = a.ctl;
  const PolicyDev *P = a.pol;
  const int k = c->k;
  const bool active = !c->fell_back;
  const bool training = active && P->kind == POL_QTRAIN;
  const bool want_feat = active && (P->kind == POL_MLP || P->roll_cap > 0);
  const int act = c->action, s = c->s;
  const double rho = c->rho_new;
  if (completed) a.h.rho[k] = rho;
  double beta = 0.0;
  if (completed && !broke && !converged) {
    beta = c->sig_new / c->sigma;
    if (!isfinite(beta)) broke = true;
  }
  int stag = 0, s_next = s;
  if (!broke) {
    stag = (k >= P->w_stag) && (rho >= a.h.rho[k - P->w_stag]);
    s_next = policy_state(P, k, rho, stag);
    if (want_feat) mlp_features(P, k, a.h.rho, stag, c->last_true, act, c->feat_next);
  } else if (want_feat) {
    for (int i = 0; i < kMlpIn; ++i) c->feat_next[i] = c->feat[i];
  }
  if (converged) {
    const double rw = policy_reward(P, act, rho, true);
    if (training) q_update(P, s, act, rw);
    if (active) roll_log(P, c->feat, c->feat_next, act, rw, 1);
    c->status = c->fell_back ? 2 : 0;
    c->relres_true = rho;
    set_done(c);
    return 0;
  }
  if (broke || (stagnated && c->fallback_enabled && !c->fell_back)) {
    const double rw = -P->w2 * policy_cost(P, act) - P->w3;
    if (training) q_update(P, s, act, rw);
    if (active) roll_log(P, c->feat, c->feat_next, act, rw, 1);
    if (!c->fallback_enabled || c->fell_back) {
      c->status = 3;
      set_done(c);
      return 0;
    }
    c->fell_back = 1;
    c->fallback_at = k;
    a.h.flag[completed ? k - 1 : k] |= FL_FALLBACK;
    c->prev_action = act;
    c->mode = M_INIT;
    c->k2op = K2_NONE;
    c->k3op = K3_FOLD;
    return 0;
  }
  {
    const double rw = policy_reward(P, act, rho, false);
    if (training) {
      const double *row = &P->q[s_next * kNAct];
      q_update(P, s, act, rw + P->gamma * row[q_argmax(row)]);
    }
    if (active) roll_log(P, c->feat, c->feat_next, act, rw, 0);
  }
  if (k >= c->maxit) {
    c->status = 1;
    set_done(c);
    return 0;
  }
  c->beta = beta;
  c->sigma = c->sig_new;
  c->prev_action = act;
  c->s = s_next;
  c->k3_fa = act & 3;
  if (want_feat)
    for (int i = 0; i < kMlpIn; ++i) c->feat[i] = c->feat_next[i];
  if (c->fell_back) {
    apply_decision(a, 63, 0, false);
    return 0;
  }
  if (P->kind == POL_MLP) {
    for (int i = 0; i < kMlpIn; ++i) s_feat[i] = c->feat[i];
    return 1;
  }
  int ex = 0;
  const int na = decide_scalar(P, s_next, k, &ex);
  apply_decision(a, na, ex, false);
  return 0;
}

// Block-level wrappers: thread 0 runs the scalar step; the block joins for an
// MLP decision.
__device__ void finish_block(const Sx &a, bool completed, bool broke, bool converged, bool stagnated) {
  __shared__ int s_need;
  __shared__ float s_feat[kMlpIn], s_logits[kNAct];
  if (threadIdx.x == 0) s_need = finish_t0(a, completed, broke, converged, stagnated, s_feat);
  __syncthreads();
  if (s_need) {
    mlp_logits_block(a.pol, s_feat, s_logits);
    if (threadIdx.x == 0) apply_decision(a, argmax64f(s_logits), 0, false);
  }
}

__device__ void init_block(const Sx &a, double s64) {
  __shared__ int s_need;
  __shared__ float s_feat[kMlpIn], s_logits[kNAct];
  if (threadIdx.x == 0) s_need = init_t0(a, s64, s_feat);
  __syncthreads();
  if (s_need) {
    mlp_logits_block(a.pol, s_feat, s_logits);
    if (threadIdx.x == 0) apply_decision(a, argmax64f(s_logits), 0, true);
  }
}

__device__ void replace_block(const Sx &a, double s64) {
  __shared__ int s_f[3];
  if (threadIdx.x == 0) {
    Ctl *c = a.ctl;
    const int k = c->k;
    const double rt = sqrt(s64) / c->bnorm;
    if (c->nrep < a.h.cap_rep) {
      a.h.rep_k[c->nrep] = k;
      a.h.rep_rho[c->nrep] = rt;
    }
    c->nrep++;
    a.h.flag[k - 1] |= FL_REPLACED;
    c->last_true = rt;
    c->rho_new = rt;
    int conv = 0, broke = 0, stag = 0;
    if (rt <= c->tol) {
      conv = 1;
    } else if (!isfinite(rt)) {
      broke = 1;
    } else {
      c->sig_new = s64;
      c->rep_hist[0] = c->rep_hist[1];
      c->rep_hist[1] = c->rep_hist[2];
      c->rep_hist[2] = rt;
      c->nrep_since++;
      if (c->nrep_since >= 3 && rt >= c->rep_hist[0]) stag = 1;
    }
    s_f[0] = conv; s_f[1] = broke; s_f[2] = stag;
  }
  __syncthreads();
  finish_block(a, true, s_f[1] != 0, s_f[0] != 0, s_f[2] != 0);
}

// ---------------------------------------------------------------------------
// K1: SpMV (or fp64 residual) over a group of kGroupRows rows; one partial per
// group = the pairwise sum of its eight 256-row subtrees.
// ---------------------------------------------------------------------------
constexpr int kGroupBlocks = kVecBlock / kRowsPerBlock;   // 8 row blocks = 2048 rows

template <int FS, int TIER>
__device__ __forceinline__ void k1_iter(const KArgs &a, int g, void *lds) {
  using V = typename TierT<TIER>::type;
  const V *p;
  V *q;
  if constexpr (TIER) { p = a.v.p64; q = a.v.q64; } else { p = a.v.p32; q = a.v.q32; }
  const int fd = (a.ctl->action >> 2) & 3;
  const int n = a.A.n;
  double sub[8];
#pragma unroll 1
  for (int sb = 0; sb < kGroupBlocks / kRPT; ++sb) {
    const int r0 = (g * kGroupBlocks + sb * kRPT) * kRowsPerBlock;
    if (r0 >= n) {            // zero-padded subtrees
#pragma unroll
      for (int j = 0; j < kRPT; ++j) sub[sb * kRPT + j] = 0.0;
      continue;
    }
    const int nrows = min(kRPT * kRowsPerBlock, n - r0);
    typename AccT<FS>::type acc[kRPT];
    spmv_rows<FS, kRPT>(a.A, p, r0, nrows, lds, acc);
    V qi[kRPT], pi[kRPT];
    bool valid[kRPT];
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int lr = threadIdx.x + j * kRowsPerBlock;
      valid[j] = lr < nrows;
      qi[j] = (V)0;
      pi[j] = (V)0;
      if (valid[j]) {
        qi[j] = spmv_out<FS, V>(a.A, r0 + lr, acc[j]);
        q[r0 + lr] = qi[j];
        pi[j] = p[r0 + lr];
      }
    }
    double s2[kRPT];
    dot_leaf_multi_rt<kRPT>(fd, pi, qi, valid, s2);
#pragma unroll
    for (int j = 0; j < kRPT; ++j) sub[sb * kRPT + j] = s2[j];
  }
  if (threadIdx.x == 0) a.part1[g] = tree8_rt(fd, sub);
}

// fp64 residual r = b - A x_hi with the partial of its squared norm (start,
// replacement, final check); a replacement also stores r in the current tier.
__device__ __forceinline__ void k1_residual(const KArgs &a, int g, int mode, void *lds) {
  const int n = a.A.n;
  double sub[8];
#pragma unroll 1
  for (int sb = 0; sb < kGroupBlocks / kRPT; ++sb) {
    const int r0 = (g * kGroupBlocks + sb * kRPT) * kRowsPerBlock;
    if (r0 >= n) {
#pragma unroll
      for (int j = 0; j < kRPT; ++j) sub[sb * kRPT + j] = 0.0;
      continue;
    }
    const int nrows = min(kRPT * kRowsPerBlock, n - r0);
    double acc[kRPT];
    spmv_rows<FP64, kRPT>(a.A, (const double *)a.v.xhi, r0, nrows, lds, acc);
    double leaf[kRPT];
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int lr = threadIdx.x + j * kRowsPerBlock;
      leaf[j] = 0.0;
      if (lr < nrows) {
        const int i = r0 + lr;
        const double r = a.v.b[i] - acc[j];
        leaf[j] = r * r;
        if (mode == M_INIT) {
          a.v.r64[i] = r;
        } else if (mode == M_REPLACE) {
          if (a.ctl->tier) a.v.r64[i] = r; else a.v.r32[i] = (float)r;
        }
      }
    }
    double s2[kRPT];
    block_tree_multi<kRPT>(leaf, s2);
#pragma unroll
    for (int j = 0; j < kRPT; ++j) sub[sb * kRPT + j] = s2[j];
  }
  if (threadIdx.x == 0) a.part1[g] = tree8(sub);
}

__global__ __launch_bounds__(kBlock) void k_slot1(KArgs a) {
  const int mode = a.ctl->mode;
  if (a.slot_log && blockIdx.x == 0 && threadIdx.x == 0) a.slot_log[a.slot] = (int8_t)mode;
  if (mode == M_DONE) return;
  const int g = xcd_group(a.G1);
  if (g >= a.P2) return;
  __shared__ double lds[kLdsDoubles];
  if (mode == M_ITER) {
    const int fs = (a.ctl->action >> 4) & 3, tier = a.ctl->tier;
    switch (fs * 2 + tier) {
    case 0: k1_iter<FP16, 0>(a, g, lds); break;
    case 1: k1_iter<FP16, 1>(a, g, lds); break;
    case 2: k1_iter<BF16, 0>(a, g, lds); break;
    case 3: k1_iter<BF16, 1>(a, g, lds); break;
    case 4: k1_iter<FP32, 0>(a, g, lds); break;
    case 5: k1_iter<FP32, 1>(a, g, lds); break;
    case 6: k1_iter<FP64, 0>(a, g, lds); break;
    default: k1_iter<FP64, 1>(a, g, lds); break;
    }
  } else {
    k1_residual(a, g, mode, lds);
  }
}

// ---------------------------------------------------------------------------
// K2: nu (redundantly per block), alpha, x_lo = axpy(alpha, p, x_lo),
// r = axpy(-alpha, q, r), partial of sigma' = dot(r, r).
// ---------------------------------------------------------------------------
template <int FA, int FD>
__device__ __forceinline__ void k2_body(const KArgs &a) {
  constexpr int TIER = (FA == FP64);
  using V = typename TierT<TIER>::type;
  using Acc = typename AccT<FD>::type;
  V *xlo, *r;
  const V *p, *q;
  if constexpr (TIER) { xlo = a.v.xlo64; r = a.v.r64; p = a.v.p64; q = a.v.q64; }
  else { xlo = a.v.xlo32; r = a.v.r32; p = a.v.p32; q = a.v.q32; }
  const int n = a.A.n;
  const int base = blockIdx.x * kVecBlock + threadIdx.x * kVecPer;
  const bool full = base + 8 <= n;
  double nu = 0.0;
  if constexpr (TIER) nu = partials_total<Acc>(a.part1, a.P2);   // fp64 tier: registers first
  V pv[8], qv[8], rv[8], xv[8];
  if (full) {                       // fp32 tier: streaming loads first, they stay
    load8(p + base, pv);            // in flight while the wave reduces nu
    load8(q + base, qv);
    load8(r + base, rv);
    load8(xlo + base, xv);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = base + j;
      pv[j] = i < n ? p[i] : (V)0;
      qv[j] = i < n ? q[i] : (V)0;
      rv[j] = i < n ? r[i] : (V)0;
      xv[j] = i < n ? xlo[i] : (V)0;
    }
  }
  if constexpr (!TIER) nu = partials_total<Acc>(a.part1, a.P2);
  const double alpha = a.ctl->sigma / nu;
  if (!(nu > 0.0 && isfinite(nu)) || !isfinite(alpha)) return;   // breakdown: KS handles it
  Acc l[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    xv[j] = axpy1<FA>(alpha, pv[j], xv[j]);
    rv[j] = axpy1<FA>(-alpha, qv[j], rv[j]);
    l[j] = (full || base + j < n) ? dot_leaf<FD>(rv[j], rv[j]) : (Acc)0;
  }
  if (full) {
    store8(xlo + base, xv);
    store8(r + base, rv);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = base + j;
      if (i < n) {
        xlo[i] = xv[j];
        r[i] = rv[j];
      }
    }
  }
  const Acc t = block_tree(tree8(l));
  if (threadIdx.x == 0) a.part2[blockIdx.x] = (double)t;
}

__global__ __launch_bounds__(kBlock) void k_slot2(KArgs a) {
  const Ctl *c = a.ctl;
  if (c->mode != M_ITER) return;
  const int act = c->action;
  switch (((act & 3) << 2) | ((act >> 2) & 3)) {
  case 0: k2_body<FP16, FP16>(a); break;
  case 1: k2_body<FP16, BF16>(a); break;
  case 2: k2_body<FP16, FP32>(a); break;
  case 3: k2_body<FP16, FP64>(a); break;
  case 4: k2_body<BF16, FP16>(a); break;
  case 5: k2_body<BF16, BF16>(a); break;
  case 6: k2_body<BF16, FP32>(a); break;
  case 7: k2_body<BF16, FP64>(a); break;
  case 8: k2_body<FP32, FP16>(a); break;
  case 9: k2_body<FP32, BF16>(a); break;
  case 10: k2_body<FP32, FP32>(a); break;
  case 11: k2_body<FP32, FP64>(a); break;
  case 12: k2_body<FP64, FP16>(a); break;
  case 13: k2_body<FP64, BF16>(a); break;
  case 14: k2_body<FP64, FP32>(a); break;
  default: k2_body<FP64, FP64>(a); break;
  }
}

// ---------------------------------------------------------------------------
// KS: one block; final reductions and the scalar / policy step.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void copy_words(void *dst, const void *src, int bytes) {
  uint64_t *d = (uint64_t *)dst;
  const uint64_t *s = (const uint64_t *)src;
  for (int i = threadIdx.x; i < bytes / 8; i += kBlock) d[i] = s[i];
}

__global__ __launch_bounds__(kBlock) void k_scalar(KArgs a) {
  __shared__ Ctl sc;
  __shared__ PolicyDev sp;
  static_assert(sizeof(Ctl) % 8 == 0 && sizeof(PolicyDev) % 8 == 0, "word copies");
  copy_words(&sc, a.ctl, sizeof(Ctl));
  copy_words(&sp, a.pol, sizeof(PolicyDev));
  __syncthreads();
  const int mode = sc.mode;
  if (mode == M_DONE) return;
  const Sx x{&sc, &sp, a.h};
  Ctl *c = &sc;
  if (mode == M_ITER) {
    const int fd = (c->action >> 2) & 3;
    const double nu = reduce_partials_rt(fd, a.part1, a.P2);
    const double sig = reduce_partials_rt(fd, a.part2, a.P2);
    const double alpha = c->sigma / nu;
    if (!(nu > 0.0 && isfinite(nu)) || !isfinite(alpha)) {
      finish_block(x, false, true, false, false);
    } else {
      __shared__ int s_fin;
      if (threadIdx.x == 0) {
        c->alpha = alpha;
        c->sig_new = sig;
        c->k += 1;
        const int k = c->k;
        const double rho = sqrt(sig) / c->bnorm;
        c->rho_new = rho;
        const bool rep = (c->R > 0 && k % c->R == 0) || rho <= c->tol || !isfinite(sig);
        if (rep) {
          c->mode = M_REPLACE;
          c->k2op = K2_NONE;
          c->k3op = K3_FOLD;
          s_fin = 0;
        } else {
          s_fin = 1;
        }
      }
      __syncthreads();
      if (s_fin) finish_block(x, true, false, false, false);
    }
  } else {
    bool skip = false;
    if (mode == M_INIT && c->bnorm_ready == 0) {
      const double bb = partials_total<double>(a.part0, a.P2);
      __shared__ int s_zero;
      if (threadIdx.x == 0) {
        c->bnorm = sqrt(bb);
        c->bnorm_ready = 1;
        s_zero = 0;
        if (c->bnorm == 0.0) {
          c->zero_solution = 1;
          a.h.rho[0] = 0.0;
          c->status = 0;
          c->relres_true = 0.0;
          set_done(c);
          s_zero = 1;
        }
      }
      __syncthreads();
      skip = s_zero != 0;
    }
    if (!skip) {
      const double s64 = partials_total<double>(a.part1, a.P2);
      if (mode == M_INIT) {
        init_block(x, s64);
      } else if (mode == M_REPLACE) {
        replace_block(x, s64);
      } else if (threadIdx.x == 0) {   // M_FINAL
        c->relres_true = sqrt(s64) / c->bnorm;
        set_done(c);
      }
    }
  }
  __syncthreads();
  copy_words(a.ctl, &sc, sizeof(Ctl));
}

// ---------------------------------------------------------------------------
// K3: p = rd_fa(fma(beta, p, r)) [+ tier switch], fold, or p = r after a start
// ---------------------------------------------------------------------------
__device__ __forceinline__ void fold1(double *xhi, int i, double xl) {
  const double s = xhi[i] + xl;
  if (isfinite(s)) xhi[i] = s;
}

template <int FA>
__device__ __forceinline__ void k3_xpay(const KArgs &a, bool sw) {
  constexpr int TIER = (FA == FP64);
  using V = typename TierT<TIER>::type;
  V *p, *r, *xlo;
  if constexpr (TIER) { p = a.v.p64; r = a.v.r64; xlo = a.v.xlo64; }
  else { p = a.v.p32; r = a.v.r32; xlo = a.v.xlo32; }
  const double beta = a.ctl->beta;
  const int n = a.A.n;
  const int base = blockIdx.x * kVecBlock + threadIdx.x * kVecPer;
  if (!sw) {
    if (base + 8 <= n) {
      V pv[8], rv[8];
      load8(p + base, pv);
      load8(r + base, rv);
#pragma unroll
      for (int j = 0; j < 8; ++j) pv[j] = axpy1<FA>(beta, pv[j], rv[j]);
      store8(p + base, pv);
    } else {
      for (int j = 0; j < 8; ++j) {
        const int i = base + j;
        if (i < n) p[i] = axpy1<FA>(beta, p[i], r[i]);
      }
    }
    return;
  }
  for (int j = 0; j < 8; ++j) {
    const int i = base + j;
    if (i >= n) break;
    const V pn = axpy1<FA>(beta, p[i], r[i]);
    fold1(a.v.xhi, i, (double)xlo[i]);
    if constexpr (TIER) {   // fp64 -> fp32
      a.v.p32[i] = (float)pn;
      a.v.r32[i] = (float)r[i];
      a.v.xlo32[i] = 0.0f;
    } else {                // fp32 -> fp64
      a.v.p64[i] = (double)pn;
      a.v.r64[i] = (double)r[i];
      a.v.xlo64[i] = 0.0;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_slot3(KArgs a) {
  const Ctl *c = a.ctl;
  const int op = c->k3op;
  if (op == K3_NONE) return;
  const int n = a.A.n;
  const int base = blockIdx.x * kVecBlock + threadIdx.x * kVecPer;
  if (op == K3_FOLD) {
    const int tier = c->tier;
    for (int j = 0; j < 8; ++j) {
      const int i = base + j;
      if (i >= n) break;
      if (tier) { fold1(a.v.xhi, i, a.v.xlo64[i]); a.v.xlo64[i] = 0.0; }
      else { fold1(a.v.xhi, i, (double)a.v.xlo32[i]); a.v.xlo32[i] = 0.0f; }
    }
  } else if (op == K3_COPY) {
    const int tier = c->tier;
    for (int j = 0; j < 8; ++j) {
      const int i = base + j;
      if (i >= n) break;
      const double r = a.v.r64[i];
      if (tier) { a.v.p64[i] = r; a.v.xlo64[i] = 0.0; }
      else { const float f = (float)r; a.v.r32[i] = f; a.v.p32[i] = f; a.v.xlo32[i] = 0.0f; }
    }
  } else {
    const bool sw = c->k3switch != 0;
    switch (c->k3_fa) {
    case FP16: k3_xpay<FP16>(a, sw); break;
    case BF16: k3_xpay<BF16>(a, sw); break;
    case FP32: k3_xpay<FP32>(a, sw); break;
    default: k3_xpay<FP64>(a, sw); break;
    }
  }
}

// ---------------------------------------------------------------------------
// start / finish
// ---------------------------------------------------------------------------
// x_hi = x0, x_lo = 0, partials of b.b (pairwise fp64) for ||b||.
__global__ __launch_bounds__(kBlock) void k_start(KArgs a) {
  const int n = a.A.n;
  const int base = blockIdx.x * kVecBlock + threadIdx.x * kVecPer;
  double l[8];
  for (int j = 0; j < 8; ++j) {
    const int i = base + j;
    if (i < n) {
      a.v.xhi[i] = a.v.xout[i];
      a.v.xlo32[i] = 0.0f;
      a.v.xlo64[i] = 0.0;
      const double bi = a.v.b[i];
      l[j] = bi * bi;
    } else {
      l[j] = 0.0;
    }
  }
  const double t = block_tree(tree8(l));
  if (threadIdx.x == 0) a.part0[blockIdx.x] = t;
}

// x = x_hi + x_lo; requests the final true-residual check after a budget stop
// or a breakdown.
__global__ __launch_bounds__(kBlock) void k_finish(KArgs a) {
  const Ctl *c = a.ctl;
  const int n = a.A.n;
  const int tier = c->tier;
  const int zero = c->zero_solution;
  const int base = blockIdx.x * kVecBlock + threadIdx.x * kVecPer;
  for (int j = 0; j < 8; ++j) {
    const int i = base + j;
    if (i >= n) break;
    if (tier) { fold1(a.v.xhi, i, a.v.xlo64[i]); a.v.xlo64[i] = 0.0; }
    else { fold1(a.v.xhi, i, (double)a.v.xlo32[i]); a.v.xlo32[i] = 0.0f; }
    a.v.xout[i] = zero ? 0.0 : a.v.xhi[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (c->status == 1 || c->status == 3)) a.ctl->mode = M_FINAL;
}

// ---------------------------------------------------------------------------
// setup: shadows
// ---------------------------------------------------------------------------
// Thread per row: fp16 row exponent e (largest magnitude scaled into
// (2^14, 2^15]), fp32 = RNE(v), bf16 = RNE(v), fp16 = RNE(v 2^-e), all directly
// from fp64.
__global__ __launch_bounds__(kBlock) void k_shadows(int n, const int *rp, const double *v, float *v32,
                                                    uint16_t *vbf, uint16_t *vh, int8_t *rexp) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int s = rp[i], t = rp[i + 1];
  double mx = 0.0;
  for (int k = s; k < t; ++k) mx = fmax(mx, fabs(v[k]));
  int e = 0;
  if (mx > 0.0 && isfinite(mx)) {
    const uint64_t u = (uint64_t)__double_as_longlong(mx);
    const int ef = (int)((u >> 52) & 0x7ff);
    const uint64_t mant = u & 0xFFFFFFFFFFFFFull;
    int cexp;
    if (ef == 0) {   // fp64 subnormal maximum
      int ee;
      const double m = frexp(mx, &ee);
      cexp = (m == 0.5) ? ee - 1 : ee;
    } else {
      cexp = (ef - 1023) + (mant != 0 ? 1 : 0);
    }
    e = cexp - 15;
    e = e < -128 ? -128 : (e > 127 ? 127 : e);
  }
  rexp[i] = (int8_t)e;
  for (int k = s; k < t; ++k) {
    const double x = v[k];
    v32[k] = (float)x;
    vbf[k] = f32_to_bf16_bits_exact((float)round_narrow_f64<8, -126, 127>(x));
    vh[k] = f32_to_f16_bits_exact((float)round_narrow_f64<11, -14, 15>(ldexp(x, -e)));
  }
}

// ---------------------------------------------------------------------------
// single-op kernels (same device code paths as the solver)
// ---------------------------------------------------------------------------
template <int FS, int TIER>
__global__ __launch_bounds__(kBlock) void k_op_spmv(Mat A, const void *pv, void *qv, int P, int G) {
  using V = typename TierT<TIER>::type;
  const int blk = xcd_group(G);
  if (blk >= P) return;
  __shared__ double lds[kLdsDoubles];
  const int r0 = blk * kRowsPerBlock;
  const int rows = min(kRowsPerBlock, A.n - r0);
  typename AccT<FS>::type acc[1];
  spmv_rows<FS, 1>(A, (const V *)pv, r0, rows, lds, acc);
  if (threadIdx.x < rows) ((V *)qv)[r0 + threadIdx.x] = spmv_out<FS, V>(A, r0 + threadIdx.x, acc[0]);
}

__global__ __launch_bounds__(kBlock) void k_op_residual(Mat A, const double *b, const double *x, double *r,
                                                         int P, int G) {
  const int blk = xcd_group(G);
  if (blk >= P) return;
  __shared__ double lds[kLdsDoubles];
  const int r0 = blk * kRowsPerBlock;
  const int rows = min(kRowsPerBlock, A.n - r0);
  double acc[1];
  spmv_rows<FP64, 1>(A, x, r0, rows, lds, acc);
  if (threadIdx.x < rows) r[r0 + threadIdx.x] = b[r0 + threadIdx.x] - acc[0];
}

template <int FD, int TIER>
__global__ __launch_bounds__(kBlock) void k_op_dot(int n, const void *uv, const void *vv, double *part) {
  using V = typename TierT<TIER>::type;
  using Acc = typename AccT<FD>::type;
  const V *u = (const V *)uv, *v = (const V *)vv;
  const int base = blockIdx.x * kVecBlock + threadIdx.x * kVecPer;
  Acc l[8];
  for (int j = 0; j < 8; ++j) {
    const int i = base + j;
    l[j] = (i < n) ? dot_leaf<FD>(u[i], v[i]) : (Acc)0;
  }
  const Acc t = block_tree(tree8(l));
  if (threadIdx.x == 0) part[blockIdx.x] = (double)t;
}

__global__ __launch_bounds__(kBlock) void k_op_dot_final(int fd, const double *part, int P, double *out) {
  const double s = reduce_partials_rt(fd, part, P);
  if (threadIdx.x == 0) *out = s;
}

template <int FA>
__global__ __launch_bounds__(kBlock) void k_op_axpy(int n, double alpha, const void *uv, void *yv) {
  using V = typename TierT<FA == FP64>::type;
  const V *u = (const V *)uv;
  V *y = (V *)yv;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = axpy1<FA>(alpha, u[i], y[i]);
}

// Greedy decisions for given states (determinism checks of the policy).
__global__ __launch_bounds__(kBlock) void k_policy_decide(const PolicyDev *P, int m, const int64_t *k,
                                                          const double *rho, const int32_t *stag,
                                                          const float *feat, int32_t *state,
                                                          int32_t *action) {
  __shared__ float s_feat[kMlpIn], s_logits[kNAct];
  for (int idx = blockIdx.x; idx < m; idx += gridDim.x) {
    const int s = policy_state(P, (int)k[idx], rho[idx], stag[idx]);
    if (P->kind == POL_MLP) {
      if (threadIdx.x < kMlpIn) s_feat[threadIdx.x] = feat[(size_t)idx * kMlpIn + threadIdx.x];
      __syncthreads();
      mlp_logits_block(P, s_feat, s_logits);
      if (threadIdx.x == 0) { state[idx] = s; action[idx] = argmax64f(s_logits); }
      __syncthreads();
    } else if (threadIdx.x == 0) {
      int ex = 0;
      state[idx] = s;
      action[idx] = P->kind == POL_QTRAIN ? q_argmax(&P->q[s * kNAct]) : decide_scalar(P, s, (int)k[idx], &ex);
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_start(const KArgs &a, hipStream_t s) { hipLaunchKernelGGL(k_start, dim3(a.P2), dim3(kBlock), 0, s, a); }

void launch_k1(const KArgs &a, hipStream_t s) { hipLaunchKernelGGL(k_slot1, dim3(a.G1), dim3(kBlock), 0, s, a); }
void launch_k2(const KArgs &a, hipStream_t s) { hipLaunchKernelGGL(k_slot2, dim3(a.P2), dim3(kBlock), 0, s, a); }
void launch_ks(const KArgs &a, hipStream_t s) { hipLaunchKernelGGL(k_scalar, dim3(1), dim3(kBlock), 0, s, a); }
void launch_k3(const KArgs &a, hipStream_t s) { hipLaunchKernelGGL(k_slot3, dim3(a.P2), dim3(kBlock), 0, s, a); }

void launch_slot(const KArgs &a, hipStream_t s) {
  launch_k1(a, s);
  launch_k2(a, s);
  launch_ks(a, s);
  launch_k3(a, s);
}

void launch_finish(const KArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(a.P2), dim3(kBlock), 0, s, a);
  launch_k1(a, s);
  launch_ks(a, s);
}

void launch_shadows(int n, const int *rp, const double *v, float *v32, uint16_t *vbf, uint16_t *vh,
                    int8_t *rexp, hipStream_t s) {
  hipLaunchKernelGGL(k_shadows, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, rp, v, v32, vbf, vh,
                     rexp);
}

void launch_op_spmv(const Mat &A, int fs, int tier, const void *p, void *q, hipStream_t s) {
  const int P = (A.n + kRowsPerBlock - 1) / kRowsPerBlock;
  const int G = (P + 7) / 8 * 8;
#define MPCG_SPMV(FS, T) hipLaunchKernelGGL((k_op_spmv<FS, T>), dim3(G), dim3(kBlock), 0, s, A, p, q, P, G)
  switch (fs * 2 + tier) {
  case 0: MPCG_SPMV(FP16, 0); break;
  case 1: MPCG_SPMV(FP16, 1); break;
  case 2: MPCG_SPMV(BF16, 0); break;
  case 3: MPCG_SPMV(BF16, 1); break;
  case 4: MPCG_SPMV(FP32, 0); break;
  case 5: MPCG_SPMV(FP32, 1); break;
  case 6: MPCG_SPMV(FP64, 0); break;
  default: MPCG_SPMV(FP64, 1); break;
  }
#undef MPCG_SPMV
}

void launch_op_residual(const Mat &A, const double *b, const double *x, double *r, hipStream_t s) {
  const int P = (A.n + kRowsPerBlock - 1) / kRowsPerBlock;
  const int G = (P + 7) / 8 * 8;
  hipLaunchKernelGGL(k_op_residual, dim3(G), dim3(kBlock), 0, s, A, b, x, r, P, G);
}

void launch_op_dot(int n, int fd, int tier, const void *u, const void *v, double *part, int P2, double *out,
                   hipStream_t s) {
#define MPCG_DOT(FD, T) hipLaunchKernelGGL((k_op_dot<FD, T>), dim3(P2), dim3(kBlock), 0, s, n, u, v, part)
  switch (fd * 2 + tier) {
  case 0: MPCG_DOT(FP16, 0); break;
  case 1: MPCG_DOT(FP16, 1); break;
  case 2: MPCG_DOT(BF16, 0); break;
  case 3: MPCG_DOT(BF16, 1); break;
  case 4: MPCG_DOT(FP32, 0); break;
  case 5: MPCG_DOT(FP32, 1); break;
  case 6: MPCG_DOT(FP64, 0); break;
  default: MPCG_DOT(FP64, 1); break;
  }
#undef MPCG_DOT
  hipLaunchKernelGGL(k_op_dot_final, dim3(1), dim3(kBlock), 0, s, fd, part, P2, out);
}

void launch_op_axpy(int n, int fa, double alpha, const void *u, void *y, hipStream_t s) {
  const dim3 g((n + kBlock - 1) / kBlock);
  switch (fa) {
  case FP16: hipLaunchKernelGGL((k_op_axpy<FP16>), g, dim3(kBlock), 0, s, n, alpha, u, y); break;
  case BF16: hipLaunchKernelGGL((k_op_axpy<BF16>), g, dim3(kBlock), 0, s, n, alpha, u, y); break;
  case FP32: hipLaunchKernelGGL((k_op_axpy<FP32>), g, dim3(kBlock), 0, s, n, alpha, u, y); break;
  default: hipLaunchKernelGGL((k_op_axpy<FP64>), g, dim3(kBlock), 0, s, n, alpha, u, y); break;
  }
}

void launch_policy_decide(const PolicyDev *P, int m, const int64_t *k, const double *rho, const int32_t *stag,
                          const float *feat, int32_t *state, int32_t *action, hipStream_t s) {
  const int g = m < 1024 ? (m > 0 ? m : 1) : 1024;
  hipLaunchKernelGGL(k_policy_decide, dim3(g), dim3(kBlock), 0, s, P, m, k, rho, stag, feat, state, action);
}

}  // namespace mpcg
