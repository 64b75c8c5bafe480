// kernels.hip -- gfx950 kernels of the mixed-precision CG iteration.
//
// One CG iteration is three launches on one stream:
//   KA  SpMV q = A_fs p in the LDS-staged CSR form with the fused partial of
//       nu = p.q (in the other modes: the fp64 residual b - A x_hi of a start,
//       replacement or final check, with its squared norm).  KA only reads the
//       control block.
//   KB  scalar step on KA's partials (nu -> alpha, breakdown; or the start /
//       replacement bookkeeping), then x_lo += alpha p, r -= alpha q and the
//       partial of sigma' = r.r (or an elementwise step: p = r after a start,
//       the direction update after a replacement, a fold of x_lo into x_hi).
//   KX  scalar step on KB's partials (sigma' -> rho, replacement test, beta,
//       the policy's state, update and next action), then the direction update
//       p = rd_fa(fma(beta, p, r)) with a change of vector tier if the next
//       action needs one (or a fold of x_lo into x_hi).
// Every workgroup of KB and KX computes the scalar step identically from the
// partials; workgroup 0 commits it (control block, histories).  The control
// block is double-buffered (KA and KB read ctl[0], KB writes ctl[1], KX reads
// ctl[1] and writes ctl[0]), so no kernel reads a value its own workgroups
// write.  No kernel communicates between its own workgroups; kernel boundaries
// order every hand-off.  Policies whose step writes shared state (Q-learning
// updates, rollout logs) or evaluates the MLP run each step once, in a
// one-block kernel (KS) before KB and before KX.  The host only enqueues launches.
// Part 9 holds two-launch variants of the iteration for fixed actions.
#include <hip/hip_ext.h>

#include <mutex>
#include "kernels.hpp"
#include "launch.hpp"

// The file is compiled as nine objects in parallel (MPCG_KPART = 1..9): the
// plain SpMV kernel (1), the plain KB kernels (2), the preconditioned and
// fp64-rho KB kernels (3, 6), everything else with every host launcher (4),
// the batched kernels (5), the tf32 / emulation / bf16-vector variants of
// the SpMV (7) and of KB (8), and the single-reduction and pipelined CG with
// their launcher (9).  Without MPCG_KPART it is one object holding all of
// them.
#ifndef MPCG_KPART
#define MPCG_KPART 0
#endif
#define MPCG_IN_PART(n) (MPCG_KPART == 0 || MPCG_KPART == (n))

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
  } else if constexpr (FS == TF32) {
    load8(A.vtf + c, v);
  } else if constexpr (FS == FP8) {
    const uint2 w = *(const uint2 *)(A.v8 + c);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      v[j] = q52_bits_to_f32((uint8_t)(w.x >> (8 * j)));
      v[4 + j] = q52_bits_to_f32((uint8_t)(w.y >> (8 * j)));
    }
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
template <int FS, int RPT, typename G>
__device__ __forceinline__ void spmv_rows(const Mat &A, const G &gather, int r0, int nrows,
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
            xv[u] = gather.template get<Acc>(lc[kk - wb + u]);
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

// Gather of the SpMV's operand.
template <typename V>
struct GatherPlain {
  const V *p;
  __device__ __forceinline__ V value(int c) const { return p[c]; }
  template <typename Acc> __device__ __forceinline__ Acc get(int c) const { return to_acc<Acc>(p[c]); }
};

// Gather from a bf16 container (16-bit vector storage): exact widening.
struct GatherBf16 {
  const uint16_t *p;
  template <typename Acc> __device__ __forceinline__ Acc get(int c) const { return (Acc)bf16_bits_to_f32(p[c]); }
};

// 8 bf16 values of a 16-bit container (16 bytes, 8-aligned position), widened.
__device__ __forceinline__ void load8_bf16(const uint16_t *p, float (&v)[8]) {
  const uint4 w = *(const uint4 *)p;
  const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    v[2 * j] = bf16_bits_to_f32((uint16_t)(ws[j] & 0xffffu));
    v[2 * j + 1] = bf16_bits_to_f32((uint16_t)(ws[j] >> 16));
  }
}
// 8 bf16-representable floats stored as bits.
__device__ __forceinline__ void store8_bf16(uint16_t *p, const float (&v)[8]) {
  uint32_t ws[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
    ws[j] = (uint32_t)f32_to_bf16_bits_exact(v[2 * j]) | ((uint32_t)f32_to_bf16_bits_exact(v[2 * j + 1]) << 16);
  *(uint4 *)p = make_uint4(ws[0], ws[1], ws[2], ws[3]);
}
__device__ __forceinline__ uint16_t bf16_bits_of(double x) {   // RNE from fp64 to bf16, as bits
  return f32_to_bf16_bits_exact(rd_from_f64_to_f32<BF16>(x));
}

// p_new = rd_fa(fma_acc(rd_acc(beta), p, r)) in the tier of fa
template <typename Vo>
__device__ __forceinline__ Vo xpay_rt(int fa, double beta, Vo p, Vo r) {
  if constexpr (sizeof(Vo) == 8) {
    return __builtin_fma(beta, p, r);
  } else {
    const float t = __builtin_fmaf((float)beta, p, r);
    return rd_rt_f32(fa, t);
  }
}

// Jacobi preconditioner solve of one element, z = rd_fa(m r) in acc(fa), with
// m the fp32 reciprocal of the diagonal (fp64 vectors: the fp64 product).
template <int FA>
__device__ __forceinline__ float precond_z(float m, float r) { return rd_from_f32<FA>(m * r); }
template <int FA>
__device__ __forceinline__ double precond_z(float m, double r) { return (double)m * r; }
__device__ __forceinline__ float precond_z_rt(int fa, float m, float r) { return rd_rt_f32(fa, m * r); }
__device__ __forceinline__ double precond_z_rt(int, float m, double r) { return (double)m * r; }

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

// q_i = rd_tier(2^{e_i} acc) (e_i = 0 unless fp16 or q52)
template <int FS, typename V>
__device__ __forceinline__ V spmv_out(const Mat &A, int i, typename AccT<FS>::type acc) {
  if constexpr (FS == FP16 || FS == FP8) {
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
  case TF32: dot_leaf_multi<TF32, RPT>(u, v, valid, out); break;
  default: dot_leaf_multi<FP64, RPT>(u, v, valid, out); break;
  }
}

template <typename V>
__device__ __forceinline__ double dot_leaf_block_rt(int fd, V u, V v, bool valid) {
  switch (fd) {
  case FP16: return dot_leaf_block<FP16>(u, v, valid);
  case BF16: return dot_leaf_block<BF16>(u, v, valid);
  case FP32: return dot_leaf_block<FP32>(u, v, valid);
  case TF32: return dot_leaf_block<TF32>(u, v, valid);
  default: return dot_leaf_block<FP64>(u, v, valid);
  }
}

// Pairwise total of P partials, identical in every thread of the block.
template <typename A>
__device__ __forceinline__ double partials_total(const double *part, int P) {
  return (double)reduce_partials<A>(part, P);
}

__device__ __forceinline__ double reduce_partials_rt(int fd, const double *part, int P) {
  return fd == FP64 ? partials_total<double>(part, P) : partials_total<float>(part, P);
}

// Pairwise total of at most kVecBlock partials already loaded by the block
// (thread t holds partials 8t .. 8t+7, zero past the end): the same tree as
// reduce_partials for one segment.
template <typename A>
__device__ __forceinline__ double tree_preloaded(const double (&pv)[8]) {
  A l[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) l[j] = (A)pv[j];
  return (double)block_tree(tree8(l));
}

__device__ __forceinline__ double tree_preloaded_rt(int fd, const double (&pv)[8]) {
  return fd == FP64 ? tree_preloaded<double>(pv) : tree_preloaded<float>(pv);
}

// Thread t's 8 partials of part[0..P) (P <= kVecBlock), zero past the end.
__device__ __forceinline__ void preload_partials(const double *part, int P, double (&pv)[8]) {
  const int base = threadIdx.x * 8;
#pragma unroll
  for (int j = 0; j < 8; ++j) pv[j] = base + j < P ? part[base + j] : 0.0;
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
  return (P->cost[act_fs(a)] + P->cost[act_fd(a)]) + P->cost[act_fa(a)];
}

// Reward of a decision whose action ran n_it iterations (n_it = 1: the
// per-iteration reward of section 4.1).
__device__ double policy_reward(const PolicyDev *P, int a, double rho, bool conv, int n_it) {
  const double accterm = (rho <= P->eps_min) ? -log10_policy(P->eps_min) : -log10_policy(rho);
  double r = P->w1 * accterm - P->w2 * (policy_cost(P, a) * (double)n_it);
  if (conv) r = r + P->w3;
  return r;
}

// One Q-table per operation (section 4.1: Q_j over states x precisions for
// j = SpMV, dot, update) lives in the same table row: Q_j(s, d) = q[s][S j + d]
// with S = nfmt formats per table and d the format digit (4: tf32).
__device__ __forceinline__ int n_fmt(const PolicyDev *P) { return P->nfmt == 5 ? 5 : 4; }

__device__ __forceinline__ int argmax_n(const double *t, int S) {
  int best = 0;
  double bv = t[0];
  for (int p = 1; p < S; ++p)
    if (t[p] > bv) { best = p; bv = t[p]; }
  return best;
}

__device__ __forceinline__ int q_greedy_row(const PolicyDev *P, const double *row) {
  if (!P->per_op) return q_argmax(row);
  const int S = n_fmt(P);
  return act_compose(argmax_n(row, S), argmax_n(row + S, S), P->per_op == 2 ? FP64 : argmax_n(row + 2 * S, S));
}

// Q update of decision (s, a) toward reward R, bootstrapped from s_next
// (s_next < 0: terminal); per operation, each table toward R + gamma max_p Q_j(s', p).
__device__ void q_learn(const PolicyDev *P, int s, int a, double R, int s_next) {
  if (!P->per_op) {
    double t = R;
    if (s_next >= 0) {
      const double *row = &P->q[s_next * kNAct];
      t = R + P->gamma * row[q_argmax(row)];
    }
    double *q = &P->q[s * kNAct + a];
    *q = *q + P->lr * (t - *q);
    return;
  }
  const int S = n_fmt(P);
  const int dj[3] = {act_fmt_dig(act_fs(a)), act_fmt_dig(act_fd(a)), act_fmt_dig(act_fa(a))};
  for (int j = 0; j < (P->per_op == 2 ? 2 : 3); ++j) {
    double t = R;
    if (s_next >= 0) {
      const double *nx = &P->q[s_next * kNAct + S * j];
      t = R + P->gamma * nx[argmax_n(nx, S)];
    }
    double *q = &P->q[s * kNAct + S * j + dj[j]];
    *q = *q + P->lr * (t - *q);
  }
}

__device__ double lg_clamped(const PolicyDev *P, double r) {
  return (r <= P->eps_min) ? log10_policy(P->eps_min) : log10_policy(r);
}

// The residual history a step reads: rho_{k-i}, i = 0..7 (index clamped at
// 0) for the network features, and rho_{k - w_stag} for the stagnation flag.
// rho_k itself is the step's own value (the history entry k is written by the
// same step, by one workgroup only).  All loads are issued together.
struct HistVals {
  double lag[8];
  double stag_ref;
};

__device__ __forceinline__ void load_hist(const PolicyDev *P, const double *hr, int k, double cur, bool lags,
                                          HistVals &h) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    int idx = k - i;
    if (idx < 0) idx = 0;
    h.lag[i] = !lags ? 0.0 : idx == k ? cur : hr[idx];
  }
  h.stag_ref = k >= P->w_stag ? hr[k - P->w_stag] : 0.0;
}

__device__ void mlp_features(const PolicyDev *P, int k, const double (&hv)[8], int stag, double last_true,
                             int prev, float *f) {
  double lg[8];
  for (int i = 0; i < 8; ++i) lg[i] = lg_clamped(P, hv[i]);
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

// Greedy action of a fixed table: precomputed with the policy when the table
// has at most kQbestMax states (the same argmax, lowest index on ties), else
// from the table.
__device__ __forceinline__ int q_greedy(const PolicyDev *P, int s) {
  return s < P->n_qbest ? (int)P->qbest[s] : q_greedy_row(P, &P->q[s * kNAct]);
}

template <bool FULL>
__device__ int decide_scalar(const PolicyDev *P, int s, int k, int *explored) {
  *explored = 0;
  if constexpr (!FULL) return P->kind == POL_QTABLE ? q_greedy(P, s) : P->fixed_action;
  switch (P->kind) {
  case POL_FIXED: return P->fixed_action;
  case POL_QTABLE: return q_greedy(P, s);
  case POL_QTRAIN: {
    if (P->per_op) {   // an epsilon-greedy draw per operation, streams 2 .. 7
      const double *row = &P->q[s * kNAct];
      const int S = n_fmt(P);
      int d[3];
      for (int j = 0; j < 3; ++j) {
        if (j == 2 && P->per_op == 2) {   // updates fixed in fp64
          d[j] = FP64;
          break;
        }
        const double u0 = counter_uniform(P->seed, (uint64_t)P->episode, (uint64_t)k, (uint64_t)(2 + 2 * j));
        if (u0 < P->epsilon) {
          const double u1 = counter_uniform(P->seed, (uint64_t)P->episode, (uint64_t)k, (uint64_t)(3 + 2 * j));
          d[j] = (int)(u1 * (double)S);
          *explored = 1;
        } else {
          d[j] = argmax_n(row + S * j, S);
        }
      }
      return act_compose(d[0], d[1], d[2]);
    }
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

// Network weights staged in LDS by the one-block step kernel: each matrix
// input-major with its rows padded by one word (W1^T [16][129], W2^T
// [128][129], W3^T [128][65]), then b1, b2, b3.  At each step of the output
// chains a wave reads consecutive words, and the transposing copy writes
// words 129 (or 65) apart, both free of bank conflicts.
constexpr int kW1s = kMlpH + 1, kW2s = kMlpH + 1, kW3s = kNAct + 1;
constexpr int kNetW2 = kMlpIn * kW1s, kNetW3 = kNetW2 + kMlpH * kW2s, kNetB1 = kNetW3 + kMlpH * kW3s;
constexpr int kNetB2 = kNetB1 + kMlpH, kNetB3 = kNetB2 + kMlpH, kNetLds = kNetB3 + kNAct;

// Copy of the packed weights W1 | b1 | W2 | b2 | W3 | b3 (row-major [out][in])
// into the LDS layout above, by the whole block, in two halves: net_load
// issues every load of a thread (into registers), net_store writes them to
// LDS, so other loads issued in between share the same round trip.
struct NetRegs {
  static constexpr int n1 = kMlpH * kMlpIn / kBlock, n2 = kMlpH * kMlpH / kBlock, n3 = kNAct * kMlpH / kBlock;
  float r1[n1], r2[n2], r3[n3], rb[3];
};
static_assert(NetRegs::n1 * kBlock == kMlpH * kMlpIn && NetRegs::n2 * kBlock == kMlpH * kMlpH &&
                  NetRegs::n3 * kBlock == kNAct * kMlpH,
              "whole rounds of the block");

__device__ __forceinline__ void net_load(const float *__restrict__ g, NetRegs &r) {
  const float *W1 = g, *b1 = W1 + kMlpH * kMlpIn, *W2 = b1 + kMlpH, *b2 = W2 + kMlpH * kMlpH, *W3 = b2 + kMlpH,
              *b3 = W3 + kNAct * kMlpH;
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < NetRegs::n1; ++j) r.r1[j] = W1[t + j * kBlock];
#pragma unroll
  for (int j = 0; j < NetRegs::n2; ++j) r.r2[j] = W2[t + j * kBlock];
#pragma unroll
  for (int j = 0; j < NetRegs::n3; ++j) r.r3[j] = W3[t + j * kBlock];
  r.rb[0] = t < kMlpH ? b1[t] : 0.0f;
  r.rb[1] = t < kMlpH ? b2[t] : 0.0f;
  r.rb[2] = t < kNAct ? b3[t] : 0.0f;
}

__device__ __forceinline__ void net_store(const NetRegs &r, float *wl) {
  const int t = threadIdx.x;
#pragma unroll
  for (int j = 0; j < NetRegs::n1; ++j) {
    const int e = t + j * kBlock;
    wl[(e % kMlpIn) * kW1s + e / kMlpIn] = r.r1[j];
  }
#pragma unroll
  for (int j = 0; j < NetRegs::n2; ++j) {
    const int e = t + j * kBlock;
    wl[kNetW2 + (e % kMlpH) * kW2s + e / kMlpH] = r.r2[j];
  }
#pragma unroll
  for (int j = 0; j < NetRegs::n3; ++j) {
    const int e = t + j * kBlock;
    wl[kNetW3 + (e % kMlpH) * kW3s + e / kMlpH] = r.r3[j];
  }
  if (t < kMlpH) {
    wl[kNetB1 + t] = r.rb[0];
    wl[kNetB2 + t] = r.rb[1];
  }
  if (t < kNAct) wl[kNetB3 + t] = r.rb[2];
}

// MLP logits by one block: x = bf16(feat); h1 = bf16(gelu(W1 x + b1));
// h2 = bf16(gelu(W2 h1 + b2)); y = W3 h2 + b3.  Each output is one thread's fp32
// fma chain over its inputs in ascending order.  Weights from the policy
// (global, row-major) or, when wl is not NULL, from the staged LDS copy.
__device__ void mlp_logits_block(const PolicyDev *P, const float *feat, float *logits, const float *wl) {
  __shared__ float x[kMlpIn], h1[kMlpH], h2[kMlpH];
  const int t = threadIdx.x;
  if (t < kMlpIn) x[t] = rd_bf16_from_f32(feat[t]);
  __syncthreads();
  if (t < kMlpH) {
    float acc = 0.0f;
    if (wl) {
      for (int i = 0; i < kMlpIn; ++i) acc = __builtin_fmaf(wl[i * kW1s + t], x[i], acc);
      acc = acc + wl[kNetB1 + t];
    } else {
      for (int i = 0; i < kMlpIn; ++i) acc = __builtin_fmaf(P->W1[t * kMlpIn + i], x[i], acc);
      acc = acc + P->b1[t];
    }
    h1[t] = rd_bf16_from_f32(gelu_as(acc));
  }
  __syncthreads();
  if (t < kMlpH) {
    float acc = 0.0f;
    if (wl) {
      for (int i = 0; i < kMlpH; ++i) acc = __builtin_fmaf(wl[kNetW2 + i * kW2s + t], h1[i], acc);
      acc = acc + wl[kNetB2 + t];
    } else {
      for (int i = 0; i < kMlpH; ++i) acc = __builtin_fmaf(P->W2[t * kMlpH + i], h1[i], acc);
      acc = acc + P->b2[t];
    }
    h2[t] = rd_bf16_from_f32(gelu_as(acc));
  }
  __syncthreads();
  if (t < kNAct) {
    float acc = 0.0f;
    if (wl) {
      for (int i = 0; i < kMlpH; ++i) acc = __builtin_fmaf(wl[kNetW3 + i * kW3s + t], h2[i], acc);
      logits[t] = acc + wl[kNetB3 + t];
    } else {
      for (int i = 0; i < kMlpH; ++i) acc = __builtin_fmaf(P->W3[t * kMlpH + i], h2[i], acc);
      logits[t] = acc + P->b3[t];
    }
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
  bool writer;        // commits histories, Q updates and rollouts
  const float *wl;    // network weights staged in LDS, or NULL (read from the policy)
};
__device__ void set_done(Ctl *c) {
  c->mode = M_DONE;
    c->k3op = K3_NONE;
}

// Install the next action.  After a start/restart r is in the fp64 container
// and K3 copies it into the new tier; otherwise K3 applies p = r + beta p in the
// old tier and converts r, p if the tier changes.
template <bool FULL>
__device__ __forceinline__ void apply_decision(const Sx &a, int na, int ex, bool from_init) {
  Ctl *c = a.ctl;
  const int k = c->k;
  if (from_init && k >= c->maxit) {
    c->status = 1;
    set_done(c);
    return;
  }
  const int nt = (c->emul || act_fa(na) == FP64) ? 1 : (c->vec16 && act_fa(na) == BF16) ? 2 : 0;
  if (from_init) {
    c->k3op = K3_COPY;
    c->k3switch = 0;
    c->tier_old = 1;
  } else {
    c->k3op = K3_XPAY;
    c->k3switch = (nt != c->tier);
    c->tier_old = c->tier;
    if (c->k3switch && a.writer) a.h.flag[k - 1] |= FL_SWITCH;
  }
  c->tier = nt;
  c->action = na;
  c->explored = ex;
    if (a.writer) {
    a.h.act[k] = (uint8_t)na;
    a.h.flag[k] = ex ? FL_EXPLORED : 0;
  }
  c->cost_sum += policy_cost(a.pol, na);
  c->mode = M_ITER;
}

// Start / restart: rho_0 from the fp64 residual, first action.  Returns 1 when
// the decision needs the block's MLP forward (features left in s_feat).
template <bool FULL>
__device__ __forceinline__ int init_t0(const Sx &a, double s64, double s64z, float *s_feat) {
  Ctl *c = a.ctl;
  const PolicyDev *P = a.pol;
  const int k = c->k;
  const double rt = sqrt(s64) / c->bnorm;
  if (a.writer) a.h.rho[k] = rt;
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
  c->sigma = s64z;   // r64.r64, or r64.(M^-1 r64) with a preconditioner
  // the state (and its stagnation flag, a history read) feeds only learned
  // policies and rollouts
  const bool need_state = FULL || P->kind != POL_FIXED;
  const bool lags = FULL && (P->kind == POL_MLP || P->roll_cap > 0);
  HistVals hv;
  if (need_state) load_hist(P, a.h.rho, k, rt, lags, hv);
  const int stag = need_state && (k >= P->w_stag) && (rt >= hv.stag_ref);
  const int s = need_state ? policy_state(P, k, rt, stag) : 0;
  c->s = s;
  if (lags) mlp_features(P, k, hv.lag, stag, rt, c->prev_action, c->feat);
  c->k_dec = k;
  if (c->fell_back) {
    apply_decision<FULL>(a, 63, 0, true);
    return 0;
  }
  if constexpr (FULL) {
    if (P->kind == POL_MLP) {
      for (int i = 0; i < kMlpIn; ++i) s_feat[i] = c->feat[i];
      return 1;
    }
  }
  int ex = 0;
  const int na = decide_scalar<FULL>(P, s, k, &ex);
  apply_decision<FULL>(a, na, ex, true);
  return 0;
}

// End of an iteration (or of a failed one): history, beta, training update,
// rollout, convergence / breakdown / fallback / budget, next action.
template <bool FULL>
__device__ __forceinline__ int finish_t0(const Sx &a, bool completed, bool broke, bool converged, bool stagnated,
                         float *s_feat) {
  Ctl *c = a.ctl;
  const PolicyDev *P = a.pol;
  const int k = c->k;
  const bool active = !c->fell_back;
  const bool training = FULL && active && P->kind == POL_QTRAIN;
  const bool want_feat = FULL && active && (P->kind == POL_MLP || P->roll_cap > 0);
  const int act = c->action, s = c->s;
  const double rho = c->rho_new;
  if (completed && a.writer) a.h.rho[k] = rho;
  double beta = 0.0;
  if (completed && !broke && !converged) {
    beta = c->dir_restart ? 0.0 : c->sig_new / c->sigma;
    // with M: r^T M^-1 r > 0 for r != 0
    if (!isfinite(beta) || (c->precond && !(c->sig_new > 0.0))) broke = true;
  }
  int stag = 0, s_next = s;
  const bool need_state = FULL || P->kind != POL_FIXED;
  if (!broke && need_state) {
    HistVals hv;
    load_hist(P, a.h.rho, k, rho, want_feat, hv);
    stag = (k >= P->w_stag) && (rho >= hv.stag_ref);
    s_next = policy_state(P, k, rho, stag);
    if (want_feat) mlp_features(P, k, hv.lag, stag, c->last_true, act, c->feat_next);
  } else if (want_feat) {
    for (int i = 0; i < kMlpIn; ++i) c->feat_next[i] = c->feat[i];
  }
  // iterations run under the current decision, a failed one included
  const int n_it = (completed ? k : k + 1) - c->k_dec;
  if (converged) {
    const double rw = policy_reward(P, act, rho, true, n_it);
    if (training && a.writer) q_learn(P, s, act, rw, -1);
    if (FULL && active && a.writer) roll_log(P, c->feat, c->feat_next, act, rw, 1);
    c->status = c->fell_back ? 2 : 0;
    c->relres_true = rho;
    set_done(c);
    return 0;
  }
  if (broke || (stagnated && c->fallback_enabled && !c->fell_back)) {
    const double rw = -P->w2 * (policy_cost(P, act) * (double)n_it) - P->w3;
    if (training && a.writer) q_learn(P, s, act, rw, -1);
    if (FULL && active && a.writer) roll_log(P, c->feat, c->feat_next, act, rw, 1);
    if (!c->fallback_enabled || c->fell_back) {
      c->status = 3;
      set_done(c);
      return 0;
    }
    c->fell_back = 1;
    c->fallback_at = k;
    if (a.writer) a.h.flag[completed ? k - 1 : k] |= FL_FALLBACK;
    c->prev_action = act;
    c->mode = M_INIT;
        c->k3op = K3_FOLD;
    return 0;
  }
  // a decision ends at a multiple of the decision period, and when the budget cuts it
  const int D = P->decision_period > 1 ? P->decision_period : 1;
  const bool dec_end = (k % D == 0) || k >= c->maxit;
  if (dec_end && (training || (FULL && active && a.writer && P->roll_cap > 0))) {   // the reward has a reader
    const double rw = policy_reward(P, act, rho, false, n_it);
    if (training && a.writer) q_learn(P, s, act, rw, s_next);
    if (FULL && active && a.writer) roll_log(P, c->feat, c->feat_next, act, rw, 0);
  }
  if (k >= c->maxit) {
    c->status = 1;
    set_done(c);
    return 0;
  }
  c->beta = beta;
  c->sigma = c->sig_new;
  c->prev_action = act;
  c->k3_fa = act_fa(act);
  if (!dec_end) {                 // the action holds until the decision ends
    apply_decision<FULL>(a, act, 0, false);
    return 0;
  }
  c->s = s_next;
  c->k_dec = k;
  if (want_feat)
    for (int i = 0; i < kMlpIn; ++i) c->feat[i] = c->feat_next[i];
  if (c->fell_back) {
    apply_decision<FULL>(a, 63, 0, false);
    return 0;
  }
  if constexpr (FULL) {
    if (P->kind == POL_MLP) {
      for (int i = 0; i < kMlpIn; ++i) s_feat[i] = c->feat[i];
      return 1;
    }
  }
  int ex = 0;
  const int na = decide_scalar<FULL>(P, s_next, k, &ex);
  apply_decision<FULL>(a, na, ex, false);
  return 0;
}

// Block-level wrappers: thread 0 runs the scalar step; the block joins for an
// MLP decision.
template <bool FULL>
__device__ __forceinline__ void finish_block(const Sx &a, bool completed, bool broke, bool converged, bool stagnated) {
  __shared__ int s_need;
  __shared__ float s_feat[kMlpIn], s_logits[kNAct];
  if (threadIdx.x == 0) s_need = finish_t0<FULL>(a, completed, broke, converged, stagnated, s_feat);
  __syncthreads();
  if constexpr (FULL) {
    if (s_need) {
      mlp_logits_block(a.pol, s_feat, s_logits, a.wl);
      if (threadIdx.x == 0) apply_decision<FULL>(a, argmax64f(s_logits), 0, false);
    }
  }
}

template <bool FULL>
__device__ __forceinline__ void init_block(const Sx &a, double s64, double s64z) {
  __shared__ int s_need;
  __shared__ float s_feat[kMlpIn], s_logits[kNAct];
  if (threadIdx.x == 0) s_need = init_t0<FULL>(a, s64, s64z, s_feat);
  __syncthreads();
  if constexpr (FULL) {
    if (s_need) {
      mlp_logits_block(a.pol, s_feat, s_logits, a.wl);
      if (threadIdx.x == 0) apply_decision<FULL>(a, argmax64f(s_logits), 0, true);
    }
  }
}

template <bool FULL>
__device__ __forceinline__ void replace_block(const Sx &a, double s64, double s64z) {
  __shared__ int s_f[3];
  if (threadIdx.x == 0) {
    Ctl *c = a.ctl;
    const int k = c->k;
    const double rt = sqrt(s64) / c->bnorm;
    const double rho_rec = c->rho_new;   // the recursive residual being replaced
    if (c->nrep < a.h.cap_rep && a.writer) {
      a.h.rep_k[c->nrep] = k;
      a.h.rep_rho[c->nrep] = rt;
    }
    c->nrep++;
    if (a.writer) a.h.flag[k - 1] |= FL_REPLACED;
    c->last_true = rt;
    c->rho_new = rt;
    int conv = 0, broke = 0, stag = 0;
    if (rt <= c->tol) {
      conv = 1;
    } else if (!isfinite(rt)) {
      broke = 1;
    } else {
      c->sig_new = s64z;
      // with M, a replacement that more than doubles the residual restarts
      // the direction (p = z)
      c->dir_restart = c->precond && !(rt <= 2.0 * rho_rec);
      c->rep_hist[0] = c->rep_hist[1];
      c->rep_hist[1] = c->rep_hist[2];
      c->rep_hist[2] = rt;
      c->nrep_since++;
      if (c->nrep_since >= 3 && rt >= c->rep_hist[0]) stag = 1;
    }
    s_f[0] = conv; s_f[1] = broke; s_f[2] = stag;
  }
  __syncthreads();
  finish_block<FULL>(a, true, s_f[1] != 0, s_f[0] != 0, s_f[2] != 0);
}

// ---------------------------------------------------------------------------
// Scalar steps.  Called by every thread of a workgroup (block-uniform control
// flow); thread 0 does the scalar work on the LDS copy of the control block.
// ---------------------------------------------------------------------------
// Before KX: the end of an iteration (KB's sigma'): replacement test, then
// beta, policy update and next action.
// EXT: with the emulation reading's rounding of the totals (plain kernels
// leave it out).
template <bool FULL, bool EXT = true>
__device__ __forceinline__ void step_x(const Sx &x, const KArgs &a, const double (&pre)[8], bool have_pre) {
  Ctl *c = x.ctl;
  if (c->mode == M_DONE || !c->pend_sigma) return;
  const int fd = act_fd(c->action);
  // r.r gives rho: at the dot format, or in fp64 (rho64)
  const bool emul = EXT && c->emul;
  const int fr = (c->rho64 || emul) ? FP64 : fd;
  double sig = have_pre ? tree_preloaded_rt(fr, pre) : reduce_partials_rt(fr, a.part2, a.P2);
  // sigma' in the second partials: r.z with a preconditioner, r.r at the dot
  // format when rho is taken in fp64
  double sigz = (c->precond || c->rho64) ? reduce_partials_rt(emul ? FP64 : fd, a.part2b, a.P2) : sig;
  if constexpr (EXT) {
    if (emul) {   // emulation: fp64 totals rounded to the dot format (rho64: rho unrounded)
      if (c->precond || c->rho64) sigz = rd_rt_f64(fd, sigz);
      if (!c->rho64) sig = rd_rt_f64(fd, sig);
      if (!c->precond && !c->rho64) sigz = sig;
    }
  }
  __shared__ int s_fin;
  if (threadIdx.x == 0) {
    c->pend_sigma = 0;
    c->sig_new = sigz;
    c->dir_restart = 0;
    c->k += 1;
    const int k = c->k;
    const double rho = sqrt(sig) / c->bnorm;
    c->rho_new = rho;
    // section 5's termination (stop_rule 1): the recursive residual below tol
    // after at least 10 iterations, with no true-residual check
    const bool paper_stop = c->stop_rule == 1 && rho < c->tol && k >= 10 && isfinite(sig) && isfinite(sigz);
    const bool rep = !paper_stop && ((c->R > 0 && k % c->R == 0) || (c->stop_rule == 0 && rho <= c->tol) ||
                                     !isfinite(sig) || !isfinite(sigz));
    if (rep) {
      c->mode = M_REPLACE;
      c->k3op = c->fold_done ? K3_NONE : K3_FOLD;
      s_fin = 0;
    } else {
      s_fin = paper_stop ? 2 : 1;
    }
    c->fold_done = 0;
  }
  __syncthreads();
  if (s_fin) finish_block<FULL>(x, true, false, s_fin == 2, false);
  __syncthreads();
}

template <bool FULL>
__device__ __forceinline__ void step_x(const Sx &x, const KArgs &a) {
  const double none[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  step_x<FULL>(x, a, none, false);
}

// Before KB: KA's partials -- nu (alpha, breakdown) after an iteration, the
// residual norm after a start, replacement or final check.
template <bool FULL, bool EXT = true>
__device__ __forceinline__ void step_b(const Sx &x, const KArgs &a, const double (&pre)[8], bool have_pre) {
  Ctl *c = x.ctl;
  const int la = c->mode;   // what KA has just executed
  if (la == M_ITER) {
    const int fd = act_fd(c->action);
    // emulation: the fp64 total rounded to the dot format
    const bool emul = EXT && c->emul;
    const int fn = emul ? FP64 : fd;
    double nu = have_pre ? tree_preloaded_rt(fn, pre) : reduce_partials_rt(fn, a.part1, a.P1);
    if constexpr (EXT) {
      if (emul) nu = rd_rt_f64(fd, nu);
    }
    const double alpha = c->sigma / nu;
    if (!(nu > 0.0 && isfinite(nu)) || !isfinite(alpha)) {
      finish_block<FULL>(x, false, true, false, false);
      __syncthreads();
      if (threadIdx.x == 0) c->b_op = B_EXEC;
    } else if (threadIdx.x == 0) {
      c->alpha = alpha;
      c->b_op = B_AXPY;
    }
  } else if (la == M_INIT || la == M_REPLACE || la == M_FINAL) {
    if (la == M_INIT && !c->bnorm_ready) {   // first start: ||b|| from the start kernel
      const double bb = partials_total<double>(a.part0, a.P2);
      if (threadIdx.x == 0) {
        c->bnorm = sqrt(bb);
        c->bnorm_ready = 1;
      }
      __syncthreads();
      if (c->bnorm == 0.0) {
        if (threadIdx.x == 0) {
          c->zero_solution = 1;
          if (x.writer) a.h.rho[0] = 0.0;
          c->status = 0;
          c->relres_true = 0.0;
          set_done(c);
          c->b_op = B_NONE;
        }
        __syncthreads();
        return;
      }
    }
    const double s64 = have_pre ? tree_preloaded<double>(pre) : partials_total<double>(a.part1, a.P1);
    const double s64z = (c->precond && la != M_FINAL) ? partials_total<double>(a.part1b, a.P1) : s64;
    if (la == M_INIT) {
      init_block<FULL>(x, s64, s64z);
    } else if (la == M_REPLACE) {
      replace_block<FULL>(x, s64, s64z);
    } else if (threadIdx.x == 0) {
      c->relres_true = sqrt(s64) / c->bnorm;
      set_done(c);
    }
    __syncthreads();
    if (threadIdx.x == 0) c->b_op = B_EXEC;
  } else if (threadIdx.x == 0) {
    c->b_op = B_NONE;
  }
  __syncthreads();
}

template <bool FULL>
__device__ __forceinline__ void step_b(const Sx &x, const KArgs &a) {
  const double none[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  step_b<FULL>(x, a, none, false);
}

__device__ __forceinline__ void copy_words(void *dst, const void *src, int bytes) {
  uint64_t *d = (uint64_t *)dst;
  const uint64_t *s = (const uint64_t *)src;
  for (int i = threadIdx.x; i < bytes / 8; i += kBlock) d[i] = s[i];
}

__device__ __forceinline__ void fold1(double *xhi, int i, double xl) {
  const double s = xhi[i] + xl;
  if (isfinite(s)) xhi[i] = s;
}

template <int RPT>
__device__ __forceinline__ double subtrees_rt(int fd, const double (&s)[RPT]) {
  if constexpr (RPT == 1) {
    return s[0];
  } else {
    static_assert(RPT == 2, "pairwise combination written for two subtrees");
    if (fd == FP64) return s[0] + s[1];
    return (double)((float)s[0] + (float)s[1]);
  }
}

// ---------------------------------------------------------------------------
// KA: SpMV over a group of consecutive rows per workgroup (a.grows rows, a
// power of two from 512 to 2048), software-pipelined: the group's row pointers
// are staged in LDS once, and while the rows of one window of CSR entries run
// their gathers and fma chains, the next window's values and column indices
// are already in flight into registers.  Each 512-row sub-block ends with an
// epilogue (output, partials); the group partial is the pairwise sum of its
// sub-block partials, i.e. an aligned subtree of the whole vector's tree.
// ---------------------------------------------------------------------------
constexpr int kMaxGroupRows = 2048;

// LDS window of the group SpMV: values kept in their storage format (16-bit
// formats as raw bits, widened when read), 4096 entries for 16-bit formats,
// 2048 otherwise; 24 KiB of values and indices in every case.
template <int FS> struct LdsWin { using type = float; static constexpr int cap = 2048; };
template <> struct LdsWin<FP64> { using type = double; static constexpr int cap = 2048; };
template <> struct LdsWin<BF16> { using type = uint16_t; static constexpr int cap = 4096; };
template <> struct LdsWin<FP16> { using type = uint16_t; static constexpr int cap = 4096; };
template <> struct LdsWin<FP8> { using type = uint8_t; static constexpr int cap = 4096; };
constexpr int kLdsWinBytes = 24576;
constexpr int kLdsKa = (kLdsWinBytes + (kMaxGroupRows + 4) * 4) / 8;   // doubles

template <int FS> struct RawVals { float v[8]; };
template <> struct RawVals<FP64> { double v[8]; };
template <> struct RawVals<FP16> { uint4 w; };
template <> struct RawVals<BF16> { uint4 w; };
template <> struct RawVals<FP8> { uint2 w; };

template <int FS>
__device__ __forceinline__ void raw_load(const Mat &A, int c, RawVals<FS> &r) {
  if constexpr (FS == FP64) load8(A.v64 + c, r.v);
  else if constexpr (FS == FP32) load8(A.v32 + c, r.v);
  else if constexpr (FS == TF32) load8(A.vtf + c, r.v);
  else if constexpr (FS == FP8) r.w = *(const uint2 *)(A.v8 + c);
  else r.w = *(const uint4 *)((FS == BF16 ? A.vbf : A.vh) + c);
}

template <int FS>
__device__ __forceinline__ void raw_to_lds(const RawVals<FS> &r, typename LdsWin<FS>::type *p) {
  if constexpr (FS == FP64 || FS == FP32 || FS == TF32) lds_store8(p, r.v);
  else if constexpr (FS == FP8) *(uint2 *)p = r.w;
  else *(uint4 *)p = r.w;
}

// One stored value, widened to the accumulation type (exact).
template <int FS>
__device__ __forceinline__ typename AccT<FS>::type lds_widen(typename LdsWin<FS>::type x) {
  if constexpr (FS == BF16) return bf16_bits_to_f32(x);
  else if constexpr (FS == FP16) return f16_bits_to_f32(x);
  else if constexpr (FS == FP8) return q52_bits_to_f32(x);
  else return x;
}

__device__ __forceinline__ double add_rt(int fd, double x, double y) {
  if (fd == FP64) return x + y;
  return (double)((float)x + (float)y);
}

// Pairwise sum of the sub-block partials t[0..3] of a group of `grows` rows.
__device__ __forceinline__ double group_tree(int fd, int grows, const double (&t)[4]) {
  if (grows <= 512) return t[0];
  if (grows <= 1024) return add_rt(fd, t[0], t[1]);
  return add_rt(fd, add_rt(fd, t[0], t[1]), add_rt(fd, t[2], t[3]));
}

// Prefetch of one window: up to two 8-entry chunks per thread, held in
// registers (values in their storage format; column indices as int32, or as
// 16-bit deltas col - row when DC, one int4 per chunk).
template <int FS, int NCH, bool DC>
__device__ __forceinline__ void win_load(const Mat &A, int wb, int we, RawVals<FS> &v0, RawVals<FS> &v1,
                                         int4 &c0a, int4 &c0b, int4 &c1a, int4 &c1b) {
  const int c0 = wb + threadIdx.x * 8;
  if constexpr (DC && (FS == BF16 || FS == FP16)) {
    // interleaved value | delta words: 32 bytes per 8 entries, one stream
    const uint32_t *pk = FS == BF16 ? A.pbf : A.ph;
    if (c0 < we) {
      c0a = *(const int4 *)(pk + c0);
      c0b = *(const int4 *)(pk + c0 + 4);
    }
    if constexpr (NCH == 2) {
      const int c1 = c0 + kVecBlock;
      if (c1 < we) {
        c1a = *(const int4 *)(pk + c1);
        c1b = *(const int4 *)(pk + c1 + 4);
      }
    }
    return;
  }
  if (c0 < we) {
    raw_load<FS>(A, c0, v0);
    if constexpr (DC) {
      c0a = *(const int4 *)(A.dc + c0);
    } else {
      c0a = *(const int4 *)(A.ci + c0);
      c0b = *(const int4 *)(A.ci + c0 + 4);
    }
  }
  if constexpr (NCH == 2) {
    const int c1 = c0 + kVecBlock;
    if (c1 < we) {
      raw_load<FS>(A, c1, v1);
      if constexpr (DC) {
        c1a = *(const int4 *)(A.dc + c1);
      } else {
        c1a = *(const int4 *)(A.ci + c1);
        c1b = *(const int4 *)(A.ci + c1 + 4);
      }
    }
  }
}

template <int FS, int NCH, bool DC>
__device__ __forceinline__ void win_store(int wb, int we, const RawVals<FS> &v0, const RawVals<FS> &v1,
                                          int4 c0a, int4 c0b, int4 c1a, int4 c1b,
                                          typename LdsWin<FS>::type *lv, void *lc) {
  const int o0 = threadIdx.x * 8;
  if constexpr (DC && (FS == BF16 || FS == FP16)) {
    uint32_t *lp = (uint32_t *)lv;   // the interleaved words as they are
    if (wb + o0 < we) {
      *(int4 *)(lp + o0) = c0a;
      *(int4 *)(lp + o0 + 4) = c0b;
    }
    if constexpr (NCH == 2) {
      const int o1 = o0 + kVecBlock;
      if (wb + o1 < we) {
        *(int4 *)(lp + o1) = c1a;
        *(int4 *)(lp + o1 + 4) = c1b;
      }
    }
    return;
  }
  if (wb + o0 < we) {
    raw_to_lds<FS>(v0, lv + o0);
    if constexpr (DC) {
      *(int4 *)((int16_t *)lc + o0) = c0a;
    } else {
      *(int4 *)((int *)lc + o0) = c0a;
      *(int4 *)((int *)lc + o0 + 4) = c0b;
    }
  }
  if constexpr (NCH == 2) {
    const int o1 = o0 + kVecBlock;
    if (wb + o1 < we) {
      raw_to_lds<FS>(v1, lv + o1);
      if constexpr (DC) {
        *(int4 *)((int16_t *)lc + o1) = c1a;
      } else {
        *(int4 *)((int *)lc + o1) = c1a;
        *(int4 *)((int *)lc + o1 + 4) = c1b;
      }
    }
  }
}

// Column of window entry e of a row `row`: the stored index, or row + delta.
template <bool DC>
__device__ __forceinline__ int win_col(const void *lc, int e, int row) {
  if constexpr (DC) return row + (int)((const int16_t *)lc)[e];
  else return ((const int *)lc)[e];
}

// pref(sb) issues sub-block sb's own-row loads ahead of time: for sb = 0
// before the row pointers are staged, for later sub-blocks together with the
// prefetch of their first window.  pre(sb) runs when sub-block sb starts,
// epi(sb, acc) when its rows are complete.  All three are called by every
// thread (block-uniform).
template <int FS, bool DC, typename G, typename Pref, typename Pre, typename Epi>
__device__ __forceinline__ void spmv_group(const Mat &A, const G &gather, int g0, int grows, void *lds_raw,
                                           Pref &&pref, Pre &&pre, Epi &&epi) {
  using Acc = typename AccT<FS>::type;
  using L = typename LdsWin<FS>::type;
  constexpr int CAP = LdsWin<FS>::cap;
  constexpr int NCH = CAP / kVecBlock;
  constexpr bool PACK = DC && (FS == BF16 || FS == FP16);   // value | delta << 16 words
  static_assert(NCH == 1 || NCH == 2, "window of one or two chunks per thread");
  static_assert(CAP * (sizeof(L) + 4) <= kLdsWinBytes, "window fits its LDS");
  L *lv = (L *)lds_raw;
  void *lc = (void *)(lv + CAP);
  const uint32_t *lp = (const uint32_t *)lds_raw;
  int *lrp = (int *)((char *)lds_raw + kLdsWinBytes);
  const int tid = threadIdx.x;
  pref(0);
  for (int i = tid; i <= grows; i += kBlock) lrp[i] = A.rp[g0 + i];
  __syncthreads();
  const int nsb = (grows + kKaRows - 1) / kKaRows;
  RawVals<FS> v0, v1;
  int4 c0a, c0b, c1a, c1b;
  int sb = 0;
  int ke = lrp[min(kKaRows, grows)];
  int wb = lrp[0] & ~7;
  win_load<FS, NCH, DC>(A, wb, min(wb + CAP, ke), v0, v1, c0a, c0b, c1a, c1b);
  Acc acc[kRPT];
  int my_s[kRPT], my_e[kRPT], my_row[kRPT];
  auto rows_of = [&](int s) {
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int lr = s * kKaRows + tid + j * kRowsPerBlock;
      acc[j] = (Acc)0;
      my_s[j] = 0;
      my_e[j] = 0;
      my_row[j] = g0 + lr;
      if (lr < grows) {
        my_s[j] = lrp[lr];
        my_e[j] = lrp[lr + 1];
      }
    }
  };
  rows_of(0);
  pre(0);
  while (true) {
    const int we = min(wb + CAP, ke);
    win_store<FS, NCH, DC>(wb, we, v0, v1, c0a, c0b, c1a, c1b, lv, lc);
    __syncthreads();
    // the next window: the rest of this sub-block, or the start of the next one
    int nsb_ = sb, nwb = wb + CAP, nke = ke;
    if (we >= ke) {
      nsb_ = sb + 1;
      if (nsb_ < nsb) {
        nwb = lrp[nsb_ * kKaRows] & ~7;
        nke = lrp[min((nsb_ + 1) * kKaRows, grows)];
      }
    }
    // The next window's loads are issued right after this window's first
    // gathers: waiting for those gathers (in-order counters) then does not
    // wait for the prefetch, which stays in flight through the fma chains.
    bool pf = nsb_ < nsb;
    if constexpr (sizeof(Acc) == 4) {
      // the thread's rows advance together, eight entries each per step, so
      // the gathers of all its rows are in flight at once
      int lo[kRPT], hi[kRPT], steps = 0;
#pragma unroll
      for (int j = 0; j < kRPT; ++j) {
        lo[j] = max(my_s[j], wb);
        hi[j] = min(my_e[j], we);
        steps = max(steps, (hi[j] - lo[j] + 7) >> 3);
      }
      for (int st = 0; st < steps; ++st) {
        Acc xv[kRPT][8], vv[kRPT][8];
        int cnt[kRPT];
#pragma unroll
        for (int j = 0; j < kRPT; ++j) {
          const int kk = lo[j] + st * 8;
          cnt[j] = hi[j] - kk;
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (u < cnt[j]) {
              if constexpr (PACK) {
                const uint32_t e = lp[kk - wb + u];
                vv[j][u] = lds_widen<FS>((L)(e & 0xffffu));
                xv[j][u] = gather.template get<Acc>(my_row[j] + (int)(int16_t)(e >> 16));
              } else {
                vv[j][u] = lds_widen<FS>(lv[kk - wb + u]);
                xv[j][u] = gather.template get<Acc>(win_col<DC>(lc, kk - wb + u, my_row[j]));
              }
            }
          }
        }
        if (pf) {
          win_load<FS, NCH, DC>(A, nwb, min(nwb + CAP, nke), v0, v1, c0a, c0b, c1a, c1b);
          if (nsb_ != sb) pref(nsb_);
          pf = false;
        }
#pragma unroll
        for (int j = 0; j < kRPT; ++j)
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (u < cnt[j]) acc[j] = fma_acc(vv[j][u], xv[j][u], acc[j]);
      }
    } else {
      // fp64: one row at a time (register budget)
#pragma unroll
      for (int j = 0; j < kRPT; ++j) {
        const int lo = max(my_s[j], wb), hi = min(my_e[j], we);
        for (int kk = lo; kk < hi; kk += 8) {
          const int cnt = hi - kk;
          Acc xv[8], vv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (u < cnt) {
              vv[u] = lds_widen<FS>(lv[kk - wb + u]);
              xv[u] = gather.template get<Acc>(win_col<DC>(lc, kk - wb + u, my_row[j]));
            }
          }
          if (pf) {
            win_load<FS, NCH, DC>(A, nwb, min(nwb + CAP, nke), v0, v1, c0a, c0b, c1a, c1b);
            if (nsb_ != sb) pref(nsb_);
            pf = false;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (u < cnt) acc[j] = fma_acc(vv[u], xv[u], acc[j]);
        }
      }
    }
    if (pf) {
      win_load<FS, NCH, DC>(A, nwb, min(nwb + CAP, nke), v0, v1, c0a, c0b, c1a, c1b);
      if (nsb_ != sb) pref(nsb_);
    }
    if (we >= ke) {
      epi(sb, acc);
      if (nsb_ >= nsb) break;
      rows_of(nsb_);
      pre(nsb_);
    }
    __syncthreads();   // the LDS window is refilled next
    sb = nsb_;
    wb = nwb;
    ke = nke;
  }
}

// EMUL: the paper's emulation reading, an fp64 SpMV whose q_i are rounded to
// the action's SpMV format, and the nu partials in fp64.
// P16: p in the bf16 container (16-bit vector storage), q in fp32.
template <int FS, int TIER, bool EMUL = false, bool P16 = false>
__device__ __forceinline__ void ka_iter(const KArgs &a, const Ctl &S, int g, void *lds) {
  using V = typename TierT<TIER>::type;
  using Acc = typename AccT<FS>::type;
  static_assert(!EMUL || (FS == FP64 && TIER == 1), "emulation runs the fp64 path");
  const V *p;
  V *q;
  if constexpr (TIER) { p = a.v.p64; q = a.v.q64; } else { p = a.v.p32; q = a.v.q32; }
  const int fd = EMUL ? FP64 : act_fd(S.action);
  const int fs_round = act_fs(S.action);
  const int n = a.A.n;
  const int g0 = g * a.grows;
  const int grows = min(a.grows, n - g0);
  V pi[kRPT], pn[kRPT];   // own elements of p: current sub-block, next sub-block
  int8_t ex[kRPT];
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  auto pref = [&](int sb) {
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int lr = sb * kKaRows + threadIdx.x + j * kRowsPerBlock;
      if constexpr (P16) pn[j] = lr < grows ? (V)bf16_bits_to_f32(a.v.p16[g0 + lr]) : (V)0;
      else pn[j] = lr < grows ? p[g0 + lr] : (V)0;
    }
  };
  auto pre = [&](int sb) {
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int lr = sb * kKaRows + threadIdx.x + j * kRowsPerBlock;
      pi[j] = pn[j];
      ex[j] = 0;
      if constexpr (FS == FP16 || FS == FP8) {
        if (lr < grows) ex[j] = a.A.rexp[g0 + lr];
      }
    }
  };
  auto epi = [&](int sb, Acc (&acc)[kRPT]) {
    V qi[kRPT];
    bool valid[kRPT];
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int lr = sb * kKaRows + threadIdx.x + j * kRowsPerBlock;
      valid[j] = lr < grows;
      qi[j] = (V)0;
      if (valid[j]) {
        if constexpr (FS == FP16 || FS == FP8) qi[j] = (V)ldexp((double)acc[j], (int)ex[j]);
        else qi[j] = (V)acc[j];
        if constexpr (EMUL) qi[j] = rd_rt_f64(fs_round, qi[j]);
        q[g0 + lr] = qi[j];
      }
    }
    double s2[kRPT];
    dot_leaf_multi_rt<kRPT>(fd, pi, qi, valid, s2);
    const double s = subtrees_rt<kRPT>(fd, s2);
    t[0] = sb == 0 ? s : t[0];
    t[1] = sb == 1 ? s : t[1];
    t[2] = sb == 2 ? s : t[2];
    t[3] = sb == 3 ? s : t[3];
  };
  if constexpr (P16) {
    if (a.A.dc) spmv_group<FS, true>(a.A, GatherBf16{a.v.p16}, g0, grows, lds, pref, pre, epi);
    else spmv_group<FS, false>(a.A, GatherBf16{a.v.p16}, g0, grows, lds, pref, pre, epi);
  } else {
    if (a.A.dc) spmv_group<FS, true>(a.A, GatherPlain<V>{p}, g0, grows, lds, pref, pre, epi);
    else spmv_group<FS, false>(a.A, GatherPlain<V>{p}, g0, grows, lds, pref, pre, epi);
  }
  if (threadIdx.x == 0) a.part1[g] = group_tree(fd, a.grows, t);
}

// fp64 residual r = b - A x_hi with the partial of its squared norm (start,
// replacement, final check); a start stores r in the fp64 container, a
// replacement in the current tier.
__device__ __forceinline__ void ka_residual(const KArgs &a, const Ctl &S, int g, int mode, void *lds) {
  const int n = a.A.n;
  const int g0 = g * a.grows;
  const int grows = min(a.grows, n - g0);
  // with a preconditioner a start or replacement also sums r64.(M^-1 r64)
  const bool pc = S.precond && (mode == M_INIT || mode == M_REPLACE);
  double bi[kRPT];
  float mi[kRPT];
  double t[4] = {0.0, 0.0, 0.0, 0.0}, tz[4] = {0.0, 0.0, 0.0, 0.0};
  auto pre = [&](int sb) {
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int lr = sb * kKaRows + threadIdx.x + j * kRowsPerBlock;
      bi[j] = lr < grows ? a.v.b[g0 + lr] : 0.0;
      mi[j] = (pc && lr < grows) ? a.A.minv[g0 + lr] : 0.0f;
    }
  };
  auto epi = [&](int sb, double (&acc)[kRPT]) {
    double leaf[kRPT], leafz[kRPT];
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int lr = sb * kKaRows + threadIdx.x + j * kRowsPerBlock;
      leaf[j] = 0.0;
      leafz[j] = 0.0;
      if (lr < grows) {
        const int i = g0 + lr;
        const double r = bi[j] - acc[j];
        leaf[j] = r * r;
        leafz[j] = r * ((double)mi[j] * r);
        if (mode == M_INIT) {
          a.v.r64[i] = r;
        } else if (mode == M_REPLACE) {
          if (S.tier == 1) a.v.r64[i] = r;
          else if (S.tier == 2) a.v.r16[i] = bf16_bits_of(r);
          else a.v.r32[i] = (float)r;
        }
      }
    }
    double s2[kRPT];
    block_tree_multi<kRPT>(leaf, s2);
    const double s = subtrees_rt<kRPT>(FP64, s2);
    t[0] = sb == 0 ? s : t[0];
    t[1] = sb == 1 ? s : t[1];
    t[2] = sb == 2 ? s : t[2];
    t[3] = sb == 3 ? s : t[3];
    if (pc) {
      block_tree_multi<kRPT>(leafz, s2);
      const double sz = subtrees_rt<kRPT>(FP64, s2);
      tz[0] = sb == 0 ? sz : tz[0];
      tz[1] = sb == 1 ? sz : tz[1];
      tz[2] = sb == 2 ? sz : tz[2];
      tz[3] = sb == 3 ? sz : tz[3];
    }
  };
  auto pref = [](int) {};
  if (a.A.dc) spmv_group<FP64, true>(a.A, GatherPlain<double>{a.v.xhi}, g0, grows, lds, pref, pre, epi);
  else spmv_group<FP64, false>(a.A, GatherPlain<double>{a.v.xhi}, g0, grows, lds, pref, pre, epi);
  if (threadIdx.x == 0) {
    a.part1[g] = group_tree(FP64, a.grows, t);
    if (pc) a.part1b[g] = group_tree(FP64, a.grows, tz);
  }
}

// x_hi += x_lo, x_lo = 0 over one 2048-element group (current tier).
__device__ __forceinline__ void fold_group(const KArgs &a, int tier, int g) {
  const int n = a.A.n;
  const int base = g * kVecBlock + threadIdx.x * kVecPer;
  for (int j = 0; j < 8; ++j) {
    const int i = base + j;
    if (i >= n) break;
    if (tier == 1) { fold1(a.v.xhi, i, a.v.xlo64[i]); a.v.xlo64[i] = 0.0; }
    else if (tier == 2) { fold1(a.v.xhi, i, (double)bf16_bits_to_f32(a.v.x16[i])); a.v.x16[i] = 0; }
    else { fold1(a.v.xhi, i, (double)a.v.xlo32[i]); a.v.xlo32[i] = 0.0f; }
  }
}

// KA's work on row group g of one system.
// V16: the variant that also runs iterations whose p is in the bf16
// container (16-bit vector storage, tier 2).
// EXT: the tf32 formats and the emulation reading (kernels launched when the
// policy or the options can use them; the plain variant keeps its code small).
template <bool V16 = false, bool EXT = true>
__device__ __forceinline__ void ka_body(const KArgs &a, int g, double *lds) {
  const Ctl &S = a.ctl[0];
  const int mode = S.mode;
  if (a.slot_log && g == 0 && threadIdx.x == 0) a.slot_log[a.slot] = (int8_t)mode;
  if (V16 && mode == M_ITER && S.tier == 2) {
    if constexpr (V16) {
      switch (act_fs(S.action)) {
      case FP16: ka_iter<FP16, 0, false, true>(a, S, g, lds); break;
      case BF16: ka_iter<BF16, 0, false, true>(a, S, g, lds); break;
      case FP32: ka_iter<FP32, 0, false, true>(a, S, g, lds); break;
      case FP8: ka_iter<FP8, 0, false, true>(a, S, g, lds); break;
      case TF32: ka_iter<TF32, 0, false, true>(a, S, g, lds); break;
      default: ka_iter<FP64, 0, false, true>(a, S, g, lds); break;
      }
    }
  } else if (EXT && mode == M_ITER && S.emul) {
    if constexpr (EXT) ka_iter<FP64, 1, true>(a, S, g, lds);
  } else if (EXT && mode == M_ITER && act_fs(S.action) == TF32) {
    if constexpr (EXT) {
      if (S.tier) ka_iter<TF32, 1>(a, S, g, lds);
      else ka_iter<TF32, 0>(a, S, g, lds);
    }
  } else if (mode == M_ITER) {
    const int fs = act_fs(S.action);   // 4: q52 storage
    switch (fs * 2 + S.tier) {
    case 8: ka_iter<FP8, 0>(a, S, g, lds); break;
    case 9: ka_iter<FP8, 1>(a, S, g, lds); break;
    case 0: ka_iter<FP16, 0>(a, S, g, lds); break;
    case 1: ka_iter<FP16, 1>(a, S, g, lds); break;
    case 2: ka_iter<BF16, 0>(a, S, g, lds); break;
    case 3: ka_iter<BF16, 1>(a, S, g, lds); break;
    case 4: ka_iter<FP32, 0>(a, S, g, lds); break;
    case 5: ka_iter<FP32, 1>(a, S, g, lds); break;
    case 6: ka_iter<FP64, 0>(a, S, g, lds); break;
    default: ka_iter<FP64, 1>(a, S, g, lds); break;
    }
  } else if (mode == M_INIT || mode == M_REPLACE || mode == M_FINAL) {
    ka_residual(a, S, g, mode, lds);
  }
}

// Kernels launched from part 4, defined in the other parts.
__global__ __launch_bounds__(kBlock, 2) void k_batched(const BatchSys *sys, const int32_t *order, int nsys,
                                                     int32_t *queue);
__global__ __launch_bounds__(kBlock) void k_a_lock(const BatchSys *sys, const SysBlk *tab, int ntab, int nround);
__global__ __launch_bounds__(kBlock) void k_b_lock(const BatchSys *sys, const SysBlk *tab, int ntab);
__global__ __launch_bounds__(kBlock) void k_x_lock(const BatchSys *sys, const SysBlk *tab, int ntab);
__global__ __launch_bounds__(kBlock) void k_step_b_lock(const BatchSys *sys, const int32_t *act);
__global__ __launch_bounds__(kBlock) void k_step_x_lock(const BatchSys *sys, const int32_t *act);
__global__ __launch_bounds__(kBlock) void k_start_lock(const BatchSys *sys, const SysBlk *tab);
__global__ __launch_bounds__(kBlock) void k_finish_lock(const BatchSys *sys, const SysBlk *tab);
__global__ __launch_bounds__(kBlock) void k_modes_lock(const BatchSys *sys, const int32_t *act, int nact,
                                                       int32_t *modes);

__global__ __launch_bounds__(kBlock) void k_a(KArgs a);
__global__ __launch_bounds__(kBlock) void k_a_ext(KArgs a);
__global__ __launch_bounds__(kBlock) void k_a16(KArgs a);
__global__ __launch_bounds__(kBlock) void k_b_ext(KArgs a);
__global__ __launch_bounds__(kBlock) void k_b_full_ext(KArgs a);
__global__ __launch_bounds__(kBlock) void k_b(KArgs a);
__global__ __launch_bounds__(kBlock) void k_b16(KArgs a);
__global__ __launch_bounds__(kBlock) void k_b_full(KArgs a);
__global__ __launch_bounds__(kBlock) void k_b_full16(KArgs a);
__global__ __launch_bounds__(kBlock) void k_b_pc(KArgs a);
__global__ __launch_bounds__(kBlock) void k_b_full_pc(KArgs a);
__global__ __launch_bounds__(kBlock) void k_b_r64(KArgs a);
__global__ __launch_bounds__(kBlock) void k_b_full_r64(KArgs a);
__global__ __launch_bounds__(kBlock) void k_b_pc_r64(KArgs a);
__global__ __launch_bounds__(kBlock) void k_b_full_pc_r64(KArgs a);

#if MPCG_IN_PART(1)
__global__ __launch_bounds__(kBlock) void k_a(KArgs a) {
  const int g = xcd_group(a.G1);
  if (g >= a.P1) return;
  __shared__ double lds[kLdsKa];
  ka_body<false, false>(a, g, lds);
}
#endif  // part 1

#if MPCG_IN_PART(7)
// the tf32 / emulation variant and the bf16-vector variant
__global__ __launch_bounds__(kBlock) void k_a_ext(KArgs a) {
  const int g = xcd_group(a.G1);
  if (g >= a.P1) return;
  __shared__ double lds[kLdsKa];
  ka_body<false, true>(a, g, lds);
}

__global__ __launch_bounds__(kBlock) void k_a16(KArgs a) {
  const int g = xcd_group(a.G1);
  if (g >= a.P1) return;
  __shared__ double lds[kLdsKa];
  ka_body<true, true>(a, g, lds);
}
#endif  // part 7

// ---------------------------------------------------------------------------
// KB: x_lo = axpy(alpha, p, x_lo), r = axpy(-alpha, q, r), partial of
// sigma' = dot(r, r); when the next iteration number is a multiple of the
// replacement period, x_lo is also folded into x_hi here (the replacement that
// follows begins with that fold).
// ---------------------------------------------------------------------------
template <typename V>
__device__ __forceinline__ void load8_tail(const V *p, int base, int n, bool full, V (&v)[8]) {
  if (full) {
    load8(p + base, v);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = base + j < n ? p[base + j] : (V)0;
  }
}

// x_lo and r updates and the sigma' partial on operands already loaded; with
// a preconditioner (PC) also z = M^-1 r and the partial of r.z.  With R64 the
// r.r partial (rho) is taken in fp64 and sigma' (r.r, or r.z with PC) at the
// dot format goes to the second partial.
template <int FA, int FD, bool PC, bool R64, bool EXT, typename V>
__device__ __forceinline__ void kb_axpy_vals(const KArgs &a, const Ctl &S, bool fold_now, int blk, const V (&pv)[8],
                                             const V (&qv)[8], V (&rv)[8], V (&xv)[8]) {
  constexpr int TIER = (FA == FP64);
  static_assert(sizeof(V) == sizeof(typename TierT<TIER>::type), "operands in the tier of fa");
  using Acc = typename AccT<FD>::type;
  constexpr int FR = R64 ? FP64 : FD;
  using AccR = typename AccT<FR>::type;
  V *xlo, *r;
  if constexpr (TIER) { xlo = a.v.xlo64; r = a.v.r64; }
  else { xlo = a.v.xlo32; r = a.v.r32; }
  const double alpha = S.alpha;
  const int n = a.A.n;
  const int base = blk * kVecBlock + threadIdx.x * kVecPer;
  const bool full = base + 8 <= n;
  AccR l[8];
  Acc lz[8];
  float mv[8];
  if constexpr (PC) load8_tail(a.A.minv, base, n, full, mv);
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    xv[j] = axpy1<FA>(alpha, pv[j], xv[j]);
    rv[j] = axpy1<FA>(-alpha, qv[j], rv[j]);
    if constexpr (FA == FP64 && EXT) {
      if (S.emul) {   // emulation: each fp64 update rounded to the update format
        xv[j] = rd_rt_f64(act_fa(S.action), xv[j]);
        rv[j] = rd_rt_f64(act_fa(S.action), rv[j]);
      }
    }
    l[j] = (full || base + j < n) ? dot_leaf<FR>(rv[j], rv[j]) : (AccR)0;
    if constexpr (PC) {
      V zj = precond_z<FA>(mv[j], rv[j]);
      if constexpr (FA == FP64 && EXT) {
        if (S.emul) zj = rd_rt_f64(act_fa(S.action), zj);
      }
      lz[j] = (full || base + j < n) ? dot_leaf<FD>(rv[j], zj) : (Acc)0;
    }
    else if constexpr (R64) lz[j] = (full || base + j < n) ? dot_leaf<FD>(rv[j], rv[j]) : (Acc)0;
  }
  if (fold_now) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = base + j;
      if (i < n) fold1(a.v.xhi, i, (double)xv[j]);
      xv[j] = (V)0;
    }
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
  const AccR t = block_tree(tree8(l));
  if (threadIdx.x == 0) a.part2[blk] = (double)t;
  if constexpr (PC || R64) {
    const Acc tz = block_tree(tree8(lz));
    if (threadIdx.x == 0) a.part2b[blk] = (double)tz;
  }
}

template <int FA, int FD, bool PC, bool R64, bool EXT = true>
__device__ __forceinline__ void kb_axpy(const KArgs &a, const Ctl &S, bool fold_now, int blk) {
  constexpr int TIER = (FA == FP64);
  using V = typename TierT<TIER>::type;
  const V *p, *q, *r, *xlo;
  if constexpr (TIER) { xlo = a.v.xlo64; r = a.v.r64; p = a.v.p64; q = a.v.q64; }
  else { xlo = a.v.xlo32; r = a.v.r32; p = a.v.p32; q = a.v.q32; }
  const int n = a.A.n;
  const int base = blk * kVecBlock + threadIdx.x * kVecPer;
  const bool full = base + 8 <= n;
  V pv[8], qv[8], rv[8], xv[8];
  load8_tail(p, base, n, full, pv);
  load8_tail(q, base, n, full, qv);
  load8_tail(r, base, n, full, rv);
  load8_tail(xlo, base, n, full, xv);
  kb_axpy_vals<FA, FD, PC, R64, EXT>(a, S, fold_now, blk, pv, qv, rv, xv);
}

// Elementwise steps (KB or KX): p = r = rd_tier(r64) after a start; the
// direction update, with a tier change when the next action needs one; the
// fold of x_lo into x_hi before a replacement or a restart.  With a
// preconditioner (PC) the direction takes z = M^-1 r in place of r (p_0 = z_0;
// p = z when the direction restarts).
// V16: also the bf16 containers (tier 2; no preconditioner there).
template <bool PC = false, bool V16 = false, bool EXT = true>
__device__ __forceinline__ void exec_elementwise(const KArgs &a, const Ctl &S, int blk) {
  [[maybe_unused]] const bool emul = EXT && S.emul;   // the emulation reading: EXT kernels only
  const int op = S.k3op;
  const int n = a.A.n;
  const int base = blk * kVecBlock + threadIdx.x * kVecPer;
  if (op == K3_FOLD) {
    fold_group(a, S.tier, blk);
  } else if (V16 && op == K3_COPY && S.tier == 2) {   // r = p = rd_bf16(r64), x_lo = 0
    for (int j = 0; j < 8; ++j) {
      const int i = base + j;
      if (i >= n) break;
      const uint16_t rb = bf16_bits_of(a.v.r64[i]);
      a.v.r16[i] = rb;
      a.v.p16[i] = rb;
      a.v.x16[i] = 0;
    }
  } else if (V16 && op == K3_XPAY && !S.k3switch && base + 8 <= n && S.tier_old == 2) {
    float pv[8], rv[8];
    load8_bf16(a.v.p16 + base, pv);
    load8_bf16(a.v.r16 + base, rv);
    const int fa = S.k3_fa;
    const float bf = (float)S.beta;
#pragma unroll
    for (int j = 0; j < 8; ++j) pv[j] = rd_rt_f32(fa, __builtin_fmaf(bf, pv[j], rv[j]));
    store8_bf16(a.v.p16 + base, pv);
  } else if (V16 && op == K3_XPAY) {
    // any pair of containers: the direction update in the old tier, then (on
    // a tier change) the fold of x_lo and r, p rounded into the new tier
    const int told = S.tier_old, nt = S.tier;
    for (int j = 0; j < 8; ++j) {
      const int i = base + j;
      if (i >= n) break;
      double pn, rold, xold;
      if (told == 1) {
        pn = xpay_rt<double>(S.k3_fa, S.beta, a.v.p64[i], a.v.r64[i]);
        rold = a.v.r64[i];
        xold = a.v.xlo64[i];
      } else {
        const float pp = told == 2 ? bf16_bits_to_f32(a.v.p16[i]) : a.v.p32[i];
        const float rr = told == 2 ? bf16_bits_to_f32(a.v.r16[i]) : a.v.r32[i];
        pn = (double)xpay_rt<float>(S.k3_fa, S.beta, pp, rr);
        rold = (double)rr;
        xold = told == 2 ? (double)bf16_bits_to_f32(a.v.x16[i]) : (double)a.v.xlo32[i];
      }
      const int to = S.k3switch ? nt : told;
      if (S.k3switch) fold1(a.v.xhi, i, xold);
      if (to == 1) {
        a.v.p64[i] = pn;
        if (S.k3switch) { a.v.r64[i] = rold; a.v.xlo64[i] = 0.0; }
      } else if (to == 2) {
        a.v.p16[i] = bf16_bits_of(pn);
        if (S.k3switch) { a.v.r16[i] = bf16_bits_of(rold); a.v.x16[i] = 0; }
      } else {
        a.v.p32[i] = (float)pn;
        if (S.k3switch) { a.v.r32[i] = (float)rold; a.v.xlo32[i] = 0.0f; }
      }
    }
  } else if (op == K3_COPY) {
    for (int j = 0; j < 8; ++j) {
      const int i = base + j;
      if (i >= n) break;
      const double r = a.v.r64[i];
      if (S.tier) {
        if constexpr (EXT) {
          a.v.p64[i] = PC ? (emul ? rd_rt_f64(act_fa(S.action), precond_z_rt(FP64, a.A.minv[i], r))
                                  : precond_z_rt(FP64, a.A.minv[i], r))
                          : r;
        } else {
          a.v.p64[i] = PC ? precond_z_rt(FP64, a.A.minv[i], r) : r;
        }
        a.v.xlo64[i] = 0.0;
      } else {
        const float f = (float)r;
        a.v.r32[i] = f;
        a.v.p32[i] = PC ? precond_z_rt(act_fa(S.action), a.A.minv[i], f) : f;
        a.v.xlo32[i] = 0.0f;
      }
    }
  } else if (op == K3_XPAY && !S.k3switch && base + 8 <= n) {   // the common case, vectorised
    float mv[8];
    if constexpr (PC) load8(a.A.minv + base, mv);
    if (S.tier_old) {
      double pv[8], rv[8];
      load8(a.v.p64 + base, pv);
      load8(a.v.r64 + base, rv);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if constexpr (PC) {
          double z = precond_z_rt(FP64, mv[j], rv[j]);
          if constexpr (EXT) {
            if (emul) z = rd_rt_f64(S.k3_fa, z);
          }
          pv[j] = S.dir_restart ? z : xpay_rt<double>(S.k3_fa, S.beta, pv[j], z);
        } else {
          pv[j] = xpay_rt<double>(S.k3_fa, S.beta, pv[j], rv[j]);
        }
        if constexpr (EXT) {
          if (emul && !(PC && S.dir_restart)) pv[j] = rd_rt_f64(S.k3_fa, pv[j]);
        }
      }
      store8(a.v.p64 + base, pv);
    } else {
      float pv[8], rv[8];
      load8(a.v.p32 + base, pv);
      load8(a.v.r32 + base, rv);
      const int fa = S.k3_fa;
      const float bf = (float)S.beta;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if constexpr (PC) {
          const float z = precond_z_rt(fa, mv[j], rv[j]);
          const float t = __builtin_fmaf(bf, pv[j], z);
          pv[j] = S.dir_restart ? z : rd_rt_f32(fa, t);
        } else {
          const float t = __builtin_fmaf(bf, pv[j], rv[j]);
          pv[j] = rd_rt_f32(fa, t);
        }
      }
      store8(a.v.p32 + base, pv);
    }
  } else if (op == K3_XPAY) {
    const int told = S.tier_old;
    for (int j = 0; j < 8; ++j) {
      const int i = base + j;
      if (i >= n) break;
      if (told) {
        double pn;
        if constexpr (PC) {
          double z = precond_z_rt(FP64, a.A.minv[i], a.v.r64[i]);
          if constexpr (EXT) {
            if (emul) z = rd_rt_f64(S.k3_fa, z);
          }
          pn = S.dir_restart ? z : xpay_rt<double>(S.k3_fa, S.beta, a.v.p64[i], z);
        } else {
          pn = xpay_rt<double>(S.k3_fa, S.beta, a.v.p64[i], a.v.r64[i]);
        }
        if constexpr (EXT) {
          if (emul && !(PC && S.dir_restart)) pn = rd_rt_f64(S.k3_fa, pn);
        }
        if (S.k3switch) {
          fold1(a.v.xhi, i, a.v.xlo64[i]);
          a.v.p32[i] = (float)pn;
          a.v.r32[i] = (float)a.v.r64[i];
          a.v.xlo32[i] = 0.0f;
        } else {
          a.v.p64[i] = pn;
        }
      } else {
        float pn;
        if constexpr (PC) {
          const float z = precond_z_rt(S.k3_fa, a.A.minv[i], a.v.r32[i]);
          pn = S.dir_restart ? z : xpay_rt<float>(S.k3_fa, S.beta, a.v.p32[i], z);
        } else {
          pn = xpay_rt<float>(S.k3_fa, S.beta, a.v.p32[i], a.v.r32[i]);
        }
        if (S.k3switch) {
          fold1(a.v.xhi, i, (double)a.v.xlo32[i]);
          a.v.p64[i] = (double)pn;
          a.v.r64[i] = (double)a.v.r32[i];
          a.v.xlo64[i] = 0.0;
        } else {
          a.v.p32[i] = pn;
        }
      }
    }
  }
}

#define MPCG_KB_CASE(FA, FD) \
  case (FA) * 8 + (FD): kb_axpy<FA, FD, PC, R64, EXT>(a, S, fold_now, blk); break;
#define MPCG_KB_VALS(FA, FD) \
  case (FA) * 8 + (FD): kb_axpy_vals<FA, FD, PC, R64, EXT>(a, S, fold_now, blk, pv, qv, rv, xv); break;

// KB's vector work for 2048-element block blk.
// x_lo and r updates with bf16 updates in the bf16 containers (16-bit vector
// storage), and the sigma' partial: the arithmetic of the fp32-container path.
template <int FD>
__device__ __forceinline__ void kb_axpy16(const KArgs &a, const Ctl &S, bool fold_now, int blk) {
  using Acc = typename AccT<FD>::type;
  const int n = a.A.n;
  const int base = blk * kVecBlock + threadIdx.x * kVecPer;
  const bool full = base + 8 <= n;
  float pv[8], qv[8], rv[8], xv[8];
  if (full) {
    load8_bf16(a.v.p16 + base, pv);
    load8(a.v.q32 + base, qv);
    load8_bf16(a.v.r16 + base, rv);
    load8_bf16(a.v.x16 + base, xv);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = base + j;
      const bool in = i < n;
      pv[j] = in ? bf16_bits_to_f32(a.v.p16[i]) : 0.0f;
      qv[j] = in ? a.v.q32[i] : 0.0f;
      rv[j] = in ? bf16_bits_to_f32(a.v.r16[i]) : 0.0f;
      xv[j] = in ? bf16_bits_to_f32(a.v.x16[i]) : 0.0f;
    }
  }
  const double alpha = S.alpha;
  Acc l[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    xv[j] = axpy1<BF16>(alpha, pv[j], xv[j]);
    rv[j] = axpy1<BF16>(-alpha, qv[j], rv[j]);
    l[j] = (full || base + j < n) ? dot_leaf<FD>(rv[j], rv[j]) : (Acc)0;
  }
  if (fold_now) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = base + j;
      if (i < n) fold1(a.v.xhi, i, (double)xv[j]);
      xv[j] = 0.0f;
    }
  }
  if (full) {
    store8_bf16(a.v.x16 + base, xv);
    store8_bf16(a.v.r16 + base, rv);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = base + j;
      if (i < n) {
        a.v.x16[i] = f32_to_bf16_bits_exact(xv[j]);
        a.v.r16[i] = f32_to_bf16_bits_exact(rv[j]);
      }
    }
  }
  const Acc t = block_tree(tree8(l));
  if (threadIdx.x == 0) a.part2[blk] = (double)t;
}

template <bool PC = false, bool R64 = false, bool V16 = false, bool EXT = true>
__device__ __forceinline__ void kb_work(const KArgs &a, const Ctl &S, int bop, bool fold_now, int blk) {
  if (V16 && bop == B_AXPY && S.tier == 2) {
    if constexpr (V16) {
      switch (act_fd(S.action)) {
      case FP16: kb_axpy16<FP16>(a, S, fold_now, blk); break;
      case BF16: kb_axpy16<BF16>(a, S, fold_now, blk); break;
      case FP32: kb_axpy16<FP32>(a, S, fold_now, blk); break;
      case TF32: kb_axpy16<TF32>(a, S, fold_now, blk); break;
      default: kb_axpy16<FP64>(a, S, fold_now, blk); break;
      }
    }
  } else if (bop == B_AXPY) {
    const int act = S.action;
    const int key = (EXT && S.emul) ? FP64 * 8 + FP64 : act_fa(act) * 8 + act_fd(act);
    if (EXT && (act_fa(act) == TF32 || act_fd(act) == TF32) && !S.emul) {
      if constexpr (EXT) {
        switch (key) {
          MPCG_KB_CASE(FP16, TF32) MPCG_KB_CASE(BF16, TF32) MPCG_KB_CASE(FP32, TF32) MPCG_KB_CASE(FP64, TF32)
          MPCG_KB_CASE(TF32, FP16) MPCG_KB_CASE(TF32, BF16) MPCG_KB_CASE(TF32, FP32) MPCG_KB_CASE(TF32, FP64)
          MPCG_KB_CASE(TF32, TF32)
        default: break;
        }
      }
    } else {
      switch (key) {
        MPCG_KB_CASE(FP16, FP16) MPCG_KB_CASE(FP16, BF16) MPCG_KB_CASE(FP16, FP32) MPCG_KB_CASE(FP16, FP64)
        MPCG_KB_CASE(BF16, FP16) MPCG_KB_CASE(BF16, BF16) MPCG_KB_CASE(BF16, FP32) MPCG_KB_CASE(BF16, FP64)
        MPCG_KB_CASE(FP32, FP16) MPCG_KB_CASE(FP32, BF16) MPCG_KB_CASE(FP32, FP32) MPCG_KB_CASE(FP32, FP64)
        MPCG_KB_CASE(FP64, FP16) MPCG_KB_CASE(FP64, BF16) MPCG_KB_CASE(FP64, FP32) MPCG_KB_CASE(FP64, FP64)
      default: break;
      }
    }
  } else if (bop == B_EXEC) {
    exec_elementwise<PC, V16, EXT>(a, S, blk);
  }
}

// Control-block bookkeeping at the end of KB's work.
__device__ __forceinline__ void kb_commit(Ctl &S, int bop, bool fold_now) {
  if (bop == B_AXPY) {
    S.pend_sigma = 1;
    S.fold_done = fold_now ? 1 : 0;
  } else if (bop == B_EXEC) {
    S.k3op = K3_NONE;
  }
  S.b_op = B_NONE;
  S.step_done = 0;
}

// KB's work on vector block blk of one system; block 0 commits the state.
// The step's partials are loaded together with the control block.
template <bool FULL = false, bool PC = false, bool R64 = false, bool V16 = false, bool EXT = true>
__device__ __forceinline__ void kb_body(const KArgs &a, int blk) {
  __shared__ Ctl S;
  __shared__ PolicyDev SP;
  double pre[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const bool fast = a.P1 <= kVecBlock;
  if (fast) preload_partials(a.part1, a.P1, pre);
  copy_words(&S, &a.ctl[0], sizeof(Ctl));
  copy_words(&SP, a.pol, sizeof(PolicyDev));
  __syncthreads();
  const Sx x{&S, &SP, a.h, blk == 0};
  const int base = blk * kVecBlock + threadIdx.x * kVecPer;
  const bool blk_full = (blk + 1) * kVecBlock <= a.A.n;   // block-uniform
  if (!S.step_done && S.mode == M_ITER && !(EXT && S.emul) && S.tier == 0 && act_fa(S.action) != FP64 && blk_full) {
    // an iteration in the fp32 containers on a whole block: the four operands
    // are in flight while the alpha step runs
    float pv[8], qv[8], rv[8], xv[8];
    __builtin_amdgcn_sched_barrier(0);
    load8(a.v.p32 + base, pv);
    load8(a.v.q32 + base, qv);
    load8(a.v.r32 + base, rv);
    load8(a.v.xlo32 + base, xv);
    __builtin_amdgcn_sched_barrier(0);
    step_b<FULL, EXT>(x, a, pre, fast);
    const int bop = S.b_op;
    const bool fold_now = (bop == B_AXPY) && S.R > 0 && (S.k + 1) % S.R == 0;
    if (bop == B_AXPY) {
      const int act = S.action;
      if (EXT && (act_fa(act) == TF32 || act_fd(act) == TF32)) {
        if constexpr (EXT) {
          switch (act_fa(act) * 8 + act_fd(act)) {
            MPCG_KB_VALS(FP16, TF32) MPCG_KB_VALS(BF16, TF32) MPCG_KB_VALS(FP32, TF32)
            MPCG_KB_VALS(TF32, FP16) MPCG_KB_VALS(TF32, BF16) MPCG_KB_VALS(TF32, FP32) MPCG_KB_VALS(TF32, FP64)
            MPCG_KB_VALS(TF32, TF32)
          default: break;
          }
        }
      } else {
        switch (act_fa(act) * 8 + act_fd(act)) {
          MPCG_KB_VALS(FP16, FP16) MPCG_KB_VALS(FP16, BF16) MPCG_KB_VALS(FP16, FP32) MPCG_KB_VALS(FP16, FP64)
          MPCG_KB_VALS(BF16, FP16) MPCG_KB_VALS(BF16, BF16) MPCG_KB_VALS(BF16, FP32) MPCG_KB_VALS(BF16, FP64)
          MPCG_KB_VALS(FP32, FP16) MPCG_KB_VALS(FP32, BF16) MPCG_KB_VALS(FP32, FP32) MPCG_KB_VALS(FP32, FP64)
        default: break;
        }
      }
    } else {
      kb_work<PC, R64, V16, EXT>(a, S, bop, fold_now, blk);
    }
    if (blk == 0) {
      __syncthreads();
      if (threadIdx.x == 0) kb_commit(S, bop, fold_now);
      __syncthreads();
      copy_words(&a.ctl[1], &S, sizeof(Ctl));
    }
    return;
  }
  if (!S.step_done) step_b<FULL, EXT>(x, a, pre, fast);
  const int bop = S.b_op;
  const bool fold_now = (bop == B_AXPY) && S.R > 0 && (S.k + 1) % S.R == 0;
  kb_work<PC, R64, V16, EXT>(a, S, bop, fold_now, blk);
  if (blk == 0) {   // commit the state after this kernel for KX
    __syncthreads();
    if (threadIdx.x == 0) kb_commit(S, bop, fold_now);
    __syncthreads();
    copy_words(&a.ctl[1], &S, sizeof(Ctl));
  }
}

// KX's work on vector block blk: end-of-iteration step, then the pending
// elementwise operation; block 0 commits the state.  The partials come with
// the control block, and the direction update's operands are issued before
// the step's arithmetic, so the step's latency overlaps the vector loads.
template <int TIER, bool PC, bool V16 = false, bool EXT = true>
__device__ __forceinline__ void kx_iter_pre(const KArgs &a, const Sx &x, Ctl &S, int blk, const double (&pre)[8],
                                            bool have_pre) {
  using V = typename TierT<TIER>::type;
  const int n = a.A.n;
  const int base = blk * kVecBlock + threadIdx.x * kVecPer;
  const bool full = base + 8 <= n;
  V pv[8], rv[8];
  float mv[8];
  __builtin_amdgcn_sched_barrier(0);
  if (full) {
    if constexpr (TIER) { load8(a.v.p64 + base, pv); load8(a.v.r64 + base, rv); }
    else { load8(a.v.p32 + base, pv); load8(a.v.r32 + base, rv); }
    if constexpr (PC) load8(a.A.minv + base, mv);
  }
  __builtin_amdgcn_sched_barrier(0);
  step_x<false, EXT>(x, a, pre, have_pre);
  if (S.k3op == K3_XPAY && !S.k3switch && full) {
    if constexpr (TIER) {
      const double beta = S.beta;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if constexpr (PC) {
          double z = precond_z<FP64>(mv[j], rv[j]);
          if constexpr (EXT) {
            if (S.emul) z = rd_rt_f64(S.k3_fa, z);
          }
          pv[j] = S.dir_restart ? z : __builtin_fma(beta, pv[j], z);
        } else {
          pv[j] = __builtin_fma(beta, pv[j], rv[j]);
        }
        if constexpr (EXT) {
          if (S.emul && !(PC && S.dir_restart)) pv[j] = rd_rt_f64(S.k3_fa, pv[j]);
        }
      }
      store8(a.v.p64 + base, pv);
    } else {
      const int fa = S.k3_fa;
      const float bf = (float)S.beta;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if constexpr (PC) {
          const float z = precond_z_rt(fa, mv[j], rv[j]);
          const float t = __builtin_fmaf(bf, pv[j], z);
          pv[j] = S.dir_restart ? z : rd_rt_f32(fa, t);
        } else {
          const float t = __builtin_fmaf(bf, pv[j], rv[j]);
          pv[j] = rd_rt_f32(fa, t);
        }
      }
      store8(a.v.p32 + base, pv);
    }
  } else {
    exec_elementwise<PC, V16, EXT>(a, S, blk);
  }
}

// KX's work on a block whose r and p are in the bf16 containers (tier 2):
// the step, then the direction update on the operands already loaded.
__device__ __forceinline__ void kx_iter16(const KArgs &a, const Sx &x, Ctl &S, int blk, const double (&pre)[8],
                                          bool have_pre) {
  const int n = a.A.n;
  const int base = blk * kVecBlock + threadIdx.x * kVecPer;
  const bool full = base + 8 <= n;
  float pv[8], rv[8];
  __builtin_amdgcn_sched_barrier(0);
  if (full) {
    load8_bf16(a.v.p16 + base, pv);
    load8_bf16(a.v.r16 + base, rv);
  }
  __builtin_amdgcn_sched_barrier(0);
  step_x<false>(x, a, pre, have_pre);
  if (S.k3op == K3_XPAY && !S.k3switch && full) {
    const int fa = S.k3_fa;
    const float bf = (float)S.beta;
#pragma unroll
    for (int j = 0; j < 8; ++j) pv[j] = rd_rt_f32(fa, __builtin_fmaf(bf, pv[j], rv[j]));
    store8_bf16(a.v.p16 + base, pv);
  } else {
    exec_elementwise<false, true>(a, S, blk);
  }
}

template <bool PC = false, bool V16 = false, bool EXT = true>
__device__ __forceinline__ void kx_body(const KArgs &a, int blk) {
  __shared__ Ctl S;
  __shared__ PolicyDev SP;
  double pre[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const bool fast = a.P2 <= kVecBlock;
  if (fast) preload_partials(a.part2, a.P2, pre);
  copy_words(&S, &a.ctl[1], sizeof(Ctl));
  copy_words(&SP, a.pol, sizeof(PolicyDev));
  __syncthreads();
  const Sx x{&S, &SP, a.h, blk == 0, nullptr};
  if (!S.step_done && S.pend_sigma) {
    if (V16 && S.tier == 2) kx_iter16(a, x, S, blk, pre, fast);
    else if (S.tier) kx_iter_pre<1, PC, V16, EXT>(a, x, S, blk, pre, fast);
    else kx_iter_pre<0, PC, V16, EXT>(a, x, S, blk, pre, fast);
  } else {
    if (!S.step_done) step_x<false, EXT>(x, a, pre, fast);
    exec_elementwise<PC, V16, EXT>(a, S, blk);
  }
  if (blk == 0) {   // commit the state after this kernel for the next KA and KB
    __syncthreads();
    if (threadIdx.x == 0) {
      S.k3op = K3_NONE;
      S.step_done = 0;
    }
    __syncthreads();
    copy_words(&a.ctl[0], &S, sizeof(Ctl));
  }
}

#if MPCG_IN_PART(2)
__global__ __launch_bounds__(kBlock) void k_b(KArgs a) { kb_body<false, false, false, false, false>(a, blockIdx.x); }

// KB whose replicated step is the full one (state features, the network's
// decision at a start or a stop, rollout log by workgroup 0): for policies
// that read but never write shared policy state during a solve.  Their
// end-of-iteration decision runs once, in the one-block step kernel before KX.
__global__ __launch_bounds__(kBlock) void k_b_full(KArgs a) { kb_body<true, false, false, false, false>(a, blockIdx.x); }
#endif  // part 2

#if MPCG_IN_PART(8)
// The tf32 / emulation variants and the bf16 vector tier (16-bit vector storage).
__global__ __launch_bounds__(kBlock) void k_b_ext(KArgs a) { kb_body<false, false, false, false, true>(a, blockIdx.x); }
__global__ __launch_bounds__(kBlock) void k_b_full_ext(KArgs a) { kb_body<true, false, false, false, true>(a, blockIdx.x); }
__global__ __launch_bounds__(kBlock) void k_b16(KArgs a) { kb_body<false, false, false, true>(a, blockIdx.x); }
__global__ __launch_bounds__(kBlock) void k_b_full16(KArgs a) { kb_body<true, false, false, true>(a, blockIdx.x); }
#endif  // part 8

#if MPCG_IN_PART(3)
// The Jacobi-preconditioned variants of KB (separate kernels, so the
// unpreconditioned ones keep their register budget).
__global__ __launch_bounds__(kBlock) void k_b_pc(KArgs a) { kb_body<false, true>(a, blockIdx.x); }
__global__ __launch_bounds__(kBlock) void k_b_full_pc(KArgs a) { kb_body<true, true>(a, blockIdx.x); }
// KB with rho from an fp64 r.r (the residual norm kept in fp64) and sigma' at
// the dot format in the second partial.
__global__ __launch_bounds__(kBlock) void k_b_r64(KArgs a) { kb_body<false, false, true>(a, blockIdx.x); }
#endif  // part 3

#if MPCG_IN_PART(6)
__global__ __launch_bounds__(kBlock) void k_b_full_r64(KArgs a) { kb_body<true, false, true>(a, blockIdx.x); }
__global__ __launch_bounds__(kBlock) void k_b_pc_r64(KArgs a) { kb_body<false, true, true>(a, blockIdx.x); }
__global__ __launch_bounds__(kBlock) void k_b_full_pc_r64(KArgs a) { kb_body<true, true, true>(a, blockIdx.x); }
#endif  // part 6

#if MPCG_IN_PART(4) || MPCG_KPART == 5   // device steps shared with the batched kernels
#if MPCG_IN_PART(4)
__global__ __launch_bounds__(kBlock) void k_x(KArgs a) { kx_body<false, false, false>(a, blockIdx.x); }
__global__ __launch_bounds__(kBlock) void k_x_ext(KArgs a) { kx_body<false, false, true>(a, blockIdx.x); }
#endif
// the bf16 vector tier (16-bit vector storage) and the Jacobi-preconditioned KX
#if MPCG_IN_PART(4)
__global__ __launch_bounds__(kBlock) void k_x16(KArgs a) { kx_body<false, true>(a, blockIdx.x); }
#endif
#if MPCG_IN_PART(4)
__global__ __launch_bounds__(kBlock) void k_x_pc(KArgs a) { kx_body<true>(a, blockIdx.x); }
#endif
#undef MPCG_KB_CASE
#undef MPCG_KB_VALS

// One-block step kernels for policies whose step writes shared state or
// evaluates the network: the step runs once, then KA / KB skip theirs.
__device__ __forceinline__ void step_b_body(const KArgs &a) {
  __shared__ Ctl S;
  __shared__ PolicyDev SP;
  double pre[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const bool fast = a.P1 <= kVecBlock;
  if (fast) preload_partials(a.part1, a.P1, pre);
  copy_words(&S, &a.ctl[0], sizeof(Ctl));
  copy_words(&SP, a.pol, sizeof(PolicyDev));
  __syncthreads();
  const Sx x{&S, &SP, a.h, true, nullptr};
  step_b<true>(x, a, pre, fast);
  if (threadIdx.x == 0) S.step_done = 1;
  __syncthreads();
  copy_words(&a.ctl[0], &S, sizeof(Ctl));
}

// wl: LDS for the network weights (staged here, in the same round trip as the
// control block and the partials), or NULL.
__device__ __forceinline__ void step_x_body(const KArgs &a, float *wl = nullptr) {
  __shared__ Ctl S;
  __shared__ PolicyDev SP;
  NetRegs nr;
  if (wl) net_load(a.net, nr);
  double pre[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const bool fast = a.P2 <= kVecBlock;
  if (fast) preload_partials(a.part2, a.P2, pre);
  copy_words(&S, &a.ctl[1], sizeof(Ctl));
  copy_words(&SP, a.pol, sizeof(PolicyDev));
  if (wl) net_store(nr, wl);
  __syncthreads();
  const Sx x{&S, &SP, a.h, true, wl};
  step_x<true>(x, a, pre, fast);
  if (threadIdx.x == 0) S.step_done = 1;
  __syncthreads();
  copy_words(&a.ctl[1], &S, sizeof(Ctl));
}

#if MPCG_IN_PART(4)
__global__ __launch_bounds__(kBlock) void k_step_b(KArgs a) { step_b_body(a); }
#endif

#if MPCG_IN_PART(4)
__global__ __launch_bounds__(kBlock) void k_step_x(KArgs a) { step_x_body(a); }
#endif

// The one-block step of a network policy, with the weights staged in LDS.
#if MPCG_IN_PART(4)
__global__ __launch_bounds__(kBlock) void k_step_x_net(KArgs a) {
  __shared__ float wl[kNetLds];
  step_x_body(a, wl);
}
#endif

// ---------------------------------------------------------------------------
// start / finish
// ---------------------------------------------------------------------------
// x_hi = x0, x_lo = 0, partials of b.b (pairwise fp64) for ||b|| (block blk).
__device__ __forceinline__ void start_block(const KArgs &a, int blk) {
  const int n = a.A.n;
  const int base = blk * kVecBlock + threadIdx.x * kVecPer;
  double l[8];
  for (int j = 0; j < 8; ++j) {
    const int i = base + j;
    if (i < n) {
      a.v.xhi[i] = a.v.xout[i];
      a.v.xlo32[i] = 0.0f;
      a.v.xlo64[i] = 0.0;
      if (a.v.x16) a.v.x16[i] = 0;
      const double bi = a.v.b[i];
      l[j] = bi * bi;
    } else {
      l[j] = 0.0;
    }
  }
  const double t = block_tree(tree8(l));
  if (threadIdx.x == 0) a.part0[blk] = t;
}

#if MPCG_IN_PART(4)
__global__ __launch_bounds__(kBlock) void k_start(KArgs a) { start_block(a, blockIdx.x); }
#endif

// x = x_hi + x_lo over block blk (tier and zero-solution flag of the final state).
__device__ __forceinline__ void finish_block_x(const KArgs &a, int tier, int zero, int blk) {
  const int n = a.A.n;
  const int base = blk * kVecBlock + threadIdx.x * kVecPer;
  for (int j = 0; j < 8; ++j) {
    const int i = base + j;
    if (i >= n) break;
    if (tier == 1) { fold1(a.v.xhi, i, a.v.xlo64[i]); a.v.xlo64[i] = 0.0; }
    else if (tier == 2) { fold1(a.v.xhi, i, (double)bf16_bits_to_f32(a.v.x16[i])); a.v.x16[i] = 0; }
    else { fold1(a.v.xhi, i, (double)a.v.xlo32[i]); a.v.xlo32[i] = 0.0f; }
    a.v.xout[i] = zero ? 0.0 : a.v.xhi[i];
  }
}

// Requests the final true-residual check after a budget stop or a breakdown.
__device__ __forceinline__ void request_final(Ctl *c) {
  // a budget stop, a breakdown, or a convergence on the recursive residual
  // (stop_rule 1) gets the true residual of the final x
  if (c->status == 1 || c->status == 3 || (c->stop_rule == 1 && !c->zero_solution && c->k > 0 &&
                                           (c->status == 0 || c->status == 2))) {
    c->mode = M_FINAL;
    c->k3op = K3_NONE;
    c->pend_sigma = 0;
    c->step_done = 0;
  }
}

// x = x_hi + x_lo; requests the final true-residual check after a budget stop
// or a breakdown.
#if MPCG_IN_PART(4)
__global__ __launch_bounds__(kBlock) void k_finish(KArgs a) {
  const Ctl *c = &a.ctl[0];
  finish_block_x(a, c->tier, c->zero_solution, blockIdx.x);
  if (blockIdx.x == 0 && threadIdx.x == 0) request_final(&a.ctl[0]);
}
#endif

#endif  // parts 4, 5

#if MPCG_IN_PART(5)
// ---------------------------------------------------------------------------
// Batched persistent solve: each workgroup takes whole systems from a queue
// (an atomic counter over a host-given order) and runs the same slot program as
// the three-kernel path -- SpMV pass, alpha step and axpy pass, beta/policy step
// and direction-update pass -- over all of the system's row groups and vector
// blocks, with workgroup barriers in place of kernel boundaries.  Every
// operation, reduction tree and step is the one of the single-system path, so
// each system's result is bit-identical to its own mpcg_solve.  The slot loop
// of a system is bounded (max_slots), and a workgroup leaves when the queue is
// empty, so every wave exits.
// ---------------------------------------------------------------------------
template <int FS, int TIER>
__device__ __forceinline__ void ka_iter_all(const KArgs &a, const Ctl &S, void *lds) {
  for (int g = 0; g < a.P1; ++g) {
    ka_iter<FS, TIER>(a, S, g, lds);
    __syncthreads();
  }
}

__device__ __forceinline__ void ka_pass(const KArgs &a, const Ctl &S, void *lds) {
  const int mode = S.mode;
  if (mode == M_ITER) {
    const int fs = (S.action >> 4) & 7;
    switch (fs * 2 + S.tier) {
    case 8: ka_iter_all<FP8, 0>(a, S, lds); break;
    case 9: ka_iter_all<FP8, 1>(a, S, lds); break;
    case 0: ka_iter_all<FP16, 0>(a, S, lds); break;
    case 1: ka_iter_all<FP16, 1>(a, S, lds); break;
    case 2: ka_iter_all<BF16, 0>(a, S, lds); break;
    case 3: ka_iter_all<BF16, 1>(a, S, lds); break;
    case 4: ka_iter_all<FP32, 0>(a, S, lds); break;
    case 5: ka_iter_all<FP32, 1>(a, S, lds); break;
    case 6: ka_iter_all<FP64, 0>(a, S, lds); break;
    default: ka_iter_all<FP64, 1>(a, S, lds); break;
    }
  } else if (mode == M_INIT || mode == M_REPLACE || mode == M_FINAL) {
    for (int g = 0; g < a.P1; ++g) {
      ka_residual(a, S, g, mode, lds);
      __syncthreads();
    }
  }
}

template <int FA, int FD>
__device__ __forceinline__ void kb_axpy_all(const KArgs &a, const Ctl &S, bool fold_now) {
  for (int blk = 0; blk < a.P2; ++blk) kb_axpy<FA, FD, false, false, false>(a, S, fold_now, blk);
}

#define MPCG_KB_ALL(FA, FD) \
  case (FA) * 4 + (FD): kb_axpy_all<FA, FD>(a, S, fold_now); break;

__device__ __forceinline__ void kb_pass(const KArgs &a, const Ctl &S, int bop, bool fold_now) {
  if (bop == B_AXPY) {
    const int act = S.action;
    switch ((act & 3) * 4 + ((act >> 2) & 3)) {
      MPCG_KB_ALL(FP16, FP16) MPCG_KB_ALL(FP16, BF16) MPCG_KB_ALL(FP16, FP32) MPCG_KB_ALL(FP16, FP64)
      MPCG_KB_ALL(BF16, FP16) MPCG_KB_ALL(BF16, BF16) MPCG_KB_ALL(BF16, FP32) MPCG_KB_ALL(BF16, FP64)
      MPCG_KB_ALL(FP32, FP16) MPCG_KB_ALL(FP32, BF16) MPCG_KB_ALL(FP32, FP32) MPCG_KB_ALL(FP32, FP64)
      MPCG_KB_ALL(FP64, FP16) MPCG_KB_ALL(FP64, BF16) MPCG_KB_ALL(FP64, FP32) MPCG_KB_ALL(FP64, FP64)
    default: break;
    }
  } else if (bop == B_EXEC) {
    for (int blk = 0; blk < a.P2; ++blk) exec_elementwise(a, S, blk);
  }
}
#undef MPCG_KB_ALL

__global__ __launch_bounds__(kBlock, 2) void k_batched(const BatchSys *sys, const int32_t *order, int nsys,
                                                     int32_t *queue) {
  __shared__ Ctl S;
  __shared__ PolicyDev SP;
  __shared__ double lds[kLdsKa];
  __shared__ int s_idx;
  while (true) {
    if (threadIdx.x == 0) s_idx = __hip_atomic_fetch_add(queue, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int qi = __builtin_amdgcn_readfirstlane(s_idx);
    __syncthreads();
    if (qi >= nsys) break;
    const int si = __builtin_amdgcn_readfirstlane(order[qi]);
    const KArgs &a = sys[si].a;
    const int max_slots = sys[si].max_slots;
    copy_words(&SP, a.pol, sizeof(PolicyDev));
    copy_words(&S, &a.ctl[0], sizeof(Ctl));
    __syncthreads();
    const Sx x{&S, &SP, a.h, true, nullptr};
    for (int blk = 0; blk < a.P2; ++blk) start_block(a, blk);
    __syncthreads();
    int slots = 0;
    while (S.mode != M_DONE && slots < max_slots) {
      ++slots;
      ka_pass(a, S, lds);
      step_b<true>(x, a);
      const int bop = S.b_op;
      const bool fold_now = (bop == B_AXPY) && S.R > 0 && (S.k + 1) % S.R == 0;
      kb_pass(a, S, bop, fold_now);
      __syncthreads();
      if (threadIdx.x == 0) kb_commit(S, bop, fold_now);
      __syncthreads();
      step_x<true>(x, a);
      for (int blk = 0; blk < a.P2; ++blk) exec_elementwise(a, S, blk);
      __syncthreads();
      if (threadIdx.x == 0) {
        S.k3op = K3_NONE;
        S.step_done = 0;
      }
      __syncthreads();
    }
    const bool finished = S.mode == M_DONE;
    for (int blk = 0; blk < a.P2; ++blk) finish_block_x(a, S.tier, S.zero_solution, blk);
    __syncthreads();
    if (threadIdx.x == 0 && finished) request_final(&S);
    __syncthreads();
    if (S.mode == M_FINAL) {
      ka_pass(a, S, lds);
      step_b<true>(x, a);
    }
    __syncthreads();
    if (threadIdx.x == 0 && !finished) S.status = -1;   // slot budget exhausted (not expected)
    __syncthreads();
    copy_words(&a.ctl[1], &S, sizeof(Ctl));
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Batched lockstep: the three kernels of an iteration over the row groups or
// vector blocks of many systems at once.  Entry t of a table names (system,
// group or block); each workgroup runs the single-system body on it, so every
// system computes exactly what its own solve computes.  Systems that are done
// return at once; the host drops them from the tables as it learns of them.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_a_lock(const BatchSys *sys, const SysBlk *tab, int ntab, int nround) {
  const int t = xcd_group(nround);
  if (t >= ntab) return;
  const int si = __builtin_amdgcn_readfirstlane(tab[t].sys);
  const int g = __builtin_amdgcn_readfirstlane(tab[t].idx);
  __shared__ double lds[kLdsKa];
  ka_body(sys[si].a, g, lds);
}

__global__ __launch_bounds__(kBlock) void k_b_lock(const BatchSys *sys, const SysBlk *tab, int ntab) {
  const int si = __builtin_amdgcn_readfirstlane(tab[blockIdx.x].sys);
  const int blk = __builtin_amdgcn_readfirstlane(tab[blockIdx.x].idx);
  kb_body(sys[si].a, blk);
}

__global__ __launch_bounds__(kBlock) void k_x_lock(const BatchSys *sys, const SysBlk *tab, int ntab) {
  const int si = __builtin_amdgcn_readfirstlane(tab[blockIdx.x].sys);
  const int blk = __builtin_amdgcn_readfirstlane(tab[blockIdx.x].idx);
  kx_body(sys[si].a, blk);
}

__global__ __launch_bounds__(kBlock) void k_step_b_lock(const BatchSys *sys, const int32_t *act) {
  step_b_body(sys[__builtin_amdgcn_readfirstlane(act[blockIdx.x])].a);
}

__global__ __launch_bounds__(kBlock) void k_step_x_lock(const BatchSys *sys, const int32_t *act) {
  step_x_body(sys[__builtin_amdgcn_readfirstlane(act[blockIdx.x])].a);
}

__global__ __launch_bounds__(kBlock) void k_start_lock(const BatchSys *sys, const SysBlk *tab) {
  const int si = __builtin_amdgcn_readfirstlane(tab[blockIdx.x].sys);
  start_block(sys[si].a, __builtin_amdgcn_readfirstlane(tab[blockIdx.x].idx));
}

__global__ __launch_bounds__(kBlock) void k_finish_lock(const BatchSys *sys, const SysBlk *tab) {
  const int si = __builtin_amdgcn_readfirstlane(tab[blockIdx.x].sys);
  const int blk = __builtin_amdgcn_readfirstlane(tab[blockIdx.x].idx);
  const KArgs &a = sys[si].a;
  const Ctl *c = &a.ctl[0];
  finish_block_x(a, c->tier, c->zero_solution, blk);
  if (blk == 0 && threadIdx.x == 0) request_final(&a.ctl[0]);
}

// modes[i] = mode of system act[i] after the last iteration kernel.
__global__ __launch_bounds__(kBlock) void k_modes_lock(const BatchSys *sys, const int32_t *act, int nact,
                                                        int32_t *modes) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < nact) modes[i] = sys[act[i]].a.ctl[0].mode;
}

#endif  // part 5

#if MPCG_IN_PART(4)
// ---------------------------------------------------------------------------
// setup: 16-bit column deltas dc[k] = col[k] - row, thread per row; *bad = 1
// when a delta leaves the int16 range (the caller then drops the array).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_dcol(int n, const int *rp, const int *ci, int16_t *dc, int *bad) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    const int d = ci[k] - i;
    if (d < -32768 || d > 32767) {
      *bad = 1;
      dc[k] = 0;
    } else {
      dc[k] = (int16_t)d;
    }
  }
}

// Interleaved value | delta << 16 words of a 16-bit shadow (entries in [0, np)).
__global__ __launch_bounds__(kBlock) void k_pack16(int np, const uint16_t *v, const int16_t *dc, uint32_t *out) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k < np) out[k] = (uint32_t)v[k] | ((uint32_t)(uint16_t)dc[k] << 16);
}

void launch_pack16(int np, const uint16_t *v, const int16_t *dc, uint32_t *out, hipStream_t s) {
  if (np > 0) hipLaunchKernelGGL(k_pack16, dim3((np + kBlock - 1) / kBlock), dim3(kBlock), 0, s, np, v, dc, out);
}

void launch_dcol(int n, const int *rp, const int *ci, int16_t *dc, int *bad, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_dcol, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, rp, ci, dc, bad);
}

// ---------------------------------------------------------------------------
// setup: shadows
// ---------------------------------------------------------------------------
// Thread per row: fp16 row exponent e (largest magnitude scaled into
// (2^14, 2^15]), fp32 = RNE(v), bf16 = RNE(v), fp16 = RNE(v 2^-e), all directly
// from fp64.
__global__ __launch_bounds__(kBlock) void k_shadows(int n, const int *rp, const int *ci, const double *v,
                                                    float *v32, uint16_t *vbf, uint16_t *vh, uint8_t *v8,
                                                    float *vtf, int8_t *rexp, float *minv) {
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
  float mi = 0.0f;   // Jacobi: the fp64 reciprocal of the diagonal, rounded to fp32
  for (int k = s; k < t; ++k) {
    const double x = v[k];
    if (ci[k] == i) mi = (float)(1.0 / x);
    v32[k] = (float)x;
    vbf[k] = f32_to_bf16_bits_exact((float)round_narrow_f64<8, -126, 127>(x));
    vh[k] = f32_to_f16_bits_exact((float)round_narrow_f64<11, -14, 15>(ldexp(x, -e)));
    // q52 (t = 3, same exponent range as fp16): its value's fp16 encoding has
    // a zero low byte, and the high byte is the q52 encoding
    v8[k] = (uint8_t)(f32_to_f16_bits_exact((float)round_narrow_f64<3, -14, 15>(ldexp(x, -e))) >> 8);
    vtf[k] = rd_from_f64_to_f32<TF32>(x);   // fp32's range: no row scale
  }
  minv[i] = mi;
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
  const GatherPlain<V> gp{(const V *)pv};
  spmv_rows<FS, 1>(A, gp, r0, rows, lds, acc);
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
  const GatherPlain<double> gp{x};
  spmv_rows<FP64, 1>(A, gp, r0, rows, lds, acc);
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
      mlp_logits_block(P, s_feat, s_logits, nullptr);
      if (threadIdx.x == 0) { state[idx] = s; action[idx] = argmax64f(s_logits); }
      __syncthreads();
    } else if (threadIdx.x == 0) {
      int ex = 0;
      state[idx] = s;
      action[idx] = P->kind == POL_QTRAIN ? q_greedy_row(P, &P->q[s * kNAct]) : decide_scalar<true>(P, s, (int)k[idx], &ex);
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_start(const KArgs &a, hipStream_t s) { hipLaunchKernelGGL(k_start, dim3(a.P2), dim3(kBlock), 0, s, a); }
// Optional events (e0, e1) take the kernel's own start and stop times.
template <typename K>
static void launch_timed(K kern, int grid, const KArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (e0) hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, e0, e1, 0, a);
  else hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), 0, s, a);
}
void launch_ka(const KArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  launch_timed(a.vec16 ? k_a16 : a.ext ? k_a_ext : k_a, a.G1, a, s, e0, e1);
}
void launch_kb(const KArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (a.rho64 && a.precond) launch_timed(a.full ? k_b_full_pc_r64 : k_b_pc_r64, a.P2, a, s, e0, e1);
  else if (a.rho64) launch_timed(a.full ? k_b_full_r64 : k_b_r64, a.P2, a, s, e0, e1);
  else if (a.precond) launch_timed(a.full ? k_b_full_pc : k_b_pc, a.P2, a, s, e0, e1);
  else if (a.vec16) launch_timed(a.full ? k_b_full16 : k_b16, a.P2, a, s, e0, e1);
  else if (a.ext) launch_timed(a.full ? k_b_full_ext : k_b_ext, a.P2, a, s, e0, e1);
  else launch_timed(a.full ? k_b_full : k_b, a.P2, a, s, e0, e1);
}
void launch_kx(const KArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  launch_timed(a.precond ? k_x_pc : a.vec16 ? k_x16 : a.ext ? k_x_ext : k_x, a.P2, a, s, e0, e1);
}
void launch_step_b(const KArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) { launch_timed(k_step_b, 1, a, s, e0, e1); }
void launch_step_x(const KArgs &a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  launch_timed(a.net ? k_step_x_net : k_step_x, 1, a, s, e0, e1);
}

void launch_slot(const KArgs &a, hipStream_t s) {
  launch_ka(a, s);
  if (a.slow) launch_step_b(a, s);
  launch_kb(a, s);
  if (a.slow || a.full) launch_step_x(a, s);
  launch_kx(a, s);
}

void launch_finish(const KArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(a.P2), dim3(kBlock), 0, s, a);
  launch_ka(a, s);
  if (a.slow) launch_step_b(a, s);
  launch_kb(a, s);
}

void launch_batched(const BatchSys *sys, const int32_t *order, int nsys, int32_t *queue, int grid,
                    hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (e0) hipExtLaunchKernelGGL(k_batched, dim3(grid), dim3(kBlock), 0, s, e0, e1, 0, sys, order, nsys, queue);
  else hipLaunchKernelGGL(k_batched, dim3(grid), dim3(kBlock), 0, s, sys, order, nsys, queue);
}

void launch_lock_slot(const BatchSys *sys, const SysBlk *tka, int nka, const SysBlk *tvb, int nvb,
                      const int32_t *act, int nact, int slow, hipStream_t s) {
  const int nr = (nka + 7) / 8 * 8;
  if (nka > 0) hipLaunchKernelGGL(k_a_lock, dim3(nr), dim3(kBlock), 0, s, sys, tka, nka, nr);
  if (slow && nact > 0) hipLaunchKernelGGL(k_step_b_lock, dim3(nact), dim3(kBlock), 0, s, sys, act);
  if (nvb > 0) hipLaunchKernelGGL(k_b_lock, dim3(nvb), dim3(kBlock), 0, s, sys, tvb, nvb);
  if (slow && nact > 0) hipLaunchKernelGGL(k_step_x_lock, dim3(nact), dim3(kBlock), 0, s, sys, act);
  if (nvb > 0) hipLaunchKernelGGL(k_x_lock, dim3(nvb), dim3(kBlock), 0, s, sys, tvb, nvb);
}

void launch_lock_start(const BatchSys *sys, const SysBlk *tvb, int nvb, hipStream_t s) {
  if (nvb > 0) hipLaunchKernelGGL(k_start_lock, dim3(nvb), dim3(kBlock), 0, s, sys, tvb);
}

void launch_lock_finish(const BatchSys *sys, const SysBlk *tka, int nka, const SysBlk *tvb, int nvb,
                        const int32_t *act, int nact, int slow, hipStream_t s) {
  if (nvb > 0) hipLaunchKernelGGL(k_finish_lock, dim3(nvb), dim3(kBlock), 0, s, sys, tvb);
  const int nr = (nka + 7) / 8 * 8;
  if (nka > 0) hipLaunchKernelGGL(k_a_lock, dim3(nr), dim3(kBlock), 0, s, sys, tka, nka, nr);
  if (slow && nact > 0) hipLaunchKernelGGL(k_step_b_lock, dim3(nact), dim3(kBlock), 0, s, sys, act);
  if (nvb > 0) hipLaunchKernelGGL(k_b_lock, dim3(nvb), dim3(kBlock), 0, s, sys, tvb, nvb);
}

void launch_lock_modes(const BatchSys *sys, const int32_t *act, int nact, int32_t *modes, hipStream_t s) {
  if (nact > 0) hipLaunchKernelGGL(k_modes_lock, dim3((nact + kBlock - 1) / kBlock), dim3(kBlock), 0, s, sys, act,
                                   nact, modes);
}

void launch_shadows(int n, const int *rp, const int *ci, const double *v, float *v32, uint16_t *vbf,
                    uint16_t *vh, uint8_t *v8, float *vtf, int8_t *rexp, float *minv, hipStream_t s) {
  hipLaunchKernelGGL(k_shadows, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, rp, ci, v, v32, vbf, vh,
                     v8, vtf, rexp, minv);
}

void launch_op_spmv(const Mat &A, int fs, int tier, const void *p, void *q, hipStream_t s) {
  const int P = (A.n + kRowsPerBlock - 1) / kRowsPerBlock;
  const int G = (P + 7) / 8 * 8;
#define MPCG_SPMV(FS, T) hipLaunchKernelGGL((k_op_spmv<FS, T>), dim3(G), dim3(kBlock), 0, s, A, p, q, P, G)
  switch (fs * 2 + tier) {
  case 10: MPCG_SPMV(TF32, 0); break;
  case 11: MPCG_SPMV(TF32, 1); break;
  case 8: MPCG_SPMV(FP8, 0); break;
  case 9: MPCG_SPMV(FP8, 1); break;
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
  case 10: MPCG_DOT(TF32, 0); break;
  case 11: MPCG_DOT(TF32, 1); break;
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

// ---------------------------------------------------------------------------
// Measurement: the floor of an SpMV over the same index stream.  A flat pass
// over the CSR entries: thread t of block b takes entries b*2048 + t + 256 j,
// j < 8 (coalesced index and bf16 value loads), issues the eight gathers of p
// together, and sums the products.  No row structure, no reductions: only the
// matrix stream and one gather per entry with the most gathers in flight.  The
// sum is stored only if it is NaN (never, for finite p), so no output traffic
// is made, and the loads cannot be removed.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_gather_floor(const int *__restrict__ col, const uint16_t *__restrict__ val,
                                                         const float *__restrict__ p, int nnz,
                                                         float *__restrict__ sink) {
  const int base = blockIdx.x * kVecBlock + threadIdx.x;
  int c[8];
  float v[8], x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int i = base + kBlock * j;
    c[j] = i < nnz ? col[i] : 0;
    v[j] = i < nnz ? bf16_bits_to_f32(val[i]) : 0.0f;
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = p[c[j]];
  float acc = 0.0f;
#pragma unroll
  for (int j = 0; j < 8; ++j) acc = __builtin_fmaf(v[j], x[j], acc);
  if (acc != acc) sink[0] = acc;
}

void launch_gather_floor(const Mat &A, const float *p, float *sink, hipStream_t s) {
  const int grid = (A.nnz + kVecBlock - 1) / kVecBlock;
  hipLaunchKernelGGL(k_gather_floor, dim3(grid), dim3(kBlock), 0, s, A.ci, A.vbf, p, A.nnz, sink);
}

// ---------------------------------------------------------------------------
// The dot product without allocation: the same two kernels as launch_op_dot,
// with the block partials in a file-scope device array instead of handle
// memory.  In host code `scratch` names a host-side stand-in, not device
// memory: its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// ever passed to kernels.  Every call on one device shares that device's
// array, so calls that overlap on one device race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kNoAllocPartials];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of this device's scratch array (looked up on first use).
static hipError_t scratch_address(double **out) {
  *out = nullptr;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double *)ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_op_dot_noalloc(int n, int fd, int tier, const void *u, const void *v, double *out,
                                 hipStream_t s) {
  const int P2 = (n + kVecBlock - 1) / kVecBlock;
  if (P2 > kNoAllocPartials) return hipErrorInvalidValue;
  double *part = nullptr;
  const hipError_t e = scratch_address(&part);
  if (e != hipSuccess) return e;
  launch_op_dot(n, fd, tier, u, v, part, P2, out, s);
  return hipGetLastError();
}

void launch_op_axpy(int n, int fa, double alpha, const void *u, void *y, hipStream_t s) {
  const dim3 g((n + kBlock - 1) / kBlock);
  switch (fa) {
  case FP16: hipLaunchKernelGGL((k_op_axpy<FP16>), g, dim3(kBlock), 0, s, n, alpha, u, y); break;
  case BF16: hipLaunchKernelGGL((k_op_axpy<BF16>), g, dim3(kBlock), 0, s, n, alpha, u, y); break;
  case FP32: hipLaunchKernelGGL((k_op_axpy<FP32>), g, dim3(kBlock), 0, s, n, alpha, u, y); break;
  case TF32: hipLaunchKernelGGL((k_op_axpy<TF32>), g, dim3(kBlock), 0, s, n, alpha, u, y); break;
  default: hipLaunchKernelGGL((k_op_axpy<FP64>), g, dim3(kBlock), 0, s, n, alpha, u, y); break;
  }
}

void launch_policy_decide(const PolicyDev *P, int m, const int64_t *k, const double *rho, const int32_t *stag,
                          const float *feat, int32_t *state, int32_t *action, hipStream_t s) {
  const int g = m < 1024 ? (m > 0 ? m : 1) : 1024;
  hipLaunchKernelGGL(k_policy_decide, dim3(g), dim3(kBlock), 0, s, P, m, k, rho, stag, feat, state, action);
}

#endif  // part 4


#if MPCG_IN_PART(9)
// ---------------------------------------------------------------------------
// Single-reduction CG (Chronopoulos and Gear, 1989).  Section 3's iteration
// rearranged so that its one SpMV, w = A r, is followed by both inner
// products, gamma = r.r and delta = r.w, whose partials KS1 takes in the
// SpMV's epilogue; s = A p is carried by a recurrence:
//   beta = gamma / gamma_old, alpha = gamma / (delta - beta gamma / alpha_old),
//   p = r + beta p, s = w + beta s, x_lo += alpha p, r -= alpha s.
// One iteration is two launches with one grid-wide dependency each (three in
// the main solver) and the same vector traffic: KS1 reads r and writes w,
// KS2 reads r, w, p, s, x_lo and writes p, s, x_lo, r.  A true-residual
// replacement folds x_lo into x_hi (in the KS2 before it), replaces r by
// rd(b - A x_hi), and the KS1 after it also recomputes s = A p.
// Pipelined CG (Ghysels and Vanroose, 2014), the PIPE kernels: w = A r and
// z = A s are recurrences too, KS1 runs q = A w with the partials of r.r and
// w.r, KS2 the six updates z = q + beta z, s = w + beta s, p = r + beta p,
// x_lo += alpha p, r -= alpha s, w -= alpha z; after a start or replacement
// a sync phase computes w = A r and s = A p, and the next KS1 also z = A s.
// Both: fixed actions of the four-format set and q52 storage; no policy,
// fallback or preconditioner.  Every workgroup of KS2 runs the scalar step
// identically from KS1's partials; workgroup 0 commits the state to the
// other half of the double buffer and writes the histories.
// ---------------------------------------------------------------------------

// The subtree sums of two dots over the same rows, u.v1 and u.v2, in one LDS
// round (each subtree is summed as by dot_leaf_multi).
template <int FD, int RPT, typename V>
__device__ __forceinline__ void dot_leaf_multi2(const V (&u)[RPT], const V (&v1)[RPT], const V (&v2)[RPT],
                                                const bool (&valid)[RPT], double (&o1)[RPT], double (&o2)[RPT]) {
  using A = typename AccT<FD>::type;
  A l[2 * RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    l[j] = valid[j] ? dot_leaf<FD>(u[j], v1[j]) : (A)0;
    l[RPT + j] = valid[j] ? dot_leaf<FD>(u[j], v2[j]) : (A)0;
  }
  double out[2 * RPT];
  block_tree_multi<2 * RPT>(l, out);
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    o1[j] = out[j];
    o2[j] = out[RPT + j];
  }
}

template <int RPT, typename V>
__device__ __forceinline__ void dot_leaf_multi2_rt(int fd, const V (&u)[RPT], const V (&v1)[RPT], const V (&v2)[RPT],
                                                   const bool (&valid)[RPT], double (&o1)[RPT], double (&o2)[RPT]) {
  switch (fd) {
  case FP16: dot_leaf_multi2<FP16, RPT>(u, v1, v2, valid, o1, o2); break;
  case BF16: dot_leaf_multi2<BF16, RPT>(u, v1, v2, valid, o1, o2); break;
  case FP32: dot_leaf_multi2<FP32, RPT>(u, v1, v2, valid, o1, o2); break;
  default: dot_leaf_multi2<FP64, RPT>(u, v1, v2, valid, o1, o2); break;
  }
}

// y = A_fs x over row group g, rounded to the tier (a second SpMV of a
// KS1: s = A p, z = A s, w = A r; no partials).
template <int FS, int TIER>
__device__ __forceinline__ void sr_spmv_plain(const SrArgs &a, int g, void *lds, const typename TierT<TIER>::type *x,
                                              typename TierT<TIER>::type *y) {
  using V = typename TierT<TIER>::type;
  using Acc = typename AccT<FS>::type;
  const int n = a.A.n;
  const int g0 = g * a.grows;
  const int grows = min(a.grows, n - g0);
  int8_t ex[kRPT];
  auto pref = [](int) {};
  auto pre = [&](int sb) {
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      ex[j] = 0;
      if constexpr (FS == FP16 || FS == FP8) {
        const int lr = sb * kKaRows + threadIdx.x + j * kRowsPerBlock;
        if (lr < grows) ex[j] = a.A.rexp[g0 + lr];
      }
    }
  };
  auto epi = [&](int sb, Acc (&acc)[kRPT]) {
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int lr = sb * kKaRows + threadIdx.x + j * kRowsPerBlock;
      if (lr < grows) {
        if constexpr (FS == FP16 || FS == FP8) y[g0 + lr] = (V)ldexp((double)acc[j], (int)ex[j]);
        else y[g0 + lr] = (V)acc[j];
      }
    }
  };
  if (a.A.dc) spmv_group<FS, true>(a.A, GatherPlain<V>{x}, g0, grows, lds, pref, pre, epi);
  else spmv_group<FS, false>(a.A, GatherPlain<V>{x}, g0, grows, lds, pref, pre, epi);
}

// KS1 of an iteration: w = A_fs r over row group g with the group partials
// of gamma and delta at the dot format; with_s: then s = A_fs p.
template <int FS, int TIER>
__device__ __forceinline__ void sr_spmv(const SrArgs &a, const SrCtl &S, int g, void *lds, bool with_s) {
  using V = typename TierT<TIER>::type;
  using Acc = typename AccT<FS>::type;
  const V *r, *p;
  V *w, *sv;
  if constexpr (TIER) { r = a.v.r64; w = a.v.q64; p = a.v.p64; sv = a.s64; }
  else { r = a.v.r32; w = a.v.q32; p = a.v.p32; sv = a.s32; }
  const int fd = S.fd;
  const int n = a.A.n;
  const int g0 = g * a.grows;
  const int grows = min(a.grows, n - g0);
  V ri[kRPT], rn[kRPT];   // own elements of r: current sub-block, next sub-block
  int8_t ex[kRPT];
  double tg[4] = {0.0, 0.0, 0.0, 0.0}, td[4] = {0.0, 0.0, 0.0, 0.0};
  auto pref = [&](int sb) {
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int lr = sb * kKaRows + threadIdx.x + j * kRowsPerBlock;
      rn[j] = lr < grows ? r[g0 + lr] : (V)0;
    }
  };
  auto pre = [&](int sb) {
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int lr = sb * kKaRows + threadIdx.x + j * kRowsPerBlock;
      ri[j] = rn[j];
      ex[j] = 0;
      if constexpr (FS == FP16 || FS == FP8) {
        if (lr < grows) ex[j] = a.A.rexp[g0 + lr];
      }
    }
  };
  auto epi = [&](int sb, Acc (&acc)[kRPT]) {
    V wi[kRPT];
    bool valid[kRPT];
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int lr = sb * kKaRows + threadIdx.x + j * kRowsPerBlock;
      valid[j] = lr < grows;
      wi[j] = (V)0;
      if (valid[j]) {
        if constexpr (FS == FP16 || FS == FP8) wi[j] = (V)ldexp((double)acc[j], (int)ex[j]);
        else wi[j] = (V)acc[j];
        w[g0 + lr] = wi[j];
      }
    }
    double s2g[kRPT], s2d[kRPT];
    dot_leaf_multi2_rt<kRPT>(fd, ri, ri, wi, valid, s2g, s2d);
    const double sg = subtrees_rt<kRPT>(fd, s2g);
    const double sd = subtrees_rt<kRPT>(fd, s2d);
    tg[0] = sb == 0 ? sg : tg[0];
    tg[1] = sb == 1 ? sg : tg[1];
    tg[2] = sb == 2 ? sg : tg[2];
    tg[3] = sb == 3 ? sg : tg[3];
    td[0] = sb == 0 ? sd : td[0];
    td[1] = sb == 1 ? sd : td[1];
    td[2] = sb == 2 ? sd : td[2];
    td[3] = sb == 3 ? sd : td[3];
  };
  if (a.A.dc) spmv_group<FS, true>(a.A, GatherPlain<V>{r}, g0, grows, lds, pref, pre, epi);
  else spmv_group<FS, false>(a.A, GatherPlain<V>{r}, g0, grows, lds, pref, pre, epi);
  if (threadIdx.x == 0) {
    a.pg[g] = group_tree(fd, a.grows, tg);
    a.pd[g] = group_tree(fd, a.grows, td);
  }
  if (!with_s) return;
  __syncthreads();   // the LDS window is staged again
  sr_spmv_plain<FS, TIER>(a, g, lds, p, sv);
}

// KS1 of a pipelined iteration: q = A_fs w over row group g with the group
// partials of gamma = r.r and delta = w.r at the dot format; with_z: then
// z = A_fs s (the first iteration after a replacement).
template <int FS, int TIER>
__device__ __forceinline__ void pc_spmv(const SrArgs &a, const SrCtl &S, int g, void *lds, bool with_z) {
  using V = typename TierT<TIER>::type;
  using Acc = typename AccT<FS>::type;
  const V *r, *w, *sv;
  V *q, *z;
  if constexpr (TIER) { r = a.v.r64; w = a.w64; sv = a.s64; q = a.v.q64; z = a.z64; }
  else { r = a.v.r32; w = a.w32; sv = a.s32; q = a.v.q32; z = a.z32; }
  const int fd = S.fd;
  const int n = a.A.n;
  const int g0 = g * a.grows;
  const int grows = min(a.grows, n - g0);
  V ri[kRPT], rn[kRPT], wi[kRPT], wn[kRPT];   // own elements of r and w: current, next sub-block
  int8_t ex[kRPT];
  double tg[4] = {0.0, 0.0, 0.0, 0.0}, td[4] = {0.0, 0.0, 0.0, 0.0};
  auto pref = [&](int sb) {
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int lr = sb * kKaRows + threadIdx.x + j * kRowsPerBlock;
      rn[j] = lr < grows ? r[g0 + lr] : (V)0;
      wn[j] = lr < grows ? w[g0 + lr] : (V)0;
    }
  };
  auto pre = [&](int sb) {
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int lr = sb * kKaRows + threadIdx.x + j * kRowsPerBlock;
      ri[j] = rn[j];
      wi[j] = wn[j];
      ex[j] = 0;
      if constexpr (FS == FP16 || FS == FP8) {
        if (lr < grows) ex[j] = a.A.rexp[g0 + lr];
      }
    }
  };
  auto epi = [&](int sb, Acc (&acc)[kRPT]) {
    bool valid[kRPT];
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int lr = sb * kKaRows + threadIdx.x + j * kRowsPerBlock;
      valid[j] = lr < grows;
      if (valid[j]) {
        if constexpr (FS == FP16 || FS == FP8) q[g0 + lr] = (V)ldexp((double)acc[j], (int)ex[j]);
        else q[g0 + lr] = (V)acc[j];
      }
    }
    double s2g[kRPT], s2d[kRPT];
    dot_leaf_multi2_rt<kRPT>(fd, ri, ri, wi, valid, s2g, s2d);
    const double sg = subtrees_rt<kRPT>(fd, s2g);
    const double sd = subtrees_rt<kRPT>(fd, s2d);
    tg[0] = sb == 0 ? sg : tg[0];
    tg[1] = sb == 1 ? sg : tg[1];
    tg[2] = sb == 2 ? sg : tg[2];
    tg[3] = sb == 3 ? sg : tg[3];
    td[0] = sb == 0 ? sd : td[0];
    td[1] = sb == 1 ? sd : td[1];
    td[2] = sb == 2 ? sd : td[2];
    td[3] = sb == 3 ? sd : td[3];
  };
  if (a.A.dc) spmv_group<FS, true>(a.A, GatherPlain<V>{w}, g0, grows, lds, pref, pre, epi);
  else spmv_group<FS, false>(a.A, GatherPlain<V>{w}, g0, grows, lds, pref, pre, epi);
  if (threadIdx.x == 0) {
    a.pg[g] = group_tree(fd, a.grows, tg);
    a.pd[g] = group_tree(fd, a.grows, td);
  }
  if (!with_z) return;
  __syncthreads();
  sr_spmv_plain<FS, TIER>(a, g, lds, sv, z);
}

// KS1 after a start or replacement of the pipelined iteration: w = A_fs r,
// and s = A_fs p unless the next step is the first.
template <int FS, int TIER>
__device__ __forceinline__ void pc_sync(const SrArgs &a, const SrCtl &S, int g, void *lds) {
  if constexpr (TIER) {
    sr_spmv_plain<FS, 1>(a, g, lds, a.v.r64, a.w64);
    if (!S.first) {
      __syncthreads();
      sr_spmv_plain<FS, 1>(a, g, lds, a.v.p64, a.s64);
    }
  } else {
    sr_spmv_plain<FS, 0>(a, g, lds, a.v.r32, a.w32);
    if (!S.first) {
      __syncthreads();
      sr_spmv_plain<FS, 0>(a, g, lds, a.v.p32, a.s32);
    }
  }
}

// KS1 of a start, replacement or final check: r64 = b - A x in fp64 over row
// group g with the partial of ||r64||^2; r = rd_tier(r64) (not at the final
// check).  A start reads the caller's x, copies it to x_hi, clears x_lo and
// takes the partial of ||b||^2 too.
__device__ __forceinline__ void sr_residual(const SrArgs &a, const SrCtl &S, int g, void *lds) {
  const int n = a.A.n;
  const int g0 = g * a.grows;
  const int grows = min(a.grows, n - g0);
  const bool start = S.mode == SR_START, fin = S.mode == SR_FINAL;
  const int tier = S.tier;
  double bi[kRPT];
  double t[4] = {0.0, 0.0, 0.0, 0.0}, tb[4] = {0.0, 0.0, 0.0, 0.0};
  auto pref = [](int) {};
  auto pre = [&](int sb) {
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int lr = sb * kKaRows + threadIdx.x + j * kRowsPerBlock;
      bi[j] = lr < grows ? a.v.b[g0 + lr] : 0.0;
    }
  };
  auto epi = [&](int sb, double (&acc)[kRPT]) {
    double leaf[kRPT], leafb[kRPT];
#pragma unroll
    for (int j = 0; j < kRPT; ++j) {
      const int lr = sb * kKaRows + threadIdx.x + j * kRowsPerBlock;
      leaf[j] = 0.0;
      leafb[j] = 0.0;
      if (lr < grows) {
        const int i = g0 + lr;
        const double r = bi[j] - acc[j];
        leaf[j] = r * r;
        leafb[j] = bi[j] * bi[j];
        if (start) {
          a.v.xhi[i] = a.v.xout[i];
          if (tier) a.v.xlo64[i] = 0.0;
          else a.v.xlo32[i] = 0.0f;
        }
        if (!fin) {
          if (tier) a.v.r64[i] = r;
          else a.v.r32[i] = (float)r;
        }
      }
    }
    double s2[kRPT];
    block_tree_multi<kRPT>(leaf, s2);
    const double s = subtrees_rt<kRPT>(FP64, s2);
    t[0] = sb == 0 ? s : t[0];
    t[1] = sb == 1 ? s : t[1];
    t[2] = sb == 2 ? s : t[2];
    t[3] = sb == 3 ? s : t[3];
    if (start) {
      block_tree_multi<kRPT>(leafb, s2);
      const double sbb = subtrees_rt<kRPT>(FP64, s2);
      tb[0] = sb == 0 ? sbb : tb[0];
      tb[1] = sb == 1 ? sbb : tb[1];
      tb[2] = sb == 2 ? sbb : tb[2];
      tb[3] = sb == 3 ? sbb : tb[3];
    }
  };
  const double *x = start ? a.v.xout : a.v.xhi;
  if (a.A.dc) spmv_group<FP64, true>(a.A, GatherPlain<double>{x}, g0, grows, lds, pref, pre, epi);
  else spmv_group<FP64, false>(a.A, GatherPlain<double>{x}, g0, grows, lds, pref, pre, epi);
  if (threadIdx.x == 0) {
    a.pg[g] = group_tree(FP64, a.grows, t);
    if (start) a.pd[g] = group_tree(FP64, a.grows, tb);
  }
}

#define MPCG_PC_CASES(FN, ...)                          \
  switch (S.fs * 2 + S.tier) {                          \
  case FP16 * 2: FN<FP16, 0>(__VA_ARGS__); break;       \
  case FP16 * 2 + 1: FN<FP16, 1>(__VA_ARGS__); break;   \
  case BF16 * 2: FN<BF16, 0>(__VA_ARGS__); break;       \
  case BF16 * 2 + 1: FN<BF16, 1>(__VA_ARGS__); break;   \
  case FP32 * 2: FN<FP32, 0>(__VA_ARGS__); break;       \
  case FP32 * 2 + 1: FN<FP32, 1>(__VA_ARGS__); break;   \
  case FP64 * 2: FN<FP64, 0>(__VA_ARGS__); break;       \
  case FP64 * 2 + 1: FN<FP64, 1>(__VA_ARGS__); break;   \
  case FP8 * 2: FN<FP8, 0>(__VA_ARGS__); break;         \
  case FP8 * 2 + 1: FN<FP8, 1>(__VA_ARGS__); break;     \
  default: break;                                       \
  }

// PIPE: the pipelined iteration's KS1 (a separate kernel, so the
// single-reduction one keeps its registers).
template <bool PIPE>
__global__ __launch_bounds__(kBlock) void k_sr1(SrArgs a) {
  const int g = xcd_group(a.G1);
  if (g >= a.P1) return;
  __shared__ double lds[kLdsKa];
  const SrCtl &S = a.ctl[a.par];
  const int mode = S.mode;
  if constexpr (PIPE) {
    if (mode == SR_ITER) {
      const bool with_z = S.sync && !S.first;
      MPCG_PC_CASES(pc_spmv, a, S, g, lds, with_z)
    } else if (mode == PC_W) {
      MPCG_PC_CASES(pc_sync, a, S, g, lds)
    } else if (mode == SR_START || mode == SR_RESID || mode == SR_FINAL) {
      sr_residual(a, S, g, lds);
    }
    return;
  }
  if (mode == SR_ITER || mode == SR_SYNC) {
    const bool with_s = mode == SR_SYNC && !S.first;
    switch (S.fs * 2 + S.tier) {
    case FP16 * 2: sr_spmv<FP16, 0>(a, S, g, lds, with_s); break;
    case FP16 * 2 + 1: sr_spmv<FP16, 1>(a, S, g, lds, with_s); break;
    case BF16 * 2: sr_spmv<BF16, 0>(a, S, g, lds, with_s); break;
    case BF16 * 2 + 1: sr_spmv<BF16, 1>(a, S, g, lds, with_s); break;
    case FP32 * 2: sr_spmv<FP32, 0>(a, S, g, lds, with_s); break;
    case FP32 * 2 + 1: sr_spmv<FP32, 1>(a, S, g, lds, with_s); break;
    case FP64 * 2: sr_spmv<FP64, 0>(a, S, g, lds, with_s); break;
    case FP64 * 2 + 1: sr_spmv<FP64, 1>(a, S, g, lds, with_s); break;
    case FP8 * 2: sr_spmv<FP8, 0>(a, S, g, lds, with_s); break;
    case FP8 * 2 + 1: sr_spmv<FP8, 1>(a, S, g, lds, with_s); break;
    default: break;
    }
  } else if (mode == SR_START || mode == SR_RESID || mode == SR_FINAL) {
    sr_residual(a, S, g, lds);
  }
}

// KS2's operands of one thread (8 consecutive elements of block blk) in the
// container of the update format.
template <int FA>
struct SrVals {
  using V = typename TierT<FA == FP64>::type;
  V r[8], w[8], p[8], s[8], x[8];
};

template <int FA>
__device__ __forceinline__ void sr_vecs(const SrArgs &a, typename SrVals<FA>::V *&r, typename SrVals<FA>::V *&w,
                                        typename SrVals<FA>::V *&p, typename SrVals<FA>::V *&s,
                                        typename SrVals<FA>::V *&xl) {
  if constexpr (FA == FP64) { r = a.v.r64; w = a.v.q64; p = a.v.p64; s = a.s64; xl = a.v.xlo64; }
  else { r = a.v.r32; w = a.v.q32; p = a.v.p32; s = a.s32; xl = a.v.xlo32; }
}

// Issues the loads of r, w, p, s and x_lo (p and s are read on the first step
// too, where they are not used).
template <int FA>
__device__ __forceinline__ void sr_load(const SrArgs &a, int base, SrVals<FA> &v) {
  using V = typename SrVals<FA>::V;
  V *r, *w, *p, *s, *xl;
  sr_vecs<FA>(a, r, w, p, s, xl);
  const int n = a.A.n;
  if (base + 8 <= n) {
    load8(r + base, v.r);
    load8(w + base, v.w);
    load8(p + base, v.p);
    load8(s + base, v.s);
    load8(xl + base, v.x);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = base + j;
      const bool in = i < n;
      v.r[j] = in ? r[i] : (V)0;
      v.w[j] = in ? w[i] : (V)0;
      v.p[j] = in ? p[i] : (V)0;
      v.s[j] = in ? s[i] : (V)0;
      v.x[j] = in ? xl[i] : (V)0;
    }
  }
}

// The direction and recurrence updates (copies on the first step), x_lo and
// r, and the fold of x_lo into x_hi before a replacement.
template <int FA>
__device__ __forceinline__ void sr_update(const SrArgs &a, int base, SrVals<FA> &v, double alpha, double beta,
                                          bool first, bool fold) {
  using V = typename SrVals<FA>::V;
  V *r, *w, *p, *s, *xl;
  sr_vecs<FA>(a, r, w, p, s, xl);
  const int n = a.A.n;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const V pn = first ? v.r[j] : xpay_rt<V>(FA, beta, v.p[j], v.r[j]);
    const V sn = first ? v.w[j] : xpay_rt<V>(FA, beta, v.s[j], v.w[j]);
    v.x[j] = axpy1<FA>(alpha, pn, v.x[j]);
    v.r[j] = axpy1<FA>(-alpha, sn, v.r[j]);
    v.p[j] = pn;
    v.s[j] = sn;
  }
  if (fold) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (base + j < n) fold1(a.v.xhi, base + j, (double)v.x[j]);
      v.x[j] = (V)0;
    }
  }
  if (base + 8 <= n) {
    store8(p + base, v.p);
    store8(s + base, v.s);
    store8(xl + base, v.x);
    store8(r + base, v.r);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = base + j;
      if (i < n) {
        p[i] = v.p[j];
        s[i] = v.s[j];
        xl[i] = v.x[j];
        r[i] = v.r[j];
      }
    }
  }
}

template <int FA>
__device__ __forceinline__ void sr_fold(const SrArgs &a, int base, SrVals<FA> &v) {
  using V = typename SrVals<FA>::V;
  V *r, *w, *p, *s, *xl;
  sr_vecs<FA>(a, r, w, p, s, xl);
  const int n = a.A.n;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int i = base + j;
    if (i < n) {
      fold1(a.v.xhi, i, (double)v.x[j]);
      xl[i] = (V)0;
    }
  }
}

// The state after KS2, identical in every thread.
struct SrNext {
  int mode, status, k, nrep, sync;
  bool upd, zero;
  double bnorm, last_true, relres, rho, gamma, alpha;
};

__device__ __forceinline__ SrNext sr_next_of(const SrCtl &S) {
  SrNext x;
  x.mode = S.mode;
  x.status = S.status;
  x.k = S.k;
  x.nrep = S.nrep;
  x.sync = S.sync;
  x.upd = false;
  x.zero = false;
  x.bnorm = S.bnorm;
  x.last_true = S.last_true;
  x.relres = S.relres_true;
  x.rho = S.rho_new;
  x.gamma = 0.0;
  x.alpha = 0.0;
  return x;
}

// KS2 after an iteration's KS1: gamma, delta -> rho (replacement or budget
// test), beta, alpha (breakdown test), then the updates of block blk, whose
// operands are loaded before the step.
template <int FA>
__device__ __forceinline__ SrNext sr2_iter(const SrArgs &a, const SrCtl &S, int blk, const double (&pg)[8],
                                           const double (&pd)[8], bool fast) {
  const int base = blk * kVecBlock + threadIdx.x * kVecPer;
  SrVals<FA> v;
  const bool live = base < a.A.n;
  __builtin_amdgcn_sched_barrier(0);
  if (live) sr_load<FA>(a, base, v);
  __builtin_amdgcn_sched_barrier(0);
  SrNext x = sr_next_of(S);
  const bool writer = blk == 0 && threadIdx.x == 0;
  const int k = S.k;
  const int fd = S.fd;
  const bool first = S.first != 0;
  const double gamma = fast ? tree_preloaded_rt(fd, pg) : reduce_partials_rt(fd, a.pg, a.P1);
  const double delta = fast ? tree_preloaded_rt(fd, pd) : reduce_partials_rt(fd, a.pd, a.P1);
  bool fold = false, go = true;
  if (S.mode == SR_ITER) {
    x.rho = sqrt(gamma) / S.bnorm;
    if (writer) a.h.rho[k] = x.rho;
    if (x.rho <= S.tol) {
      fold = true;
      x.mode = SR_RESID;
      go = false;
    } else if (k >= S.maxit) {
      x.status = 1;
      fold = true;
      x.mode = SR_FINAL;
      go = false;
    }
  }
  double alpha = 0.0, beta = 0.0;
  if (go) {
    beta = first ? 0.0 : gamma / S.gamma_old;
    const double den = first ? delta : delta - beta * gamma / S.alpha_old;
    alpha = gamma / den;
    if (!(den > 0.0) || !isfinite(alpha) || !isfinite(beta) || !isfinite(gamma)) {
      x.status = 3;
      fold = true;
      x.mode = SR_FINAL;
    } else {
      x.upd = true;
      x.gamma = gamma;
      x.alpha = alpha;
      if (writer) {
        a.h.act[k] = (uint8_t)S.action;
        a.h.flag[k] = 0;
      }
      x.k = k + 1;
      fold = S.R > 0 && x.k % S.R == 0;
      x.mode = fold ? SR_RESID : SR_ITER;
    }
  }
  if (live) {
    if (x.upd) sr_update<FA>(a, base, v, alpha, beta, first, fold);
    else if (fold) sr_fold<FA>(a, base, v);
  }
  return x;
}

// The pipelined iteration's KS2 operands of one thread: q, z, w, s, r, p, x_lo.
template <int FA>
struct PcVals {
  using V = typename TierT<FA == FP64>::type;
  V q[8], z[8], w[8], s[8], r[8], p[8], x[8];
};

template <int FA>
struct PcPtr {
  using V = typename TierT<FA == FP64>::type;
  V *q, *z, *w, *s, *r, *p, *x;
  __device__ explicit PcPtr(const SrArgs &a) {
    if constexpr (FA == FP64) { q = a.v.q64; z = a.z64; w = a.w64; s = a.s64; r = a.v.r64; p = a.v.p64; x = a.v.xlo64; }
    else { q = a.v.q32; z = a.z32; w = a.w32; s = a.s32; r = a.v.r32; p = a.v.p32; x = a.v.xlo32; }
  }
};

template <int FA>
__device__ __forceinline__ void pc_load(const SrArgs &a, int base, PcVals<FA> &v) {
  using V = typename PcVals<FA>::V;
  const PcPtr<FA> P(a);
  const int n = a.A.n;
  if (base + 8 <= n) {
    load8(P.q + base, v.q);
    load8(P.z + base, v.z);
    load8(P.w + base, v.w);
    load8(P.s + base, v.s);
    load8(P.r + base, v.r);
    load8(P.p + base, v.p);
    load8(P.x + base, v.x);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = base + j;
      const bool in = i < n;
      v.q[j] = in ? P.q[i] : (V)0;
      v.z[j] = in ? P.z[i] : (V)0;
      v.w[j] = in ? P.w[i] : (V)0;
      v.s[j] = in ? P.s[i] : (V)0;
      v.r[j] = in ? P.r[i] : (V)0;
      v.p[j] = in ? P.p[i] : (V)0;
      v.x[j] = in ? P.x[i] : (V)0;
    }
  }
}

// z = q + beta z, s = w + beta s, p = r + beta p (copies on the first step),
// x_lo += alpha p, r -= alpha s, w -= alpha z; the fold before a replacement.
template <int FA>
__device__ __forceinline__ void pc_update(const SrArgs &a, int base, PcVals<FA> &v, double alpha, double beta,
                                          bool first, bool fold) {
  using V = typename PcVals<FA>::V;
  const PcPtr<FA> P(a);
  const int n = a.A.n;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const V zn = first ? v.q[j] : xpay_rt<V>(FA, beta, v.z[j], v.q[j]);
    const V sn = first ? v.w[j] : xpay_rt<V>(FA, beta, v.s[j], v.w[j]);
    const V pn = first ? v.r[j] : xpay_rt<V>(FA, beta, v.p[j], v.r[j]);
    v.x[j] = axpy1<FA>(alpha, pn, v.x[j]);
    v.r[j] = axpy1<FA>(-alpha, sn, v.r[j]);
    v.w[j] = axpy1<FA>(-alpha, zn, v.w[j]);
    v.z[j] = zn;
    v.s[j] = sn;
    v.p[j] = pn;
  }
  if (fold) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (base + j < n) fold1(a.v.xhi, base + j, (double)v.x[j]);
      v.x[j] = (V)0;
    }
  }
  if (base + 8 <= n) {
    store8(P.z + base, v.z);
    store8(P.s + base, v.s);
    store8(P.p + base, v.p);
    store8(P.x + base, v.x);
    store8(P.r + base, v.r);
    store8(P.w + base, v.w);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = base + j;
      if (i < n) {
        P.z[i] = v.z[j];
        P.s[i] = v.s[j];
        P.p[i] = v.p[j];
        P.x[i] = v.x[j];
        P.r[i] = v.r[j];
        P.w[i] = v.w[j];
      }
    }
  }
}

// KS2 after a pipelined iteration's KS1: gamma, delta -> rho (replacement or
// budget test, except on the first iteration after a start or replacement),
// beta, alpha (breakdown test), then the updates of block blk.
template <int FA>
__device__ __forceinline__ SrNext pc2_iter(const SrArgs &a, const SrCtl &S, int blk, const double (&pg)[8],
                                           const double (&pd)[8], bool fast) {
  const int base = blk * kVecBlock + threadIdx.x * kVecPer;
  PcVals<FA> v;
  const bool live = base < a.A.n;
  __builtin_amdgcn_sched_barrier(0);
  if (live) pc_load<FA>(a, base, v);
  __builtin_amdgcn_sched_barrier(0);
  SrNext x = sr_next_of(S);
  const bool writer = blk == 0 && threadIdx.x == 0;
  const int k = S.k;
  const int fd = S.fd;
  const bool first = S.first != 0;
  const double gamma = fast ? tree_preloaded_rt(fd, pg) : reduce_partials_rt(fd, a.pg, a.P1);
  const double delta = fast ? tree_preloaded_rt(fd, pd) : reduce_partials_rt(fd, a.pd, a.P1);
  bool fold = false, go = true;
  if (!S.sync) {
    x.rho = sqrt(gamma) / S.bnorm;
    if (writer) a.h.rho[k] = x.rho;
    if (x.rho <= S.tol) {
      fold = true;
      x.mode = SR_RESID;
      go = false;
    } else if (k >= S.maxit) {
      x.status = 1;
      fold = true;
      x.mode = SR_FINAL;
      go = false;
    }
  }
  double alpha = 0.0, beta = 0.0;
  if (go) {
    beta = first ? 0.0 : gamma / S.gamma_old;
    const double den = first ? delta : delta - beta * gamma / S.alpha_old;
    alpha = gamma / den;
    if (!(den > 0.0) || !isfinite(alpha) || !isfinite(beta) || !isfinite(gamma)) {
      x.status = 3;
      fold = true;
      x.mode = SR_FINAL;
    } else {
      x.upd = true;
      x.sync = 0;
      x.gamma = gamma;
      x.alpha = alpha;
      if (writer) {
        a.h.act[k] = (uint8_t)S.action;
        a.h.flag[k] = 0;
      }
      x.k = k + 1;
      fold = S.R > 0 && x.k % S.R == 0;
      x.mode = fold ? SR_RESID : SR_ITER;
    }
  }
  if (live) {
    if (x.upd) {
      pc_update<FA>(a, base, v, alpha, beta, first, fold);
    } else if (fold) {
      const PcPtr<FA> P(a);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int i = base + j;
        if (i < a.A.n) {
          fold1(a.v.xhi, i, (double)v.x[j]);
          P.x[i] = (typename PcVals<FA>::V)0;
        }
      }
    }
  }
  return x;
}

// KS2 after a start, replacement or final check: the true relres and the
// stop tests; at the stop the caller's x receives x_hi (or 0 when b = 0).
__device__ __forceinline__ SrNext sr2_resid(const SrArgs &a, const SrCtl &S, int blk, const double (&pg)[8],
                                            const double (&pd)[8], bool fast) {
  SrNext x = sr_next_of(S);
  const bool writer = blk == 0 && threadIdx.x == 0;
  const int mode = S.mode, k = S.k;
  const double s64 = fast ? tree_preloaded<double>(pg) : partials_total<double>(a.pg, a.P1);
  if (mode == SR_START) x.bnorm = sqrt(fast ? tree_preloaded<double>(pd) : partials_total<double>(a.pd, a.P1));
  bool out = false;
  if (mode == SR_START && x.bnorm == 0.0) {
    x.zero = true;
    out = true;
    x.status = 0;
    x.relres = 0.0;
    x.mode = SR_DONE;
    if (writer) a.h.rho[0] = 0.0;
  } else {
    const double rt = sqrt(s64) / x.bnorm;
    if (mode == SR_FINAL) {
      x.relres = rt;
      out = true;
      x.mode = SR_DONE;
    } else {
      if (writer) {
        a.h.rho[k] = rt;
        if (mode == SR_RESID) {
          if (x.nrep < a.h.cap_rep) {
            a.h.rep_k[x.nrep] = k;
            a.h.rep_rho[x.nrep] = rt;
          }
          if (k > 0) a.h.flag[k - 1] |= FL_REPLACED;
        }
      }
      if (mode == SR_RESID) x.nrep++;
      x.last_true = rt;
      x.rho = rt;
      x.mode = S.pipe ? PC_W : SR_SYNC;
      if (rt <= S.tol || !isfinite(rt) || k >= S.maxit) {
        x.status = rt <= S.tol ? 0 : !isfinite(rt) ? 3 : 1;
        x.relres = rt;
        out = true;
        x.mode = SR_DONE;
      }
    }
  }
  if (out) {
    const int n = a.A.n;
    const int base = blk * kVecBlock + threadIdx.x * kVecPer;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (base + j < n) a.v.xout[base + j] = x.zero ? 0.0 : a.v.xhi[base + j];
  }
  return x;
}

// TIER: the container of the action's update format (a fixed action keeps
// one tier for the whole solve), so the fp32 kernel holds no fp64 operands;
// PIPE: the pipelined iteration.
template <int TIER, bool PIPE>
__global__ __launch_bounds__(kBlock) void k_sr2(SrArgs a) {
  __shared__ SrCtl S;
  const int blk = blockIdx.x;
  const bool fast = a.P1 <= kVecBlock;
  double pg[8] = {0, 0, 0, 0, 0, 0, 0, 0}, pd[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (fast) {
    preload_partials(a.pg, a.P1, pg);
    preload_partials(a.pd, a.P1, pd);
  }
  copy_words(&S, &a.ctl[a.par], sizeof(SrCtl));
  __syncthreads();
  const int mode = S.mode;
  SrNext x;
  if (PIPE && mode == SR_ITER) {
    if constexpr (PIPE) {
      if constexpr (TIER) {
        x = pc2_iter<FP64>(a, S, blk, pg, pd, fast);
      } else {
        switch (S.fa) {
        case FP16: x = pc2_iter<FP16>(a, S, blk, pg, pd, fast); break;
        case BF16: x = pc2_iter<BF16>(a, S, blk, pg, pd, fast); break;
        default: x = pc2_iter<FP32>(a, S, blk, pg, pd, fast); break;
        }
      }
    }
  } else if (PIPE && mode == PC_W) {
    x = sr_next_of(S);
    x.mode = SR_ITER;
    x.sync = 1;
  } else if (!PIPE && (mode == SR_ITER || mode == SR_SYNC)) {
    if constexpr (TIER) {
      x = sr2_iter<FP64>(a, S, blk, pg, pd, fast);
    } else {
      switch (S.fa) {
      case FP16: x = sr2_iter<FP16>(a, S, blk, pg, pd, fast); break;
      case BF16: x = sr2_iter<BF16>(a, S, blk, pg, pd, fast); break;
      default: x = sr2_iter<FP32>(a, S, blk, pg, pd, fast); break;
      }
    }
  } else if (mode == SR_START || mode == SR_RESID || mode == SR_FINAL) {
    x = sr2_resid(a, S, blk, pg, pd, fast);
  } else {
    x = sr_next_of(S);
  }
  __syncthreads();   // every thread has read S
  if (threadIdx.x == 0) {
    S.mode = x.mode;
    S.status = x.status;
    S.k = x.k;
    S.nrep = x.nrep;
    S.bnorm = x.bnorm;
    S.last_true = x.last_true;
    S.relres_true = x.relres;
    S.rho_new = x.rho;
    S.sync = x.sync;
    if (x.zero) S.zero_solution = 1;
    if (x.upd) {
      S.gamma_old = x.gamma;
      S.alpha_old = x.alpha;
      S.first = 0;
    }
  }
  __syncthreads();
  if (blk == 0) copy_words(&a.ctl[a.par ^ 1], &S, sizeof(SrCtl));
}

void launch_sr_slot(const SrArgs &a, hipStream_t s) {
  if (a.pipe) {
    hipLaunchKernelGGL(k_sr1<true>, dim3(a.G1), dim3(kBlock), 0, s, a);
    if (a.tier) hipLaunchKernelGGL((k_sr2<1, true>), dim3(a.P2), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_sr2<0, true>), dim3(a.P2), dim3(kBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_sr1<false>, dim3(a.G1), dim3(kBlock), 0, s, a);
    if (a.tier) hipLaunchKernelGGL((k_sr2<1, false>), dim3(a.P2), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_sr2<0, false>), dim3(a.P2), dim3(kBlock), 0, s, a);
  }
}
#undef MPCG_PC_CASES
#endif  // part 9

}  // namespace mpcg
