// mlp.hip -- training of the MLP precision policy on gfx950 matrix cores.
//
// Network: 16 features -> 128 -> 128 -> 64 action values, GELU (erf form,
// Abramowitz & Stegun 7.1.28), as in the decision path of the solver.
// Training is fitted Q-iteration, the function-approximation form of the
// Q-learning update of section 4.1: targets y = r + gamma (1 - done) max_a
// Q_frozen(s', a) with the weights frozen at the start of each epoch, loss
// mean 1/2 (Q(s, a) - y)^2 on the taken action, Adam on fp32 master weights.
//
// Every product runs on v_mfma_f32_16x16x16_bf16: bfloat16 operands (features,
// weights, activations, and the gradient operands dY, dZ2, dZ1), fp32
// accumulation.  One workgroup (4 waves) takes 64 samples through the forward
// and backward passes with the activations in LDS and writes its partial
// weight gradients; a second kernel sums the partials in a fixed order and
// applies Adam, then refreshes the bfloat16 weight copies (row-major and
// transposed, so every matrix-core operand is read as 4 contiguous values).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev.hpp"
#include "mlp.hpp"

namespace mpcg {

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;   // samples per workgroup

__device__ __forceinline__ uint16_t bf16_bits(float x) { return (uint16_t)(__float_as_uint(rd_bf16_from_f32(x)) >> 16); }
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// GELU and its exact derivative (A&S 7.1.28 erf), fp32.
__device__ __forceinline__ void gelu_and_grad(float x, float &g, float &dg) {
  const float a1 = 0.0705230784f, a2 = 0.0422820123f, a3 = 0.0092705272f;
  const float a4 = 0.0001520143f, a5 = 0.0002765672f, a6 = 0.0000430638f;
  const float z = x * 0.70710678118654752f;
  const float t = fabsf(z);
  const float poly = fmaf(fmaf(fmaf(fmaf(fmaf(a6, t, a5), t, a4), t, a3), t, a2), t, a1);
  const float d = fmaf(poly, t, 1.0f);
  const float dd = fmaf(fmaf(fmaf(fmaf(fmaf(6.0f * a6, t, 5.0f * a5), t, 4.0f * a4), t, 3.0f * a3), t, 2.0f * a2), t, a1);
  const float d2 = d * d, d4 = d2 * d2, d8 = d4 * d4, d16 = d8 * d8;
  float erfv = 1.0f - 1.0f / d16;
  if (z < 0.0f) erfv = -erfv;
  g = 0.5f * x * (1.0f + erfv);
  const float derf = 16.0f * dd / (d16 * d);
  dg = 0.5f * (1.0f + erfv) + 0.5f * x * derf * 0.70710678118654752f;
}

__device__ __forceinline__ float4_t mfma(short4_t a, short4_t b, float4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Operand fetches for a 16x16x16 step.  Lane l: row/column l % 16, k block
// 4 (l / 16) .. + 3.
__device__ __forceinline__ short4_t ld4(const uint16_t *p) {   // 4 contiguous bf16 (8-byte aligned)
  const uint2 w = *(const uint2 *)p;
  short4_t r;
  r[0] = (short)(w.x & 0xffff); r[1] = (short)(w.x >> 16);
  r[2] = (short)(w.y & 0xffff); r[3] = (short)(w.y >> 16);
  return r;
}
__device__ __forceinline__ short4_t ld4s(const uint16_t *p, int stride) {   // 4 values, stride apart
  short4_t r;
  r[0] = (short)p[0]; r[1] = (short)p[stride]; r[2] = (short)p[2 * stride]; r[3] = (short)p[3 * stride];
  return r;
}

// LDS of the forward/backward kernel (64 samples).
struct MlpLds {
  uint16_t xb[kTile][kMlpIn];       // features, bf16
  uint16_t h1[kTile][kMlpH];        // GELU(Z1) bf16; later dZ1 bf16
  uint16_t h2[kTile][kMlpH];        // GELU(Z2) bf16
  float g1[kTile][kMlpH];           // GELU'(Z1); later dZ1 fp32
  float g2[kTile][kMlpH];           // GELU'(Z2); later dZ2 fp32
  uint16_t dy[kTile][kNAct];        // dY bf16
  uint16_t dz2[kTile][kMlpH];       // dZ2 bf16
  float q[kTile];                   // Q(s, a) of the taken action
  float diff[kTile];                // (Q - y) / B
};

// Forward of 64 samples through the three layers: h1, g1, h2, g2 in LDS;
// the action values Y go to y_out (global, may be NULL) and, for the taken
// action, to L.q (when act != NULL); when ymax != NULL the row maxima of Y.
__device__ void mlp_forward_tile(const MlpWeights &W, const float *feat, int s0, int n, MlpLds &L,
                                 const int32_t *act, float *y_out, float *ymax) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, kb = lane >> 4;
  for (int e = tid; e < kTile * kMlpIn; e += kBlock) {
    const int s = e / kMlpIn, i = e % kMlpIn;
    const float v = (s0 + s < n) ? feat[(size_t)(s0 + s) * kMlpIn + i] : 0.0f;
    L.xb[s][i] = bf16_bits(v);
  }
  __syncthreads();
  const int r0 = wave * 16;   // this wave's 16 samples
  // layer 1: Z1 = x W1^T + b1
  for (int nt = 0; nt < kMlpH / 16; ++nt) {
    float4_t c = {0.f, 0.f, 0.f, 0.f};
    c = mfma(ld4(&L.xb[r0 + li][4 * kb]), ld4(W.w1b + (nt * 16 + li) * kMlpIn + 4 * kb), c);
    const int col = nt * 16 + li;
    for (int r = 0; r < 4; ++r) {
      float g, dg;
      gelu_and_grad(c[r] + W.b1[col], g, dg);
      L.h1[r0 + 4 * kb + r][col] = bf16_bits(g);
      L.g1[r0 + 4 * kb + r][col] = dg;
    }
  }
  __syncthreads();
  // layer 2: Z2 = h1 W2^T + b2
  for (int nt = 0; nt < kMlpH / 16; ++nt) {
    float4_t c = {0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < kMlpH / 16; ++ks)
      c = mfma(ld4(&L.h1[r0 + li][16 * ks + 4 * kb]), ld4(W.w2b + (nt * 16 + li) * kMlpH + 16 * ks + 4 * kb), c);
    const int col = nt * 16 + li;
    for (int r = 0; r < 4; ++r) {
      float g, dg;
      gelu_and_grad(c[r] + W.b2[col], g, dg);
      L.h2[r0 + 4 * kb + r][col] = bf16_bits(g);
      L.g2[r0 + 4 * kb + r][col] = dg;
    }
  }
  __syncthreads();
  // layer 3: Y = h2 W3^T + b3
  float m[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int nt = 0; nt < kNAct / 16; ++nt) {
    float4_t c = {0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < kMlpH / 16; ++ks)
      c = mfma(ld4(&L.h2[r0 + li][16 * ks + 4 * kb]), ld4(W.w3b + (nt * 16 + li) * kMlpH + 16 * ks + 4 * kb), c);
    const int col = nt * 16 + li;
    for (int r = 0; r < 4; ++r) {
      const int s = r0 + 4 * kb + r;
      const float y = c[r] + W.b3[col];
      if (y_out && s0 + s < n) y_out[(size_t)(s0 + s) * kNAct + col] = y;
      if (act && s0 + s < n && (act[s0 + s] & (kNAct - 1)) == col) L.q[s] = y;
      m[r] = fmaxf(m[r], y);
    }
  }
  if (ymax) {
    // row maxima: each sample's 64 values sit in the 16 lanes of one k block
    for (int r = 0; r < 4; ++r) {
      float v = m[r];
      for (int off = 1; off < 16; off <<= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
      const int s = r0 + 4 * kb + r;
      if (li == 0 && s0 + s < n) ymax[s0 + s] = v;
    }
  }
}

// y_t = r_t + gamma (1 - done_t) max_a Q(next_t, a) with the given weights, or
// the raw action values when logits != NULL.
__global__ __launch_bounds__(kBlock) void k_mlp_forward(MlpWeights W, const float *feat, int n, float *logits,
                                                       const float *rew, const uint8_t *done, float gamma,
                                                       float *target, float *ymax_buf) {
  __shared__ MlpLds L;
  const int s0 = blockIdx.x * kTile;
  mlp_forward_tile(W, feat, s0, n, L, nullptr, logits, target ? ymax_buf : nullptr);
  if (target) {
    __syncthreads();
    for (int s = threadIdx.x; s < kTile; s += kBlock) {
      const int i = s0 + s;
      if (i < n) target[i] = rew[i] + gamma * (done[i] ? 0.0f : ymax_buf[i]);
    }
  }
}

// Forward + backward of 64 samples (batch of B samples starting at b0): the
// workgroup's partial gradients go to part[blockIdx.x][param], in the
// parameter order W1 | b1 | W2 | b2 | W3 | b3; its partial loss to
// part_loss[blockIdx.x].
__global__ __launch_bounds__(kBlock) void k_mlp_grad(MlpWeights W, const float *feat, const int32_t *act,
                                                    const float *target, int b0, int B, float *part,
                                                    float *part_loss) {
  __shared__ MlpLds L;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, kb = lane >> 4;
  const int s0 = b0 + blockIdx.x * kTile;
  const int n = b0 + B;
  mlp_forward_tile(W, feat, s0, n, L, act, nullptr, nullptr);
  for (int e = tid; e < kTile * kNAct; e += kBlock) L.dy[e / kNAct][e % kNAct] = 0;
  __syncthreads();
  float *g = part + (size_t)blockIdx.x * kMlpParams;
  float *gW1 = g, *gb1 = gW1 + kMlpH * kMlpIn, *gW2 = gb1 + kMlpH, *gb2 = gW2 + kMlpH * kMlpH;
  float *gW3 = gb2 + kMlpH, *gb3 = gW3 + kNAct * kMlpH;
  const float invB = 1.0f / (float)B;
  if (tid < kTile) {
    const int i = s0 + tid;
    const float d = (L.q[tid] - target[i]);
    L.diff[tid] = d * invB;
    L.dy[tid][act[i] & (kNAct - 1)] = bf16_bits(d * invB);
  }
  __syncthreads();
  if (tid == 0) {
    float l = 0.0f;
    for (int s = 0; s < kTile; ++s) {
      const float d = L.diff[s] * (float)B;
      l = fmaf(0.5f * d, d, l);
    }
    part_loss[blockIdx.x] = l * invB;
  }
  // db3: per action, the diffs of the samples that took it, in sample order
  for (int a = tid; a < kNAct; a += kBlock) {
    float sacc = 0.0f;
    for (int s = 0; s < kTile; ++s)
      if ((act[s0 + s] & (kNAct - 1)) == a) sacc += L.diff[s];
    gb3[a] = sacc;
  }
  // dW3[out][in] = dY^T h2 : M = 64 actions, N = 128, K = 64 samples
  for (int t = wave; t < (kNAct / 16) * (kMlpH / 16); t += 4) {
    const int mt = t / (kMlpH / 16), nt = t % (kMlpH / 16);
    float4_t c = {0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < kTile / 16; ++ks)
      c = mfma(ld4s(&L.dy[16 * ks + 4 * kb][mt * 16 + li], kNAct), ld4s(&L.h2[16 * ks + 4 * kb][nt * 16 + li], kMlpH), c);
    for (int r = 0; r < 4; ++r) gW3[(mt * 16 + 4 * kb + r) * kMlpH + nt * 16 + li] = c[r];
  }
  // dH2 = dY W3 : M = 64 samples, N = 128, K = 64 actions; dZ2 = dH2 GELU'(Z2)
  const int r0 = wave * 16;
  for (int nt = 0; nt < kMlpH / 16; ++nt) {
    float4_t c = {0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < kNAct / 16; ++ks)
      c = mfma(ld4(&L.dy[r0 + li][16 * ks + 4 * kb]), ld4(W.w3t + (nt * 16 + li) * kNAct + 16 * ks + 4 * kb), c);
    const int col = nt * 16 + li;
    for (int r = 0; r < 4; ++r) {
      const int s = r0 + 4 * kb + r;
      const float dz = c[r] * L.g2[s][col];
      L.g2[s][col] = dz;
      L.dz2[s][col] = bf16_bits(dz);
    }
  }
  __syncthreads();
  for (int j = tid; j < kMlpH; j += kBlock) {
    float sacc = 0.0f;
    for (int s = 0; s < kTile; ++s) sacc += L.g2[s][j];
    gb2[j] = sacc;
  }
  // dW2[j2][j1] = dZ2^T h1 : M = 128, N = 128, K = 64 samples
  for (int t = wave; t < (kMlpH / 16) * (kMlpH / 16); t += 4) {
    const int mt = t / (kMlpH / 16), nt = t % (kMlpH / 16);
    float4_t c = {0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < kTile / 16; ++ks)
      c = mfma(ld4s(&L.dz2[16 * ks + 4 * kb][mt * 16 + li], kMlpH), ld4s(&L.h1[16 * ks + 4 * kb][nt * 16 + li], kMlpH), c);
    for (int r = 0; r < 4; ++r) gW2[(mt * 16 + 4 * kb + r) * kMlpH + nt * 16 + li] = c[r];
  }
  __syncthreads();   // h1 is overwritten with dZ1 below
  // dH1 = dZ2 W2 : M = 64 samples, N = 128, K = 128; dZ1 = dH1 GELU'(Z1)
  for (int nt = 0; nt < kMlpH / 16; ++nt) {
    float4_t c = {0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < kMlpH / 16; ++ks)
      c = mfma(ld4(&L.dz2[r0 + li][16 * ks + 4 * kb]), ld4(W.w2t + (nt * 16 + li) * kMlpH + 16 * ks + 4 * kb), c);
    const int col = nt * 16 + li;
    for (int r = 0; r < 4; ++r) {
      const int s = r0 + 4 * kb + r;
      const float dz = c[r] * L.g1[s][col];
      L.g1[s][col] = dz;
      L.h1[s][col] = bf16_bits(dz);
    }
  }
  __syncthreads();
  for (int j = tid; j < kMlpH; j += kBlock) {
    float sacc = 0.0f;
    for (int s = 0; s < kTile; ++s) sacc += L.g1[s][j];
    gb1[j] = sacc;
  }
  // dW1[j1][i] = dZ1^T x : M = 128, N = 16, K = 64 samples
  for (int mt = wave; mt < kMlpH / 16; mt += 4) {
    float4_t c = {0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < kTile / 16; ++ks)
      c = mfma(ld4s(&L.h1[16 * ks + 4 * kb][mt * 16 + li], kMlpH), ld4s(&L.xb[16 * ks + 4 * kb][li], kMlpIn), c);
    for (int r = 0; r < 4; ++r) gW1[(mt * 16 + 4 * kb + r) * kMlpIn + li] = c[r];
  }
}

// bfloat16 copies (row-major and transposed) of parameter p in `dst`.
__device__ void mlp_store_copy(const MlpWeights &dst, int p, float w) {
  const int o1 = kMlpH * kMlpIn, o2 = o1 + kMlpH, o3 = o2 + kMlpH * kMlpH, o4 = o3 + kMlpH, o5 = o4 + kNAct * kMlpH;
  if (p < o1) {
    const int j = p / kMlpIn, i = p % kMlpIn;
    dst.w1b[j * kMlpIn + i] = bf16_bits(w);
  } else if (p < o2) {
    dst.b1[p - o1] = w;
  } else if (p < o3) {
    const int q = p - o2, j = q / kMlpH, i = q % kMlpH;
    dst.w2b[j * kMlpH + i] = bf16_bits(w);
    dst.w2t[i * kMlpH + j] = bf16_bits(w);
  } else if (p < o4) {
    dst.b2[p - o3] = w;
  } else if (p < o5) {
    const int q = p - o4, a = q / kMlpH, i = q % kMlpH;
    dst.w3b[a * kMlpH + i] = bf16_bits(w);
    dst.w3t[i * kNAct + a] = bf16_bits(w);
  } else {
    dst.b3[p - o5] = w;
  }
}

// Sums the partials of nwg workgroups in workgroup order; with adam != 0
// applies one Adam step to the fp32 master parameters (step t) and refreshes
// the bfloat16 copies; otherwise writes the summed gradient to grad_out.
__global__ __launch_bounds__(kBlock) void k_mlp_update(MlpState st, const float *part, const float *part_loss,
                                                      int nwg, int adam, int t, float lr, float b1, float b2,
                                                      float eps, float *grad_out, float *loss_out) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0 && loss_out) {
    float l = 0.0f;
    for (int w = 0; w < nwg; ++w) l += part_loss[w];
    *loss_out = l;
  }
  if (p >= kMlpParams) return;
  float gs = 0.0f;
  for (int w = 0; w < nwg; ++w) gs += part[(size_t)w * kMlpParams + p];
  if (!adam) {
    grad_out[p] = gs;
    return;
  }
  const float m = b1 * st.m[p] + (1.0f - b1) * gs;
  const float v = b2 * st.v[p] + (1.0f - b2) * gs * gs;
  st.m[p] = m;
  st.v[p] = v;
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  const float w = st.master[p] - lr * (m / c1) / (sqrtf(v / c2) + eps);
  st.master[p] = w;
  mlp_store_copy(st.cur, p, w);
}

// dst copies from fp32 parameters (initialisation, frozen copies).
__global__ __launch_bounds__(kBlock) void k_mlp_copies(MlpWeights dst, const float *params) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p < kMlpParams) mlp_store_copy(dst, p, params[p]);
}

void launch_mlp_copies(const MlpWeights &dst, const float *params, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_copies, dim3((kMlpParams + kBlock - 1) / kBlock), dim3(kBlock), 0, s, dst, params);
}

void launch_mlp_forward(const MlpWeights &W, const float *feat, int n, float *logits, const float *rew,
                        const uint8_t *done, float gamma, float *target, float *ymax_buf, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mlp_forward, dim3((n + kTile - 1) / kTile), dim3(kBlock), 0, s, W, feat, n, logits, rew,
                     done, gamma, target, ymax_buf);
}

void launch_mlp_grad(const MlpWeights &W, const float *feat, const int32_t *act, const float *target, int b0, int B,
                     float *part, float *part_loss, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_grad, dim3(B / kTile), dim3(kBlock), 0, s, W, feat, act, target, b0, B, part, part_loss);
}

void launch_mlp_update(const MlpState &st, const float *part, const float *part_loss, int nwg, int adam, int t,
                       float lr, float b1, float b2, float eps, float *grad_out, float *loss_out, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_update, dim3((kMlpParams + kBlock - 1) / kBlock), dim3(kBlock), 0, s, st, part, part_loss,
                     nwg, adam, t, lr, b1, b2, eps, grad_out, loss_out);
}

}  // namespace mpcg
