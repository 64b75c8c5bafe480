// dev.hpp -- device building blocks for gfx950: format rounding, tier loads,
// pairwise (tree) reductions in a fixed order, and the scalar arithmetic of the
// precision policy.  Everything here is IEEE basic operations in a fixed order,
// so results are reproducible bit for bit.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace mpcg {

// Formats.  FP8 is Table 1's quarter precision q52 (5 exponent bits, 2
// fraction bits: the top byte of an fp16), used only as matrix storage.  TF32
// (section 5's format set) has fp32's exponent range and fp16's 11-bit
// significand; gfx950 has no tf32 arithmetic or storage, so its values are
// rounded to it and held in fp32 containers.
enum { FP16 = 0, BF16 = 1, FP32 = 2, FP64 = 3, FP8 = 4, TF32 = 5 };

// Actions.  0..63: 16 f_s + 4 f_d + f_a over {fp16, bf16, fp32, fp64};
// 64..79: a q52 SpMV with 4 f_d + f_a; 128..252: 128 + 25 d_s + 5 d_d + d_a
// over the digits {0: fp16, 1: bf16, 2: fp32, 3: fp64, 4: tf32} (an action
// without a tf32 digit keeps its 0..63 code).
__host__ __device__ inline int act_dig_fmt(int d) { return d == 4 ? TF32 : d; }
__host__ __device__ inline int act_fmt_dig(int f) { return f == TF32 ? 4 : f; }
__host__ __device__ inline int act_fs(int a) { return a < 64 ? (a >> 4) & 3 : a < 80 ? FP8 : act_dig_fmt((a - 128) / 25); }
__host__ __device__ inline int act_fd(int a) { return a < 80 ? (a >> 2) & 3 : act_dig_fmt(((a - 128) / 5) % 5); }
__host__ __device__ inline int act_fa(int a) { return a < 80 ? a & 3 : act_dig_fmt((a - 128) % 5); }
__host__ __device__ inline int act_compose(int ds, int dd, int da) {
  return (ds == 4 || dd == 4 || da == 4) ? 128 + 25 * ds + 5 * dd + da : 16 * ds + 4 * dd + da;
}
__host__ __device__ inline bool act_valid(int a) { return (a >= 0 && a < 80) || (a >= 128 && a <= 252); }

constexpr int kBlock = 256;          // threads per block, every kernel
constexpr int kWaves = kBlock / 64;  // 64-wide wavefronts
constexpr int kVecPer = 8;           // elements per thread in vector kernels
constexpr int kVecBlock = kBlock * kVecPer;   // 2048 elements per vector block
constexpr int kRowsPerBlock = kBlock;         // SpMV: one row per thread

// ---------------------------------------------------------------------------
// Round-to-nearest-even to a narrow binary format with T significand bits and
// exponent range [EMIN, EMAX] (Table 1), graded underflow, overflow to
// infinity, NaN/inf passed through.  Integer operations on the bit pattern.
// ---------------------------------------------------------------------------
template <int T, int EMIN, int EMAX>
__device__ __forceinline__ double round_narrow_f64(double x) {
  const uint64_t u = (uint64_t)__double_as_longlong(x);
  const uint64_t sign = u & 0x8000000000000000ull;
  const int e = (int)((u >> 52) & 0x7ff);
  if (e == 0x7ff) return x;
  if (e == 0) return __longlong_as_double((long long)sign);   // |x| < 2^-1022: rounds to 0
  const int E = e - 1023;
  const double inf = __longlong_as_double(0x7ff0000000000000ll);
  if (E > EMAX) return sign ? -inf : inf;
  const uint64_t M = (u & 0xFFFFFFFFFFFFFull) | 0x10000000000000ull;   // 53 bits
  const int qexp = (E < EMIN ? EMIN : E) - (T - 1);
  const int shift = qexp - (E - 52);
  if (shift >= 54) return __longlong_as_double((long long)sign);
  uint64_t q = M >> shift;
  const uint64_t rem = M & ((1ull << shift) - 1ull);
  const uint64_t half = 1ull << (shift - 1);
  if (rem > half || (rem == half && (q & 1ull))) q += 1ull;
  double y = ldexp((double)q, qexp);
  const double xmax = ldexp(2.0 - ldexp(1.0, 1 - T), EMAX);
  if (y > xmax) y = inf;
  return sign ? -y : y;
}

// fp32 source, fp16 target (32-bit integer path).
__device__ __forceinline__ float rd_f16_from_f32(float x) {
  const uint32_t u = __float_as_uint(x);
  const uint32_t sign = u & 0x80000000u;
  const int e = (int)((u >> 23) & 0xff);
  if (e == 0xff) return x;
  if (e == 0) return __uint_as_float(sign);        // fp32 subnormal: below fp16's range
  const int E = e - 127;
  if (E > 15) return __uint_as_float(sign | 0x7f800000u);
  const uint32_t M = (u & 0x7fffffu) | 0x800000u;  // 24 bits
  const int qexp = (E < -14 ? -14 : E) - 10;
  const int shift = qexp - (E - 23);
  if (shift >= 25) return __uint_as_float(sign);
  uint32_t q = M >> shift;
  const uint32_t rem = M & ((1u << shift) - 1u);
  const uint32_t half = 1u << (shift - 1);
  if (rem > half || (rem == half && (q & 1u))) q += 1u;
  float y = ldexpf((float)q, qexp);
  if (y > 65504.0f) y = __uint_as_float(0x7f800000u);
  return sign ? -y : y;
}

// fp32 source, bf16 target: bf16 shares fp32's exponent range, so RNE is a
// carry into bit 16 (subnormals included); inf/nan passed through.
__device__ __forceinline__ float rd_bf16_from_f32(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// fp32 source, tf32 target: fp32's exponent range with 11 significant bits,
// so RNE is a carry into bit 13 (subnormals included, overflow carries into
// the infinity pattern); inf/nan passed through.
__device__ __forceinline__ float rd_tf32_from_f32(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;
  u += 0xfffu + ((u >> 13) & 1u);
  return __uint_as_float(u & 0xffffe000u);
}

template <int F>
__device__ __forceinline__ float rd_from_f32(float x) {
  if constexpr (F == FP16) return rd_f16_from_f32(x);
  else if constexpr (F == BF16) return rd_bf16_from_f32(x);
  else if constexpr (F == TF32) return rd_tf32_from_f32(x);
  else return x;
}

template <int F>
__device__ __forceinline__ float rd_from_f64_to_f32(double x) {
  if constexpr (F == FP16) return (float)round_narrow_f64<11, -14, 15>(x);
  else if constexpr (F == BF16) return (float)round_narrow_f64<8, -126, 127>(x);
  else if constexpr (F == TF32) return (float)round_narrow_f64<11, -126, 127>(x);
  else return (float)x;   // v_cvt_f32_f64: RNE
}

// Runtime-format rounding of an fp64 value to format f, as a double (the
// paper's emulation reading rounds each operation's fp64 result).
__device__ __forceinline__ double rd_rt_f64(int f, double x) {
  switch (f) {
  case FP16: return round_narrow_f64<11, -14, 15>(x);
  case BF16: return round_narrow_f64<8, -126, 127>(x);
  case FP32: return (double)(float)x;
  case TF32: return round_narrow_f64<11, -126, 127>(x);
  default: return x;
  }
}

// Runtime-format rounding of an fp32 value (fp32 and fp64 formats: unchanged).
__device__ __forceinline__ float rd_rt_f32(int f, float t) {
  return f == FP16 ? rd_f16_from_f32(t) : f == BF16 ? rd_bf16_from_f32(t) : f == TF32 ? rd_tf32_from_f32(t) : t;
}

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float f16_bits_to_f32(uint16_t b) {
  _Float16 h = __builtin_bit_cast(_Float16, b);
  return (float)h;        // exact widening
}
// q52 bits: exactly the upper byte of the fp16 encoding of the same value.
__device__ __forceinline__ float q52_bits_to_f32(uint8_t b) { return f16_bits_to_f32((uint16_t)((uint16_t)b << 8)); }
__device__ __forceinline__ uint16_t f32_to_bf16_bits_exact(float x) {   // x already bf16-representable
  return (uint16_t)(__float_as_uint(x) >> 16);
}
__device__ __forceinline__ uint16_t f32_to_f16_bits_exact(float x) {    // x already fp16-representable
  _Float16 h = (_Float16)x;
  return __builtin_bit_cast(uint16_t, h);
}

// ---------------------------------------------------------------------------
// Tier containers: float (tier 0) or double (tier 1).
// ---------------------------------------------------------------------------
template <int TIER> struct TierT { using type = float; };
template <> struct TierT<1> { using type = double; };

template <int F> struct AccT { using type = float; };
template <> struct AccT<FP64> { using type = double; };

// Leaf of dot_f: rd_acc(rd_f(u) * rd_f(v)).
template <int FD, typename V>
__device__ __forceinline__ typename AccT<FD>::type dot_leaf(V u, V v) {
  if constexpr (FD == FP64) {
    return (double)u * (double)v;
  } else if constexpr (sizeof(V) == 4) {
    return rd_from_f32<FD>(u) * rd_from_f32<FD>(v);
  } else {
    return rd_from_f64_to_f32<FD>(u) * rd_from_f64_to_f32<FD>(v);
  }
}

// ---------------------------------------------------------------------------
// Pairwise reductions.  The whole vector is one recursive-halving tree over
// its zero-padded power-of-two length; any aligned power-of-two block of it is
// a subtree.  A thread holding an aligned chunk, a 64-lane tree that adds
// sibling subtrees (x + y = y + x bit for bit) and a fixed combination of the
// block's waves reproduce that tree exactly.
// ---------------------------------------------------------------------------
template <typename A>
__device__ __forceinline__ A tree8(const A (&l)[8]) {
  return ((l[0] + l[1]) + (l[2] + l[3])) + ((l[4] + l[5]) + (l[6] + l[7]));
}

// A DPP lane permutation (every source lane exists, so every lane is written).
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_value(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Tree over the 64 lanes, total in every lane.  Lane pairs, then pairs of
// pairs, are combined by quad permutations; quads within each 8-lane half-row
// by the half-row mirror (lane i <-> 7 - i); halves of each 16-lane row by the
// row mirror (i <-> 15 - i).  After each step every lane of a subtree holds its
// sum; the four row sums then combine as (r0 + r1) + (r2 + r3).
template <typename A>
__device__ __forceinline__ A wave_tree(A v) {
  v = v + dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]: lanes t, t ^ 1
  v = v + dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]: lanes t, t ^ 2
  v = v + dpp_move<0x141>(v);   // row_half_mirror
  v = v + dpp_move<0x140>(v);   // row_mirror
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Block of kBlock threads, each holding the sum of an aligned subtree of equal
// size, consecutive by thread index.  Returns the block subtree (all threads).
template <typename A>
__device__ __forceinline__ A block_tree(A v) {
  __shared__ A wsum[kWaves];
  v = wave_tree(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wsum[wave] = v;
  __syncthreads();
  A t = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
  __syncthreads();
  return t;
}

// Pairwise sum of P partials (P >= 1) by one block, as the tree over
// next_pow2(P) zero-padded leaves.  Segments of kVecBlock partials are aligned
// subtrees; their sums combine by recursive halving.
template <typename A>
__device__ A reduce_partials(const double *part, int P) {
  __shared__ A seg[64];
  int Pp = 1;
  while (Pp < P) Pp <<= 1;
  const int nseg = Pp <= kVecBlock ? 1 : Pp / kVecBlock;
  for (int s = 0; s < nseg; ++s) {
    A l[8];
    const int base = s * kVecBlock + threadIdx.x * kVecPer;
#pragma unroll
    for (int j = 0; j < 8; ++j) l[j] = (base + j < P) ? (A)part[base + j] : (A)0;
    A t = block_tree(tree8(l));
    if (threadIdx.x == 0) seg[s] = t;
  }
  __syncthreads();
  A total;
  if (threadIdx.x == 0) {
    for (int len = nseg; len > 1; len >>= 1)
      for (int i = 0; i < len / 2; ++i) seg[i] = seg[2 * i] + seg[2 * i + 1];
  }
  __syncthreads();
  total = seg[0];
  __syncthreads();
  return total;
}

// ---------------------------------------------------------------------------
// Policy arithmetic.
// ---------------------------------------------------------------------------
// Decimal logarithm: x = m 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s),
// s = (m-1)/(m+1), atanh(s) = s * sum_{j=0..11} s^{2j}/(2j+1) by Horner with fma.
__device__ inline double log10_policy(double x) {
  const double LN2 = 0.693147180559945309417232121458176568;
  const double LOG10E = 0.434294481903251827651128918916605082;
  const double SQRT_HALF = 0.707106781186547524400844362104849039;
  if (!(x > 0.0) || !isfinite(x)) return __longlong_as_double(0x7ff8000000000000ll);
  int e;
  double m = frexp(x, &e);
  if (m < SQRT_HALF) {
    m = m * 2.0;
    e = e - 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double s2 = s * s;
  double h = 1.0 / 23.0;
  for (int j = 10; j >= 0; --j) h = fma(h, s2, 1.0 / (double)(2 * j + 1));
  const double ln = fma((double)e, LN2, 2.0 * s * h);
  return ln * LOG10E;
}

// SplitMix64 output function (Steele, Lea, Flood 2014), chained as a counter hash.
__device__ __forceinline__ uint64_t splitmix_out(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double counter_uniform(uint64_t seed, uint64_t episode, uint64_t k,
                                                  uint64_t stream) {
  uint64_t h = splitmix_out(seed);
  h = splitmix_out(h ^ episode);
  h = splitmix_out(h ^ k);
  h = splitmix_out(h ^ stream);
  return (double)(h >> 11) * 0x1.0p-53;
}

// GELU (erf form), erf by Abramowitz & Stegun 7.1.28 (|error| <= 3e-7).
__device__ __forceinline__ float gelu_as(float x) {
  const float a1 = 0.0705230784f, a2 = 0.0422820123f, a3 = 0.0092705272f;
  const float a4 = 0.0001520143f, a5 = 0.0002765672f, a6 = 0.0000430638f;
  const float z = x * 0.70710678118654752f;
  const float t = fabsf(z);
  const float poly = fmaf(fmaf(fmaf(fmaf(fmaf(a6, t, a5), t, a4), t, a3), t, a2), t, a1);
  const float d = fmaf(poly, t, 1.0f);
  const float d2 = d * d, d4 = d2 * d2, d8 = d4 * d4, d16 = d8 * d8;
  float erfv = 1.0f - 1.0f / d16;
  if (z < 0.0f) erfv = -erfv;
  return 0.5f * x * (1.0f + erfv);
}

}  // namespace mpcg
