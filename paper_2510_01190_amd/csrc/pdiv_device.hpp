// Device helpers shared by the libpdiv kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace pdiv {

// ---------------------------------------------------------------------------
// Storage types.  Moment planes may be float32, float16 or bfloat16; all
// arithmetic is float32.  bfloat16 is handled as its raw 16 bits.
// ---------------------------------------------------------------------------
struct bf16_t {
  uint16_t bits;
};

__device__ __forceinline__ float to_f32(float x) { return x; }
__device__ __forceinline__ float to_f32(__half x) { return __half2float(x); }
__device__ __forceinline__ float to_f32(bf16_t x) {
  return __uint_as_float(static_cast<uint32_t>(x.bits) << 16);
}

template <typename T>
__device__ __forceinline__ T from_f32(float x);
template <>
__device__ __forceinline__ float from_f32<float>(float x) { return x; }
template <>
__device__ __forceinline__ __half from_f32<__half>(float x) { return __float2half_rn(x); }
template <>
__device__ __forceinline__ bf16_t from_f32<bf16_t>(float x) {
  // round to nearest even on the 16 dropped bits; NaN stays a quiet NaN
  uint32_t u = __float_as_uint(x);
  bf16_t r;
  if ((u & 0x7fffffffu) > 0x7f800000u) {
    r.bits = static_cast<uint16_t>((u >> 16) | 0x40u);
  } else {
    u += 0x7fffu + ((u >> 16) & 1u);
    r.bits = static_cast<uint16_t>(u >> 16);
  }
  return r;
}

template <typename T>
__device__ __forceinline__ float ld(const T* __restrict__ p, int64_t i) {
  return to_f32(p[i]);
}

// ---------------------------------------------------------------------------
// Eq. 2 and Eq. 3 at one vertex (Section 3.1).  The caller supplies the two
// U neighbours along x and the two V neighbours along y, already clamped at
// the boundary, and the matching coefficients: cxm = 1/(2dx) inside and 1/dx
// on the x boundary (one-sided difference), cxv = cxm^2; likewise cym, cyv.
// Contraction is off so every caller rounds the same way: the fused kernel
// and the two-step path give bitwise equal results.
// ---------------------------------------------------------------------------
struct DivGauss {
  float mean, var;
};

__device__ __forceinline__ DivGauss div_gauss(float mu_xl, float mu_xr, float var_xl,
                                              float var_xr, float mv_yl, float mv_yr,
                                              float var_yl, float var_yr, float cxm, float cxv,
                                              float cym, float cyv) {
#pragma clang fp contract(off)
  DivGauss g;
  float mx = (mu_xr - mu_xl) * cxm;
  float my = (mv_yr - mv_yl) * cym;
  float vx = (var_xr + var_xl) * cxv;
  float vy = (var_yr + var_yl) * cyv;
  g.mean = mx + my;
  g.var = vx + vy;
  return g;
}

// ---------------------------------------------------------------------------
// Per-corner Gaussian tails for the level-crossing probability.
//
// For a corner X ~ N(mu, var) and isovalue c the corner is above with
// probability a = P(X >= c) and below with b = P(X < c) = 1 - a.  Only the
// smaller of the two is evaluated directly, t = erfc(|c - mu| / (sigma sqrt 2))/2
// <= 1/2; the larger is 1 - t, which has no cancellation since it is >= 1/2.
// A corner with var == 0 is deterministic (t = 0, above iff mu >= c).
// ---------------------------------------------------------------------------
struct Corner {
  float mean;  // mu
  float r;     // 1 / (sigma sqrt 2); 0 for a deterministic corner
  bool det;    // var == 0
};

__device__ __forceinline__ Corner make_corner(DivGauss g) {
  Corner c;
  c.mean = g.mean;
  c.det = (g.var == 0.0f);
  // rsqrt of a negative variance is NaN, which then propagates to the LCP
  c.r = c.det ? 0.0f : __frsqrt_rn(2.0f * g.var);
  return c;
}

struct AB {
  float a, b;  // P(above), P(below)
};

__device__ __forceinline__ AB corner_probs(const Corner& k, float c) {
  float y = fabsf((c - k.mean) * k.r);
  float t = k.det ? 0.0f : 0.5f * erfcf(y);
  bool above = (k.mean >= c);
  float s = 1.0f - t;
  AB p;
  p.a = above ? s : t;
  p.b = above ? t : s;
  return p;
}

// Vertical pair of corners (lo = row j, hi = row j+1) of one column:
//   Pa = a_lo a_hi (both above), Qa = 1 - Pa = b_lo + a_lo b_hi, and the same
//   with a and b swapped.  Every term is non-negative, so Qa and Qb carry
//   full relative accuracy even when Pa or Pb is within rounding of 1.
struct Pair {
  float pa, qa, pb, qb;
};

__device__ __forceinline__ Pair make_pair(AB lo, AB hi) {
  Pair p;
  p.pa = lo.a * hi.a;
  p.qa = fmaf(lo.a, hi.b, lo.b);
  p.pb = lo.b * hi.b;
  p.qb = fmaf(lo.b, hi.a, lo.a);
  return p;
}

// LCP of the cell made of the left pair L and the right pair R:
//   A = Pa_L Pa_R (all above), 1 - A = Qa_L + Pa_L Qa_R, same for B (all below);
//   LCP = (1 - A) - B if A >= B, else (1 - B) - A.
// If A >= B some corner has a >= b, hence B <= b_k = min(a_k, b_k) <= LCP, so
// the subtraction loses at most a bit: relative accuracy holds near 0.
__device__ __forceinline__ float cell_lcp(const Pair& L, const Pair& R) {
  float A = L.pa * R.pa;
  float B = L.pb * R.pb;
  float oneMinusA = fmaf(L.pa, R.qa, L.qa);
  float oneMinusB = fmaf(L.pb, R.qb, L.qb);
  return (A >= B) ? (oneMinusA - B) : (oneMinusB - A);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011).  One round maps
// (x0,x1,x2,x3) with key (k0,k1) to (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2),
// hi(M0 x0) ^ x3 ^ k1, lo(M0 x0)); the key advances by (W0, W1) between rounds.
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = static_cast<uint64_t>(M0) * c.x;
    uint64_t p1 = static_cast<uint64_t>(M1) * c.z;
    U4 n;
    n.x = static_cast<uint32_t>(p1 >> 32) ^ c.y ^ k0;
    n.y = static_cast<uint32_t>(p1);
    n.z = static_cast<uint32_t>(p0 >> 32) ^ c.w ^ k1;
    n.w = static_cast<uint32_t>(p0);
    c = n;
    k0 += W0;
    k1 += W1;
  }
  return c;
}

// Box-Muller (1958): u1 = (wa + 1) 2^-32 in (0, 1], u2 = wb 2^-32 in [0, 1);
// r = sqrt(-2 ln u1); (r cos 2 pi u2, r sin 2 pi u2).  The hardware sine and
// cosine take their argument in revolutions, so u2 is passed as is.
struct F2 {
  float x, y;
};

__device__ __forceinline__ F2 box_muller(uint32_t wa, uint32_t wb) {
  constexpr float two_m32 = 2.3283064365386963e-10f;  // 2^-32
  float u1 = fmaf(static_cast<float>(wa), two_m32, two_m32);
  float u2 = static_cast<float>(wb) * two_m32;
  float r = __fsqrt_rn(-2.0f * __logf(u1));
  F2 z;
  z.x = r * __builtin_amdgcn_cosf(u2);
  z.y = r * __builtin_amdgcn_sinf(u2);
  return z;
}

}  // namespace pdiv
