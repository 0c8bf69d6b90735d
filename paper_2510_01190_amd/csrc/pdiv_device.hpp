// Device helpers shared by the libpdiv kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <type_traits>

#include "tail_coeffs.hpp"

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

// Element idx of a row that starts at `row`, addressed as row + 32-bit byte
// offset: with a wave-uniform row pointer this is a scalar base plus a
// per-lane 32-bit offset, with no 64-bit address arithmetic per lane.
// Rows are at most 2^29 elements, so the byte offset fits in 32 bits.
template <typename T>
__device__ __forceinline__ T* at(T* row, uint32_t idx) {
  using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return reinterpret_cast<T*>(reinterpret_cast<B*>(row) + idx * uint32_t(sizeof(T)));
}

// Float stores through a buffer resource: `row` is wave-uniform (the
// descriptor lives in scalar registers), `byte_off` the per-lane offset, and
// the record count bounds the row: stores at byte offsets >= `bytes` are
// dropped by the buffer hardware, each dword checked on its own.  Lanes that
// must not store are pointed at an offset past any row, so the stores need
// no branch (a divergent branch around a store makes the compiler wait for
// every outstanding memory operation, stores included, before the next load
// can be used).  Descriptor word 3 is the raw 32-bit buffer format of
// gfx9-family targets.
//
// STREAM selects the streaming cache policy: non-temporal (nt) with the sc1
// scope bit.  It pays only when every store writes whole 128-byte lines
// (rows starting on a line): then the output, written once, does not push
// the input rows out of the caches.  Measured on gfx950, fused kernel at
// 8192^2, K = 16, rows interleaved by isovalue: 1.09 ms with sc1+nt, 1.14 ms
// with nt alone, 1.13-1.15 ms with sc1 or sc0+sc1 alone, 1.18 ms with the
// default policy.  Where rows start inside a line, neighbouring tiles write
// the two parts of the lines where rows meet, the parts merge in L2 only if
// the line stays there, and the default policy is the fastest (dense rows:
// 1.45 ms, against 1.99 ms with sc1 and 2.63 ms with sc1+nt).
template <bool STREAM>
struct RowWriter {
  static constexpr int kPolicy = STREAM ? 0x12 : 0;  // 0x12: sc1 | nt (0x10 | 0x2)
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ RowWriter(float* row, uint32_t bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(row, 0, static_cast<int>(bytes), 0x00020000)) {}
  __device__ __forceinline__ void put(float v, uint32_t byte_off) const {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, static_cast<int>(byte_off), 0,
                                          kPolicy);
  }
  // two consecutive floats; a pair whose second float lies past the row
  // stores the first
  __device__ __forceinline__ void put2(float lo, float hi, uint32_t byte_off) const {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 v = {__float_as_uint(lo), __float_as_uint(hi)};
    __builtin_amdgcn_raw_buffer_store_b64(v, r, static_cast<int>(byte_off), 0, kPolicy);
  }
};

// Lane L receives lane L-1's value (wave_shr:1) or lane L+1's (wave_shl:1);
// a lane with no source keeps its own.  The source lane must be active: call
// these outside lane-dependent branches (a DPP read inside one finds its
// partner lane switched off and returns the lane's own value).
__device__ __forceinline__ float dpp_from_left(float x) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_from_right(float x) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x), 0x130, 0xf, 0xf, false));
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
// smaller of the two is evaluated directly, Q = erfc(|mu - c| / (sigma sqrt 2))/2
// <= 1/2; the larger is 1 - Q, which has no cancellation since it is >= 1/2.
//
// Q comes from gauss_tail_scaled(): a branch-free fit (see gen_tail.py)
//   t = 1/(1 + KP y'),  Q = t 2^(-y'^2 + C(t)),  y' = |mu - c| sqrt(log2 e)/(sigma sqrt 2),
// one reciprocal, one base-2 exponential and nine fused multiply-adds.
// A corner with var == 0 is deterministic: its tail argument is made +inf
// (t = 0, Q = 0), so it is above iff mu >= c, at no extra cost per isovalue.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float gauss_tail_scaled(float y) {
  const float t = __builtin_amdgcn_rcpf(fmaf(tail::KP, y, 1.0f));
  float p = tail::C7;
  p = fmaf(p, t, tail::C6);
  p = fmaf(p, t, tail::C5);
  p = fmaf(p, t, tail::C4);
  p = fmaf(p, t, tail::C3);
  p = fmaf(p, t, tail::C2);
  p = fmaf(p, t, tail::C1);
  p = fmaf(p, t, tail::C0);
  return t * __builtin_amdgcn_exp2f(fmaf(-y, y, p));
}

struct Corner {
  float mean;  // mu
  float rs;    // sqrt(log2 e) / (sigma sqrt 2); 0 for a deterministic corner
  float z0;    // 0, or +inf for a deterministic corner
};

__device__ __forceinline__ Corner make_corner(DivGauss g) {
  constexpr float kTwoLn2 = 1.38629436112f;  // 2 ln 2 = 2 / log2(e)
  Corner c;
  c.mean = g.mean + 0.0f;  // -0 becomes +0 (the side test reads the sign bit)
  const bool det = (g.var == 0.0f);
  // The hardware reciprocal square root (rsqrtf wraps it in a rescaling of
  // tiny arguments that costs five more instructions per corner and row).
  // For normal arguments the result is the same; an argument too small for
  // it gives +inf, clamped to the largest float so that |mu - c| = 0 still
  // gives a tail argument of 0, not NaN.  A negative variance gives NaN,
  // which the clamp keeps and which then propagates to the LCP.
  const float r = __builtin_amdgcn_rsqf(g.var * kTwoLn2);
  constexpr float kMax = 3.40282347e38f;
  c.rs = det ? 0.0f : (r > kMax ? kMax : r);
  c.z0 = det ? __builtin_inff() : 0.0f;
  return c;
}

struct AB {
  float a, b;  // P(above), P(below)
  int below;   // all ones if mu < c, else 0
};

// Bitwise select (m & x) | (~m & y), one v_bfi_b32.  Written as an
// instruction because the compiler turns the mask expression back into a
// compare and two conditional moves.
__device__ __forceinline__ float bit_select(int m, float x, float y) {
  float r;
  asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(m), "v"(x), "v"(y));
  return r;
}

// The side test reads the sign bit of d = mu - c.  make_corner stores mu + 0
// (no -0), so mu == c gives d = +0: above, the >= rule.
__device__ __forceinline__ AB corner_probs(const Corner& k, float c) {
  const float d = k.mean - c;
  const float q = gauss_tail_scaled(fmaf(fabsf(d), k.rs, k.z0));
  const float s = 1.0f - q;
  AB p;
  p.below = __float_as_int(d) >> 31;
  p.a = bit_select(p.below, q, s);
  p.b = bit_select(p.below, s, q);
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
//   LCP = (1 - A) - B if some corner is above, else (1 - B) - A.
// `ref_below` is the side of any one corner of the cell.  For every corner k,
// LCP >= min(a_k, b_k) (fix the other three corners: the all-same-side mass is
// at most max(a_k, b_k)).  If corner k is above, B <= b_k <= LCP, so
// (1 - A) - B subtracts at most half of 1 - A and keeps its relative accuracy
// near 0; symmetrically when it is below.
__device__ __forceinline__ float cell_lcp(const Pair& L, const Pair& R, bool ref_below) {
  const float A = L.pa * R.pa;
  const float B = L.pb * R.pb;
  const float oneMinusA = fmaf(L.pa, R.qa, L.qa);
  const float oneMinusB = fmaf(L.pb, R.qb, L.qb);
  return ref_below ? (oneMinusB - A) : (oneMinusA - B);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011).  One round maps
// (x0,x1,x2,x3) with key (k0,k1) to (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2),
// hi(M0 x0) ^ x3 ^ k1, lo(M0 x0)); the key advances by (W0, W1) between rounds.
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t x, y, z, w;
};

// a ^ b ^ k with k wave-uniform, in one instruction: gfx950's three-input
// bitwise operation with truth table 0x96 (odd parity).  Left to itself the
// compiler issues two two-input xors here.
__device__ __forceinline__ uint32_t xor3_uniform(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
}

// The keys k0, k1 are wave-uniform (kernel arguments).
__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = static_cast<uint64_t>(M0) * c.x;
    uint64_t p1 = static_cast<uint64_t>(M1) * c.z;
    U4 n;
    n.x = xor3_uniform(static_cast<uint32_t>(p1 >> 32), c.y, k0);
    n.y = static_cast<uint32_t>(p1);
    n.z = xor3_uniform(static_cast<uint32_t>(p0 >> 32), c.w, k1);
    n.w = static_cast<uint32_t>(p0);
    c = n;
    k0 += W0;
    k1 += W1;
  }
  return c;
}

// Box-Muller (1958): u1 = (wa + 1) 2^-32 in (0, 1], u2 = wb 2^-32 in [0, 1);
// r = sqrt(-2 ln u1); (r cos 2 pi u2, r sin 2 pi u2).  The hardware sine and
// cosine take their argument in revolutions, so u2 is passed as is.  r is
// sqrt(-2 ln 2 log2 u1) with the hardware base-2 logarithm and square root:
// u1 >= 2^-32 and -2 ln u1 <= 44.4 are normal (or zero), so neither needs
// the library functions' rescaling of tiny arguments, which cost 14 more
// instructions per pair of normals.
struct F2 {
  float x, y;
};

__device__ __forceinline__ F2 box_muller(uint32_t wa, uint32_t wb) {
  constexpr float two_m32 = 2.3283064365386963e-10f;  // 2^-32
  float u1 = fmaf(static_cast<float>(wa), two_m32, two_m32);
  float u2 = static_cast<float>(wb) * two_m32;
  constexpr float kMinus2Ln2 = -1.38629436112f;  // -2 ln 2
  const float r = __builtin_amdgcn_sqrtf(kMinus2Ln2 * __builtin_amdgcn_logf(u1));
  F2 z;
  z.x = r * __builtin_amdgcn_cosf(u2);
  z.y = r * __builtin_amdgcn_sinf(u2);
  return z;
}

}  // namespace pdiv
