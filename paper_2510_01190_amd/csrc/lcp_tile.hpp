// Column-walking tile of the closed-form LCP (Eq. 2-3 and the level-crossing
// probability of Section 3.1), shared by the single-field kernel and the
// batched persistent kernel so that both give bitwise the same maps.
//
// A wave owns 127 vertex columns x0..x0+126, i.e. the 126 cells between
// them, over a band of cell rows.  Lane L holds two vertex columns, A = x0 + L
// and B = x0 + 63 + L (lane 63's A column repeats lane 0's B column), and
// walks down the band one vertex row at a time.  For each isovalue it
// evaluates each corner's tail once per row, pairs it with the previous row's
// (vertical pairs, kept in registers) and forms the cells (A, A+1) and
// (B, B+1), taking the right-hand pairs from lane L+1 by lane shuffles.  Lanes
// 0..62 store; each of the two stores writes 63 consecutive cells of one
// output row, which keeps the write stream contiguous (stride-2 lane patterns
// through buffer stores cost a factor of three in write bandwidth); stores
// are masked by their buffer record range, not by branches.  The next row's
// input loads are issued before the current row is computed.
#pragma once

#include "pdiv_device.hpp"
#include "pdiv_internal.hpp"

namespace pdiv {

constexpr int kWave = 64;
constexpr int kHalf = kWave - 1;          // cells per half-strip
constexpr int kCellsPerWave = 2 * kHalf;  // 126

// The values one vertex reads: for the fused path the U neighbours along x
// and the V neighbours along y of Eq. 2-3 (boundary-clamped), for the
// two-step path its divergence mean and variance.  Loading them is split from
// using them so that the next row's loads are in flight while the current
// row is computed.
template <bool FUSED>
struct Raw;
template <>
struct Raw<true> {
  float mu_l, mu_r, vu_l, vu_r, mv_l, mv_r, vv_l, vv_r;
};
template <>
struct Raw<false> {
  float mean, var;
};

// Row pointers are formed from the (wave-uniform) row index first, so each
// load is a scalar base plus a 32-bit per-lane column offset.
template <typename T>
__device__ __forceinline__ void load_raw(Raw<true>& r, const T* __restrict__ mu,
                                         const T* __restrict__ vu, const T* __restrict__ mv,
                                         const T* __restrict__ vv, int ny, int nx, uint32_t x,
                                         uint32_t xl, uint32_t xr, int j) {
  const int yl = j > 0 ? j - 1 : 0;
  const int yr = j < ny - 1 ? j + 1 : ny - 1;
  const int64_t r0 = static_cast<int64_t>(j) * nx;
  const int64_t rl = static_cast<int64_t>(yl) * nx;
  const int64_t rr = static_cast<int64_t>(yr) * nx;
  r.mu_l = to_f32(*at(mu + r0, xl));
  r.mu_r = to_f32(*at(mu + r0, xr));
  r.vu_l = to_f32(*at(vu + r0, xl));
  r.vu_r = to_f32(*at(vu + r0, xr));
  r.mv_l = to_f32(*at(mv + rl, x));
  r.mv_r = to_f32(*at(mv + rr, x));
  r.vv_l = to_f32(*at(vv + rl, x));
  r.vv_r = to_f32(*at(vv + rr, x));
}

template <typename T>
__device__ __forceinline__ void load_raw(Raw<false>& r, const T* __restrict__ dm,
                                         const T* __restrict__ dv, const T* __restrict__,
                                         const T* __restrict__, int, int nx, uint32_t x,
                                         uint32_t, uint32_t, int j) {
  const int64_t r0 = static_cast<int64_t>(j) * nx;
  r.mean = to_f32(*at(dm + r0, x));
  r.var = to_f32(*at(dv + r0, x));
}

// Eq. 2-3 at vertex (x, j) with the one-sided differences of Eq. 1 on the
// boundary (bx: x is a boundary column; j decides the y boundary).
__device__ __forceinline__ DivGauss raw_div(const Raw<true>& r, bool bx, int j, int ny,
                                            const StencilCoef& k) {
  const bool by = (j == 0) | (j == ny - 1);
  return div_gauss(r.mu_l, r.mu_r, r.vu_l, r.vu_r, r.mv_l, r.mv_r, r.vv_l, r.vv_r,
                   bx ? k.cxm_bd : k.cxm_in, bx ? k.cxv_bd : k.cxv_in,
                   by ? k.cym_bd : k.cym_in, by ? k.cyv_bd : k.cyv_in);
}
__device__ __forceinline__ DivGauss raw_div(const Raw<false>& r, bool, int, int,
                                            const StencilCoef&) {
  DivGauss g;
  g.mean = r.mean;
  g.var = r.var;
  return g;
}

// Neighbour columns of x for the x differences, clamped at the boundary.
struct Col {
  uint32_t x, xl, xr;
  bool bx;
};
__device__ __forceinline__ Col make_col(uint32_t x, int nx) {
  const uint32_t last = uint32_t(nx - 1);
  Col c;
  c.x = x;
  c.xl = x > 0 ? x - 1 : 0;
  c.xr = x < last ? x + 1 : last;
  c.bx = (x == 0) | (x == last);
  return c;
}

// Lane L receives lane L+1's value (DPP wave_shl:1; lane 63 receives 0 and
// stores nothing).  A register move in the vector ALU, no LDS round trip.
__device__ __forceinline__ float from_right(float v) {
  constexpr int kWaveShl1 = 0x130;
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), kWaveShl1, 0xf, 0xf, true));
}

__device__ __forceinline__ Pair pair_from_right(const Pair& p) {
  Pair r;
  r.pa = from_right(p.pa);
  r.qa = from_right(p.qa);
  r.pb = from_right(p.pb);
  r.qb = from_right(p.qb);
  return r;
}

// One vertex row step: the corners of row j+1 (from raw values loaded one
// step earlier) for the lane's two columns, their pairs with row j (prev_*),
// and the lane's two cells for every isovalue; the new corners go to next_*.
// off_a, off_b are the byte offsets of the lane's two cells within a row.
// LCP of the cell whose left column pair is p (this lane) and whose right
// column pair is lane L+1's p, read through the DPP operand of each
// instruction (wave_shl:1: lane L reads lane L+1):
//   up = (Qa + Pa Qa') - Pb Pb' = (1 - A) - B,  dn = (Qb + Pb Qb') - Pa Pa' = (1 - B) - A,
//   LCP = below ? dn : up   (below: integer mask, all ones if the reference corner is below).
// s_nop 1 gives the two wait states a DPP read needs after a VALU write of
// its source register.  qa and qb are consumed in place.
__device__ __forceinline__ float cell_lcp_dpp(Pair p, int below) {
  float l;
  asm volatile(
      "s_nop 1\n\t"
      "v_fmac_f32_dpp %1, %1, %3 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %2, %2, %4 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %1, -%4, %4 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %2, -%3, %3 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_bfi_b32 %0, %5, %2, %1"
      : "=v"(l), "+v"(p.qa), "+v"(p.qb)
      : "v"(p.pa), "v"(p.pb), "v"(below));
  return l;
}

template <int KC, bool FUSED>
__device__ __forceinline__ void row_step(const Raw<FUSED>& raw_a, const Raw<FUSED>& raw_b,
                                         const Col& ca_col, const Col& cb_col, int ny, int nx,
                                         const StencilCoef& k, const IsoChunk& iso,
                                         int n_store, float* __restrict__ out, int64_t plane,
                                         int j,
                                         uint32_t off_a, uint32_t off_b,
                                         const AB (&prev_a)[KC], const AB (&prev_b)[KC],
                                         AB (&next_a)[KC], AB (&next_b)[KC]) {
  const Corner ca = make_corner(raw_div(raw_a, ca_col.bx, j + 1, ny, k));
  const Corner cb = make_corner(raw_div(raw_b, cb_col.bx, j + 1, ny, k));
  float* __restrict__ orow = out + static_cast<int64_t>(j) * (nx - 1);
  const uint32_t row_bytes = uint32_t(nx - 1) * 4u;
#pragma unroll
  for (int q = 0; q < KC; ++q) {
    const AB cur_a = corner_probs(ca, iso.c[q]);
    const AB cur_b = corner_probs(cb, iso.c[q]);
    const Pair pa = make_pair(prev_a[q], cur_a);
    const Pair pb = make_pair(prev_b[q], cur_b);
    const float l0 = cell_lcp_dpp(pa, cur_a.below);
    const float l1 = cell_lcp_dpp(pb, cur_b.below);
    // planes past n_store (a batch's padding) get an empty record range
    const RowWriter w(orow + q * plane, q < n_store ? row_bytes : 0u);
    w.put(l0, off_a);
    w.put(l1, off_b);
    next_a[q] = cur_a;
    next_b[q] = cur_b;
  }
}

// One tile: cell columns [x0, x0+126) of strip `strip` (x0 = 126 strip),
// cell rows [j0, j1), for the KC isovalues in `iso`; only the first n_store
// isovalue planes are written (a batch pads its isovalue set to KC).  Must be
// called with wave-uniform arguments by all 64 lanes of a wave.
template <int KC, bool FUSED, typename T>
__device__ __forceinline__ void lcp_tile(const T* __restrict__ p0, const T* __restrict__ p1,
                                         const T* __restrict__ p2, const T* __restrict__ p3,
                                         int ny, int nx, const StencilCoef& k,
                                         const IsoChunk& iso, int n_store,
                                         float* __restrict__ out, int64_t plane, int strip,
                                         int j0, int j1) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t xa = uint32_t(strip * kCellsPerWave) + lane;  // A column
  const uint32_t xb = xa + kHalf;                               // B column
  const uint32_t last = uint32_t(nx - 1);
  const Col ca = make_col(xa < last ? xa : last, nx);  // columns past the edge load a
  const Col cb = make_col(xb < last ? xb : last, nx);  // valid column and store nothing
  // byte offsets of the lane's two cells in an output row; lane 63 and cells
  // past the right edge get an offset far beyond any row (rows are < 2^31
  // bytes), so the buffer hardware drops their stores
  constexpr uint32_t kDrop = 0x7ffffff0u;
  const uint32_t off_a = (lane < kHalf) & (xa < last) ? xa * 4u : kDrop;
  const uint32_t off_b = (lane < kHalf) & (xb < last) ? xb * 4u : kDrop;

  AB ra[KC], rb[KC], sa[KC], sb[KC];
  Raw<FUSED> xa0, xb0, xa1, xb1;
  load_raw(xa0, p0, p1, p2, p3, ny, nx, ca.x, ca.xl, ca.xr, j0);
  load_raw(xb0, p0, p1, p2, p3, ny, nx, cb.x, cb.xl, cb.xr, j0);
  load_raw(xa1, p0, p1, p2, p3, ny, nx, ca.x, ca.xl, ca.xr, j0 + 1);
  load_raw(xb1, p0, p1, p2, p3, ny, nx, cb.x, cb.xl, cb.xr, j0 + 1);
  {
    const Corner c0 = make_corner(raw_div(xa0, ca.bx, j0, ny, k));
    const Corner c1 = make_corner(raw_div(xb0, cb.bx, j0, ny, k));
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      ra[q] = corner_probs(c0, iso.c[q]);
      rb[q] = corner_probs(c1, iso.c[q]);
    }
  }
  // Two rows per trip: the carried corners alternate between two register
  // sets, and the raw loads of the row after next are issued before the next
  // row is computed.  A trip has no branches (the prefetch row is clamped to
  // the band's last row) and the first trip is peeled off the loop, so every
  // path into the loop body has the same loads and stores in flight and the
  // compiler waits for exactly the loads a row needs, never for the stores
  // of the row before.  An odd last row is done after the loop.
  auto trip = [&](int j) {
    load_raw(xa0, p0, p1, p2, p3, ny, nx, ca.x, ca.xl, ca.xr, j + 2);
    load_raw(xb0, p0, p1, p2, p3, ny, nx, cb.x, cb.xl, cb.xr, j + 2);
    row_step<KC, FUSED>(xa1, xb1, ca, cb, ny, nx, k, iso, n_store, out, plane, j, off_a,
                        off_b, ra, rb, sa, sb);
    const int jn = min(j + 3, j1);
    load_raw(xa1, p0, p1, p2, p3, ny, nx, ca.x, ca.xl, ca.xr, jn);
    load_raw(xb1, p0, p1, p2, p3, ny, nx, cb.x, cb.xl, cb.xr, jn);
    row_step<KC, FUSED>(xa0, xb0, ca, cb, ny, nx, k, iso, n_store, out, plane, j + 1, off_a,
                        off_b, sa, sb, ra, rb);
  };
  int j = j0;
  if (j + 2 <= j1) {
    trip(j);
    for (j += 2; j + 2 <= j1; j += 2) trip(j);
  }
  if (j < j1)  // xa1/xb1 hold row j + 1 == j1
    row_step<KC, FUSED>(xa1, xb1, ca, cb, ny, nx, k, iso, n_store, out, plane, j, off_a,
                        off_b, ra, rb, sa, sb);
}

}  // namespace pdiv
