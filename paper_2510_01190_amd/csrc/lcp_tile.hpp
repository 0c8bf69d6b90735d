// Column-walking tiles of the closed-form LCP (Eq. 2-3 and the level-crossing
// probability of Section 3.1), shared by the single-field kernel and the
// batched persistent kernel so that both give bitwise the same maps.  A wave
// walks a strip of cells down a band of cell rows, one vertex row at a time:
// for each isovalue it evaluates each corner's tail once per row, pairs it
// with the previous row's (vertical pairs, kept in registers) and forms the
// cells from the pairs of neighbouring columns, read from the lane to the
// right through DPP.  The next row's input loads are issued before the
// current row is computed, and stores are masked by their buffer record range
// (checked per dword), not by branches.  Two strip layouts, the same
// arithmetic (so the same bits), and two store policies for the paired one:
//
// Paired (lcp_tile_paired), for outputs whose rows start on 128-byte lines: a
// wave owns the 128 cells [x0, x0+128), x0 = 128 strip, i.e. vertex columns
// x0..x0+128.  Lane L holds the adjacent columns E = x0+2L and O = x0+2L+1,
// forms cell 2L from its own two columns and cell 2L+1 from O and lane L+1's
// E, and writes both with one 8-byte store: one store instruction covers 512
// contiguous bytes, whole lines.  The 129th column x0+128, right neighbour of
// lane 63's last cell, belongs to no lane: a seam step per row has lanes 2q
// and 2q+1 evaluate columns x0+127 and x0+128 at isovalue q, lane 2q forms
// cell x0+127 for isovalue q with the same arithmetic, and lane 63 takes it
// over with one readlane/writelane per isovalue (about 7% more vector ALU
// work at 16 isovalues).  On gfx950 such stores sustain about 5.4 TB/s.
//
// The fused kernel also takes the paired tile for rows that start inside a
// line (dense [K][ny-1][nx-1] maps, odd pitches), with the default store
// policy: a strip's 8-byte stores then fill the lines in its middle and leave
// the two lines it shares with the neighbouring strips to be completed in L2
// by the neighbour (XCD-contiguous strips share an L2).  It runs the same
// arithmetic with the LDS-staged rows, launched at two waves per SIMD (the
// launcher reserves LDS: fewer waves writing at once complete more shared
// lines in L2); at 8192^2 into dense maps it takes 0.46 / 0.73 / 1.35 ms at
// 4 / 8 / 16 isovalues (0.50 / 0.80 / 1.455 ms at three waves per SIMD)
// against 0.40 / 0.66 / 1.07 ms into line-aligned rows (with the streaming
// policy 0.578 / 0.974 / 1.760 ms at three waves; the split tile 1.51 ms at
// 16).
//
// Split (lcp_tile_split), for the other outputs (the two-step path on rows
// that start inside a line, and small maps with few isovalues, where a
// launch's fixed cost dominates and is lower for this tile: use_paired_tile
// below): a wave owns 127 vertex columns, the 126 cells [x0, x0+126),
// x0 = 126 strip.  Lane L holds columns A = x0+L and B = x0+63+L (lane 63's
// A repeats lane 0's B), forms cells (A, A+1) and (B, B+1) with the right
// pair from lane L+1, and lanes 0..62 write 63 consecutive cells per store.
// No seam step.
#pragma once

#include "pdiv_device.hpp"
#include "pdiv_internal.hpp"

namespace pdiv {

constexpr int kWave = 64;
constexpr int kPairedCells = 2 * kWave;     // 128 cells per wave
constexpr int kSplitHalf = kWave - 1;       // 63 cells per half-strip
constexpr int kSplitCells = 2 * kSplitHalf; // 126 cells per wave
__host__ __device__ constexpr int cells_per_wave(bool paired) {
  return paired ? kPairedCells : kSplitCells;
}

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

// Neighbour columns of x for the x differences, clamped at the boundary, as
// byte offsets into a row of elements of `size` bytes.
struct Col {
  uint32_t x, xl, xr;  // byte offsets
  bool bx;             // x is a boundary column
};
__device__ __forceinline__ Col make_col(uint32_t x, int nx, uint32_t size) {
  const uint32_t last = uint32_t(nx - 1);
  Col c;
  c.x = x * size;
  c.xl = (x > 0 ? x - 1 : 0) * size;
  c.xr = (x < last ? x + 1 : last) * size;
  c.bx = (x == 0) | (x == last);
  return c;
}

// Input rows are read through buffer resources: the row base lives in
// scalar registers and each lane supplies its column's 32-bit byte offset,
// which is fixed for the whole walk, so a load needs no per-lane 64-bit
// address arithmetic (and no address registers).
template <typename T>
struct RowReader {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ RowReader(const T* row, int nx)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(row), 0,
                                            static_cast<int>(uint32_t(nx) * sizeof(T)),
                                            0x00020000)) {}
  // byte_off: per lane; so: a wave-uniform byte offset added to it
  __device__ __forceinline__ float get(uint32_t byte_off, uint32_t so = 0) const;
};
template <>
__device__ __forceinline__ float RowReader<float>::get(uint32_t o, uint32_t so) const {
  return __uint_as_float(
      __builtin_amdgcn_raw_buffer_load_b32(r, static_cast<int>(o), static_cast<int>(so), 0));
}
template <>
__device__ __forceinline__ float RowReader<__half>::get(uint32_t o, uint32_t so) const {
  return __half2float(__ushort_as_half(
      __builtin_amdgcn_raw_buffer_load_b16(r, static_cast<int>(o), static_cast<int>(so), 0)));
}
template <>
__device__ __forceinline__ float RowReader<bf16_t>::get(uint32_t o, uint32_t so) const {
  return __uint_as_float(static_cast<uint32_t>(__builtin_amdgcn_raw_buffer_load_b16(
                             r, static_cast<int>(o), static_cast<int>(so), 0))
                         << 16);
}

template <typename T>
__device__ __forceinline__ void load_raw(Raw<true>& r, const T* __restrict__ mu,
                                         const T* __restrict__ vu, const T* __restrict__ mv,
                                         const T* __restrict__ vv, int ny, int nx,
                                         const Col& c, int j) {
  const int yl = j > 0 ? j - 1 : 0;
  const int yr = j < ny - 1 ? j + 1 : ny - 1;
  const RowReader<T> u0(mu + static_cast<int64_t>(j) * nx, nx);
  const RowReader<T> w0(vu + static_cast<int64_t>(j) * nx, nx);
  const RowReader<T> ul(mv + static_cast<int64_t>(yl) * nx, nx);
  const RowReader<T> ur(mv + static_cast<int64_t>(yr) * nx, nx);
  const RowReader<T> wl(vv + static_cast<int64_t>(yl) * nx, nx);
  const RowReader<T> wr(vv + static_cast<int64_t>(yr) * nx, nx);
  r.mu_l = u0.get(c.xl);
  r.mu_r = u0.get(c.xr);
  r.vu_l = w0.get(c.xl);
  r.vu_r = w0.get(c.xr);
  r.mv_l = ul.get(c.x);
  r.mv_r = ur.get(c.x);
  r.vv_l = wl.get(c.x);
  r.vv_r = wr.get(c.x);
}

template <typename T>
__device__ __forceinline__ void load_raw(Raw<false>& r, const T* __restrict__ dm,
                                         const T* __restrict__ dv, const T* __restrict__,
                                         const T* __restrict__, int, int nx, const Col& c,
                                         int j) {
  r.mean = RowReader<T>(dm + static_cast<int64_t>(j) * nx, nx).get(c.x);
  r.var = RowReader<T>(dv + static_cast<int64_t>(j) * nx, nx).get(c.x);
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


// Cell LCP from the vertical pairs of its left (l) and right (r) columns:
//   1 - A = Qa_l + Pa_l Qa_r,  1 - B = Qb_l + Pb_l Qb_r,  A = Pa_l Pa_r,  B = Pb_l Pb_r,
//   LCP = below ? (1 - B) - A : (1 - A) - B
// (below: integer mask, all ones if the cell's reference corner, the left
// column's corner in the lower row of the walk, is below the isovalue).  The
// form subtracts the product that is at most the smaller tail, so the result
// keeps its relative accuracy for LCP near 0 and near 1.
__device__ __forceinline__ float cell_lcp_local(const Pair& l, const Pair& r, int below) {
  float ua = fmaf(l.pa, r.qa, l.qa);
  float ub = fmaf(l.pb, r.qb, l.qb);
  ua = fmaf(-l.pb, r.pb, ua);
  ub = fmaf(-l.pa, r.pa, ub);
  return bit_select(below, ub, ua);
}

// The same cell formula with the right column in lane L+1, read through the
// DPP operand of each instruction (wave_shl:1: lane L reads lane L+1; lane
// 63 has no source lane and leaves its result undefined).  cell_lcp_dpp reads
// the right pair from the same registers as the left (the seam step);
// cell_lcp_dpp_next takes the left pair from this lane's O column (o) and
// the right one from lane L+1's E column (e).
// s_nop 1 gives the two wait states a DPP read needs after a VALU write of
// its source register.  The left pair's qa and qb are consumed in place.
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

__device__ __forceinline__ float cell_lcp_dpp_next(Pair o, const Pair& e, int below) {
  float l;
  asm volatile(
      "s_nop 1\n\t"
      "v_fmac_f32_dpp %1, %3, %5 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %2, %4, %6 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %1, -%7, %6 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %2, -%8, %5 wave_shl:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_bfi_b32 %0, %9, %2, %1"
      : "=v"(l), "+v"(o.qa), "+v"(o.qb)
      : "v"(e.qa), "v"(e.qb), "v"(o.pa), "v"(o.pb), "v"(e.pb), "v"(e.pa), "v"(below));
  return l;
}

// v with lane 63 replaced by the wave-uniform value s (v_writelane_b32; the
// lane select is an inline constant, so the SGPR written by the readlane
// that produces s is only a data operand and needs no wait states).
__device__ __forceinline__ float to_lane63(float v, int s) {
  asm("v_writelane_b32 %0, %1, 63" : "+v"(v) : "s"(s));
  return v;
}

// Corner probabilities carried from one vertex row to the next, per
// isovalue: the lane's columns E and O and its seam column (paired layout).
template <int KC>
struct PairedCarry {
  AB e[KC], o[KC], s;
};

// Paired layout, the cells of one row step: given the corners of row j+1 for
// the lane's columns E and O and its seam column, their pairs with row j
// (prev_*; row j+1's corner probabilities go to next_*), and the lane's two
// cells for every isovalue.  prev and next may be the same set (updated in
// place: a register move per carried value and row, since the old and new
// values are live together) or two sets that the walk alternates (no moves,
// more registers).  off is the byte offset of the lane's first cell within an
// output row.
template <int KC, bool STREAM>
__device__ __forceinline__ void row_cells_paired(const Corner& ke, const Corner& ko,
                                                 const Corner& ks, const IsoChunk& iso,
                                                 float c_seam, int n_store,
                                                 float* __restrict__ out, int64_t plane,
                                                 int64_t pitch, uint32_t row_bytes, int j,
                                                 uint32_t off, const AB (&prev_e)[KC],
                                                 const AB (&prev_o)[KC], const AB& prev_s,
                                                 AB (&next_e)[KC], AB (&next_o)[KC],
                                                 AB& next_s) {
  // seam: lane 2q holds cell x0+127 at isovalue q
  const AB cur_s = corner_probs(ks, c_seam);
  const float seam = cell_lcp_dpp(make_pair(prev_s, cur_s), cur_s.below);
  next_s = cur_s;
  float* __restrict__ orow = out + static_cast<int64_t>(j) * pitch;
#pragma unroll
  for (int q = 0; q < KC; ++q) {
    const AB cur_e = corner_probs(ke, iso.c[q]);
    const AB cur_o = corner_probs(ko, iso.c[q]);
    const Pair pe = make_pair(prev_e[q], cur_e);
    const Pair po = make_pair(prev_o[q], cur_o);
    const float l_e = cell_lcp_local(pe, po, cur_e.below);
    float l_o = cell_lcp_dpp_next(po, pe, cur_o.below);
    l_o = to_lane63(l_o, __builtin_amdgcn_readlane(__float_as_int(seam), 2 * q));
    // planes past n_store (a batch's padding) get an empty record range
    const RowWriter<STREAM> w(orow + q * plane, q < n_store ? row_bytes : 0u);
    w.put2(l_e, l_o, off);
    next_e[q] = cur_e;
    next_o[q] = cur_o;
    // Keep the isovalues in order: left alone the scheduler evaluates the
    // tails of later isovalues early and holds them, which costs 25 VGPRs
    // and the third wave per SIMD.
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Paired layout, one vertex row step from raw values loaded earlier.
template <int KC, bool FUSED, bool STREAM>
__device__ __forceinline__ void row_step_paired(const Raw<FUSED>& raw_e, const Raw<FUSED>& raw_o,
                                                const Raw<FUSED>& raw_s, const Col& ce,
                                                const Col& co, const Col& cs, int ny,
                                                const StencilCoef& k, const IsoChunk& iso,
                                                float c_seam, int n_store,
                                                float* __restrict__ out, int64_t plane,
                                                int64_t pitch, uint32_t row_bytes, int j,
                                                uint32_t off, const AB (&prev_e)[KC],
                                                const AB (&prev_o)[KC], const AB& prev_s,
                                                AB (&next_e)[KC], AB (&next_o)[KC], AB& next_s) {
  row_cells_paired<KC, STREAM>(make_corner(raw_div(raw_e, ce.bx, j + 1, ny, k)),
                               make_corner(raw_div(raw_o, co.bx, j + 1, ny, k)),
                               make_corner(raw_div(raw_s, cs.bx, j + 1, ny, k)), iso, c_seam,
                               n_store, out, plane, pitch, row_bytes, j, off, prev_e, prev_o,
                               prev_s, next_e, next_o, next_s);
}

// Paired tile: cell columns [x0, x0+128) of strip `strip` (x0 = 128 strip),
// cell rows [j0, j1), for the KC isovalues in `iso`; only the first n_store
// isovalue planes are written (a batch pads its isovalue set to KC).  Output
// row j of plane q starts at out + q plane + j pitch.  Must be called with
// wave-uniform arguments by all 64 lanes of a wave; KC <= 32.  STREAM: store
// with the non-temporal policy (for outputs whose rows start on 128-byte lines).
template <int KC, bool FUSED, bool STREAM, typename T>
__device__ __forceinline__ void lcp_tile_paired(const T* __restrict__ p0, const T* __restrict__ p1,
                                         const T* __restrict__ p2, const T* __restrict__ p3,
                                         int ny, int nx, const StencilCoef& k,
                                         const IsoChunk& iso, int n_store,
                                         float* __restrict__ out, int64_t plane, int64_t pitch,
                                         int strip, int j0, int j1) {
  static_assert(2 * KC <= kWave, "the seam step needs two lanes per isovalue");
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t last = uint32_t(nx - 1);                      // also the cell count
  const uint32_t xe = uint32_t(strip) * kPairedCells + 2 * lane;  // E column
  const uint32_t xs = uint32_t(strip) * kPairedCells + (kPairedCells - 1) + (lane & 1);
  // columns past the edge load a valid column and store nothing
  const Col ce = make_col(min(xe, last), nx, sizeof(T));
  const Col co = make_col(min(xe + 1, last), nx, sizeof(T));
  const Col cs = make_col(min(xs, last), nx, sizeof(T));
  // cells past the right edge: an offset beyond any row (rows are < 2^31
  // bytes) drops the store; the record range drops a lone second cell
  constexpr uint32_t kDrop = 0x7ffffff0u;
  const uint32_t off = xe < last ? xe * 4u : kDrop;
  const uint32_t row_bytes = last * 4u;
  // isovalue of the lane's seam evaluation: q = L / 2
  const int qs = min(int(lane >> 1), KC - 1);
  float c_seam = iso.c[0];
#pragma unroll
  for (int q = 1; q < KC; ++q) c_seam = (qs == q) ? iso.c[q] : c_seam;

  // corner probabilities of the walk's current vertex row, two alternating sets
  PairedCarry<KC> ca, cb;
  Raw<FUSED> e0, o0, s0, e1, o1, s1;
  auto load3 = [&](Raw<FUSED>& re, Raw<FUSED>& ro, Raw<FUSED>& rs_, int j) {
    load_raw(re, p0, p1, p2, p3, ny, nx, ce, j);
    load_raw(ro, p0, p1, p2, p3, ny, nx, co, j);
    load_raw(rs_, p0, p1, p2, p3, ny, nx, cs, j);
  };
  auto step = [&](const Raw<FUSED>& re, const Raw<FUSED>& ro, const Raw<FUSED>& rs_, int j,
                  const PairedCarry<KC>& prev, PairedCarry<KC>& next) {
    row_step_paired<KC, FUSED, STREAM>(re, ro, rs_, ce, co, cs, ny, k, iso, c_seam, n_store,
                                       out, plane, pitch, row_bytes, j, off, prev.e, prev.o,
                                       prev.s, next.e, next.o, next.s);
  };
  load3(e0, o0, s0, j0);
  load3(e1, o1, s1, j0 + 1);
  {
    const Corner c0 = make_corner(raw_div(e0, ce.bx, j0, ny, k));
    const Corner c1 = make_corner(raw_div(o0, co.bx, j0, ny, k));
    const Corner c2 = make_corner(raw_div(s0, cs.bx, j0, ny, k));
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      ca.e[q] = corner_probs(c0, iso.c[q]);
      ca.o[q] = corner_probs(c1, iso.c[q]);
    }
    ca.s = corner_probs(c2, c_seam);
  }
  // Two rows per trip: the raw loads of the row after next are issued before
  // the next row is computed.  A trip has no branches (the prefetch row is
  // clamped to the band's last row) and the first trip is peeled off the
  // loop, so every path into the loop body has the same loads and stores in
  // flight and the compiler waits for exactly the loads a row needs, never
  // for the stores of the row before.  An odd last row is done after the loop.
  auto trip = [&](int j) {
    load3(e0, o0, s0, j + 2);
    step(e1, o1, s1, j, ca, cb);
    load3(e1, o1, s1, min(j + 3, j1));
    step(e0, o0, s0, j + 1, cb, ca);
  };
  int j = j0;
  if (j + 2 <= j1) {
    trip(j);
    for (j += 2; j + 2 <= j1; j += 2) trip(j);
  }
  if (j < j1) step(e1, o1, s1, j, ca, cb);  // e1.. hold row j + 1 == j1
}

// ---------------------------------------------------------------------------
// Paired tile, fused: input rows staged through LDS.
//
// The fused tile needs, per vertex row, the four moment planes over the strip's
// columns x0-1 .. x0+129 (x differences and the seam).  Instead of per-lane
// loads into registers, each row is copied once into a per-wave LDS ring by
// direct memory-to-LDS loads (buffer_load ... lds: 64 lanes x 4 bytes per
// instruction, 3 per plane and row), kRingRows - 3 = 2 row steps ahead of
// its first use, and the stencil values are read from LDS.  This takes the
// in-flight rows out of the vector registers (three waves per SIMD instead of
// two) and deepens the prefetch.  Slot layout (dwords): array a (mu, var_u,
// mv, var_v) index i = column - (x0 - 1) at 132 a + i, i < 131; the third
// load of a plane runs on lanes 0..2 only.  With one stride per plane, a
// lane reads every plane at one base address plus immediate offsets.  A
// 16-bit element loads the same way
// (each lane still writes one dword, the value zero-extended), so the layout
// does not depend on the storage type.
//
// The compiler does not order these loads with later LDS reads, so each step
// waits explicitly (s_waitcnt vmcnt) for the one row it is about to read.
// Every step issues the same memory operations in the same order (12 row
// loads, then KC stores), so the count of operations issued after a given row
// load is a constant: a row read at step j was loaded at step j - 2, followed
// by 2 KC + 24 operations (KC <= 16 keeps this within the counter's 63).
// ---------------------------------------------------------------------------
constexpr int kRingRows = 5;
constexpr int kPlaneStride = 132;  // dwords per plane in a slot (131 used)
constexpr int kSlotFloats = 4 * kPlaneStride;
constexpr int kRowLoads = 12;      // memory-to-LDS loads per staged row
constexpr int kTileWaves = 4;  // waves per block of the kernels that run tiles

typedef __attribute__((address_space(3))) float lds_float;
typedef __attribute__((address_space(3))) char lds_char;

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}


typedef __attribute__((address_space(3))) uint32_t lds_u32;

// One memory-to-LDS load of an element of B bytes per lane (the builtins
// take the size as a literal).
template <int B>
__device__ __forceinline__ void load_to_lds(__amdgpu_buffer_rsrc_t r, lds_float* dst,
                                            uint32_t voff) {
  if constexpr (B == 4)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, dst, 4, voff, 0, 0, 0);
  else
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, dst, 2, voff, 0, 0, 0);
}

// ring entry at byte offset off as float32 (a 16-bit element sits in the low
// half of its dword)
template <typename T>
__device__ __forceinline__ float lds_at(const lds_char* base, uint32_t off) {
  const uint32_t w = *reinterpret_cast<const lds_u32*>(base + off);
  if constexpr (std::is_same<T, float>::value)
    return __uint_as_float(w);
  else if constexpr (std::is_same<T, __half>::value)
    return __half2float(__ushort_as_half(static_cast<unsigned short>(w)));
  else
    return __uint_as_float(w << 16);
}

// POISON (a checking mode, pdiv_set_debug): every ring slot is filled with
// NaN before its row's loads are issued, so a step that read its rows before
// the loads had landed (a wait count too lax for the code the compiler made)
// would see NaN, which reaches the map, instead of an older row's values.
template <int KC, bool STREAM, typename T, bool POISON = false>
__device__ __forceinline__ void lcp_tile_paired_lds(const T* __restrict__ mu,
                                                    const T* __restrict__ vu,
                                                    const T* __restrict__ mv,
                                                    const T* __restrict__ vv, int ny, int nx,
                                                    const StencilCoef& k, const IsoChunk& iso,
                                                    int n_store, float* __restrict__ out,
                                                    int64_t plane, int64_t pitch, int strip,
                                                    int j0, int j1) {
  static_assert(2 * KC <= kWave && 2 * (kRowLoads + KC) <= 63, "seam lanes and the wait count");
  __shared__ float ring_block[kTileWaves * kRingRows * kSlotFloats];
  const uint32_t lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  lds_float* ring = (lds_float*)(ring_block) + wave * (kRingRows * kSlotFloats);
  const int last = nx - 1;
  const int x0 = strip * kPairedCells;
  // row loads: lane L of chunk c reads column x0 - 1 + 64 c + L (clamped)
  constexpr uint32_t kSize = sizeof(T);
  const uint32_t voff0 = uint32_t(min(max(x0 - 1 + int(lane), 0), last)) * kSize;
  const uint32_t voff1 = uint32_t(min(max(x0 + 63 + int(lane), 0), last)) * kSize;
  const uint32_t voff2 = uint32_t(min(max(x0 + 127 + int(lane), 0), last)) * kSize;
  const uint32_t rb = uint32_t(nx) * kSize;

  auto load_row = [&](int rho) {  // logical row rho = vertex row j0 - 1 + rho, clamped
    const int y = min(max(j0 - 1 + rho, 0), ny - 1);
    lds_float* slot = ring + (rho % kRingRows) * kSlotFloats;
    if constexpr (POISON) {
      lds_u32* const words = reinterpret_cast<lds_u32*>(slot);
      for (uint32_t w = lane; w < uint32_t(kSlotFloats); w += kWave) words[w] = 0x7fc00000u;
      // the NaNs are in LDS before any row data can land on them
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    }
    const int64_t ro = static_cast<int64_t>(y) * nx;
    const T* planes[4] = {mu, vu, mv, vv};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<T*>(planes[a] + ro), 0, static_cast<int>(rb), 0x00020000);
      load_to_lds<sizeof(T)>(r, slot + a * kPlaneStride, voff0);
      load_to_lds<sizeof(T)>(r, slot + a * kPlaneStride + 64, voff1);
      // indices 128..130 only: lanes 3.. would write into the next plane
      if (lane < 3) load_to_lds<sizeof(T)>(r, slot + a * kPlaneStride + 128, voff2);
    }
  };

  // per lane: indices of columns E = x0 + 2L, O = E + 1, seam S = x0+127+(L&1)
  // byte offsets: plane a at a * kPlaneStride * 4, index i at 4 i
  const uint32_t ie = 2 * lane + 1, is = 128 + (lane & 1);
  const uint32_t be = ie * 4, bs = is * 4;
  constexpr uint32_t kP = kPlaneStride * 4;
  const uint32_t xe = uint32_t(x0) + 2 * lane, xs = uint32_t(x0) + 127 + (lane & 1);
  const uint32_t ulast = uint32_t(last);
  const bool bx_e = (min(xe, ulast) == 0) | (min(xe, ulast) == ulast);
  const bool bx_o = (min(xe + 1, ulast) == ulast);
  const bool bx_s = (min(xs, ulast) == ulast);
  constexpr uint32_t kDrop = 0x7ffffff0u;
  const uint32_t off = xe < ulast ? xe * 4u : kDrop;
  const uint32_t row_bytes = ulast * 4u;
  const int qs = min(int(lane >> 1), KC - 1);
  float c_seam = iso.c[0];
#pragma unroll
  for (int q = 1; q < KC; ++q) c_seam = (qs == q) ? iso.c[q] : c_seam;

  // corners of vertex row r = j0 - 1 + rho (slots rho - 1, rho, rho + 1)
  struct C3 {
    Corner e, o, s;
  };
  auto corners = [&](int rho, int r) {
    const lds_char* up = reinterpret_cast<const lds_char*>(ring + ((rho - 1) % kRingRows) * kSlotFloats);
    const lds_char* at = reinterpret_cast<const lds_char*>(ring + (rho % kRingRows) * kSlotFloats);
    const lds_char* dn = reinterpret_cast<const lds_char*>(ring + ((rho + 1) % kRingRows) * kSlotFloats);
    const bool by = (r == 0) | (r == ny - 1);
    const float cym = by ? k.cym_bd : k.cym_in, cyv = by ? k.cyv_bd : k.cyv_in;
    // column at byte offset b: U neighbours at b -/+ 4 (planes 0, 1), V at b
    // in the rows above and below (planes 2, 3)
    auto one = [&](uint32_t b, bool bx) {
      return make_corner(div_gauss(lds_at<T>(at, b - 4), lds_at<T>(at, b + 4),
                                   lds_at<T>(at, b - 4 + kP), lds_at<T>(at, b + 4 + kP),
                                   lds_at<T>(up, b + 2 * kP), lds_at<T>(dn, b + 2 * kP),
                                   lds_at<T>(up, b + 3 * kP), lds_at<T>(dn, b + 3 * kP),
                                   bx ? k.cxm_bd : k.cxm_in, bx ? k.cxv_bd : k.cxv_in, cym, cyv));
    };
    C3 c;
    c.e = one(be, bx_e);
    c.o = one(be + 4, bx_o);
    c.s = one(bs, bx_s);
    return c;
  };

  // Two alternating carried sets, as in the register tiles (a single set
  // updated in place costs 64 register moves per row at K = 16).
  PairedCarry<KC> ca, cb;
#pragma unroll
  for (int rho = 0; rho < kRingRows; ++rho) load_row(rho);
  wait_vmcnt<2 * kRowLoads>();  // rows 0..2 are in LDS (rows 3 and 4 may be in flight)
  {
    const C3 c = corners(1, j0);
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      ca.e[q] = corner_probs(c.e, iso.c[q]);
      ca.o[q] = corner_probs(c.o, iso.c[q]);
    }
    ca.s = corner_probs(c.s, c_seam);
  }
  // Cell row j: corners of vertex row j + 1 = logical row j - j0 + 2, which
  // needs logical rows up to j - j0 + 3; the load issued first is row
  // j - j0 + 5, for the step two rows on.
  auto step = [&](int j) {
    const int rho = j - j0 + 2;
    load_row(rho + 3);
    return rho;
  };
  auto cells = [&](int j, int rho, const PairedCarry<KC>& p, PairedCarry<KC>& n) {
    const C3 c = corners(rho, j + 1);
    row_cells_paired<KC, STREAM>(c.e, c.o, c.s, iso, c_seam, n_store, out, plane, pitch,
                                 row_bytes, j, off, p.e, p.o, p.s, n.e, n.o, n.s);
  };
  // The first two rows read rows loaded before the loop, with fewer
  // operations issued after them: wait as in the prologue (stricter).  Then
  // two rows per trip, the carried sets alternating; an odd last row after.
  int j = j0;
  if (j < j1) {
    const int r0 = step(j);
    wait_vmcnt<2 * kRowLoads>();
    cells(j, r0, ca, cb);
    if (++j < j1) {
      const int r1 = step(j);
      wait_vmcnt<2 * kRowLoads>();
      cells(j, r1, cb, ca);
      ++j;
    }
  }
  for (; j + 2 <= j1; j += 2) {
    const int r0 = step(j);
    wait_vmcnt<2 * (kRowLoads + KC)>();
    cells(j, r0, ca, cb);
    const int r1 = step(j + 1);
    wait_vmcnt<2 * (kRowLoads + KC)>();
    cells(j + 1, r1, cb, ca);
  }
  if (j < j1) {
    const int r0 = step(j);
    wait_vmcnt<2 * (kRowLoads + KC)>();
    cells(j, r0, ca, cb);
  }
  // The loads of rows past the band are still in flight.  Let them land
  // before the ring is reused (the batch kernel's next tile writes the same
  // slots) or released with the wave: only the last step's KC stores, issued
  // after the last load, may remain outstanding.
  wait_vmcnt<KC>();
}

// Split layout, one vertex row step: the corners of row j+1 for the lane's
// columns A and B, their pairs with row j (cor_*, which then take row j+1's
// corners), and the lane's two cells for every isovalue; off_a, off_b are the
// byte offsets of the lane's cells within an output row.
template <int KC, bool FUSED>
__device__ __forceinline__ void row_step_split(const Raw<FUSED>& raw_a, const Raw<FUSED>& raw_b,
                                               const Col& ca, const Col& cb, int ny,
                                               const StencilCoef& k, const IsoChunk& iso,
                                               int n_store, float* __restrict__ out,
                                               int64_t plane, int64_t pitch, uint32_t row_bytes,
                                               int j, uint32_t off_a, uint32_t off_b,
                                               const AB (&prev_a)[KC], const AB (&prev_b)[KC],
                                               AB (&next_a)[KC], AB (&next_b)[KC]) {
  const Corner ka = make_corner(raw_div(raw_a, ca.bx, j + 1, ny, k));
  const Corner kb = make_corner(raw_div(raw_b, cb.bx, j + 1, ny, k));
  float* __restrict__ orow = out + static_cast<int64_t>(j) * pitch;
#pragma unroll
  for (int q = 0; q < KC; ++q) {
    const AB cur_a = corner_probs(ka, iso.c[q]);
    const AB cur_b = corner_probs(kb, iso.c[q]);
    const float l0 = cell_lcp_dpp(make_pair(prev_a[q], cur_a), cur_a.below);
    const float l1 = cell_lcp_dpp(make_pair(prev_b[q], cur_b), cur_b.below);
    // planes past n_store (a batch's padding) get an empty record range
    const RowWriter<false> w(orow + q * plane, q < n_store ? row_bytes : 0u);
    w.put(l0, off_a);
    w.put(l1, off_b);
    next_a[q] = cur_a;
    next_b[q] = cur_b;
  }
}

// Split tile: cell columns [x0, x0+126) of strip `strip` (x0 = 126 strip),
// cell rows [j0, j1); arguments as for lcp_tile_paired.
template <int KC, bool FUSED, typename T>
__device__ __forceinline__ void lcp_tile_split(const T* __restrict__ p0, const T* __restrict__ p1,
                                               const T* __restrict__ p2, const T* __restrict__ p3,
                                               int ny, int nx, const StencilCoef& k,
                                               const IsoChunk& iso, int n_store,
                                               float* __restrict__ out, int64_t plane,
                                               int64_t pitch, int strip, int j0, int j1) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t xa = uint32_t(strip) * kSplitCells + lane;  // A column
  const uint32_t xb = xa + kSplitHalf;                        // B column
  const uint32_t last = uint32_t(nx - 1);
  const Col ca = make_col(min(xa, last), nx, sizeof(T));  // columns past the edge load a
  const Col cb = make_col(min(xb, last), nx, sizeof(T));  // valid column, store nothing
  // lane 63 and cells past the right edge get an offset beyond any row
  constexpr uint32_t kDrop = 0x7ffffff0u;
  const uint32_t off_a = ((lane < kSplitHalf) & (xa < last)) ? xa * 4u : kDrop;
  const uint32_t off_b = ((lane < kSplitHalf) & (xb < last)) ? xb * 4u : kDrop;
  const uint32_t row_bytes = last * 4u;

  AB pa[KC], pb[KC], qa[KC], qb[KC];  // two alternating sets
  Raw<FUSED> a0, b0, a1, b1;
  load_raw(a0, p0, p1, p2, p3, ny, nx, ca, j0);
  load_raw(b0, p0, p1, p2, p3, ny, nx, cb, j0);
  load_raw(a1, p0, p1, p2, p3, ny, nx, ca, j0 + 1);
  load_raw(b1, p0, p1, p2, p3, ny, nx, cb, j0 + 1);
  {
    const Corner c0 = make_corner(raw_div(a0, ca.bx, j0, ny, k));
    const Corner c1 = make_corner(raw_div(b0, cb.bx, j0, ny, k));
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      pa[q] = corner_probs(c0, iso.c[q]);
      pb[q] = corner_probs(c1, iso.c[q]);
    }
  }
  auto step = [&](const Raw<FUSED>& ra, const Raw<FUSED>& rb, int j, const AB (&prev_a)[KC],
                  const AB (&prev_b)[KC], AB (&next_a)[KC], AB (&next_b)[KC]) {
    row_step_split<KC, FUSED>(ra, rb, ca, cb, ny, k, iso, n_store, out, plane, pitch,
                              row_bytes, j, off_a, off_b, prev_a, prev_b, next_a, next_b);
  };
  // two rows per trip, as in the paired tile
  auto trip = [&](int j) {
    load_raw(a0, p0, p1, p2, p3, ny, nx, ca, j + 2);
    load_raw(b0, p0, p1, p2, p3, ny, nx, cb, j + 2);
    step(a1, b1, j, pa, pb, qa, qb);
    const int jn = min(j + 3, j1);
    load_raw(a1, p0, p1, p2, p3, ny, nx, ca, jn);
    load_raw(b1, p0, p1, p2, p3, ny, nx, cb, jn);
    step(a0, b0, j + 1, qa, qb, pa, pb);
  };
  int j = j0;
  if (j + 2 <= j1) {
    trip(j);
    for (j += 2; j + 2 <= j1; j += 2) trip(j);
  }
  if (j < j1) step(a1, b1, j, pa, pb, qa, qb);  // a1/b1 hold row j + 1 == j1
}

// Layout choice: the paired tile when every output row starts on a 128-byte
// line (base aligned, row pitch and plane stride multiples of 32 floats) and
// either there are at least 8 isovalues or the map has at least 2^22 cells
// (use_paired_tile); under the same size rule the fused kernel also takes it
// for other rows (use_paired_unaligned), with the default store policy.
// On large maps its whole-line stores outweigh the seam step at any
// isovalue count (8192^2, rows interleaved, paired against split: 0.269 /
// 0.293 ms at 1 isovalue, 0.318 / 0.360 ms at 2, 0.430 / 0.497 ms at 4;
// 4096^2: 62 / 76 us at 1, 103 / 142 us at 4); on small maps with few
// isovalues the launch is dominated by its fixed cost, which is lower for
// the split tile (up to 1024^2: 16 against 24 us at 1 isovalue, 26 against
// 35 us at 4).
inline bool use_paired_tile(const float* out, int64_t pitch, int64_t plane, int kc,
                            int64_t cells) {
  return (reinterpret_cast<uintptr_t>(out) % 128 == 0) && (pitch % 32 == 0) &&
         (plane % 32 == 0) && (kc >= 8 || cells >= (int64_t(1) << 22));
}
inline bool use_paired_unaligned(int kc, int64_t cells) {
  return kc >= 8 || cells >= (int64_t(1) << 22);
}

// The tile of layout PAIRED.  STREAM: non-temporal stores (for rows that
// start on 128-byte lines; the unaligned paired tile of the fused kernel
// stores with the default policy).
template <int KC, bool FUSED, bool PAIRED, typename T, bool POISON = false, bool STREAM = PAIRED>
__device__ __forceinline__ void lcp_tile(const T* __restrict__ p0, const T* __restrict__ p1,
                                         const T* __restrict__ p2, const T* __restrict__ p3,
                                         int ny, int nx, const StencilCoef& k,
                                         const IsoChunk& iso, int n_store,
                                         float* __restrict__ out, int64_t plane, int64_t pitch,
                                         int strip, int j0, int j1) {
  static_assert(PAIRED || !STREAM, "the split tile stores with the default policy");
  if constexpr (PAIRED && FUSED)
    lcp_tile_paired_lds<KC, STREAM, T, POISON>(p0, p1, p2, p3, ny, nx, k, iso, n_store, out,
                                                plane, pitch, strip, j0, j1);
  else if constexpr (PAIRED)
    lcp_tile_paired<KC, FUSED, STREAM>(p0, p1, p2, p3, ny, nx, k, iso, n_store, out, plane, pitch,
                                       strip, j0, j1);
  else
    lcp_tile_split<KC, FUSED>(p0, p1, p2, p3, ny, nx, k, iso, n_store, out, plane, pitch, strip,
                              j0, j1);
}

}  // namespace pdiv
