// The path extended to 3D vector fields, the paper's stated future work
// (Section 5): the divergence Gaussian gains the z term of Eq. 2 and Eq. 3
// (dW/dz differenced like the other two axes), and a cell is a hexahedron
// whose level-crossing probability is 1 - prod_8 P(above) - prod_8 P(below).
//
// Kernels:
//   divergence3d_kernel  Eq. 2-3 with the z term, one vertex per lane; HBM
//                        bound: 6 planes read, 2 written.
//   lcp3d_kernel         8-corner LCP from the divergence Gaussians.  A wave
//                        holds a strip of 64 vertex columns (63 cells) and LZ
//                        consecutive cell layers k0..k0+LZ-1 and walks a band
//                        of rows along y.  At each row it evaluates the
//                        corner tails once for the LZ+1 z-levels it holds,
//                        pairs them along z, joins each z-pair with the one
//                        of the previous row (carried in registers) and
//                        combines the resulting 4-corner column with the
//                        right neighbour's through DPP, so every tail serves
//                        the cells on both sides of its vertex in x, y and,
//                        inside the wave, z.
#include <hip/hip_runtime.h>

#include "lcp_tile.hpp"
#include "pdiv_device.hpp"
#include "pdiv_internal.hpp"

namespace pdiv {

StencilCoef3 make_coef3(double dx, double dy, double dz) {
  StencilCoef3 k;
  k.xy = make_coef(dx, dy);
  k.czm_in = static_cast<float>(1.0 / (2.0 * dz));
  k.czv_in = static_cast<float>(1.0 / (4.0 * dz * dz));
  k.czm_bd = static_cast<float>(1.0 / dz);
  k.czv_bd = static_cast<float>(1.0 / (dz * dz));
  return k;
}

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;
// z slices per divergence3d wave: each chunk re-reads W at its two ends, and
// longer chunks mean fewer waves.  At 512^3 float32: 8, 12, 16, 32, 64
// slices take 0.877, 0.852, 0.901, 0.962, 0.976 ms.
constexpr int kZChunk = 12;
// Vertex rows per band: 32, except 16 for the two-step kernel on rows that
// do not start on lines, where the shorter walks (twice the waves, the first
// row of each band peeled) measured faster (512^3 dense maps: 0.396 / 0.911 /
// 3.152 ms at 1 / 4 / 16 isovalues against 0.408 / 0.958 / 3.377 ms with
// 32); line-aligned rows are unchanged by it and the fused kernel on dense
// rows gains nothing (0.985 / 1.482 / 3.955 against 0.980 / 1.496 / 3.879).
template <bool FUSED, bool LINES>
constexpr int band_rows3() {
  return (LINES || FUSED) ? 32 : 16;
}
constexpr int kMinBandRows3 = 16;

// Eq. 2-3 with the z term at one vertex; the neighbours are already clamped
// at the boundary and the coefficients chosen (1/(2h) inside, 1/h on a
// boundary plane).  Contraction is off so the rounding is fixed.
__device__ __forceinline__ DivGauss div_gauss3(float mu_xl, float mu_xr, float vu_xl,
                                               float vu_xr, float mv_yl, float mv_yr,
                                               float vv_yl, float vv_yr, float mw_zl,
                                               float mw_zr, float vw_zl, float vw_zr, float cxm,
                                               float cxv, float cym, float cyv, float czm,
                                               float czv) {
#pragma clang fp contract(off)
  const float mx = (mu_xr - mu_xl) * cxm;
  const float my = (mv_yr - mv_yl) * cym;
  const float mz = (mw_zr - mw_zl) * czm;
  const float vx = (vu_xr + vu_xl) * cxv;
  const float vy = (vv_yr + vv_yl) * cyv;
  const float vz = (vw_zr + vw_zl) * czv;
  DivGauss g;
  g.mean = (mx + my) + mz;
  g.var = (vx + vy) + vz;
  return g;
}

// Grid: blocks of 4 waves over (x block of 64 columns, 4 consecutive rows
// y, a chunk of kZChunk slices z), x block fastest, in XCD-contiguous block
// order (blocks are dealt round-robin to the 8 XCDs; this gives each XCD a
// contiguous run, so blocks that share neighbour rows share an L2).  A wave
// walks z along its row: W's values at z-1, z, z+1 stay in a three-deep
// register window, so each is loaded once per chunk instead of once per use;
// V's rows y-1, y+1 are those of the block's other waves (found in cache).
// Every vertex sees the same inputs and operations as a straight evaluation
// of Eq. 2-3 with clamped neighbours.
template <typename T>
__global__ __launch_bounds__(kBlock) void divergence3d_kernel(
    const T* __restrict__ mu, const T* __restrict__ vu, const T* __restrict__ mv,
    const T* __restrict__ vv, const T* __restrict__ mw, const T* __restrict__ vw, int nz, int ny,
    int nx, StencilCoef3 k, float* __restrict__ dmean, float* __restrict__ dvar, int n_xb,
    int n_yq) {
  const int nb = gridDim.x, xcd = blockIdx.x % 8, q8 = nb / 8, r8 = nb % 8;
  const int blk = xcd * q8 + min(xcd, r8) + blockIdx.x / 8;
  const int xb = blk % n_xb;
  const int rest = blk / n_xb;
  const int y = (rest % n_yq) * kWavesPerBlock + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int z0 = (rest / n_yq) * kZChunk;
  const int x = xb * 64 + (threadIdx.x & 63);
  if (y >= ny || x >= nx) return;
  const int z1 = min(z0 + kZChunk, nz);
  const Col c = make_col(uint32_t(x), nx, sizeof(T));
  const int yl = y > 0 ? y - 1 : 0, yr = y < ny - 1 ? y + 1 : ny - 1;
  const bool by = (y == 0) | (y == ny - 1);
  const float cym = by ? k.xy.cym_bd : k.xy.cym_in, cyv = by ? k.xy.cyv_bd : k.xy.cyv_in;
  const float cxm = c.bx ? k.xy.cxm_bd : k.xy.cxm_in, cxv = c.bx ? k.xy.cxv_bd : k.xy.cxv_in;
  const int64_t plane = int64_t(ny) * nx;
  const int64_t off_y = int64_t(y) * nx;
  auto w_at = [&](int z, float& m, float& v) {
    const int64_t row = int64_t(z) * plane + off_y;
    m = RowReader<T>(mw + row, nx).get(c.x);
    v = RowReader<T>(vw + row, nx).get(c.x);
  };
  float wm_prev, wv_prev, wm_cur, wv_cur, wm_next, wv_next;
  w_at(z0, wm_cur, wv_cur);
  if (z0 > 0) {
    w_at(z0 - 1, wm_prev, wv_prev);
  } else {
    wm_prev = wm_cur;
    wv_prev = wv_cur;
  }
  for (int z = z0; z < z1; ++z) {
    w_at(z < nz - 1 ? z + 1 : nz - 1, wm_next, wv_next);
    const int64_t row = int64_t(z) * plane + off_y;
    const int64_t row_yl = int64_t(z) * plane + int64_t(yl) * nx;
    const int64_t row_yr = int64_t(z) * plane + int64_t(yr) * nx;
    const RowReader<T> u0(mu + row, nx), s0(vu + row, nx);
    const RowReader<T> v_l(mv + row_yl, nx), v_r(mv + row_yr, nx);
    const RowReader<T> t_l(vv + row_yl, nx), t_r(vv + row_yr, nx);
    const bool bz = (z == 0) | (z == nz - 1);
    // clamped z neighbours: (0, 1) at z = 0, (nz-2, nz-1) at z = nz-1
    const float mzl = z > 0 ? wm_prev : wm_cur, vzl = z > 0 ? wv_prev : wv_cur;
    const float mzr = z < nz - 1 ? wm_next : wm_cur, vzr = z < nz - 1 ? wv_next : wv_cur;
    const DivGauss g = div_gauss3(u0.get(c.xl), u0.get(c.xr), s0.get(c.xl), s0.get(c.xr),
                                  v_l.get(c.x), v_r.get(c.x), t_l.get(c.x), t_r.get(c.x), mzl,
                                  mzr, vzl, vzr, cxm, cxv, cym, cyv,
                                  bz ? k.czm_bd : k.czm_in, bz ? k.czv_bd : k.czv_in);
    __builtin_nontemporal_store(g.mean, dmean + row + x);
    __builtin_nontemporal_store(g.var, dvar + row + x);
    wm_prev = wm_cur;
    wv_prev = wv_cur;
    wm_cur = wm_next;
    wv_cur = wv_next;
  }
}

// The 8 corners of a pair of 4-corner groups (lo, hi): the products multiply
// and 1 - prod telescopes as Q_lo + P_lo Q_hi (every term non-negative).
__device__ __forceinline__ Pair join_pairs(const Pair& lo, const Pair& hi) {
  Pair p;
  p.pa = lo.pa * hi.pa;
  p.qa = fmaf(lo.pa, hi.qa, lo.qa);
  p.pb = lo.pb * hi.pb;
  p.qb = fmaf(lo.pb, hi.qb, lo.qb);
  return p;
}

// The input planes of one launch: the two divergence volumes (dm, dv as
// float) or, fused, the six moment volumes of type T.
struct Planes6 {
  const void* p[6];
};

// One vertex row's inputs for a lane's column at the L+1 levels it holds,
// loaded a row ahead of their use.  Two-step: the divergence mean and
// variance per level.  Fused: U's x neighbours (mean, variance) and V's next
// row per level, and W at the levels one below to one above the held ones
// (level t + 1 of the array is held level t; adjacent held levels share W).
template <int L, bool FUSED>
struct Row3;
template <int L>
struct Row3<L, false> {
  float m[L + 1], v[L + 1];
};
template <int L>
struct Row3<L, true> {
  float ul[L + 1], ur[L + 1], sl[L + 1], sr[L + 1];
  float vm[L + 1], vv[L + 1];
  float wm[L + 3], wv[L + 3];
};

// Fused: V's rows clamp(j-1) and j per held level, carried from row to row
// so that each V row is loaded once per walk.
template <int L>
struct VWin {
  float m[L + 1][2], v[L + 1][2];
};

// Eq. 2-3 (fused) or the loaded Gaussians (two-step) of the held levels at
// row j, as corners; bz[l]: level l is a z boundary plane.  Moves the V
// window one row.
template <int L, bool FUSED>
__device__ __forceinline__ void row_corners(const Row3<L, FUSED>& r, VWin<L>& w,
                                            const bool (&bz)[L + 1], float cxm, float cxv,
                                            float cym, float cyv, const StencilCoef3& k,
                                            Corner (&c)[L + 1]) {
#pragma unroll
  for (int l = 0; l <= L; ++l) {
    DivGauss g;
    if constexpr (FUSED) {
      g = div_gauss3(r.ul[l], r.ur[l], r.sl[l], r.sr[l], w.m[l][0], r.vm[l], w.v[l][0], r.vv[l],
                     r.wm[l], r.wm[l + 2], r.wv[l], r.wv[l + 2], cxm, cxv, cym, cyv,
                     bz[l] ? k.czm_bd : k.czm_in, bz[l] ? k.czv_bd : k.czv_in);
      w.m[l][0] = w.m[l][1];
      w.v[l][0] = w.v[l][1];
      w.m[l][1] = r.vm[l];
      w.v[l][1] = r.vv[l];
    } else {
      g.mean = r.m[l];
      g.var = r.v[l];
    }
    c[l] = make_corner(g);
  }
}

// A reader over plane p from level `lev`, row `row` to the end of the
// volume (at most 2^31 - 1 bytes): loads reach the levels above `lev`
// through their offsets (the caller keeps 7 levels within 2^31 bytes).
template <typename T>
__device__ __forceinline__ RowReader<T> vol_reader(const void* p, int lev, int row, int nz,
                                                   int nx, int64_t vplane) {
  const T* base = static_cast<const T*>(p) + int64_t(lev) * vplane + int64_t(row) * nx;
  const int64_t left = (int64_t(nz) - lev) * vplane - int64_t(row) * nx;
  const int64_t cap = int64_t(0x7fffffff / sizeof(T));
  return RowReader<T>(base, int(left < cap ? left : cap));
}

// The planes' readers of one row: level lb, row j (U, W; the two-step
// divergence volumes) and row clamp(j+1) (V), shared by the wave's column
// and the seam.
template <bool FUSED, typename T>
struct Rows3 {
  RowReader<T> u, s, vm, vv, wm, wv;
  __device__ __forceinline__ Rows3(const Planes6& src, int lb, int j, int nz, int ny, int nx,
                                   int64_t vplane)
      : u(vol_reader<T>(src.p[0], lb, j, nz, nx, vplane)),
        s(vol_reader<T>(src.p[1], lb, j, nz, nx, vplane)),
        vm(vol_reader<T>(src.p[FUSED ? 2 : 0], lb, j < ny - 1 ? j + 1 : ny - 1, nz, nx, vplane)),
        vv(vol_reader<T>(src.p[FUSED ? 3 : 1], lb, j < ny - 1 ? j + 1 : ny - 1, nz, nx, vplane)),
        wm(vol_reader<T>(src.p[FUSED ? 4 : 0], lb, j, nz, nx, vplane)),
        wv(vol_reader<T>(src.p[FUSED ? 5 : 1], lb, j, nz, nx, vplane)) {}
};

// One row's inputs at L+1 held levels.  lo[t]: byte offset of level t
// relative to level lb (W's level t - 1 for the fused W array, whose level
// t + 1 is held level t); wave-uniform for the wave's own column (scalar
// offsets), per lane for the seam (added to the column offset).
template <int L, bool UNIFORM, typename T>
__device__ __forceinline__ void load_levels(Row3<L, false>& r, const Rows3<false, T>& rd,
                                            const uint32_t* lo, const Col& c) {
#pragma unroll
  for (int l = 0; l <= L; ++l) {
    r.m[l] = UNIFORM ? rd.u.get(c.x, lo[l]) : rd.u.get(c.x + lo[l]);
    r.v[l] = UNIFORM ? rd.s.get(c.x, lo[l]) : rd.s.get(c.x + lo[l]);
  }
}
template <int L, bool UNIFORM, typename T>
__device__ __forceinline__ void load_levels(Row3<L, true>& r, const Rows3<true, T>& rd,
                                            const uint32_t* lw, const Col& c) {
  auto get = [&](const RowReader<T>& x, uint32_t col, uint32_t lev) {
    return UNIFORM ? x.get(col, lev) : x.get(col + lev);
  };
#pragma unroll
  for (int t = 0; t < L + 3; ++t) {
    r.wm[t] = get(rd.wm, c.x, lw[t]);
    r.wv[t] = get(rd.wv, c.x, lw[t]);
  }
#pragma unroll
  for (int l = 0; l <= L; ++l) {
    r.ul[l] = get(rd.u, c.xl, lw[l + 1]);
    r.ur[l] = get(rd.u, c.xr, lw[l + 1]);
    r.sl[l] = get(rd.s, c.xl, lw[l + 1]);
    r.sr[l] = get(rd.s, c.xr, lw[l + 1]);
    r.vm[l] = get(rd.vm, c.x, lw[l + 1]);
    r.vv[l] = get(rd.vv, c.x, lw[l + 1]);
  }
}

// Waves: strip (fastest), then layer group, then band, over an XCD-aware
// block order: blocks are dealt round-robin to the 8 XCDs, each with its own
// L2, so each XCD is given a contiguous run of blocks and the strips that
// share an output row's cache lines write them through the same L2
// (measured at 512^3: 1.03 ms against 1.19 ms with layer groups fastest at
// 4 isovalues).  Every lane stays active through the DPP reads:
// lanes past the grid clamp their column.  Loads and stores go through
// buffer resources with a scalar row base and a per-lane byte offset; a
// store row is sized to the strip's cells, so the buffer hardware drops the
// stores of lanes past the grid (no branch around them).  Each row's inputs
// are loaded one row ahead, so their latency overlaps the previous row's
// arithmetic.
//
// Two strip layouts, the same arithmetic (so the same bits):
//   LINES = false: lane L holds vertex column x0+L, x0 = 63 strip; the wave
//     forms the 63 cells [x0, x0+63) (lane 63 has no cell), for any row pitch.
//   LINES = true, for outputs whose rows start on 128-byte lines: x0 = 64
//     strip and lane 63 forms cell x0+63 too, so each store instruction
//     writes 256 contiguous bytes, two whole lines.  Its right column x0+64
//     belongs to no lane: a seam step has lanes 2i and 2i+1 (i = q LZ + l)
//     evaluate columns x0+63 and x0+64 at levels l and l+1 for isovalue q,
//     lane 2i forms that cell with the cell formula of every other lane, and
//     lane 63 takes it over with one readlane/writelane per (q, l).  Needs
//     2 KC LZ <= 64.
// FUSED: each row's corners come from Eq. 2-3 with the z term evaluated on
// the spot from the six moment volumes (the divergence never reaches HBM),
// with the operands and order of divergence3d_kernel, so the maps are
// bitwise the two-step result.
// With 8 corners the float32 combination can land an ulp outside [0, 1]
// where the probability is 0 or 1; the exact value is inside, so clamping
// only removes error.  The IEEE 754-2019 maximum and minimum (v_maximum3_f32,
// v_minimum3_f32 on gfx950) return NaN for a NaN operand, so a NaN LCP stays
// NaN, in two instructions.
__device__ __forceinline__ float clamp01(float v) {
  return __builtin_elementwise_minimum(__builtin_elementwise_maximum(v, 0.0f), 1.0f);
}

template <int KC, int LZ, bool FUSED, bool LINES, typename T>
__global__ __launch_bounds__(kBlock) void lcp3d_kernel(Planes6 src, int nz, int ny, int nx,
                                                       StencilCoef3 k, IsoChunk iso,
                                                       float* __restrict__ out, int64_t pitch,
                                                       int64_t plane, int n_groups, int n_strips,
                                                       int n_bands) {
  static_assert(!LINES || 2 * KC * LZ <= 64, "the seam step needs two lanes per (q, l)");
  constexpr int kW = LINES ? 64 : 63;  // cells per strip
  const int nb = gridDim.x, xcd = blockIdx.x % 8, q8 = nb / 8, r8 = nb % 8;
  const int blk = xcd * q8 + min(xcd, r8) + blockIdx.x / 8;
  const int wave = __builtin_amdgcn_readfirstlane(blk * kWavesPerBlock + (threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int strip = wave % n_strips;
  const int rest = wave / n_strips;
  const int grp = rest % n_groups;
  const int band = rest / n_groups;
  if (band >= n_bands) return;
  const int k0 = grp * LZ;
  const int nl = min(LZ, nz - 1 - k0);
  const int j0 = band * band_rows3<FUSED, LINES>();
  const int j1 = min(j0 + band_rows3<FUSED, LINES>(), ny - 1);
  const int x0 = strip * kW;
  const uint32_t store_bytes = uint32_t(min(kW, nx - 1 - x0)) * 4u;
  const uint32_t soff = uint32_t(lane) * 4u;
  const int64_t layer = int64_t(ny - 1) * pitch;
  const int64_t vplane = int64_t(ny) * nx;
  const Col col = make_col(uint32_t(min(x0 + lane, nx - 1)), nx, sizeof(T));
  const float cxm = col.bx ? k.xy.cxm_bd : k.xy.cxm_in;
  const float cxv = col.bx ? k.xy.cxv_bd : k.xy.cxv_in;
  bool bz[LZ + 1];
#pragma unroll
  for (int l = 0; l <= LZ; ++l) {
    const int kk = min(k0 + l, nz - 1);
    bz[l] = (kk == 0) | (kk == nz - 1);
  }

  // seam lanes: (q, l) = (si / LZ, si % LZ), column x0+63 (even lane) or
  // x0+64 (odd lane), levels k0+l and k0+l+1
  const int si = min(lane >> 1, KC * LZ - 1);
  const int sq = si / LZ, sl = si % LZ;
  float c_seam = iso.c[0];
#pragma unroll
  for (int q = 1; q < KC; ++q) c_seam = (sq == q) ? iso.c[q] : c_seam;
  const Col cs = make_col(uint32_t(min(x0 + 63 + (lane & 1), nx - 1)), nx, sizeof(T));
  const float sxm = cs.bx ? k.xy.cxm_bd : k.xy.cxm_in;
  const float sxv = cs.bx ? k.xy.cxv_bd : k.xy.cxv_in;
  bool sbz[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int kk = min(k0 + sl + t, nz - 1);
    sbz[t] = (kk == 0) | (kk == nz - 1);
  }
  // Level offsets (bytes) from the readers' base level lb.  Fused: W's
  // levels clamp(k0-1+t), t < LZ+3 (held level l is t = l+1); two-step: the
  // held levels.  The seam's per lane, from its first level k0+sl.
  const int lb = FUSED ? max(k0 - 1, 0) : k0;
  const uint32_t pb = uint32_t(vplane) * uint32_t(sizeof(T));
  constexpr int kLv = FUSED ? LZ + 3 : LZ + 1;
  uint32_t lo[kLv], slo[FUSED ? 4 : 2];
#pragma unroll
  for (int t = 0; t < kLv; ++t)
    lo[t] = uint32_t((FUSED ? min(max(k0 - 1 + t, 0), nz - 1) : min(k0 + t, nz - 1)) - lb) * pb;
#pragma unroll
  for (int t = 0; t < (FUSED ? 4 : 2); ++t)
    slo[t] = uint32_t((FUSED ? min(max(k0 + sl - 1 + t, 0), nz - 1) : min(k0 + sl + t, nz - 1)) -
                      lb) * pb;

  VWin<LZ> win;
  VWin<1> swin;
  if constexpr (FUSED) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int y = h == 0 ? (j0 > 0 ? j0 - 1 : 0) : j0;
      const RowReader<T> vm = vol_reader<T>(src.p[2], lb, y, nz, nx, vplane);
      const RowReader<T> vv = vol_reader<T>(src.p[3], lb, y, nz, nx, vplane);
#pragma unroll
      for (int l = 0; l <= LZ; ++l) {
        win.m[l][h] = vm.get(col.x, lo[l + 1]);
        win.v[l][h] = vv.get(col.x, lo[l + 1]);
      }
      if constexpr (LINES) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          swin.m[t][h] = vm.get(cs.x + slo[t + 1]);
          swin.v[t][h] = vv.get(cs.x + slo[t + 1]);
        }
      }
    }
  }
  Row3<LZ, FUSED> raw;
  Row3<1, FUSED> sraw;
  auto load = [&](int j) {
    const Rows3<FUSED, T> rd(src, lb, j, nz, ny, nx, vplane);
    load_levels<LZ, true, T>(raw, rd, lo, col);
    if constexpr (LINES) load_levels<1, false, T>(sraw, rd, slo, cs);
  };
  load(j0);
  // Corner probabilities of the previous vertex row per held level and
  // isovalue (the seam's per lane).  A cell joins, at each of its two
  // levels, the corners of rows j-1 and j into a pair, joins the two levels'
  // pairs into its column's 4 corners, and combines them with the right
  // column's through DPP.
  AB prev[LZ + 1][KC];
  AB sprev[2];
  auto cym_of = [&](int j) {
    const bool by = (j == 0) | (j == ny - 1);
    return by ? k.xy.cym_bd : k.xy.cym_in;
  };
  auto cyv_of = [&](int j) {
    const bool by = (j == 0) | (j == ny - 1);
    return by ? k.xy.cyv_bd : k.xy.cyv_in;
  };
  {  // the band's first vertex row: corners only (j1 > j0 always)
    Corner c[LZ + 1];
    row_corners<LZ, FUSED>(raw, win, bz, cxm, cxv, cym_of(j0), cyv_of(j0), k, c);
    Corner sc[2];
    if constexpr (LINES)
      row_corners<1, FUSED>(sraw, swin, sbz, sxm, sxv, cym_of(j0), cyv_of(j0), k, sc);
    load(j0 + 1);
#pragma unroll
    for (int q = 0; q < KC; ++q)
#pragma unroll
      for (int l = 0; l <= LZ; ++l) prev[l][q] = corner_probs(c[l], iso.c[q]);
    if constexpr (LINES) {
      sprev[0] = corner_probs(sc[0], c_seam);
      sprev[1] = corner_probs(sc[1], c_seam);
    }
  }
  // layers past the volume's end get an empty record range (stores dropped)
  uint32_t layer_bytes[LZ];
#pragma unroll
  for (int l = 0; l < LZ; ++l) layer_bytes[l] = l < nl ? store_bytes : 0u;
  // One row step: prev holds row j-1's probabilities, row j's go to next
  // (which may be prev itself: each is read before it is overwritten).
  auto row = [&](int j, const AB (&prev)[LZ + 1][KC], AB (&next)[LZ + 1][KC],
                 const AB (&sprev)[2], AB (&snext)[2]) {
    Corner c[LZ + 1];
    row_corners<LZ, FUSED>(raw, win, bz, cxm, cxv, cym_of(j), cyv_of(j), k, c);
    Corner sc[2];
    if constexpr (LINES)
      row_corners<1, FUSED>(sraw, swin, sbz, sxm, sxv, cym_of(j), cyv_of(j), k, sc);
    if (j < j1) load(j + 1);
    // seam: lane 2i holds cell x0+63 of layer l at isovalue q
    float seam = 0.0f;
    if constexpr (LINES) {
      const AB a0 = corner_probs(sc[0], c_seam);
      const AB a1 = corner_probs(sc[1], c_seam);
      seam = cell_lcp_dpp(join_pairs(make_pair(sprev[0], a0), make_pair(sprev[1], a1)),
                          a0.below);
      seam = clamp01(seam);
      snext[0] = a0;
      snext[1] = a1;
    }
    float* const row_out = out + int64_t(k0) * layer + int64_t(j - 1) * pitch + x0;
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      Pair yp[LZ + 1];
      int below[LZ];
#pragma unroll
      for (int l = 0; l <= LZ; ++l) {
        const AB ab = corner_probs(c[l], iso.c[q]);
        yp[l] = make_pair(prev[l][q], ab);
        if (l < LZ) below[l] = ab.below;
        next[l][q] = ab;
      }
#pragma unroll
      for (int l = 0; l < LZ; ++l) {
        float v = cell_lcp_dpp(join_pairs(yp[l], yp[l + 1]), below[l]);
        v = clamp01(v);
        if constexpr (LINES)
          v = to_lane63(v, __builtin_amdgcn_readlane(__float_as_int(seam), 2 * (q * LZ + l)));
        RowWriter<LINES>(row_out + int64_t(q) * plane + int64_t(l) * layer, layer_bytes[l])
            .put(v, soff);
      }
    }
  };
  if constexpr (KC == 4 && !FUSED) {
    // 4 isovalues: two sets, alternated (no copies, registers to spare; 0.782
    // against 0.790 ms with one set at 512^3); at 1 and 2 one set's lower
    // register count (63 / 79 VGPRs: 8 / 6 waves per SIMD) pays for its
    // copies on a random field (0.364 against 0.381 ms at 1 isovalue, 0.495
    // against 0.502 at 2) and is neutral on the smooth benchmark field
    AB prev2[LZ + 1][KC];
    AB sprev2[2];
    int j = j0 + 1;
    for (; j + 1 <= j1; j += 2) {
      row(j, prev, prev2, sprev, sprev2);
      row(j + 1, prev2, prev, sprev2, sprev);
    }
    if (j <= j1) row(j, prev, prev2, sprev, sprev2);
  } else {
    // one set updated in place (a copy per value, one wave more per SIMD)
    for (int j = j0 + 1; j <= j1; ++j) row(j, prev, prev, sprev, sprev);
  }
}

template <int KC, int LZ, bool FUSED, bool LINES, typename T>
hipError_t launch_lcp3d_kc(const Planes6& src, int nz, int ny, int nx, const StencilCoef3& k,
                           const IsoChunk& iso, float* out, int64_t pitch, int64_t plane,
                           hipStream_t s) {
  constexpr int kW = LINES ? 64 : 63;
  const int n_groups = (nz - 1 + LZ - 1) / LZ;
  const int n_strips = (nx - 1 + kW - 1) / kW;
  constexpr int kRows = band_rows3<FUSED, LINES>();
  const int n_bands = (ny - 1 + kRows - 1) / kRows;
  const int64_t waves = int64_t(n_groups) * n_strips * n_bands;
  const int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
  if (!launch_fits(blocks, kBlock)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((lcp3d_kernel<KC, LZ, FUSED, LINES, T>), dim3(unsigned(blocks)), dim3(kBlock),
                     0, s, src, nz, ny, nx, k, iso, out, pitch, plane, n_groups, n_strips,
                     n_bands);
  return hipGetLastError();
}

}  // namespace

int64_t lcp3d_blocks(int64_t nz, int64_t ny, int64_t nx, int kc) {
  const int lz = kc <= 4 ? 4 : 2;  // the fewest layers any launch uses
  const int64_t waves = ((nz - 1 + lz - 1) / lz) * ((nx - 1 + 62) / 63) *
                        ((ny - 1 + kMinBandRows3 - 1) / kMinBandRows3);
  return (waves + kWavesPerBlock - 1) / kWavesPerBlock;
}

bool lcp3d_slice_fits(int64_t ny, int64_t nx, size_t elem_bytes) {
  return 7 * ny * nx * int64_t(elem_bytes) < (int64_t(1) << 31);
}

int64_t divergence3d_blocks(int64_t nz, int64_t ny, int64_t nx) {
  return ((nx + 63) / 64) * ((ny + kWavesPerBlock - 1) / kWavesPerBlock) *
         ((nz + kZChunk - 1) / kZChunk);
}

hipError_t launch_divergence3d(const void* mu, const void* vu, const void* mv, const void* vv,
                               const void* mw, const void* vw, pdiv_dtype dt, int64_t nz,
                               int64_t ny, int64_t nx, const StencilCoef3& k, float* dmean,
                               float* dvar, hipStream_t s) {
  const int n_xb = int((nx + 63) / 64);
  const int n_yq = int((ny + kWavesPerBlock - 1) / kWavesPerBlock);
  const int64_t blocks = divergence3d_blocks(nz, ny, nx);
  if (!launch_fits(blocks, kBlock)) return hipErrorInvalidConfiguration;
  const dim3 grid{unsigned(blocks)}, block{unsigned(kBlock)};
  const int z = int(nz), y = int(ny), x = int(nx);
#define PDIV_DIV3(T)                                                                         \
  hipLaunchKernelGGL(divergence3d_kernel<T>, grid, block, 0, s, static_cast<const T*>(mu),   \
                     static_cast<const T*>(vu), static_cast<const T*>(mv),                   \
                     static_cast<const T*>(vv), static_cast<const T*>(mw),                   \
                     static_cast<const T*>(vw), z, y, x, k, dmean, dvar, n_xb, n_yq)
  switch (dt) {
    case PDIV_F32: PDIV_DIV3(float); break;
    case PDIV_F16: PDIV_DIV3(__half); break;
    case PDIV_BF16: PDIV_DIV3(bf16_t); break;
    default: return hipErrorInvalidValue;
  }
#undef PDIV_DIV3
  return hipGetLastError();
}

namespace {

template <bool FUSED, bool LINES, typename T>
hipError_t launch_lcp3d_kcs(const Planes6& src, int z, int y, int x, const StencilCoef3& k,
                            const IsoChunk& iso, int kc, float* out, int64_t pitch, int64_t plane,
                            hipStream_t s) {
  switch (kc) {
    case 1: return launch_lcp3d_kc<1, 4, FUSED, LINES, T>(src, z, y, x, k, iso, out, pitch, plane, s);
    case 2: return launch_lcp3d_kc<2, 4, FUSED, LINES, T>(src, z, y, x, k, iso, out, pitch, plane, s);
    case 4: return launch_lcp3d_kc<4, 4, FUSED, LINES, T>(src, z, y, x, k, iso, out, pitch, plane, s);
    // two-step: 4 layers at 8 isovalues (16 come as two launches); fused: the
    // moment rows' registers leave room for 2 layers at 8 and 16
    case 8:
      if constexpr (FUSED)
        return launch_lcp3d_kc<8, 2, FUSED, LINES, T>(src, z, y, x, k, iso, out, pitch, plane, s);
      else
        return launch_lcp3d_kc<8, 4, FUSED, LINES, T>(src, z, y, x, k, iso, out, pitch, plane, s);
    case 16:
      if constexpr (FUSED)
        return launch_lcp3d_kc<16, 2, FUSED, LINES, T>(src, z, y, x, k, iso, out, pitch, plane, s);
      else
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

// The line-aligned tile when every output row starts on a 128-byte line.
template <bool FUSED, typename T>
hipError_t launch_lcp3d_any(const Planes6& src, int64_t nz, int64_t ny, int64_t nx,
                            const StencilCoef3& k, const IsoChunk& iso, int kc, float* out_k0,
                            int64_t pitch, int64_t plane, hipStream_t s) {
  if (!lcp3d_slice_fits(ny, nx, sizeof(T))) return hipErrorInvalidValue;
  const int z = int(nz), y = int(ny), x = int(nx);
  const bool lines = (reinterpret_cast<uintptr_t>(out_k0) % 128 == 0) && pitch % 32 == 0 &&
                     plane % 32 == 0;
  return lines ? launch_lcp3d_kcs<FUSED, true, T>(src, z, y, x, k, iso, kc, out_k0, pitch, plane, s)
               : launch_lcp3d_kcs<FUSED, false, T>(src, z, y, x, k, iso, kc, out_k0, pitch, plane, s);
}

}  // namespace

hipError_t launch_lcp3d(const float* dm, const float* dv, int64_t nz, int64_t ny, int64_t nx,
                        const IsoChunk& iso, int kc, float* out_k0, int64_t pitch, int64_t plane,
                        hipStream_t s) {
  const Planes6 src{{dm, dv, nullptr, nullptr, nullptr, nullptr}};
  return launch_lcp3d_any<false, float>(src, nz, ny, nx, StencilCoef3{}, iso, kc, out_k0, pitch,
                                        plane, s);
}

hipError_t launch_lcp3d_fused(const void* const* planes, pdiv_dtype dt, int64_t nz, int64_t ny,
                              int64_t nx, const StencilCoef3& k, const IsoChunk& iso, int kc,
                              float* out_k0, int64_t pitch, int64_t plane, hipStream_t s) {
  const Planes6 src{{planes[0], planes[1], planes[2], planes[3], planes[4], planes[5]}};
  switch (dt) {
    case PDIV_F32:
      return launch_lcp3d_any<true, float>(src, nz, ny, nx, k, iso, kc, out_k0, pitch, plane, s);
    case PDIV_F16:
      return launch_lcp3d_any<true, __half>(src, nz, ny, nx, k, iso, kc, out_k0, pitch, plane, s);
    case PDIV_BF16:
      return launch_lcp3d_any<true, bf16_t>(src, nz, ny, nx, k, iso, kc, out_k0, pitch, plane, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pdiv
