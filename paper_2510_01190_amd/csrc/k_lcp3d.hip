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
constexpr int kBandRows3 = 32;

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

// Waves: strip (fastest), then layer group, then band, over an XCD-aware
// block order: blocks are dealt round-robin to the 8 XCDs, each with its own
// L2, so each XCD is given a contiguous run of blocks and the strips that
// share an output row's cache lines write them through the same L2
// (measured at 512^3: 1.03 ms against 1.19 ms with layer groups fastest at
// 4 isovalues).  Every lane stays active through the DPP reads:
// lanes past the grid clamp their column.  Loads and stores go through
// buffer resources with a scalar row base and a per-lane byte offset; a
// store row is sized to the strip's cells, so the buffer hardware drops the
// stores of lane 63 and of lanes past the grid (no branch around them).
// Each row's inputs are loaded one row ahead, so their latency overlaps the
// previous row's arithmetic.
// The input planes of one launch: the two divergence volumes (dm, dv as
// float) or, fused, the six moment volumes of type T.
struct Planes6 {
  const void* p[6];
};

// FUSED: each row's corners come from Eq. 2-3 with the z term evaluated on
// the spot from the six moment volumes (the divergence never reaches HBM):
// U's x neighbours and V's y neighbours are read directly, W once per row at
// the levels k0-1 .. k0+LZ+1 and shared by adjacent levels; the operands and
// their order are those of divergence3d_kernel, so the maps are bitwise the
// two-step result.
template <int KC, int LZ, bool FUSED, typename T>
__global__ __launch_bounds__(kBlock) void lcp3d_kernel(Planes6 src, int nz, int ny, int nx,
                                                       StencilCoef3 k, IsoChunk iso,
                                                       float* __restrict__ out, int64_t plane,
                                                       int n_groups, int n_strips, int n_bands) {
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
  const int j0 = band * kBandRows3;
  const int j1 = min(j0 + kBandRows3, ny - 1);
  const int x0 = strip * 63;
  const uint32_t xoff = uint32_t(min(x0 + lane, nx - 1)) * 4u;
  const uint32_t store_bytes = uint32_t(min(63, nx - 1 - x0)) * 4u;
  const uint32_t soff = uint32_t(lane) * 4u;
  const int64_t cells_x = nx - 1;
  const int64_t layer = int64_t(ny - 1) * cells_x;
  const int64_t vplane = int64_t(ny) * nx;
  float pm[LZ + 1], pv[LZ + 1];
  const Col col = make_col(uint32_t(min(x0 + lane, nx - 1)), nx, sizeof(T));
  const float cxm = col.bx ? k.xy.cxm_bd : k.xy.cxm_in;
  const float cxv = col.bx ? k.xy.cxv_bd : k.xy.cxv_in;
  // FUSED: V at rows clamp(j-1) and j of every level, carried from row to
  // row, so each V row is loaded once per wave
  float vwin_m[LZ + 1][2], vwin_v[LZ + 1][2];
  if constexpr (FUSED) {
    const T* const mv = static_cast<const T*>(src.p[2]);
    const T* const vv = static_cast<const T*>(src.p[3]);
#pragma unroll
    for (int l = 0; l <= LZ; ++l) {
      const int kk = min(k0 + l, nz - 1);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int y = h == 0 ? (j0 > 0 ? j0 - 1 : 0) : j0;
        const int64_t row = int64_t(kk) * vplane + int64_t(y) * nx;
        vwin_m[l][h] = RowReader<T>(mv + row, nx).get(col.x);
        vwin_v[l][h] = RowReader<T>(vv + row, nx).get(col.x);
      }
    }
  }
  auto load_row = [&](int j) {
    if constexpr (FUSED) {
      const T* const mu = static_cast<const T*>(src.p[0]);
      const T* const vu = static_cast<const T*>(src.p[1]);
      const T* const mv = static_cast<const T*>(src.p[2]);
      const T* const vv = static_cast<const T*>(src.p[3]);
      const T* const mw = static_cast<const T*>(src.p[4]);
      const T* const vw = static_cast<const T*>(src.p[5]);
      const int yr = j < ny - 1 ? j + 1 : ny - 1;
      const bool by = (j == 0) | (j == ny - 1);
      const float cym = by ? k.xy.cym_bd : k.xy.cym_in, cyv = by ? k.xy.cyv_bd : k.xy.cyv_in;
      // W at levels clamp(k0 - 1 + t), t = 0 .. LZ + 2: level k0 + l has its
      // clamped z neighbours at t = l and t = l + 2
      float wm[LZ + 3], wv[LZ + 3];
#pragma unroll
      for (int t = 0; t < LZ + 3; ++t) {
        const int lev = min(max(k0 - 1 + t, 0), nz - 1);
        const int64_t row = int64_t(lev) * vplane + int64_t(j) * nx;
        wm[t] = RowReader<T>(mw + row, nx).get(col.x);
        wv[t] = RowReader<T>(vw + row, nx).get(col.x);
      }
#pragma unroll
      for (int l = 0; l <= LZ; ++l) {
        const int kk = min(k0 + l, nz - 1);
        const int64_t row = int64_t(kk) * vplane + int64_t(j) * nx;
        const int64_t row_yr = int64_t(kk) * vplane + int64_t(yr) * nx;
        const RowReader<T> u0(mu + row, nx), s0(vu + row, nx);
        const float vmr = RowReader<T>(mv + row_yr, nx).get(col.x);
        const float vvr = RowReader<T>(vv + row_yr, nx).get(col.x);
        const bool bz = (kk == 0) | (kk == nz - 1);
        const DivGauss g = div_gauss3(
            u0.get(col.xl), u0.get(col.xr), s0.get(col.xl), s0.get(col.xr), vwin_m[l][0], vmr,
            vwin_v[l][0], vvr, wm[l], wm[l + 2], wv[l], wv[l + 2], cxm, cxv, cym, cyv,
            bz ? k.czm_bd : k.czm_in, bz ? k.czv_bd : k.czv_in);
        pm[l] = g.mean;
        pv[l] = g.var;
        // the window moves one row: rows clamp(j), clamp(j+1) become the
        // next row's lower and centre rows
        vwin_m[l][0] = vwin_m[l][1];
        vwin_v[l][0] = vwin_v[l][1];
        vwin_m[l][1] = vmr;
        vwin_v[l][1] = vvr;
      }
    } else {
      const float* const dm = static_cast<const float*>(src.p[0]);
      const float* const dv = static_cast<const float*>(src.p[1]);
#pragma unroll
      for (int l = 0; l <= LZ; ++l) {
        const int64_t row = int64_t(min(k0 + l, nz - 1)) * vplane + int64_t(j) * nx;
        pm[l] = RowReader<float>(dm + row, nx).get(xoff);
        pv[l] = RowReader<float>(dv + row, nx).get(xoff);
      }
    }
  };
  load_row(j0);
  Pair carry[LZ][KC];
  for (int j = j0; j <= j1; ++j) {
    Corner c[LZ + 1];
#pragma unroll
    for (int l = 0; l <= LZ; ++l) {
      DivGauss g;
      g.mean = pm[l];
      g.var = pv[l];
      c[l] = make_corner(g);
    }
    if (j < j1) load_row(j + 1);
    float* const row_out = out + int64_t(k0) * layer + int64_t(j - 1) * cells_x + x0;
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      AB ab[LZ + 1];
#pragma unroll
      for (int l = 0; l <= LZ; ++l) ab[l] = corner_probs(c[l], iso.c[q]);
#pragma unroll
      for (int l = 0; l < LZ; ++l) {
        const Pair zp = make_pair(ab[l], ab[l + 1]);
        if (j > j0) {
          float v = cell_lcp_dpp(join_pairs(carry[l][q], zp), ab[l].below);
          // with 8 corners the float32 combination can land an ulp outside
          // [0, 1] where the probability is 0 or 1; the exact value is inside,
          // so clamping only removes error (NaN fails both tests and stays)
          v = v < 0.0f ? 0.0f : v;
          v = v > 1.0f ? 1.0f : v;
          if (l < nl)
            RowWriter<false>(row_out + int64_t(q) * plane + int64_t(l) * layer, store_bytes)
                .put(v, soff);
        }
        carry[l][q] = zp;
      }
    }
  }
}

template <int KC, int LZ, bool FUSED, typename T>
hipError_t launch_lcp3d_kc(const Planes6& src, int nz, int ny, int nx, const StencilCoef3& k,
                           const IsoChunk& iso, float* out, int64_t plane, hipStream_t s) {
  const int n_groups = (nz - 1 + LZ - 1) / LZ;
  const int n_strips = (nx - 1 + 62) / 63;
  const int n_bands = (ny - 1 + kBandRows3 - 1) / kBandRows3;
  const int64_t waves = int64_t(n_groups) * n_strips * n_bands;
  const int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
  if (!launch_fits(blocks, kBlock)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((lcp3d_kernel<KC, LZ, FUSED, T>), dim3(unsigned(blocks)), dim3(kBlock), 0, s,
                     src, nz, ny, nx, k, iso, out, plane, n_groups, n_strips, n_bands);
  return hipGetLastError();
}

}  // namespace

int64_t lcp3d_blocks(int64_t nz, int64_t ny, int64_t nx, int kc) {
  const int lz = kc <= 4 ? 4 : 2;
  const int64_t waves = ((nz - 1 + lz - 1) / lz) * ((nx - 1 + 62) / 63) *
                        ((ny - 1 + kBandRows3 - 1) / kBandRows3);
  return (waves + kWavesPerBlock - 1) / kWavesPerBlock;
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

template <bool FUSED, typename T>
hipError_t launch_lcp3d_any(const Planes6& src, int64_t nz, int64_t ny, int64_t nx,
                            const StencilCoef3& k, const IsoChunk& iso, int kc, float* out_k0,
                            int64_t plane, hipStream_t s) {
  const int z = int(nz), y = int(ny), x = int(nx);
  switch (kc) {
    case 1: return launch_lcp3d_kc<1, 4, FUSED, T>(src, z, y, x, k, iso, out_k0, plane, s);
    case 2: return launch_lcp3d_kc<2, 4, FUSED, T>(src, z, y, x, k, iso, out_k0, plane, s);
    case 4: return launch_lcp3d_kc<4, 4, FUSED, T>(src, z, y, x, k, iso, out_k0, plane, s);
    case 8: return launch_lcp3d_kc<8, 2, FUSED, T>(src, z, y, x, k, iso, out_k0, plane, s);
    case 16: return launch_lcp3d_kc<16, 2, FUSED, T>(src, z, y, x, k, iso, out_k0, plane, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_lcp3d(const float* dm, const float* dv, int64_t nz, int64_t ny, int64_t nx,
                        const IsoChunk& iso, int kc, float* out_k0, int64_t plane,
                        hipStream_t s) {
  const Planes6 src{{dm, dv, nullptr, nullptr, nullptr, nullptr}};
  return launch_lcp3d_any<false, float>(src, nz, ny, nx, StencilCoef3{}, iso, kc, out_k0, plane,
                                        s);
}

hipError_t launch_lcp3d_fused(const void* const* planes, pdiv_dtype dt, int64_t nz, int64_t ny,
                              int64_t nx, const StencilCoef3& k, const IsoChunk& iso, int kc,
                              float* out_k0, int64_t plane, hipStream_t s) {
  const Planes6 src{{planes[0], planes[1], planes[2], planes[3], planes[4], planes[5]}};
  switch (dt) {
    case PDIV_F32: return launch_lcp3d_any<true, float>(src, nz, ny, nx, k, iso, kc, out_k0, plane, s);
    case PDIV_F16: return launch_lcp3d_any<true, __half>(src, nz, ny, nx, k, iso, kc, out_k0, plane, s);
    case PDIV_BF16: return launch_lcp3d_any<true, bf16_t>(src, nz, ny, nx, k, iso, kc, out_k0, plane, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pdiv
