// Divergence Gaussians (Eq. 2-3) and the closed-form level-crossing
// probability (Section 3.1), standalone and fused.
//
// Column-walking tiles: a wave owns 128 consecutive vertex columns, i.e. the
// 127 cells between them, over a band of cell rows.  Lane L holds vertex
// columns x0 + 2L and x0 + 2L + 1 and walks down the band one vertex row at a
// time.  For each isovalue it evaluates each corner's tail once per row,
// pairs it with the previous row's (vertical pairs, kept in registers) and
// forms its two cells: the left one from its own two columns, the right one
// with the first column of lane L+1, fetched by a lane shuffle.  Lane 63's
// right cell belongs to the next strip and is not stored.  The kernel is
// bound by the per-(corner, isovalue) tail and per-(cell, isovalue) combine
// arithmetic and by the LCP stores, which are written once with
// non-temporal stores (the maps are not re-read by this kernel).
#include "pdiv_device.hpp"
#include "pdiv_internal.hpp"

namespace pdiv {

StencilCoef make_coef(double dx, double dy) {
  StencilCoef k;
  k.cxm_in = static_cast<float>(1.0 / (2.0 * dx));
  k.cxv_in = static_cast<float>(1.0 / (4.0 * dx * dx));
  k.cxm_bd = static_cast<float>(1.0 / dx);
  k.cxv_bd = static_cast<float>(1.0 / (dx * dx));
  k.cym_in = static_cast<float>(1.0 / (2.0 * dy));
  k.cyv_in = static_cast<float>(1.0 / (4.0 * dy * dy));
  k.cym_bd = static_cast<float>(1.0 / dy);
  k.cyv_bd = static_cast<float>(1.0 / (dy * dy));
  return k;
}

LcpShape default_lcp_shape(int64_t ny, int64_t nx, int n_iso) {
  (void)nx;
  (void)n_iso;
  LcpShape s;
  s.band_rows = ny > 4096 ? 64 : 32;
  return s;
}

namespace {

constexpr int kWave = 64;
constexpr int kColsPerLane = 2;
constexpr int kCellsPerWave = kWave * kColsPerLane - 1;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

// Divergence Gaussian of vertex (x, j) from the moment planes, with the
// one-sided differences of Eq. 1 on the boundary.  Row pointers are formed
// from the row index first so that, when j is uniform across the wave, the
// address is a scalar base plus a 32-bit per-lane column offset.
template <typename T>
__device__ __forceinline__ DivGauss vertex_from_moments(const T* __restrict__ mu,
                                                        const T* __restrict__ vu,
                                                        const T* __restrict__ mv,
                                                        const T* __restrict__ vv, int ny,
                                                        int nx, uint32_t x, int j,
                                                        const StencilCoef& k) {
  const uint32_t xl = x > 0 ? x - 1 : 0;
  const uint32_t xr = x < uint32_t(nx - 1) ? x + 1 : uint32_t(nx - 1);
  const int yl = j > 0 ? j - 1 : 0;
  const int yr = j < ny - 1 ? j + 1 : ny - 1;
  const bool bx = (x == 0) | (x == uint32_t(nx - 1));
  const bool by = (j == 0) | (j == ny - 1);
  const int64_t r0 = static_cast<int64_t>(j) * nx;
  const int64_t rl = static_cast<int64_t>(yl) * nx;
  const int64_t rr = static_cast<int64_t>(yr) * nx;
  return div_gauss(to_f32(*at(mu + r0, xl)), to_f32(*at(mu + r0, xr)), to_f32(*at(vu + r0, xl)),
                   to_f32(*at(vu + r0, xr)), to_f32(*at(mv + rl, x)), to_f32(*at(mv + rr, x)),
                   to_f32(*at(vv + rl, x)), to_f32(*at(vv + rr, x)), bx ? k.cxm_bd : k.cxm_in,
                   bx ? k.cxv_bd : k.cxv_in, by ? k.cym_bd : k.cym_in,
                   by ? k.cyv_bd : k.cyv_in);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void divergence_kernel(const T* __restrict__ mu,
                                                            const T* __restrict__ vu,
                                                            const T* __restrict__ mv,
                                                            const T* __restrict__ vv, int ny,
                                                            int nx, StencilCoef k,
                                                            float* __restrict__ dmean,
                                                            float* __restrict__ dvar,
                                                            int rows_per_thread) {
  const int x = blockIdx.x * kWave + (threadIdx.x & 63);
  const int j0 = (blockIdx.y * kWavesPerBlock + (threadIdx.x >> 6)) * rows_per_thread;
  if (x >= nx) return;
  const int j1 = min(j0 + rows_per_thread, ny);
  for (int j = j0; j < j1; ++j) {
    DivGauss g = vertex_from_moments(mu, vu, mv, vv, ny, nx, uint32_t(x), j, k);
    const int64_t o = static_cast<int64_t>(j) * nx + x;
    __builtin_nontemporal_store(g.mean, dmean + o);
    __builtin_nontemporal_store(g.var, dvar + o);
  }
}

template <bool FUSED, typename T>
__device__ __forceinline__ Corner load_corner(const T* __restrict__ p0, const T* __restrict__ p1,
                                              const T* __restrict__ p2,
                                              const T* __restrict__ p3, int ny, int nx,
                                              uint32_t x, int j, const StencilCoef& k) {
  if constexpr (FUSED) {
    return make_corner(vertex_from_moments(p0, p1, p2, p3, ny, nx, x, j, k));
  } else {
    const int64_t r0 = static_cast<int64_t>(j) * nx;
    DivGauss g;
    g.mean = to_f32(*at(p0 + r0, x));
    g.var = to_f32(*at(p1 + r0, x));
    return make_corner(g);
  }
}

__device__ __forceinline__ Pair pair_from_right(const Pair& p) {
  Pair r;
  r.pa = __shfl_down(p.pa, 1, kWave);
  r.qa = __shfl_down(p.qa, 1, kWave);
  r.pb = __shfl_down(p.pb, 1, kWave);
  r.qb = __shfl_down(p.qb, 1, kWave);
  return r;
}

// One vertex row step: corners of row j+1 for the lane's two columns, their
// pairs with row j (prev_*), the lane's two cells for every isovalue; the new
// corners replace the old ones in next_*.
template <int KC, bool FUSED, typename T>
__device__ __forceinline__ void row_step(const T* __restrict__ p0, const T* __restrict__ p1,
                                         const T* __restrict__ p2, const T* __restrict__ p3,
                                         int ny, int nx, const StencilCoef& k,
                                         const IsoChunk& iso, float* __restrict__ out,
                                         int64_t plane, int j, uint32_t xa_c, uint32_t xb_c,
                                         uint32_t xa, bool store_a, bool store_b,
                                         const AB (&prev_a)[KC], const AB (&prev_b)[KC],
                                         AB (&next_a)[KC], AB (&next_b)[KC]) {
  const Corner ca = load_corner<FUSED>(p0, p1, p2, p3, ny, nx, xa_c, j + 1, k);
  const Corner cb = load_corner<FUSED>(p0, p1, p2, p3, ny, nx, xb_c, j + 1, k);
  float* __restrict__ orow = out + static_cast<int64_t>(j) * (nx - 1);
#pragma unroll
  for (int q = 0; q < KC; ++q) {
    const AB cur_a = corner_probs(ca, iso.c[q]);
    const AB cur_b = corner_probs(cb, iso.c[q]);
    const Pair pa = make_pair(prev_a[q], cur_a);
    const Pair pb = make_pair(prev_b[q], cur_b);
    const Pair right = pair_from_right(pa);
    const float l0 = cell_lcp(pa, pb, cur_a.below);
    const float l1 = cell_lcp(pb, right, cur_b.below);
    const RowWriter w(orow + q * plane);
    if (store_a) w.put(l0, xa * 4u);
    if (store_b) w.put(l1, xa * 4u + 4u);
    next_a[q] = cur_a;
    next_b[q] = cur_b;
  }
}

template <int KC, bool FUSED, typename T>
__global__ __launch_bounds__(kBlock) void lcp_kernel(const T* __restrict__ p0,
                                                     const T* __restrict__ p1,
                                                     const T* __restrict__ p2,
                                                     const T* __restrict__ p3, int ny, int nx,
                                                     StencilCoef k, IsoChunk iso,
                                                     float* __restrict__ out, int64_t plane,
                                                     int band_rows, int n_strips,
                                                     int n_bands) {
  const uint32_t lane = threadIdx.x & 63;
  // the wave index is uniform: row indices and row base pointers stay scalar
  const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock +
                                                  (threadIdx.x >> 6));
  const int strip = wave % n_strips;
  const int band = wave / n_strips;
  if (band >= n_bands) return;
  const uint32_t xa = uint32_t(strip * kCellsPerWave) + kColsPerLane * lane;  // first column
  const uint32_t xb = xa + 1;                                                 // second column
  const uint32_t last = uint32_t(nx - 1);
  const uint32_t xa_c = xa < last ? xa : last;  // columns past the edge load a valid column
  const uint32_t xb_c = xb < last ? xb : last;
  const bool store_a = xa < last;
  const bool store_b = (lane < kWave - 1) & (xb < last);
  const int j0 = band * band_rows;
  const int j1 = min(j0 + band_rows, ny - 1);

  AB ra[KC], rb[KC], sa[KC], sb[KC];
  {
    const Corner ca = load_corner<FUSED>(p0, p1, p2, p3, ny, nx, xa_c, j0, k);
    const Corner cb = load_corner<FUSED>(p0, p1, p2, p3, ny, nx, xb_c, j0, k);
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      ra[q] = corner_probs(ca, iso.c[q]);
      rb[q] = corner_probs(cb, iso.c[q]);
    }
  }
  // two rows per trip so the carried corners alternate between two register
  // sets instead of being copied
  for (int j = j0; j < j1; j += 2) {
    row_step<KC, FUSED>(p0, p1, p2, p3, ny, nx, k, iso, out, plane, j, xa_c, xb_c, xa,
                        store_a, store_b, ra, rb, sa, sb);
    if (j + 1 < j1)
      row_step<KC, FUSED>(p0, p1, p2, p3, ny, nx, k, iso, out, plane, j + 1, xa_c, xb_c, xa,
                          store_a, store_b, sa, sb, ra, rb);
  }
}

template <int KC, bool FUSED, typename T>
hipError_t launch_kc(const void* p0, const void* p1, const void* p2, const void* p3, int ny,
                     int nx, const StencilCoef& k, const IsoChunk& iso, float* out,
                     LcpShape shape, hipStream_t s) {
  const int n_strips = (nx - 1 + kCellsPerWave - 1) / kCellsPerWave;
  const int n_bands = (ny - 1 + shape.band_rows - 1) / shape.band_rows;
  const int64_t waves = static_cast<int64_t>(n_strips) * n_bands;
  const unsigned blocks = static_cast<unsigned>((waves + kWavesPerBlock - 1) / kWavesPerBlock);
  const int64_t plane = static_cast<int64_t>(ny - 1) * (nx - 1);
  hipLaunchKernelGGL((lcp_kernel<KC, FUSED, T>), dim3(blocks), dim3(kBlock), 0, s,
                     static_cast<const T*>(p0), static_cast<const T*>(p1),
                     static_cast<const T*>(p2), static_cast<const T*>(p3), ny, nx, k, iso, out,
                     plane, shape.band_rows, n_strips, n_bands);
  return hipGetLastError();
}

template <bool FUSED, typename T>
hipError_t launch_any(const void* p0, const void* p1, const void* p2, const void* p3, int ny,
                      int nx, const StencilCoef& k, const IsoChunk& iso, int kc, float* out,
                      LcpShape shape, hipStream_t s) {
  switch (kc) {
    case 1: return launch_kc<1, FUSED, T>(p0, p1, p2, p3, ny, nx, k, iso, out, shape, s);
    case 2: return launch_kc<2, FUSED, T>(p0, p1, p2, p3, ny, nx, k, iso, out, shape, s);
    case 4: return launch_kc<4, FUSED, T>(p0, p1, p2, p3, ny, nx, k, iso, out, shape, s);
    case 8: return launch_kc<8, FUSED, T>(p0, p1, p2, p3, ny, nx, k, iso, out, shape, s);
    case 16: return launch_kc<16, FUSED, T>(p0, p1, p2, p3, ny, nx, k, iso, out, shape, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_divergence(const void* mu, const void* vu, const void* mv, const void* vv,
                             pdiv_dtype dt, int64_t ny, int64_t nx, const StencilCoef& k,
                             float* dmean, float* dvar, hipStream_t s) {
  constexpr int rows = 16;
  dim3 grid(static_cast<unsigned>((nx + kWave - 1) / kWave),
            static_cast<unsigned>((ny + rows * kWavesPerBlock - 1) / (rows * kWavesPerBlock)));
  const int iny = static_cast<int>(ny), inx = static_cast<int>(nx);
  switch (dt) {
    case PDIV_F32:
      hipLaunchKernelGGL(divergence_kernel<float>, grid, dim3(kBlock), 0, s,
                         static_cast<const float*>(mu), static_cast<const float*>(vu),
                         static_cast<const float*>(mv), static_cast<const float*>(vv), iny, inx,
                         k, dmean, dvar, rows);
      break;
    case PDIV_F16:
      hipLaunchKernelGGL(divergence_kernel<__half>, grid, dim3(kBlock), 0, s,
                         static_cast<const __half*>(mu), static_cast<const __half*>(vu),
                         static_cast<const __half*>(mv), static_cast<const __half*>(vv), iny,
                         inx, k, dmean, dvar, rows);
      break;
    case PDIV_BF16:
      hipLaunchKernelGGL(divergence_kernel<bf16_t>, grid, dim3(kBlock), 0, s,
                         static_cast<const bf16_t*>(mu), static_cast<const bf16_t*>(vu),
                         static_cast<const bf16_t*>(mv), static_cast<const bf16_t*>(vv), iny,
                         inx, k, dmean, dvar, rows);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_lcp(bool fused, const void* p0, const void* p1, const void* p2,
                      const void* p3, pdiv_dtype dt, int64_t ny, int64_t nx,
                      const StencilCoef& k, const IsoChunk& iso, int kc, float* lcp_k0,
                      LcpShape shape, hipStream_t s) {
  const int iny = static_cast<int>(ny), inx = static_cast<int>(nx);
  if (!fused)
    return launch_any<false, float>(p0, p1, p2, p3, iny, inx, k, iso, kc, lcp_k0, shape, s);
  switch (dt) {
    case PDIV_F32:
      return launch_any<true, float>(p0, p1, p2, p3, iny, inx, k, iso, kc, lcp_k0, shape, s);
    case PDIV_F16:
      return launch_any<true, __half>(p0, p1, p2, p3, iny, inx, k, iso, kc, lcp_k0, shape, s);
    case PDIV_BF16:
      return launch_any<true, bf16_t>(p0, p1, p2, p3, iny, inx, k, iso, kc, lcp_k0, shape, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace pdiv
