// Divergence Gaussians (Eq. 2-3) and the closed-form level-crossing
// probability (Section 3.1), standalone and fused.
//
// Column-walking tiles: a wave owns 64 consecutive vertex columns, i.e. the 63
// cells between them, over a band of cell rows.  Lane L holds vertex column
// x0 + L and walks down the band one vertex row at a time.  For each isovalue
// it evaluates the corner tail once per vertex and row, pairs it with the
// previous row's (vertical pair, kept in registers) and takes the right-hand
// pair of the cell from lane L+1 by a lane shuffle; lane 63 only feeds lane
// 62.  Each LCP value is stored once, coalesced across the wave (64
// consecutive floats of one output row), with a non-temporal store.
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
constexpr int kCellsPerWave = kWave - 1;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

// Divergence Gaussian of vertex (x, j) from the moment planes, with the
// one-sided differences of Eq. 1 on the boundary.
template <typename T>
__device__ __forceinline__ DivGauss vertex_from_moments(const T* __restrict__ mu,
                                                        const T* __restrict__ vu,
                                                        const T* __restrict__ mv,
                                                        const T* __restrict__ vv, int ny,
                                                        int nx, int x, int j,
                                                        const StencilCoef& k) {
  const int xl = x > 0 ? x - 1 : 0;
  const int xr = x < nx - 1 ? x + 1 : nx - 1;
  const int yl = j > 0 ? j - 1 : 0;
  const int yr = j < ny - 1 ? j + 1 : ny - 1;
  const bool bx = (x == 0) | (x == nx - 1);
  const bool by = (j == 0) | (j == ny - 1);
  const int64_t row = static_cast<int64_t>(j) * nx;
  return div_gauss(ld(mu, row + xl), ld(mu, row + xr), ld(vu, row + xl), ld(vu, row + xr),
                   ld(mv, static_cast<int64_t>(yl) * nx + x),
                   ld(mv, static_cast<int64_t>(yr) * nx + x),
                   ld(vv, static_cast<int64_t>(yl) * nx + x),
                   ld(vv, static_cast<int64_t>(yr) * nx + x), bx ? k.cxm_bd : k.cxm_in,
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
    DivGauss g = vertex_from_moments(mu, vu, mv, vv, ny, nx, x, j, k);
    const int64_t o = static_cast<int64_t>(j) * nx + x;
    __builtin_nontemporal_store(g.mean, dmean + o);
    __builtin_nontemporal_store(g.var, dvar + o);
  }
}

template <bool FUSED, typename T>
__device__ __forceinline__ Corner load_corner(const T* __restrict__ p0, const T* __restrict__ p1,
                                              const T* __restrict__ p2,
                                              const T* __restrict__ p3, int ny, int nx, int x,
                                              int j, const StencilCoef& k) {
  if constexpr (FUSED) {
    return make_corner(vertex_from_moments(p0, p1, p2, p3, ny, nx, x, j, k));
  } else {
    const int64_t o = static_cast<int64_t>(j) * nx + x;
    DivGauss g;
    g.mean = ld(p0, o);
    g.var = ld(p1, o);
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

template <int KC, bool FUSED, typename T>
__global__ __launch_bounds__(kBlock) void lcp_kernel(const T* __restrict__ p0,
                                                     const T* __restrict__ p1,
                                                     const T* __restrict__ p2,
                                                     const T* __restrict__ p3, int ny, int nx,
                                                     StencilCoef k, IsoChunk iso,
                                                     float* __restrict__ out, int64_t plane,
                                                     int band_rows, int n_strips,
                                                     int n_bands) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  const int strip = wave % n_strips;
  const int band = wave / n_strips;
  if (band >= n_bands) return;  // uniform per wave
  const int x = strip * kCellsPerWave + lane;
  const int xc = x < nx ? x : nx - 1;  // lanes past the edge load a valid column
  const bool store = (lane < kCellsPerWave) & (x < nx - 1);
  const int ncx = nx - 1;
  const int j0 = band * band_rows;
  const int j1 = min(j0 + band_rows, ny - 1);

  AB prev[KC];
  {
    const Corner c = load_corner<FUSED>(p0, p1, p2, p3, ny, nx, xc, j0, k);
#pragma unroll
    for (int q = 0; q < KC; ++q) prev[q] = corner_probs(c, iso.c[q]);
  }
  for (int j = j0; j < j1; ++j) {
    const Corner c = load_corner<FUSED>(p0, p1, p2, p3, ny, nx, xc, j + 1, k);
    float* orow = out + static_cast<int64_t>(j) * ncx + x;
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      const AB cur = corner_probs(c, iso.c[q]);
      const Pair left = make_pair(prev[q], cur);
      const Pair right = pair_from_right(left);
      const float l = cell_lcp(left, right);
      if (store) __builtin_nontemporal_store(l, orow + q * plane);
      prev[q] = cur;
    }
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
#define PDIV_KC(N) \
  case N: return launch_kc<N, FUSED, T>(p0, p1, p2, p3, ny, nx, k, iso, out, shape, s);
    PDIV_KC(1) PDIV_KC(2) PDIV_KC(3) PDIV_KC(4) PDIV_KC(5) PDIV_KC(6) PDIV_KC(7) PDIV_KC(8)
    PDIV_KC(9) PDIV_KC(10) PDIV_KC(11) PDIV_KC(12) PDIV_KC(13) PDIV_KC(14) PDIV_KC(15)
    PDIV_KC(16)
#undef PDIV_KC
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
