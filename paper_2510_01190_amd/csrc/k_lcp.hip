// Divergence Gaussians (Eq. 2-3) and the closed-form level-crossing
// probability (Section 3.1), standalone and fused, for one field.  The tile
// walk itself lives in lcp_tile.hpp; here a grid of waves covers the field's
// strips x bands, one tile per wave.
#include <atomic>
#include <type_traits>

#include "lcp_tile.hpp"

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

static std::atomic<int> g_band_rows_override{0};

void set_band_rows_override(int rows) { g_band_rows_override.store(rows); }

// Rows per band: each band re-reads two halo rows and re-evaluates one corner
// row, and short bands give more waves to even out the tail of the launch.
// On gfx950, 8191 x 8191 cells at K = 16: the paired tile (64 strips) ran
// 1.26 ms with 64-row bands against 1.32 (48 rows), 1.37 (96) and 1.30 (128);
// the split tile (65 strips, dense rows) 1.45 ms with 16-row bands against
// 1.50 (8) and 1.55 (64).  0 in band_rows: this choice, made per layout.
LcpShape default_lcp_shape(int64_t ny, int64_t nx, int n_iso) {
  (void)nx;
  (void)n_iso;
  (void)ny;
  LcpShape s;
  s.band_rows = g_band_rows_override.load();
  s.poison = (debug_flags() & PDIV_DEBUG_POISON_LDS) != 0;
  return s;
}

int band_rows_for(const LcpShape& s, int64_t ny, bool paired) {
  if (s.band_rows > 0) return s.band_rows;
  if (ny <= 4096) return 32;
  return paired ? 64 : 16;
}

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

// Eq. 2-3 at every vertex.  A wave walks rows_per_thread rows of a strip of
// columns and keeps V's rows clamp(j-1), j, clamp(j+1) in a register window,
// so each V row is loaded once.  U's x neighbours depend on the storage:
//   32-bit  the strip is 64 columns; each lane loads its two neighbours,
//           which the L1 serves from the lines of the row already in flight;
//   16-bit  the strip is 62 columns in 64 lanes (lanes 0 and 63 hold the x
//           halo); each lane loads only its own column and takes the
//           neighbours from the adjacent lanes through DPP, with every lane
//           active, so no load straddles a cache line.
// Measured at 8192^2: the DPP form takes 0.39 ms for 16-bit storage against
// 0.55 ms with neighbour loads, but 0.49 ms for 32-bit against 0.36 ms (its
// 62-column strips put the row segments off cache-line boundaries).  Either
// way the operands are those of a straight evaluation with clamped
// neighbours.
template <typename T>
__global__ __launch_bounds__(kBlock) void divergence_kernel(const T* __restrict__ mu,
                                                            const T* __restrict__ vu,
                                                            const T* __restrict__ mv,
                                                            const T* __restrict__ vv, int ny,
                                                            int nx, StencilCoef k,
                                                            float* __restrict__ dmean,
                                                            float* __restrict__ dvar,
                                                            int rows_per_thread) {
  constexpr bool kDpp = sizeof(T) == 2;
  constexpr int kStrip = kDpp ? kWave - 2 : kWave;
  const int lane = threadIdx.x & 63;
  const int x = int(blockIdx.x) * kStrip + lane - (kDpp ? 1 : 0);
  // the wave index is uniform: row pointers stay scalar, and whole waves
  // leave together, so every DPP partner lane is active
  const int j0 =
      __builtin_amdgcn_readfirstlane(blockIdx.y * kWavesPerBlock + (threadIdx.x >> 6)) *
      rows_per_thread;
  if (j0 >= ny) return;
  if (!kDpp && x >= nx) return;
  const int j1 = min(j0 + rows_per_thread, ny);
  const Col c = make_col(uint32_t(x < 0 ? 0 : min(x, nx - 1)), nx, sizeof(T));
  const bool store = (x < nx) & (!kDpp | ((lane >= 1) & (lane <= kWave - 2)));
  auto v_at = [&](int y, float& m, float& v) {
    const int64_t row = static_cast<int64_t>(y) * nx;
    m = RowReader<T>(mv + row, nx).get(c.x);
    v = RowReader<T>(vv + row, nx).get(c.x);
  };
  float vm_l, vv_l, vm_c, vv_c, vm_r, vv_r;
  v_at(j0 > 0 ? j0 - 1 : 0, vm_l, vv_l);
  v_at(j0, vm_c, vv_c);
  for (int j = j0; j < j1; ++j) {
    v_at(j < ny - 1 ? j + 1 : ny - 1, vm_r, vv_r);
    const int64_t row = static_cast<int64_t>(j) * nx;
    const RowReader<T> u0(mu + row, nx);
    const RowReader<T> w0(vu + row, nx);
    Raw<true> r;
    if constexpr (kDpp) {
      const float um = u0.get(c.x);
      const float us = w0.get(c.x);
      const float um_l = dpp_from_left(um), um_r = dpp_from_right(um);
      const float us_l = dpp_from_left(us), us_r = dpp_from_right(us);
      r.mu_l = x == 0 ? um : um_l;
      r.mu_r = x == nx - 1 ? um : um_r;
      r.vu_l = x == 0 ? us : us_l;
      r.vu_r = x == nx - 1 ? us : us_r;
    } else {
      r.mu_l = u0.get(c.xl);
      r.mu_r = u0.get(c.xr);
      r.vu_l = w0.get(c.xl);
      r.vu_r = w0.get(c.xr);
    }
    r.mv_l = vm_l;
    r.mv_r = vm_r;
    r.vv_l = vv_l;
    r.vv_r = vv_r;
    const DivGauss g = raw_div(r, c.bx, j, ny, k);
    if (store) {
      __builtin_nontemporal_store(g.mean, dmean + row + x);
      __builtin_nontemporal_store(g.var, dvar + row + x);
    }
    vm_l = vm_c;
    vv_l = vv_c;
    vm_c = vm_r;
    vv_c = vv_r;
  }
}

template <int KC, bool FUSED, bool PAIRED, typename T, bool POISON = false,
          bool STREAM = PAIRED>
__device__ __forceinline__ void lcp_body(const T* __restrict__ p0,
                                                     const T* __restrict__ p1,
                                                     const T* __restrict__ p2,
                                                     const T* __restrict__ p3, int ny, int nx,
                                                     StencilCoef k, IsoChunk iso,
                                                     float* __restrict__ out, int64_t plane,
                                                     int64_t pitch, int band_rows, int n_strips,
                                                     int n_bands) {
  // Blocks are dealt round-robin to the 8 XCDs (block b runs on XCD b % 8),
  // each with its own L2.  Give each XCD a contiguous run of tiles, so that
  // neighbouring strips, whose output rows meet inside a cache line, write
  // that line through the same L2.  The map is a bijection on [0, gridDim.x).
  const int nb = gridDim.x, xcd = blockIdx.x % 8, q8 = nb / 8, r8 = nb % 8;
  const int blk = xcd * q8 + min(xcd, r8) + blockIdx.x / 8;
  // the wave index is uniform: row indices and row base pointers stay scalar
  const int wave = __builtin_amdgcn_readfirstlane(blk * kWavesPerBlock + (threadIdx.x >> 6));
  const int strip = wave % n_strips;
  const int band = wave / n_strips;
  if (band >= n_bands) return;
  const int j0 = band * band_rows;
  lcp_tile<KC, FUSED, PAIRED, T, POISON, STREAM>(p0, p1, p2, p3, ny, nx, k, iso, KC, out, plane,
                                                 pitch, strip, j0, min(j0 + band_rows, ny - 1));
}

// Paired-layout kernel: asks the compiler for three waves per SIMD (at most
// 168 VGPRs); with the alternating carried sets the tile needs one more, and
// one spill costs less than the third wave's absence or the per-row moves of
// a single set (measured on gfx950 at 8192^2, K = 16: 1.144 ms against 1.151).
// STREAM = false: the fused kernel on rows that start inside a line.
template <int KC, bool FUSED, typename T, bool POISON = false, bool STREAM = true>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void lcp_kernel_paired(
    const T* __restrict__ p0, const T* __restrict__ p1, const T* __restrict__ p2,
    const T* __restrict__ p3, int ny, int nx, StencilCoef k, IsoChunk iso, float* __restrict__ out,
    int64_t plane, int64_t pitch, int band_rows, int n_strips, int n_bands) {
  lcp_body<KC, FUSED, true, T, POISON, STREAM>(p0, p1, p2, p3, ny, nx, k, iso, out, plane, pitch,
                                               band_rows, n_strips, n_bands);
}

// Split-layout kernel (its tile has no LDS ring; two waves per SIMD).
template <int KC, bool FUSED, typename T>
__global__ __launch_bounds__(kBlock) void lcp_kernel_split(
    const T* __restrict__ p0, const T* __restrict__ p1, const T* __restrict__ p2,
    const T* __restrict__ p3, int ny, int nx, StencilCoef k, IsoChunk iso, float* __restrict__ out,
    int64_t plane, int64_t pitch, int band_rows, int n_strips, int n_bands) {
  lcp_body<KC, FUSED, false>(p0, p1, p2, p3, ny, nx, k, iso, out, plane, pitch, band_rows,
                             n_strips, n_bands);
}

// Dynamic LDS that leaves room for only two 4-wave blocks of `kernel` per CU
// (160 KiB of LDS: 3 x 54 KiB does not fit), i.e. two waves per SIMD instead
// of the three its registers allow.  The fused kernel's stores into rows that
// start inside a 128-byte line, and its launches at up to 4 isovalues, run
// faster with fewer waves writing at once (8192^2 at 16 isovalues into dense
// maps: 1.35 against 1.45 ms; at 8: 0.73 against 0.80 ms; line-aligned rows
// at 4 isovalues: 0.403 against 0.418 ms; line-aligned at 16: unchanged).
// Zero if the attributes cannot be read (the launch then runs at the usual
// occupancy).
template <typename Kernel>
size_t two_waves_per_simd_lds(Kernel kernel) {
  hipFuncAttributes a{};
  if (hipFuncGetAttributes(&a, reinterpret_cast<const void*>(kernel)) != hipSuccess) {
    (void)hipGetLastError();  // not the launch's error
    return 0;
  }
  constexpr size_t kPerBlock = 54 * 1024;
  return a.sharedSizeBytes < kPerBlock ? kPerBlock - a.sharedSizeBytes : 0;
}

template <int KC, bool FUSED, typename T>
hipError_t launch_kc(const void* p0, const void* p1, const void* p2, const void* p3, int ny,
                     int nx, const StencilCoef& k, const IsoChunk& iso, float* out,
                     int64_t pitch, int64_t plane, LcpShape shape, hipStream_t s) {
  const int64_t n_cells = int64_t(ny - 1) * (nx - 1);
  const bool lines = use_paired_tile(out, pitch, plane, KC, n_cells);
  // the fused kernel takes the paired tile on other rows too (default policy)
  const bool unaligned = FUSED && !lines && use_paired_unaligned(KC, n_cells);
  const bool paired = lines || unaligned;
  const int cells = cells_per_wave(paired);
  const int band_rows = band_rows_for(shape, ny, paired);
  const int n_strips = (nx - 1 + cells - 1) / cells;
  const int n_bands = (ny - 1 + band_rows - 1) / band_rows;
  const int64_t waves = static_cast<int64_t>(n_strips) * n_bands;
  if (!launch_fits((waves + kWavesPerBlock - 1) / kWavesPerBlock, kBlock))
    return hipErrorInvalidConfiguration;
  const unsigned blocks = static_cast<unsigned>((waves + kWavesPerBlock - 1) / kWavesPerBlock);
  if constexpr (FUSED && std::is_same<T, float>::value) {
    // the checking variant exists for the fused float32 kernel only
    if (paired && shape.poison) {
      if (unaligned)
        hipLaunchKernelGGL((lcp_kernel_paired<KC, FUSED, T, true, false>), dim3(blocks),
                           dim3(kBlock), 0, s, static_cast<const T*>(p0),
                           static_cast<const T*>(p1), static_cast<const T*>(p2),
                           static_cast<const T*>(p3), ny, nx, k, iso, out, plane, pitch,
                           band_rows, n_strips, n_bands);
      else
        hipLaunchKernelGGL((lcp_kernel_paired<KC, FUSED, T, true>), dim3(blocks), dim3(kBlock),
                           0, s, static_cast<const T*>(p0), static_cast<const T*>(p1),
                           static_cast<const T*>(p2), static_cast<const T*>(p3), ny, nx, k, iso,
                           out, plane, pitch, band_rows, n_strips, n_bands);
      return hipGetLastError();
    }
  }
  if constexpr (FUSED) {
    if (unaligned) {
      static const size_t lds =
          two_waves_per_simd_lds(lcp_kernel_paired<KC, FUSED, T, false, false>);
      hipLaunchKernelGGL((lcp_kernel_paired<KC, FUSED, T, false, false>), dim3(blocks),
                         dim3(kBlock), lds, s, static_cast<const T*>(p0),
                         static_cast<const T*>(p1), static_cast<const T*>(p2),
                         static_cast<const T*>(p3), ny, nx, k, iso, out, plane, pitch, band_rows,
                         n_strips, n_bands);
      return hipGetLastError();
    }
  }
  if (paired) {
    size_t lds = 0;
    if constexpr (FUSED && KC <= 4) {
      static const size_t two = two_waves_per_simd_lds(lcp_kernel_paired<KC, FUSED, T>);
      lds = two;
    }
    hipLaunchKernelGGL((lcp_kernel_paired<KC, FUSED, T>), dim3(blocks), dim3(kBlock), lds, s,
                       static_cast<const T*>(p0), static_cast<const T*>(p1),
                       static_cast<const T*>(p2), static_cast<const T*>(p3), ny, nx, k, iso, out,
                       plane, pitch, band_rows, n_strips, n_bands);
  }
  else
    hipLaunchKernelGGL((lcp_kernel_split<KC, FUSED, T>), dim3(blocks), dim3(kBlock), 0, s,
                       static_cast<const T*>(p0), static_cast<const T*>(p1),
                       static_cast<const T*>(p2), static_cast<const T*>(p3), ny, nx, k, iso, out,
                       plane, pitch, band_rows, n_strips, n_bands);
  return hipGetLastError();
}

template <bool FUSED, typename T>
hipError_t launch_any(const void* p0, const void* p1, const void* p2, const void* p3, int ny,
                      int nx, const StencilCoef& k, const IsoChunk& iso, int kc, float* out,
                      int64_t pitch, int64_t plane, LcpShape shape, hipStream_t s) {
  switch (kc) {
    case 1: return launch_kc<1, FUSED, T>(p0, p1, p2, p3, ny, nx, k, iso, out, pitch, plane, shape, s);
    case 2: return launch_kc<2, FUSED, T>(p0, p1, p2, p3, ny, nx, k, iso, out, pitch, plane, shape, s);
    case 4: return launch_kc<4, FUSED, T>(p0, p1, p2, p3, ny, nx, k, iso, out, pitch, plane, shape, s);
    case 8: return launch_kc<8, FUSED, T>(p0, p1, p2, p3, ny, nx, k, iso, out, pitch, plane, shape, s);
    case 16: return launch_kc<16, FUSED, T>(p0, p1, p2, p3, ny, nx, k, iso, out, pitch, plane, shape, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_divergence(const void* mu, const void* vu, const void* mv, const void* vv,
                             pdiv_dtype dt, int64_t ny, int64_t nx, const StencilCoef& k,
                             float* dmean, float* dvar, hipStream_t s) {
  // rows per wave: at 8192^2 float32 takes 0.314 / 0.311 / 0.309 / 0.317 ms
  // with 8 / 16 / 12 / 24 rows, 16-bit storage 0.310 / 0.347 / 0.366 / 0.377 ms
  const int rows = dt == PDIV_F32 ? 16 : 8;
  // strips of 64 columns for 32-bit storage, of 62 for 16-bit (DPP halo)
  const int64_t strip = dt == PDIV_F32 ? kWave : kWave - 2;
  dim3 grid(static_cast<unsigned>((nx + strip - 1) / strip),
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
                      int64_t pitch, int64_t plane, LcpShape shape, hipStream_t s) {
  const int iny = static_cast<int>(ny), inx = static_cast<int>(nx);
  if (!fused)
    return launch_any<false, float>(p0, p1, p2, p3, iny, inx, k, iso, kc, lcp_k0, pitch, plane, shape, s);
  switch (dt) {
    case PDIV_F32:
      return launch_any<true, float>(p0, p1, p2, p3, iny, inx, k, iso, kc, lcp_k0, pitch, plane, shape, s);
    case PDIV_F16:
      return launch_any<true, __half>(p0, p1, p2, p3, iny, inx, k, iso, kc, lcp_k0, pitch, plane, shape, s);
    case PDIV_BF16:
      return launch_any<true, bf16_t>(p0, p1, p2, p3, iny, inx, k, iso, kc, lcp_k0, pitch, plane, shape, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace pdiv
