// The Red Sea pre-stage (Section 4): for every ensemble member the pixelwise
// gradient of the velocity magnitude, fitted per point with a Gaussian over
// the members -- the field whose divergence uncertainty the path then
// analyses.  Fused: the members' speed and gradient never reach HBM; each
// member value is read once (plus halos), the fit accumulates in registers.
//
// Tile: 64 columns x0-1 .. x0+62 (lanes 1..62 produce outputs, lanes 0 and
// 63 are the x halo) by a band of kBand output rows, one tile per block.
// The block's four waves split the members into four contiguous runs; per
// member a wave loads the band's rows and the two halo rows (one load per
// lane and component), takes the speed once per point, forms the x
// difference from the neighbouring lanes through DPP and the y difference
// from the rows in registers (Eq. 1's scheme: central inside, one-sided on
// the boundary), and updates a float32 Welford fit of gx and gy per point.
// The four partial fits then meet in LDS and wave w merges those of output
// rows w and w + 4 in run order (the pairwise update of Chan, Golub and
// LeVeque), so each member value is still read once and a tile has four
// waves in flight.  Measured at 721 x 1440 x 50, float32: one wave per
// 4-row tile walking all members 0.120 ms; four waves per 4-row tile
// 0.105 ms; per 8-row tile (two halo rows per eight output rows, not per
// four) 0.099 ms; per 16-row tile 0.107 ms (254 registers); eight waves per
// 8-row tile 0.101 ms.
#include <hip/hip_runtime.h>

#include "pdiv_device.hpp"
#include "pdiv_internal.hpp"

namespace pdiv {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kBand = 8;
constexpr int kStrip = 62;
static_assert(kBand % kWavesPerBlock == 0, "the merge gives each wave whole output rows");

// first member of wave w's run
__device__ __forceinline__ int member_run_start(int w, int m_members) {
  return int(int64_t(w) * m_members / kWavesPerBlock);
}

// (mean, m2) over n_a values merged with (mean_b, m2_b) over n_b values;
// n_a may be 0 (then mean and m2 are 0 and the result is exactly b's)
__device__ __forceinline__ void merge_fit(float& mean, float& m2, int n_a, float mean_b,
                                          float m2_b, int n_b) {
  if (n_b == 0) return;
  const float d = mean_b - mean;
  const float f_b = static_cast<float>(n_b) / static_cast<float>(n_a + n_b);
  mean = fmaf(d, f_b, mean);
  m2 = (m2 + m2_b) + d * d * (static_cast<float>(n_a) * f_b);
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kBlock) void speed_gradient_moments_kernel(
    const Tin* __restrict__ u, const Tin* __restrict__ v, int m_members, int ny, int nx,
    int64_t stride, StencilCoef k, float inv_dof, Tout* __restrict__ mgx,
    Tout* __restrict__ vgx, Tout* __restrict__ mgy, Tout* __restrict__ vgy, int n_strips) {
  // partial fits: [wave][row of the band][mean_x, m2_x, mean_y, m2_y][lane]
  __shared__ float part[kWavesPerBlock][kBand][4][64];
  // Blocks are dealt round-robin to the 8 XCDs, each with its own L2; give
  // each XCD a contiguous run of tiles, so that the halo rows two bands
  // share are fetched into one L2.  The map is a bijection on [0, gridDim.x).
  const int nb = gridDim.x, xcd = blockIdx.x % 8, q8 = nb / 8, r8 = nb % 8;
  const int blk = xcd * q8 + min(xcd, r8) + blockIdx.x / 8;
  const int strip = blk % n_strips;
  const int band = blk / n_strips;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int x = strip * kStrip - 1 + lane;
  const int xc = x < 0 ? 0 : (x > nx - 1 ? nx - 1 : x);
  const bool bx = (x == 0) | (x == nx - 1);
  const float cxm = bx ? k.cxm_bd : k.cxm_in;
  const int y0 = band * kBand;
  float mean_x[kBand], m2_x[kBand], mean_y[kBand], m2_y[kBand];
#pragma unroll
  for (int r = 0; r < kBand; ++r) mean_x[r] = m2_x[r] = mean_y[r] = m2_y[r] = 0.0f;
  // speeds of the band's rows (and the two halo rows) for one member
  auto speeds = [&](int m, float (&s)[kBand + 2]) {
    const Tin* const um = u + int64_t(m) * stride;
    const Tin* const vm = v + int64_t(m) * stride;
    float a[kBand + 2], b[kBand + 2];
#pragma unroll
    for (int r = 0; r < kBand + 2; ++r) {
      int yy = y0 - 1 + r;
      yy = yy < 0 ? 0 : (yy > ny - 1 ? ny - 1 : yy);
      const int64_t o = int64_t(yy) * nx + xc;
      a[r] = to_f32(um[o]);
      b[r] = to_f32(vm[o]);
    }
#pragma unroll
    for (int r = 0; r < kBand + 2; ++r) s[r] = sqrtf(fmaf(a[r], a[r], b[r] * b[r]));
  };
  // the i-th member of the run folded into the running fit (Welford)
  auto update = [&](int i, const float (&s)[kBand + 2]) {
    const float inv = 1.0f / static_cast<float>(i + 1);
#pragma unroll
    for (int r = 0; r < kBand; ++r) {
      const int y = y0 + r;
      const float own = s[r + 1];
      // both neighbours read with every lane active: a DPP read inside a
      // lane-dependent branch would find its partner lane switched off
      const float left = dpp_from_left(own);
      const float right = dpp_from_right(own);
      const float sl = x == 0 ? own : left;
      const float sr = x == nx - 1 ? own : right;
      const float gx = (sr - sl) * cxm;
      const bool by = (y == 0) | (y == ny - 1);
      const float lo = y == 0 ? own : s[r];
      const float hi = y >= ny - 1 ? own : s[r + 2];
      const float gy = (hi - lo) * (by ? k.cym_bd : k.cym_in);
      float d = gx - mean_x[r];
      mean_x[r] = fmaf(d, inv, mean_x[r]);
      m2_x[r] = fmaf(d, gx - mean_x[r], m2_x[r]);
      float e = gy - mean_y[r];
      mean_y[r] = fmaf(e, inv, mean_y[r]);
      m2_y[r] = fmaf(e, gy - mean_y[r], m2_y[r]);
    }
  };
  const int m_lo = member_run_start(w, m_members);
  const int m_hi = member_run_start(w + 1, m_members);
  for (int m = m_lo; m < m_hi; ++m) {
    float s[kBand + 2];
    speeds(m, s);
    update(m - m_lo, s);
  }
#pragma unroll
  for (int r = 0; r < kBand; ++r) {
    part[w][r][0][lane] = mean_x[r];
    part[w][r][1][lane] = m2_x[r];
    part[w][r][2][lane] = mean_y[r];
    part[w][r][3][lane] = m2_y[r];
  }
  __syncthreads();
  if (lane == 0 || lane == 63 || x >= nx) return;
  // wave w now owns output rows y0 + w, y0 + w + 4, ...: the runs' fits
  // merged in run order
#pragma unroll
  for (int r = w; r < kBand; r += kWavesPerBlock) {
    const int y = y0 + r;
    if (y >= ny) break;
    float mx = 0.0f, qx = 0.0f, my = 0.0f, qy = 0.0f;
    int n = 0;
#pragma unroll
    for (int p = 0; p < kWavesPerBlock; ++p) {
      const int np = member_run_start(p + 1, m_members) - member_run_start(p, m_members);
      merge_fit(mx, qx, n, part[p][r][0][lane], part[p][r][1][lane], np);
      merge_fit(my, qy, n, part[p][r][2][lane], part[p][r][3][lane], np);
      n += np;
    }
    const int64_t o = int64_t(y) * nx + x;
    mgx[o] = from_f32<Tout>(mx);
    vgx[o] = from_f32<Tout>(qx * inv_dof);
    mgy[o] = from_f32<Tout>(my);
    vgy[o] = from_f32<Tout>(qy * inv_dof);
  }
}

template <typename Tin, typename Tout>
hipError_t launch_sg(const void* u, const void* v, int64_t m, int64_t ny, int64_t nx,
                     int64_t stride, const StencilCoef& k, int ddof, void* mgx, void* vgx,
                     void* mgy, void* vgy, hipStream_t s) {
  const float inv_dof = static_cast<float>(1.0 / static_cast<double>(m - ddof));
  const int n_strips = int((nx + kStrip - 1) / kStrip);
  const int64_t blocks = speed_gradient_blocks(ny, nx);  // one per tile
  if (!launch_fits(blocks, kBlock)) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((speed_gradient_moments_kernel<Tin, Tout>), dim3(unsigned(blocks)),
                     dim3(kBlock), 0, s, static_cast<const Tin*>(u), static_cast<const Tin*>(v),
                     int(m), int(ny), int(nx), stride, k, inv_dof, static_cast<Tout*>(mgx),
                     static_cast<Tout*>(vgx), static_cast<Tout*>(mgy), static_cast<Tout*>(vgy),
                     n_strips);
  return hipGetLastError();
}

template <typename Tin>
hipError_t launch_sg_out(const void* u, const void* v, int64_t m, int64_t ny, int64_t nx,
                         int64_t stride, const StencilCoef& k, int ddof, void* mgx, void* vgx,
                         void* mgy, void* vgy, pdiv_dtype out_dt, hipStream_t s) {
  switch (out_dt) {
    case PDIV_F32: return launch_sg<Tin, float>(u, v, m, ny, nx, stride, k, ddof, mgx, vgx, mgy, vgy, s);
    case PDIV_F16: return launch_sg<Tin, __half>(u, v, m, ny, nx, stride, k, ddof, mgx, vgx, mgy, vgy, s);
    case PDIV_BF16: return launch_sg<Tin, bf16_t>(u, v, m, ny, nx, stride, k, ddof, mgx, vgx, mgy, vgy, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int64_t speed_gradient_blocks(int64_t ny, int64_t nx) {
  return ((nx + kStrip - 1) / kStrip) * ((ny + kBand - 1) / kBand);
}

hipError_t launch_speed_gradient_moments(const void* u, const void* v, pdiv_dtype in_dt,
                                         int64_t m, int64_t ny, int64_t nx, int64_t stride,
                                         const StencilCoef& k, int ddof, void* mgx, void* vgx,
                                         void* mgy, void* vgy, pdiv_dtype out_dt,
                                         hipStream_t s) {
  switch (in_dt) {
    case PDIV_F32: return launch_sg_out<float>(u, v, m, ny, nx, stride, k, ddof, mgx, vgx, mgy, vgy, out_dt, s);
    case PDIV_F16: return launch_sg_out<__half>(u, v, m, ny, nx, stride, k, ddof, mgx, vgx, mgy, vgy, out_dt, s);
    case PDIV_BF16: return launch_sg_out<bf16_t>(u, v, m, ny, nx, stride, k, ddof, mgx, vgx, mgy, vgy, out_dt, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pdiv
