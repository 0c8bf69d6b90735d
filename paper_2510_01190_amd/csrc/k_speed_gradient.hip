// The Red Sea pre-stage (Section 4): for every ensemble member the pixelwise
// gradient of the velocity magnitude, fitted per point with a Gaussian over
// the members -- the field whose divergence uncertainty the path then
// analyses.  Fused: the members' speed and gradient never reach HBM; each
// member value is read once (plus halos), the fit accumulates in registers.
//
// Tile: a wave holds 64 columns x0-1 .. x0+62 (lanes 1..62 produce outputs,
// lanes 0 and 63 are the x halo) and a band of kBand output rows.  Per
// member it loads the band's rows and the two halo rows (one load per lane
// and component), takes the speed once per point, forms the x difference
// from the neighbouring lanes through DPP and the y difference from the
// rows in registers (Eq. 1's scheme: central inside, one-sided on the
// boundary), and updates a float32 Welford fit of gx and gy per point.
#include <hip/hip_runtime.h>

#include "pdiv_device.hpp"
#include "pdiv_internal.hpp"

namespace pdiv {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kBand = 4;
constexpr int kStrip = 62;
// Members walked one at a time: at 721 x 1440 x 50 this runs 7 waves per
// SIMD and takes 0.121 ms; issuing the loads of 2 or 4 members together
// needs more registers (5 or 3 waves per SIMD) and takes 0.144 or 0.222 ms.
constexpr int kUnroll = 1;

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kBlock) void speed_gradient_moments_kernel(
    const Tin* __restrict__ u, const Tin* __restrict__ v, int m_members, int ny, int nx,
    int64_t stride, StencilCoef k, float inv_dof, Tout* __restrict__ mgx,
    Tout* __restrict__ vgx, Tout* __restrict__ mgy, Tout* __restrict__ vgy, int n_strips,
    int n_bands) {
  const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
  const int strip = wave % n_strips;
  const int band = wave / n_strips;
  if (band >= n_bands) return;  // wave-uniform: whole waves leave, DPP partners stay together
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
  // one member's gradients folded into the running fit (Welford)
  auto update = [&](int m, const float (&s)[kBand + 2]) {
    const float inv = 1.0f / static_cast<float>(m + 1);
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
  // kUnroll members' loads are issued together, so their latencies overlap
  int m = 0;
  for (; m + kUnroll <= m_members; m += kUnroll) {
    float s[kUnroll][kBand + 2];
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) speeds(m + q, s[q]);
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) update(m + q, s[q]);
  }
  for (; m < m_members; ++m) {
    float s[kBand + 2];
    speeds(m, s);
    update(m, s);
  }
  if (lane == 0 || lane == 63 || x >= nx) return;
#pragma unroll
  for (int r = 0; r < kBand; ++r) {
    const int y = y0 + r;
    if (y < ny) {
      const int64_t o = int64_t(y) * nx + x;
      mgx[o] = from_f32<Tout>(mean_x[r]);
      vgx[o] = from_f32<Tout>(m2_x[r] * inv_dof);
      mgy[o] = from_f32<Tout>(mean_y[r]);
      vgy[o] = from_f32<Tout>(m2_y[r] * inv_dof);
    }
  }
}

template <typename Tin, typename Tout>
hipError_t launch_sg(const void* u, const void* v, int64_t m, int64_t ny, int64_t nx,
                     int64_t stride, const StencilCoef& k, int ddof, void* mgx, void* vgx,
                     void* mgy, void* vgy, hipStream_t s) {
  const float inv_dof = static_cast<float>(1.0 / static_cast<double>(m - ddof));
  const int n_strips = int((nx + kStrip - 1) / kStrip);
  const int n_bands = int((ny + kBand - 1) / kBand);
  const int64_t blocks = (int64_t(n_strips) * n_bands + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > 0x7fffffff / kWavesPerBlock) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((speed_gradient_moments_kernel<Tin, Tout>), dim3(unsigned(blocks)),
                     dim3(kBlock), 0, s, static_cast<const Tin*>(u), static_cast<const Tin*>(v),
                     int(m), int(ny), int(nx), stride, k, inv_dof, static_cast<Tout*>(mgx),
                     static_cast<Tout*>(vgx), static_cast<Tout*>(mgy), static_cast<Tout*>(vgy),
                     n_strips, n_bands);
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
  return (((nx + kStrip - 1) / kStrip) * ((ny + kBand - 1) / kBand) + kWavesPerBlock - 1) /
         kWavesPerBlock;
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
