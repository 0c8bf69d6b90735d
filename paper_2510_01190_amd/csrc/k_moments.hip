// Per-point Gaussian fit over ensemble members (the fit that precedes Eq. 2-3;
// Sections 3 and 4).  Pure HBM streaming: every member value is read once.
//
// Layout: member m of a component is a plane of n_points values starting at
// element m*stride.  The fit is pointwise, so the grid is treated as a flat
// array: thread t owns VEC consecutive points and walks the members with a
// float32 Welford update (mean += d/n, M2 += d (x - mean)), which needs no
// second pass and keeps its accuracy when |mean| >> sigma.
#include "pdiv_device.hpp"
#include "pdiv_internal.hpp"

namespace pdiv {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float half_bits_to_f32(uint32_t b) {
  return __half2float(__ushort_as_half(static_cast<unsigned short>(b)));
}
__device__ __forceinline__ float bf16_bits_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

// Four consecutive values starting at element i (i a multiple of 4, base
// 4-element aligned), streamed past the caches.
__device__ __forceinline__ void load4(const float* __restrict__ p, int64_t i, float (&x)[4]) {
  const f32x4 w = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p + i));
  x[0] = w.x; x[1] = w.y; x[2] = w.z; x[3] = w.w;
}
__device__ __forceinline__ void load4(const __half* __restrict__ p, int64_t i, float (&x)[4]) {
  const u32x2 w = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p + i));
  x[0] = half_bits_to_f32(w.x & 0xffffu); x[1] = half_bits_to_f32(w.x >> 16);
  x[2] = half_bits_to_f32(w.y & 0xffffu); x[3] = half_bits_to_f32(w.y >> 16);
}
__device__ __forceinline__ void load4(const bf16_t* __restrict__ p, int64_t i, float (&x)[4]) {
  const u32x2 w = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p + i));
  x[0] = bf16_bits_to_f32(w.x & 0xffffu); x[1] = bf16_bits_to_f32(w.x >> 16);
  x[2] = bf16_bits_to_f32(w.y & 0xffffu); x[3] = bf16_bits_to_f32(w.y >> 16);
}
template <typename T>
__device__ __forceinline__ void load_vec(const T* __restrict__ p, int64_t i, float (&x)[4]) {
  load4(p, i, x);
}
template <typename T>
__device__ __forceinline__ void load_vec(const T* __restrict__ p, int64_t i, float (&x)[1]) {
  x[0] = to_f32(p[i]);
}

template <typename Tin, typename Tout, int VEC, int UNROLL>
__global__ __launch_bounds__(256) void moments_kernel(const Tin* __restrict__ u,
                                                      const Tin* __restrict__ v, int m_members,
                                                      int64_t n_points, int64_t stride,
                                                      float inv_dof, Tout* __restrict__ mu,
                                                      Tout* __restrict__ vu,
                                                      Tout* __restrict__ mv,
                                                      Tout* __restrict__ vv) {
  const int64_t p0 = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) * VEC;
  if (p0 >= n_points) return;
  const bool full = (p0 + VEC <= n_points);

  float mean_u[VEC], m2_u[VEC], mean_v[VEC], m2_v[VEC];
#pragma unroll
  for (int q = 0; q < VEC; ++q) mean_u[q] = m2_u[q] = mean_v[q] = m2_v[q] = 0.0f;

  int m = 0;
  if (full) {
    for (; m + UNROLL <= m_members; m += UNROLL) {
      float xu[UNROLL][VEC], xv[UNROLL][VEC];
#pragma unroll
      for (int r = 0; r < UNROLL; ++r) {
        load_vec<Tin>(u, (m + r) * stride + p0, xu[r]);
        load_vec<Tin>(v, (m + r) * stride + p0, xv[r]);
      }
#pragma unroll
      for (int r = 0; r < UNROLL; ++r) {
        const float inv = 1.0f / static_cast<float>(m + r + 1);
#pragma unroll
        for (int q = 0; q < VEC; ++q) {
          float d = xu[r][q] - mean_u[q];
          mean_u[q] = fmaf(d, inv, mean_u[q]);
          m2_u[q] = fmaf(d, xu[r][q] - mean_u[q], m2_u[q]);
          float e = xv[r][q] - mean_v[q];
          mean_v[q] = fmaf(e, inv, mean_v[q]);
          m2_v[q] = fmaf(e, xv[r][q] - mean_v[q], m2_v[q]);
        }
      }
    }
  }
  for (; m < m_members; ++m) {
    const float inv = 1.0f / static_cast<float>(m + 1);
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      if (p0 + q < n_points) {
        float x = ld(u, m * stride + p0 + q);
        float d = x - mean_u[q];
        mean_u[q] = fmaf(d, inv, mean_u[q]);
        m2_u[q] = fmaf(d, x - mean_u[q], m2_u[q]);
        float y = ld(v, m * stride + p0 + q);
        float e = y - mean_v[q];
        mean_v[q] = fmaf(e, inv, mean_v[q]);
        m2_v[q] = fmaf(e, y - mean_v[q], m2_v[q]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < VEC; ++q) {
    if (p0 + q < n_points) {
      mu[p0 + q] = from_f32<Tout>(mean_u[q]);
      vu[p0 + q] = from_f32<Tout>(m2_u[q] * inv_dof);
      mv[p0 + q] = from_f32<Tout>(mean_v[q]);
      vv[p0 + q] = from_f32<Tout>(m2_v[q] * inv_dof);
    }
  }
}

template <typename Tin, typename Tout>
hipError_t launch_typed(const void* u, const void* v, int64_t m, int64_t n, int64_t stride,
                        int ddof, void* mu, void* vu, void* mv, void* vv, hipStream_t s) {
  const float inv_dof = static_cast<float>(1.0 / static_cast<double>(m - ddof));
  const size_t align = sizeof(Tin) * 4;
  const bool vec4 = (stride % 4 == 0) && (reinterpret_cast<uintptr_t>(u) % align == 0) &&
                    (reinterpret_cast<uintptr_t>(v) % align == 0);
  constexpr int kBlock = 256;
  if (vec4) {
    const int64_t threads = (n + 3) / 4;
    if (!launch_fits((threads + kBlock - 1) / kBlock, kBlock)) return hipErrorInvalidConfiguration;
    dim3 grid(static_cast<unsigned>((threads + kBlock - 1) / kBlock));
    hipLaunchKernelGGL((moments_kernel<Tin, Tout, 4, 4>), grid, dim3(kBlock), 0, s,
                       static_cast<const Tin*>(u), static_cast<const Tin*>(v),
                       static_cast<int>(m), n, stride, inv_dof, static_cast<Tout*>(mu),
                       static_cast<Tout*>(vu), static_cast<Tout*>(mv), static_cast<Tout*>(vv));
  } else {
    if (!launch_fits((n + kBlock - 1) / kBlock, kBlock)) return hipErrorInvalidConfiguration;
    dim3 grid(static_cast<unsigned>((n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL((moments_kernel<Tin, Tout, 1, 8>), grid, dim3(kBlock), 0, s,
                       static_cast<const Tin*>(u), static_cast<const Tin*>(v),
                       static_cast<int>(m), n, stride, inv_dof, static_cast<Tout*>(mu),
                       static_cast<Tout*>(vu), static_cast<Tout*>(mv), static_cast<Tout*>(vv));
  }
  return hipGetLastError();
}

template <typename Tin>
hipError_t launch_in(const void* u, const void* v, int64_t m, int64_t n, int64_t stride,
                     int ddof, void* mu, void* vu, void* mv, void* vv, pdiv_dtype out,
                     hipStream_t s) {
  switch (out) {
    case PDIV_F32: return launch_typed<Tin, float>(u, v, m, n, stride, ddof, mu, vu, mv, vv, s);
    case PDIV_F16: return launch_typed<Tin, __half>(u, v, m, n, stride, ddof, mu, vu, mv, vv, s);
    case PDIV_BF16: return launch_typed<Tin, bf16_t>(u, v, m, n, stride, ddof, mu, vu, mv, vv, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_moments(const void* u, const void* v, pdiv_dtype in_dtype, int64_t m,
                          int64_t n_points, int64_t stride, int ddof, void* mu, void* vu,
                          void* mv, void* vv, pdiv_dtype out_dtype, hipStream_t s) {
  switch (in_dtype) {
    case PDIV_F32:
      return launch_in<float>(u, v, m, n_points, stride, ddof, mu, vu, mv, vv, out_dtype, s);
    case PDIV_F16:
      return launch_in<__half>(u, v, m, n_points, stride, ddof, mu, vu, mv, vv, out_dtype, s);
    case PDIV_BF16:
      return launch_in<bf16_t>(u, v, m, n_points, stride, ddof, mu, vu, mv, vv, out_dtype, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace pdiv
