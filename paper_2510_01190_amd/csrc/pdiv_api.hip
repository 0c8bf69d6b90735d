// C ABI of libpdiv: argument validation, dtype dispatch and launch of the
// core calls.  Every check runs before any HIP call, so a rejected call
// touches neither the device nor the outputs.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "pdiv_device.hpp"
#include "pdiv_internal.hpp"

namespace pdiv {

thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

pdiv_status invalid(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return PDIV_ERR_INVALID;
}

// --- checking modes --------------------------------------------------------
uint32_t initial_debug_flags() {
  uint32_t f = 0;
  const char* c = std::getenv("PDIV_DEBUG_CHECKS");
  if (c && *c && std::strcmp(c, "0") != 0) f |= PDIV_DEBUG_CHECK_INPUTS;
  const char* l = std::getenv("PDIV_LOG");
  if (l && *l && std::strcmp(l, "0") != 0) f |= PDIV_DEBUG_LOG;
  return f;
}
std::atomic<uint32_t> g_debug{initial_debug_flags()};
uint32_t debug_flags() { return g_debug.load(std::memory_order_relaxed); }
void set_debug_flags(uint32_t flags) { g_debug.store(flags, std::memory_order_relaxed); }

// One line per core call on stderr under PDIV_DEBUG_LOG.
void log_call(const char* fmt, ...) {
  if (!(debug_flags() & PDIV_DEBUG_LOG)) return;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "[pdiv] %s\n", buf);
}

pdiv_status device_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return PDIV_OK;
  set_error("%s: %s", what, hipGetErrorString(e));
  return PDIV_ERR_DEVICE;
}

// Grid limits of the kernels' launch geometry: nx <= 2^29 (a row's byte
// offset fits in 32 bits), ny <= 2^21.
constexpr int64_t kMaxNx = int64_t(1) << 29;
constexpr int64_t kMaxNy = int64_t(1) << 21;

pdiv_status check_grid(int64_t ny, int64_t nx) {
  if (ny < 2 || nx < 2) return invalid("grid must be at least 2x2 (got ny=%lld nx=%lld)",
                                       (long long)ny, (long long)nx);
  if (nx > kMaxNx || ny > kMaxNy)
    return invalid("grid too large (ny=%lld > 2^21 or nx=%lld > 2^29)", (long long)ny,
                   (long long)nx);
  return PDIV_OK;
}

pdiv_status check_spacing(double dx, double dy) {
  if (!(std::isfinite(dx) && dx > 0.0) || !(std::isfinite(dy) && dy > 0.0))
    return invalid("dx and dy must be finite and > 0 (got %g, %g)", dx, dy);
  return PDIV_OK;
}

pdiv_status check_dtype(pdiv_dtype d, const char* name) {
  if (d != PDIV_F32 && d != PDIV_F16 && d != PDIV_BF16)
    return invalid("%s: unknown dtype %d", name, (int)d);
  return PDIV_OK;
}

pdiv_status check_iso(const float* iso, int32_t n) {
  if (iso == nullptr) return invalid("isovalues_host is NULL");
  if (n < 1 || n > PDIV_MAX_ISO) return invalid("n_iso must be in [1, %d] (got %d)", PDIV_MAX_ISO, n);
  return PDIV_OK;
}

pdiv_status check_layout(int64_t row_pitch, int64_t plane_stride, int64_t ny, int64_t nx,
                         int32_t n_iso, OutLayout* out) {
  const int64_t cells = nx - 1, rows = ny - 1;
  const int64_t pitch = row_pitch == 0 ? cells : row_pitch;
  if (pitch < cells || pitch > (int64_t(1) << 52))
    return invalid("lcp_row_pitch must be 0 or in [nx - 1, 2^52] (got %lld, nx=%lld)",
                   (long long)row_pitch, (long long)nx);
  // rows x pitch is bounded in double (exact up to 2^53, so the comparison is
  // exact) before the int64 product is formed
  if (double(rows) * double(pitch) > double(int64_t(1) << 52))
    return invalid("LCP output layout is too large (rows x pitch > 2^52 floats)");
  const int64_t map = rows * pitch;
  const int64_t plane = plane_stride == 0 ? map : plane_stride;
  if (plane < 0 || plane > (int64_t(1) << 52))
    return invalid("lcp_plane_stride must be 0 or in [1, 2^52] (got %lld)",
                   (long long)plane_stride);
  const bool apart = plane >= map;
  const bool interleaved = plane >= cells && pitch >= int64_t(n_iso) * plane;
  if (!apart && !interleaved)
    return invalid("lcp_plane_stride %lld with lcp_row_pitch %lld makes the %d maps of "
                   "%lld x %lld cells overlap", (long long)plane, (long long)pitch, n_iso,
                   (long long)rows, (long long)cells);
  // last element: (n_iso - 1) plane + (rows - 1) pitch + cells - 1
  const double last = double(n_iso - 1) * double(plane) + double(rows - 1) * double(pitch) +
                      double(cells);
  if (last * 4.0 >= double(int64_t(1) << 56)) return invalid("LCP output layout is too large");
  out->pitch = pitch;
  out->plane = plane;
  return PDIV_OK;
}

pdiv_status check_grid3(int64_t nz, int64_t ny, int64_t nx) {
  if (nz < 2 || ny < 2 || nx < 2)
    return invalid("grid must be at least 2x2x2 (got nz=%lld ny=%lld nx=%lld)", (long long)nz,
                   (long long)ny, (long long)nx);
  if (nx > kMaxNx || ny > kMaxNy || nz > kMaxNy)
    return invalid("grid too large (nz, ny > 2^21 or nx > 2^29)");
  if (double(nz) * double(ny) * double(nx) > double(int64_t(1) << 40) ||
      !launch_fits(divergence3d_blocks(nz, ny, nx), 256) ||
      !launch_fits(lcp3d_blocks(nz, ny, nx, 16), 256))
    return invalid("grid of %lld x %lld x %lld points is too large for one launch",
                   (long long)nz, (long long)ny, (long long)nx);
  return PDIV_OK;
}

#define PDIV_TRY(expr)                \
  do {                                \
    pdiv_status st_ = (expr);         \
    if (st_ != PDIV_OK) return st_;   \
  } while (0)

#define PDIV_NONNULL(p) \
  do {                  \
    if ((p) == nullptr) return invalid("%s is NULL", #p); \
  } while (0)

// A float output: non-null and 4-byte aligned (the kernels store whole
// floats, two at a time on the paired tiles).
#define PDIV_FLOATS(p)                                                          \
  do {                                                                          \
    PDIV_NONNULL(p);                                                            \
    if (reinterpret_cast<uintptr_t>(p) % 4 != 0)                                \
      return invalid("%s must be 4-byte aligned (a float array)", #p);          \
  } while (0)

pdiv_status lcp_chunks(bool fused, const void* p0, const void* p1, const void* p2,
                       const void* p3, pdiv_dtype dt, int64_t ny, int64_t nx, double dx,
                       double dy, const float* iso_host, int32_t n_iso, float* lcp,
                       OutLayout lo, hipStream_t s) {
  const StencilCoef k = make_coef(dx, dy);
  const int64_t plane = lo.plane;
  const LcpShape shape = default_lcp_shape(ny, nx, n_iso);
  // chunks of 16, 8, 4, 2, 1 isovalues (the kernel is instantiated for these)
  for (int32_t k0 = 0; k0 < n_iso;) {
    const int left = n_iso - k0;
    const int kc = left >= 16 ? 16 : left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
    IsoChunk c;
    for (int q = 0; q < kIsoChunk; ++q) c.c[q] = iso_host[k0 + (q < kc ? q : kc - 1)];
    hipError_t e = launch_lcp(fused, p0, p1, p2, p3, dt, ny, nx, k, c, kc, lcp + k0 * plane,
                              lo.pitch, plane, shape, s);
    if (e != hipSuccess) return device_status(e, "LCP launch");
    k0 += kc;
  }
  return PDIV_OK;
}

pdiv_status check_spaghetti(const void* u_members, const void* v_members, pdiv_dtype in_dtype,
                            int64_t n_members, int64_t ny, int64_t nx, int64_t* member_stride,
                            double dx, double dy, const int64_t* row_offsets,
                            const float* segments, int64_t max_segments) {
  PDIV_NONNULL(u_members);
  PDIV_NONNULL(v_members);
  PDIV_NONNULL(row_offsets);
  PDIV_TRY(check_dtype(in_dtype, "in_dtype"));
  PDIV_TRY(check_grid(ny, nx));
  PDIV_TRY(check_spacing(dx, dy));
  // the per-member divergence runs a thread per point of 64-column strips,
  // the contour passes 64 threads per cell row, both over all members' rows
  // rounded up to a block's 4: (n_members*ny + 3) * nx_r < 2^32 per launch
  const int64_t nx_r = (nx + 63) / 64 * 64;
  if (n_members < 1 || n_members > (int64_t(0xffffffff) / nx_r - 3) / ny)
    return invalid("n_members must be >= 1 with n_members*ny*nx (nx rounded up to 64) < 2^32 "
                   "(got %lld)", (long long)n_members);
  const int64_t n = ny * nx;
  if (*member_stride == 0) *member_stride = n;
  if (*member_stride < n)
    return invalid("member_stride %lld < ny*nx %lld", (long long)*member_stride, (long long)n);
  if (max_segments < 0) return invalid("max_segments must be >= 0 (got %lld)",
                                       (long long)max_segments);
  if (max_segments > 0 && segments == nullptr) return invalid("segments is NULL");
  if (max_segments > 0 && reinterpret_cast<uintptr_t>(segments) % 16 != 0)
    return invalid("segments must be 16-byte aligned");
  return PDIV_OK;
}

// Every member's Eq. 1 divergence into div (n_members planes of ny*nx
// floats), then all members' contours from it.
hipError_t run_spaghetti(const void* u_members, const void* v_members, pdiv_dtype in_dtype,
                         int64_t n_members, int64_t ny, int64_t nx, int64_t member_stride,
                         double dx, double dy, float isovalue, float* div,
                         int64_t* row_offsets, float* segments, int64_t max_segments,
                         hipStream_t s) {
  hipError_t e = launch_members_divergence(u_members, v_members, in_dtype, n_members, ny, nx,
                                           member_stride, make_coef(dx, dy), div, s);
  return e != hipSuccess ? e
                         : launch_isocontours(div, n_members, ny * nx, ny, nx, isovalue,
                                              row_offsets, segments, max_segments, s);
}

// ---------------------------------------------------------------------------
// PDIV_DEBUG_CHECK_INPUTS: a scan of the moment (or divergence) planes for
// non-finite values and negative variances, counted in a device word.
// ---------------------------------------------------------------------------
static __device__ unsigned int check_count;

__global__ void check_zero_kernel(unsigned int* c) { *c = 0u; }

template <typename T>
__global__ __launch_bounds__(256) void check_planes_kernel(const T* __restrict__ m0,
                                                           const T* __restrict__ v0,
                                                           const T* __restrict__ m1,
                                                           const T* __restrict__ v1, int64_t n,
                                                           unsigned int* __restrict__ bad) {
  unsigned int b = 0;
  for (int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x; p < n;
       p += int64_t(gridDim.x) * 256) {
    const float a = to_f32(m0[p]), c = to_f32(m1[p]), va = to_f32(v0[p]), vc = to_f32(v1[p]);
    b |= unsigned(!__builtin_isfinite(a)) | unsigned(!__builtin_isfinite(c)) |
         unsigned(!(__builtin_isfinite(va) && va >= 0.0f)) |
         unsigned(!(__builtin_isfinite(vc) && vc >= 0.0f));
  }
  if (b) atomicAdd(bad, 1u);
}

std::mutex g_check_mu;
unsigned int* g_check_ptr[64] = {};

// Scans the planes of a call under PDIV_DEBUG_CHECK_INPUTS (waits for the
// stream); PDIV_OK when every value is admissible.
pdiv_status check_inputs(const void* m0, const void* v0, const void* m1, const void* v1,
                         pdiv_dtype dt, int64_t n, hipStream_t s, const char* call) {
  if (!(debug_flags() & PDIV_DEBUG_CHECK_INPUTS)) return PDIV_OK;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_status(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) {
    set_error("device index %d beyond the checking table", dev);
    return PDIV_ERR_UNSUPPORTED;
  }
  unsigned int* cnt = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_check_mu);
    if (!g_check_ptr[dev]) {
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(check_count));
      if (e != hipSuccess) return device_status(e, "hipGetSymbolAddress(check_count)");
      g_check_ptr[dev] = static_cast<unsigned int*>(p);
    }
    cnt = g_check_ptr[dev];
  }
  const unsigned grid = unsigned(std::min<int64_t>((n + 255) / 256, 4096));
  hipLaunchKernelGGL(check_zero_kernel, dim3(1), dim3(1), 0, s, cnt);
  switch (dt) {
    case PDIV_F32:
      hipLaunchKernelGGL(check_planes_kernel<float>, dim3(grid), dim3(256), 0, s,
                         static_cast<const float*>(m0), static_cast<const float*>(v0),
                         static_cast<const float*>(m1), static_cast<const float*>(v1), n, cnt);
      break;
    case PDIV_F16:
      hipLaunchKernelGGL(check_planes_kernel<__half>, dim3(grid), dim3(256), 0, s,
                         static_cast<const __half*>(m0), static_cast<const __half*>(v0),
                         static_cast<const __half*>(m1), static_cast<const __half*>(v1), n, cnt);
      break;
    default:
      hipLaunchKernelGGL(check_planes_kernel<bf16_t>, dim3(grid), dim3(256), 0, s,
                         static_cast<const bf16_t*>(m0), static_cast<const bf16_t*>(v0),
                         static_cast<const bf16_t*>(m1), static_cast<const bf16_t*>(v1), n, cnt);
      break;
  }
  unsigned int host = 0;
  e = hipGetLastError();
  e = e != hipSuccess ? e : hipMemcpyAsync(&host, cnt, sizeof host, hipMemcpyDeviceToHost, s);
  e = e != hipSuccess ? e : hipStreamSynchronize(s);
  if (e != hipSuccess) return device_status(e, "input check");
  if (host) return invalid("%s: input planes hold non-finite values or negative variances", call);
  return PDIV_OK;
}

// ---------------------------------------------------------------------------
// Workspace of pdiv_spaghetti_noalloc: the members' divergence planes live in
// this file-scope device array instead of a caller's buffer.  Its name is a
// host-side stand-in in host code; the device address of each GPU's copy is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and only that address is handed to kernels.
// ---------------------------------------------------------------------------
constexpr int64_t kScratchFloats = int64_t(1) << 24;  // 64 MiB per device
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

pdiv_status scratch_for_current_device(float** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_status(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index %d beyond the %d devices the workspace table holds", dev,
              kMaxDevices);
    return PDIV_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return device_status(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return PDIV_OK;
}

}  // namespace pdiv

using namespace pdiv;

extern "C" {

const char* pdiv_version(void) { return "0.1.0"; }

pdiv_status pdiv_set_lcp_band_rows(int32_t rows) {
  g_last_error.clear();
  if (rows < 0 || rows > 4096) return invalid("band rows must be in [0, 4096] (got %d)", rows);
  set_band_rows_override(rows);
  return PDIV_OK;
}

pdiv_status pdiv_set_debug(uint32_t flags) {
  g_last_error.clear();
  const uint32_t known = PDIV_DEBUG_POISON_LDS | PDIV_DEBUG_CHECK_INPUTS | PDIV_DEBUG_LOG;
  if (flags & ~known) return invalid("unknown debug flags 0x%x", flags & ~known);
  set_debug_flags(flags);
  return PDIV_OK;
}

const char* pdiv_last_error(void) { return g_last_error.c_str(); }

const char* pdiv_status_string(pdiv_status s) {
  switch (s) {
    case PDIV_OK: return "ok";
    case PDIV_ERR_INVALID: return "invalid argument";
    case PDIV_ERR_UNSUPPORTED: return "unsupported";
    case PDIV_ERR_NOMEM: return "out of memory";
    case PDIV_ERR_DEVICE: return "device error";
    case PDIV_ERR_BUSY: return "busy";
    case PDIV_ERR_TIMEOUT: return "timeout";
  }
  return "unknown status";
}

pdiv_status pdiv_moments(const void* u_members, const void* v_members, pdiv_dtype in_dtype,
                         int64_t n_members, int64_t ny, int64_t nx, int64_t member_stride,
                         int32_t ddof, void* mean_u, void* var_u, void* mean_v, void* var_v,
                         pdiv_dtype out_dtype, pdiv_stream stream) {
  g_last_error.clear();
  log_call("pdiv_moments members=%lld ny=%lld nx=%lld in=%d out=%d ddof=%d", (long long)n_members,
           (long long)ny, (long long)nx, int(in_dtype), int(out_dtype), ddof);
  PDIV_NONNULL(u_members);
  PDIV_NONNULL(v_members);
  PDIV_NONNULL(mean_u);
  PDIV_NONNULL(var_u);
  PDIV_NONNULL(mean_v);
  PDIV_NONNULL(var_v);
  PDIV_TRY(check_dtype(in_dtype, "in_dtype"));
  PDIV_TRY(check_dtype(out_dtype, "out_dtype"));
  if (ny < 1 || nx < 1 || ny > kMaxNy || nx > kMaxNx)
    return invalid("bad grid ny=%lld nx=%lld", (long long)ny, (long long)nx);
  if (ddof != 0 && ddof != 1) return invalid("ddof must be 0 or 1 (got %d)", ddof);
  if (n_members <= ddof || n_members > (int64_t(1) << 30))
    return invalid("n_members must be in (ddof, 2^30] (got %lld)", (long long)n_members);
  const int64_t n = ny * nx;
  if (member_stride == 0) member_stride = n;
  if (member_stride < n)
    return invalid("member_stride %lld < ny*nx %lld", (long long)member_stride, (long long)n);
  return device_status(launch_moments(u_members, v_members, in_dtype, n_members, n,
                                      member_stride, ddof, mean_u, var_u, mean_v, var_v,
                                      out_dtype, static_cast<hipStream_t>(stream)),
                       "moments launch");
}

pdiv_status pdiv_speed_gradient_moments(const void* u_members, const void* v_members,
                                        pdiv_dtype in_dtype, int64_t n_members, int64_t ny,
                                        int64_t nx, int64_t member_stride, double dx, double dy,
                                        int32_t ddof, void* mean_gx, void* var_gx,
                                        void* mean_gy, void* var_gy, pdiv_dtype out_dtype,
                                        pdiv_stream stream) {
  g_last_error.clear();
  log_call("pdiv_speed_gradient_moments members=%lld ny=%lld nx=%lld in=%d", (long long)n_members,
           (long long)ny, (long long)nx, int(in_dtype));
  PDIV_NONNULL(u_members);
  PDIV_NONNULL(v_members);
  PDIV_NONNULL(mean_gx);
  PDIV_NONNULL(var_gx);
  PDIV_NONNULL(mean_gy);
  PDIV_NONNULL(var_gy);
  PDIV_TRY(check_dtype(in_dtype, "in_dtype"));
  PDIV_TRY(check_dtype(out_dtype, "out_dtype"));
  PDIV_TRY(check_grid(ny, nx));
  PDIV_TRY(check_spacing(dx, dy));
  if (ddof != 0 && ddof != 1) return invalid("ddof must be 0 or 1 (got %d)", ddof);
  if (n_members <= ddof || n_members > (int64_t(1) << 30))
    return invalid("n_members must be in (ddof, 2^30] (got %lld)", (long long)n_members);
  const int64_t n = ny * nx;
  if (member_stride == 0) member_stride = n;
  if (member_stride < n)
    return invalid("member_stride %lld < ny*nx %lld", (long long)member_stride, (long long)n);
  if (!launch_fits(speed_gradient_blocks(ny, nx), 256))
    return invalid("grid of %lld x %lld points is too large for one launch", (long long)ny,
                   (long long)nx);
  return device_status(
      launch_speed_gradient_moments(u_members, v_members, in_dtype, n_members, ny, nx,
                                    member_stride, make_coef(dx, dy), ddof, mean_gx, var_gx,
                                    mean_gy, var_gy, out_dtype, static_cast<hipStream_t>(stream)),
      "speed-gradient launch");
}

pdiv_status pdiv_divergence_gaussian(const void* mean_u, const void* var_u, const void* mean_v,
                                     const void* var_v, pdiv_dtype in_dtype, int64_t ny,
                                     int64_t nx, double dx, double dy, float* div_mean,
                                     float* div_var, pdiv_stream stream) {
  g_last_error.clear();
  log_call("pdiv_divergence_gaussian ny=%lld nx=%lld in=%d", (long long)ny, (long long)nx,
           int(in_dtype));
  PDIV_NONNULL(mean_u);
  PDIV_NONNULL(var_u);
  PDIV_NONNULL(mean_v);
  PDIV_NONNULL(var_v);
  PDIV_NONNULL(div_mean);
  PDIV_NONNULL(div_var);
  PDIV_TRY(check_dtype(in_dtype, "in_dtype"));
  PDIV_TRY(check_grid(ny, nx));
  PDIV_TRY(check_spacing(dx, dy));
  PDIV_TRY(check_inputs(mean_u, var_u, mean_v, var_v, in_dtype, ny * nx,
                        static_cast<hipStream_t>(stream), "pdiv_divergence_gaussian"));
  return device_status(launch_divergence(mean_u, var_u, mean_v, var_v, in_dtype, ny, nx,
                                         make_coef(dx, dy), div_mean, div_var,
                                         static_cast<hipStream_t>(stream)),
                       "divergence launch");
}

pdiv_status pdiv_lcp(const float* div_mean, const float* div_var, int64_t ny, int64_t nx,
                     const float* isovalues_host, int32_t n_iso, float* lcp,
                     int64_t lcp_row_pitch, int64_t lcp_plane_stride, pdiv_stream stream) {
  g_last_error.clear();
  log_call("pdiv_lcp ny=%lld nx=%lld n_iso=%d pitch=%lld plane=%lld", (long long)ny,
           (long long)nx, n_iso, (long long)lcp_row_pitch, (long long)lcp_plane_stride);
  PDIV_NONNULL(div_mean);
  PDIV_NONNULL(div_var);
  PDIV_FLOATS(lcp);
  PDIV_TRY(check_grid(ny, nx));
  PDIV_TRY(check_iso(isovalues_host, n_iso));
  OutLayout lo;
  PDIV_TRY(check_layout(lcp_row_pitch, lcp_plane_stride, ny, nx, n_iso, &lo));
  PDIV_TRY(check_inputs(div_mean, div_var, div_mean, div_var, PDIV_F32, ny * nx,
                        static_cast<hipStream_t>(stream), "pdiv_lcp"));
  return lcp_chunks(false, div_mean, div_var, nullptr, nullptr, PDIV_F32, ny, nx, 1.0, 1.0,
                    isovalues_host, n_iso, lcp, lo, static_cast<hipStream_t>(stream));
}

pdiv_status pdiv_lcp_from_moments(const void* mean_u, const void* var_u, const void* mean_v,
                                  const void* var_v, pdiv_dtype in_dtype, int64_t ny,
                                  int64_t nx, double dx, double dy,
                                  const float* isovalues_host, int32_t n_iso, float* lcp,
                                  int64_t lcp_row_pitch, int64_t lcp_plane_stride,
                                  pdiv_stream stream) {
  g_last_error.clear();
  log_call("pdiv_lcp_from_moments ny=%lld nx=%lld in=%d n_iso=%d pitch=%lld plane=%lld",
           (long long)ny, (long long)nx, int(in_dtype), n_iso, (long long)lcp_row_pitch,
           (long long)lcp_plane_stride);
  PDIV_NONNULL(mean_u);
  PDIV_NONNULL(var_u);
  PDIV_NONNULL(mean_v);
  PDIV_NONNULL(var_v);
  PDIV_FLOATS(lcp);
  PDIV_TRY(check_dtype(in_dtype, "in_dtype"));
  PDIV_TRY(check_grid(ny, nx));
  PDIV_TRY(check_spacing(dx, dy));
  PDIV_TRY(check_iso(isovalues_host, n_iso));
  OutLayout lo;
  PDIV_TRY(check_layout(lcp_row_pitch, lcp_plane_stride, ny, nx, n_iso, &lo));
  PDIV_TRY(check_inputs(mean_u, var_u, mean_v, var_v, in_dtype, ny * nx,
                        static_cast<hipStream_t>(stream), "pdiv_lcp_from_moments"));
  return lcp_chunks(true, mean_u, var_u, mean_v, var_v, in_dtype, ny, nx, dx, dy,
                    isovalues_host, n_iso, lcp, lo, static_cast<hipStream_t>(stream));
}

pdiv_status pdiv_isocontour(const float* field, int64_t ny, int64_t nx, float isovalue,
                            int64_t* row_offsets, float* segments, int64_t max_segments,
                            pdiv_stream stream) {
  g_last_error.clear();
  log_call("pdiv_isocontour ny=%lld nx=%lld max_segments=%lld", (long long)ny, (long long)nx,
           (long long)max_segments);
  PDIV_NONNULL(field);
  PDIV_NONNULL(row_offsets);
  PDIV_TRY(check_grid(ny, nx));
  if (max_segments < 0) return invalid("max_segments must be >= 0 (got %lld)",
                                       (long long)max_segments);
  if (max_segments > 0 && segments == nullptr) return invalid("segments is NULL");
  if (max_segments > 0 && reinterpret_cast<uintptr_t>(segments) % 16 != 0)
    return invalid("segments must be 16-byte aligned");
  return device_status(launch_isocontour(field, ny, nx, isovalue, row_offsets, segments,
                                         max_segments, static_cast<hipStream_t>(stream)),
                       "isocontour launch");
}

pdiv_status pdiv_spaghetti(const void* u_members, const void* v_members, pdiv_dtype in_dtype,
                           int64_t n_members, int64_t ny, int64_t nx, int64_t member_stride,
                           double dx, double dy, float isovalue, float* div_workspace,
                           int64_t* row_offsets, float* segments, int64_t max_segments,
                           pdiv_stream stream) {
  g_last_error.clear();
  log_call("pdiv_spaghetti members=%lld ny=%lld nx=%lld", (long long)n_members, (long long)ny,
           (long long)nx);
  PDIV_NONNULL(div_workspace);
  PDIV_TRY(check_spaghetti(u_members, v_members, in_dtype, n_members, ny, nx, &member_stride,
                           dx, dy, row_offsets, segments, max_segments));
  return device_status(run_spaghetti(u_members, v_members, in_dtype, n_members, ny, nx,
                                     member_stride, dx, dy, isovalue, div_workspace,
                                     row_offsets, segments, max_segments,
                                     static_cast<hipStream_t>(stream)),
                       "spaghetti launch");
}

pdiv_status pdiv_spaghetti_noalloc(const void* u_members, const void* v_members,
                                   pdiv_dtype in_dtype, int64_t n_members, int64_t ny,
                                   int64_t nx, int64_t member_stride, double dx, double dy,
                                   float isovalue, int64_t* row_offsets, float* segments,
                                   int64_t max_segments, pdiv_stream stream) {
  g_last_error.clear();
  log_call("pdiv_spaghetti_noalloc members=%lld ny=%lld nx=%lld", (long long)n_members,
           (long long)ny, (long long)nx);
  PDIV_TRY(check_spaghetti(u_members, v_members, in_dtype, n_members, ny, nx, &member_stride,
                           dx, dy, row_offsets, segments, max_segments));
  if (n_members * ny * nx > kScratchFloats)
    return invalid("n_members*ny*nx = %lld exceeds the %lld floats of the library's own "
                   "workspace; use pdiv_spaghetti with a caller workspace",
                   (long long)(n_members * ny * nx), (long long)kScratchFloats);
  float* div = nullptr;
  PDIV_TRY(scratch_for_current_device(&div));
  return device_status(run_spaghetti(u_members, v_members, in_dtype, n_members, ny, nx,
                                     member_stride, dx, dy, isovalue, div, row_offsets,
                                     segments, max_segments, static_cast<hipStream_t>(stream)),
                       "spaghetti launch");
}

pdiv_status pdiv_divergence_gaussian_3d(const void* mean_u, const void* var_u,
                                        const void* mean_v, const void* var_v,
                                        const void* mean_w, const void* var_w,
                                        pdiv_dtype in_dtype, int64_t nz, int64_t ny, int64_t nx,
                                        double dx, double dy, double dz, float* div_mean,
                                        float* div_var, pdiv_stream stream) {
  g_last_error.clear();
  log_call("pdiv_divergence_gaussian_3d nz=%lld ny=%lld nx=%lld", (long long)nz, (long long)ny,
           (long long)nx);
  PDIV_NONNULL(mean_u);
  PDIV_NONNULL(var_u);
  PDIV_NONNULL(mean_v);
  PDIV_NONNULL(var_v);
  PDIV_NONNULL(mean_w);
  PDIV_NONNULL(var_w);
  PDIV_NONNULL(div_mean);
  PDIV_NONNULL(div_var);
  PDIV_TRY(check_dtype(in_dtype, "in_dtype"));
  PDIV_TRY(check_grid3(nz, ny, nx));
  PDIV_TRY(check_spacing(dx, dy));
  if (!(std::isfinite(dz) && dz > 0.0)) return invalid("dz must be finite and > 0 (got %g)", dz);
  return device_status(launch_divergence3d(mean_u, var_u, mean_v, var_v, mean_w, var_w,
                                           in_dtype, nz, ny, nx, make_coef3(dx, dy, dz),
                                           div_mean, div_var, static_cast<hipStream_t>(stream)),
                       "3D divergence launch");
}

namespace {

// Output layout of the 3D maps: rows of `pitch` floats (0: nx-1, dense),
// layers (ny-1) pitch apart, maps `plane` floats apart (0: the layers of one
// map back to back).  Maps may not overlap.
pdiv_status check_layout3(int64_t row_pitch, int64_t plane_stride, int64_t nz, int64_t ny,
                          int64_t nx, int32_t n_iso, OutLayout* out) {
  const int64_t cells = nx - 1;
  const int64_t pitch = row_pitch == 0 ? cells : row_pitch;
  if (pitch < cells || pitch > (int64_t(1) << 52))
    return invalid("lcp_row_pitch must be 0 or in [nx - 1, 2^52] (got %lld, nx=%lld)",
                   (long long)row_pitch, (long long)nx);
  const double map_d = double(nz - 1) * double(ny - 1) * double(pitch);
  if (map_d > double(int64_t(1) << 52))
    return invalid("LCP output layout is too large (layers x rows x pitch > 2^52 floats)");
  const int64_t map = (nz - 1) * (ny - 1) * pitch;
  const int64_t plane = plane_stride == 0 ? map : plane_stride;
  if (plane < map || plane > (int64_t(1) << 52))
    return invalid("lcp_plane_stride must be 0 or in [(nz-1)(ny-1) row pitch, 2^52] (got %lld)",
                   (long long)plane_stride);
  if ((double(n_iso - 1) * double(plane) + map_d) * 4.0 >= double(int64_t(1) << 56))
    return invalid("LCP output layout is too large");
  out->pitch = pitch;
  out->plane = plane;
  return PDIV_OK;
}

// Isovalue chunks for the 3D LCP launches: 8, 4, 2, 1 for the two-step form
// (a wave carries four cell layers at up to 8 isovalues; at 16 it could
// carry only two, and the tails of the extra shared z levels cost more than
// reading the divergence volumes twice), 16, 8, 4, 2, 1 fused (the six
// moment volumes are read once).  planes is null for the two-step form (dm,
// dv given), else the six moment volumes.
pdiv_status lcp3d_chunks(const float* dm, const float* dv, const void* const* planes,
                         pdiv_dtype dt, int64_t nz, int64_t ny, int64_t nx,
                         const StencilCoef3& k, const float* iso_host, int32_t n_iso,
                         float* lcp, const OutLayout& lo, hipStream_t s) {
  for (int32_t k0 = 0; k0 < n_iso;) {
    const int left = n_iso - k0;
    const int kc = (left >= 16 && planes) ? 16 : left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
    IsoChunk c;
    for (int q = 0; q < kIsoChunk; ++q) c.c[q] = iso_host[k0 + (q < kc ? q : kc - 1)];
    float* const out = lcp + k0 * lo.plane;
    const hipError_t e =
        planes ? launch_lcp3d_fused(planes, dt, nz, ny, nx, k, c, kc, out, lo.pitch, lo.plane, s)
               : launch_lcp3d(dm, dv, nz, ny, nx, c, kc, out, lo.pitch, lo.plane, s);
    if (e != hipSuccess) return device_status(e, "3D LCP launch");
    k0 += kc;
  }
  return PDIV_OK;
}

}  // namespace

pdiv_status pdiv_lcp_3d(const float* div_mean, const float* div_var, int64_t nz, int64_t ny,
                        int64_t nx, const float* isovalues_host, int32_t n_iso, float* lcp,
                        int64_t lcp_row_pitch, int64_t lcp_plane_stride, pdiv_stream stream) {
  g_last_error.clear();
  log_call("pdiv_lcp_3d nz=%lld ny=%lld nx=%lld n_iso=%d", (long long)nz, (long long)ny,
           (long long)nx, n_iso);
  PDIV_NONNULL(div_mean);
  PDIV_NONNULL(div_var);
  PDIV_FLOATS(lcp);
  PDIV_TRY(check_grid3(nz, ny, nx));
  PDIV_TRY(check_iso(isovalues_host, n_iso));
  if (!lcp3d_slice_fits(ny, nx, 4))
    return invalid("3D LCP slices are limited to 7 ny nx x 4 bytes < 2^31 (ny=%lld, nx=%lld)",
                   (long long)ny, (long long)nx);
  OutLayout lo;
  PDIV_TRY(check_layout3(lcp_row_pitch, lcp_plane_stride, nz, ny, nx, n_iso, &lo));
  return lcp3d_chunks(div_mean, div_var, nullptr, PDIV_F32, nz, ny, nx, StencilCoef3{},
                      isovalues_host, n_iso, lcp, lo, static_cast<hipStream_t>(stream));
}

pdiv_status pdiv_lcp_3d_from_moments(const void* mean_u, const void* var_u, const void* mean_v,
                                     const void* var_v, const void* mean_w, const void* var_w,
                                     pdiv_dtype in_dtype, int64_t nz, int64_t ny, int64_t nx,
                                     double dx, double dy, double dz,
                                     const float* isovalues_host, int32_t n_iso, float* lcp,
                                     int64_t lcp_row_pitch, int64_t lcp_plane_stride,
                                     pdiv_stream stream) {
  g_last_error.clear();
  log_call("pdiv_lcp_3d_from_moments nz=%lld ny=%lld nx=%lld n_iso=%d", (long long)nz,
           (long long)ny, (long long)nx, n_iso);
  PDIV_NONNULL(mean_u);
  PDIV_NONNULL(var_u);
  PDIV_NONNULL(mean_v);
  PDIV_NONNULL(var_v);
  PDIV_NONNULL(mean_w);
  PDIV_NONNULL(var_w);
  PDIV_FLOATS(lcp);
  PDIV_TRY(check_dtype(in_dtype, "in_dtype"));
  PDIV_TRY(check_grid3(nz, ny, nx));
  PDIV_TRY(check_spacing(dx, dy));
  if (!(std::isfinite(dz) && dz > 0.0)) return invalid("dz must be finite and > 0 (got %g)", dz);
  PDIV_TRY(check_iso(isovalues_host, n_iso));
  if (!lcp3d_slice_fits(ny, nx, in_dtype == PDIV_F32 ? 4 : 2))
    return invalid("3D LCP slices are limited to 7 ny nx x element bytes < 2^31 (ny=%lld, "
                   "nx=%lld)", (long long)ny, (long long)nx);
  OutLayout lo;
  PDIV_TRY(check_layout3(lcp_row_pitch, lcp_plane_stride, nz, ny, nx, n_iso, &lo));
  const void* const planes[6] = {mean_u, var_u, mean_v, var_v, mean_w, var_w};
  return lcp3d_chunks(nullptr, nullptr, planes, in_dtype, nz, ny, nx, make_coef3(dx, dy, dz),
                      isovalues_host, n_iso, lcp, lo, static_cast<hipStream_t>(stream));
}

pdiv_status pdiv_mc_lcp(const void* mean_u, const void* var_u, const void* mean_v,
                        const void* var_v, pdiv_dtype in_dtype, int64_t ny, int64_t nx,
                        double dx, double dy, const float* isovalues_host, int32_t n_iso,
                        int64_t n_samples, uint64_t seed, uint32_t mode, float* lcp,
                        pdiv_stream stream) {
  g_last_error.clear();
  log_call("pdiv_mc_lcp ny=%lld nx=%lld n_iso=%d samples=%lld mode=%u", (long long)ny,
           (long long)nx, n_iso, (long long)n_samples, mode);
  PDIV_NONNULL(mean_u);
  PDIV_NONNULL(var_u);
  PDIV_NONNULL(mean_v);
  PDIV_NONNULL(var_v);
  PDIV_FLOATS(lcp);
  PDIV_TRY(check_dtype(in_dtype, "in_dtype"));
  PDIV_TRY(check_grid(ny, nx));
  PDIV_TRY(check_spacing(dx, dy));
  PDIV_TRY(check_iso(isovalues_host, n_iso));
  if (ny * nx >= (int64_t(1) << 32))
    return invalid("Monte Carlo needs ny*nx < 2^32 (point index is a 32-bit counter word)");
  if (n_samples < 1 || n_samples >= (int64_t(1) << 31))
    return invalid("n_samples must be in [1, 2^31) (got %lld)", (long long)n_samples);
  if (mode != PDIV_MC_VECTOR && mode != PDIV_MC_VERTEX)
    return invalid("mode must be PDIV_MC_VECTOR (0) or PDIV_MC_VERTEX (1) (got %u)", mode);
  if (!launch_fits(mc_tiles_x(nx), 256) || !launch_fits(mc_tiles_y(ny), 256))
    return invalid("grid of %lld x %lld points is too large for one Monte Carlo launch",
                   (long long)ny, (long long)nx);
  PDIV_TRY(check_inputs(mean_u, var_u, mean_v, var_v, in_dtype, ny * nx,
                        static_cast<hipStream_t>(stream), "pdiv_mc_lcp"));
  const StencilCoef k = make_coef(dx, dy);
  const int64_t plane = (ny - 1) * (nx - 1);
  for (int32_t k0 = 0; k0 < n_iso; k0 += kIsoChunk) {
    const int kc = (n_iso - k0) < kIsoChunk ? (n_iso - k0) : kIsoChunk;
    IsoChunk c;
    for (int q = 0; q < kIsoChunk; ++q) c.c[q] = isovalues_host[k0 + (q < kc ? q : kc - 1)];
    hipError_t e = launch_mc(mean_u, var_u, mean_v, var_v, in_dtype, ny, nx, k, c, kc,
                             n_samples, seed, mode, lcp + k0 * plane,
                             static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_status(e, "Monte Carlo launch");
  }
  return PDIV_OK;
}

pdiv_status pdiv_mc_sample_field(const void* mean_u, const void* var_u, const void* mean_v,
                                 const void* var_v, pdiv_dtype in_dtype, int64_t ny, int64_t nx,
                                 int64_t sample, uint64_t seed, float* u_s, float* v_s,
                                 pdiv_stream stream) {
  g_last_error.clear();
  PDIV_NONNULL(mean_u);
  PDIV_NONNULL(var_u);
  PDIV_NONNULL(mean_v);
  PDIV_NONNULL(var_v);
  PDIV_NONNULL(u_s);
  PDIV_NONNULL(v_s);
  PDIV_TRY(check_dtype(in_dtype, "in_dtype"));
  PDIV_TRY(check_grid(ny, nx));
  if (ny * nx >= (int64_t(1) << 32)) return invalid("ny*nx must be < 2^32");
  if (sample < 0 || sample >= (int64_t(1) << 31)) return invalid("sample out of range");
  return device_status(launch_mc_sample(mean_u, var_u, mean_v, var_v, in_dtype, ny, nx, sample,
                                        seed, u_s, v_s, static_cast<hipStream_t>(stream)),
                       "sample launch");
}

}  // extern "C"
