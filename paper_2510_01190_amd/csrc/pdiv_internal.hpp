// Host-side interface between the C ABI (pdiv_api.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/pdiv.h"

namespace pdiv {

// Message of the last failing call on this thread (pdiv_last_error).
extern thread_local std::string g_last_error;
// Records a message for pdiv_last_error.
void set_error(const char* fmt, ...);
// Records a message and returns PDIV_ERR_INVALID.
pdiv_status invalid(const char* fmt, ...);
// PDIV_OK for hipSuccess; otherwise records the HIP error and returns PDIV_ERR_DEVICE.
pdiv_status device_status(hipError_t e, const char* what);

// Isovalues of one launch, passed by value in the kernel arguments so that
// every wave reads them from scalar registers.
constexpr int kIsoChunk = 16;
// A dispatch covers at most 2^32 - 1 work-items per grid dimension; a 1D
// launch of `blocks` blocks of `threads` threads fits iff this holds.
inline bool launch_fits(int64_t blocks, int threads) {
  return blocks >= 0 && blocks <= int64_t(0xffffffff) / threads;
}

struct IsoChunk {
  float c[kIsoChunk];
};

// Finite-difference coefficients of Eq. 1-3 in float32: m = 1/(2h) inside,
// 1/h on the boundary; v = m^2.
struct StencilCoef {
  float cxm_in, cxv_in, cxm_bd, cxv_bd;
  float cym_in, cyv_in, cym_bd, cyv_bd;
};
StencilCoef make_coef(double dx, double dy);

// Output layout of the LCP maps in floats: row pitch (0: dense, nx - 1; else
// >= nx - 1) and plane stride (0: (ny - 1) row pitch).  The maps may be apart
// (plane stride >= (ny - 1) row pitch) or interleaved by rows (plane stride
// >= nx - 1 and row pitch >= n_iso plane stride); any other pair makes maps
// overlap.  check_layout validates (PDIV_ERR_INVALID with a message) and
// resolves the zeros.
struct OutLayout {
  int64_t pitch, plane;
};
pdiv_status check_layout(int64_t row_pitch, int64_t plane_stride, int64_t ny, int64_t nx,
                         int32_t n_iso, OutLayout* out);

// Tile shape of the column-walking LCP kernels: one wave covers a strip of
// 128 (paired layout) or 126 cells (split layout) over a band of `band_rows`
// cell rows; 0 lets the launcher choose per layout.
struct LcpShape {
  int band_rows;
  bool poison;  // PDIV_DEBUG_POISON_LDS: NaN-fill the LDS ring slots
};
LcpShape default_lcp_shape(int64_t ny, int64_t nx, int n_iso);
void set_band_rows_override(int rows);

// Process-wide checking modes (PDIV_DEBUG_* of pdiv_set_debug; the
// environment variables PDIV_DEBUG_CHECKS and PDIV_LOG set their bits at
// load).
uint32_t debug_flags();
void set_debug_flags(uint32_t flags);

hipError_t launch_moments(const void* u, const void* v, pdiv_dtype in_dtype, int64_t m,
                          int64_t n_points, int64_t stride, int ddof, void* mu, void* vu,
                          void* mv, void* vv, pdiv_dtype out_dtype, hipStream_t s);

hipError_t launch_divergence(const void* mu, const void* vu, const void* mv, const void* vv,
                             pdiv_dtype dt, int64_t ny, int64_t nx, const StencilCoef& k,
                             float* dmean, float* dvar, hipStream_t s);

// LCP for isovalues [k0, k0+kc) (kc <= 16): from divergence Gaussians
// (fused = false, planes dmean/dvar as float) or from moments (fused = true).
// Output rows are `pitch` floats apart, planes `plane` floats.
hipError_t launch_lcp(bool fused, const void* p0, const void* p1, const void* p2,
                      const void* p3, pdiv_dtype dt, int64_t ny, int64_t nx,
                      const StencilCoef& k, const IsoChunk& iso, int kc, float* lcp_k0,
                      int64_t pitch, int64_t plane, LcpShape shape, hipStream_t s);

// Monte Carlo LCP, mode PDIV_MC_VECTOR (the paper's sampling of the vectors)
// or PDIV_MC_VERTEX (each vertex divergence drawn on its own).  The launch is
// mc_tiles_x(nx) x mc_tiles_y(ny) blocks of 256 threads.
int64_t mc_tiles_x(int64_t nx);
int64_t mc_tiles_y(int64_t ny);
hipError_t launch_mc(const void* mu, const void* vu, const void* mv, const void* vv,
                     pdiv_dtype dt, int64_t ny, int64_t nx, const StencilCoef& k,
                     const IsoChunk& iso, int kc, int64_t n_samples, uint64_t seed,
                     uint32_t mode, float* lcp_k0, hipStream_t s);

hipError_t launch_mc_sample(const void* mu, const void* vu, const void* mv, const void* vv,
                            pdiv_dtype dt, int64_t ny, int64_t nx, int64_t sample,
                            uint64_t seed, float* us, float* vs, hipStream_t s);

// Red Sea pre-stage: per member the gradient of the speed by Eq. 1's
// differences, fitted per point over the members (Welford, float32).
int64_t speed_gradient_blocks(int64_t ny, int64_t nx);
hipError_t launch_speed_gradient_moments(const void* u, const void* v, pdiv_dtype in_dt,
                                         int64_t m, int64_t ny, int64_t nx, int64_t stride,
                                         const StencilCoef& k, int ddof, void* mgx, void* vgx,
                                         void* mgy, void* vgy, pdiv_dtype out_dt,
                                         hipStream_t s);

// Marching-squares isocontour of a [ny][nx] float32 field: row_offsets (ny
// entries) receives each cell row's first segment index and the total at
// [ny-1]; segments [max_segments][4] (x0, y0, x1, y1), the ones past
// max_segments not written.
hipError_t launch_isocontour(const float* field, int64_t ny, int64_t nx, float c,
                             int64_t* row_offsets, float* segments, int64_t max_segments,
                             hipStream_t s);
// The same over n_fields fields field_stride floats apart (row_offsets:
// n_fields (ny-1) + 1 entries, field-major).
hipError_t launch_isocontours(const float* fields, int64_t n_fields, int64_t field_stride,
                              int64_t ny, int64_t nx, float c, int64_t* row_offsets,
                              float* segments, int64_t max_segments, hipStream_t s);
// Eq. 1 of each of m members (deterministic fields) into div [m][ny][nx].
hipError_t launch_members_divergence(const void* u, const void* v, pdiv_dtype dt, int64_t m,
                                     int64_t ny, int64_t nx, int64_t stride,
                                     const StencilCoef& k, float* div, hipStream_t s);

// 3D extension: the coefficients of the x and y differences plus z's.
struct StencilCoef3 {
  StencilCoef xy;
  float czm_in, czv_in, czm_bd, czv_bd;
};
StencilCoef3 make_coef3(double dx, double dy, double dz);

// Blocks of the 3D launches (the API rejects grids whose launch would not fit).
int64_t divergence3d_blocks(int64_t nz, int64_t ny, int64_t nx);
int64_t lcp3d_blocks(int64_t nz, int64_t ny, int64_t nx, int kc);
// The 3D LCP walks reach up to 7 z levels of a plane from one buffer base
// (32-bit offsets): 7 ny nx elem_bytes < 2^31.
bool lcp3d_slice_fits(int64_t ny, int64_t nx, size_t elem_bytes);

hipError_t launch_divergence3d(const void* mu, const void* vu, const void* mv, const void* vv,
                               const void* mw, const void* vw, pdiv_dtype dt, int64_t nz,
                               int64_t ny, int64_t nx, const StencilCoef3& k, float* dmean,
                               float* dvar, hipStream_t s);

// 8-corner LCP for isovalues [k0, k0+kc) (kc in {1, 2, 4, 8, 16}) from 3D
// divergence Gaussians; maps [kc][nz-1][ny-1][nx-1], rows `pitch` floats
// apart, layers (ny-1) pitch, maps `plane` floats apart.
hipError_t launch_lcp3d(const float* dm, const float* dv, int64_t nz, int64_t ny, int64_t nx,
                        const IsoChunk& iso, int kc, float* out_k0, int64_t pitch,
                        int64_t plane, hipStream_t s);
// The same from the six moment volumes (mean_u, var_u, mean_v, var_v,
// mean_w, var_w) of type dt, Eq. 2-3 evaluated on the spot.
hipError_t launch_lcp3d_fused(const void* const* planes, pdiv_dtype dt, int64_t nz, int64_t ny,
                              int64_t nx, const StencilCoef3& k, const IsoChunk& iso, int kc,
                              float* out_k0, int64_t pitch, int64_t plane, hipStream_t s);

}  // namespace pdiv
