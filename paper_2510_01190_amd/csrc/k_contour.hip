// Isocontour geometry by marching squares: the mean-field contour of the
// divergence and the per-member contours of a spaghetti plot (Section 4,
// the figures' geometry).  Rules: a corner is above iff its value >= c; the
// case index sums 1, 2, 4, 8 for the corners (i,j), (i+1,j), (i+1,j+1),
// (i,j+1) that are above; a crossed edge from corner value p to q gets the
// point at t = (c - p) / (q - p); the two saddle cases are split by the cell
// centre ((v00 + v10) + (v11 + v01)) / 4.  Segments are listed cell by cell
// in row-major order, so the output is deterministic:
//   count  one wave per cell row: segments of the row;
//   scan   one block: exclusive scan of the row counts, total at the end;
//   write  one wave per cell row: each lane's segments at the row's offset
//          plus the count of the lanes before it (ballot + prefix count).
#include <hip/hip_runtime.h>

#include "pdiv_device.hpp"
#include "pdiv_internal.hpp"

namespace pdiv {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kScanBlock = 1024;
constexpr int kScanItems = 8;  // consecutive rows per scan thread
// A wave walks its cell row in chunks of 64 cells, kUnroll chunks at a time:
// their loads are unconditional (clamped to the last cell) and issued
// together before any of them is classified, so that the row's walk is not
// one dependent load round per chunk.  At 8192^2 (6 M segments) the three
// passes take 0.370 ms one chunk at a time, 0.345 / 0.324 / 0.316 ms with
// 2 / 4 / 8 chunks.
constexpr int kUnroll = 8;

// Edges: 0 bottom (i,j)-(i+1,j), 1 right (i+1,j)-(i+1,j+1), 2 top
// (i,j+1)-(i+1,j+1), 3 left (i,j)-(i,j+1).  Nibble `case` of kEdgeA / kEdgeB
// holds the two edges of the case's segment (the saddles 5 and 10 and the
// empty cases 0 and 15 are decided apart).
constexpr uint64_t kEdgeA = 0x0303100220013030ull;
constexpr uint64_t kEdgeB = 0x0011202332021100ull;

struct Cell {
  int n;       // segments: 0, 1 or 2
  int a0, b0;  // edges of the first segment
  int a1, b1;  // edges of the second (saddles)
};

__device__ __forceinline__ Cell classify(float v00, float v10, float v11, float v01, float c) {
  const int cs = int(v00 >= c) | (int(v10 >= c) << 1) | (int(v11 >= c) << 2) | (int(v01 >= c) << 3);
  Cell r;
  r.a0 = int((kEdgeA >> (4 * cs)) & 15u);
  r.b0 = int((kEdgeB >> (4 * cs)) & 15u);
  r.a1 = r.b1 = 0;
  r.n = (cs == 0 || cs == 15) ? 0 : 1;
  if (cs == 5 || cs == 10) {
#pragma clang fp contract(off)
    const float centre = ((v00 + v10) + (v11 + v01)) * 0.25f;
    // the corners on the centre's side connect through the cell; the
    // contour cuts off the other two
    const bool join_diag = (cs == 5) == (centre >= c);
    r.n = 2;
    r.a0 = join_diag ? 0 : 3;
    r.b0 = join_diag ? 1 : 0;
    r.a1 = join_diag ? 2 : 1;
    r.b1 = join_diag ? 3 : 2;
  }
  return r;
}

__device__ __forceinline__ float2 edge_point(int e, int i, int j, float v00, float v10, float v11,
                                             float v01, float c) {
  switch (e) {
    case 0: return make_float2(float(i) + (c - v00) / (v10 - v00), float(j));
    case 1: return make_float2(float(i + 1), float(j) + (c - v10) / (v11 - v10));
    case 2: return make_float2(float(i) + (c - v01) / (v11 - v01), float(j + 1));
    default: return make_float2(float(i), float(j) + (c - v00) / (v01 - v00));
  }
}

struct Corners {
  float v00, v10, v11, v01;
};

__device__ __forceinline__ Corners corners(const float* __restrict__ f, int nx, int j, int i) {
  const int64_t o = int64_t(j) * nx + i;
  Corners k;
  k.v00 = f[o];
  k.v10 = f[o + 1];
  k.v01 = f[o + nx];
  k.v11 = f[o + nx + 1];
  return k;
}

// Rows r = 0 .. n_fields (ny - 1) - 1 of n_fields fields stored field_stride
// floats apart: cell row j = r mod (ny - 1) of field r / (ny - 1).
__global__ __launch_bounds__(kBlock) void contour_count_kernel(const float* __restrict__ f0, int ny,
                                                               int nx, int64_t field_stride,
                                                               int rows, float c,
                                                               int64_t* __restrict__ counts) {
  const int r = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (r >= rows) return;
  const int j = r % (ny - 1);
  const float* const f = f0 + int64_t(r / (ny - 1)) * field_stride;
  const int lane = threadIdx.x & 63;
  int n = 0;
  for (int i0 = 0; i0 < nx - 1; i0 += 64 * kUnroll) {
    Corners k[kUnroll];
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) k[q] = corners(f, nx, j, min(i0 + 64 * q + lane, nx - 2));
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      const int ni = classify(k[q].v00, k[q].v10, k[q].v11, k[q].v01, c).n;
      n += i0 + 64 * q + lane < nx - 1 ? ni : 0;
    }
  }
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) n += __shfl_xor(n, s, 64);
  if (lane == 0) counts[r] = n;
}

// Exclusive scan of counts[0 .. n) in place, total to counts[n]; one block.
// Per pass thread t sums its kScanItems consecutive counts, the block scans
// the thread sums (Hillis-Steele in LDS), and each thread writes its items'
// offsets from its own prefix.
__global__ __launch_bounds__(kScanBlock) void contour_scan_kernel(int64_t* __restrict__ counts,
                                                                  int n) {
  __shared__ int64_t buf[kScanBlock];
  const int t = threadIdx.x;
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += int64_t(kScanBlock) * kScanItems) {
    const int64_t first = base + int64_t(t) * kScanItems;
    int64_t x[kScanItems];
    int64_t sum = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
      x[q] = first + q < n ? counts[first + q] : 0;
      sum += x[q];
    }
    buf[t] = sum;
    __syncthreads();
    for (int d = 1; d < kScanBlock; d <<= 1) {
      const int64_t y = t >= d ? buf[t - d] : 0;
      __syncthreads();
      buf[t] += y;
      __syncthreads();
    }
    int64_t run = carry + buf[t] - sum;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
      if (first + q < n) counts[first + q] = run;
      run += x[q];
    }
    carry += buf[kScanBlock - 1];
    __syncthreads();
  }
  if (t == 0) counts[n] = carry;
}

__global__ __launch_bounds__(kBlock) void contour_write_kernel(
    const float* __restrict__ f0, int ny, int nx, int64_t field_stride, int rows, float c,
    const int64_t* __restrict__ offsets, float4* __restrict__ segs, int64_t max_segs) {
  const int r = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (r >= rows) return;
  const int j = r % (ny - 1);
  const float* const f = f0 + int64_t(r / (ny - 1)) * field_stride;
  const int lane = threadIdx.x & 63;
  const uint64_t below_me = __lanemask_lt();
  int64_t k = offsets[r];
  // every lane walks the same number of chunks, so the ballots see the wave
  for (int i00 = 0; i00 < nx - 1; i00 += 64 * kUnroll) {
    Corners vs[kUnroll];
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) vs[q] = corners(f, nx, j, min(i00 + 64 * q + lane, nx - 2));
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      const int i = i00 + 64 * q + lane;
      const Corners& v = vs[q];
      Cell cell = classify(v.v00, v.v10, v.v11, v.v01, c);
      if (i >= nx - 1) cell.n = 0;
      const uint64_t one = __ballot(cell.n >= 1);
      const uint64_t two = __ballot(cell.n >= 2);
      const int64_t at = k + __popcll(one & below_me) + __popcll(two & below_me);
      if (cell.n >= 1 && at < max_segs) {
        const float2 p = edge_point(cell.a0, i, j, v.v00, v.v10, v.v11, v.v01, c);
        const float2 q2 = edge_point(cell.b0, i, j, v.v00, v.v10, v.v11, v.v01, c);
        segs[at] = make_float4(p.x, p.y, q2.x, q2.y);
      }
      if (cell.n >= 2 && at + 1 < max_segs) {
        const float2 p = edge_point(cell.a1, i, j, v.v00, v.v10, v.v11, v.v01, c);
        const float2 q2 = edge_point(cell.b1, i, j, v.v00, v.v10, v.v11, v.v01, c);
        segs[at + 1] = make_float4(p.x, p.y, q2.x, q2.y);
      }
      k += __popcll(one) + __popcll(two);
    }
  }
}

// Eq. 1 on every member of an ensemble (each member a deterministic field):
// the x and y differences with the coefficients of Eq. 2 and its rounding,
// so each divergence is bitwise the mean of a zero-variance Eq. 2.  Grid:
// x blocks of 64 columns, one row per wave, members outermost.
template <typename T>
__global__ __launch_bounds__(kBlock) void members_divergence_kernel(
    const T* __restrict__ u, const T* __restrict__ v, int ny, int nx, int64_t stride,
    StencilCoef k, float* __restrict__ div, int n_xb, int rows) {
  const int xb = blockIdx.x % n_xb;
  const int r = (blockIdx.x / n_xb) * kWavesPerBlock + (threadIdx.x >> 6);
  const int x = xb * 64 + (threadIdx.x & 63);
  if (r >= rows || x >= nx) return;
  const int m = r / ny, y = r % ny;
  const T* const um = u + int64_t(m) * stride;
  const T* const vm = v + int64_t(m) * stride;
  const int xl = x > 0 ? x - 1 : 0, xr = x < nx - 1 ? x + 1 : nx - 1;
  const int yl = y > 0 ? y - 1 : 0, yr = y < ny - 1 ? y + 1 : ny - 1;
  const bool bx = (x == 0) | (x == nx - 1), by = (y == 0) | (y == ny - 1);
  const float a_r = to_f32(um[int64_t(y) * nx + xr]), a_l = to_f32(um[int64_t(y) * nx + xl]);
  const float b_r = to_f32(vm[int64_t(yr) * nx + x]), b_l = to_f32(vm[int64_t(yl) * nx + x]);
  const float cx = bx ? k.cxm_bd : k.cxm_in, cy = by ? k.cym_bd : k.cym_in;
  float d;
  {
#pragma clang fp contract(off)
    d = (a_r - a_l) * cx + (b_r - b_l) * cy;
  }
  div[int64_t(m) * ny * nx + int64_t(y) * nx + x] = d;
}

}  // namespace

hipError_t launch_isocontours(const float* fields, int64_t n_fields, int64_t field_stride,
                              int64_t ny, int64_t nx, float c, int64_t* row_offsets,
                              float* segments, int64_t max_segments, hipStream_t s) {
  const int64_t rows64 = n_fields * (ny - 1);
  if (rows64 > 0x7fffffff || !launch_fits((rows64 + kWavesPerBlock - 1) / kWavesPerBlock, kBlock))
    return hipErrorInvalidConfiguration;
  const int rows = int(rows64);
  const unsigned blocks = unsigned((rows + kWavesPerBlock - 1) / kWavesPerBlock);
  hipLaunchKernelGGL(contour_count_kernel, dim3(blocks), dim3(kBlock), 0, s, fields, int(ny),
                     int(nx), field_stride, rows, c, row_offsets);
  hipLaunchKernelGGL(contour_scan_kernel, dim3(1), dim3(kScanBlock), 0, s, row_offsets, rows);
  hipLaunchKernelGGL(contour_write_kernel, dim3(blocks), dim3(kBlock), 0, s, fields, int(ny),
                     int(nx), field_stride, rows, c, row_offsets,
                     reinterpret_cast<float4*>(segments), max_segments);
  return hipGetLastError();
}

hipError_t launch_isocontour(const float* field, int64_t ny, int64_t nx, float c,
                             int64_t* row_offsets, float* segments, int64_t max_segments,
                             hipStream_t s) {
  return launch_isocontours(field, 1, ny * nx, ny, nx, c, row_offsets, segments, max_segments,
                            s);
}

hipError_t launch_members_divergence(const void* u, const void* v, pdiv_dtype dt, int64_t m,
                                     int64_t ny, int64_t nx, int64_t stride,
                                     const StencilCoef& k, float* div, hipStream_t s) {
  const int n_xb = int((nx + 63) / 64);
  const int64_t blocks64 = int64_t(n_xb) * ((m * ny + kWavesPerBlock - 1) / kWavesPerBlock);
  if (m * ny > 0x7fffffff || !launch_fits(blocks64, kBlock)) return hipErrorInvalidConfiguration;
  const int rows = int(m * ny);
  const unsigned blocks = unsigned(blocks64);
#define PDIV_MDIV(T)                                                                           \
  hipLaunchKernelGGL(members_divergence_kernel<T>, dim3(blocks), dim3(kBlock), 0, s,           \
                     static_cast<const T*>(u), static_cast<const T*>(v), int(ny), int(nx),     \
                     stride, k, div, n_xb, rows)
  switch (dt) {
    case PDIV_F32: PDIV_MDIV(float); break;
    case PDIV_F16: PDIV_MDIV(__half); break;
    case PDIV_BF16: PDIV_MDIV(bf16_t); break;
    default: return hipErrorInvalidValue;
  }
#undef PDIV_MDIV
  return hipGetLastError();
}

}  // namespace pdiv
