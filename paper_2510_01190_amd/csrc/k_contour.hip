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
//   write  one wave per cell row: a batch's segments are listed in LDS in
//          output order (ballot + prefix count), then computed and stored
//          64 at a time from the row's offset on.
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
// one dependent load round per chunk (at 8192^2 with 6 M segments the three
// passes took 0.370 ms one chunk at a time, 0.345 / 0.324 / 0.316 ms with
// 2 / 4 / 8 chunks).
constexpr int kUnroll = 8;

// Edges: 0 bottom (i,j)-(i+1,j), 1 right (i+1,j)-(i+1,j+1), 2 top
// (i,j+1)-(i+1,j+1), 3 left (i,j)-(i,j+1).  Nibble `case` of kEdgeA / kEdgeB
// holds the two edges of the case's segment (the saddles 5 and 10 and the
// empty cases 0 and 15 are decided apart).
constexpr uint64_t kEdgeA = 0x0303100220013030ull;
constexpr uint64_t kEdgeB = 0x0011202332021100ull;

struct Corners {
  float v00, v10, v11, v01;
};

// Edges (a, b) of a cell's first (second = false) or second segment, from
// its case index.  The two saddle cases are split by the cell centre: the
// corners on the centre's side connect through the cell and the contour
// cuts off the other two.
__device__ __forceinline__ void segment_edges(int cs, bool second, const Corners& v, float c,
                                              int& a, int& b) {
  a = int((kEdgeA >> (4 * cs)) & 15u);
  b = int((kEdgeB >> (4 * cs)) & 15u);
  if (cs == 5 || cs == 10) {
#pragma clang fp contract(off)
    const float centre = ((v.v00 + v.v10) + (v.v11 + v.v01)) * 0.25f;
    const bool join_diag = (cs == 5) == (centre >= c);
    if (!second) {
      a = join_diag ? 0 : 3;
      b = join_diag ? 1 : 0;
    } else {
      a = join_diag ? 2 : 1;
      b = join_diag ? 3 : 2;
    }
  }
}

// The crossing point on edge e: its end values p -> q are picked by selects
// and one division runs on them, the same for every lane whichever edge it
// holds.  Bottom (i,j)-(i+1,j) and top (i,j+1)-(i+1,j+1) run along x, right
// (i+1,j)-(i+1,j+1) and left (i,j)-(i,j+1) along y.
__device__ __forceinline__ float2 edge_point(int e, int i, int j, float v00, float v10, float v11,
                                             float v01, float c) {
  const bool along_x = (e == 0) | (e == 2);
  const float p = e == 0 ? v00 : e == 1 ? v10 : e == 2 ? v01 : v00;
  const float q = e == 0 ? v10 : e == 1 ? v11 : e == 2 ? v11 : v01;
  const float t = (c - p) / (q - p);
  const float fx = float(i + (e == 1 ? 1 : 0));
  const float fy = float(j + (e == 2 ? 1 : 0));
  return along_x ? make_float2(fx + t, fy) : make_float2(fx, fy + t);
}

// Segments per case index, two bits each: none for 0 and 15, two for the
// saddles 5 and 10, one otherwise.
constexpr uint32_t kSegCount = 0x15655954u;

// The two vertex rows of cell row j, read through buffer resources: the row
// bases live in scalar registers and a lane's loads share one 32-bit byte
// offset (the right-hand corners at +4 bytes), so a load needs no per-lane
// 64-bit address arithmetic.
// v with lane 63 replaced by the wave-uniform s (v_writelane_b32).
__device__ __forceinline__ float with_lane63(float v, int s) {
  asm("v_writelane_b32 %0, %1, 63" : "+v"(v) : "s"(s));
  return v;
}

struct RowPair {
  __amdgpu_buffer_rsrc_t lo, hi;
  __device__ __forceinline__ RowPair(const float* f, int nx, int j)
      : lo(__builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(f) + int64_t(j) * nx, 0,
                                             static_cast<int>(uint32_t(nx) * 4u), 0x00020000)),
        hi(__builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(f) + int64_t(j + 1) * nx, 0,
                                             static_cast<int>(uint32_t(nx) * 4u), 0x00020000)) {}
  // corners of cell i (0 <= i <= nx - 2)
  __device__ __forceinline__ Corners at(int i) const {
    const int o = i * 4;
    Corners k;
    k.v00 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(lo, o, 0, 0));
    k.v10 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(lo, o + 4, 0, 0));
    k.v01 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(hi, o, 0, 0));
    k.v11 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(hi, o + 4, 0, 0));
    return k;
  }
  __device__ __forceinline__ float2 vertices(int x) const {
    const int o = x * 4;
    return make_float2(__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(lo, o, 0, 0)),
                       __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(hi, o, 0, 0)));
  }
  // Corners of the cells i0 + 64 q + lane, q < U: each lane loads its
  // column's two vertices only (whole-line loads) and takes the right-hand
  // corners from lane + 1 through DPP; lane 63 takes them from lane 0 of
  // the next chunk, and the batch's last chunk from one more column, read
  // at the same address by every lane.  Columns are clamped to nx - 1, so
  // cells past the row's end get corners from valid columns (and are not
  // counted).  All lanes of the wave must be active.
  template <int U>
  __device__ __forceinline__ void batch(int i0, int lane, int nx, Corners (&k)[U]) const {
    float2 v[U];
#pragma unroll
    for (int q = 0; q < U; ++q) v[q] = vertices(min(i0 + 64 * q + lane, nx - 1));
    const float2 e = vertices(min(i0 + 64 * U, nx - 1));
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int s_lo = q + 1 < U ? __builtin_amdgcn_readlane(__float_as_int(v[q + 1].x), 0)
                                 : __builtin_amdgcn_readfirstlane(__float_as_int(e.x));
      const int s_hi = q + 1 < U ? __builtin_amdgcn_readlane(__float_as_int(v[q + 1].y), 0)
                                 : __builtin_amdgcn_readfirstlane(__float_as_int(e.y));
      k[q].v00 = v[q].x;
      k[q].v01 = v[q].y;
      k[q].v10 = with_lane63(dpp_from_right(v[q].x), s_lo);
      k[q].v11 = with_lane63(dpp_from_right(v[q].y), s_hi);
    }
  }
};

// Row of this wave.  Blocks are dealt round-robin to the 8 XCDs (block b
// runs on XCD b mod 8), each with its own L2; renumbering the blocks so
// that each XCD takes a contiguous run of rows lets the two rows that
// share a vertex row read it through one L2.  A bijection on the blocks.
__device__ __forceinline__ int wave_row() {
  const int nb = gridDim.x, xcd = blockIdx.x % 8, q8 = nb / 8, r8 = nb % 8;
  const int blk = xcd * q8 + min(xcd, r8) + blockIdx.x / 8;
  // uniform across the wave, which the compiler must know: the row's buffer
  // descriptors then stay in scalar registers (a descriptor computed from a
  // lane-varying value makes every buffer access a loop over its values)
  return __builtin_amdgcn_readfirstlane(blk * kWavesPerBlock + (threadIdx.x >> 6));
}

__device__ __forceinline__ int case_index(const Corners& k, float c) {
  return int(k.v00 >= c) | (int(k.v10 >= c) << 1) | (int(k.v11 >= c) << 2) |
         (int(k.v01 >= c) << 3);
}

// Rows r = 0 .. n_fields (ny - 1) - 1 of n_fields fields stored field_stride
// floats apart: cell row j = r mod (ny - 1) of field r / (ny - 1).
__global__ __launch_bounds__(kBlock) void contour_count_kernel(const float* __restrict__ f0, int ny,
                                                               int nx, int64_t field_stride,
                                                               int rows, float c,
                                                               int64_t* __restrict__ counts) {
  const int r = wave_row();
  if (r >= rows) return;
  const int j = r % (ny - 1);
  const RowPair rp(f0 + int64_t(r / (ny - 1)) * field_stride, nx, j);
  const int lane = threadIdx.x & 63;
  int n = 0;
  for (int i0 = 0; i0 < nx - 1; i0 += 64 * kUnroll) {
    Corners k[kUnroll];
    rp.batch(i0, lane, nx, k);
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      const int ni = int((kSegCount >> (2 * case_index(k[q], c))) & 3u);
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

// Write pass, one wave per cell row, 8 chunks of 64 cells per batch.  The
// batch's cells are classified lane by lane; the segments they hold are
// listed in LDS in output order (cell, then its first and second segment),
// each entry the cell's column within the batch and the segment's two edges;
// then lanes take the listed segments 64 at a time, load their cell's
// corners again (from the caches) and compute and store the points.  The
// divisions of the edge points so run once per 64 segments, not once per 64
// cells of which a few hold one, and the stores are contiguous.
constexpr int kList = 64 * kUnroll * 2;  // segments of a batch, at most

__global__ __launch_bounds__(kBlock) void contour_write_kernel(
    const float* __restrict__ f0, int ny, int nx, int64_t field_stride, int rows, float c,
    const int64_t* __restrict__ offsets, float4* __restrict__ segs, int64_t max_segs) {
  __shared__ uint32_t list_block[kWavesPerBlock][kList + 1];  // + a slot for discards
  const int r = wave_row();
  if (r >= rows) return;
  uint32_t* const list = list_block[threadIdx.x >> 6];
  const int j = r % (ny - 1);
  const RowPair rp(f0 + int64_t(r / (ny - 1)) * field_stride, nx, j);
  const int lane = threadIdx.x & 63;
  const uint64_t below_me = __lanemask_lt();
  constexpr uint32_t kDrop = 0x7ffffff0u;
  int64_t k = offsets[r];
  // every lane walks the same number of batches, so the ballots see the wave
  for (int i00 = 0; i00 < nx - 1; i00 += 64 * kUnroll) {
    Corners vs[kUnroll];
    rp.batch(i00, lane, nx, vs);
    uint32_t nb = 0;  // segments of the batch listed so far (wave-uniform)
    // entry: the cell's column within the batch, its case index, and
    // whether it is the cell's second segment
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
      const int di = 64 * q + lane;
      const int cs = case_index(vs[q], c);
      const int n = i00 + di < nx - 1 ? int((kSegCount >> (2 * cs)) & 3u) : 0;
      const uint64_t one = __ballot(n >= 1);
      const uint64_t two = __ballot(n >= 2);
      const uint32_t slot = nb + uint32_t(__popcll(one & below_me) + __popcll(two & below_me));
      const uint32_t e = (uint32_t(di) << 5) | (uint32_t(cs) << 1);
      list[n >= 1 ? slot : kList] = e;
      list[n >= 2 ? slot + 1 : kList] = e | 1u;
      nb += uint32_t(__popcll(one) + __popcll(two));
    }
    // the list is written and read by this wave only, in order
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t e0 = 0; e0 < nb; e0 += 64) {
      const uint32_t idx = e0 + uint32_t(lane);
      const bool ok = idx < nb;
      const uint32_t w = list[ok ? idx : kList];
      const int i = min(i00 + int(w >> 5), nx - 2);  // a discarded lane's column is clamped
      const Corners v = rp.at(i);
      int ea, eb;
      segment_edges(int((w >> 1) & 15u), (w & 1u) != 0, v, c, ea, eb);
      const float2 p = edge_point(ea, i, j, v.v00, v.v10, v.v11, v.v01, c);
      const float2 q2 = edge_point(eb, i, j, v.v00, v.v10, v.v11, v.v01, c);
      // this group's segments are [k + e0, k + e0 + 64), cut at max_segs
      const int64_t first = k + int64_t(e0);
      const int64_t room = max_segs - first;
      const uint32_t bytes = room <= 0 ? 0u : uint32_t(min(room, int64_t(64))) * 16u;
      const __amdgpu_buffer_rsrc_t out = __builtin_amdgcn_make_buffer_rsrc(
          segs + (room <= 0 ? 0 : first), 0, int(bytes), 0x00020000);
      typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
      const u32x4 val = {__float_as_uint(p.x), __float_as_uint(p.y), __float_as_uint(q2.x),
                         __float_as_uint(q2.y)};
      __builtin_amdgcn_raw_buffer_store_b128(val, out, int(ok ? uint32_t(lane) * 16u : kDrop), 0,
                                             0);
    }
    k += int64_t(nb);
    // the next batch rewrites the list only after these reads
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
