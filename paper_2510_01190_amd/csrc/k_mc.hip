// Monte Carlo level-crossing probability, the paper's comparison method
// (Sections 3.2 and 4): sample the uncertain vectors at every grid point,
// take each sample's divergence by Eq. 1, count per cell how often the
// isocontour crosses it.
//
// A workgroup owns a 32x32 tile of cells.  Per pair of samples it draws U and
// V at every grid point of the tile and its one-point halo (one Philox4x32-10
// call per point gives both samples of the pair), writes them to LDS, forms
// the divergence of both samples at the tile's 33x33 vertices, and tests the
// 32x32 cells against every isovalue, accumulating integer counts in
// registers.  Samples are regenerated from their counters, never stored, so
// neighbouring tiles see identical values at shared points.  This path is
// bound by vector ALU work (integer multiplies, transcendentals, compares),
// not by memory.
//
// Crossing test at 8 or 16 isovalues (ranked): with the isovalues in ascending
// order, a vertex's rank r(d) = #{q : c_q <= d} says that it is above exactly
// the isovalues q < r(d) (>= counts as above), so a cell is crossed exactly
// at the isovalues rmin <= q < rmax, rmin and rmax the smallest and largest
// rank of its corners.  Each vertex's rank comes from a branch-free binary
// search (log2 K LDS lookups in a breadth-first table, one compare with the
// largest isovalue); each cell's crossed set is the bit mask [rmin, rmax);
// the masks of 32/K cells share a 32-bit word and are counted in bit-sliced
// counters (bit plane b holds bit b of every count): a 4-plane counter takes
// each pair of samples with a handful of logic operations and is added into
// a 16-plane counter before it can overflow (every 7 pairs; every 6 in the
// vertex mode, which takes samples four at a time).  At 16 isovalues about a
// third of the instructions of 16 compares and a carry-add per isovalue and
// cell, for the same counts.  Both sampling modes use it; chunks of 1, 2 or
// 4 isovalues, chunks holding a NaN isovalue and runs of more than 65535
// samples take the direct test.
//
// Vertex-level sampling (PDIV_MC_VERTEX) draws each vertex divergence on its
// own from the Gaussian of Eq. 2-3 instead, so the four corners of every cell
// are independent -- the closed form's model, which it converges to on every
// cell, boundary cells included (where the paper's vector-level sampling
// shares grid points between the one-sided differences).
#include "mc_rank.hpp"
#include "pdiv_device.hpp"
#include "pdiv_internal.hpp"

namespace pdiv {
namespace {

constexpr int TX = 32, TY = 32;            // cells per tile
constexpr int VX = TX + 1, VY = TY + 1;    // vertices per tile
constexpr int PX = TX + 3, PY = TY + 3;    // grid points (vertices + halo)
constexpr int NP = PX * PY;
constexpr int NV = VX * VY;
constexpr int kBlock = 256;
constexpr int PPT = (NP + kBlock - 1) / kBlock;  // points per thread
constexpr int VPT = (NV + kBlock - 1) / kBlock;  // vertices per thread
constexpr int CPT = (TX * TY) / kBlock;          // cells per thread

// One sample value U = mu + sigma z, rounded twice (no contraction), as the
// float32 definition of the draw.
__device__ __forceinline__ float draw(float mu, float sd, float z) {
#pragma clang fp contract(off)
  return mu + sd * z;
}

// Eq. 1 for one sample from the U neighbours along x and V neighbours along y.
__device__ __forceinline__ float fd_div(float ul, float ur, float vl, float vr, float cxm,
                                        float cym) {
#pragma clang fp contract(off)
  return (ur - ul) * cxm + (vr - vl) * cym;
}

// #{q : c_q <= d} over the K sorted isovalues (0..K); NaN ranks 0, below
// every isovalue, as every >= comparison with it is false.  The walk keeps
// the node's byte offset a = 4i in the table (children at 2a and 2a + 4), so
// each level is one LDS read, a compare, a select and a shift-add.
template <int K>
__device__ __forceinline__ uint32_t rank_of(float d, const float* tree, float top) {
  const char* base = reinterpret_cast<const char*>(tree);
  uint32_t a = 4u;
#pragma unroll
  for (int k = 1; k < K; k *= 2) {
    const float t = *reinterpret_cast<const float*>(base + a);
    a = 2u * a + (d >= t ? 4u : 0u);
  }
  return (a >> 2) - uint32_t(K) + (d >= top ? 1u : 0u);
}

// RANK (8 or 16 isovalue slots, at most 65535 samples): the ranked crossing
// test; the divergence slots hold each vertex's rank instead of its value.
template <int KC, bool RANK, typename T>
__global__ __launch_bounds__(kBlock) void mc_kernel(const T* __restrict__ mu,
                                                    const T* __restrict__ vu,
                                                    const T* __restrict__ mv,
                                                    const T* __restrict__ vv, int ny, int nx,
                                                    StencilCoef k, IsoChunk iso, RankTable rt,
                                                    int n_store, int n_samples, uint32_t key0,
                                                    uint32_t key1, float* __restrict__ out,
                                                    int64_t plane) {
  static_assert(!RANK || KC == 8 || KC == 16, "the ranked test takes 8 or 16 slots");
  constexpr int kPer = 32 / KC;             // ranked: cells per counter word
  constexpr int kWords = RANK ? CPT / kPer : 1;
  __shared__ float sU[2][NP];
  __shared__ float sV[2][NP];
  __shared__ float sD[2][NV];
  __shared__ float sTree[16];

  const int tid = threadIdx.x;
  if (RANK && tid < KC) sTree[tid] = rt.tree[tid];  // read after the first barrier
  const int x0 = blockIdx.x * TX;
  const int y0 = blockIdx.y * TY;

  float pmu[PPT], psu[PPT], pmv[PPT], psv[PPT];
  uint32_t pid[PPT];
  bool pin[PPT];
#pragma unroll
  for (int m = 0; m < PPT; ++m) {
    const int p = tid + m * kBlock;
    const int gx = x0 - 1 + p % PX;
    const int gy = y0 - 1 + p / PX;
    pin[m] = (p < NP) & (gx >= 0) & (gx < nx) & (gy >= 0) & (gy < ny);
    pmu[m] = psu[m] = pmv[m] = psv[m] = 0.0f;
    pid[m] = 0;
    if (pin[m]) {
      const int64_t o = static_cast<int64_t>(gy) * nx + gx;
      pid[m] = static_cast<uint32_t>(o);
      pmu[m] = ld(mu, o);
      psu[m] = __fsqrt_rn(ld(vu, o));
      pmv[m] = ld(mv, o);
      psv[m] = __fsqrt_rn(ld(vv, o));
    }
  }

  constexpr int kCnt = RANK ? 1 : CPT;  // direct counters (unused when ranked)
  uint32_t cnt[kCnt][KC];
#pragma unroll
  for (int m = 0; m < kCnt; ++m)
#pragma unroll
    for (int q = 0; q < KC; ++q) cnt[m][q] = 0;
  Sliced sl[kWords];  // ranked: cell m in word m / kPer at bit (m % kPer) KC
#pragma unroll
  for (int w = 0; w < kWords; ++w) sliced_clear(sl[w]);

  const int n_pairs = (n_samples + 1) >> 1;
  for (int pr = 0; pr < n_pairs; ++pr) {
    // 1. draw both samples of the pair at every point of tile + halo
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
      if (pin[m]) {
        const int p = tid + m * kBlock;
        U4 c;
        c.x = pid[m];
        c.y = static_cast<uint32_t>(pr);
        c.z = 0u;
        c.w = 0u;
        const U4 w = philox4x32_10(c, key0, key1);
        const F2 z0 = box_muller(w.x, w.y);
        const F2 z1 = box_muller(w.z, w.w);
        sU[0][p] = draw(pmu[m], psu[m], z0.x);
        sV[0][p] = draw(pmv[m], psv[m], z0.y);
        sU[1][p] = draw(pmu[m], psu[m], z1.x);
        sV[1][p] = draw(pmv[m], psv[m], z1.y);
      }
    }
    __syncthreads();
    // 2. divergence of both samples at the tile's vertices (one-sided on the
    //    grid boundary, exactly as Eq. 1 is read for the closed form)
#pragma unroll
    for (int m = 0; m < VPT; ++m) {
      const int v = tid + m * kBlock;
      if (v < NV) {
        const int gx = x0 + v % VX;
        const int gy = y0 + v / VX;
        if (gx < nx && gy < ny) {
          const int xl = gx > 0 ? gx - 1 : 0;
          const int xr = gx < nx - 1 ? gx + 1 : nx - 1;
          const int yl = gy > 0 ? gy - 1 : 0;
          const int yr = gy < ny - 1 ? gy + 1 : ny - 1;
          const bool bx = (gx == 0) | (gx == nx - 1);
          const bool by = (gy == 0) | (gy == ny - 1);
          const float cxm = bx ? k.cxm_bd : k.cxm_in;
          const float cym = by ? k.cym_bd : k.cym_in;
          const int py = gy - (y0 - 1), px = gx - (x0 - 1);
          const int il = py * PX + (xl - (x0 - 1));
          const int ir = py * PX + (xr - (x0 - 1));
          const int jl = (yl - (y0 - 1)) * PX + px;
          const int jr = (yr - (y0 - 1)) * PX + px;
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const float d = fd_div(sU[s][il], sU[s][ir], sV[s][jl], sV[s][jr], cxm, cym);
            sD[s][v] = RANK ? __uint_as_float(rank_of<KC>(d, sTree, rt.tree[0])) : d;
          }
        }
      }
    }
    __syncthreads();
    // 3. crossing test per cell: not all four corners on one side (>= is above)
    if constexpr (RANK) {
      uint32_t word[2][kWords];
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int w = 0; w < kWords; ++w) word[s][w] = 0u;
#pragma unroll
      for (int m = 0; m < CPT; ++m) {
        const int cidx = tid + m * kBlock;
        const int cx = cidx % TX, cy = cidx / TX;
        if (x0 + cx < nx - 1 && y0 + cy < ny - 1) {
          const int v00 = cy * VX + cx;
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            if (2 * pr + s < n_samples) {
              const uint32_t mk = crossed_mask(
                  __float_as_uint(sD[s][v00]), __float_as_uint(sD[s][v00 + 1]),
                  __float_as_uint(sD[s][v00 + VX]), __float_as_uint(sD[s][v00 + VX + 1]));
              word[s][m / kPer] |= mk << (KC * (m % kPer));
            }
          }
        }
      }
#pragma unroll
      for (int w = 0; w < kWords; ++w) sliced_add2(sl[w], word[0][w], word[1][w]);
      if (pr % 7 == 6) {
#pragma unroll
        for (int w = 0; w < kWords; ++w) sliced_flush(sl[w]);
      }
    } else {
#pragma unroll
      for (int m = 0; m < CPT; ++m) {
        const int cidx = tid + m * kBlock;
        const int cx = cidx % TX, cy = cidx / TX;
        if (x0 + cx < nx - 1 && y0 + cy < ny - 1) {
          const int v00 = cy * VX + cx;
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            if (2 * pr + s < n_samples) {
              const float d0 = sD[s][v00], d1 = sD[s][v00 + 1];
              const float d2 = sD[s][v00 + VX], d3 = sD[s][v00 + VX + 1];
              const float lo = fminf(fminf(d0, d1), fminf(d2, d3));
              const float hi = fmaxf(fmaxf(d0, d1), fmaxf(d2, d3));
#pragma unroll
              for (int q = 0; q < KC; ++q)
                cnt[m][q] += static_cast<uint32_t>((lo < iso.c[q]) & (hi >= iso.c[q]));
            }
          }
        }
      }
    }
    __syncthreads();
  }

  const float fs = static_cast<float>(n_samples);
  if constexpr (RANK) {
#pragma unroll
    for (int w = 0; w < kWords; ++w) sliced_flush(sl[w]);
  }
#pragma unroll
  for (int m = 0; m < CPT; ++m) {
    const int cidx = tid + m * kBlock;
    const int gx = x0 + cidx % TX, gy = y0 + cidx / TX;
    if (gx < nx - 1 && gy < ny - 1) {
      float* o = out + static_cast<int64_t>(gy) * (nx - 1) + gx;
#pragma unroll
      for (int q = 0; q < KC; ++q) {
        if (q < n_store) {
          if constexpr (RANK)
            o[rt.perm[q] * plane] =
                static_cast<float>(sliced_count(sl[m / kPer], q + KC * (m % kPer))) / fs;
          else
            o[q * plane] = static_cast<float>(cnt[m][q]) / fs;
        }
      }
    }
  }
}

// Vertex-level sampling.  Each thread holds the divergence Gaussians of its
// vertices of the tile (Eq. 2-3 evaluated as in the closed-form path).  Per
// group of four samples one Philox4x32-10 call per vertex, at counter
// (vertex index, group, 1, 0), gives four normals by two Box-Muller pairs:
// (w0, w1) for samples 4g and 4g+1, (w2, w3) for 4g+2 and 4g+3.  RANK: the
// ranked crossing test of mc_kernel (the slots hold each vertex's rank).
template <int KC, bool RANK, typename T>
__global__ __launch_bounds__(kBlock) void mc_vertex_kernel(const T* __restrict__ mu,
                                                           const T* __restrict__ vu,
                                                           const T* __restrict__ mv,
                                                           const T* __restrict__ vv, int ny,
                                                           int nx, StencilCoef k, IsoChunk iso,
                                                           int n_store, int n_samples,
                                                           uint32_t key0, uint32_t key1,
                                                           RankTable rt,
                                                           float* __restrict__ out,
                                                           int64_t plane) {
  static_assert(!RANK || KC == 8 || KC == 16, "the ranked test takes 8 or 16 slots");
  constexpr int kPer = 32 / KC;
  constexpr int kWords = RANK ? CPT / kPer : 1;
  __shared__ float sD[4][NV];
  __shared__ float sTree[16];

  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * TX;
  const int y0 = blockIdx.y * TY;

  float dm[VPT], ds[VPT];
  uint32_t vid[VPT];
  bool vin[VPT];
#pragma unroll
  for (int m = 0; m < VPT; ++m) {
    const int v = tid + m * kBlock;
    const int gx = x0 + v % VX;
    const int gy = y0 + v / VX;
    vin[m] = (v < NV) & (gx < nx) & (gy < ny);
    dm[m] = ds[m] = 0.0f;
    vid[m] = 0;
    if (vin[m]) {
      const int xl = gx > 0 ? gx - 1 : 0;
      const int xr = gx < nx - 1 ? gx + 1 : nx - 1;
      const int yl = gy > 0 ? gy - 1 : 0;
      const int yr = gy < ny - 1 ? gy + 1 : ny - 1;
      const bool bx = (gx == 0) | (gx == nx - 1);
      const bool by = (gy == 0) | (gy == ny - 1);
      const int64_t row = static_cast<int64_t>(gy) * nx;
      const int64_t rl = static_cast<int64_t>(yl) * nx, rr = static_cast<int64_t>(yr) * nx;
      const DivGauss g =
          div_gauss(ld(mu, row + xl), ld(mu, row + xr), ld(vu, row + xl), ld(vu, row + xr),
                    ld(mv, rl + gx), ld(mv, rr + gx), ld(vv, rl + gx), ld(vv, rr + gx),
                    bx ? k.cxm_bd : k.cxm_in, bx ? k.cxv_bd : k.cxv_in,
                    by ? k.cym_bd : k.cym_in, by ? k.cyv_bd : k.cyv_in);
      dm[m] = g.mean;
      ds[m] = __fsqrt_rn(g.var);
      vid[m] = static_cast<uint32_t>(row + gx);
    }
  }

  constexpr int kCnt = RANK ? 1 : CPT;
  uint32_t cnt[kCnt][KC];
#pragma unroll
  for (int m = 0; m < kCnt; ++m)
#pragma unroll
    for (int q = 0; q < KC; ++q) cnt[m][q] = 0;
  Sliced sl[kWords];
#pragma unroll
  for (int w = 0; w < kWords; ++w) sliced_clear(sl[w]);
  if constexpr (RANK) {
    if (tid < KC) sTree[tid] = rt.tree[tid];
    __syncthreads();
  }

  const int n_groups = (n_samples + 3) >> 2;
  for (int gr = 0; gr < n_groups; ++gr) {
#pragma unroll
    for (int m = 0; m < VPT; ++m) {
      if (vin[m]) {
        const int v = tid + m * kBlock;
        U4 c;
        c.x = vid[m];
        c.y = static_cast<uint32_t>(gr);
        c.z = 1u;
        c.w = 0u;
        const U4 w = philox4x32_10(c, key0, key1);
        const F2 z01 = box_muller(w.x, w.y);
        const F2 z23 = box_muller(w.z, w.w);
        const float d[4] = {draw(dm[m], ds[m], z01.x), draw(dm[m], ds[m], z01.y),
                            draw(dm[m], ds[m], z23.x), draw(dm[m], ds[m], z23.y)};
#pragma unroll
        for (int s = 0; s < 4; ++s)
          sD[s][v] = RANK ? __uint_as_float(rank_of<KC>(d[s], sTree, rt.tree[0])) : d[s];
      }
    }
    __syncthreads();
    if constexpr (RANK) {
      uint32_t word[4][kWords];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int w = 0; w < kWords; ++w) word[s][w] = 0u;
#pragma unroll
      for (int m = 0; m < CPT; ++m) {
        const int cidx = tid + m * kBlock;
        const int cx = cidx % TX, cy = cidx / TX;
        if (x0 + cx < nx - 1 && y0 + cy < ny - 1) {
          const int v00 = cy * VX + cx;
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            if (4 * gr + s < n_samples) {
              const uint32_t mk = crossed_mask(
                  __float_as_uint(sD[s][v00]), __float_as_uint(sD[s][v00 + 1]),
                  __float_as_uint(sD[s][v00 + VX]), __float_as_uint(sD[s][v00 + VX + 1]));
              word[s][m / kPer] |= mk << (KC * (m % kPer));
            }
          }
        }
      }
      // two sample pairs per group: the 4-plane counter takes at most 7
      // pairs, so it is flushed after every third group (6 pairs)
#pragma unroll
      for (int w = 0; w < kWords; ++w) {
        sliced_add2(sl[w], word[0][w], word[1][w]);
        sliced_add2(sl[w], word[2][w], word[3][w]);
      }
      if (gr % 3 == 2) {
#pragma unroll
        for (int w = 0; w < kWords; ++w) sliced_flush(sl[w]);
      }
    } else {
#pragma unroll
      for (int m = 0; m < CPT; ++m) {
        const int cidx = tid + m * kBlock;
        const int cx = cidx % TX, cy = cidx / TX;
        if (x0 + cx < nx - 1 && y0 + cy < ny - 1) {
          const int v00 = cy * VX + cx;
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            if (4 * gr + s < n_samples) {
              const float d0 = sD[s][v00], d1 = sD[s][v00 + 1];
              const float d2 = sD[s][v00 + VX], d3 = sD[s][v00 + VX + 1];
              const float lo = fminf(fminf(d0, d1), fminf(d2, d3));
              const float hi = fmaxf(fmaxf(d0, d1), fmaxf(d2, d3));
#pragma unroll
              for (int q = 0; q < KC; ++q)
                cnt[m][q] += static_cast<uint32_t>((lo < iso.c[q]) & (hi >= iso.c[q]));
            }
          }
        }
      }
    }
    __syncthreads();
  }

  const float fs = static_cast<float>(n_samples);
  if constexpr (RANK) {
#pragma unroll
    for (int w = 0; w < kWords; ++w) sliced_flush(sl[w]);
  }
#pragma unroll
  for (int m = 0; m < CPT; ++m) {
    const int cidx = tid + m * kBlock;
    const int gx = x0 + cidx % TX, gy = y0 + cidx / TX;
    if (gx < nx - 1 && gy < ny - 1) {
      float* o = out + static_cast<int64_t>(gy) * (nx - 1) + gx;
#pragma unroll
      for (int q = 0; q < KC; ++q) {
        if (q < n_store) {
          if constexpr (RANK)
            o[rt.perm[q] * plane] =
                static_cast<float>(sliced_count(sl[m / kPer], q + KC * (m % kPer))) / fs;
          else
            o[q * plane] = static_cast<float>(cnt[m][q]) / fs;
        }
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void mc_sample_kernel(const T* __restrict__ mu,
                                                           const T* __restrict__ vu,
                                                           const T* __restrict__ mv,
                                                           const T* __restrict__ vv,
                                                           int64_t n, uint32_t pair, int odd,
                                                           uint32_t key0, uint32_t key1,
                                                           float* __restrict__ us,
                                                           float* __restrict__ vs) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (p >= n) return;
  U4 c;
  c.x = static_cast<uint32_t>(p);
  c.y = pair;
  c.z = 0u;
  c.w = 0u;
  const U4 w = philox4x32_10(c, key0, key1);
  const F2 z = odd ? box_muller(w.z, w.w) : box_muller(w.x, w.y);
  us[p] = draw(ld(mu, p), __fsqrt_rn(ld(vu, p)), z.x);
  vs[p] = draw(ld(mv, p), __fsqrt_rn(ld(vv, p)), z.y);
}

template <int KC, typename T>
hipError_t launch_kc(const void* mu, const void* vu, const void* mv, const void* vv, int ny,
                     int nx, const StencilCoef& k, const IsoChunk& iso, int kc, int n_samples,
                     uint64_t seed, bool vertex, float* out, hipStream_t s) {
  dim3 grid(static_cast<unsigned>(mc_tiles_x(nx)), static_cast<unsigned>(mc_tiles_y(ny)));
  const int64_t plane = static_cast<int64_t>(ny - 1) * (nx - 1);
  RankTable rt{};
  if constexpr (KC == 8 || KC == 16) {
    if (n_samples <= 65535 && rank_table(iso.c, kc, KC, &rt)) {
      if (vertex)
        hipLaunchKernelGGL((mc_vertex_kernel<KC, true, T>), grid, dim3(kBlock), 0, s,
                           static_cast<const T*>(mu), static_cast<const T*>(vu),
                           static_cast<const T*>(mv), static_cast<const T*>(vv), ny, nx, k, iso,
                           kc, n_samples, static_cast<uint32_t>(seed),
                           static_cast<uint32_t>(seed >> 32), rt, out, plane);
      else
        hipLaunchKernelGGL((mc_kernel<KC, true, T>), grid, dim3(kBlock), 0, s,
                           static_cast<const T*>(mu), static_cast<const T*>(vu),
                           static_cast<const T*>(mv), static_cast<const T*>(vv), ny, nx, k, iso,
                           rt, kc, n_samples, static_cast<uint32_t>(seed),
                           static_cast<uint32_t>(seed >> 32), out, plane);
      return hipGetLastError();
    }
  }
  if (vertex)
    hipLaunchKernelGGL((mc_vertex_kernel<KC, false, T>), grid, dim3(kBlock), 0, s,
                       static_cast<const T*>(mu), static_cast<const T*>(vu),
                       static_cast<const T*>(mv), static_cast<const T*>(vv), ny, nx, k, iso, kc,
                       n_samples, static_cast<uint32_t>(seed),
                       static_cast<uint32_t>(seed >> 32), rt, out, plane);
  else
    hipLaunchKernelGGL((mc_kernel<KC, false, T>), grid, dim3(kBlock), 0, s,
                       static_cast<const T*>(mu), static_cast<const T*>(vu),
                       static_cast<const T*>(mv), static_cast<const T*>(vv), ny, nx, k, iso, rt,
                       kc, n_samples, static_cast<uint32_t>(seed),
                       static_cast<uint32_t>(seed >> 32), out, plane);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_typed(const void* mu, const void* vu, const void* mv, const void* vv, int ny,
                        int nx, const StencilCoef& k, const IsoChunk& iso, int kc,
                        int n_samples, uint64_t seed, bool vertex, float* out, hipStream_t s) {
  // isovalue counts are bucketed to 1, 2, 4, 8, 16; the caller pads the
  // unused isovalue slots and only the first kc planes are stored
  const int kb = kc <= 1 ? 1 : kc <= 2 ? 2 : kc <= 4 ? 4 : kc <= 8 ? 8 : 16;
  switch (kb) {
    case 1: return launch_kc<1, T>(mu, vu, mv, vv, ny, nx, k, iso, kc, n_samples, seed, vertex, out, s);
    case 2: return launch_kc<2, T>(mu, vu, mv, vv, ny, nx, k, iso, kc, n_samples, seed, vertex, out, s);
    case 4: return launch_kc<4, T>(mu, vu, mv, vv, ny, nx, k, iso, kc, n_samples, seed, vertex, out, s);
    case 8: return launch_kc<8, T>(mu, vu, mv, vv, ny, nx, k, iso, kc, n_samples, seed, vertex, out, s);
    case 16: return launch_kc<16, T>(mu, vu, mv, vv, ny, nx, k, iso, kc, n_samples, seed, vertex, out, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

int64_t mc_tiles_x(int64_t nx) { return (nx - 1 + TX - 1) / TX; }
int64_t mc_tiles_y(int64_t ny) { return (ny - 1 + TY - 1) / TY; }

hipError_t launch_mc(const void* mu, const void* vu, const void* mv, const void* vv,
                     pdiv_dtype dt, int64_t ny, int64_t nx, const StencilCoef& k,
                     const IsoChunk& iso, int kc, int64_t n_samples, uint64_t seed,
                     uint32_t mode, float* lcp_k0, hipStream_t s) {
  const int iny = static_cast<int>(ny), inx = static_cast<int>(nx);
  const int ns = static_cast<int>(n_samples);
  const bool vx = mode == PDIV_MC_VERTEX;
  switch (dt) {
    case PDIV_F32: return launch_typed<float>(mu, vu, mv, vv, iny, inx, k, iso, kc, ns, seed, vx, lcp_k0, s);
    case PDIV_F16: return launch_typed<__half>(mu, vu, mv, vv, iny, inx, k, iso, kc, ns, seed, vx, lcp_k0, s);
    case PDIV_BF16: return launch_typed<bf16_t>(mu, vu, mv, vv, iny, inx, k, iso, kc, ns, seed, vx, lcp_k0, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_mc_sample(const void* mu, const void* vu, const void* mv, const void* vv,
                            pdiv_dtype dt, int64_t ny, int64_t nx, int64_t sample,
                            uint64_t seed, float* us, float* vs, hipStream_t s) {
  const int64_t n = ny * nx;
  if (!launch_fits((n + kBlock - 1) / kBlock, kBlock)) return hipErrorInvalidConfiguration;
  dim3 grid(static_cast<unsigned>((n + kBlock - 1) / kBlock));
  const uint32_t pair = static_cast<uint32_t>(sample >> 1);
  const int odd = static_cast<int>(sample & 1);
  const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
  switch (dt) {
    case PDIV_F32:
      hipLaunchKernelGGL(mc_sample_kernel<float>, grid, dim3(kBlock), 0, s,
                         static_cast<const float*>(mu), static_cast<const float*>(vu),
                         static_cast<const float*>(mv), static_cast<const float*>(vv), n, pair,
                         odd, k0, k1, us, vs);
      break;
    case PDIV_F16:
      hipLaunchKernelGGL(mc_sample_kernel<__half>, grid, dim3(kBlock), 0, s,
                         static_cast<const __half*>(mu), static_cast<const __half*>(vu),
                         static_cast<const __half*>(mv), static_cast<const __half*>(vv), n,
                         pair, odd, k0, k1, us, vs);
      break;
    case PDIV_BF16:
      hipLaunchKernelGGL(mc_sample_kernel<bf16_t>, grid, dim3(kBlock), 0, s,
                         static_cast<const bf16_t*>(mu), static_cast<const bf16_t*>(vu),
                         static_cast<const bf16_t*>(mv), static_cast<const bf16_t*>(vv), n,
                         pair, odd, k0, k1, us, vs);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pdiv
