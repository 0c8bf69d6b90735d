// Batched persistent launch: many independent fields of uneven size, each with
// its own isovalues, in one kernel launch.  The paper's GPU timing is
// dominated by launch overhead on a small field (Section 4, Red Sea); a batch
// pays one launch for all of them and keeps every CU busy across field
// boundaries.
//
// Every field is cut into the column-walking tiles of lcp_tile.hpp (126-cell
// strips x band_rows-row bands).  Tile counts are prefix-summed over the
// fields; a grid sized to the device's resident capacity walks the global tile
// index with a stride of the total wave count (static, deterministic, no
// counters to reset, so the launch can be captured and replayed as a graph).
// A wave finds its field by binary search over the prefix table with scalar
// loads.  Results are bitwise those of the single-field kernels: the same tile
// code computes every cell.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "batch_internal.hpp"
#include "lcp_tile.hpp"

namespace pdiv {

namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

template <int KC, bool FUSED, bool PAIRED, typename T>
__global__ __launch_bounds__(kBlock) void batch_kernel(const BatchField* __restrict__ fields,
                                                       int n_fields, int64_t n_tiles,
                                                       int band_rows) {
  // XCD-aware order, as in the single-field kernel: block b runs on XCD b % 8,
  // so renumber blocks to give each XCD a contiguous range of wave slots and
  // hence runs of neighbouring tiles (their output rows share cache lines).
  const int nb = gridDim.x, xcd = blockIdx.x % 8, q8 = nb / 8, r8 = nb % 8;
  const int blk = xcd * q8 + min(xcd, r8) + blockIdx.x / 8;
  const int64_t wave = __builtin_amdgcn_readfirstlane(blk * kWavesPerBlock + (threadIdx.x >> 6));
  const int64_t n_waves = int64_t(gridDim.x) * kWavesPerBlock;
  for (int64_t t = wave; t < n_tiles; t += n_waves) {
    // field of tile t: the last f with fields[f].tile_begin <= t
    int lo = 0, hi = n_fields - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (fields[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
    }
    const BatchField& F = fields[lo];
    const int64_t local = t - F.tile_begin;
    const int strip = static_cast<int>(local % F.n_strips);
    const int band = static_cast<int>(local / F.n_strips);
    IsoChunk iso;
#pragma unroll
    for (int q = 0; q < KC; ++q) iso.c[q] = F.iso[q < F.n_iso ? q : F.n_iso - 1];
    const int j0 = band * band_rows;
    lcp_tile<KC, FUSED, PAIRED>(static_cast<const T*>(F.p0), static_cast<const T*>(F.p1),
                        static_cast<const T*>(F.p2), static_cast<const T*>(F.p3), F.ny, F.nx,
                        F.coef, iso, F.n_iso, F.lcp, F.plane, F.pitch, strip, j0,
                        min(j0 + band_rows, F.ny - 1));
  }
}

template <bool FUSED, bool PAIRED, typename T>
const void* kernel_for(int kc) {
  switch (kc) {
    case 1: return reinterpret_cast<const void*>(&batch_kernel<1, FUSED, PAIRED, T>);
    case 2: return reinterpret_cast<const void*>(&batch_kernel<2, FUSED, PAIRED, T>);
    case 4: return reinterpret_cast<const void*>(&batch_kernel<4, FUSED, PAIRED, T>);
    case 8: return reinterpret_cast<const void*>(&batch_kernel<8, FUSED, PAIRED, T>);
    case 16: return reinterpret_cast<const void*>(&batch_kernel<16, FUSED, PAIRED, T>);
  }
  return nullptr;
}

template <bool PAIRED>
const void* kernel_for_dtype(bool fused, pdiv_dtype dt, int kc) {
  if (!fused) return kernel_for<false, PAIRED, float>(kc);
  switch (dt) {
    case PDIV_F32: return kernel_for<true, PAIRED, float>(kc);
    case PDIV_F16: return kernel_for<true, PAIRED, __half>(kc);
    case PDIV_BF16: return kernel_for<true, PAIRED, bf16_t>(kc);
  }
  return nullptr;
}

}  // namespace

int iso_bucket(int n) { return n <= 1 ? 1 : n <= 2 ? 2 : n <= 4 ? 4 : n <= 8 ? 8 : 16; }

const void* batch_kernel_ptr(bool fused, pdiv_dtype dt, int kc, bool paired) {
  return paired ? kernel_for_dtype<true>(fused, dt, kc) : kernel_for_dtype<false>(fused, dt, kc);
}

bool all_rows_on_lines(const std::vector<BatchField>& f) {
  for (auto& x : f)
    if (reinterpret_cast<uintptr_t>(x.lcp) % 128 != 0 || x.pitch % 32 != 0 || x.plane % 32 != 0)
      return false;
  return true;
}

int64_t fill_tiles(std::vector<BatchField>& f, int band_rows, bool paired) {
  const int cells = cells_per_wave(paired);
  int64_t t = 0;
  for (auto& x : f) {
    x.n_strips = static_cast<int>((x.nx - 1 + cells - 1) / cells);
    const int n_bands = (x.ny - 1 + band_rows - 1) / band_rows;
    x.tile_begin = t;
    t += int64_t(x.n_strips) * n_bands;
  }
  return t;
}

int resident_blocks(const void* kernel) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 1024;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return cus * per_cu;
}

hipError_t launch_batch(const void* kernel, const BatchField* dev_fields, int n_fields,
                        int64_t n_tiles, int band_rows, int grid, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  void* args[] = {const_cast<BatchField**>(&dev_fields), &n_fields, &n_tiles, &band_rows};
  return hipLaunchKernel(kernel, dim3(grid), dim3(kBlock), args, 0, s);
}

}  // namespace pdiv

// ---------------------------------------------------------------------------
// Host side of the pdiv_batch_* calls.
// ---------------------------------------------------------------------------
using namespace pdiv;

struct pdiv_batch_s {
  std::vector<BatchField> fields;
  BatchField* dev = nullptr;
  const void* kernel = nullptr;
  int64_t n_tiles = 0;
  int band_rows = 16;
  int grid = 1;
  bool paired = false;      // tile layout (paired needs every output row on a line)
  bool lines = false;       // every field's output rows start on 128-byte lines
  pdiv_dtype dtype = PDIV_F32;
  int kc = 1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;
  hipEvent_t done = nullptr;
};

namespace {

// Autotune cache: in memory for the process, and in a JSON file when
// PDIV_TUNE_CACHE names one.  Key: dtype, isovalue bucket, whether the
// outputs are line-aligned, and the size class (log2 of total cells, log2 of
// the mean field side).  Value: band rows, grid multiplier, tile layout.
struct Tune {
  int band_rows, grid_mult, paired;
};
std::mutex g_tune_mu;
std::map<std::string, Tune> g_tune;
bool g_tune_loaded = false;

std::string tune_key(pdiv_dtype dt, int kc, bool lines, const std::vector<BatchField>& f) {
  double cells = 0, side = 0;
  for (auto& x : f) {
    cells += double(x.ny - 1) * double(x.nx - 1);
    side += std::sqrt(double(x.ny) * double(x.nx));
  }
  side /= std::max<size_t>(1, f.size());
  std::ostringstream o;
  o << "gfx950/batch/dt" << int(dt) << "/k" << kc << "/l" << int(lines) << "/c"
    << int(std::log2(cells + 1)) << "/s" << int(std::log2(side + 1));
  return o.str();
}

void tune_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("PDIV_TUNE_CACHE");
  if (!path) return;
  std::ifstream in(path);
  std::string line;
  // one entry per line: "key": [band_rows, grid_mult, paired],
  while (std::getline(in, line)) {
    const size_t a = line.find('"'), b = line.find('"', a + 1), c = line.find('[', b);
    if (a == std::string::npos || b == std::string::npos || c == std::string::npos) continue;
    int br = 0, gm = 0, pr = 0;
    if (std::sscanf(line.c_str() + c, "[%d, %d, %d]", &br, &gm, &pr) == 3 && br > 0 && gm > 0 &&
        (pr == 0 || pr == 1))
      g_tune[line.substr(a + 1, b - a - 1)] = {br, gm, pr};
  }
}

void tune_save() {
  const char* path = std::getenv("PDIV_TUNE_CACHE");
  if (!path) return;
  std::ofstream out(path);
  out << "{\n";
  size_t i = 0;
  for (auto& e : g_tune)
    out << "  \"" << e.first << "\": [" << e.second.band_rows << ", " << e.second.grid_mult
        << ", " << e.second.paired << "]" << (++i < g_tune.size() ? "," : "") << "\n";
  out << "}\n";
}

pdiv_status upload(pdiv_batch b) {
  if (b->dev) {
    if (hipFree(b->dev) != hipSuccess) return PDIV_ERR_DEVICE;
    b->dev = nullptr;
  }
  const size_t bytes = sizeof(BatchField) * b->fields.size();
  if (hipMalloc(&b->dev, bytes) != hipSuccess) {
    b->dev = nullptr;
    (void)hipGetLastError();
    invalid("batch: cannot allocate the %zu-byte field table", bytes);
    return PDIV_ERR_NOMEM;
  }
  return device_status(hipMemcpy(b->dev, b->fields.data(), bytes, hipMemcpyHostToDevice),
                       "batch table upload");
}

void release(pdiv_batch b) {
  if (b->done) (void)hipEventSynchronize(b->done);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  if (b->done) (void)hipEventDestroy(b->done);
  if (b->dev) (void)hipFree(b->dev);
  delete b;
}

// Sets the batch's layout and band height and fills its tile table.
void shape(pdiv_batch b, bool paired, int band_rows) {
  b->paired = paired;
  b->kernel = batch_kernel_ptr(true, b->dtype, b->kc, paired);
  b->band_rows = band_rows;
  b->n_tiles = fill_tiles(b->fields, band_rows, paired);
}

// Times the candidate shapes on the batch itself (the launches write the
// batch's own outputs) and keeps the fastest: band rows x grid size, and both
// tile layouts when every output row starts on a line.
pdiv_status autotune(pdiv_batch b, hipStream_t s) {
  const std::string key = tune_key(b->dtype, b->kc, b->lines, b->fields);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_load();
    auto it = g_tune.find(key);
    if (it != g_tune.end() && (b->lines || !it->second.paired)) {
      shape(b, it->second.paired != 0, it->second.band_rows);
      b->grid = std::max(1, resident_blocks(b->kernel) * it->second.grid_mult / 2);
      return upload(b);
    }
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return device_status(hipGetLastError(), "autotune events");
  float best = 1e30f;
  Tune win{16, 2, 0};
  pdiv_status st = PDIV_OK;
  for (int paired = 0; paired <= (b->lines ? 1 : 0) && st == PDIV_OK; ++paired) {
    for (int br : {8, 16, 32, 64}) {
      shape(b, paired != 0, br);
      const int base = resident_blocks(b->kernel);
      if ((st = upload(b)) != PDIV_OK) break;
      for (int gm : {1, 2, 4}) {  // grid = gm/2 x resident capacity
        const int grid = std::max(1, base * gm / 2);
        hipError_t e = launch_batch(b->kernel, b->dev, int(b->fields.size()), b->n_tiles, br,
                                    grid, s);  // warm
        e = e != hipSuccess ? e : hipEventRecord(e0, s);
        for (int r = 0; r < 3 && e == hipSuccess; ++r)
          e = launch_batch(b->kernel, b->dev, int(b->fields.size()), b->n_tiles, br, grid, s);
        e = e != hipSuccess ? e : hipEventRecord(e1, s);
        e = e != hipSuccess ? e : hipEventSynchronize(e1);
        float ms = 0;
        e = e != hipSuccess ? e : hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          st = device_status(e, "autotune launch");
          break;
        }
        if (ms < best) {
          best = ms;
          win = {br, gm, paired};
        }
      }
      if (st != PDIV_OK) break;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != PDIV_OK) return st;
  shape(b, win.paired != 0, win.band_rows);
  b->grid = std::max(1, resident_blocks(b->kernel) * win.grid_mult / 2);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[key] = win;
    tune_save();
  }
  return upload(b);
}

}  // namespace

extern "C" {

pdiv_status pdiv_batch_create(const pdiv_field* fields_host, int32_t n_fields, pdiv_dtype dtype,
                              uint32_t flags, pdiv_stream stream, pdiv_batch* out) {
  g_last_error.clear();
  if (out == nullptr) return invalid("out is NULL");
  *out = nullptr;
  if (fields_host == nullptr) return invalid("fields_host is NULL");
  if (n_fields < 1 || n_fields > (1 << 24)) return invalid("n_fields must be in [1, 2^24]");
  if (dtype != PDIV_F32 && dtype != PDIV_F16 && dtype != PDIV_BF16)
    return invalid("unknown dtype %d", int(dtype));
  if (flags & ~(PDIV_BATCH_GRAPH | PDIV_BATCH_AUTOTUNE)) return invalid("unknown flags");
  std::vector<BatchField> fv(n_fields);
  int kc = 1;
  for (int32_t i = 0; i < n_fields; ++i) {
    const pdiv_field& f = fields_host[i];
    if (!f.mean_u || !f.var_u || !f.mean_v || !f.var_v || !f.isovalues || !f.lcp)
      return invalid("field %d: NULL pointer", i);
    if (f.ny < 2 || f.nx < 2 || f.ny > (int64_t(1) << 21) || f.nx > (int64_t(1) << 29))
      return invalid("field %d: bad grid %lld x %lld", i, (long long)f.ny, (long long)f.nx);
    if (!(std::isfinite(f.dx) && f.dx > 0) || !(std::isfinite(f.dy) && f.dy > 0))
      return invalid("field %d: dx and dy must be finite and > 0", i);
    if (f.n_iso < 1 || f.n_iso > kIsoChunk)
      return invalid("field %d: n_iso must be in [1, %d]", i, kIsoChunk);
    OutLayout lo;
    if (check_layout(f.lcp_row_pitch, f.lcp_plane_stride, f.ny, f.nx, f.n_iso, &lo) != PDIV_OK)
      return invalid("field %d: %s", i, std::string(pdiv_last_error()).c_str());
    BatchField& x = fv[i];
    x.p0 = f.mean_u;
    x.p1 = f.var_u;
    x.p2 = f.mean_v;
    x.p3 = f.var_v;
    x.lcp = f.lcp;
    x.iso = f.isovalues;
    x.ny = static_cast<int>(f.ny);
    x.nx = static_cast<int>(f.nx);
    x.n_iso = f.n_iso;
    x.pitch = lo.pitch;
    x.plane = lo.plane;
    x.coef = make_coef(f.dx, f.dy);
    kc = std::max(kc, iso_bucket(f.n_iso));
  }
  pdiv_batch b = new pdiv_batch_s();
  b->fields = std::move(fv);
  b->dtype = dtype;
  b->kc = kc;
  b->lines = all_rows_on_lines(b->fields);
  hipStream_t s = static_cast<hipStream_t>(stream);
  pdiv_status st = PDIV_OK;
  if (flags & PDIV_BATCH_AUTOTUNE) {
    st = autotune(b, s);
  } else {
    shape(b, b->lines && kc >= 8, 16);
    b->grid = resident_blocks(b->kernel);
    st = upload(b);
  }
  if (st == PDIV_OK && hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess)
    st = device_status(hipGetLastError(), "batch event");
  if (st == PDIV_OK && (flags & PDIV_BATCH_GRAPH)) {
    // capture on a private stream (default priority) so the caller's stream
    // is never in capture mode
    hipError_t e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    e = e != hipSuccess ? e : hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t le = launch_batch(b->kernel, b->dev, int(b->fields.size()), b->n_tiles,
                                   b->band_rows, b->grid, b->capture);
      e = hipStreamEndCapture(b->capture, &b->graph);
      if (le != hipSuccess) e = le;
    }
    e = e != hipSuccess ? e : hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) st = device_status(e, "batch graph capture");
  }
  if (st != PDIV_OK) {
    release(b);
    return st;
  }
  *out = b;
  return PDIV_OK;
}

pdiv_status pdiv_batch_launch(pdiv_batch b, pdiv_stream stream) {
  g_last_error.clear();
  if (b == nullptr) return invalid("batch is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = b->exec ? hipGraphLaunch(b->exec, s)
                         : launch_batch(b->kernel, b->dev, int(b->fields.size()), b->n_tiles,
                                        b->band_rows, b->grid, s);
  if (e == hipSuccess) e = hipEventRecord(b->done, s);
  return device_status(e, "batch launch");
}

pdiv_status pdiv_batch_info(pdiv_batch b, int32_t* band_rows, int32_t* strip_cells,
                            int64_t* n_tiles) {
  g_last_error.clear();
  if (b == nullptr) return invalid("batch is NULL");
  if (band_rows) *band_rows = b->band_rows;
  if (strip_cells) *strip_cells = cells_per_wave(b->paired);
  if (n_tiles) *n_tiles = b->n_tiles;
  return PDIV_OK;
}

pdiv_status pdiv_batch_destroy(pdiv_batch b) {
  g_last_error.clear();
  if (b == nullptr) return invalid("batch is NULL");
  release(b);
  return PDIV_OK;
}

}  // extern "C"
