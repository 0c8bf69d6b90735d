// Shared by the batched launch and the server: the per-field descriptor the
// persistent kernel reads, and the host helpers that build and launch it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "pdiv_internal.hpp"

namespace pdiv {

// One field of a batch, as the persistent kernel reads it (scalar loads).
// Fused batches point p0..p3 at the moment planes (mean U, var U, mean V,
// var V); two-step batches point p0, p1 at the divergence mean and variance.
struct alignas(16) BatchField {
  const void* p0;
  const void* p1;
  const void* p2;
  const void* p3;
  float* lcp;          // [n_iso][ny-1] rows of pitch floats
  const float* iso;    // n_iso isovalues (device)
  int ny, nx;
  int n_iso;           // 1..16
  int n_strips;        // filled by fill_tiles
  int64_t plane;       // (ny-1) pitch
  int64_t pitch;       // output row pitch in floats, >= nx-1
  int64_t tile_begin;  // first global tile index of the field (fill_tiles)
  StencilCoef coef;
};

int iso_bucket(int n);
// Kernel for a batch: fused (moments of dtype dt) or two-step (float planes),
// paired or split tile layout.
const void* batch_kernel_ptr(bool fused, pdiv_dtype dt, int kc, bool paired);
// Every field's output rows start on 128-byte lines (the paired layout's need).
bool all_rows_on_lines(const std::vector<BatchField>& f);
// Sets n_strips and tile_begin for band_rows-row bands of the layout's strips;
// returns the tile count.
int64_t fill_tiles(std::vector<BatchField>& f, int band_rows, bool paired);
// Blocks of the kernel resident on the whole device at once.
int resident_blocks(const void* kernel);
hipError_t launch_batch(const void* kernel, const BatchField* dev_fields, int n_fields,
                        int64_t n_tiles, int band_rows, int grid, hipStream_t s);

}  // namespace pdiv
