/*
 * pdiv.h -- C ABI of libpdiv, the gfx950 (MI355X) implementation of the
 * probabilistic local-divergence path of Ouermi et al., "Efficient
 * Probabilistic Visualization of Local Divergence of 2D Vector Fields with
 * Independent Gaussian Uncertainty".
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Grids are uniform with spacing dx, dy (Section 3).  A field is stored as
 *    row-major [ny][nx] planes with x (index i) fastest; U is the x component
 *    and V the y component of the vector field.  Cell (i, j), 0 <= i < nx-1,
 *    0 <= j < ny-1, has corners (i,j), (i+1,j), (i,j+1), (i+1,j+1).
 *  - LCP outputs are float32 planes [n_iso][ny-1][nx-1], one per isovalue,
 *    densely packed.
 *  - Pointers without a _host suffix are DEVICE pointers (hipMalloc'd or
 *    torch CUDA tensors) owned by the caller.  The core calls allocate
 *    nothing and keep no state between calls.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Every call is
 *    asynchronous on that stream: it validates its arguments, enqueues
 *    kernels and returns.  Host arrays (isovalues_host) are copied into
 *    kernel arguments before the call returns and may be reused at once.
 *  - Errors: every size and pointer argument is checked synchronously before
 *    anything is enqueued; a bad argument returns PDIV_ERR_INVALID and leaves
 *    the outputs untouched, with a message in pdiv_last_error().  A failed
 *    launch returns PDIV_ERR_DEVICE.  Faults inside kernels surface at the
 *    caller's next synchronisation, as with any HIP kernel.  Value
 *    preconditions (variances >= 0 and finite) are the caller's: NaN inputs
 *    give NaN outputs.  No C++ exception crosses this ABI.
 *  - The core calls are thread-safe.
 */
#ifndef PDIV_H_
#define PDIV_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pdiv_status {
  PDIV_OK = 0,
  PDIV_ERR_INVALID = 1,     /* bad argument; nothing was enqueued            */
  PDIV_ERR_UNSUPPORTED = 2, /* valid request the library cannot serve       */
  PDIV_ERR_NOMEM = 3,       /* an owned allocation (batch, server) failed    */
  PDIV_ERR_DEVICE = 4,      /* HIP runtime or launch error                   */
  PDIV_ERR_BUSY = 5,        /* server: admission refused (budget or queue)   */
  PDIV_ERR_TIMEOUT = 6      /* server: wait timed out                        */
} pdiv_status;

/* Storage type of the moment planes (mean and variance of U and V).  All
 * arithmetic is float32 whatever the storage type.  An int32_t rather than an
 * enum type, so that every value a caller passes is well defined on the
 * library's side; values other than these are rejected with
 * PDIV_ERR_INVALID. */
typedef int32_t pdiv_dtype;
enum { PDIV_F32 = 0, PDIV_F16 = 1, PDIV_BF16 = 2 };

/* Largest isovalue count one call accepts. */
#define PDIV_MAX_ISO 256

/* A hipStream_t, kept opaque so this header needs no HIP headers. */
typedef void* pdiv_stream;

/* ------------------------------------------------------------------------
 * Core calls
 * ------------------------------------------------------------------------ */

/* (a) Per-point Gaussian fit over ensemble members.
 *
 * Section 3 models each vector component at each grid point as an independent
 * Gaussian N(mu, sigma^2); Section 4 fits it over 15 (wind) and 20 (Red Sea)
 * ensemble members.  For every point p and component x in {U, V}:
 *     mean = (1/M) sum_m x_m(p),   var = sum_m (x_m(p) - mean)^2 / (M - ddof).
 * u_members, v_members: [n_members] planes of ny*nx values of in_dtype, plane
 *   m starting at element m*member_stride (member_stride = 0 means ny*nx;
 *   otherwise member_stride >= ny*nx).
 * ddof: 0 or 1 (1 = unbiased sample variance); n_members > ddof.
 * mean_u, var_u, mean_v, var_v: outputs, ny*nx values of out_dtype each.
 * Accumulation is float32 (streaming Welford); out_dtype rounds once at the
 * store (round to nearest even). */
pdiv_status pdiv_moments(const void* u_members, const void* v_members, pdiv_dtype in_dtype,
                         int64_t n_members, int64_t ny, int64_t nx, int64_t member_stride,
                         int32_t ddof, void* mean_u, void* var_u, void* mean_v, void* var_v,
                         pdiv_dtype out_dtype, pdiv_stream stream);

/* The Red Sea pre-stage (Section 4): for every member, the pixelwise gradient
 * of the velocity magnitude, gx = d|F|/dx and gy = d|F|/dy with |F| =
 * sqrt(u^2 + v^2), differenced like Eq. 1 (central inside, first-order
 * one-sided at the boundary; the paper does not state the scheme), then
 * fitted per point over the members like pdiv_moments: mean and variance of
 * gx and gy.  The gradient vectors are the field whose divergence
 * uncertainty the path analyses next (pass the four outputs to
 * pdiv_lcp_from_moments as mean_u, var_u, mean_v, var_v).  Fused: the
 * members' speeds and gradients never reach memory.  Arguments as in
 * pdiv_moments, plus the grid spacing dx, dy (finite, > 0); ny, nx >= 2. */
pdiv_status pdiv_speed_gradient_moments(const void* u_members, const void* v_members,
                                        pdiv_dtype in_dtype, int64_t n_members, int64_t ny,
                                        int64_t nx, int64_t member_stride, double dx, double dy,
                                        int32_t ddof, void* mean_gx, void* var_gx,
                                        void* mean_gy, void* var_gy, pdiv_dtype out_dtype,
                                        pdiv_stream stream);

/* (b) Divergence Gaussian at every vertex: Eq. 2 (mean) and Eq. 3 (variance)
 * of Section 3.1, from the finite-difference divergence of Eq. 1.  Interior
 * vertices use the central difference; at i = 0, i = nx-1, j = 0, j = ny-1 the
 * difference along that axis is the first-order forward/backward one,
 * e.g. mean_x = (mu^U(1,j) - mu^U(0,j))/dx, var_x = (var^U(1,j) + var^U(0,j))/dx^2.
 * Inputs: four [ny][nx] planes of in_dtype; dx, dy finite and > 0.
 * Outputs: div_mean, div_var, [ny][nx] float32. */
pdiv_status pdiv_divergence_gaussian(const void* mean_u, const void* var_u, const void* mean_v,
                                     const void* var_v, pdiv_dtype in_dtype, int64_t ny,
                                     int64_t nx, double dx, double dy, float* div_mean,
                                     float* div_var, pdiv_stream stream);

/* (c) Closed-form level-crossing probability (Section 3.1, the
 * independent-Gaussian LCP of Poethkow et al.): for every cell and isovalue c,
 *     LCP = 1 - prod_k P(X_k >= c) - prod_k P(X_k < c)
 * over the cell's four corners X_k ~ N(div_mean, div_var).  A corner with
 * variance 0 is deterministic and counts as above iff its mean >= c, so zero
 * variance gives the marching-squares crossing indicator.  Evaluated in
 * float32 with one Gaussian tail per corner and isovalue and a cancellation-
 * free combination, so cells near 0 and near 1 keep their relative accuracy.
 * div_mean, div_var: [ny][nx] float32; isovalues_host: n_iso floats in host
 * memory, 1 <= n_iso <= PDIV_MAX_ISO; lcp: n_iso maps of ny-1 rows of nx-1
 * float32 cells (device memory, 4-byte aligned like any float array; a
 * misaligned pointer is rejected), cell (q, j, i) at
 * lcp[q*plane_stride + j*row_pitch + i].
 * lcp_row_pitch: floats between rows (0: nx-1, dense; larger values pad the
 * rows, and padding is never written).  lcp_plane_stride: floats between maps
 * (0: (ny-1)*row_pitch); maps may also be interleaved by rows (plane stride
 * >= nx-1 and row pitch >= n_iso*plane stride, i.e. a [ny-1][n_iso][pitch]
 * buffer); layouts whose maps overlap are rejected.  When the row pitch and
 * plane stride are multiples of 32 floats and lcp is 128-byte aligned, every
 * store writes whole cache lines, which the kernel needs for its full write
 * bandwidth (on other rows the lines that neighbouring strips share are
 * completed in L2: 8192^2 dense maps at 16 isovalues take about 1.27x the
 * time); rows interleaved by isovalue write faster still on gfx950. */
pdiv_status pdiv_lcp(const float* div_mean, const float* div_var, int64_t ny, int64_t nx,
                     const float* isovalues_host, int32_t n_iso, float* lcp,
                     int64_t lcp_row_pitch, int64_t lcp_plane_stride, pdiv_stream stream);

/* Sampling modes of pdiv_mc_lcp. */
enum {
  PDIV_MC_VECTOR = 0, /* the paper's Monte Carlo: sample the vectors (Sections 3.2, 4)  */
  PDIV_MC_VERTEX = 1  /* test mode: sample each vertex divergence on its own            */
};

/* (d) Monte Carlo LCP, the paper's comparison (Sections 3.2 and 4): count
 * per cell and isovalue the samples whose four corner divergences are not
 * all on one side of c (>= counts as above); lcp = count / n_samples.
 *
 * mode PDIV_MC_VECTOR (the paper's): draw n_samples samples of the uncertain
 * vectors at every grid point and take the divergence of each sample by
 * Eq. 1 (one-sided at the boundary).  Sample s at point p = j*nx + i uses
 * Philox4x32-10 keyed by seed (low word, high word) at counter
 * (p, s/2, 0, 0); output words (w0, w1) feed a Box-Muller pair giving the U
 * and V normals of even s, (w2, w3) those of odd s.
 * U = mean_u + sqrt(var_u) * z, likewise V.
 *
 * mode PDIV_MC_VERTEX: draw every vertex divergence on its own from
 * N(mean, var) of Eq. 2-3 (as pdiv_divergence_gaussian computes them), so the
 * four corners of a cell are independent -- the closed form's model, to
 * which this mode converges on every cell, boundary cells included (the
 * vector mode shares grid points between neighbouring one-sided
 * differences there).  Sample s at vertex p uses counter (p, s/4, 1, 0);
 * Box-Muller on (w0, w1) gives the normals of samples 4q and 4q+1, on
 * (w2, w3) those of 4q+2 and 4q+3; value = mean + sqrt(var) * z.
 *
 * Requires ny*nx < 2^32 and 1 <= n_samples < 2^31; any other mode is
 * PDIV_ERR_INVALID.  Other arguments as in pdiv_divergence_gaussian and
 * pdiv_lcp; lcp is dense [n_iso][ny-1][nx-1]. */
pdiv_status pdiv_mc_lcp(const void* mean_u, const void* var_u, const void* mean_v,
                        const void* var_v, pdiv_dtype in_dtype, int64_t ny, int64_t nx,
                        double dx, double dy, const float* isovalues_host, int32_t n_iso,
                        int64_t n_samples, uint64_t seed, uint32_t mode, float* lcp,
                        pdiv_stream stream);

/* (b)+(c) fused: Eq. 2-3 and the closed-form LCP in one pass over the moment
 * planes; the divergence Gaussians never leave the chip.  Gives bitwise the
 * same LCP as pdiv_divergence_gaussian followed by pdiv_lcp; the output
 * layout (lcp_row_pitch, lcp_plane_stride) is that of pdiv_lcp. */
pdiv_status pdiv_lcp_from_moments(const void* mean_u, const void* var_u, const void* mean_v,
                                  const void* var_v, pdiv_dtype in_dtype, int64_t ny,
                                  int64_t nx, double dx, double dy,
                                  const float* isovalues_host, int32_t n_iso, float* lcp,
                                  int64_t lcp_row_pitch, int64_t lcp_plane_stride,
                                  pdiv_stream stream);

/* Diagnostic: sample s of the uncertain field exactly as pdiv_mc_lcp draws it
 * (same generator, counters and transform): u_s, v_s are [ny][nx] float32. */
pdiv_status pdiv_mc_sample_field(const void* mean_u, const void* var_u, const void* mean_v,
                                 const void* var_v, pdiv_dtype in_dtype, int64_t ny, int64_t nx,
                                 int64_t sample, uint64_t seed, float* u_s, float* v_s,
                                 pdiv_stream stream);

/* Isocontour geometry (Section 4's figures: the mean-field contour of the
 * divergence and the per-member contours of a spaghetti plot) by marching
 * squares; the paper does not state the extraction, the rules here are the
 * textbook ones: a corner is above iff its value >= isovalue; the case index
 * sums 1, 2, 4, 8 for the corners (i,j), (i+1,j), (i+1,j+1), (i,j+1) that
 * are above; a crossed edge from corner value p to q gets the point at
 * t = (isovalue - p) / (q - p) along it; the two saddle cases are split by
 * the cell centre ((v00 + v10) + (v11 + v01)) / 4 (the two corners on the
 * centre's side connect).  Segments (x0, y0, x1, y1) in grid units (x = i,
 * y = j) are listed cell by cell in row-major order, so the output is
 * deterministic.
 * field: [ny][nx] float32 (device).  row_offsets: ny int64 (device,
 * caller-allocated workspace and result): entry j < ny-1 receives the index
 * of cell row j's first segment, entry ny-1 the total count.  segments:
 * [max_segments][4] float32 (device, 16-byte aligned; may be NULL when
 * max_segments is 0);
 * segments past max_segments are not written, so a caller can size the
 * buffer from a first call with max_segments = 0.  A NaN isovalue or field
 * value never counts as above. */
pdiv_status pdiv_isocontour(const float* field, int64_t ny, int64_t nx, float isovalue,
                            int64_t* row_offsets, float* segments, int64_t max_segments,
                            pdiv_stream stream);

/* Spaghetti plot in one call: the divergence of every member by Eq. 1 (each
 * member a deterministic field; bitwise the mean of pdiv_divergence_gaussian
 * with zero variances) into div_workspace, then every member's isocontour
 * at isovalue, as pdiv_isocontour computes it.  u_members, v_members as in
 * pdiv_moments; div_workspace: n_members*ny*nx float32 (device, caller-
 * allocated); row_offsets: n_members*(ny-1) + 1 int64 (device): entry
 * m*(ny-1) + j receives the first segment of member m's cell row j, the last
 * entry the total, so member m's segments are
 * [row_offsets[m*(ny-1)], row_offsets[(m+1)*(ny-1)]); segments and
 * max_segments as in pdiv_isocontour.  n_members*ny*nx, with nx rounded up
 * to a multiple of 64, must be below 2^32 (one launch's thread count). */
pdiv_status pdiv_spaghetti(const void* u_members, const void* v_members, pdiv_dtype in_dtype,
                           int64_t n_members, int64_t ny, int64_t nx, int64_t member_stride,
                           double dx, double dy, float isovalue, float* div_workspace,
                           int64_t* row_offsets, float* segments, int64_t max_segments,
                           pdiv_stream stream);

/* pdiv_spaghetti for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no div_workspace argument.  The members' divergence planes go to a
 * workspace the library holds itself, a static device array of 2^24 floats
 * (64 MiB) on each GPU it runs on, kept until the process ends; the call
 * allocates nothing.  n_members*ny*nx must be at most 2^24 floats, else
 * PDIV_ERR_INVALID (nothing enqueued); the other arguments, checks and
 * results are those of pdiv_spaghetti, bit for bit.  Every call on one GPU
 * shares that GPU's workspace and leaves its contents there: calls whose
 * work overlaps on the device (issued on different streams, or from
 * different threads without ordering) race, so order them on one stream or
 * synchronise between them. */
pdiv_status pdiv_spaghetti_noalloc(const void* u_members, const void* v_members,
                                   pdiv_dtype in_dtype, int64_t n_members, int64_t ny,
                                   int64_t nx, int64_t member_stride, double dx, double dy,
                                   float isovalue, int64_t* row_offsets, float* segments,
                                   int64_t max_segments, pdiv_stream stream);

/* ------------------------------------------------------------------------
 * 3D vector fields, the extension the paper names as future work (Section 5).
 * Nothing in the method changes but the dimension: the divergence adds
 * dW/dz, differenced like the other two axes, and a cell is a hexahedron.
 * Grids are row-major [nz][ny][nx] (x fastest); 2 <= nz, ny <= 2^21,
 * 2 <= nx <= 2^29, at most 2^40 points; larger grids are PDIV_ERR_INVALID.
 * ------------------------------------------------------------------------ */

/* Eq. 2 and Eq. 3 with the z term at every vertex: mean = sum over the three
 * axes of the central difference of the axis's own component's means (step
 * 2h inside, first-order one-sided with step h on the two boundary planes of
 * that axis), variance = the sum of the squared weights times the neighbour
 * variances.  U, V, W are the x, y, z components; their six [nz][ny][nx]
 * planes are in_dtype (device); div_mean, div_var: [nz][ny][nx] float32
 * (device).  dx, dy, dz: finite and > 0. */
pdiv_status pdiv_divergence_gaussian_3d(const void* mean_u, const void* var_u,
                                        const void* mean_v, const void* var_v,
                                        const void* mean_w, const void* var_w,
                                        pdiv_dtype in_dtype, int64_t nz, int64_t ny, int64_t nx,
                                        double dx, double dy, double dz, float* div_mean,
                                        float* div_var, pdiv_stream stream);

/* Level-crossing probability of every hexahedral cell: the probability that
 * the c-isosurface passes through a cell whose 8 corners hold independent
 * Gaussians, 1 - prod_8 P(X >= c) - prod_8 P(X < c) (Section 3.1's formula
 * with 8 corners; >= counts as above; a zero-variance corner is
 * deterministic, so zero variance everywhere gives the marching-cubes
 * crossing indicator).  Evaluated in float32 with one Gaussian tail per
 * corner and isovalue and the cancellation-free pairwise combination.
 * div_mean, div_var: [nz][ny][nx] float32 (device); isovalues_host: n_iso
 * floats in host memory, 1 <= n_iso <= PDIV_MAX_ISO; lcp: n_iso maps of
 * float32 cells (device), cell (q, k, j, i) -- corners (i+a, j+b, k+c), a, b,
 * c in {0, 1} -- at lcp[q*plane_stride + (k*(ny-1) + j)*row_pitch + i].
 * lcp_row_pitch: floats between rows (0: nx-1, dense; larger values pad the
 * rows, and padding is never written); lcp_plane_stride: floats between maps
 * (0: (nz-1)*(ny-1)*row_pitch; smaller values are PDIV_ERR_INVALID).  Rows
 * that all start on 128-byte lines (lcp 128-byte aligned, row pitch and
 * plane stride multiples of 32) are written as whole lines, the fastest
 * layout on gfx950; every layout gives bitwise the same values.  A walk
 * reads up to 7 z slices from one 32-bit-addressed base, so 7*ny*nx*4 bytes
 * (2 bytes per element for 16-bit moments in the fused call) must stay
 * below 2^31; larger slices are PDIV_ERR_INVALID. */
pdiv_status pdiv_lcp_3d(const float* div_mean, const float* div_var, int64_t nz, int64_t ny,
                        int64_t nx, const float* isovalues_host, int32_t n_iso, float* lcp,
                        int64_t lcp_row_pitch, int64_t lcp_plane_stride, pdiv_stream stream);

/* The two 3D steps fused: Eq. 2-3 with the z term and the 8-corner LCP in
 * one pass over the six moment volumes (the divergence Gaussians never leave
 * the chip).  Gives bitwise the same maps as pdiv_divergence_gaussian_3d
 * followed by pdiv_lcp_3d.  Arguments as in those two calls. */
pdiv_status pdiv_lcp_3d_from_moments(const void* mean_u, const void* var_u, const void* mean_v,
                                     const void* var_v, const void* mean_w, const void* var_w,
                                     pdiv_dtype in_dtype, int64_t nz, int64_t ny, int64_t nx,
                                     double dx, double dy, double dz,
                                     const float* isovalues_host, int32_t n_iso, float* lcp,
                                     int64_t lcp_row_pitch, int64_t lcp_plane_stride,
                                     pdiv_stream stream);

/* ------------------------------------------------------------------------
 * Batched launch: many independent fields of uneven size, each with its own
 * isovalues, in ONE persistent kernel (fused Eq. 2-3 + closed-form LCP).
 * The paper's GPU run is dominated by launch overhead on a small field
 * (Section 4, Red Sea); a batch amortises one launch over all fields.
 * ------------------------------------------------------------------------ */

typedef struct pdiv_field {
  const void* mean_u;      /* [ny][nx] planes of the batch's dtype (device)       */
  const void* var_u;
  const void* mean_v;
  const void* var_v;
  int64_t ny, nx;          /* >= 2 each                                           */
  double dx, dy;           /* finite, > 0                                         */
  const float* isovalues;  /* n_iso float32 isovalues, DEVICE memory, read at each
                              launch (update them between launches to move a slider) */
  int32_t n_iso;           /* 1 .. 16                                             */
  float* lcp;              /* float32 output (device): n_iso planes of ny-1 rows  */
  int64_t lcp_row_pitch;   /* output layout as for pdiv_lcp: floats between rows */
  int64_t lcp_plane_stride;/* ... and between maps (0 = (ny-1)*row pitch)         */
} pdiv_field;

typedef struct pdiv_batch_s* pdiv_batch;

/* Flags for pdiv_batch_create. */
#define PDIV_BATCH_GRAPH 1u    /* capture the launch in a hipGraph, replay it     */
#define PDIV_BATCH_AUTOTUNE 2u /* time the candidate tile shapes on this batch and
                                  keep the fastest (cached per shape class)       */

/* Builds the tile table for fields_host[0..n) (host array, copied), uploads it,
 * and with PDIV_BATCH_GRAPH captures the launch on `stream`.  The batch owns
 * its device tables and graph; the fields' buffers stay the caller's and must
 * outlive the batch.  Returns PDIV_ERR_INVALID on a bad field, PDIV_ERR_NOMEM
 * if a table allocation fails. */
pdiv_status pdiv_batch_create(const pdiv_field* fields_host, int32_t n_fields, pdiv_dtype dtype,
                              uint32_t flags, pdiv_stream stream, pdiv_batch* out);
/* Enqueues one pass over every field of the batch on `stream`. */
pdiv_status pdiv_batch_launch(pdiv_batch batch, pdiv_stream stream);
/* Tile shape chosen for the batch: cell rows per band, cells per wave strip
 * (128: paired layout, for outputs whose rows all start on 128-byte lines;
 * 126: split layout) and the number of tiles. */
pdiv_status pdiv_batch_info(pdiv_batch batch, int32_t* band_rows, int32_t* strip_cells,
                            int64_t* n_tiles);
/* Releases the batch (synchronises its stream first). */
pdiv_status pdiv_batch_destroy(pdiv_batch batch);

/* ------------------------------------------------------------------------
 * Server: continuous batching of LCP requests over fields kept resident on
 * the device.  A worker thread admits requests as HBM budget and stream slots
 * free up, merges the isovalue-slider requests that are waiting into batched
 * launches, overlaps them on n_streams streams, and completes tickets from
 * device events.
 * ------------------------------------------------------------------------ */

typedef struct pdiv_server_s* pdiv_server;

typedef struct pdiv_server_stats_t {
  uint64_t done;            /* completed requests                                */
  uint64_t failed;          /* requests that ended with an error                 */
  uint64_t launches;        /* kernel launches issued for LCP requests           */
  double p50_us, p99_us;    /* latency, from the put_field / submit_lcp call to
                               the worker seeing the result on the device      */
  double p50_new_us, p99_new_us;       /* ... for new-field requests             */
  double p50_slider_us, p99_slider_us; /* ... for slider requests                */
  double lcp_cells;         /* LCP values produced                               */
  size_t resident_bytes;    /* device bytes held now (fields + in-flight scratch) */
  size_t peak_bytes;        /* high-water mark of resident_bytes                 */
} pdiv_server_stats_t;

/* hbm_budget: bytes the server may hold on the device (resident divergence
 * Gaussians, 8 B per point, plus staging of fields being uploaded).
 * n_streams: 1..8 compute streams.  Slider launches should not share a
 * hardware queue with the upload stream, or they wait behind its host-to-device
 * copies (milliseconds per large field): keep n_streams + 2 (the upload stream
 * and the application's own stream) within the device's hardware queues per
 * process (4 by default on ROCm; GPU_MAX_HW_QUEUES).  For tests of the
 * failure paths, the environment variable PDIV_FAULT=<point>:<n>[,...] read
 * here makes the n-th start of <point> (server_launch: a merged slider
 * launch; server_upload: a new field's upload) fail on the host before
 * anything is enqueued; the requests it carries finish with
 * PDIV_ERR_DEVICE. */
pdiv_status pdiv_server_create(size_t hbm_budget, int32_t n_streams, pdiv_server* out);
/* New field from host moment planes (pageable or pinned host memory, dtype as
 * given, [ny][nx] each): uploaded, reduced to its divergence Gaussians
 * (Eq. 2-3) and kept resident under id.  The host planes are copied (on
 * several threads for large fields) into pinned staging before the call
 * returns; the call waits while the staging pool is full.  Returns PDIV_ERR_BUSY if the field can never fit the budget;
 * otherwise the request waits for room (evicting least recently used fields
 * that no pending request names). */
pdiv_status pdiv_server_put_field(pdiv_server srv, uint64_t id, const void* mean_u_host,
                                  const void* var_u_host, const void* mean_v_host,
                                  const void* var_v_host, pdiv_dtype dtype, int64_t ny,
                                  int64_t nx, double dx, double dy, uint64_t* ticket);
/* Sizes the pinned host staging pool: makes sure it holds `count` free
 * buffers, each large enough for a new field of up to max_points points of
 * dtype, and touches their pages, so that pdiv_server_put_field reuses them
 * instead of allocating.  From then on the pool keeps to the bytes it holds
 * after this call (by default it grows to 2 GiB): a put_field that finds no
 * free buffer waits until an upload returns one; only a field larger than
 * every buffer, with none in use, allocates past that.  Returns
 * PDIV_ERR_NOMEM if pinned memory runs out. */
pdiv_status pdiv_server_reserve_staging(pdiv_server srv, int64_t max_points, pdiv_dtype dtype,
                                        int32_t count);
/* Slider request: LCP maps of resident field id at n_iso (1..16) isovalues
 * (host array, copied) into out, a device buffer of n_iso*(ny-1)*(nx-1) floats
 * that must stay valid until the ticket completes. */
pdiv_status pdiv_server_submit_lcp(pdiv_server srv, uint64_t id, const float* isovalues_host,
                                   int32_t n_iso, float* out, uint64_t* ticket);
/* Waits up to timeout_us (< 0: forever) for a ticket; *result receives the
 * request's own status.  Returns PDIV_ERR_TIMEOUT if it is still running. */
pdiv_status pdiv_server_wait(pdiv_server srv, uint64_t ticket, int64_t timeout_us,
                             pdiv_status* result);
pdiv_status pdiv_server_stats(pdiv_server srv, pdiv_server_stats_t* out);
/* Drains every pending request, then frees all device memory of the server. */
pdiv_status pdiv_server_destroy(pdiv_server srv);

/* ------------------------------------------------------------------------
 * Tuning
 * ------------------------------------------------------------------------ */
/* Cell rows per wave band of the closed-form LCP kernels (pdiv_lcp,
 * pdiv_lcp_from_moments), process-wide; 0 restores the built-in choice.
 * Results do not depend on it.  Returns PDIV_ERR_INVALID outside [0, 4096]. */
pdiv_status pdiv_set_lcp_band_rows(int32_t rows);

/* ------------------------------------------------------------------------
 * Checking modes (process-wide; for debugging, not for timing)
 * ------------------------------------------------------------------------ */
/* The fused float32 LCP kernel with rows on 128-byte lines fills each slot
 * of its LDS row ring with NaN before the row's loads are issued: a read
 * that ran ahead of its load would give NaN maps instead of stale values. */
#define PDIV_DEBUG_POISON_LDS 1u
/* Before any work, pdiv_divergence_gaussian, pdiv_lcp, pdiv_lcp_from_moments
 * and pdiv_mc_lcp scan their input planes on the device and return
 * PDIV_ERR_INVALID if a mean or a variance is not finite or a variance is
 * negative (the value preconditions that are otherwise the caller's).  The
 * scan waits for the stream, so these calls become synchronous.  Also set by
 * the environment variable PDIV_DEBUG_CHECKS=1 when the library loads. */
#define PDIV_DEBUG_CHECK_INPUTS 2u
/* Each core call writes one line (its name and sizes) to stderr.  Also set
 * by the environment variable PDIV_LOG=1 when the library loads. */
#define PDIV_DEBUG_LOG 4u
/* Sets the checking modes (an OR of PDIV_DEBUG_*; 0 switches all off).
 * Returns PDIV_ERR_INVALID for unknown bits. */
pdiv_status pdiv_set_debug(uint32_t flags);

/* ------------------------------------------------------------------------
 * Status
 * ------------------------------------------------------------------------ */
const char* pdiv_status_string(pdiv_status s);
/* Message of the last failing call on this thread ("" if none). */
const char* pdiv_last_error(void);
/* Library version, e.g. "0.1.0". */
const char* pdiv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PDIV_H_ */
