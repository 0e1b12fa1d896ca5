/* cddt.h -- C ABI of libcddt: Compressed Directional Distance Transform ray
 * casting and the particle-filter beam sensor model on AMD Instinct MI355X.
 *
 * Method: Walsh & Karaman, "CDDT: Fast Approximate 2D Ray Casting for
 * Accelerated Localization".  Sec. III defines the ray cast on an occupancy
 * grid; Sec. IV defines the DDT/CDDT, its direct construction (Sec. IV-A),
 * the query (Sec. IV-B), the theta/theta+pi symmetry, edge map and overlap
 * check (Sec. IV-C) and the incremental obstacle update (Sec. IV-D); Sec. VI
 * uses the casts in a beam-model particle filter with 61 rays per particle.
 *
 * Conventions for every call:
 *  - Bulk arrays are DEVICE pointers unless the parameter name ends in _h
 *    (host memory).  The caller owns every buffer it passes in; the library
 *    owns the structure behind a cddt_map / cddt_plan / cddt_server.
 *  - Every call returns cddt_status: 0 on success, a negative code on failure.
 *    Nothing aborts and nothing throws across the ABI.  cddt_last_error()
 *    returns a thread-local message describing the last failure.
 *  - Argument validation happens on the host before any GPU work is queued:
 *    an invalid call returns CDDT_EINVAL and has no side effects.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls on a stream
 *    are asynchronous unless stated otherwise; outputs are valid once the
 *    stream reaches the call.  A cddt_map is not thread-safe: order all calls
 *    that use one map on one stream (or synchronise between streams).
 *  - Device data (poses, angles, observations) is never validated on the host;
 *    it has defined results instead (see cddt_cast).
 *
 * Numerical contract (bit-exact; the reading of the paper is fixed here):
 *  - Cells (i, j) cover [i, i+1) x [j, j+1); the grid is row-major occ[j*W+i];
 *    theta is measured from +x toward +y; lengths are in cells.
 *  - theta_bins = n bins over the full circle; the n/2 slices 0 <= s < n/2
 *    are stored and bin k >= n/2 is answered from slice k - n/2 by searching
 *    backwards (Sec. IV-C symmetry).
 *  - Direction table: C[s] = llround(cos(2 pi s/n) 2^30), S[s] likewise with
 *    sin, computed on the host in double.
 *  - Zero point of cell (i, j) in slice s: Z = ((2i+1) C + (2j+1) S) >> 15,
 *    the along-ray coordinate of the cell centre in units of 2^-16 cell.
 *    It is stored in every band r ("CDDT bin") that the rotated cell square's
 *    lateral extent [Yc - Hs, Yc + Hs) overlaps, with Yc = (2j+1) C - (2i+1) S,
 *    Hs = |C| + |S| (units 2^-31) and bands [r, r+1) half-open.
 *  - Query (x, y, theta), all float32: the answer is 0 if |theta| >= 1e6 or
 *    theta is not finite, if (x, y) is outside [0, W) x [0, H) or not finite,
 *    or if the cell under (x, y) is occupied (overlap check, full grid).
 *    Otherwise xf = floor(x 2^16), yf = floor(y 2^16), bin
 *    k = floor(fl(fl(theta * K) + 0.5f)) mod n with K = (float)(n / (2 pi))
 *    and no fused multiply-add, Xq = (xf C + yf S) >> 30,
 *    r = (yf C - xf S) >> 46.  For k < n/2 the answer uses the smallest zero
 *    point Z > Xq in band r, otherwise the largest Z < Xq; the range is
 *    min(max_range, (|Z - Xq| + 2^15) >> 16), or max_range when no such Z.
 *  - Construction uses the edge map (occupied cells with at least one free or
 *    off-map 8-neighbour) unless CDDT_FLAG_FULL_MAP is given.
 */
#ifndef CDDT_H
#define CDDT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cddt_status;
enum {
  CDDT_OK = 0,
  CDDT_EINVAL = -1,   /* invalid argument; nothing was done */
  CDDT_ENOMEM = -2,   /* device allocation failed or the structure exceeds 2^32 entries */
  CDDT_EDEVICE = -3,  /* a HIP runtime call failed; the message names it */
  CDDT_EBUSY = -4,    /* server admission refused (budget or slots exhausted) */
  CDDT_EINTERNAL = -5 /* consistency check failed inside the library */
};

/* Construction flags. */
enum {
  CDDT_FLAG_FULL_MAP = 1u << 0, /* project every occupied cell, not only the edge map */
  CDDT_FLAG_STATIC = 1u << 1,   /* no per-row slack: smallest structure, updates rebuild */
  CDDT_FLAG_BUCKETS = 1u << 2,  /* add the bucket index described below */
  CDDT_FLAG_ZP16 = 1u << 3,     /* 16-bit zero points in the bucket index (below) */
  CDDT_FLAG_PRUNE = 1u << 4     /* PCDDT: drop zero points no grid state returns (below) */
};
/* Bucket index (an addition to Sec. IV-A's bins, same results): every band
 * of every stored slice is cut into fixed-width buckets along the slice
 * direction, 2^k cells wide, starting at the lowest projection of the map
 * rectangle onto that slice.  Each bucket is one 128-byte line holding its
 * zero points, the last zero point before it and the first one after it, so
 * a band search reads one line, addressed from the band and the query's
 * projection alone (no header read).  A bucket with more than 30 zero points
 * sends its searches to the band's sorted search lines instead.  Costs
 * rows * buckets-per-band * 128 bytes, about 1.8 * (theta_bins / 2) *
 * width * height * 128 / 2^k bytes for a square map; kept current by
 * cddt_update.  k (4..10) goes in bits 8..11 of flags; 0 selects k = 7.
 * Narrower buckets hold fewer zero points, so fewer searches need more than
 * a line's first half (on room/corridor floors about 2% at k = 6, 10% at
 * k = 7, 40% at k = 8) at twice the memory per step down in k. */
#define CDDT_BUCKET_LOG2(k) ((uint32_t)(k) << 8)
/* 16-bit zero points (Sec. IV-C suggests them at a small precision loss;
 * needs CDDT_FLAG_BUCKETS): the bucket lines hold each zero point as a 16-bit
 * index of its 1/8-cell bin (60 per line, so buckets can be twice as wide for
 * the same overflow rate), and every query answers as if each zero point Z of
 * slice s were the centre of its bin, zlo + 8192 floor((Z - zlo) / 8192) +
 * 4096 (Q16), zlo = (min(0, W 2^16 C) + min(0, H 2^16 S)) >> 30.  Ranges then
 * differ from the exact ones by at most one cell except for rays that start
 * within about 1/8 cell of a zero point of their band.  cddt_export still
 * returns the exact zero points. */
/* PCDDT (Sec. IV-C, pruning; needs CDDT_FLAG_STATIC, not with
 * CDDT_FLAG_ZP16): after construction one cast is made from every discrete
 * state, the centre (i + 1/2, j + 1/2) of every free cell under every theta
 * bin, and each band keeps only the distinct zero points some state returned
 * (30-40% fewer on room maps).  Casts from those states (and from those
 * centres at any theta) return exactly what the full structure returns; other
 * queries may see past a dropped zero point.  cddt_update applies the ops to
 * the grid and rebuilds and prunes the whole structure; cddt_export returns
 * the pruned bands. */

/* Device memory for the structure.  alloc returns a device pointer of at
 * least `bytes` bytes (NULL on failure); free releases it.  Both are called
 * from the thread that calls into the library.  NULL allocator -> hipMalloc. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} cddt_allocator;

typedef struct cddt_map_s* cddt_map;

typedef struct {
  int32_t width, height, theta_bins, slices;
  uint32_t flags, reserved;
  int64_t rows;          /* bands over all stored slices */
  int64_t edge_cells;    /* cells projected (edge map, or all occupied cells) */
  int64_t zero_points;   /* stored zero points (sum of row lengths) */
  int64_t capacity;      /* allocated zero-point slots (>= zero_points; slack for updates) */
  int64_t max_row_len;
  int64_t device_bytes;  /* bytes the map holds on the device (bucket index included) */
  int64_t rebuilds;      /* updates that overflowed a row and re-laid the structure */
  int64_t bucket_lines;  /* lines of the bucket index (0 without CDDT_FLAG_BUCKETS) */
  int64_t bucket_overflow; /* buckets whose searches use the band's search lines */
  int32_t bucket_log2;   /* bucket width 2^k cells (0 without the index) */
  int32_t reserved2;
} cddt_stats;

/* Build a CDDT from an occupancy grid (Sec. IV-A: erosion to the edge map,
 * projection of every edge cell into every stored slice, per-band sort).
 *   occ        device, W*H bytes, row-major occ[j*W + i], nonzero = occupied;
 *              copied into the map (the caller may free it after the call).
 *   width,height  1..16384.   theta_bins  even, 2..8192.
 *   flags      CDDT_FLAG_*.   alloc  nullable (hipMalloc).
 * Blocks until the structure is built (sizes are read back to allocate).
 * Errors: EINVAL (arguments), ENOMEM, EDEVICE. */
cddt_status cddt_create(const uint8_t* occ, int32_t width, int32_t height, int32_t theta_bins,
                        uint32_t flags, const cddt_allocator* alloc, void* stream,
                        cddt_map* out_h);

/* Wait for the map's outstanding work and release it.  NULL is accepted. */
cddt_status cddt_destroy(cddt_map m);

/* Incremental obstacle update (Sec. IV-D).  Op k sets cell (xs_h[k], ys_h[k])
 * to occupied if values_h[k] != 0, else free; ops apply in array order, so
 * the last write to a cell wins.  Cells within one step of a changed cell are
 * re-classified against the edge map and their zero points removed from or
 * inserted into every slice and band they cover, so the structure afterwards
 * equals cddt_create on the new grid (same rows as multisets).  A row that
 * runs out of slack moves to a spare area at the end of the structure; only
 * when that is used up is the whole structure rebuilt.
 *   xs_h, ys_h, values_h  host arrays of n_ops (n_ops >= 0).
 * Blocks until applied.  Errors: EINVAL if any op is off the map (none is
 * applied), ENOMEM, EDEVICE. */
cddt_status cddt_update(cddt_map m, const int32_t* xs_h, const int32_t* ys_h,
                        const uint8_t* values_h, int64_t n_ops, void* stream);

/* Ray casts (Sec. IV-B query, Sec. IV-C symmetry and overlap check).
 *   x, y, theta  device float32[n] (structure of arrays).
 *   max_range    0..65535.   ranges_out  device int32[n].
 * n = 0 is a no-op.  Asynchronous. */
cddt_status cddt_cast(cddt_map m, const float* x, const float* y, const float* theta, int64_t n,
                      int32_t max_range, int32_t* ranges_out, void* stream);

/* Beam-model sensor weights (Sec. VI): for each particle p,
 *   logw_out[p] = sum_r log_table[clamp(obs_ranges[r], 0, M) * (M + 1) + d_pr]
 * where d_pr = cast(px[p], py[p], fl(ptheta[p] + ray_offsets[r])) with max
 * range M.  The sum is float32 in a fixed order that depends only on n_rays.
 *   px, py, ptheta  device float32[n_particles].
 *   ray_offsets     device float32[n_rays], 1 <= n_rays <= 1024.
 *   obs_ranges      device int32[n_rays].
 *   log_table       device float32[(M+1)*(M+1)], row-major [observed][expected].
 *   pair_offset     0, or P such that rays r and r+P point in opposite
 *                   directions: when their bins fall in the same slice, one
 *                   search answers both (Sec. IV-C radial pairing).  Results
 *                   do not depend on it.  See cddt_pair_offset.
 *   logw_out        device float32[n_particles].
 *   ranges_out      nullable device int32[n_particles * n_rays], [p][r].
 * Asynchronous. */
cddt_status cddt_weight(cddt_map m, const float* px, const float* py, const float* ptheta,
                        int64_t n_particles, const float* ray_offsets, int32_t n_rays,
                        int32_t pair_offset, const int32_t* obs_ranges, const float* log_table,
                        int32_t max_range, float* logw_out, int32_t* ranges_out, void* stream);

/* Helper for cddt_weight: the offset P (1 <= P < n_rays) that pairs the most
 * rays r, r+P whose bearings differ by pi (within 1e-4 rad), or 0.
 *   offsets_h  host float32[n_rays].  Returns the offset (>= 0). */
int32_t cddt_pair_offset(const float* offsets_h, int32_t n_rays);

/* Structure facts.  out_h: host.  Errors: EINVAL. */
cddt_status cddt_info(cddt_map m, cddt_stats* out_h);

/* The per-slice tables (host arrays of theta_bins/2 entries each): direction
 * C, S (2^30 fixed point), lowest band index, band count, and K. */
cddt_status cddt_slice_table(cddt_map m, int32_t* c_h, int32_t* s_h, int32_t* row_min_h,
                             int32_t* nrows_h, float* k_scale_h);

/* Canonical copy of the structure (Sec. IV-A: per stored slice, per band,
 * the ascending zero points) as compressed rows with the slack removed:
 *   row_start_h  host int64[rows + 1]: offset of each band's first zero point
 *                in zeros_h, in (slice, band) order; row_start_h[rows] is the
 *                total (int64: a structure may hold more than 2^31 points);
 *   row_len_h    host int32[rows]: band lengths;
 *   zeros_h      host int32[zero_points]: all bands concatenated, each band
 *                ascending (duplicates kept).
 * Any of the three may be NULL.  Blocks.  Errors: EINVAL, EDEVICE. */
cddt_status cddt_export(cddt_map m, int64_t* row_start_h, int32_t* row_len_h, int32_t* zeros_h);

/* Current occupancy grid (host uint8[W*H]).  Blocks. */
cddt_status cddt_export_grid(cddt_map m, uint8_t* occ_h);

/* The bucket index lines (inspection helper; the line format follows the
 * bucket index's description above): lines_h receives bucket_lines x 32
 * int32 (band r's bucket b at line r * buckets-per-band + b), n_ints must be
 * exactly that.  A map updated incrementally holds the same lines as a fresh
 * build of its grid.  Blocks.  Errors: EINVAL (NULL, no bucket index, wrong
 * size). */
cddt_status cddt_export_buckets(cddt_map m, int32_t* lines_h, int64_t n_ints);

/* ---------------------------------------------------------------------------
 * Many filters in one persistent launch.
 * A plan fixes a set of filters (each one cddt_weight call: its own map,
 * particles, rays, observations and table).  Running a plan launches one
 * persistent kernel whose waves pull tiles of particles from a device work
 * counter until all filters are done; results are bit-identical to one
 * cddt_weight per filter.  Running is capture-safe (kernel launches only, no
 * allocation, memset or synchronisation), so a run can be recorded into a
 * hipGraph and replayed each filter step with new data in the same buffers.
 * Maps of a plan may be updated between runs (cddt_update on the plan's
 * stream, or synchronised with it).  An update that re-lays a map's whole
 * structure (static and pruned maps, or a full spare area) moves its band
 * arrays; cddt_plan_run, cddt_plan_run_mcl, cddt_plan_replay, cddt_plan_time
 * and cddt_plan_run_plain notice this and upload the plan's descriptors again
 * on their stream before launching, so a captured graph keeps working (its
 * kernels read the descriptors from device memory).  Only the plan calls do
 * this: a graph replayed with hipGraphLaunch directly after such an update
 * reads freed memory.
 * ------------------------------------------------------------------------- */
typedef struct {
  cddt_map map;
  const float *px, *py, *ptheta;
  int64_t n_particles;
  const float* ray_offsets;
  int32_t n_rays;
  int32_t pair_offset;
  const int32_t* obs_ranges;
  const float* log_table;
  int32_t max_range;
  int32_t reserved;
  float* logw_out;
  int32_t* ranges_out; /* nullable */
} cddt_filter;

typedef struct {
  int32_t particles_per_tile; /* particles a wave takes per queue pop (1..256) */
  int32_t waves_per_block;    /* 1..8 */
  int32_t blocks_per_cu;      /* persistent blocks per compute unit (1..32) */
  int32_t search_mode;        /* 0: one lane per band search, one particle per wave at a time;
                                 1..5: eight lanes per search, this many searches per 8-lane
                                 group in flight; 6 / 7 / 8: one lane per search, the searches
                                 of 4 / 8 / 16 particles queued in LDS and drained together;
                                 9 / 10: as 7 / 8 with two searches per lane per round */
} cddt_tuning;

typedef struct cddt_plan_s* cddt_plan;

/* filters_h: host array of n_filters (1..65536) descriptors, copied.
 * tuning_h: nullable (library default).  Allocates the device descriptor
 * table and work counter; blocks until they are uploaded. */
cddt_status cddt_plan_create(const cddt_filter* filters_h, int32_t n_filters,
                             const cddt_tuning* tuning_h, void* stream, cddt_plan* out_h);
cddt_status cddt_plan_set_tuning(cddt_plan p, const cddt_tuning* tuning_h);
cddt_status cddt_plan_get_tuning(cddt_plan p, cddt_tuning* tuning_h);
/* One persistent launch (plus a one-thread counter reset kernel). */
cddt_status cddt_plan_run(cddt_plan p, void* stream);
/* Record one run into a hipGraph (replacing any previous one) / replay it. */
cddt_status cddt_plan_capture(cddt_plan p, void* stream);
cddt_status cddt_plan_replay(cddt_plan p, void* stream);
/* Run the plan with the given tuning `reps` times and return the mean kernel
 * milliseconds measured with HIP events on `stream` (used by the autotuner).
 * Blocks. */
cddt_status cddt_plan_time(cddt_plan p, const cddt_tuning* tuning_h, int32_t reps, void* stream,
                           float* ms_h);
/* The same filters as plain launches: one cddt_weight per filter, in order. */
cddt_status cddt_plan_run_plain(cddt_plan p, void* stream);
cddt_status cddt_plan_destroy(cddt_plan p);

/* Tunings found by an autotuner, kept in the library for the rest of the
 * process and keyed by a signature of the filter set (device, filter count,
 * particle total to the nearest power of two, the set of theta bin counts and
 * of structure layouts).  cddt_plan_create and cddt_batch_weight called
 * without a tuning use the tuning recorded for their filter set, else the
 * library default.  get returns that tuning and found_h = 1 if one was
 * recorded (found_h may be NULL).  Errors: EINVAL. */
cddt_status cddt_tuning_cache_put(const cddt_filter* filters_h, int32_t n_filters, const cddt_tuning* tuning_h);
cddt_status cddt_tuning_cache_get(const cddt_filter* filters_h, int32_t n_filters, cddt_tuning* tuning_h,
                                  int32_t* found_h);

/* The batched step in one call, without a plan: the sensor-model weights of
 * every filter (each the cddt_weight of Sec. VI's beam model over Sec. IV-B
 * casts) in one persistent launch, bit-identical to one cddt_weight per
 * filter and to a plan over the same filters and tuning.
 *   filters_h  host array of n_filters (1..65536) descriptors, read during
 *              the call only.
 *   tuning_h   nullable: NULL takes the tuning recorded for this filter set
 *              by cddt_tuning_cache_put (the autotuner's), else the library
 *              default.
 * The descriptors reach the device as kernel arguments, so a call enqueues
 * kernel launches only (one short launch per 20 filters, then the persistent
 * kernel): no copy, no synchronisation, and no allocation once the stream's
 * workspace holds n_filters descriptors.  A call can therefore be captured
 * into a hipGraph; its replays use the descriptors of the capture (update a
 * map that re-lays its structure, then capture again).
 * Workspace: library-owned device memory per (device, stream), counters plus
 * 168 bytes per filter, grown to the next power of two of at least 64
 * filters by the first call that needs more; growing synchronises the stream
 * first and is refused (EINVAL) while the stream is capturing.  Calls on one
 * stream are ordered; calls on different streams have separate workspaces.
 * A graph captured before the stream's workspace grew must not be replayed.
 * Errors: EINVAL (filters, tuning, capture), ENOMEM, EDEVICE. */
cddt_status cddt_batch_weight(const cddt_filter* filters_h, int32_t n_filters, const cddt_tuning* tuning_h,
                              void* stream);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call as cddt_batch_weight, same arguments and bit-identical results, with
 * its workspace (tile counters, prefix sums, descriptors) in a fixed device
 * array of the library, about 170 KiB per device, held from the first call
 * on a device until the process ends.  The call allocates nothing and does
 * not synchronise.  n_filters at most 1024 (EINVAL beyond).  Every call on a
 * device shares that array: calls that overlap on one device (different
 * streams, or graphs replayed concurrently) race and give wrong results;
 * order them on one stream.  The array keeps the last call's contents; each
 * call rewrites all it reads (its first kernel clears the counters).
 * Errors: EINVAL (filters, tuning, more than 1024 filters), EDEVICE. */
cddt_status cddt_batch_weight_noalloc(const cddt_filter* filters_h, int32_t n_filters,
                                      const cddt_tuning* tuning_h, void* stream);

/* ---------------------------------------------------------------------------
 * The particle-filter steps around the sensor model.  The paper's Monte
 * Carlo localization update moves every particle by the odometry, weighs it
 * with the sensor model and resamples by the weights (Sec. I, Sec. VI) but
 * gives no formulas for the first and last step; the library fixes them:
 *
 *   motion     odometry (dx, dy, dtheta) in the robot frame, noise drawn by
 *              the caller; in double precision
 *                x' = ((x + cos(th) dx) - sin(th) dy) + ex
 *                y' = ((y + sin(th) dx) + cos(th) dy) + ey
 *                th' = (th + dtheta) + eth, wrapped to [-pi, pi)
 *              each rounded once to float32;
 *   resample   systematic resampling with one uniform draw u (32 bits): the
 *              integer weights q_k = floor(2^20 exp(l_k - max finite l))
 *              (0 for a non-finite l_k; all 1 if no l_k is finite), T = sum,
 *              s = floor((u >> 12) T / 2^20); particle k fills the output
 *              slots [a_k, a_(k+1)), a_k = ceil((n C_k - s) / T) clamped at 0,
 *              C_k = q_0 + ... + q_(k-1).  Copies keep source order.
 *
 * exp, sin and cos are evaluated by range reduction and Taylor series in a
 * fixed order of double operations, so results are reproducible bit for bit.
 * ------------------------------------------------------------------------- */

/* Move n particles in place.  px, py, ptheta: device float32[n];
 * noise: device float32[3n] = (ex[n], ey[n], eth[n]).  Asynchronous.
 * Errors: EINVAL. */
cddt_status cddt_motion(float* px, float* py, float* ptheta, int64_t n, float dx, float dy, float dtheta,
                        const float* noise, void* stream);

/* Systematic resampling of one filter (n <= 2^20).  logw: device float32[n];
 * px/py/ptheta in and *_out: device float32[n], not overlapping;
 * idx_out: device int32[n], the source particle of every output.  One
 * workgroup; asynchronous.  Errors: EINVAL. */
cddt_status cddt_resample(const float* logw, int64_t n, uint32_t u, const float* px, const float* py,
                          const float* ptheta, float* px_out, float* py_out, float* ptheta_out, int32_t* idx_out,
                          void* stream);

/* A whole filter step for every filter of a plan: motion, the batched
 * log-weights (written to each filter's logw_out) and resampling of each
 * filter's poses in place (every filter n <= 2^20).  The step's inputs are
 * device arrays the caller rewrites between steps: odom float32[3 F]
 * ((dx, dy, dtheta) per filter), u uint32[F], noise float32[3 P] (filter f's
 * (ex, ey, eth) blocks of n_f each, at 3 * (n_0 + ... + n_(f-1))), P = total
 * particles.  set_mcl stores the pointers (and allocates the plan's
 * resampling scratch on first use: 16 bytes per particle); it drops any
 * captured graph.  run_mcl enqueues the step; capture_mcl captures it into
 * the plan's graph (replayed with cddt_plan_replay).  Errors: EINVAL,
 * ENOMEM. */
cddt_status cddt_plan_set_mcl(cddt_plan p, const float* odom, const uint32_t* u, const float* noise);
cddt_status cddt_plan_run_mcl(cddt_plan p, void* stream);
cddt_status cddt_plan_capture_mcl(cddt_plan p, void* stream);

/* Number of compute units of the current device (for tuning spaces). */
int32_t cddt_device_cus(void);

/* ---------------------------------------------------------------------------
 * Measurement helpers for the paper's query-time benchmarks (Sec. VI: casts
 * from a uniformly spaced grid over the (x, y, theta) states and from uniformly
 * random states, reported per query) and its dense lookup-table comparator
 * (Sec. II-III: the range of every discrete state stored in a 3-D table).
 * ------------------------------------------------------------------------- */
/* Rate of the device's constant wall clock in kHz (0 if it cannot be read). */
int32_t cddt_device_clock_khz(void);
/* cddt_cast (same kernels, same ranges) that also writes, per ray, the
 * wall-clock ticks its wave spent from loading the ray to its result:
 * ticks_out device int32[n].  Errors as cddt_cast. */
cddt_status cddt_cast_timed(cddt_map m, const float* x, const float* y, const float* theta, int64_t n,
                            int32_t max_range, int32_t* ranges_out, int32_t* ticks_out, void* stream);
/* Dense table of m's casts: lut[(k * H + j) * W + i] = the cast from the centre
 * (i + 1/2, j + 1/2) of cell (i, j) at the bin centre angle (float)(2 pi k / n),
 * for every bin k < n (0 in occupied cells).  lut: caller-owned device
 * uint16[n * W * H] (n * W * H * 2 bytes).  Asynchronous.  Errors: EINVAL. */
cddt_status cddt_lut_build(cddt_map m, int32_t max_range, uint16_t* lut, void* stream);
/* Table lookups: each query gets the same guards as a cast (0 when theta is
 * not finite or |theta| >= 1e6, or (x, y) is off the W x H map), then the
 * entry of its cell (floor(x), floor(y)) and bin (the cast's theta binning).
 * ticks_out: nullable, as in cddt_cast_timed.  Asynchronous.  Errors: EINVAL. */
cddt_status cddt_lut_cast(const uint16_t* lut, int32_t width, int32_t height, int32_t theta_bins, const float* x,
                          const float* y, const float* theta, int64_t n, int32_t* ranges_out, int32_t* ticks_out,
                          void* stream);
/* The cell-walk comparator (Bresenham's line family, Sec. II; here the exact
 * traversal of Amanatides and Woo): from (x, y) along (cos theta, sin theta),
 * theta not binned, the cells in the order the exact ray enters them (ties
 * step in y) are read from m's occupancy grid until the first occupied one;
 * the range is its entry distance rounded half up and capped at max_range
 * (max_range when the ray leaves the map first), 0 under the cast's guards.
 * Double precision; sin and cos by range reduction and a Taylor series in a
 * fixed order of operations.  ticks_out nullable, as in cddt_cast_timed.
 * Asynchronous.  Errors: EINVAL. */
cddt_status cddt_march_cast(cddt_map m, const float* x, const float* y, const float* theta, int64_t n,
                            int32_t max_range, int32_t* ranges_out, int32_t* ticks_out, void* stream);

/* Measurement helper, not part of the method: the band search's memory access
 * pattern without the search.  Groups of 8 lanes read whole 128-byte lines
 * (16 bytes per lane) at hashed random line indices of `buf`, keeping `depth`
 * (1, 2, 4 or 8) independent lines in flight; blocks x 256 threads, each group
 * reading steps*depth lines.  The achieved line rate x 128 bytes is the
 * achievable random-gather bandwidth.
 *   buf   device, `bytes` bytes (a multiple of 128, < 2^39).
 *   sink  device int32[blocks * 256] (receives a checksum per thread).
 * Asynchronous.  Errors: EINVAL. */
cddt_status cddt_probe_gather(const void* buf, int64_t bytes, int32_t blocks, int32_t steps, int32_t depth,
                              uint32_t seed, int32_t* sink, void* stream);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching over resident maps.
 * A server keeps maps resident and accepts requests (one robot's particles
 * and one scan) from host threads, in one of two modes.  Results are
 * bit-identical to running each request alone in either.
 *
 * Lanes (resident = 0): a scheduler thread admits queued requests whenever a
 * batch slot and enough of the staging budget are free, packs every admitted
 * request into one persistent batched launch on one of `n_lanes` streams, and
 * keeps up to n_lanes batches in flight, so requests that arrive while others
 * run are admitted as slots and memory free up and their work overlaps on the
 * device.
 *
 * Resident (resident = 1): one persistent kernel stays on the device while
 * there is work and admits requests as they are published.  A request takes
 * one of `max_batch` ring slots (each budget_bytes / max_batch bytes of
 * pinned, device-mapped host memory for its inputs and log-weights; a request
 * that does not fit is refused with EBUSY, one that finds no free slot waits),
 * is written there by the submitting thread and published at once; the
 * kernel's waves take its tiles as they come, among every other request's,
 * and the last tile writes the request's completion word back to host memory.
 * No launch or copy happens per request.  A request's tiles hold the
 * tuning's particles_per_tile particles while the ring holds fewer tiles than
 * the kernel has waves, and four times as many (at most 256) beyond that,
 * which trades a little latency for throughput under load.  The kernel leaves
 * about a millisecond after the last request finished and is launched again
 * by the next one.  Takes search modes 0, 6, 7 and 8; n_lanes must be 1.
 * ------------------------------------------------------------------------- */
typedef struct cddt_server_s* cddt_server;

typedef struct {
  int64_t budget_bytes;     /* device staging budget for request inputs/outputs */
  int32_t n_lanes;          /* batches in flight (streams), 1..4 (HIP's hardware queues per
                               process); a lane's batch writes its results straight into
                               pinned host memory, so it uses no copy engine */
  int32_t max_batch;        /* requests per batch, 1..4096 (resident: ring slots, 1..65536) */
  int32_t max_rays;         /* rays per request, 1..1024 */
  int32_t resident;         /* 0: lanes of batches; 1: one resident kernel fed through a ring */
  cddt_tuning tuning;       /* persistent-kernel tuning for server batches */
} cddt_server_config;

typedef struct {
  int64_t submitted, completed, rejected;
  int64_t batches;          /* batches launched (resident: kernel launches) */
  int64_t rays;
  int64_t peak_bytes;       /* highest staging bytes in use */
  double busy_seconds;      /* wall time with at least one batch in flight */
  double device_seconds;    /* sum over batches of device time, input copy start to batch kernel end */
  double max_batch_seconds; /* the slowest batch's device time */
} cddt_server_stats;

/* maps_h: host array of n_maps resident maps (not owned).  Per map: its ray
 * layout (offsets float32[n_rays], pair offset), its log table (device
 * float32[(M+1)^2]) and max range.  offsets_h are host arrays, copied. */
cddt_status cddt_server_create(const cddt_map* maps_h, int32_t n_maps,
                               const float* const* offsets_h, const int32_t* n_rays_h,
                               const float* const* log_tables, const int32_t* max_range_h,
                               const cddt_server_config* config_h, cddt_server* out_h);
/* Queue one request (host memory, copied before return): particle poses
 * px/py/ptheta_h[n_particles], observations obs_h[n_rays of the map].
 * Returns the request id (>= 0) in *id_h.  EBUSY if the request alone
 * exceeds the budget; otherwise it waits in the queue until admitted. */
cddt_status cddt_server_submit(cddt_server s, int32_t map_index, const float* px_h,
                               const float* py_h, const float* ptheta_h, int32_t n_particles,
                               const int32_t* obs_h, int64_t* id_h);
/* Measurement helper (an open-loop load generator), not part of the method:
 * submits request i at_h[i] seconds after the call starts (offsets not
 * decreasing) from the calling thread, exactly as cddt_server_submit would,
 * and records that scheduled arrival as its submit time, so latency is
 * measured from the arrival even when a submission runs late.  Arrays are host arrays of n entries; request i reads
 * px_h[i], py_h[i], ptheta_h[i] (count_h[i] floats each) and obs_h[i].  Blocks
 * until the last request is submitted; ids_h[i] receives the id, or -1 if the
 * request was refused (EBUSY).  Errors: EINVAL (nothing submitted). */
cddt_status cddt_server_replay(cddt_server s, int32_t n, const int32_t* map_h, const int32_t* count_h,
                               const float* const* px_h, const float* const* py_h,
                               const float* const* ptheta_h, const int32_t* const* obs_h,
                               const double* at_h, int64_t* ids_h);
/* The same load generator with n_threads (1..16) submitting threads: thread k
 * (the caller for k = 0) submits the requests i with i mod n_threads == k, each
 * at its own arrival time, so arrivals faster than one thread can submit are
 * still offered on time.  cddt_server_replay is the one-thread case.  Errors:
 * EINVAL (nothing submitted). */
cddt_status cddt_server_replay_threads(cddt_server s, int32_t n_threads, int32_t n, const int32_t* map_h,
                                       const int32_t* count_h, const float* const* px_h,
                                       const float* const* py_h, const float* const* ptheta_h,
                                       const int32_t* const* obs_h, const double* at_h, int64_t* ids_h);
/* Non-blocking: 1 if the request finished (logw copied to logw_h, which must
 * hold n_particles floats, and the request released), 0 if not yet. */
cddt_status cddt_server_poll(cddt_server s, int64_t id, float* logw_h, int32_t* done_h);
/* Blocking form of poll. */
cddt_status cddt_server_wait(cddt_server s, int64_t id, float* logw_h);
/* Completion time of a finished request, seconds since server creation
 * (result visible on the host), and its submit time.  Kept for the 65536 most
 * recent completions (a fixed ring, so a long-running server holds bounded
 * memory); EINVAL for a request not finished or completed longer ago. */
cddt_status cddt_server_times(cddt_server s, int64_t id, double* submit_h, double* done_h);
cddt_status cddt_server_stats_get(cddt_server s, cddt_server_stats* out_h);
/* Seconds since server creation on the server's clock. */
double cddt_server_now(cddt_server s);
/* Drain in-flight work, stop the scheduler and release staging memory. */
cddt_status cddt_server_destroy(cddt_server s);

/* Thread-local description of the last error (never NULL). */
const char* cddt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CDDT_H */
