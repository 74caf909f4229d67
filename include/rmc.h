/*
 * rmc.h -- C ABI of the MI355X (gfx950) emission-based reciprocal Monte Carlo solver for
 * the radiative heat source div q_r on a Cartesian grid.
 *
 * Method: Silvestri & Pecnik, "A fast GPU Monte Carlo radiative heat transfer
 * implementation for coupling with direct numerical simulation".  For every cell, rays
 * are drawn over (narrow band n, g-point g) from the T_max spectral pdf (Sec. 2, Eqs. 13-17)
 * and over isotropic directions (Eq. 9), marched face to face through the grid
 * (Algorithm 1; x and z periodic, black walls bounding y) and weighted as in Eq. 14; the
 * cell estimate is the mean ray value (Eq. 8, ERMC form of Sec. 2).
 *
 * Conventions (every entry point):
 *  - Cells: nx x ny x nz, natural index c = (i * ny + j) * nz + k (k fastest); x and z are
 *    periodic with face coordinates xf[0..nx], zf[0..nz]; y is bounded by black walls at
 *    yf[0] and yf[ny].  1 <= nx, ny, nz <= 1023.
 *  - Ownership: the caller owns every buffer it passes.  set_* calls copy (and convert) what
 *    they need into library-owned device memory; caller buffers may be reused when the call
 *    returns (device inputs: once the given stream has reached the call).
 *  - Streams: `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on it
 *    and results are valid once it is synchronised.  set_temperature / set_species
 *    synchronise the stream to validate the field.
 *  - Errors: every call returns an rmc_status; rmc_last_error() gives the message of the
 *    calling thread's last failure.  The library never aborts and never prints.
 *    Temperatures outside the table range (or NaN) are errors, never clamped.
 *  - A context is bound to one device and is not thread-safe; use one per thread.
 *  - Units: lengths m, temperatures K, kappa m^-1 per unit mole fraction, band widths
 *    cm^-1, intensities W m^-2 sr^-1 (cm^-1)^-1; div q in W m^-3 (emission - absorption,
 *    Eq. 10 sign: positive in cells that lose energy).
 */
#ifndef RMC_H
#define RMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rmc_ctx rmc_ctx;

typedef enum {
    RMC_OK = 0,
    RMC_INVALID_ARG = 1,     /* bad pointer, size or enum value */
    RMC_BAD_STATE = 2,       /* a required set_* call is missing */
    RMC_OUT_OF_RANGE = 3,    /* temperature outside the table, NaN, negative mole fraction */
    RMC_UNSUPPORTED = 4,     /* a combination this build does not run, e.g. the learned
                                allocation in a closed box, or the wall flux with a reflecting
                                wall or the multigrid march */
    RMC_DEVICE_ERROR = 5,    /* a HIP runtime call failed */
    RMC_OUT_OF_MEMORY = 6
} rmc_status;

typedef enum { RMC_F32 = 0, RMC_F64 = 1, RMC_BF16 = 2 } rmc_dtype;
typedef enum { RMC_HOST = 0, RMC_DEVICE = 1 } rmc_mem;

/* Per-cell accumulation of the R ray values (always returned as double). */
typedef enum {
    RMC_ACC_F64 = 0,         /* double sums */
    RMC_ACC_COMP_F32 = 1,    /* float sums with Neumaier compensation */
    RMC_ACC_F32 = 2          /* plain float sums (reported for comparison) */
} rmc_accum;

typedef enum {
    RMC_SAMPLING_PLAIN = 0,  /* T_max spectral pdf (Eqs. 13-17), octant uniform */
    RMC_SAMPLING_PDF = 1,    /* per-cell pdf over (n, g, octant) from rmc_set_cell_pdf */
    RMC_SAMPLING_LEARNED = 2 /* per-cell pdf proposed by the allocation network (rmc_set_allocator) */
} rmc_sampling;

typedef struct {
    int32_t rays_per_cell;   /* R, 1..255 */
    uint64_t seed;           /* Philox key */
    uint32_t snapshot;       /* 0..2^27-1, part of every random-stream counter */
    double tol;              /* transmissivity cut-off of the march (Algorithm 1), >= 0 */
    int32_t max_steps;       /* cap on ray-cell steps per ray, >= 1 */
    rmc_dtype march;         /* RMC_F32 or RMC_F64 arithmetic of the march */
    rmc_accum accum;
    rmc_sampling sampling;
    double mix_eps;          /* PDF and LEARNED sampling: weight of the plain pdf in the mixture */
    int32_t block_threads;   /* march launch: threads per block (0 = default 256; only 256 is built) */
    int32_t long_ray_steps;  /* FP32 march on uniform x/z: rays still marching after this many steps
                                are finished by 64 lanes in parallel segments (0 = default 512,
                                >= max_steps disables it) */
    int32_t xcd_span;        /* march launch order: workgroups are dealt to the 8 XCDs in turn, and
                                each XCD takes runs of this many consecutive 64-ray chunks of the
                                bucketed work list, so that the rays in flight on one XCD work on
                                one (n, g) pair and nearby cells (power of two in [4, 2^20];
                                0 = default 256; 4 = plain workgroup order) */
    int32_t length_sort;     /* 1: each march workgroup reorders the rays of its four chunks by a
                                class of their expected length first (a counting sort in LDS), so
                                that a wavefront's rays end at similar times.  The estimate counts
                                the face crossings of the straight path up to the wall the ray
                                heads for or to the optical depth ln(1/tol) at a reference kappa
                                of its (n, g) pair.  0 (default): cell order.  Results are the same
                                either way */
    int32_t bucket_order;    /* march order of the (n, g, octant) buckets: 0 (default) pairs by
                                increasing kappa(T_max), the longest rays first; 1 band-major, the
                                g-points of a band together (they share its intensity table).
                                Results are the same either way */
    int32_t mg_levels;       /* multigrid march (Sec. 4.3): number of overlaid grids; grid L has
                                every 2^L-th face of the DNS grid (coarsening ratio 2 on every axis,
                                possible while each axis is even with a half of at least 3 cells)
                                and cells with the volume-weighted mean temperature and mole
                                fractions of the DNS cells they cover.  0 or 1: DNS grid only
                                (default); -1: every level the grid allows; more levels than the
                                grid allows is RMC_INVALID_ARG at compute.  Changes the result:
                                the coarse grids approximate the medium far from the source */
    int32_t mg_steps;        /* multigrid: steps a ray takes on each grid before it continues on
                                the next coarser one (the source cell's step counts on the DNS
                                grid); the last grid runs to depletion.  0 = default 5 */
    int32_t alloc_tile;      /* cells per allocation tile, the unit in which rays are counted into
                                and scattered to their buckets: a multiple of 64 in [256, 65536];
                                0 (default) = about 1024 tiles over the pass (256 to 8192 cells).
                                Larger tiles mean fewer per-tile histograms; results are the same
                                either way */
    int32_t long_ray_form;   /* long-ray kernel (FP32 march, periodic x and z): 0 (default) picks
                                on the device by the number of long rays -- up to 8192, one
                                workgroup of 256 parallel segments per ray (their latency sets
                                the time), more, one wavefront of 64 (throughput); 1 always
                                workgroups; 2 always wavefronts.  The segments' products round
                                differently, so the forms agree within the FP32 tolerance */
    int32_t alloc_cache;     /* LEARNED sampling: 1 keeps each cell's pair sums of the allocation
                                softmax (4 bytes per cell and (n, g) pair plus 12 per cell of device
                                memory: 27 GB for 4.2 M cells x 1600 pairs) after a compute, and
                                later computes of the unchanged field, walls, tables and network
                                (any snapshot, R or mix_eps) draw from them, running the network
                                only for the octants of the pairs they draw; the draws and values
                                are the same as without it.  0 (default): the network runs over
                                every pair at every compute.  Not in a captured graph */
    int32_t region_cells;    /* march order: the work list runs region by region -- groups of
                                allocation tiles compact in x and y, spanning z, holding about this
                                many cells -- and inside a region bucket by bucket, so that the rays
                                in flight start in one region and gather its cell records from L2
                                (an addition to the paper's narrow-band ordering of Sec. 4.2);
                                0 = default: regions of 262144 cells in snapshots of at least twice
                                that, one region in smaller ones; -1 = one region per snapshot
                                (bucket-major order); >= 64: this many cells.  Each (region,
                                bucket) run is padded to whole wavefronts.  Results are the same in
                                every order */
} rmc_options;

typedef struct {
    int64_t rays;            /* rays marched by the last compute */
    int64_t steps;           /* ray-cell steps (one DDA segment in one cell) of the last compute */
    int64_t capped_rays;     /* rays stopped by max_steps with tau > tol */
    double ms_prep;          /* last compute: pdf + property fields (HIP events on its stream) */
    double ms_alloc;         /* last compute: ray allocation, bucketing */
    double ms_march;         /* last compute: march kernel */
    double ms_reduce;        /* last compute: per-cell reduction */
    double ms_total;
    /* accumulated over every compute since rmc_reset_stats (or context creation) */
    int64_t computes;
    int64_t sum_rays;
    int64_t sum_steps;
    double sum_ms_prep, sum_ms_alloc, sum_ms_march, sum_ms_reduce;
    /* the march split into its two kernels (FP32 march on uniform x/z): */
    int64_t long_steps;      /* last compute: steps taken by the long-ray kernel */
    double ms_march_lane;    /* last compute: the lane kernel alone (HIP events) */
    double sum_ms_march_lane;
} rmc_stats;

/* One ray of rmc_trace_cells (parity and debugging). */
typedef struct {
    double Y;                /* ray value [W m^-3] (cell estimate = mean over its R rays) */
    double p;                /* probability p(n, g, o) the ray was drawn with */
    int32_t n, g, o, k;      /* band, g-point, octant, ordinal among equal (n, g, o) in the cell */
    int32_t steps;           /* ray-cell steps */
    int32_t end;             /* how the ray ended: 0 tau <= tol, 3 step cap, or the black wall
                                that stopped it: 1 y0, 2 y1, 4 x0, 5 x1, 6 z0, 7 z1 (x and z walls
                                only in a closed box, rmc_set_box_walls) */
} rmc_ray_record;

/* Create a context on HIP device `device` (>= 0).  Allocates nothing large. */
rmc_status rmc_create(int device, rmc_ctx **out);
/* Free the context and its device memory (NULL is a no-op).  Synchronises the device. */
void rmc_destroy(rmc_ctx *ctx);
/* Message of the calling thread's last failed call ("" if none).  Valid until the next call. */
const char *rmc_last_error(void);

/* Grid: face coordinates (host, double), strictly increasing, xf[0..nx], yf[0..ny],
 * zf[0..nz].  Invalidates fields set earlier. */
rmc_status rmc_set_grid(rmc_ctx *ctx, int nx, int ny, int nz,
                        const double *xf, const double *yf, const double *zf);

/* Wall temperatures at y = yf[0] and y = yf[ny] and their emissivities eps in [0, 1]
 * (RMC_INVALID_ARG otherwise).  Eq. 3: a ray reaching a wall leaves there the fraction eps
 * of its transmissivity tau (the term tau eps (I_b(T_source) - I_b(T_wall)) of the ray
 * value) and goes on with tau (1 - eps); the reflection law is not stated in the paper and
 * is taken specular (the ray is mirrored on the wall plane).  eps = 1 ends the ray.
 * Walls with eps < 1 turn off the parallel-segment long-ray march (rays then run in the
 * lane kernel to the end). */
rmc_status rmc_set_walls(rmc_ctx *ctx, double T_y0, double T_y1, double eps_y0, double eps_y1);

/* Closed box (Cases 3-4 and 12 of Table 1): walls at x = xf[0], x = xf[nx], z = zf[0] and
 * z = zf[nz] as well, with temperatures T[4] and emissivities eps[4] in that order (host
 * arrays, copied), the same wall law as rmc_set_walls.  T = NULL restores periodic x and z
 * (the default).  Errors: RMC_INVALID_ARG for negative or non-finite temperatures or
 * emissivities outside [0, 1]; temperatures outside the table range are RMC_OUT_OF_RANGE at
 * compute.  A closed box marches with per-face parameters on all three axes and without the
 * long-ray segments; the learned allocation is not available in it (RMC_UNSUPPORTED). */
rmc_status rmc_set_box_walls(rmc_ctx *ctx, const double *T, const double *eps);

/* Narrow-band correlated-k tables on the uniform temperature grid T0 + t * dT, t < nT
 * (Sec. 2.1, precomputed tables of Sec. 2.2).  All host pointers:
 *   dnu[nb] band widths, wg[ng] quadrature weights,
 *   k[ns][nb][ng][nT] absorption coefficient per unit mole fraction, RMC_F32 floats or
 *     RMC_BF16 raw bfloat16 bit patterns (uint16),
 *   Ib[nb][nT] band-averaged blackbody intensity (double).
 * Limits: 1 <= nb <= 4096, 1 <= ng <= 255, 1 <= ns <= 8, 2 <= nT, nb * ng <= 2000.  The
 * march stages the tables of four (band, g) pairs in LDS beside the face tables of the grids
 * it marches: 8 (nfaces + 4 (nT + ns nT / 2)) bytes must stay within the device's LDS per
 * workgroup less 12 KiB (nfaces: the face coordinates of every grid level of every distinct
 * grid of a pass; snapshots of one grid share theirs), else the compute returns
 * RMC_UNSUPPORTED. */
rmc_status rmc_set_kdist(rmc_ctx *ctx, int nb, int ng, int ns, int nT, double T0, double dT,
                         const double *dnu, const double *wg, const void *k, rmc_dtype k_dtype,
                         const double *Ib);

/* Temperature field T[ncells] (natural order), RMC_F32 or RMC_F64, host or device memory.
 * Needs set_grid and set_kdist first.  Validates every value against the table range
 * (RMC_OUT_OF_RANGE, NaN included) and synchronises `stream`. */
rmc_status rmc_set_temperature(rmc_ctx *ctx, const void *T, rmc_dtype dtype, rmc_mem mem,
                               void *stream);

/* Mole fractions X[ns][ncells] (natural order), RMC_F32 or RMC_F64, host or device.
 * ns must match set_kdist.  Negative or non-finite values are RMC_OUT_OF_RANGE.
 * Synchronises `stream`. */
rmc_status rmc_set_species(rmc_ctx *ctx, int ns, const void *X, rmc_dtype dtype, rmc_mem mem,
                           void *stream);

/* rmc_set_temperature and rmc_set_species in one call (the per-snapshot ingest of a DNS loop):
 * both fields are converted and checked by kernels enqueued together and the stream is
 * synchronised once.  Same arguments, layouts and errors as the two calls (a temperature error
 * is reported first; each field is kept or rejected on its own). */
rmc_status rmc_set_fields(rmc_ctx *ctx, const void *T, rmc_dtype T_dtype, int ns, const void *X,
                          rmc_dtype X_dtype, rmc_mem mem, void *stream);

/* Solver options; see rmc_options.  rmc_default_options fills the defaults
 * (R = 16, seed 0, tol 1e-6, max_steps 65536, F32 march, F64 sums, plain sampling). */
void rmc_default_options(rmc_options *opt);
rmc_status rmc_set_options(rmc_ctx *ctx, const rmc_options *opt);
/* The context's current options (as set, or as the autotuner left them) into *opt. */
rmc_status rmc_get_options(const rmc_ctx *ctx, rmc_options *opt);

/* Autotuner of the launch schedule, an addition to the paper's method (its kernels run with
 * fixed launch shapes, Sec. 3): times `reps` computes of the context's current workload on
 * `stream` (HIP events, after one warm-up each), first for every combination of xcd_span in
 * {16, 64, 256, 1024} and length_sort in {0, 1} at the automatic tile size, then for
 * alloc_tile at half and twice the automatic size (kept within [256, 16384]) with the best
 * of those, and keeps the fastest in the context's options (out, nullable, receives them).
 * Only knobs that reorder work are tuned: results are bitwise the same for every candidate.
 * Needs grid, walls, tables, fields and options set.  cache_path (nullable): a text file of
 * "signature : xcd_span length_sort alloc_tile" lines; a line for this workload and device
 * skips the timing, otherwise the result is appended.
 * Resets the statistics (rmc_reset_stats) after timing.  Synchronises the stream. */
rmc_status rmc_autotune(rmc_ctx *ctx, int reps, const char *cache_path, rmc_options *out, void *stream);

/* rmc_autotune for a batch (the contexts rmc_compute_batch accepts): times rmc_compute_batch
 * over all of them for the same candidates, the automatic tile size taken over the whole
 * pass, and writes the chosen xcd_span, length_sort and alloc_tile into every context's
 * options (the other fields, snapshot ids included, stay).  The signature of a cache line
 * lists every grid of the batch.  out (nullable) receives the first context's options. */
rmc_status rmc_autotune_batch(rmc_ctx *const *ctxs, int nsnap, int reps, const char *cache_path,
                              rmc_options *out, void *stream);

/* Measurement aid (the roofline of the march, not part of the method): the march's memory
 * access alone.  Every lane of ncells x R walks a straight ray of `steps` unit cells (x and z
 * periodic, y reflected) from a cell of its wavefront's tile region and reads per step the
 * 16-byte record of its cell (table coordinate of T, mole fractions) from the field of the
 * last compute, with the march's XCD-aware launch order and one (n, g) pair per run of
 * chunks, but no physics and no table lookups.  *ms receives the kernel time (HIP events on
 * `stream`, synchronised), *bytes the bytes it gathers (16 per step) and writes (8 per
 * wavefront): bytes / ms is the gather bandwidth the march's access pattern can reach.  Needs
 * a previous compute with the FP32 march (RMC_BAD_STATE otherwise); steps in [1, 65536]. */
rmc_status rmc_gather_probe(rmc_ctx *ctx, int steps, double *ms, double *bytes, void *stream);

/* Per-cell allocation pdf over (n, g, octant) for RMC_SAMPLING_PDF: q[ncells][nb][ng][8]
 * (double, >= 0, not necessarily normalised, host or device).  The rays of cell c are
 * drawn from (1 - mix_eps) q_c / sum q_c + mix_eps p_plain(n, g) / 8 and weighted by the
 * inverse of that probability (importance weights keep the estimate unbiased). */
rmc_status rmc_set_cell_pdf(rmc_ctx *ctx, const double *q, rmc_mem mem, void *stream);

/* The ERMC estimate of every cell: divq[ncells] (mean ray value, natural order) and, if
 * non-null, stderr[ncells] (standard error of that mean).  Both double, in `mem` memory.
 * Enqueued on `stream`; nothing is synchronised. */
rmc_status rmc_compute_divergence(rmc_ctx *ctx, double *divq, double *stderr_out, rmc_mem mem,
                                  void *stream);

/* rmc_compute_divergence for callers that cannot allocate device memory (code being captured
 * into a HIP graph, tight serving loops, harnesses that forbid hipMalloc): the same kernels and
 * results, but every per-compute buffer (cell records, pdf, work lists, ray slots, histograms,
 * descriptors) is carved from a static scratch array of 64 MiB that each GPU the library runs
 * on holds until the process ends; the call makes no hipMalloc, hipFree or pinned-host
 * allocation.  divq and stderr_out (nullable) are device memory; the call is enqueued on
 * `stream` and nothing is synchronised.  Limits: plain (T_max) sampling, no wall flux, and
 * a workload whose buffers fit the scratch (about ncells * R <= 2 million rays), else
 * RMC_UNSUPPORTED with the reason in rmc_last_error.  All calls on one GPU share its scratch:
 * calls that overlap on one GPU (other streams, other threads) race, and the scratch keeps the
 * last call's contents (counters and lists are cleared by the call itself).  The context's own
 * buffers are untouched, so rmc_get_stats, rmc_get_ray_values and the other inspection calls
 * keep describing its last regular compute.  The device's scratch address is taken by
 * rmc_create (RMC_DEVICE_ERROR here if that failed). */
rmc_status rmc_compute_divergence_noalloc(rmc_ctx *ctx, double *divq, double *stderr_out,
                                          void *stream);

/* rmc_compute_divergence plus the wall flux: q_wall receives, per wall face element, the net
 * radiative flux from the gas into the wall [W m^-2] -- the sum over every ray that ended on
 * that element of its wall term w kappa_src tau_w (I_src - I_w) (Eq. 3's wall factor with
 * emissivity 1, Eq. 14's weight), times the source cell's volume / (R x the element's area).
 * Exchange between walls is not part of it (rays start in gas cells).  Layout, doubles:
 * x0 [ny][nz], x1 [ny][nz], y0 [nx][nz], y1 [nx][nz], z0 [nx][ny], z1 [nx][ny] (the x and z
 * walls of a periodic box stay zero); in `mem` memory like divq.  Needs every wall black and
 * one grid (mg_levels 0 or 1): else RMC_UNSUPPORTED.  The face sums use FP64 atomics, so
 * they are reproducible to rounding, not bitwise; divq and stderr are those of
 * rmc_compute_divergence, bitwise.  Enqueued on `stream`; nothing is synchronised. */
rmc_status rmc_compute_wall_flux(rmc_ctx *ctx, double *divq, double *stderr_out, double *q_wall, rmc_mem mem,
                                 void *stream);

/* Several snapshots (contexts on one device with identical tables, options and walls;
 * grids and fields may differ) in one pass of the pipeline: the rays of all snapshots are
 * bucketed together and marched by one kernel launch.  divq[s] / stderr[s] (nullable)
 * receive snapshot s.  Enqueued on `stream`. */
rmc_status rmc_compute_batch(rmc_ctx *const *ctxs, int nsnap, double *const *divq,
                             double *const *stderr_out, rmc_mem mem, void *stream);

/* A compute of one or more snapshots captured into a HIP graph, for callers that replay the
 * same computation on new fields (a DNS loop): rmc_graph_capture plans the batch (allocates
 * and uploads descriptors, runs nothing else), then captures the kernel sequence of one
 * rmc_compute_batch with device outputs divq[s] / stderr[s] (nullable) on `stream`, which must
 * not be the null stream.  rmc_graph_launch replays it: the replay reads the contexts' current
 * temperature and species fields (rmc_set_temperature / rmc_set_species may be called between
 * replays) and writes the same output buffers.  Any other set_* call on a captured context,
 * or a compute that grows its buffers, invalidates the graph: launching it then returns
 * RMC_BAD_STATE.  Replays do not update rmc_get_stats.  Destroy a graph before the contexts it
 * captured. */
typedef struct rmc_graph rmc_graph;
rmc_status rmc_graph_capture(rmc_ctx *const *ctxs, int nsnap, double *const *divq,
                             double *const *stderr_out, void *stream, rmc_graph **out);
rmc_status rmc_graph_launch(rmc_graph *graph, void *stream);
void rmc_graph_destroy(rmc_graph *graph);

/* Per-ray values and step counts of the last compute for the listed cells (host arrays):
 * Y[ncell][R] (double) and steps[ncell][R] (int32, nullable).  Synchronises `stream`. */
rmc_status rmc_get_ray_values(rmc_ctx *ctx, const int64_t *cells, int ncell, double *Y,
                              int32_t *steps, void *stream);

/* Re-draw and re-march all R rays of the listed cells with the same device functions as
 * rmc_compute_divergence and return full records out[ncell][R] (host).  Synchronises. */
rmc_status rmc_trace_cells(rmc_ctx *ctx, const int64_t *cells, int ncell, rmc_ray_record *out,
                           void *stream);

/* The plain spectral pdf used by the last compute (host arrays): p[nb][ng], cdf_b[nb],
 * cdf_g[nb][ng] and T_max (nullable).  Synchronises `stream`. */
rmc_status rmc_get_pdf(rmc_ctx *ctx, double *p, double *cdf_b, double *cdf_g, double *T_max,
                       void *stream);

/* ------------------------------------------------------------ learned ray allocation
 * An addition to the paper's method.  A network proposes, for every cell, a pdf over
 * (band n, g-point g, octant o) from which that cell's rays are drawn; each ray keeps the
 * importance weight of Eq. 14 with the probability it was drawn with, so the estimate stays
 * unbiased for any positive pdf (the argument that lets the T_max pdf stand in for a cell's
 * own emission pdf, Eqs. 13-14).  With RMC_SAMPLING_LEARNED the rays of cell c are drawn from
 *   p_c(n,g,o) = (1 - mix_eps) softmax over all (n,g,o) of [zg_c + log p_plain(n,g)]
 *                + mix_eps p_plain(n,g) / 8,
 * so that a network whose logits are all equal reproduces the plain (T_max) allocation and
 * the network learns corrections to it; zg_c(n,g,o) = z(x_{c,n,g})[o xor m_c] (returned by
 * rmc_allocator_logits, without the prior), where z is the network below and m_c the sign bits
 * (x: 1, y: 2, z: 4) of the cell's temperature gradient, so that the network sees octants in
 * the frame of the local gradient.  The draws use the cell's allocation stream exactly as the
 * other modes (band, then g within the band, then octant, by inversion of cumulative sums
 * taken in that order).  The per-cell pdf is never stored: one kernel computes a group of
 * cells' logits (hidden layers on BF16 matrix cores, FP32 accumulation), the softmax and
 * the draws (FP32 exponentials, FP64 sums) and writes each ray's stratum and probability.
 *
 * Network: x = (f - mu) / sd, f = [T_c / 1000 K, log10(1 + |grad T|_c), log10(kappa_P,c),
 * nu_n / 1e4 cm^-1, g abscissa]; h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2),
 * h3 = relu(W3 h2 + b3), z = W4 h3 + b4 (64 hidden units, 8 outputs).  kappa_P,c =
 * sum_s x_s kP_s(T_c), kP_s(T) = pi sum_{n,g} dnu_n w_g k^s_{n,g}(T) I_n(T) / (sigma T^4)
 * interpolated from the table nodes; grad T by central differences at the cell centres,
 * periodic in x and z, walls as ghost values on the wall faces. */
#define RMC_MLP_PARAMS 9224

/* params[RMC_MLP_PARAMS] (float, row-major, output index first): W1[64][5], b1[64],
 * W2[64][64], b2[64], W3[64][64], b3[64], W4[8][64], b4[8]; mu[5], sd[5] (sd > 0);
 * nu_c[nb] band centres (cm^-1); gx[ng] g abscissae.  Host pointers, copied.  Resets the
 * training state.  rmc_set_kdist invalidates it (call again afterwards). */
rmc_status rmc_set_allocator(rmc_ctx *ctx, const float *params, const float *mu, const float *sd,
                             const double *nu_c, const double *gx);
/* The current parameters (host float[RMC_MLP_PARAMS]). */
rmc_status rmc_get_allocator(rmc_ctx *ctx, float *params);

/* Raw features of the current fields: feat[ncells][3] (float: T / 1000, log10(1 + |grad T|),
 * log10(max(kappa_P, 1e-30))) and mask[ncells] (uint8: sign bits of grad T), natural cell
 * order, in `mem` memory.  Host outputs synchronise the stream. */
rmc_status rmc_get_features(rmc_ctx *ctx, float *feat, uint8_t *mask, rmc_mem mem, void *stream);

/* The global-octant logits zg[ncell][nb][ng][8] (host float) of the listed cells, computed
 * by the inference kernel of the learned mode.  Synchronises. */
rmc_status rmc_allocator_logits(rmc_ctx *ctx, const int64_t *cells, int ncell, float *zg, void *stream);

/* Draws of the last compute with RMC_SAMPLING_LEARNED for the listed cells (host arrays):
 * stratum[ncell][R] = (n * ng + g) * 8 + o and p[ncell][R], the probability each ray was drawn
 * with.  Synchronises. */
rmc_status rmc_get_ray_draws(rmc_ctx *ctx, const int64_t *cells, int ncell, int32_t *stratum, double *p,
                             void *stream);

/* Training data of one step (all device pointers): ncell cells with raw features
 * feat[ncell][3] and masks mask[ncell]; pplain[nb * ng] the plain pdf of the run the rays
 * came from; nsamp rays drawn with that plain pdf, sorted by cell: ray i belongs to cell
 * cell_of[i] (0 <= cell_of < ncell, non-decreasing), lies in stratum[i] = (n*ng + g)*8 + o,
 * and has h[i] = Y_i p0_i (its value times the probability p0[i] it was drawn with).  At most
 * 1024 rays per cell.  ray_cost[nsamp] (nullable): the cost of each ray, for instance its
 * number of steps plus a fixed overhead. */
typedef struct {
    int32_t ncell, nsamp;
    const float *feat;
    const uint8_t *mask;
    const double *pplain;
    const int32_t *cell_of, *stratum;
    const double *h, *p0;
    const double *ray_cost;
} rmc_train_batch;

/* Loss of the batch under the current parameters and its gradient (host float
 * grad[RMC_MLP_PARAMS], nullable), from the FP32 training kernels.  Per cell c with samples
 * (i over its rays, p_c the learned pdf above, c_i = ray_cost[i] or 1 without ray_cost):
 *   M_c(p) = mean_i h_i^2 / (p0_i p(s_i)),   C_c(p) = mean_i c_i p(s_i) / p0_i,
 * unbiased estimates, from the plain rays, of the second moment of the cell's ray value and of
 * the expected cost of a ray were its rays drawn from p; and over the batch the ratio
 *   L = [sum_c M_c(p_c)] [sum_c C_c(p_c)] / ([sum_c M_c(p0)] [sum_c C_c(p0)])
 * (C = 1 without ray_cost): the work to reach a given RMS error of the whole field (squared
 * error sum_c Var_c / R, work R sum_c C_c) relative to the plain allocation's.  For one cell
 * its minimiser over pdfs is p_s proportional to sqrt(E[h^2 | s] / E[c | s]).  Synchronises.
 * RMC_INVALID_ARG if the samples are not sorted by cell. */
rmc_status rmc_train_grad(rmc_ctx *ctx, const rmc_train_batch *batch, double *loss, float *grad, void *stream);
/* One Adam step (Kingma & Ba; beta 0.9 / 0.999, eps 1e-8) of learning rate lr on the batch;
 * loss (nullable) is the loss before the step.  Synchronises. */
rmc_status rmc_train_step(rmc_ctx *ctx, const rmc_train_batch *batch, float lr, double *loss, void *stream);
/* nstep Adam steps in one call: step i takes batches[i] (device data as for rmc_train_step,
 * every pointer valid until the call returns) with learning rate lr[i] (host array); losses
 * (host, nullable) receives the loss of each batch before its step.  The steps are enqueued
 * back to back on `stream` with no synchronisation in between; the call synchronises once at
 * the end.  The host checks of every batch run before anything is enqueued; a batch that
 * fails the device-side sample checks (unsorted, out of range, more than 1024 rays in a cell)
 * makes the call return that error after all steps ran (the parameters then hold the steps'
 * result and should be reset with rmc_set_allocator). */
rmc_status rmc_train_steps(rmc_ctx *ctx, const rmc_train_batch *batches, int nstep, const float *lr,
                           double *losses, void *stream);

/* Counters and phase timings of the last compute and accumulated since the last reset.
 * Waits for every compute enqueued so far to finish. */
rmc_status rmc_get_stats(rmc_ctx *ctx, rmc_stats *out);
/* Wait for pending computes, then zero the accumulated counters and timings. */
rmc_status rmc_reset_stats(rmc_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* RMC_H */
