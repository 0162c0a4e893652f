/*
 * stencil.h -- C ABI of the MI355X (gfx950) temporally blocked stencil engine.
 *
 * The operation (paper Section 2.1, Listings 1-3): T out-of-place Jacobi steps
 *
 *     U^s(i) = sum_{p in P} w_p * U^{s-1}(i + p),   s = 1..T,
 *
 * on a 2D or 3D grid whose halo of width r is a Dirichlet boundary held at its
 * initial values. Temporal blocking (paper Sections 2.1.2-2.1.3, 3, 4) fuses
 * several steps per pass over HBM; the result does not depend on the blocking.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Coefficients: `coeffs` is a host array of (2r+1)^ndim doubles, the dense
 *   coefficient box, row-major, slowest offset first: offset (p_0..p_{d-1})
 *   sits at index sum_j (p_j + r) * (2r+1)^(d-1-j). An entry that is exactly
 *   0.0 is an absent point (no load, no term). The library copies the
 *   coefficients; the caller may free them on return. Single-precision plans
 *   round every coefficient to float (nearest even) once.
 * Summation: each cell adds its terms in that dense-box order, starting from
 *   +0.0, with one fused multiply-add per term. A box with no non-zero entry
 *   is a stencil of no points: every step sets the interior to +0.0.
 * Arrays: `in` and `out` are device pointers (caller-owned, never freed or
 *   retained) to contiguous padded arrays of extents n_j + 2r per dimension,
 *   slowest first, x fastest, in the plan's dtype. `in` is never written.
 *   `out` receives the whole padded grid: U^T on the interior and the halo
 *   copied from `in`. `in` and `out` must not overlap.
 * Streams: `stream` is a hipStream_t (NULL = the default stream). All device
 *   work is enqueued on it and the call returns after enqueueing.
 * Errors: every function returns a stencil_status; nothing throws across the
 *   ABI. Argument errors are detected before any device call.
 *   stencil_last_error() returns a thread-local message for the last failure.
 * Threading: plans are immutable after creation and may be shared between
 *   threads; concurrent executions of one plan need distinct workspaces.
 */
#ifndef STENCIL_H
#define STENCIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STENCIL_OK = 0,
  STENCIL_ERR_INVALID = -1,     /* bad argument (null pointer, ndim, radius, T, extent, dtype) */
  STENCIL_ERR_UNSUPPORTED = -2, /* valid request with no implementation */
  STENCIL_ERR_ALIAS = -3,       /* in and out overlap */
  STENCIL_ERR_NOMEM = -4,       /* device or host allocation failed */
  STENCIL_ERR_DEVICE = -5,      /* a HIP call failed */
  STENCIL_ERR_BUDGET = -6,      /* request exceeds a memory budget */
  STENCIL_ERR_TIMEOUT = -7      /* a bounded device wait expired */
} stencil_status;

typedef enum { STENCIL_F32 = 0, STENCIL_F64 = 1 } stencil_dtype;

/* Interior extents, slowest first; ndim is 2 or 3 (n[2] ignored for 2D). */
typedef struct {
  int32_t ndim;
  int64_t n[3];
} stencil_shape;

/* Optional tuning hint; zero fields mean "choose automatically" (from the
 * autotuner's cache when it holds an entry for this stencil class and size,
 * else the planner's defaults).
 * depth: time steps fused per pass over HBM (paper Section 6.2).
 * tile[0]: rows (2D) or planes (3D) per streamed segment; tile[1..2] reserved.
 * flags: STENCIL_FLAG_NAIVE forces one plain step per pass;
 *        STENCIL_FLAG_NO_CACHE ignores the autotuner's cache;
 *        STENCIL_FLAG_PERSISTENT runs all passes of a blocked plan in one
 *        persistent launch (one workgroup per CU), each pass starting once the
 *        grid-wide count of finished tiles of the previous pass is complete (the
 *        inter-pass grid synchronisation of paper Section 2.1.3, bounded by a
 *        watchdog that stencil_sync reports); ignored for other schemes;
 *        STENCIL_FLAG_UNIFORM_TILES keeps the two edge strips of a blocked 2D
 *        plan at the interior segment length. By default their tiles, which
 *        also apply the Dirichlet columns and so cost more per row, are cut
 *        into shorter segments that take the wave slots the interior tiles
 *        leave free, so that no pass waits on them. The flag also tells the
 *        planner that the plan's tiles share the device with other jobs, so
 *        its depth choice does not charge for a round of tiles this grid
 *        alone would leave part-empty (batches and the server set this flag:
 *        their jobs share the slots);
 *        STENCIL_FLAG_DEVICE_TILING asks a 3D plan for device tiling (paper
 *        Section 4.1, "one tile at a time"): the interior xy plane is split
 *        into 64 x 16 tiles without overlap, one workgroup each, all resident
 *        at once (at most one per CU), every workgroup streams the whole z
 *        extent through all levels and the tiles exchange their r-wide edges
 *        of every level through global memory after each z-step, each tile
 *        publishing one progress counter that its neighbours wait on
 *        (bounded by the watchdog; stencil_sync reports an expiry). Applies
 *        when x is a multiple of 64, y a multiple of 16, the tiles fit the
 *        CUs, the padded grid is below 4 GiB, and the stencil is a radius-1
 *        or radius-2 star or a radius-1 box; otherwise the plan falls back to
 *        the overlapped tiles. STENCIL_FLAG_OVERLAPPED_TILING forbids device
 *        tiling. Without either flag the planner chooses. */
typedef struct {
  int32_t tile[3];
  int32_t depth;
  int32_t flags;
} stencil_tuning;

#define STENCIL_FLAG_NAIVE 1
#define STENCIL_FLAG_NO_CACHE 2
#define STENCIL_FLAG_PERSISTENT 4
#define STENCIL_FLAG_UNIFORM_TILES 8
#define STENCIL_FLAG_DEVICE_TILING 16
#define STENCIL_FLAG_OVERLAPPED_TILING 32

/* Execution scheme chosen by a plan. */
typedef enum {
  STENCIL_SCHEME_COPY = 0,       /* T = 0: out := in */
  STENCIL_SCHEME_NAIVE = 1,      /* one step per pass, no temporal blocking */
  STENCIL_SCHEME_BLOCKED_2D = 2, /* overlapped wave tiles streamed along y (tb2d) */
  STENCIL_SCHEME_BLOCKED_3D = 3, /* overlapped 64x64 workgroup tiles streamed along z (tb3d) */
  STENCIL_SCHEME_DEVICE_3D = 4   /* device tiling: 64x16 tiles exchanging edges every z-step (tb3d_dev) */
} stencil_scheme;

/* Pattern classes of the coefficient box. */
typedef enum { STENCIL_STAR = 0, STENCIL_BOX = 1, STENCIL_GENERAL = 2 } stencil_pattern;

/* What a plan will do (for inspection, tests and benchmarks). */
typedef struct {
  int32_t scheme;        /* stencil_scheme */
  int32_t pattern;       /* stencil_pattern */
  int32_t points;        /* non-zero coefficients k */
  int32_t depth;         /* steps per pass (largest pass) */
  int64_t passes;        /* passes over HBM */
  int32_t tiles;         /* wave tiles per pass (blocked schemes) */
  int32_t strips;        /* column strips (2D) or xy tiles (3D) */
  int32_t seg_len;       /* rows (2D) or planes (3D) per streamed segment */
  int32_t cols_per_lane; /* x cells held by one lane */
  int32_t redundant_lanes; /* lanes of overlap on each open tile side */
  int32_t grid, block;   /* launch shape of the main kernel */
  int64_t cells;         /* interior cells */
  int64_t padded_bytes;  /* bytes of one padded array */
  int64_t workspace_bytes;
  int32_t edge_seg_len;  /* rows per segment of the two edge strips (2D) */
  int32_t edge_tiles;    /* tiles of the edge strips when they have their own
                            segments (2D), else 0 */
  double model_cells_per_s; /* the model's predicted rate of a full-depth pass
                               (valid cell-updates / s; 0 for plain schemes) */
} stencil_plan_info;

typedef struct stencil_plan_s* stencil_plan_t;

/* Build a plan (host only, no device memory is touched except to read the
 * device's properties). `hint` may be NULL. On success *plan owns host memory
 * released by stencil_plan_destroy. */
stencil_status stencil_plan(stencil_plan_t* plan, const double* coeffs, int32_t radius,
                            const stencil_shape* shape, stencil_dtype dtype, int64_t T,
                            const stencil_tuning* hint);

/* Bytes of device workspace stencil_execute needs (0 when none). */
stencil_status stencil_plan_workspace(stencil_plan_t plan, size_t* bytes);

/* Describe the plan's decisions. */
stencil_status stencil_plan_describe(stencil_plan_t plan, stencil_plan_info* info);

/* Run the plan: in -> out on `stream`, using `workspace` (device memory of at
 * least stencil_plan_workspace bytes, may be NULL when that is 0, must not
 * overlap in or out). */
stencil_status stencil_execute(stencil_plan_t plan, const void* in, void* out, void* workspace,
                               void* stream);

stencil_status stencil_plan_destroy(stencil_plan_t plan);

/* One-shot: plan, stream-ordered workspace allocation, execute, release. */
stencil_status stencil_run(const double* coeffs, int32_t radius, const stencil_shape* shape,
                           stencil_dtype dtype, int64_t T, const void* in, void* out, void* stream);

/* For callers that cannot allocate device memory (work recorded under stream
 * capture, tight serving loops, hosts that forbid allocation): stencil_run
 * with the same arguments and results, bit for bit, that makes no device
 * allocation or release. A plan of two or more passes uses, as its ping-pong
 * workspace, a library-owned device region of STENCIL_NOALLOC_SCRATCH_BYTES
 * (64 MiB), one per GPU, held from the first call on that GPU until the
 * process ends. Plans whose workspace (one padded grid) is larger are
 * rejected with STENCIL_ERR_INVALID and a message naming the limit; single-
 * pass plans need no workspace and have no size limit. Calls that overlap on
 * one GPU (two streams or threads at once) share the region and race: the
 * caller serialises them. Other errors as stencil_run. */
#define STENCIL_NOALLOC_SCRATCH_BYTES (64ull << 20)
stencil_status stencil_run_noalloc(const double* coeffs, int32_t radius, const stencil_shape* shape,
                                   stencil_dtype dtype, int64_t T, const void* in, void* out,
                                   void* stream);

/* ---- Batched execution (many independent grids in persistent launches) ----
 *
 * A job is one stencil_run request: coefficients (host, copied at submit),
 * radius, interior shape, dtype, T, device arrays in / out (same conventions
 * as stencil_run; `in` never written, `out` receives the padded result), a
 * caller tag, and an optional depth hint (0 = planner's choice).
 * stencil_batch_submit validates and plans every job (per_job_status[i] gets
 * the job's status; invalid jobs are skipped), checks that no two jobs share
 * memory, and enqueues on `stream`: one halo-frame copy launch, then one
 * persistent launch per kernel variant in use, whose workgroups pull
 * (job, pass, tile) items from a shared work list; a tile waits until its
 * job's previous pass is complete (paper Section 4.1, tile-by-tile execution,
 * applied across grids). Jobs without a blocked variant run with the plain
 * kernel on the same stream. Workspace and control memory are allocated and
 * released stream-ordered. Returns STENCIL_OK if at least the valid jobs were
 * enqueued, STENCIL_ERR_INVALID if no job is valid or an argument is NULL,
 * STENCIL_ERR_ALIAS if jobs overlap. A bounded device wait that expires is
 * reported by the next stencil_sync on that stream. */
typedef struct {
  const double* coeffs;
  int32_t radius;
  stencil_shape shape;
  stencil_dtype dtype;
  int64_t T;
  const void* in;
  void* out;
  uint64_t tag;
  int32_t depth; /* 0: planner's choice */
} stencil_job;

stencil_status stencil_batch_submit(const stencil_job* jobs, int32_t n, void* stream,
                                    stencil_status* per_job_status);

/* Host only: describes the plan stencil_batch_submit runs `job` with (scheme,
 * depth, passes, tiles; its in/out pointers are not read). Batched plans use
 * uniform tiles of the batch's segment lengths, are capped at the fused
 * kernel's depth for their variant, and take their depth from the model as
 * if the device were full (the other jobs fill it). STENCIL_ERR_INVALID for
 * NULL arguments; planning errors as stencil_plan. */
stencil_status stencil_batch_describe(const stencil_job* job, stencil_plan_info* info);

/* Wait for `stream` and report device-side failures of the library's kernels
 * enqueued on that stream since the last call on it: STENCIL_ERR_TIMEOUT if a
 * bounded wait expired (the affected results are undefined), STENCIL_ERR_DEVICE
 * if the stream reports an error, else STENCIL_OK. Each launch has its own
 * error word, so an expiry never affects the waits of other launches; a small
 * kernel after each launch folds it into a report word of the stream, which
 * this call reads and clears. The watchdog limit is 5 s per wait, or
 * STENCIL_WATCHDOG_US microseconds when that environment variable is set
 * (read at each launch). */
stencil_status stencil_sync(void* stream);

/* Diagnostic: average time of one device-wide synchronisation of a grid of
 * one workgroup per CU through a counter in device memory (the mechanism
 * that separates passes in persistent launches; the paper's T_Dsync, Section
 * 5.2.2), over `rounds` barriers in one launch after a warm-up launch.
 * Synchronises `stream`. Errors: STENCIL_ERR_INVALID (rounds < 1, NULL
 * result, rounds above 1e6), STENCIL_ERR_TIMEOUT (a bounded wait expired),
 * device errors. */
stencil_status stencil_probe_grid_sync(int32_t rounds, void* stream, double* seconds_per_sync);

/* ---- Microbenchmarks for the model's parameters (paper Section 5.1: the
 * bandwidths B_gm and B_sm; Section 6.1: latencies, whose product with a
 * throughput is the parallelism a kernel needs by Little's law; Section
 * 5.2.2: the cost of a synchronisation). Each allocates its own device
 * memory stream-ordered on `stream`, times its kernels with events on it,
 * synchronises it and releases the memory before returning. Errors:
 * STENCIL_ERR_INVALID (arguments), STENCIL_ERR_NOMEM, STENCIL_ERR_DEVICE,
 * STENCIL_ERR_TIMEOUT (a bounded wait of the neighbour probe expired). ----
 *
 * stencil_probe_copy: reachable HBM bandwidth, (read + write bytes) / s of a
 *   streaming device copy of `bytes` (1 MiB .. 64 GiB; 2 x bytes allocated)
 *   with 128-bit loads and stores: the best run over four kernel variants
 *   (4 or 8 loads in flight per lane, non-temporal or ordinary accesses) and
 *   grids of 4 to 32 workgroups per CU, three timed runs each.
 * stencil_probe_latency: seconds per link of a dependent chain, one lane:
 *   STENCIL_PROBE_HBM_LATENCY loads that jump across a 1 GiB buffer (beyond
 *   the last-level cache), STENCIL_PROBE_LDS_LATENCY loads from LDS,
 *   STENCIL_PROBE_FMA64_LATENCY FP64 fused multiply-adds. The difference of
 *   two chain lengths cancels the launch cost.
 * stencil_probe_lds_bandwidth: bytes / s of conflict-free 128-bit LDS reads
 *   over all CUs (two workgroups per CU).
 * stencil_probe_neighbor_sync: one workgroup per CU on a 2D torus; in each of
 *   `rounds` rounds a workgroup writes `payload_bytes` (0 .. 1 MiB), publishes
 *   its round counter, waits for its four neighbours' counters (bounded by a
 *   5 s watchdog) and reads their payloads. mode 0 publishes with an
 *   agent-scope release (a write-back of the L2) and polls with acquires;
 *   mode 1 writes the payload through to the coherence point, waits for those
 *   stores and publishes with a plain counter store, the scheme of the 3D
 *   device-tiled pass. *seconds_per_round is the average round; *mismatches
 *   counts payload words read that did not carry their round's value (0 when
 *   the publication scheme is sound). */
#define STENCIL_PROBE_HBM_LATENCY 0
#define STENCIL_PROBE_LDS_LATENCY 1
#define STENCIL_PROBE_FMA64_LATENCY 2

stencil_status stencil_probe_copy(int64_t bytes, void* stream, double* bytes_per_s);
stencil_status stencil_probe_latency(int32_t kind, void* stream, double* seconds);
stencil_status stencil_probe_lds_bandwidth(void* stream, double* bytes_per_s);
stencil_status stencil_probe_neighbor_sync(int32_t mode, int32_t rounds, int32_t payload_bytes, void* stream,
                                           double* seconds_per_round, uint64_t* mismatches);

/* ---- Practical attainable performance model (paper Section 5, Section 6) ----
 *
 * Times of the three pressure points for one tile step of depth t:
 *   T_gm  = a_gm * D_gm / B_gm * S          (global memory, Section 5.1)
 *   T_sm  = a_sm * D_sm * t / B_sm * S      (on-chip memory; skipped if B_sm <= 0)
 *   T_cmp = a_cmp * D_cmp * t / thr_cmp     (arithmetic)
 * T_stencil = max of the three; P = D_all * t / T_stencil (cells/s); the valid
 * proportion V is (tile - 2 t rad) / tile per tiled dimension for SM tiling
 * (Section 5.2.1, both sides of a tile lose t*rad cells) and
 * T_stencil / (T_stencil + n_sync * t_dsync) for device tiling (Section 5.2.2);
 * PP = P * V. Also reported: the desired depth of Section 6.2 (smallest t that
 * moves the bound off global memory; device tiling counts the tile halo in
 * D_gm) and the minimum square device tile of Section 6.4. Units are the
 * caller's, used consistently (bytes/s, flop/s, seconds, cells).
 * Returns STENCIL_ERR_INVALID for NULL pointers or non-positive B_gm, thr_cmp,
 * cell_bytes or t. */
#define STENCIL_MODEL_NO_TILING 0
#define STENCIL_MODEL_SM_TILING 1
#define STENCIL_MODEL_DEVICE_TILING 2

typedef struct {
  double B_gm, B_sm, thr_cmp; /* bandwidths (bytes/s) and compute throughput (flop/s) */
  double cell_bytes;          /* S */
  double a_gm, a_sm, a_cmp;   /* accesses per cell (global, on-chip) and flops per cell */
  double D_gm, D_sm, D_cmp, D_all; /* cells counted for each term and in P */
  double t;                   /* temporal depth */
  int32_t tiling;             /* STENCIL_MODEL_* */
  int32_t tiled_dims;         /* dimensions with overlapped tiles (1 for 2D, 2 for 3D) */
  double tile[2];             /* tile extents (cells) */
  double rad;                 /* stencil radius */
  double t_dsync;             /* seconds per device-wide synchronisation */
  double n_sync;              /* synchronisations per tile step (1 with lazy streaming) */
} stencil_model_params;

typedef struct {
  double T_gm, T_sm, T_cmp, T_stencil;
  double P, V, PP;
  double t_desired, min_tile;
  int32_t bottleneck;         /* 0 global memory, 1 on-chip memory, 2 compute */
} stencil_model_result;

stencil_status stencil_model_eval(const stencil_model_params* params, stencil_model_result* result);

/* ---- Machine parameters of the model and the model-driven planner ----
 *
 * A process-wide set of the model's inputs (paper Section 5.1: bandwidths and
 * compute throughput; Section 5.2.2: synchronisation costs; Section 6.1:
 * latencies). The defaults are MI355X values measured with the probes above:
 * copy bandwidth, LDS bandwidth, device-wide barrier, neighbour-counter round,
 * chain latencies; the vector FP64 peak is 256 CUs x 4 SIMDs x 16 lanes x 2
 * flops at the clock measured under the stencil kernels (2.15 GHz), and FP32
 * runs at the same rate as built (packed FP32 is not used).
 *
 * Without a depth hint or an autotuner entry, stencil_plan chooses among the
 * feasible candidates (2D: every compiled depth; 3D: every compiled depth of
 * the overlapped tiles and, where it applies and is not forbidden, of device
 * tiling) the one whose predicted rate is highest. The prediction
 * (stencil_plan_info.model_cells_per_s) counts the candidate's own HBM
 * traffic, LDS traffic and flops, redundant margin cells included (the valid
 * proportion of Section 5.2.1), and for device tiling one neighbour
 * synchronisation per z-step (Section 5.2.2); the desired depth of Section
 * 6.2 and the deeper-versus-wider trade-off of Section 6.4 follow from
 * maximising it.
 *
 * stencil_machine_get copies the current set; stencil_machine_set replaces it
 * (NULL restores the defaults; STENCIL_ERR_INVALID for non-positive
 * bandwidths, peaks or CU count, or negative sync times);
 * stencil_machine_calibrate runs the probes on `stream` (synchronising it),
 * stores the measured values and returns the new set in *out (may be NULL). */
typedef struct {
  double hbm_bytes_per_s;  /* B_gm: streaming copy (read + write bytes / s) */
  double lds_bytes_per_s;  /* B_sm: LDS reads over all CUs */
  double fp64_flops;       /* vector FP64 FMA peak (flop/s) */
  double fp32_flops;       /* vector FP32 FMA peak as built (flop/s) */
  double grid_sync_s;      /* T_Dsync: one device-wide barrier */
  double neighbor_sync_s;  /* one neighbour-counter round of the device-tiled exchange */
  double hbm_latency_s, lds_latency_s, fma_latency_s; /* dependent-chain latencies */
  int32_t cus;             /* compute units */
} stencil_machine;

stencil_status stencil_machine_get(stencil_machine* out);
stencil_status stencil_machine_set(const stencil_machine* m);
stencil_status stencil_machine_calibrate(void* stream, stencil_machine* out);

/* ---- Autotuner (paper Section 3.4: empirical depth search; Sections 5-6:
 * the model prunes) ----
 *
 * stencil_tune times candidate (scheme, depth, segment) plans of the blocked
 * kernels for this stencil class and grid shape on `stream` and stores the
 * fastest in a process-wide cache keyed by (gfx arch, CU count, ndim, pattern
 * class, radius, points, dtype, half-octave size bucket per axis, single or
 * batched). Candidates: every compiled depth, each with the planner's segment
 * for it and (single grids) half and double that; for single 3D grids also
 * every depth of device tiling where it applies. Candidates whose model rate
 * (stencil_plan_info.model_cells_per_s: the plan's own traffic, flops and
 * valid proportion under the current stencil_machine parameters) is below 60%
 * of the best model rate are not timed. STENCIL_TUNE_BATCH tunes the depth used by
 * stencil_batch_submit, timing a batch of replicas of the grid that fills the
 * device; STENCIL_TUNE_FORCE re-measures a cached entry. The tuner allocates
 * and frees its own device buffers (in, out(s), workspace of the padded size)
 * and synchronises `stream`; results never depend on the choice (blocking is
 * exact). Errors: STENCIL_ERR_INVALID (arguments), STENCIL_ERR_UNSUPPORTED (no
 * blocked kernel for this stencil and shape), STENCIL_ERR_NOMEM, device errors.
 *
 * Plans without a hint and batch jobs with depth 0 use the cached choice
 * (depth, segment and, for 3D, scheme; a caller's scheme flag wins).
 * stencil_tune_lookup reports it in out->depth, out->tile[0] and out->flags
 * (found = 0 when absent); the cache is saved
 * to and merged from a JSON file ({"entries": [{"key", "depth", "seg", ...}]});
 * stencil_tune_cache_key writes the key of a request into buf. */
#define STENCIL_TUNE_BATCH 1
#define STENCIL_TUNE_FORCE 2

typedef struct {
  int32_t depth;            /* chosen steps per pass */
  int32_t seg_len;          /* chosen rows/planes per segment (0: planner's) */
  double seconds_per_step;  /* measured, per grid */
  double model_cells_per_s; /* model rate of the chosen candidate */
  int32_t candidates;       /* candidates timed */
  int32_t from_cache;       /* 1 if answered from the cache */
  int32_t flags;            /* chosen scheme: STENCIL_FLAG_DEVICE_TILING or
                               STENCIL_FLAG_OVERLAPPED_TILING (3D), else 0 */
} stencil_tune_result;

stencil_status stencil_tune(const double* coeffs, int32_t radius, const stencil_shape* shape,
                            stencil_dtype dtype, int32_t flags, void* stream,
                            stencil_tune_result* result);
stencil_status stencil_tune_lookup(const double* coeffs, int32_t radius, const stencil_shape* shape,
                                   stencil_dtype dtype, int32_t flags, stencil_tuning* out,
                                   int32_t* found);
stencil_status stencil_tune_cache_key(const double* coeffs, int32_t radius, const stencil_shape* shape,
                                      stencil_dtype dtype, int32_t flags, char* buf, size_t len);
stencil_status stencil_tune_cache_load(const char* path, int32_t* loaded);
stencil_status stencil_tune_cache_save(const char* path);
stencil_status stencil_tune_cache_clear(void);

/* ---- Serving loop (continuous batching of stencil requests) ----
 *
 * A server owns one HIP device, a compute stream, a copy stream and a
 * scheduler thread. Requests (a stencil_job whose in/out are ignored, plus the
 * padded input grid in host memory, copied at submit so the caller may reuse
 * it) wait in a FIFO queue. Admission: a request enters when a slot is free
 * and the device memory it needs (two padded grids plus one batch workspace
 * per round in flight, held until its result is collected) fits in the HBM
 * budget; the input is copied to the device on the copy stream while rounds
 * run. Each round runs the next quantum (at most quantum_passes passes of the
 * request's temporal depth) of every resident request in one
 * stencil_batch_submit, so a request that arrives mid-round starts at the
 * next round composed after its admission and its work shares the device
 * with the others'. With rounds_in_flight = 2 the next round is composed and
 * enqueued shortly before the running one is expected to end, which hides
 * the host's work between rounds (lower latency under moderate load) but
 * makes rounds smaller under saturation (lower capacity); with 1 (the
 * default) it is composed when the running one has ended. A quantum
 * is quantum_passes passes; with
 * round_target_s > 0 it is at least the request's fair share of a round of
 * that duration (the throughput measured over past rounds, divided by the
 * resident requests and the request's cells, in whole passes). Latency is measured from submit to the end of
 * the round that completes the request; results stay on the device until
 * stencil_server_poll collects them. Results equal stencil_run's bit for bit
 * (running T steps as several quanta is the same arithmetic).
 *
 * stencil_server_create: budget > 0, max_slots >= 1; quantum_passes <= 0
 *   means 4; round_target_s <= 0 turns the fair share off; rounds_in_flight
 *   <= 0 means 1, and above 2 is STENCIL_ERR_INVALID. Fails with
 *   STENCIL_ERR_DEVICE when the device is unusable.
 * stencil_server_submit: STENCIL_ERR_BUDGET if the request alone exceeds the
 *   budget, STENCIL_ERR_INVALID for a bad job (as stencil_plan) or NULL
 *   arguments; otherwise returns a ticket.
 * stencil_server_poll: *done = 0 while pending; once done, copies the padded
 *   result to host_out (if not NULL), stores the latency, releases the
 *   request's device memory and forgets the ticket (*done = 1). Returns the
 *   request's own error (e.g. STENCIL_ERR_TIMEOUT) if it failed, and
 *   STENCIL_ERR_INVALID for an unknown ticket. stencil_server_wait blocks
 *   until the request is done, then behaves like poll.
 * stencil_server_stats: counters and latency percentiles over the requests
 *   completed so far (nearest-rank p50 / p99).
 * stencil_server_destroy: stops the scheduler, waits for the rounds in
 *   flight, drops pending requests and releases all device memory. */
typedef struct stencil_server_s* stencil_server_t;

typedef struct {
  int32_t device;            /* HIP device ordinal */
  int32_t max_slots;         /* resident requests at most */
  int32_t quantum_passes;    /* passes per request per round (<= 0: 4) */
  uint64_t hbm_budget_bytes; /* device memory for resident requests */
  double round_target_s;     /* > 0: fair share of a round of this duration */
  int32_t rounds_in_flight;  /* rounds enqueued at a time, 1 or 2 (<= 0: 1) */
} stencil_server_config;

typedef struct {
  uint64_t submitted, admitted, completed, failed, rejected, rounds;
  int32_t active, queued, max_active;
  uint64_t hbm_in_use, hbm_peak;
  double cell_updates;       /* completed requests' cells x T */
  double busy_s;             /* rounds' device time */
  double wall_s;             /* first submit to last completion */
  double p50_s, p99_s, mean_s, max_s; /* latency of completed requests */
} stencil_server_statistics;

stencil_status stencil_server_create(const stencil_server_config* config, stencil_server_t* server);
stencil_status stencil_server_submit(stencil_server_t server, const stencil_job* job,
                                     const void* host_in, uint64_t* ticket);
stencil_status stencil_server_poll(stencil_server_t server, uint64_t ticket, void* host_out,
                                   int32_t* done, double* latency_s);
stencil_status stencil_server_wait(stencil_server_t server, uint64_t ticket, void* host_out,
                                   double* latency_s);
stencil_status stencil_server_stats(stencil_server_t server, stencil_server_statistics* stats);
stencil_status stencil_server_destroy(stencil_server_t server);

/* Thread-local description of the last failure on this thread ("" if none). */
const char* stencil_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STENCIL_H */
