/* bbc — Bernstein-bound caustics on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the bound-driven caustic estimator of "Bernstein Bounds for
 * Caustics" (arXiv 2504.19163).  Three stages run on one GPU:
 *
 *   1. For every (point emitter, specular triangle) tuple the receiver
 *      position u_k(u1) and the path irradiance E_k(u1) are rational functions
 *      of the barycentric coordinates u1 of the specular vertex (Sec. 4.3-4.4;
 *      refraction replaces sqrt(beta) by a linear approximant plus remainder
 *      variables, Sec. 4.3).
 *   2. Each tuple's domain is subdivided adaptively and interval bounds of
 *      u_k and E_k are read off the Bernstein coefficients of numerator and
 *      denominator (Sec. 4.1, Eq. eq_bbound; Sec. 6.1 subdivision and domain
 *      initialisation); the leaves are splatted into a receiver grid that
 *      stores, per cell and tuple, the per-tuple bound E~ (Eq. eq_pertuple_b;
 *      Sec. 6.1 bound storage).
 *   3. Per shading point, the tuples of its cell are sampled with the
 *      variance-bound-optimal probabilities P_T = min(gamma E~_T, 1)
 *      (Sec. 5.4), the selected tuples are root-found by Newton iteration in
 *      the triangle domain (Sec. 6.1), and Alg. 1 returns the unbiased
 *      estimate sum_{T in S} E(T) / P_T.
 *
 * Arithmetic: every bound carries running error bounds and is rounded
 * outward.  Position-only bounds (tuple classification, domain
 * initialisation) run in FP32 and re-evaluate a box in FP64 when a
 * denominator coefficient cannot be given a sign; subdivision boxes, whose
 * irradiance denominator cancels by orders of magnitude, run in FP64 (the
 * same issue rate as unpacked FP32 on this GPU).  Newton iterates in FP32 and
 * every accepted root is polished and weighted in FP64.
 *
 * Conventions
 *  - Every entry point returns a bbc_status; 0 is success.  On failure
 *    bbc_last_error() returns a thread-local message.  Arguments are validated
 *    before any work is enqueued; no C++ exception crosses this ABI.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued asynchronously on it; device outputs are valid once the
 *    stream has been synchronised.
 *  - Arrays are structure-of-arrays FP32.  A `memory` field says whether the
 *    arrays of a struct are host (BBC_MEM_HOST) or device (BBC_MEM_DEVICE)
 *    pointers; the library copies what it keeps, so inputs are only borrowed
 *    for the duration of the call.
 *  - Tuples are numbered emitter * n_tri + triangle.
 */
#ifndef BBC_H
#define BBC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bbc_status;
#define BBC_OK 0
#define BBC_EINVAL (-1)       /* bad argument (null pointer, n < 0, spp < 1, degenerate receiver, eta <= 0) */
#define BBC_ENOMEM (-2)       /* device or host allocation failed */
#define BBC_EBUDGET (-3)      /* serving: a request can never fit the memory budget */
#define BBC_EDEVICE (-4)      /* HIP runtime error; text in bbc_last_error() */
#define BBC_EUNSUPPORTED (-5) /* reserved: a chain type this library does not handle */
#define BBC_EQUEUE (-6)       /* a device work queue or buffer overflowed its capacity */

#define BBC_CHAIN_R 0  /* one specular reflection */
#define BBC_CHAIN_T 1  /* one specular refraction */
#define BBC_CHAIN_RR 2 /* two specular reflections */

#define BBC_MEM_HOST 0
#define BBC_MEM_DEVICE 1

/* Specular casters and the planar receiver (symbols of Sec. 4.2, Table 1).
 * pos: [9][n_tri] rows p0.x p0.y p0.z p1.x ... p2.z; nrm: [9][n_tri] vertex
 * normals n0, n1, n2 (interpolated un-normalised, Eq. eq_ni).  The receiver is
 * the parallelogram x = q0 + u f1 + v f2 with (u, v) in [0,1]^2, its texture
 * space (Sec. 6.1, bound storage).  eta is the ratio of indices of refraction
 * eta' (incident over transmitted side) used by BBC_CHAIN_T (Eq.
 * eq_refr_rational); vertex normals must face the incident side. */
typedef struct {
  int32_t chain;  /* BBC_CHAIN_* */
  int32_t memory; /* BBC_MEM_* for pos/nrm/pos2/nrm2 */
  int64_t n_tri;
  const float* pos;
  const float* nrm;
  int64_t n_tri2; /* BBC_CHAIN_RR: second specular surface */
  const float* pos2;
  const float* nrm2;
  float eta;
  float q0[3], f1[3], f2[3];
} bbc_scene;

/* Emitters: pos [3][n], intensity I0 [n] (Sec. 4.4).  Point lights when edges
 * is NULL.  Otherwise area lights (the emitter variable of the implementation
 * section's area-light remark; single reflection only, EINVAL for the other
 * chains): edges [6][n] holds a and b of the parallelogram
 * pos + z1 a + z2 b, (z1, z2) in [0,1]^2, every point of which emits with
 * intensity I0; the irradiance is the mean over (z1, z2).  Bounds hold for
 * the whole light; a query draws one light point per selected pair. */
typedef struct {
  int32_t memory; /* BBC_MEM_* for pos, I0 and edges */
  int64_t n;
  const float* pos;
  const float* I0;
  const float* edges; /* nullable */
} bbc_emitters;

/* Subdivision and storage controls (Sec. 6.1).  Defaults: max_depth 8,
 * sigma 1e-4, alpha 2 (single scattering), grid_res 512, init_pieces 100,
 * init_levels 4, cover_frac 0.5. */
typedef struct {
  int32_t max_depth;   /* depth cap, counted from the initialised root box */
  float sigma;         /* stop when the clipped position-bound area (in receiver units) < sigma */
  float alpha;         /* stop when E_hi / E_lo < alpha (E_lo > 0) */
  int32_t grid_res;    /* receiver grid is grid_res x grid_res cells over [0,1]^2 (1..4096) */
  int32_t init_pieces; /* domain initialisation keeps at most this many boxes */
  int32_t init_levels; /* and descends at most this many levels */
  int32_t flags;       /* BBC_FLAG_* */
  float cover_frac;    /* bound storage: a tuple whose leaves' closed cell rectangles add up to at
                          least cover_frac * grid_res^2 cells is stored once, in a cover-all list
                          read by every shading point after its cell's list, with the largest E_hi
                          of its leaves (default 0.5; 0 keeps every tuple in the cells) */
} bbc_subdiv_params;
#define BBC_FLAG_FIXED_DEPTH 1  /* only the depth cap stops subdivision (parity mode) */
#define BBC_FLAG_NO_REMAINDER 2 /* refraction without remainder variables (ablation; bounds may be invalid) */
/* refraction: irradiance bound by implicit differentiation of the specular
 * polynomials F (Snell's law) and G (coplanarity) over the box times its
 * position bound (Sec. 4.4, "Implicit differentiation"), rounded outward;
 * the other chains ignore it */
#define BBC_FLAG_IMPLICIT_IRR 4
/* two reflections: degree reduction (Sec. 6.1, "Degree reduction") of the
 * irradiance ratio Den^3 / det M, whose degree (46, 46) exceeds the threshold
 * 40: both polynomials are replaced by least-squares approximants of degree
 * (16, 16) plus a remainder variable each, and the ratio is bounded over
 * (16, 16, 1, 1); the other chains ignore it */
#define BBC_FLAG_DEGREE_REDUCTION 8

typedef struct bbc_bounds bbc_bounds;

/* Stage 1 and 2: build the bound hierarchy and receiver grid of a scene.
 * The scene and emitter arrays are copied into library-owned device memory.
 * *out receives an opaque handle owned by the library until bbc_free_bounds.
 * Returns BBC_EQUEUE if a capacity in `params` order of magnitude is exceeded
 * even after the library's automatic regrowth.
 *
 * Two reflections (BBC_CHAIN_RR): tuples are (emitter, t1, t2) with t1 on
 * the first surface and t2 on the second, numbered (emitter * n_tri + t1) *
 * n_tri2 + t2 (below 2^32).  Tuple construction (Sec. 6.1) keeps the pairs
 * whose interval bound of (x2 - x1) x d~1 covers zero; this costs one host
 * synchronisation, since the pair count sizes the per-tuple buffers.  The
 * irradiance bound of this chain (Sec. 4.4, with u1 as the parameter: det M
 * of degree 46 per axis over Den^3) takes the ratio's coefficient signs as
 * computed in FP64; a box whose det M changes sign gets E = [0, inf). */
bbc_status bbc_build_bounds(const bbc_scene* scene, const bbc_emitters* emitters, const bbc_subdiv_params* params,
                            void* stream, bbc_bounds** out);

/* Rebuild in place: same as bbc_build_bounds but reuses the device buffers of
 * an existing handle (no allocation when capacities suffice). */
bbc_status bbc_rebuild_bounds(bbc_bounds* b, const bbc_scene* scene, const bbc_emitters* emitters,
                              const bbc_subdiv_params* params, void* stream);

/* Release a handle; bbc_free_bounds(NULL) is a no-op. */
bbc_status bbc_free_bounds(bbc_bounds* b);

typedef struct {
  int64_t n_tuples;       /* emitters x triangles */
  int64_t n_live_tuples;  /* tuples with a root box after domain initialisation */
  int64_t n_boxes;        /* boxes bounded during subdivision */
  int64_t n_leaves;
  int64_t n_grid_entries; /* (cell, tuple) records plus the cover-all list's */
  int64_t n_inf_leaves;   /* leaves with an infinite irradiance bound */
  int64_t n_fp64_boxes;   /* boxes re-evaluated in FP64 (sign-uncertain denominators) */
  int64_t device_bytes;   /* device memory held by the handle */
  int32_t grid_res;
  int32_t max_depth_reached;
  int64_t n_cover_tuples; /* tuples stored in the cover-all list instead of the cells */
} bbc_bounds_info_t;
bbc_status bbc_bounds_info(const bbc_bounds* b, bbc_bounds_info_t* out);

/* Persist a built hierarchy so that a later process can query it without
 * rebuilding (the bounds depend only on the scene, Sec. 6.1, so one build
 * serves every query of that scene).
 *
 * bbc_bounds_save writes the scene and emitter copies, the subdivision
 * parameters, the build counters and every array the queries and exports
 * read (tuple records, root boxes, leaves grouped by tuple, receiver grid,
 * and for two reflections the second surface and the pair numbers) to the
 * file at `path` (created or truncated).  The file is little-endian in the
 * layout of this library version: magic "BBCBOUND", version 1, a header,
 * one length-prefixed section per array, and a trailing FNV-1a-64 hash of
 * all preceding bytes.  The handle must hold a completed build (the last
 * build or rebuild returned BBC_OK).  EINVAL for a null argument or when the
 * file cannot be written; EDEVICE if a device copy fails.
 *
 * bbc_bounds_load reads such a file into a new handle on the current device
 * (copies ordered on `stream`, which is synchronised before return) and
 * stores it in *out (NULL on failure).  The file is checked before any
 * device memory is written: magic, version, header counts, every section's
 * size, the hash, and that every offset, tuple number, pair number and box
 * code stays inside its array; any failure gives EINVAL with the reason in
 * bbc_last_error().  ENOMEM if device memory runs out.  A loaded handle
 * answers queries, exports and bbc_bounds_info like the saved one, and
 * bbc_rebuild_bounds works on it as on any other handle. */
bbc_status bbc_bounds_save(const bbc_bounds* b, const char* path);
bbc_status bbc_bounds_load(const char* path, void* stream, bbc_bounds** out);

/* Copy the leaves to host memory (arrays of length n_leaves, any may be NULL):
 * tuple[n], code[n] (depth << 28 | iu << 14 | iv, the box index inside the
 * tuple's root box), box[n][4] (u0,u1,v0,v1 of u1), ukbox[n][4] (u_lo,u_hi,
 * v_lo,v_hi clipped to [0,1]^2), E[n][2] (E_lo, E_hi; E_hi may be +inf).
 * Leaves are ordered by tuple, then code. */
bbc_status bbc_export_leaves(const bbc_bounds* b, uint32_t* tuple, uint32_t* code, float* box, float* ukbox, float* E);

/* The tuples the build works on, in the numbering above, ascending: every
 * emitter x triangle for one vertex, the constructed pairs for two
 * reflections (tuple construction, Sec. 6.1).  *n receives their count; up to
 * cap of them are copied to host memory at `tuples` (nullable). */
bbc_status bbc_export_tuples(const bbc_bounds* b, uint32_t* tuples, int64_t cap, int64_t* n);

/* Copy the receiver grid to host memory: offsets[grid_res^2 + 2] and
 * n_grid_entries entries of (tuple, E~).  Slice c = cu * grid_res + cv
 * (offsets[c] .. offsets[c + 1]) is cell (cu, cv), sorted by tuple; slice
 * grid_res^2 is the cover-all list, sorted by tuple.  A shading point's
 * candidate list U is its cell's slice followed by the cover-all slice. */
bbc_status bbc_export_grid(const bbc_bounds* b, uint32_t* offsets, uint32_t* tuple, float* Et);

/* Per-query statistics (host struct, summed over the points of a call). */
typedef struct {
  int64_t n_points;
  int64_t sum_U;       /* sum of |U| (candidate tuples) */
  int64_t sum_S;       /* sum of |S| (selected tuples) */
  int64_t n_roots;     /* accepted specular paths */
  int64_t n_newton;    /* Newton starts (covering leaves of selected tuples) */
  double sum_varbound; /* sum over points of sum_U E~^2 / P (Eq. eq_varbound_u), finite parts */
  int64_t n_pairs;     /* (point, tuple) pairs root-found (= sum_S) */
  int64_t n_iter_fp32; /* FP32 path evaluations (value + Jacobian) */
  int64_t n_iter_fp64; /* FP64 path evaluations (value + Jacobian) */
} bbc_query_stats;

/* Stage 3: irradiance estimates at n shading points (Alg. 1).
 * points_dev [3][n] FP32 device array of positions on the receiver plane;
 * out_E_dev [n] FP32 device array.  spp is W, the expected number of sampled
 * tuples per point (Sec. 5.4).  Result i depends only on (bounds, points[i],
 * i, spp, seed): the Bernoulli draw for tuple T at point i is Philox4x32-10
 * keyed by (seed, i, T).  Points off the receiver return 0.  stats_host may
 * be NULL; when given, the call synchronises the stream to fill it. */
bbc_status bbc_query_irradiance(const bbc_bounds* b, const float* points_dev, int64_t n, int32_t spp, uint64_t seed,
                                float* out_E_dev, bbc_query_stats* stats_host, void* stream);

/* Same with an execution mode:
 *  BBC_QUERY_FUSED   one persistent kernel per call (default of bbc_query_irradiance)
 *  BBC_QUERY_STAGED  one launch per stage: gather+gamma, selection, Newton, accumulation
 *  BBC_QUERY_EXHAUSTIVE (or-ed in) every candidate tuple with P = 1 (position-only enumeration)
 * and, or-ed into BBC_QUERY_STAGED only (EINVAL with the fused form or with
 * EXHAUSTIVE), one of the other sampling schemes the paper compares its
 * estimator with (Sec. 5.2-5.3, the sampling-scheme comparison figure):
 *  BBC_QUERY_UNIFORM     every candidate independently with P = W'/|U|, W' = min(spp, |U|)
 *                        (position bound only)
 *  BBC_QUERY_ONE_SAMPLE  spp independent draws with P1 = E~ / sum of the finite E~; a tuple
 *                        drawn c times contributes E(T) c / (spp P1); unbounded tuples once
 *                        with P = 1
 *  BBC_QUERY_BINS        the bound-optimal P packed next-fit in list order into bins of total
 *                        at most 1, one draw per bin (at most one tuple per bin)
 * point_index_base offsets the point index used by the random stream, so a
 * request split into pieces draws exactly what it would draw whole. */
#define BBC_QUERY_FUSED 0
#define BBC_QUERY_STAGED 1
#define BBC_QUERY_EXHAUSTIVE 16
#define BBC_QUERY_UNIFORM 32
#define BBC_QUERY_ONE_SAMPLE 64
#define BBC_QUERY_BINS 96
#define BBC_QUERY_SAMPLERS 96  /* mask of the three above */
bbc_status bbc_query_irradiance_ex(const bbc_bounds* b, const float* points_dev, int64_t n, int32_t spp, uint64_t seed,
                                   int64_t point_index_base, int32_t mode, float* out_E_dev, float* stats_dev,
                                   bbc_query_stats* stats_host, void* stream);
/* stats_dev (nullable) [n][4] FP32: |U|, |S|, roots, sum_U E~^2/P per point
 * (the last is 0 for the uniform and one-sample schemes). */

/* The staged query for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments and results as bbc_query_irradiance_ex with
 * stats_host = NULL; `mode` must be BBC_QUERY_STAGED, optionally or-ed with
 * BBC_QUERY_EXHAUSTIVE or one sampler.  Results are bit-identical to that
 * call's.  The work space is a 64 MiB device array inside the library (one
 * per GPU, held until the process ends); the points run in consecutive
 * slices of as many points as it holds at the worst case (every candidate of
 * the fullest grid cell selected).  The call allocates nothing and calls no
 * allocating routine.  Every call on a GPU shares that GPU's array: calls
 * that overlap on one GPU (other streams, other host threads) race, so the
 * caller orders them.  EBUDGET when one point's worst case exceeds the array
 * (a cell of more than about 3 million candidates); EINVAL as
 * bbc_query_irradiance_ex, or when the current device is not the handle's. */
bbc_status bbc_query_irradiance_noalloc(const bbc_bounds* b, const float* points_dev, int64_t n, int32_t spp,
                                        uint64_t seed, int64_t point_index_base, int32_t mode, float* out_E_dev,
                                        float* stats_dev, void* stream);

/* Launch-shape knobs (results never depend on them; paper_2504_19163_amd/
 * autotune.py measures the launch-shape ones on a GPU and records its choice
 * per device and workload in paper_2504_19163_amd/tuning.json, which the
 * Python binding applies):
 *  BBC_TUNE_QUERY_WAVES        fused query register budget: 2 (256 VGPRs) or 4 (128) waves per SIMD
 *  BBC_TUNE_QUERY_GRID         fused query persistent workgroups (1..2^20)
 *  BBC_TUNE_BUILD_GRID_PER_CU  persistent build kernels: workgroups per compute unit (1..64),
 *                              or 0 (default) for one resident round of each kernel
 *  BBC_TUNE_QUERY_TILE         fused query shading points per wave: 16, 32 or 64
 *  BBC_TUNE_TIMING             1: record HIP events on the query stream around the
 *                              query's dominant kernel (see bbc_query_kernel_ms)
 *  BBC_TUNE_NEWTON_STEPS       staged query: FP32 Newton iterations per pass of the
 *                              pooled Newton kernel (1..20, default 4); 0 gives each
 *                              lane one selected pair for all of its starts
 *  BBC_TUNE_NEWTON_RESULTS     pooled Newton kernel: accepted roots it keeps per batch
 *                              of 64 pairs (1..96, default 96); the pairs whose roots
 *                              do not fit are redone one lane per pair (smaller values
 *                              exercise that path)
 *  BBC_TUNE_STAGED_PAIRS       staged query and serving batches: worst-case selected pairs
 *                              of one launch (1..2^28, default 2^28); a larger query or
 *                              batch runs as consecutive launches over slices of its points
 *                              (smaller values exercise that path)
 *  BBC_TUNE_GRAPH              staged query: 1 = capture each call's launches into a HIP
 *                              graph (the handle's executable graph is updated in place)
 *                              and replay it on a stream of the handle's own, ordered
 *                              after the caller's stream; 0 (default) launches directly.
 *                              Not with BBC_TUNE_TIMING (timed queries launch directly)
 *  BBC_TUNE_NEWTON_GRID_PER_CU staged query: workgroups per compute unit of the pooled
 *                              Newton kernel (1..64; 0, the default, asks the occupancy
 *                              API how many stay resident)
 *  BBC_TUNE_BUILD_GRAPH        build and rebuild: 1 = capture the launch sequence (counter
 *                              reset, level 0, domain initialisation, one subdivision launch
 *                              per depth) into the handle's HIP graph, updated in place and
 *                              replayed; 0 (default) launches directly.  Not with
 *                              BBC_TUNE_TIMING
 *  BBC_TUNE_RR_OUTLINED        two-reflection subdivision: 1 = run the box evaluation as a
 *                              called (not inlined) function; 0 (default) inlines it (about
 *                              4 % faster).  The same arithmetic: builds are identical
 *  BBC_TUNE_SUBDIV_SPLIT       single-reflection subdivision (point lights): 1 (default) = a
 *                              box that is split writes its four children's polynomials
 *                              (Pu, Pv, Q, Tn, det M, Q^3 and the solid-angle factors, with
 *                              their magnitudes and error factors), split at the midpoint in
 *                              scaled Bernstein form (Sec. 4.1), to a record each, and a child
 *                              is bounded from its record instead of from its corners (4.5 KB
 *                              of device memory per record, room for 65536 records per depth
 *                              parity at first; a build that needs more is redone with room
 *                              for them); n > 1 = the same with room for n records at first
 *                              (rounded down to a multiple of 4, at least 4; up to 2^20);
 *                              0 = every box from its corners.  The same trees; bounds agree
 *                              to rounding and remain rounded outward
 * Applies to later calls on the handle; EINVAL for an unknown knob or value. */
#define BBC_TUNE_QUERY_WAVES 1
#define BBC_TUNE_QUERY_GRID 2
#define BBC_TUNE_BUILD_GRID_PER_CU 3
#define BBC_TUNE_QUERY_TILE 4
#define BBC_TUNE_TIMING 5
#define BBC_TUNE_NEWTON_STEPS 6
#define BBC_TUNE_NEWTON_RESULTS 7
#define BBC_TUNE_STAGED_PAIRS 8
#define BBC_TUNE_GRAPH 9
#define BBC_TUNE_RR_OUTLINED 10
#define BBC_TUNE_NEWTON_GRID_PER_CU 11
#define BBC_TUNE_BUILD_GRAPH 12
#define BBC_TUNE_SUBDIV_SPLIT 13
bbc_status bbc_set_tuning(bbc_bounds* b, int32_t knob, int64_t value);
bbc_status bbc_get_tuning(const bbc_bounds* b, int32_t knob, int64_t* value);

/* Duration in milliseconds of the dominant kernel of the last query on this
 * handle (the fused kernel, or the staged form's Newton kernel summed over the
 * query's slices), measured with HIP events on the query's stream; waits for
 * those events.  EINVAL unless BBC_TUNE_TIMING is on and a query ran since. */
bbc_status bbc_query_kernel_ms(const bbc_bounds* b, float* ms);

/* Duration in milliseconds of the adaptive-subdivision launches of the last
 * build or rebuild on this handle (the step's dominant build kernel, Sec. 6.1
 * domain subdivision), measured with HIP events on the build's stream, and the
 * number of launches (nullable).  Waits for the end event.  EINVAL unless
 * BBC_TUNE_TIMING was on when the build ran. */
bbc_status bbc_build_kernel_ms(const bbc_bounds* b, float* ms, int32_t* launches);

/* ------------------------------------------------------------------ serving
 * A continuous-batching server over resident bound hierarchies (one per
 * scene).  Requests of shading points are queued by bbc_server_submit; a
 * scheduler thread inside the library admits the oldest waiting requests as
 * soon as one of max_inflight batch slots is free and their device work space
 * fits the memory budget, gathers every waiting request of the same scene
 * (in arrival order, up to max_batch_points points and max_batch_requests
 * requests) into one batch, and runs the staged query pipeline for the batch
 * on the slot's own stream, so batches of different slots overlap on the
 * device.  A batch's work space (points, results, per-point request index,
 * and the staged pipeline's buffers sized for the worst case of every
 * candidate tuple being selected) is carved from one device arena of
 * hbm_budget_bytes allocated at creation.
 *
 * Each point keeps the random stream of its own request: the draw for tuple T
 * at point i of a request is keyed by (request seed, point_index_base + i, T)
 * exactly as in bbc_query_irradiance_ex, and each point's estimate is summed
 * in the same order, so a request's result is bit-identical whether it runs
 * alone, through bbc_query_irradiance_ex, or inside any mix of requests.
 *
 * The bounds handles are borrowed: keep them alive, and do not rebuild them,
 * until bbc_server_destroy has returned.  All handles must live on the same
 * device.  Calls on one server may come from several host threads. */
typedef struct bbc_server bbc_server;

#define BBC_SERVER_PAUSED 1 /* create paused: admit nothing until bbc_server_resume */
/* replay each batch's staged launches as a HIP graph captured on the slot's
 * stream (one executable graph per slot, updated in place per batch) */
#define BBC_SERVER_GRAPH 2

typedef struct {
  int64_t hbm_budget_bytes;   /* device arena for batch work space, >= 1 MiB */
  int32_t max_inflight;       /* batch slots (one stream each), 1..16 */
  int32_t max_batch_points;   /* points in one batch, 1..2^24; a request must fit one batch */
  int32_t max_batch_requests; /* requests in one batch, 1..65535 */
  int32_t queue_capacity;     /* waiting requests before submit returns BBC_EQUEUE, >= 1 */
  int32_t mode;               /* 0 (sampled, Alg. 1), BBC_QUERY_EXHAUSTIVE or one of the samplers */
  int32_t flags;              /* BBC_SERVER_PAUSED | BBC_SERVER_GRAPH */
} bbc_server_config;

/* One request: n shading points [3][n] and n results, both host or both
 * device memory (`memory`).  The arrays are borrowed until the request is
 * complete; results are valid after bbc_server_wait or a poll that reports
 * completion. */
typedef struct {
  int32_t memory;           /* BBC_MEM_HOST or BBC_MEM_DEVICE */
  int32_t scene;            /* index into the bounds array given at creation */
  int64_t n;                /* points, 0..max_batch_points */
  const float* points;      /* [3][n] receiver-plane positions */
  float* out;               /* [n] irradiance estimates */
  int32_t spp;              /* W >= 1, the expected sample count per point */
  uint64_t seed;
  int64_t point_index_base; /* index of the first point in the random stream, >= 0 */
} bbc_request;

typedef struct {
  int64_t submitted, completed, rejected; /* rejected: EBUDGET / EQUEUE / EINVAL at submit */
  int64_t batches, points;                /* batches launched and points in them */
  double mean_batch_points, mean_batch_requests;
  double latency_p50_ms, latency_p99_ms, latency_max_ms; /* submit -> result ready, host monotonic clock */
  double batch_gpu_ms;                    /* summed device time of the batches (copies included) */
  int64_t arena_bytes, arena_peak_bytes;  /* budget and the largest part of it in use at once */
  int32_t inflight_peak;                  /* largest number of batches in flight at once */
  int32_t queue_peak;                     /* largest number of waiting requests */
} bbc_server_counters;

/* Create a server over n_bounds resident hierarchies (scene i = bounds[i]).
 * EINVAL for a bad configuration, ENOMEM if the arena or the pinned staging
 * buffers cannot be allocated.  *out is owned by the caller until
 * bbc_server_destroy. */
bbc_status bbc_server_create(bbc_bounds* const* bounds, int32_t n_bounds, const bbc_server_config* cfg,
                             bbc_server** out);
/* Queue one request; *ticket identifies it.  EBUDGET if it can never be
 * admitted (more points than max_batch_points, or more work space than the
 * whole arena); EQUEUE if queue_capacity requests are already waiting (nothing
 * is queued, the caller may retry later); EINVAL for bad arguments. */
bbc_status bbc_server_submit(bbc_server* s, const bbc_request* r, uint64_t* ticket);
/* *done = 1 if the request is complete (then the ticket is retired and the
 * return value is the request's own status), else 0 and BBC_OK.  EINVAL for
 * an unknown or retired ticket. */
bbc_status bbc_server_poll(bbc_server* s, uint64_t ticket, int32_t* done);
/* Block until the request is complete; retires the ticket and returns its
 * status.  latency_ms (nullable) receives submit-to-ready time. */
bbc_status bbc_server_wait(bbc_server* s, uint64_t ticket, double* latency_ms);
/* Start admitting requests (a server created with BBC_SERVER_PAUSED). */
bbc_status bbc_server_resume(bbc_server* s);
/* Counters and latency percentiles since creation or the last reset
 * (reset != 0 clears them after reading). */
bbc_status bbc_server_stats(bbc_server* s, bbc_server_counters* out, int32_t reset);
/* Complete every queued request, stop the scheduler and free the server.
 * NULL is a no-op. */
bbc_status bbc_server_destroy(bbc_server* s);

/* Thread-local text of the last error. */
const char* bbc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BBC_H */
