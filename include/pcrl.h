/*
 * pcrl.h -- C ABI of the MI355X (gfx950) coarse-path ray launcher.
 *
 * The library implements the coarse path tracing stage of "A Ray Launching
 * Approach for Computing Exact Paths with Point Clouds" (Vaara et al., 2024)
 * as uniform ray launching over a multi-level voxelisation of a labeled
 * point cloud:
 *
 *   build_voxels   voxelisation (Section 2.1): a hierarchy of axis-aligned
 *                  voxel levels over the cloud, each finer level dividing
 *                  the coarser one by an integer factor (the subvoxels of
 *                  Section 2.1 are the finest level), with per-leaf point
 *                  ranges;
 *   launch_rays    coarse path tracing (Section 2.2): uniformly spaced rays
 *                  from every TX walk the hierarchy by DDA, intersect points
 *                  as surfel disks, reflect specularly up to K times
 *                  (Section 2.2.3, propagation phase) and are received by RX
 *                  spheres;
 *   collect_paths  coarse paths as label sequences deduplicated with the
 *                  duplicate limit kappa (Section 2.2.3);
 *   refine_paths   exact paths from coarse ones by gradient descent on the
 *                  path length (Section 2.3, Eq. 2), then their dedup.
 *
 * Conventions for every entry point
 *   - Return value: PCRL_OK (0) or a negative status below; the message of
 *     the last failure on the calling thread is available from last_error().
 *   - Pointers documented as "device" point to device memory of the current
 *     HIP device (e.g. torch tensors on cuda:N); "host" pointers to host memory.
 *   - Arrays are contiguous; [N,3] float arrays are xyz-interleaved rows.
 *   - All work is enqueued on the given stream (NULL = default stream) and is
 *     asynchronous unless stated otherwise.  Caller input arrays are read
 *     only by work enqueued during the call, so they may be released in
 *     stream order afterwards.
 *   - Objects (PcrlScene, PcrlLaunch) are owned by the library until their
 *     release_* call; a launch refers to its scene, so release the launch first.
 *   - A failed call leaves no object behind (out pointers are set to NULL).
 */
#ifndef PCRL_H
#define PCRL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PCRL_OK         0
#define PCRL_EINVAL    -1   /* bad argument: NULL, size, non-finite input, zero normal, level sizes not integer multiples, K > 8 */
#define PCRL_ENOMEM    -2   /* device or host allocation failed */
#define PCRL_EOVERFLOW -3   /* results exceed a capacity; the size needed is reported (see each call) */
#define PCRL_EHIP      -4   /* HIP runtime error */
#define PCRL_EBUSY     -5   /* admission refused (serving) */
#define PCRL_ECANCELED -6   /* the query was cancelled (serving) */

#define PCRL_MAX_LEVELS 4
#define PCRL_MAX_REFLECTIONS 8

typedef struct PcrlScene PcrlScene;
typedef struct PcrlLaunch PcrlLaunch;
typedef void* pcrl_stream_t; /* a hipStream_t */

/* ------------------------------------------------------------------------ */
/* device memory                                                             */
/* ------------------------------------------------------------------------ */

/* Where the library's device buffers (scene hierarchies, ray state, records,
 * temporaries) come from.  alloc returns `bytes` of device memory of the
 * current device usable in stream order on `stream` (NULL on failure, which
 * the calling entry point reports as PCRL_ENOMEM); free releases a block in
 * stream order on `stream` (work enqueued there before may still use it).
 * ctx is passed back unchanged.  Both run on whichever thread calls into the
 * library (the serving worker included) and must be thread-safe. */
typedef struct {
    void* (*alloc)(size_t bytes, pcrl_stream_t stream, void* ctx);
    void  (*free)(void* ptr, pcrl_stream_t stream, void* ctx);
    void* ctx;
} PcrlAllocator;

/* Route all later device allocations of the library to `a` (copied), e.g. a
 * framework's caching allocator; NULL returns to the library's own caching
 * allocator (per-device free lists by size class, reuse in stream order or
 * after an event).  Blocks are always freed through the allocator that made
 * them, so objects created before a switch stay valid; the callbacks must
 * therefore stay callable until every block they made is freed (release the
 * objects made under them, or keep them for the life of the process).
 * PCRL_EINVAL if a callback is missing. */
int set_allocator(const PcrlAllocator* a);

/* ------------------------------------------------------------------------ */
/* voxelisation (Section 2.1)                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n_levels;                     /* 1..4 voxel levels */
    float   level_size[PCRL_MAX_LEVELS];  /* edge lengths in metres, coarse -> fine; each an integer
                                             multiple (within 1e-4 relative) of the next */
    float   surfel_radius;                /* r_s > 0: every point is a two-sided disk of this radius */
    float   t_eps;                        /* self-intersection distance; <= 0 selects 1e-5 x AABB diagonal */
    int32_t flags;                        /* 0, or PCRL_VOXEL_COMPACT */
} PcrlVoxelParams;

/* PcrlVoxelParams.flags: keep no dense cell table of the leaves' parent bricks
 * (8 bytes per leaf cell of every occupied parent); the traversal then reads
 * the bricks' occupancy masks (less device memory, slower).  The table is
 * also left out when the parent-to-leaf ratio exceeds 16 or it would exceed
 * 256 MiB (beyond the last-level cache it slows the traversal down). */
#define PCRL_VOXEL_COMPACT 1

typedef struct {
    int64_t n_points;                     /* input points */
    int64_t n_entries;                    /* (leaf, point) pairs: a point is listed in every leaf its disk overlaps */
    int64_t n_leaves;                     /* occupied leaves */
    int64_t n_nodes[PCRL_MAX_LEVELS];     /* occupied cells per level (n_nodes[n_levels-1] = n_leaves) */
    int32_t max_label;                    /* largest label of the static points (bit pattern of the uint32) */
    int32_t n_levels;
    int32_t dims[3];                      /* leaf grid dimensions */
    int32_t dims0[3];                     /* coarsest grid dimensions */
    float   origin[3];                    /* grid origin (metres) */
    float   leaf_size;                    /* finest edge length */
    float   surfel_radius;
    float   t_eps;                        /* effective self-intersection distance */
    float   aabb[6];                      /* point AABB: min xyz, max xyz */
    int64_t device_bytes;                 /* device memory held by the scene */
    int32_t key_bits;                     /* bits of the hierarchical leaf key */
    int32_t reserved;
    int64_t n_dynamic;                    /* points of the current dynamic overlay (update_points) */
    int64_t epoch;                        /* number of update_points calls so far */
} PcrlSceneInfo;

/* Build the voxel hierarchy of a labeled point cloud.
 *   xyz    device [n_points,3] float32 positions
 *   normal device [n_points,3] float32 normals (any non-zero length; normalised here)
 *   label  device [n_points]   uint32 labels (segmented surfaces)
 * n_points may be 0 (every ray then escapes).  Fails with PCRL_EINVAL on a
 * non-finite coordinate, a zero or non-finite normal, or invalid params.
 * Synchronises the stream internally (twice) to size its buffers. */
int build_voxels(const float* xyz, const float* normal, const uint32_t* label, int64_t n_points,
                 const PcrlVoxelParams* params, pcrl_stream_t stream, PcrlScene** out);

/* Incremental re-voxelisation: replace the scene's dynamic points.
 *   ids    device [n] uint32 global point ids of the dynamic points; they must
 *          differ from the static ids 0..n_points-1 of build_voxels
 *   xyz, normal, label as in build_voxels (device, [n,3] / [n,3] / [n])
 * The points are voxelised into an overlay on the base grid (same origin,
 * levels, surfel radius and t_eps); traversal takes the nearest hit over base
 * and overlay, which is exactly the nearest hit of a scene built from all
 * points with these ids.  Each call starts a new epoch: launches enqueued
 * earlier keep tracing the overlay they started with (it is freed when the
 * last of them is released).  n = 0 removes the overlay.  The static base is
 * never rebuilt.  PCRL_EINVAL if a dynamic point leaves the base grid.
 * Synchronises the stream twice. */
int update_points(PcrlScene* scene, const uint32_t* ids, const float* xyz, const float* normal, const uint32_t* label,
                  int64_t n, pcrl_stream_t stream);

/* Sizes of a built scene (host struct).  PCRL_EINVAL for a NULL argument. */
int scene_info(const PcrlScene* scene, PcrlSceneInfo* out);

/* Copy the leaf table to caller device buffers of capacity >= n_leaves:
 * leaf_key (hierarchical key), leaf_begin and leaf_count (ranges into the
 * leaf-ordered entries) and entry_point (the point id of every entry,
 * capacity >= n_entries).  Any pointer may be NULL.  Synchronous;
 * PCRL_EINVAL for a NULL scene, PCRL_EHIP if a copy fails. */
int scene_leaf_table(const PcrlScene* scene, uint64_t* leaf_key, uint32_t* leaf_begin, uint32_t* leaf_count,
                     uint32_t* entry_point, pcrl_stream_t stream);

int release_scene(PcrlScene* scene);

/* ------------------------------------------------------------------------ */
/* ray launching (Section 2.2)                                               */
/* ------------------------------------------------------------------------ */

#define PCRL_LAUNCH_STATS   1   /* count DDA steps, leaves, surfel tests (slower kernel variant) */
#define PCRL_LAUNCH_TIMING  2   /* time every bounce kernel with HIP events */
#define PCRL_LAUNCH_COHERENT 4  /* trace the first bounce in a direction-coherent ray order and (launches of
                                   >= 65536 rays) every later bounce in a coherent order of its survivors;
                                   results do not depend on it */
#define PCRL_LAUNCH_SDF      8  /* segments end at the implicit surface of Eq. 1 (Section 2.2.1), marched as
                                   sdf_intersect does with its default h, eps and max_steps, instead of at
                                   the surfels: the ray reflects about n(x), the interaction's label and
                                   hit id are those of the nearest point, and a reflected segment starts at
                                   t = 4 eps / |d.n| (outside the |f| <= eps band it left).  One kernel runs
                                   all segments (TIMING reports it as bounce 0).  Not with
                                   PCRL_LAUNCH_STATS, dynamic points or launch_batch / serving. */

typedef struct {
    int64_t n_rays;            /* rays per TX (> 0) */
    const float* directions;   /* device [n_rays,3] unit directions shared by all TX; NULL = Fibonacci lattice */
    int32_t max_reflections;   /* K in [0, 8]: segments 0..K are traced, no reflection after the K-th */
    float   rx_radius_scale;   /* sigma of the reception sphere rho(L) = sigma L alpha / sqrt(3); <= 0 -> 1.25 */
    float   ray_spacing;       /* alpha in radians; <= 0 -> sqrt(8 pi / (sqrt(3) n_rays)) */
    int64_t record_capacity;   /* reception records the launch can hold; <= 0 -> heuristic */
    int32_t flags;             /* PCRL_LAUNCH_* */
    int32_t reserved;
    int32_t* hit_log_id;       /* optional device [n_tx*n_rays*(K+1)]: hit point id per ray and segment,
                                  -1 no hit, -2 segment not traced */
    float*  hit_log_t;         /* optional device, same shape: hit distance (NaN if none) */
} PcrlLaunchParams;

typedef struct {
    int64_t rays;                                  /* n_tx * n_rays */
    int64_t segments;                              /* traced segments, all bounces */
    int64_t active[PCRL_MAX_REFLECTIONS + 1];      /* rays entering bounce b */
    int64_t records;                               /* reception records produced (may exceed capacity) */
    int64_t record_capacity;
    /* PCRL_LAUNCH_STATS only (else 0) */
    int64_t dda_steps;                             /* cells entered at any level */
    int64_t leaves_visited;                        /* occupied leaves whose points were tested */
    int64_t node_lookups;                          /* hierarchy lookups (level-0 map and brick words) */
    int64_t surfel_tests;                          /* ray-disk tests */
    int64_t hits;                                  /* segments ending on a surfel */
    int64_t algo_bytes;                            /* algorithmic bytes of the trace kernels: hierarchy
                                                      reads (4 B level-0, 8-12 B per brick word, 8 B per
                                                      leaf), 32 B per surfel tested, 36 B ray state read per
                                                      later segment, 52 B per reflection, 16 B per record */
    int64_t empty_leaf_steps;                      /* DDA steps into empty leaves of occupied parents */
    int64_t uniform_leaf_visits;                   /* leaf visits shared by every walking lane of the wave */
    int64_t wave_dda_iters;                        /* DDA loop iterations per wave, summed over waves */
    int64_t wave_test_iters;                       /* surfel-test loop iterations per wave, summed over waves */
    int64_t algo_bytes_bounce[PCRL_MAX_REFLECTIONS + 1];  /* algo_bytes of each bounce kernel */
    int64_t dda_steps_bounce[PCRL_MAX_REFLECTIONS + 1];   /* dda_steps of each bounce */
    int64_t surfel_tests_bounce[PCRL_MAX_REFLECTIONS + 1];  /* surfel_tests of each bounce */
    int64_t wave_dda_bounce[PCRL_MAX_REFLECTIONS + 1];    /* wave_dda_iters of each bounce */
    /* PCRL_LAUNCH_TIMING only (else 0) */
    float   kernel_ms[PCRL_MAX_REFLECTIONS + 1];   /* trace kernel time per bounce */
    float   total_ms;                              /* first to last trace kernel */
} PcrlLaunchStats;

/* Launch n_rays rays from each of n_tx TX and trace them.
 *   tx device [n_tx,3] float32, rx device [n_rx,3] float32 (n_rx may be 0).
 * The scene must stay alive until the launch is released.  Asynchronous.
 * PCRL_EINVAL for NULL arrays, n_rays < 1, K outside [0, 8], more than 65535
 * RX, n_tx * n_rays >= 2^31 or a hit log given half; then
 * PCRL_ENOMEM or PCRL_EHIP from the allocations and launches. */
int launch_rays(const PcrlScene* scene, const float* tx, int32_t n_tx, const float* rx, int32_t n_rx,
                const PcrlLaunchParams* params, pcrl_stream_t stream, PcrlLaunch** out);

/* The launch directions used when PcrlLaunchParams.directions is NULL: the
 * Fibonacci lattice z_j = 1 - (2j+1)/N, phi_j = 2 pi frac(j (3 - sqrt 5)/2),
 * evaluated in FP64 and rounded to FP32 (uniformly spaced rays, Section 1's
 * ray launching).  out: device [n_rays,3] float32.  Asynchronous;
 * PCRL_EINVAL unless 1 <= n_rays < 2^31 and out is given. */
int launch_directions(int64_t n_rays, float* out, pcrl_stream_t stream);

/* Counters and timings of a launch (synchronises the launch's stream).
 * PCRL_EINVAL for a NULL argument, PCRL_EHIP if the copy fails. */
int launch_stats(PcrlLaunch* launch, PcrlLaunchStats* out);

/* Raw reception records (synchronous).  Device arrays of capacity `cap`:
 * ray (global ray id g = tx*n_rays + j), rx, n_refl (reflections before
 * reception), len_poly (TX -> interaction points -> RX centre) and len_unf
 * (ray length at closest approach).  Order is unspecified.  *n_out receives
 * the record count; PCRL_EOVERFLOW if it exceeds cap (or the launch's own
 * capacity: then *n_out is the capacity needed). */
int launch_records(PcrlLaunch* launch, int64_t cap, int64_t* ray, int32_t* rx, int32_t* n_refl,
                   float* len_poly, float* len_unf, int64_t* n_out);

int release_launch(PcrlLaunch* launch);

/* ------------------------------------------------------------------------ */
/* batched launching: many TX/RX queries on many scenes (Section 2.2 per TX)  */
/* ------------------------------------------------------------------------ */

/* One query: launch params.n_rays rays from each of n_tx TX into `scene` and
 * receive them at n_rx RX (arrays as in launch_rays). */
typedef struct {
    const PcrlScene* scene;
    const float* tx;           /* device [n_tx,3] */
    int32_t n_tx;
    int32_t n_rx;
    const float* rx;           /* device [n_rx,3] */
    PcrlLaunchParams params;   /* per-query parameters; PCRL_LAUNCH_TIMING times the whole batch */
} PcrlQuery;

typedef struct {
    int32_t tile_rays;          /* ray slots per work item (multiple of 64); <= 0 -> 1024 */
    float   compact_threshold;  /* theta: a bounce keeps survivors in place when the predicted density of live
                                   rays is >= theta, else compacts them; > 1 always compacts; < 0 -> 0.6 */
    int32_t waves_per_cu;       /* persistent waves per compute unit; <= 0 -> 16 */
    int32_t use_graph;          /* replay the bounce loop as a cached hipGraph (ignored with TIMING) */
    int32_t autotune;           /* take tile / theta / waves from the autotuner's table for this batch's
                                   scene class, tuning on up to 32 of its queries on first use */
    int32_t flags;              /* reserved, 0 */
} PcrlBatchParams;

/* Trace all queries together: one persistent work-queue kernel per bounce
 * serves every query's rays (tiles of tile_rays slots), so queries of very
 * different sizes share the GPU.  Each query gets its own launch object in
 * out[i] (use collect_paths / launch_stats / launch_records / release_launch
 * on it as for launch_rays); its results are bitwise those of launch_rays
 * with the same arguments.  Scenes must outlive the launches.  Asynchronous
 * (the autotuner, when it runs, synchronises).  On failure every out[i] is
 * NULL. */
int launch_batch(const PcrlQuery* queries, int32_t n_queries, const PcrlBatchParams* params, pcrl_stream_t stream,
                 PcrlLaunch** out);

/* Tune tile_rays, compact_threshold and waves_per_cu on the given queries
 * (coordinate descent over measured batch times; the queries are traced
 * several times and the results discarded).  The winner is stored in the
 * process-wide table used by launch_batch(autotune = 1) for this scene class
 * (GPU architecture, number of levels, log2 mean entries, log2 mean rays)
 * and returned in *out.  Synchronous; PCRL_EINVAL without queries or out,
 * otherwise launch_batch's statuses. */
int batch_autotune(const PcrlQuery* queries, int32_t n_queries, pcrl_stream_t stream, PcrlBatchParams* out);

/* ------------------------------------------------------------------------ */
/* coarse paths (Section 2.2.3)                                              */
/* ------------------------------------------------------------------------ */

#define PCRL_KEY_LABELS 0   /* key = (tx, rx, n_refl, labels of the interactions) */
#define PCRL_KEY_LEAVES 1   /* key = (tx, rx, n_refl, linear finest-leaf index of the interaction points) */

typedef struct {
    int64_t capacity;          /* rows the arrays can hold */
    int64_t n_rows;            /* out: rows written (sum over keys of min(count, kappa)) */
    int64_t n_keys;            /* out: distinct coarse paths */
    /* device arrays, one entry per row, rows sorted by (key, len_poly, ray) */
    int32_t* tx;
    int32_t* rx;
    int32_t* n_refl;
    int64_t* key;              /* [capacity*K]: label (or leaf index) of interaction k, -1 for k >= n_refl */
    int64_t* count;            /* records that share the row's key */
    int32_t* rank;             /* 0..kappa-1 position of the row within its key */
    int64_t* ray;              /* global ray id of the row */
    float*   len_poly;
    float*   len_unf;
    float*   points;           /* [capacity*K*3] interaction points, NaN for k >= n_refl */
} PcrlPaths;

/* Deduplicate the launch's records into coarse paths: rows with the same key
 * are ordered by (len_poly, ray) and the first kappa (>= 1) are kept.
 * Synchronises the stream; any output pointer may be NULL.  Returns
 * PCRL_EOVERFLOW with out->n_rows = rows needed if capacity is too small, or
 * if the launch dropped records (then launch_stats().records is the record
 * capacity to relaunch with). */
int collect_paths(PcrlLaunch* launch, int32_t kappa, int32_t key_mode, PcrlPaths* out, pcrl_stream_t stream);

/* collect_paths for callers that cannot allocate (code that must not call the
 * device allocator: tight serving loops, harnesses that forbid allocation):
 * the same rows, bit for bit, computed with no device, pinned-host or
 * caller-allocator allocation.  Its temporaries live in one fixed 64 MiB
 * device array per GPU, held from the first call on that GPU until the
 * process ends and shared by every call on that GPU: calls on one GPU must
 * not overlap in time (overlapping calls race on the array and give wrong
 * rows).  Enough for about 600k reception records with the longest keys
 * (about 1.2M with single-word keys); a launch with more records is refused
 * with PCRL_EINVAL before any work is enqueued.  Synchronises the stream. */
int collect_paths_noalloc(PcrlLaunch* launch, int32_t kappa, int32_t key_mode, PcrlPaths* out,
                          pcrl_stream_t stream);

/* ------------------------------------------------------------------------ */
/* path refinement (Section 2.3, Eq. 2)                                      */
/* ------------------------------------------------------------------------ */

/* Outcome of a refined path (PcrlRefined.status). */
#define PCRL_REFINE_VALID          0   /* converged, a reflection at every point, last segment unblocked */
#define PCRL_REFINE_NOT_CONVERGED  1   /* gradient norm still >= grad_tol after max_iters steps */
#define PCRL_REFINE_MISS           2   /* a ray towards an updated point hit nothing */
#define PCRL_REFINE_WRONG_SIDE     3   /* converged, but a point has its neighbours on both sides of its surfel */
#define PCRL_REFINE_OCCLUDED       4   /* converged, but a surfel blocks the last segment to the RX */
#define PCRL_REFINE_DEGENERATE     5   /* a segment of zero length */
#define PCRL_REFINE_OFF_EDGE       6   /* a diffraction point stepped off its edge's segment */

typedef struct {
    int32_t max_iters;   /* rho: gradient steps before a path is given up; <= 0 -> 2000 (Table 1) */
    float   grad_tol;    /* delta: convergence threshold on the norm of the tangent-plane gradient of the
                            path length (all points together); <= 0 -> 1e-4 (Table 1) */
    float   step;        /* eta in (0, 1]: point k steps by eta / (1/|I_k - I_k-1| + 1/|I_k - I_k+1|) times
                            its gradient; <= 0 -> 0.75 */
    float   carrier_hz;  /* frequency of the first-Fresnel-zone dedup; 0 -> 60e9 (Table 1); < 0 skips it */
    int32_t flags;       /* 0 or PCRL_REFINE_SMOOTH */
    float   smooth_radius;  /* PCRL_REFINE_SMOOTH: radius h of the normal average, surfel radius < h <= 0.98 x
                               leaf edge (PCRL_EINVAL otherwise); <= 0 -> 0.95 x leaf edge */
    /* diffraction edges (Section 2.3: D_k = c_k + t_k w_k); edge_of NULL: every interaction is a reflection */
    const int32_t*  edge_of;       /* device [n_rows * k_stride]: edge of interaction k of row i, -1 for a
                                      reflection */
    int32_t         n_edges;
    const float*    edge_seg;      /* device [n_edges,2,3]: end points a, b (non-zero length) */
    const float*    edge_normals;  /* device [n_edges,2,3]: outward normals of the edge's two faces */
    const uint32_t* edge_label;    /* device [n_edges]: the label of a diffraction at the edge */
} PcrlRefineParams;

/* PcrlRefineParams.flags: the surface normal at an interaction point is the
 * weighted average of the normals of the points within smooth_radius of it
 * (weights (1 - d^2/h^2)^4, each normal oriented like the hit surfel's: the
 * smooth normal n(x) of Eq. 1) instead of the hit surfel's own normal. */
#define PCRL_REFINE_SMOOTH 1

typedef struct {
    int64_t  n_kept;     /* out: paths with kept[i] = 1 */
    /* caller device arrays, one entry per input row (same order) */
    int32_t* status;     /* PCRL_REFINE_* */
    int32_t* iters;      /* gradient steps taken */
    float*   grad;       /* final gradient norm (NaN after a miss) */
    float*   length;     /* f of Eq. 2 over the final points (NaN after a miss) */
    float*   points;     /* [n*K*3] final interaction points, NaN for k >= n_refl */
    int32_t* point_id;   /* [n*K] point (surfel) of each interaction, -2 - edge for a diffraction, -1 for
                            k >= n_refl */
    int64_t* key;        /* [n*K] label of each interaction (the edge's for a diffraction), -1 for k >= n_refl */
    int32_t* kept;       /* 1 for the unique exact paths: valid, shortest of its label sequence within its
                            (tx, rx, n_refl) group, and not inside the first Fresnel zones of a shorter kept
                            path of that group (every point within sqrt(lambda d1 d2 / (d1 + d2)) of the
                            shorter path's corresponding point, d1 / d2 its path lengths from TX / to RX) */
} PcrlRefined;

/* Refine coarse paths into exact paths (Section 2.3): per path, gradient
 * descent on the path length of Eq. 2 with every interaction point moving in
 * the tangent plane of its surfel, a ray traced through the voxel hierarchy
 * from the previous point towards each updated point to find the new point
 * and surfel, for at most max_iters steps; then the dedup of refined paths
 * (shortest per label sequence, then first-Fresnel-zone uniqueness in order
 * of increasing length).  With params->edge_of, an interaction with an edge
 * is a diffraction: its point D_k = a + t_k w stays on the edge's segment
 * [a, b] (w the unit direction), starting at the coarse point's projection,
 * and t_k steps along the derivative of the length along the edge; no ray
 * is traced to it; a ray leaving it starts r_s (the surfel radius) along its
 * direction, and a segment arriving at it is blocked only by a surfel hit
 * more than r_s before it; a step off [a, b] ends the path
 * (PCRL_REFINE_OFF_EDGE); a converged path also needs both neighbours of
 * every diffraction point outside the edge's wedge ((I - D) . n1 > 0 or
 * (I - D) . n2 > 0) and every segment arriving at one unblocked.
 *   scene  the scene the paths were traced in (its current overlay epoch is used)
 *   tx, rx device [n_tx,3] / [n_rx,3] float32, the arrays of the launch
 *   paths  a collect_paths result (device arrays; n_rows rows sorted by
 *          (tx, rx, n_refl), as collect_paths returns them): tx, rx, n_refl
 *          and points are read
 *   k_stride  K of the launch (points has k_stride entries per row)
 * Synchronous.  PCRL_EINVAL on a row with an index out of range or rows out
 * of order, an edge index out of range or an edge of zero length;
 * PCRL_EOVERFLOW if one (tx, rx, n_refl) group keeps more than 2048 paths
 * (the per-path outputs are still written). */
int refine_paths(const PcrlScene* scene, const float* tx, int32_t n_tx, const float* rx, int32_t n_rx,
                 const PcrlPaths* paths, int32_t k_stride, const PcrlRefineParams* params, PcrlRefined* out,
                 pcrl_stream_t stream);

/* ------------------------------------------------------------------------ */
/* intersection with the implicit surface of Eq. 1 (Section 2.2.1)           */
/* ------------------------------------------------------------------------ */

typedef struct {
    float     h;          /* neighbourhood radius of the averages, 0 < h <= 0.98 leaf edges;
                             <= 0 selects 0.95 leaf edges */
    float     eps;        /* |f| at or below this is an intersection; <= 0 selects 1e-3 leaf edges */
    int32_t   max_steps;  /* evaluations of f per leaf segment, <= 2^20; <= 0 selects 64 */
    int32_t   flags;      /* 0 */
    uint64_t* stats;      /* NULL, or device [2] to which the call adds the evaluations of f and the
                             leaf entries read (the caller zeroes it) */
} PcrlSdfParams;

/* First intersection of each ray with the point cloud's implicit surface
 * f(x) = (x - p(x)) . n(x) of Eq. 1 (Section 2.2.1): p and n are the averages
 * of the positions and (normalised, consistently oriented) normals of the
 * points within h of x, with weights (1 - |x - q|^2 / h^2)^4.  For every
 * occupied leaf the ray crosses within [0, t_hi], a segment one leaf diagonal
 * long is centred on the projection onto the ray of the centre of the box
 * around the points whose centre lies in that leaf, and clipped to
 * [t_lo, t_hi]; from its near end the position advances by |f| until
 * |f| <= eps (intersection there), or f changes sign between two samples
 * (intersection at the zero of their linear interpolation), or the segment
 * ends, or max_steps evaluations were spent.  Where no point lies within h
 * the position advances by h / 2 and no sign is compared across it.  The
 * result is the nearest intersection over all such leaves.
 *   o, d      device [n_rays,3] float32 origins and directions (any non-zero length)
 *   t_range   device [n_rays,2] float32 (t_lo, t_hi) per ray, or NULL for (0, inf)
 * Outputs (device, caller-owned):
 *   t         [n_rays] distance along the normalised direction, +inf if none
 *   point     [n_rays,3] o + t d (NaN if none)
 *   normal    [n_rays,3] n at the intersection (0 if none)
 *   leaf_cell [n_rays,3] int32 leaf cell whose segment held it (-1 if none), or NULL
 * A ray with a zero or non-finite direction or origin, or t_lo > t_hi, has
 * no intersection.  Asynchronous on `stream`, except that the first call on
 * a scene builds and keeps with the scene an index of each point in the leaf
 * of its centre (16 B per point twice, 4 B per entry) and waits for it.  Calls
 * of 65536 rays or more sort the rays by origin and direction first (outputs
 * stay in the caller's order).  PCRL_EINVAL on NULL arrays, out-of-range
 * parameters, or a scene holding dynamic points (update_points): the surface
 * is defined over the static points. */
int sdf_intersect(const PcrlScene* scene, const float* o, const float* d, const float* t_range, int64_t n_rays,
                  const PcrlSdfParams* params, float* t, float* point, float* normal, int32_t* leaf_cell,
                  pcrl_stream_t stream);

/* ------------------------------------------------------------------------ */
/* environment-driven coarse tracing with conical rays (Sections 2.1-2.2.4)  */
/* ------------------------------------------------------------------------ */

/* Low-resolution voxel grid of the intersectable entities (IEs, Section 2.1):
 * voxels of edge `voxel` from `origin`, dims voxels per axis, each divided
 * into dv^3 subvoxels (Table 1: voxel 0.5 m, D_v = 2). */
typedef struct {
    float   origin[3];
    float   voxel;
    int32_t dv;           /* 1..8 */
    int32_t dims[3];      /* voxels per axis; dims product * dv^3 < 2^31 */
} PcrlIeGrid;

typedef struct PcrlIes PcrlIes;           /* opaque: a scene's IE table (library-owned) */
typedef struct PcrlConeLaunch PcrlConeLaunch;  /* opaque: one cone-traced query (library-owned) */

typedef struct {
    int64_t n_ies;        /* IEs: point IEs ((subvoxel, label) pairs holding points), then edge pieces */
    int64_t n_edge_ies;   /* edge pieces (ie_add_edges) */
    int64_t n_voxels;     /* voxels of the grid */
    int64_t n_occupied;   /* voxels holding an IE */
    int64_t device_bytes;
} PcrlIeInfo;

/* Point IEs of a scene's static points (Section 2.1): the points of one label
 * whose position lies in one subvoxel, the subvoxel cell taken in FP32 as
 * floor((p - origin) * (1 / (voxel / dv))).  Each IE keeps its label, the
 * number of its points, a reception point (the mean of its positions) and a
 * normal (the normalised mean of their unit normals).  IEs are ordered by
 * (voxel, subvoxel within the voxel, label).  The scene must outlive the
 * table.  Synchronous.  PCRL_EINVAL: a point outside the grid, bad grid
 * parameters, a scene with dynamic points (update_points). */
int ie_build(PcrlScene* scene, const PcrlIeGrid* grid, pcrl_stream_t stream, PcrlIes** out);
/* Diffraction edges (Section 2: inserted by hand; Section 3: exterior edges
 * only): nE convex edge segments seg [nE,2,3] (device float32, end points
 * a, b), the outward normals of the two faces meeting at each edge normals
 * [nE,2,3] and a label per edge (label [nE], device).  Every edge is cut at
 * the subvoxel faces it crosses (cut parameters t = ((origin + k sv) - a) /
 * (b - a) per face plane, in FP32); each piece is an edge IE in the subvoxel
 * of its midpoint, with the edge's label, its midpoint as reception point,
 * the edge direction and the two normals.  Edge IEs get the indices after
 * the point IEs, ordered by (voxel, subvoxel, label, edge).  Once per table;
 * PCRL_EINVAL for edges outside the grid, zero-length edges, or a second
 * call.  Synchronous. */
int ie_add_edges(PcrlIes* ies, const float* seg, const float* normals, const uint32_t* label, int64_t n_edges,
                 pcrl_stream_t stream);
/* Sizes of an IE table (host struct).  PCRL_EINVAL for a NULL argument. */
int ie_info(const PcrlIes* ies, PcrlIeInfo* out);
/* Copy the IE table into caller device arrays of at least n_ies entries
 * (any may be NULL): key (voxel * dv^3 + local subvoxel) << 32 | label,
 * sub [n,3] subvoxel cell, label, count, pos [n,3], nrm [n,3].
 * PCRL_EINVAL for a NULL table, PCRL_EHIP if a copy fails. */
int ie_table(const PcrlIes* ies, uint64_t* key, int32_t* sub, uint32_t* label, uint32_t* count, float* pos,
             float* nrm, pcrl_stream_t stream);
int release_ies(PcrlIes* ies);

typedef struct {
    int32_t max_interactions;  /* K in [0, 8] (Table 1: 5) */
    float   half_angle;        /* cone half-angle in radians, (0, pi/4]; <= 0 -> 2.5 degrees */
    int32_t flags;             /* 0 */
    int32_t max_diffractions;  /* edge interactions per path, >= 0 (Section 3, simulation B: 1); edge pieces
                                  are targets only while a path has fewer */
} PcrlConeParams;

typedef struct {
    int64_t nodes[PCRL_MAX_REFLECTIONS + 1];       /* [k]: partial paths with k interactions kept */
    int64_t cones[PCRL_MAX_REFLECTIONS + 1];       /* [k]: conical rays they cast (one per reflection, the
                                                      exterior Keller-cone sectors per diffraction) */
    int64_t candidates[PCRL_MAX_REFLECTIONS + 1];  /* [k]: targets that passed the cone and plane tests
                                                      ([0]: the transmission phase's rays) */
    int64_t visible[PCRL_MAX_REFLECTIONS + 1];     /* [k]: of those, visible */
    int64_t records;                               /* receptions (paths reaching an RX) */
    double  ms_transmission, ms_propagation;       /* host wall clock of the two phases */
} PcrlConeStats;

/* Environment-driven coarse tracing of one query (Sections 2.2.2-2.2.4):
 *   transmission: from every TX a visibility ray towards every IE's
 *     reception point and every RX; a ray is blocked when a surfel disk
 *     (radius r_s, t > t_eps) is hit before it enters the target's subvoxel;
 *   propagation: every visible IE is an interaction; a conical ray leaves it
 *     (apex the reception point, axis the incoming direction mirrored about
 *     the IE's normal, half_angle); its axis is marched through the IE grid
 *     up to the voxel of the axis's first surfel hit (or the grid's exit) and
 *     every IE and RX in the voxels within one voxel of the march is a target
 *     when the cone meets its subvoxel's bounding sphere, its reception
 *     point lies in front of the separation plane at the apex (normal: the
 *     IE's normal on the reflected side, cleared by 1e-3 of a subvoxel) and
 *     a visibility ray reaches it;
 *   diffraction (max_diffractions > 0, edge IEs of ie_add_edges): an edge
 *     piece hit from direction d_in casts the Keller cone of the directions d
 *     with d . w = d_in . w (w the edge direction), cut into N = max(1,
 *     ceil(pi sin(beta) / half_angle)) sectors of azimuth 2 pi / N measured
 *     from the first face's normal; a sector is kept when its axis leaves
 *     the wedge (v . n1 >= 0 or v . n2 >= 0 for its direction v across the
 *     edge), and its two separation planes contain the edge at its bounding
 *     azimuths: a target lies in the sector iff (p - o) . n_lo >= 0 and
 *     (p - o) . n_hi < 0;
 *   partial paths reaching the same IE with the same label sequence are
 *     merged (the one of smallest SplitMix64 priority is kept), up to
 *     max_interactions; an RX target ends a coarse path.
 * tx, rx: device [n,3] float32 (1 <= n_tx <= 255, 0 <= n_rx <= 65535).
 * Synchronous; PCRL_EINVAL for bad arguments or IEs of another scene. */
int cone_launch(const PcrlIes* ies, const float* tx, int32_t n_tx, const float* rx, int32_t n_rx,
                const PcrlConeParams* params, pcrl_stream_t stream, PcrlConeLaunch** out);
/* Counts and timings of a cone launch (host struct).  PCRL_EINVAL for a NULL
 * argument. */
int cone_stats(const PcrlConeLaunch* launch, PcrlConeStats* out);
/* Partial paths with k (1..K) interactions, in their kept order (by TX,
 * label sequence, IE, priority): device arrays of at least nodes[k] entries
 * (any may be NULL): IE, parent (index in generation k-1, or the TX for
 * k = 1), TX, priority, polyline length TX -> reception points.
 * PCRL_EINVAL for a NULL launch or k outside 1..K. */
int cone_nodes(const PcrlConeLaunch* launch, int32_t k, int32_t* ie, int32_t* parent, int32_t* tx,
               uint64_t* prio, float* length, pcrl_stream_t stream);
/* Coarse paths: receptions grouped by (tx, rx, number of interactions,
 * labels), each group's count and its kappa rows of smallest priority
 * (Section 2.2.3), rows sorted by (tx, rx, n, labels, priority).  `ray` holds
 * k << 40 | node index of the row's last interaction (k = 0: the TX); len_poly
 * = len_unf = the polyline length TX -> reception points -> RX; points are
 * the reception points.  Synchronous; PCRL_EOVERFLOW with n_rows = rows
 * needed when capacity is too small. */
int cone_collect(PcrlConeLaunch* launch, int32_t kappa, PcrlPaths* out, pcrl_stream_t stream);
/* Refine the coarse paths of a cone_collect result of this launch (Section
 * 2.3): refine_paths in the launch's scene with its TX and RX, every
 * interaction at an edge piece a diffraction on that piece's edge (the
 * edges of ie_add_edges).  params->edge_* must be unset (the launch supplies
 * them).  Synchronous; PCRL_EINVAL for rows that are not the launch's. */
int refine_cone_paths(const PcrlConeLaunch* launch, const PcrlPaths* paths, const PcrlRefineParams* params,
                      PcrlRefined* out, pcrl_stream_t stream);
int release_cone(PcrlConeLaunch* launch);

/* ------------------------------------------------------------------------ */
/* serving: a request loop over one device-resident, incrementally           */
/* re-voxelised scene                                                         */
/* ------------------------------------------------------------------------ */

typedef struct PcrlServer PcrlServer;

typedef struct {
    int32_t max_inflight;       /* queries in flight at once; <= 0 -> 256 */
    int32_t n_streams;          /* admission rounds running concurrently; <= 0 -> 4 */
    int64_t hbm_budget_bytes;   /* device memory the queries in flight may use; <= 0 -> 64 GiB */
    int32_t max_batch;          /* queries per admission round; <= 0 -> 64 */
    int32_t kappa;              /* duplicate limit of every result; <= 0 -> 1 */
    int32_t key_mode;           /* PCRL_KEY_LABELS or PCRL_KEY_LEAVES */
    int32_t reserved;
    PcrlBatchParams batch;      /* launch shape of every round (see launch_batch) */
} PcrlServeParams;

typedef struct {
    int32_t status;             /* 0 pending, 1 running, 2 done, < 0 failed with that PCRL status */
    int32_t reserved;
    int64_t epoch;              /* scene epoch (update count) the query traced */
    int64_t n_rows;             /* result rows (done) */
    int64_t n_keys;             /* distinct coarse paths (done) */
    double  queue_ms;           /* submission -> admission */
    double  latency_ms;         /* submission -> result on the host */
} PcrlServeResult;

typedef struct {
    int64_t completed;
    int64_t pending;
    int32_t inflight;
    int32_t reserved;
    int64_t rounds;             /* admission rounds started */
    double  mean_batch;         /* queries per round */
    int64_t rays;               /* rays of completed queries */
    double  p50_ms, p99_ms, max_ms, mean_ms;   /* latency of completed queries */
    double  rays_per_s;         /* rays of completed queries / (last completion - first admission) */
    int64_t used_bytes;         /* memory estimate of the queries in flight */
} PcrlServeStats;

/* Start a server on `scene` (which must outlive it) with its own worker
 * thread and streams.  Queries are admitted while the stream budget, the
 * in-flight limit and the memory budget allow; each admission round packs
 * every admissible pending query into one launch_batch on a free stream, so
 * rounds overlap on the device (continuous batching).  Each query is
 * charged serve_query_bytes against hbm_budget_bytes while it is in flight.
 * PCRL_EINVAL for a NULL argument, PCRL_ENOMEM when the server cannot be
 * allocated, PCRL_EHIP when its streams cannot be created. */
int serve_create(PcrlScene* scene, const PcrlServeParams* params, PcrlServer** out);

/* Device bytes a query of n_tx TX, n_rx RX and these launch params holds
 * while it is in flight: what the server charges it against the memory
 * budget.  With R = n_tx * n_rays, the sum of its launch's blocks, each
 * rounded up to the allocator's size class (at least 512 B; a request above
 * 2^e and at most 2^(e+1) bytes takes 1.5 * 2^e or 2^(e+1)):
 *   records 16*C (C = record_capacity, or its default
 *     R*(K+1)*min(n_rx,8)/16 + 65536; 1 without RX); counters 4*(K+3);
 *   history 16*R*K (K > 0); statistics 128*(K+1) (PCRL_LAUNCH_STATS);
 *   ray state: 16*R, 16*R and 4*R per set, two sets for K >= 2, one for
 *     K = 1;
 *   directions 12*n_rays;
 *   PCRL_LAUNCH_COHERENT: bucket keys 2*n_rays, the bounce-0 order and its
 *     positions 4*n_rays each, bucket counts and starts 256 KiB each; and
 *     for R >= 65536 with K > 0 the later bounces' order 4*R, keys 2*R,
 *     positions 4*R and counts K*256 KiB;
 * plus 12*(n_tx + max(n_rx, 1)) + 64 bytes (unrounded) for the round's
 * antenna arrays and batch words.  The collection of a finished query is
 * not charged: rounds collect one query at a time, and it takes about 64 B
 * per reception record plus the result rows for that moment.  Host
 * arithmetic only (no device call).  PCRL_EINVAL for arguments that
 * serve_submit refuses. */
int serve_query_bytes(int32_t n_tx, int32_t n_rx, const PcrlLaunchParams* params, int64_t* bytes);

/* Queue one query (host arrays tx [n_tx,3], rx [n_rx,3]; params as in
 * launch_rays, Fibonacci directions, no hit log).  Returns at once with a
 * ticket.  PCRL_EBUSY if the query alone needs more than the memory budget
 * or the server is shutting down.  Thread-safe. */
int serve_submit(PcrlServer* server, const float* tx, int32_t n_tx, const float* rx, int32_t n_rx,
                 const PcrlLaunchParams* params, int64_t* ticket);

/* Frame update: replace the dynamic points (update_points on the server's
 * update stream).  Rounds admitted afterwards trace the new epoch; rounds in
 * flight finish on theirs.  Synchronous.  Thread-safe.  PCRL_EINVAL for a
 * NULL server; otherwise update_points' status. */
int serve_update(PcrlServer* server, const uint32_t* ids, const float* xyz, const float* normal, const uint32_t* label,
                 int64_t n);

/* State of a ticket; waits up to timeout_s seconds (0: no wait) for it to
 * finish.  Returns the query's failure status if it failed; PCRL_EINVAL for a
 * NULL argument or an unknown ticket. */
int serve_poll(PcrlServer* server, int64_t ticket, double timeout_s, PcrlServeResult* out);

/* Copy a finished query's coarse paths (rows as in collect_paths) into HOST
 * arrays of out->capacity rows.  PCRL_EOVERFLOW if they do not fit;
 * PCRL_EINVAL for a NULL argument or a ticket without a result (unknown or
 * not finished). */
int serve_result(PcrlServer* server, int64_t ticket, PcrlPaths* out);

/* Cancel a query.  A pending one leaves the queue at once; a running one
 * finishes its kernels (they cannot be interrupted) but its result is not
 * collected.  Either way serve_poll then reports status PCRL_ECANCELED; the
 * other queries are unaffected.  A finished query is left as it is.
 * PCRL_EINVAL for an unknown ticket. */
int serve_cancel(PcrlServer* server, int64_t ticket);

/* Forget a finished ticket (frees its host result).  An unknown ticket is
 * ignored; PCRL_EBUSY while the ticket is pending or running; PCRL_EINVAL
 * for a NULL server. */
int serve_release(PcrlServer* server, int64_t ticket);

/* Throughput and latency (p50 / p99 over completed queries).  PCRL_EINVAL
 * for a NULL argument. */
int serve_stats(PcrlServer* server, PcrlServeStats* out);

/* Finish every pending and running query, then stop the worker and free the
 * server.  NULL is ignored. */
int serve_destroy(PcrlServer* server);

/* Message of the last failed call on this thread ("" if none). */
const char* last_error(void);

/* Library version string. */
const char* pcrl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PCRL_H */
