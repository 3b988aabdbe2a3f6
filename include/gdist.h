/*
 * gdist: exact minimum / maximum distance between two rigidly posed triangle
 * meshes on an AMD Instinct MI355X (gfx950).  C ABI of libgdist.so.
 *
 * What is computed (gDist, Fan et al. 2024, Sec. 3, Eqs. 1-2):
 *   D_min = min over p in A, q in B of |p - q|,   D_max = max of the same,
 * over the closed triangles of the two meshes after their rigid poses, with
 * the Euclidean norm.  Penetrating meshes have D_min = 0 (Sec. 7).
 *
 * How: each mesh gets a perfect binary AABB tree whose leaves hold 1 or 2
 * triangles (the paper's f12-BVH, Sec. 6.3), built on the GPU from Morton
 * codes.  A query refits one tree into the other's frame, then expands the
 * BVH-vs-BVH pair tree in rounds whose depth adapts to the front size
 * (Alg. 1, Alg. 2, Sec. 5 "Adaptive Expansion Depth"), culling node pairs
 * with the conventional and enhanced AABB bounds of Sec. 4 against a running
 * best bound kept with integer atomics (Sec. 6.1, 6.4).  Leaf pairs go through
 * an exact FP32 triangle-triangle distance; every candidate within the FP32
 * error window of the best is re-evaluated in FP64 on the GPU.
 *
 * Conventions
 *   - Every call returns gdist_status_t; GDIST_OK = 0.  Nothing throws across
 *     the ABI.  gdist_last_error() returns a thread-local message describing
 *     the most recent failure of the calling thread.
 *   - Vertices are float32 triples (x,y,z), triangles uint32 triples of
 *     0-based vertex indices, both row-major and densely packed.
 *   - Poses are FP64 rigid transforms, world = R x + t, R row-major.
 *   - Triangle indices in results are the caller's original 0-based indices.
 *   - Points in results are in the world frame, FP64.
 *   - A context is bound to one device and is not thread-safe: calls on one
 *     context must not overlap.  Distinct contexts may be used concurrently
 *     (gdist_build calls on one device take turns inside the library).
 */
#ifndef GDIST_H
#define GDIST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gdist_ctx* gdist_ctx_t;
typedef uint64_t gdist_mesh_t; /* opaque handle; 0 is never a valid handle */

typedef enum { GDIST_MIN = 0, GDIST_MAX = 1 } gdist_mode_t;

typedef enum {
  GDIST_OK = 0,
  GDIST_E_INVALID = 1,  /* bad argument: sizes, indices, non-finite data, pose, mode */
  GDIST_E_HANDLE = 2,   /* unknown or released mesh handle, or null context       */
  GDIST_E_OOM = 3,      /* device or host allocation failed, or over the budget    */
  GDIST_E_CAPACITY = 4, /* traversal front / candidate storage exhausted after the
                           automatic retries with larger capacity                  */
  GDIST_E_DEVICE = 5,   /* a HIP runtime call failed or a kernel reported an error */
  GDIST_E_BUSY = 6      /* the context is in use by a running server               */
} gdist_status_t;

/* gdist_build flags */
#define GDIST_BUILD_DEVICE_PTR 1u /* verts / tris are device pointers (e.g. torch
                                     tensors on the context's device)            */
#define GDIST_BUILD_DEFORMABLE 2u /* keep the triangles' vertex indices (12 B per
                                     triangle) so gdist_update can move the
                                     vertices later                              */

/* gdist_result_t.flags */
#define GDIST_F_TIED 1u  /* more than one triangle pair lies within the tie
                            tolerance of the optimum; the reported pair is the
                            lexicographically smallest (tri_a, tri_b) of them   */
#define GDIST_F_ZERO 2u  /* min mode: the meshes touch or penetrate (distance 0) */

typedef struct {
  double R[9]; /* row-major rotation, orthonormal with det +1 */
  double t[3];
} gdist_pose_t;

typedef struct {
  double distance;      /* FP64 D_min or D_max, re-evaluated from the caller's FP32
                           vertices and FP64 poses                                 */
  double distance_fp32; /* the FP32 narrow-phase optimum (before FP64 re-eval)     */
  double err_bound;     /* bound on |distance - exact real-arithmetic optimum of the
                           FP32 input vertices under the FP64 poses|              */
  double point_a[3];    /* world-frame point on tri_a of mesh a                   */
  double point_b[3];    /* world-frame point on tri_b of mesh b (|pa-pb| is the
                           pair's own FP64 distance, within the tie tolerance of
                           `distance`)                                            */
  uint32_t tri_a, tri_b;/* caller's triangle indices of the reported pair         */
  uint32_t status;      /* gdist_status_t of this query (batched calls)           */
  uint32_t flags;       /* GDIST_F_*                                              */
  uint32_t n_candidates;/* triangle pairs re-evaluated in FP64                     */
  uint32_t n_ties;      /* pairs within the tie tolerance of the optimum           */
} gdist_result_t;

typedef struct {
  gdist_mesh_t a, b;    /* may be the same handle                                  */
  gdist_pose_t pa, pb;  /* world poses of a and b                                  */
  uint32_t mode;        /* gdist_mode_t                                            */
  uint32_t reserved;    /* must be 0                                               */
} gdist_query_desc_t;

typedef struct {
  uint32_t n_tris;      /* triangles                                               */
  uint32_t n_leaves;    /* 2^floor(log2 n_tris)                                    */
  uint32_t depth;       /* log2 n_leaves                                           */
  uint32_t reserved;
  uint64_t device_bytes;/* device memory held by the handle                        */
  float root_box[6];    /* local-frame root box: min xyz, max xyz                 */
} gdist_mesh_info_t;

/* Counters of the most recent gdist_query / gdist_query_batch call on a
 * context, summed over its queries.  Byte counts are algorithmic (what the
 * method must move, counted in the kernels), not hardware counters:
 *   bytes_traversal = 16 per entry popped + 24 per child box read (2^kA + 2^kB
 *                     per popped entry expanded kA levels in A, kB in B; each
 *                     sibling box once) + 16 per entry pushed;
 *   bytes_narrow    = 16 per leaf pair + 36 per triangle read (tA + tB per leaf
 *                     pair of leaves holding tA and tB triangles);
 *   bytes_reeval    = 144 per candidate (its two triangles). */
typedef struct {
  uint64_t rounds;          /* expansion rounds (grid-wide steps)                  */
  uint64_t entries_popped;  /* front entries expanded                              */
  uint64_t child_pairs;     /* node pairs whose bounds were evaluated              */
  uint64_t entries_pushed;  /* node pairs appended to the next front              */
  uint64_t leaf_pairs;      /* leaf pairs sent to the narrow phase                 */
  uint64_t tri_pairs;       /* triangle pairs given the separating-axis test      */
  uint64_t tri_full;        /* exact FP32 triangle-triangle evaluations            */
  uint64_t candidates;      /* candidates appended for FP64 re-evaluation          */
  uint64_t front_peak;      /* largest front (entries)                             */
  uint64_t bytes_refit;     /* refit: triangles read + boxes written               */
  uint64_t bytes_traversal; /* entries read + child boxes read + entries written   */
  uint64_t bytes_narrow;    /* leaf pairs read + their triangles read              */
  uint64_t retries;         /* capacity retries                                    */
  double ms_refit;          /* device time of the refit kernels (HIP events)       */
  double ms_traversal;      /* device time of the traversal + re-eval kernel       */
  double ms_total;          /* device time of the whole query (refit to result)    */
  double ms_traverse_kernel;/* summed device time of the k_traverse launches alone   */
  uint64_t traverse_launches;/* k_traverse launches (groups and capacity retries)     */
  uint64_t child_boxes;     /* child boxes read: sum of 2^kA + 2^kB over popped entries */
  uint64_t leaf_tris;       /* triangles read: sum of tA + tB over leaf pairs          */
  uint64_t bytes_reeval;    /* FP64 re-evaluation: 144 per candidate                   */
  uint64_t refit_trees;     /* trees refitted by the call                              */
} gdist_stats_t;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  Allocates the context's stream and
 * a small control block.  *out receives the context. */
gdist_status_t gdist_create(int device, gdist_ctx_t* out);

/* Destroy a context and every mesh and workspace it owns.  NULL is accepted. */
gdist_status_t gdist_destroy(gdist_ctx_t ctx);

/* Set a tunable.  Keys (value ranges are checked, E_INVALID otherwise):
 *   "front_capacity"  entries per front buffer (16 B each); a round expands at
 *                     most about a quarter of it, the surplus waits on the
 *                     spill stack
 *   "leaf_capacity"   leaf pairs per narrow-phase buffer (16 B each)
 *   "stack_capacity"  spill-stack entries (16 B each), initial value (2^27); doubles on
 *                     overflow up to 2^31
 *   "cand_capacity"   FP64 candidates (24 B each)
 *   "max_retries"     capacity doublings before GDIST_E_CAPACITY
 *   "group_size"      queries of a batch traversed together per launch (0 = all);
 *                     smaller groups keep their trees' boxes in the caches
 *   "expand_budget"   C of the adaptive depth rule (largest k with 4^k n < C;
 *                     default 2^22)
 *   "k_cap"           largest expansion depth per side and round (1..8, default 8)
 *   "kappa"           FP32 inflation: delta = kappa * 2^-24 * M
 *   "blocks_per_cu"   persistent-kernel workgroups per compute unit
 *   "bounds"          0 = enhanced upper bounds (paper Sec. 4), 1 = conventional
 *                     bounds only (the paper's ablation)
 *   "warm_start"      1 = temporal coherence (paper Sec. 7): the context keeps
 *                     the pair each query reported, per (mesh a, mesh b, mode),
 *                     and the next query of the same meshes evaluates that pair
 *                     first to seed its bound (frame sequences); results do not
 *                     change.  0 (default) forgets the pairs.  gdist_query and
 *                     the batch calls use it; a server does not record pairs
 *   "memory_budget"   device bytes the context may hold (0 = unlimited)
 *   "stats"           1 (default) = traversals count the work statistics that
 *                     gdist_last_stats reports (entries, child pairs, leaf and
 *                     triangle pairs, bytes); 0 = they do not (a few per cent
 *                     faster; those fields then read 0, rounds and the front
 *                     peak are still counted).  Results do not change.
 *   "cand_buffer"     candidates each wave holds in its LDS buffer before they
 *                     go to memory (0..128, default 128; 0 = every candidate
 *                     goes to memory at once).  A full buffer is pruned
 *                     against the query's current bound, then flushed.
 *                     Results do not change (small values exercise the
 *                     pruning and flushing paths).
 */
gdist_status_t gdist_set_option(gdist_ctx_t ctx, const char* key, double value);

/* Route the context's device allocations through the caller (for example a
 * framework's caching allocator): alloc(bytes, user) returns device memory or
 * NULL (then the call that needed it returns E_OOM), free_(ptr, user) releases
 * it.  Both NULL restores hipMalloc / hipFree.  Only on a context that holds
 * no device memory yet (right after gdist_create), else E_INVALID. */
gdist_status_t gdist_set_allocator(gdist_ctx_t ctx, void* (*alloc)(size_t, void*), void (*free_)(void*, void*),
                                   void* user);

/* ------------------------------------------------------------------ meshes */

/* Build the f12 tree of a mesh on the device (Morton keys, radix sort, leaf
 * emit, level reduction; Sec. 6.3).  The caller's arrays are copied; the
 * handle owns its device data until gdist_release.  Zero-area triangles are
 * accepted.  E_INVALID: n_tris == 0 or >= 2^31, n_verts == 0, an index >=
 * n_verts, or a non-finite vertex coordinate (checked on the device, reported
 * after the build's one host wait; nothing is kept).  E_DEVICE: a HIP error,
 * or a bounded wait of the sort's look-back gave up (nothing is kept).
 * Synchronous. */
gdist_status_t gdist_build(gdist_ctx_t ctx, const float* verts, uint32_t n_verts,
                           const uint32_t* tris, uint32_t n_tris, uint32_t flags,
                           gdist_mesh_t* out);

/* Deformable meshes (the method covers deformable models, Sec. 1, by refitting
 * its trees each frame, Sec. 7): give a mesh built with GDIST_BUILD_DEFORMABLE
 * new vertex positions (same n_verts, same triangles) and refit its tree in
 * place: every box is recomputed tight from the new triangles; the leaf
 * order of the original build is kept (no new sort), so a large deformation
 * may leave the tree less effective at culling but never changes a result.
 * verts: n_verts x 3
 * floats, host memory or (flags = GDIST_BUILD_DEVICE_PTR) device memory,
 * copied.  E_INVALID: a mesh built without GDIST_BUILD_DEFORMABLE, n_verts
 * other than at build time, a non-finite coordinate (the mesh is then left
 * unchanged), unknown flags.  Synchronous. */
gdist_status_t gdist_update(gdist_ctx_t ctx, gdist_mesh_t mesh, const float* verts, uint32_t n_verts,
                            uint32_t flags);

/* Release a mesh handle and its device memory.  Queued asynchronous batches
 * of the context complete first, so a handle still in flight is released
 * after the work that uses it; the warm-start pairs of the mesh are dropped.
 * E_BUSY while a server runs on the context. */
gdist_status_t gdist_release(gdist_ctx_t ctx, gdist_mesh_t mesh);

gdist_status_t gdist_mesh_info(gdist_ctx_t ctx, gdist_mesh_t mesh, gdist_mesh_info_t* out);

/* Copy a mesh's device tree to host memory (any pointer may be NULL):
 *   boxes  float[2 * n_leaves][6]: node boxes in heap order (node 1 = root,
 *          node n_leaves + j = leaf j; entry 0 unused), local frame;
 *   tris   float[n_tris][9]: triangle vertices in leaf order;
 *   orig   uint32[n_tris]: caller's index of each leaf-order triangle. */
gdist_status_t gdist_mesh_export(gdist_ctx_t ctx, gdist_mesh_t mesh, float* boxes,
                                 float* tris, uint32_t* orig);

/* ----------------------------------------------------------------- queries */

/* One query, one launch sequence, synchronous.  E_INVALID for a pose that is
 * not a proper rotation (|R^T R - I|_inf > 1e-6 or det R < 0), a non-finite
 * pose, or an unknown mode.  E_HANDLE for an unknown handle. */
gdist_status_t gdist_query(gdist_ctx_t ctx, gdist_mesh_t a, gdist_mesh_t b,
                           const gdist_pose_t* pa, const gdist_pose_t* pb,
                           gdist_mode_t mode, gdist_result_t* out);

/* gdist_query for callers that cannot allocate device memory (a serving loop
 * with a fixed footprint, code that must not call hipMalloc): the same
 * kernels and the same result as gdist_query, but every device buffer of the
 * query comes from one fixed array of 128 MiB that the library holds on each
 * GPU it runs on (set up by gdist_create, kept until the process ends); the
 * call allocates no device or pinned memory.  Limits: the smaller mesh of the
 * pair (the one refitted) has fewer than 2^20 triangles (E_INVALID
 * otherwise, before anything runs); the traversal runs on at most 64
 * workgroups with a fixed spill stack of 2^20 pairs, and a query that needs
 * more storage returns E_CAPACITY (out->status too) where gdist_query would
 * grow its storage.  All calls on one GPU share its array, which keeps the
 * last call's contents: calls that overlap on one GPU (several threads or
 * contexts of that device) race and must be serialised by the caller.
 * E_BUSY while a server runs on the context.  Synchronous. */
gdist_status_t gdist_query_noalloc(gdist_ctx_t ctx, gdist_mesh_t a, gdist_mesh_t b,
                                   const gdist_pose_t* pa, const gdist_pose_t* pb,
                                   gdist_mode_t mode, gdist_result_t* out);

/* n queries in one persistent launch (one refit launch set, one traversal
 * launch, one re-evaluation).  Each query's result equals what gdist_query
 * returns for it alone.  out[i].status carries the per-query status (a query
 * that could not complete, e.g. after E_CAPACITY, holds that status and a NaN
 * distance); the call returns the first non-OK status, or OK.  Synchronous. */
gdist_status_t gdist_query_batch(gdist_ctx_t ctx, uint32_t n, const gdist_query_desc_t* q,
                                 gdist_result_t* out);

/* One mesh against n others (the paper's future work, Sec. 8): mesh a at
 * pose pa against b[i] at pose pb[i], all in one batched call, result i in
 * out[i] (same per-query statuses and return value as gdist_query_batch).
 * b, pb and out hold n entries each, caller-owned.  Synchronous. */
gdist_status_t gdist_query_one_to_many(gdist_ctx_t ctx, gdist_mesh_t a, const gdist_pose_t* pa, uint32_t n,
                                       const gdist_mesh_t* b, const gdist_pose_t* pb, gdist_mode_t mode,
                                       gdist_result_t* out);

/* gdist_query_batch without waiting: the queries are validated (E_HANDLE /
 * E_INVALID now) and copied, then run in submission order by a worker thread
 * of the context after everything already queued on hip_stream (a hipStream_t,
 * or NULL for no ordering).  out must stay valid until gdist_sync returns;
 * it is written when the batch completes.  Any other call on the context
 * (except gdist_mesh_info and further async submissions) first waits for the
 * queued batches.  E_BUSY while a server runs on the context. */
gdist_status_t gdist_query_batch_async(gdist_ctx_t ctx, uint32_t n, const gdist_query_desc_t* q,
                                       gdist_result_t* out, void* hip_stream);

/* Wait for every batch queued with gdist_query_batch_async; then, if
 * hip_stream is not NULL, make later work on that stream wait for the
 * context's device work too.  Returns the first failure among the completed
 * batches since the previous gdist_sync (with its message), or OK. */
gdist_status_t gdist_sync(gdist_ctx_t ctx, void* hip_stream);

/* Counters of the most recent query call on this context. */
gdist_status_t gdist_last_stats(gdist_ctx_t ctx, gdist_stats_t* out);

/* ----------------------------------------------------------------- serving */
/* Continuous batching (not in the paper; it serves queries of different
 * sizes as they arrive).  A worker thread owns the context's stream and runs
 * device steps of a few traversal rounds over all queries in flight.  Between
 * steps it admits queued queries into free slots while the shared traversal
 * storage has room, and it completes every query whose traversal has drained:
 * FP64 re-evaluation, then the result is queued for gdist_server_poll.  A
 * query's result equals what gdist_query returns for it alone.  While a
 * server runs, other query calls on its context return GDIST_E_BUSY. */
typedef struct gdist_server* gdist_server_t;

/* A device step is a fixed launch sequence after admission: the traversal
 * (at most rounds_per_step rounds), per-slot live counts, completion flags,
 * FP64 re-evaluation of the completed slots, one copy of the step's report to
 * pinned host memory.  By default the server builds it once as a HIP graph
 * (again after the spill stack grows) and replays it every step: one graph
 * launch and one host wait per step.  With this flag it launches the kernels
 * one by one (same results). */
#define GDIST_SERVER_DIRECT 1u

typedef struct {
  uint32_t max_slots;       /* queries in flight, 1..512 (0 = 64)                        */
  uint32_t rounds_per_step; /* traversal rounds per device step while queries wait to be
                               admitted (0 = 4); with none waiting a step runs up to 64
                               rounds, so a lone query usually completes in one step      */
  uint64_t front_capacity;  /* entries per front and per leaf-pair buffer (0 = 2^25, at
                               most 2^28); a step's rounds expand at most about a
                               quarter of it, the surplus waits on the spill stack       */
  uint32_t cand_per_slot;   /* FP64 candidates per query (0 = 2^18, at most 2^26); a
                               query that needs more is re-run alone (see fallbacks)    */
  uint32_t max_tris;        /* largest mesh a query refits, i.e. the smaller mesh of
                               its pair (0 = largest mesh built on the context when the
                               server starts); sizes the per-slot box storage            */
  uint32_t flags;           /* GDIST_SERVER_DIRECT, or 0                                 */
  uint64_t stack_capacity;  /* spill-stack entries (0 = 2^26, at most 2^31); doubles when
                               one query overflows it alone; beyond 2^31 the query is
                               re-run alone (see fallbacks)                              */
} gdist_server_config_t;

typedef struct {
  uint64_t tag;             /* caller's tag from gdist_server_submit                      */
  uint64_t t_submit_ns;     /* steady clock (CLOCK_MONOTONIC) at submit                   */
  uint64_t t_done_ns;       /* steady clock when the result reached host memory           */
  gdist_result_t result;    /* result.status != GDIST_OK for a failed query              */
} gdist_completion_t;

typedef struct {
  uint64_t submitted, admitted, completed, failed, requeued;
  uint64_t steps, rounds;
  uint32_t active, pending; /* at the time of the call                                    */
  uint32_t concurrency;     /* current admission limit (halved after a storage overflow) */
  uint32_t fallbacks;       /* queries re-run alone through gdist_query's growing storage */
  double device_ms;         /* device time of all steps' launch sequences (HIP events)    */
  uint64_t graph_steps;     /* steps replayed from the captured graph                     */
  uint32_t graph_mode;      /* 1: steps replay the step graph; 0: kernels launched one by
                               one (GDIST_SERVER_DIRECT, or the runtime refused the graph) */
  uint32_t reserved;
} gdist_server_stats_t;

/* Start a server on ctx (config may be NULL for defaults).  Allocates all of
 * its device storage up front (only the spill stack grows later, as
 * stack_capacity says).  E_BUSY if ctx already has a server. */
gdist_status_t gdist_server_start(gdist_ctx_t ctx, const gdist_server_config_t* config, gdist_server_t* out);

/* Queue one query.  Handles, poses and mode are validated here (E_HANDLE /
 * E_INVALID); E_CAPACITY if the smaller mesh of the pair exceeds max_tris.
 * Thread-safe. */
gdist_status_t gdist_server_submit(gdist_server_t srv, const gdist_query_desc_t* q, uint64_t tag);

/* Move up to max finished queries into out[]; returns how many.  Thread-safe,
 * non-blocking. */
uint32_t gdist_server_poll(gdist_server_t srv, gdist_completion_t* out, uint32_t max);

gdist_status_t gdist_server_stats(gdist_server_t srv, gdist_server_stats_t* out);

/* Stop the worker (queries still queued or in flight are dropped), free the
 * server's storage and release the context. */
gdist_status_t gdist_server_stop(gdist_server_t srv);

/* Message for the most recent failure on the calling thread ("" if none). */
const char* gdist_last_error(void);

/* ------------------------------------------------------ device self-checks */

/* Evaluate the device box-bound routine on n box pairs (host arrays).
 * a, b: float[n][6]; out: float[n][4] = conventional lower bound of the min,
 * enhanced upper bound of the min, conventional upper bound of the max,
 * enhanced lower bound of the max (Sec. 4).  Exposed for testing. */
gdist_status_t gdist_eval_box_bounds(gdist_ctx_t ctx, uint32_t n, const float* a,
                                     const float* b, float* out);

/* Evaluate the device triangle-triangle routines on n pairs (host arrays).
 * p, q: float[n][9]; mode 0 = min, 1 = max.  out32: FP32 routine; out64: FP64
 * routine on the same inputs widened to double.  Exposed for testing. */
gdist_status_t gdist_eval_tri_tri(gdist_ctx_t ctx, uint32_t n, const float* p, const float* q,
                                  uint32_t mode, float* out32, double* out64);

#ifdef __cplusplus
}
#endif
#endif /* GDIST_H */
