/*
 * ptp.h: C ABI of the MI355X Parallel Toplesets Propagation library.
 *
 * The problem (paper Sec. 3.1): a triangle mesh T = (V, E, F) and a source set
 * S of vertices; compute for every vertex v the geodesic distance d_S(v) to S.
 * The method (Sec. 4): group the vertices into topological level sets V_r
 * (BFS hop distance r from S, Sec. 4.1), then repeatedly recompute, for every
 * vertex of the update band B_{i_k}^{j_k} (the toplesets i_k .. j_k), its
 * distance from the previous iteration's map with the planar Fast-Marching
 * update over its incident triangles (Sec. 3.2 update_step, Sec. 4.2); the
 * band grows by one topleset per iteration (Eq. upper_band) and drops its
 * first topleset once every value there changed by a relative amount below
 * the tolerance (Eq. lower_band).
 *
 * Conventions for every entry point
 *   - Device pointers are HIP device addresses on the current device; the
 *     caller owns them (typically torch tensors) and keeps them alive until
 *     the work enqueued on `stream` has finished.  The library never frees
 *     caller memory.  `stream` is a hipStream_t passed as void* (NULL = the
 *     null stream).
 *   - Inputs are read only.  Outputs are fully overwritten on PTP_OK and on
 *     PTP_ENOCONV; on any other status their contents are undefined.
 *   - Errors are reported by status code only; nothing throws or aborts
 *     across this boundary.  ptp_last_error() gives a message per plan.
 *   - A plan may be used by one host thread at a time.
 *
 * Layouts
 *   V      float32 [n][3]   vertex coordinates, row-major (x, y, z).
 *   F      int32   [f][3]   triangle vertex ids, 0 <= id < n.
 *   S      int32   [m]      source vertex ids, distinct, 0 <= id < n, m >= 1.
 *   dist   float32 [n]      distance to S; +inf where no path exists.
 *   label  int32   [n]      Voronoi label (Sec. 5.3): index into S of the
 *                           source at the root of the vertex's chain of
 *                           parents in the final map, the parent being the
 *                           vertex its value comes from under its best
 *                           triangle (the smaller input of a planar value,
 *                           the other end of an edge update; equal candidates:
 *                           the smaller vertex id; only parents before the
 *                           vertex in (distance, id) order); -1 where
 *                           unreachable.
 */
#ifndef PTP_MI355X_H
#define PTP_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PTP_OK = 0,
    PTP_EINVAL = -1,        /* bad argument, index out of range, non-finite
                               coordinate, duplicate or missing source, tol <= 0 */
    PTP_ENOMEM = -2,        /* workspace too small                            */
    PTP_EDEVICE = -3,       /* a HIP call failed or a kernel reported a fault  */
    PTP_ENOCONV = -4,       /* iteration cap reached before every topleset
                               retired; the distances so far are written       */
    PTP_EUNSUPPORTED = -5   /* sizes beyond what the library handles          */
} ptp_status;

/* Band rules (ptp_options.band_rule). */
#define PTP_BAND_PAPER 0      /* Eq. upper_band / Eq. lower_band: the band grows by one
                                 topleset per iteration and drops its first one when
                                 every value there changed by less than tol (Sec. 4.2) */
#define PTP_BAND_FIXED_HALF 1 /* the fixed band [max(1, floor((k+1)/2)), min(k, rho-1)]
                                 of the complexity analysis (Sec. 6), run for
                                 2 rho - 3 iterations (V_r is final after 2r - 1
                                 iterations on a regular mesh whose toplesets grow);
                                 tol is not used */
#define PTP_BAND_JACOBI 2     /* every topleset from 1 on, until an iteration changes
                                 no value: the fixed point d = min(d, U(d)) the
                                 iteration approximates; tol is not used */

typedef struct {
    float tol;              /* epsilon of Eq. lower_band, > 0                   */
    int32_t max_iters;      /* iteration cap; 0 -> 4 * rho + 16 (PTP_BAND_JACOBI:
                               64 * rho + 256)                                  */
    int32_t window;         /* > 0: the band holds at most `window` toplesets
                               and the ones pushed below it stop updating;
                               0: unbounded, the paper's rule                  */
    int32_t want_labels;    /* nonzero: compute Voronoi labels                  */
    int32_t workgroups;     /* persistent grid size; 0 -> chosen by the library */
    int32_t lds_bfs_max;    /* meshes of at most this many vertices run their
                               BFS in one workgroup with LDS bitmaps: 0 -> as
                               large as the device's LDS allows, -1 -> never
                               (tuning only: the toplesets are the same)     */
    int32_t band_rule;      /* PTP_BAND_*; 0 is the paper's rule              */
} ptp_options;

typedef struct {
    int32_t iterations;     /* K: iterations run                               */
    int32_t n_toplesets;    /* rho: number of toplesets (reachable levels)     */
    int32_t reachable;      /* vertices in some topleset                        */
    int32_t workgroups;     /* persistent grid size used                        */
    int64_t vertex_updates; /* U = sum over k of |B_{i_k}^{j_k}|  (Eq.
                               n_operations without the constant)             */
    int32_t certify_rounds; /* warm start: certification sweeps (0 otherwise)  */
    int32_t certify_rejected; /* warm start: bounds the certification withdrew */
    float ms_prepare;       /* device time of the last prepare (events on its
                               stream), -1 when it was not timed               */
    float ms_run;           /* device time of the last run, -1 when not timed
                               (a run enqueued under graph capture)            */
    float ms_mesh_begin;    /* this mesh's iteration began / ended, ms after
                               the first mesh of the launch began (device     */
    float ms_mesh_end;      /* clock); -1 when it did not run                   */
    int64_t evaluated_updates; /* the vertex updates whose triangles were
                               evaluated: an update of a vertex that was
                               updated in the previous iteration and none of
                               whose neighbours changed there keeps its value
                               without evaluation (the result would be the
                               same); vertex_updates counts every update of
                               the band                                      */
} ptp_stats;

typedef struct ptp_plan ptp_plan;

/* Create a plan for a mesh with n_vertices, n_faces and n_sources.  `opt` is
 * copied; NULL means tol = 1e-3 (the paper's epsilon) and defaults elsewhere.
 * Sizes: 1 <= n_vertices < 2^31 / 4, 0 <= n_faces, 6 * n_faces < 2^31,
 * 1 <= n_sources <= n_vertices.  Returns PTP_EINVAL / PTP_EUNSUPPORTED on
 * bad sizes or options; *out is NULL then. */
ptp_status ptp_plan_create(ptp_plan **out, int32_t n_vertices, int32_t n_faces,
                           int32_t n_sources, const ptp_options *opt);

/* Device workspace the plan needs, in bytes.  The caller allocates it (any
 * 256-byte aligned device buffer) and passes the same buffer to
 * ptp_prepare and every later ptp_run of this plan. */
ptp_status ptp_workspace_bytes(const ptp_plan *plan, size_t *bytes);

/* Validate the mesh and build, on the device: the vertex-triangle incidence,
 * the toplesets by BFS from S (Sec. 4.1) and the reorder of coordinates and
 * incidence into topleset order (Sec. 4.3).  Synchronises `stream` once to
 * read the validation result and the number of toplesets.  Returns
 * PTP_EINVAL for out-of-range face or source ids, non-finite coordinates or
 * duplicate sources; PTP_ENOMEM if work_bytes is too small. */
ptp_status ptp_prepare(ptp_plan *plan, const float *dV, const int32_t *dF,
                       const int32_t *dS, void *dWork, size_t work_bytes, void *stream);

/* Run the PTP iteration on a prepared plan and write dist (and label when
 * dLabel is non-NULL and the plan wants labels) in the caller's vertex
 * order.  Enqueues work only: no host synchronisation, no allocation.  The
 * outcome (PTP_OK / PTP_ENOCONV / device fault) is read by ptp_get_stats
 * after the stream has drained. */
ptp_status ptp_run(ptp_plan *plan, float *dDist, int32_t *dLabel, void *stream);

/* ptp_prepare + ptp_run + synchronise; fills *stats when non-NULL.  Returns
 * the run's outcome (PTP_OK, PTP_ENOCONV, ...). */
ptp_status ptp_solve(ptp_plan *plan, const float *dV, const int32_t *dF, const int32_t *dS,
                     void *dWork, size_t work_bytes, float *dDist, int32_t *dLabel,
                     ptp_stats *stats, void *stream);

/* ptp_solve for callers that cannot allocate device memory (code that must
 * not call hipMalloc: tight serving loops, harnesses that forbid it).  The
 * workspace is not a caller buffer but a fixed scratch array of
 * ptp_noalloc_scratch_bytes() (64 MiB) that the library holds on every
 * device it runs on until the process ends; this call allocates nothing.
 * The caller still owns V, F, S, dist and label.  PTP_ENOMEM (with a message
 * naming both sizes) when ptp_workspace_bytes of the plan exceeds the
 * scratch, that is above roughly 200k vertices.  Every call on a device
 * shares that device's scratch, and the plan keeps using it for later
 * ptp_run calls: calls that overlap on one device (other threads, other
 * streams, runs still in flight) race and give undefined results; the
 * synchronisation at the end of this call makes consecutive calls on one
 * thread safe.  Everything a solve reads from the scratch is written first
 * by the same solve, so earlier contents never matter. */
ptp_status ptp_solve_noalloc(ptp_plan *plan, const float *dV, const int32_t *dF,
                             const int32_t *dS, float *dDist, int32_t *dLabel,
                             ptp_stats *stats, void *stream);

/* Size of the fixed scratch of ptp_solve_noalloc, in bytes. */
size_t ptp_noalloc_scratch_bytes(void);

/* Synchronise the plan's last stream and report the last run: fills *stats
 * and returns its outcome. */
ptp_status ptp_get_stats(ptp_plan *plan, ptp_stats *stats);

/* The same iteration in float64 (the paper runs single and double precision,
 * Sec. 5.1): coordinates are the float32 input promoted exactly, distances and
 * the update in double (correctly rounded square root and division).
 * dDist: double [n], caller order.  Distances only: PTP_EUNSUPPORTED when the
 * plan wants labels.  Enqueues work only, like ptp_run; ptp_get_stats
 * reports it. */
ptp_status ptp_run_f64(ptp_plan *plan, double *dDist, void *stream);

/* Farthest point sampling (Sec. 5.3; cost analysis in the appendix on the
 * sampling's complexity): starting from the sources S[0, n_initial), add
 * n_sources - n_initial vertices one at a time, each the reachable vertex
 * farthest from the current set by the distance map of that set (largest
 * float32 distance, smallest vertex id on a tie).
 *   plan      single-mesh plan created with n_sources = the final count m and
 *             want_labels = 0 (PTP_EUNSUPPORTED otherwise)
 *   dS        int32 [m] device: S[0, n_initial) in, S[n_initial, m) out
 *   warm      0: every map from +inf (the paper's use); 1: every map after the
 *             first starts from the previous one, which bounds the enlarged
 *             set's map from above (no certification is needed: each of its
 *             values was set to the planar update of an earlier, larger map,
 *             and an added source only lowers updates)
 *   dDist     float [n] device: the map of the final set S[0, m)
 *   dRadius   float [m - n_initial] device or NULL: distance of each sample
 *             when it was chosen
 *   dSteps    int64 [2 (m - n_initial + 1)] device or NULL: (K, U) of every map
 * Prepares the plan (validates the mesh and S[0, n_initial)) and enqueues the
 * whole loop without host round trips, then synchronises.  PTP_EINVAL when
 * fewer than m vertices are reachable.  Afterwards the plan is prepared for
 * S[0, m) and ptp_get_stats reports the last map. */
ptp_status ptp_fps(ptp_plan *plan, const float *dV, const int32_t *dF, int32_t *dS, int32_t n_initial,
                   void *dWork, size_t work_bytes, int32_t warm, float *dDist, float *dRadius,
                   int64_t *dSteps, void *stream);

/* One Lloyd step towards a centroidal Voronoi tessellation on the geodesic
 * Voronoi cells of a labelled run (the paper proposes its method for
 * centroidal Voronoi tessellations, Sec. 7; cells from multi-source labels,
 * Sec. 5.3).  Cell s holds the vertices labelled s; vertex v weighs A_v, a
 * third of the area of its incident triangles; the centroid of s is
 * sum A_v x_v / sum A_v; the new generator is the vertex of the cell nearest
 * (Euclidean) to it, smallest id on a tie; an empty cell keeps its generator.
 * Sums and distances in float64, reduced in a fixed order (deterministic).
 *   plan      single-mesh plan; the step reads the V, F and S given to its
 *             last ptp_prepare (validated there; the caller keeps them alive)
 *   dLabel    int32 [n] labels, caller order (from ptp_run of this plan)
 *   dSout     int32 [m] the new generators (may not be the prepared S)
 *   dCentroid double [m][4] device or NULL: (x, y, z, cell area)
 * Enqueues work only. */
ptp_status ptp_lloyd_step(ptp_plan *plan, const int32_t *dLabel, int32_t *dSout, double *dCentroid,
                          void *stream);

/* The parents behind the labels of the last run, which must have computed
 * labels (PTP_EINVAL otherwise): parent[v] = the caller id of the vertex
 * v's final value comes from (see `label` above), v itself for a source, -1
 * where unreachable.  Following parents from any vertex descends the final
 * map to its nearest source along a chain of vertices (a discrete geodesic
 * path, Sec. 5.3).  dParent int32 [n] device, caller order.  Asynchronous. */
ptp_status ptp_get_parents(ptp_plan *plan, int32_t *dParent, void *stream);

/* Copy the topleset order of the last prepare into caller DEVICE buffers:
 * perm[n] = caller vertex id at each position of the order (by topleset, then
 * ascending id; unreachable vertices last), offsets[rho + 1] = start of each
 * topleset in that order.  Either pointer may be NULL.  Asynchronous on
 * `stream`. */
ptp_status ptp_get_order(ptp_plan *plan, int32_t *dPerm, int32_t *dOffsets, void *stream);

/* Copy the retirement iteration of each topleset of the last run into a
 * HOST buffer retire[rho]: the last iteration that updated V_r (0 for V_0,
 * -1 if it never retired).  Synchronises. */
ptp_status ptp_get_schedule(ptp_plan *plan, int32_t *hRetire);

/* Replace the band cap for the following runs (the `window` option:
 * > 0 caps the band at `window` toplesets, the ones pushed below it stop
 * updating; 0 is the paper's unbounded band).  Unlike a schedule this
 * changes results; it exists so that a caller can tune it against the
 * unbounded run.  PTP_EINVAL for a negative value. */
ptp_status ptp_set_window(ptp_plan *plan, int32_t window);

/* Number of toplesets found by the last prepare (host value). */
int32_t ptp_n_toplesets(const ptp_plan *plan);

const char *ptp_last_error(const ptp_plan *plan);
void ptp_plan_destroy(ptp_plan *plan);

/* ------------------------------------------------------------------------
 * Batches: many meshes (or one mesh with many source sets) solved in one
 * persistent launch.  The meshes are concatenated in the caller's arrays;
 * each descriptor gives where its rows start.  Ids inside a mesh (face
 * entries, sources) are local to that mesh.  Several descriptors may share
 * the same vertex and face rows with different sources and output offsets
 * (many source sets on one mesh).  Every mesh is solved exactly as
 * ptp_solve would solve it alone with the same options: the batch changes
 * the schedule, never the result.
 * ---------------------------------------------------------------------- */
typedef struct {
    int64_t v_off;          /* first row of this mesh in V                      */
    int64_t f_off;          /* first row in F                                  */
    int64_t s_off;          /* first entry in S                                */
    int64_t out_off;        /* first entry of its distances / labels in the outputs */
    int32_t n_vertices, n_faces, n_sources, reserved;
} ptp_mesh;

/* Work distribution of a batch over the persistent grid (tuning only; the
 * results do not depend on it).  Meshes are split by vertex count into small
 * (< small_limit, one workgroup each), medium and large (>= large_limit);
 * medium and large meshes run on groups of medium_group / large_group
 * workgroups.  Zero fields take the library's defaults. */
typedef struct {
    int32_t workgroups;     /* persistent grid size                            */
    int32_t small_limit;
    int32_t large_limit;
    int32_t medium_group;
    int32_t large_group;
    int32_t xcd_pack;       /* > 0: place each group of at most max(32,
                               xcd_pack) workgroups on one XCD (launch
                               index i runs on XCD i mod 8; such a group
                               then exchanges its data through that XCD's
                               L2); -1: consecutive indices                */
} ptp_schedule;

typedef struct ptp_batch ptp_batch;

/* Create a batch plan.  `meshes` (host, [count]) is copied.  Sizes as for
 * ptp_plan_create, per mesh; totals must stay below 2^29 vertices and 2^31 / 6
 * faces.  Returns PTP_EINVAL on bad descriptors or options. */
ptp_status ptp_batch_create(ptp_batch **out, const ptp_mesh *meshes, int32_t count,
                            const ptp_options *opt);
ptp_status ptp_batch_workspace_bytes(const ptp_batch *batch, size_t *bytes);

/* Validate every mesh and build toplesets and reorders for all of them
 * (Sec. 4.1, 4.3) in one persistent BFS launch.  dV / dF / dS are the
 * concatenated arrays (rows addressed by the descriptors).  Synchronises
 * once.  PTP_EINVAL if any mesh is invalid (ptp_batch_get_stats then reports
 * which). */
ptp_status ptp_batch_prepare(ptp_batch *batch, const float *dV, const int32_t *dF,
                             const int32_t *dS, void *dWork, size_t work_bytes, void *stream);

/* Run PTP on every mesh in one persistent launch; dDist / dLabel are indexed
 * by out_off + local vertex id.  Enqueues work only (capture-safe: kernel
 * launches only). */
ptp_status ptp_batch_run(ptp_batch *batch, float *dDist, int32_t *dLabel, void *stream);

/* ptp_run_f64 for a batch: dDist double [out_len], indexed like ptp_batch_run. */
ptp_status ptp_batch_run_f64(ptp_batch *batch, double *dDist, void *stream);

/* Synchronise and report: per-mesh stats and status (host arrays [count],
 * either may be NULL).  Returns PTP_OK, or the first non-OK mesh status. */
ptp_status ptp_batch_get_stats(ptp_batch *batch, ptp_stats *hStats, int32_t *hStatus);

/* ptp_get_parents for a batch: dParent [out_len], indexed like ptp_batch_run,
 * local (per mesh) vertex ids. */
ptp_status ptp_batch_get_parents(ptp_batch *batch, int32_t *dParent, void *stream);

/* ptp_set_window for a batch (one cap for every mesh). */
ptp_status ptp_batch_set_window(ptp_batch *batch, int32_t window);

/* Replace / read the work distribution used by the next prepare and run. */
ptp_status ptp_batch_set_schedule(ptp_batch *batch, const ptp_schedule *schedule);
ptp_status ptp_batch_get_schedule(const ptp_batch *batch, ptp_schedule *schedule);

/* Try each candidate schedule (host array [n]) on the prepared batch: one
 * run each after a warm-up, timed with device events on `stream`; keep the
 * fastest and write its index and time per candidate (host, [n] ms).  The
 * outputs are overwritten by the runs.  Synchronises. */
ptp_status ptp_batch_autotune(ptp_batch *batch, const ptp_schedule *candidates, int32_t n,
                              float *dDist, int32_t *dLabel, float *hMs, int32_t *best,
                              void *stream);

const char *ptp_batch_last_error(const ptp_batch *batch);
void ptp_batch_destroy(ptp_batch *batch);

/* ------------------------------------------------------------------------
 * Learned warm start (an extension; the paper starts every vertex but the
 * sources at +inf).  A small network predicts each vertex's distance from
 * local geometry and its BFS hop count; the prediction, inflated, is
 * certified into an upper bound and the PTP iteration starts from it.  The
 * min-relaxation of Sec. 4.2 descends from any upper bound of the fixed point
 * to that fixed point, and the band and retirement rules (Eq. upper_band,
 * Eq. lower_band) stay as in the plain run with one addition: V_r retires no
 * earlier than iteration r + 1.  Labels are not computed on this path.
 *
 * Certification: every vertex whose bound w(v) is below the planar update
 * U(w)(v) from its neighbours' bounds (Sec. 3.2 update_step) loses its bound
 * (+inf), repeated until nothing changes; the result satisfies w >= U(w) with
 * w = 0 on S, a supersolution, hence w >= the fixed point.  Any input is
 * therefore safe: a bad prediction costs time, never accuracy.
 *
 * Network (one float32 parameter vector of PTP_MLP_PARAMS values):
 *   x  = (f1 / l, hop, f3 * l) / (64, 64, 1)
 *        l   = mean edge length of the mesh (each triangle's three edges)
 *        f1  = Euclidean distance to the nearest source
 *        hop = topleset index r of the vertex (Sec. 4.1)
 *        f3  = signed discrete mean curvature: H = |K| / 2 with the sign of
 *              K . n, K the cotangent Laplacian of the position over the
 *              barycentric area (a third of the incident triangle areas),
 *              n the sum of the incident (unnormalised) face normals
 *   h1 = gelu(x W1 + b1), h2 = gelu(h1 W2 + b2), o = h2 . W3 + b3
 *   d^ = 64 l softplus(o)                      gelu with the exact erf
 *   layout [W1 3x64 | b1 64 | W2 64x64 | b2 64 | W3 64 | b3 1], matrices
 *   input-major (W[i][j] at i * cols + j).  The weight matrices are rounded
 *   to bfloat16 (nearest even) where used; layer 2 runs on the matrix cores
 *   with bfloat16 inputs (h1 rounded) and float32 accumulation; the rest is
 *   float32.
 * ---------------------------------------------------------------------- */
#define PTP_MLP_PARAMS 4481

/* Network inputs of a prepared plan in the caller's vertex order: X[n][3]
 * and scale[n] = l (-1 for unreachable vertices).  Asynchronous. */
ptp_status ptp_warm_features(ptp_plan *plan, float *dX, float *dScale, void *stream);

/* Predicted upper bound in the caller's order: upper[v] = inflate * d^(v),
 * 0 at the sources, +inf where unreachable.  inflate >= 1 (1.05 by design).
 * dParams is a device vector [PTP_MLP_PARAMS].  Asynchronous. */
ptp_status ptp_warm_predict(ptp_plan *plan, const float *dParams, float inflate, float *dUpper,
                            void *stream);

/* Certify dUpper[n] (caller order; negative or NaN entries mean no bound) and
 * run PTP from it; writes dist like ptp_run.  dUpper is read before dist is
 * written, so it may be the same buffer.  PTP_EUNSUPPORTED when the plan
 * wants labels.  Enqueues work only; ptp_get_stats reports the outcome and
 * the certification counts. */
ptp_status ptp_run_warm(ptp_plan *plan, const float *dUpper, float *dDist, void *stream);

/* The same three on a batch; arrays are indexed by out_off + local id. */
ptp_status ptp_batch_warm_features(ptp_batch *batch, float *dX, float *dScale, void *stream);
ptp_status ptp_batch_warm_predict(ptp_batch *batch, const float *dParams, float inflate,
                                  float *dUpper, void *stream);
ptp_status ptp_batch_run_warm(ptp_batch *batch, const float *dUpper, float *dDist, void *stream);

/* Number of network parameters (PTP_MLP_PARAMS). */
int32_t ptp_mlp_params(void);

/* out[i] = 64 * scale[i] * softplus(o(X[i])) for n rows X[n][3].  n = 0 is a
 * no-op.  Asynchronous. */
ptp_status ptp_mlp_apply(const float *dParams, const float *dX, const float *dScale, int64_t n,
                         float *dOut, void *stream);

/* Device scratch ptp_mlp_grad needs, in bytes. */
size_t ptp_mlp_scratch_bytes(void);

/* Training loss and its gradient over n >= 1 rows:
 *   L = (1/n) sum_i ((d^_i - target_i) / max(target_i, scale_i))^2
 * grad[PTP_MLP_PARAMS] = dL/dparams (with the bfloat16 rounding of the
 * weights taken as the identity), loss[1] = L (dLoss may be NULL).  The
 * result does not depend on scheduling (fixed reduction order).  dScratch:
 * caller device buffer of ptp_mlp_scratch_bytes(), 16-byte aligned;
 * PTP_ENOMEM if smaller.  Asynchronous. */
ptp_status ptp_mlp_grad(const float *dParams, const float *dX, const float *dScale,
                        const float *dTarget, int64_t n, void *dScratch, size_t scratch_bytes,
                        float *dGrad, float *dLoss, void *stream);

/* One Adam step (bias-corrected, step t >= 1) on the float32 parameters:
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * params -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * dM, dV [PTP_MLP_PARAMS] are the caller's moment buffers (zero at t = 1).
 * Asynchronous. */
ptp_status ptp_adam_step(float *dParams, const float *dGrad, float *dM, float *dV, int32_t t,
                         float lr, float beta1, float beta2, float eps, void *stream);

/* Library version string. */
const char *ptp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PTP_MI355X_H */
