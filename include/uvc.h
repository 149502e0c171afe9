/*
 * uvc.h -- C ABI of the MI355X irradiance-matrix library.
 *
 * The library assembles the irradiance matrix of "Optimized Coverage Planning
 * for UV Surface Disinfection" (arXiv 2103.14137): for K candidate lamp poses
 * and the N triangles of a mesh, the irradiance that each triangle receives
 * from a lamp dwelling at each pose (Sec. III-B, discrete irradiance; Sec.
 * IV-C, inverse-square law with the visibility condition), and solves the
 * relaxed dosage LP that consumes it (Sec. IV-D, relaxed LP).
 *
 * Matrix layout: the paper writes I_i(x_k) with one column per pose; this
 * library stores it pose-major, E[k * N + i] = I_i(x_k), so one paper column
 * is one row of E.
 *
 * Conventions for every entry point
 *  - Every function returns uvc_status; nothing throws across the ABI.  On a
 *    failure uvc_last_error() returns a thread-local message naming the cause.
 *  - "dev" pointers are HIP device pointers on the current device; "host"
 *    pointers are ordinary host memory.  Caller-owned buffers are borrowed for
 *    the duration of the call only.  Scenes and CSR jobs are owned by the
 *    library and released by their destroy functions.
 *  - hip_stream is a hipStream_t (NULL = the default stream).  Work is
 *    enqueued on it and the call returns without waiting, except where a
 *    function says it synchronises.
 *  - Inputs are validated before any kernel is launched: non-finite
 *    coordinates, indices out of range, zero-area triangles, source counts
 *    outside [1, 32] or non-positive powers return UVC_EINVAL.  K = 0 or
 *    N = 0 succeed with empty output.
 */
#ifndef UVC_H
#define UVC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    UVC_OK = 0,
    UVC_EINVAL = -1,        /* invalid argument (message names it)          */
    UVC_ENOMEM = -2,        /* device allocation failed                     */
    UVC_EDEVICE = -3,       /* HIP runtime error                            */
    UVC_ENOTCONV = -4,      /* LP iteration limit; best iterate returned    */
    UVC_EUNSUPPORTED = -5   /* request outside what this build supports     */
} uvc_status;

/* Thread-local description of the last failure on this thread ("" if none). */
const char* uvc_last_error(void);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int32_t uvc_version(void);

/* ------------------------------------------------------------------------
 * Scene: the mesh, its surface elements and its bounding volume hierarchy.
 * ------------------------------------------------------------------------ */
typedef struct uvc_scene uvc_scene;

/* Build a scene from a triangle mesh (Sec. III-B: the surface is a simplicial
 * complex of N triangles, one surface element per triangle).
 *   verts_xyz : n_verts x 3 FP32, row-major (x, y, z) in metres.
 *   tri_idx   : n_tris x 3 int32 vertex indices.  The right-hand normal
 *               (v1 - v0) x (v2 - v0) of every triangle must point into free
 *               space, the side lamps are on.
 *   inputs_on_device : 0 if both arrays are host memory, 1 if device memory
 *               (they are copied to the host once for validation).
 * The scene keeps its own copies; the inputs may be freed on return.  This
 * call synchronises hip_stream.  Errors: UVC_EINVAL for non-finite vertices,
 * a vertex coordinate above 2^26 in magnitude (the FP32 box tests stay
 * finite below it), indices outside [0, n_verts) or a triangle whose FP64
 * cross product is exactly zero (the message names the first such
 * triangle); UVC_ENOMEM; UVC_EDEVICE. */
uvc_status uvc_build_scene(const float* verts_xyz, int64_t n_verts,
                           const int32_t* tri_idx, int64_t n_tris,
                           int32_t inputs_on_device, void* hip_stream,
                           uvc_scene** out);

/* Scene facts: triangle count, depth of the hierarchy (root = 1) and the
 * largest absolute vertex coordinate.  Any output pointer may be NULL. */
uvc_status uvc_scene_info(const uvc_scene* scene, int64_t* n_tris,
                          int32_t* bvh_depth, float* max_abs_coord);

/* Surface elements in the input triangle order (Sec. III-B), into caller
 * device buffers: centroid c_xyz (N x 3 FP32; the FP64 mean of the three
 * vertices rounded once to FP32 -- the element's sampling point), unit
 * normal n_xyz (N x 3 FP32) and area (N FP32).  Any pointer may be NULL. */
uvc_status uvc_scene_elements(const uvc_scene* scene, float* c_xyz_dev,
                              float* n_xyz_dev, float* area_dev,
                              void* hip_stream);

/* Copy the hierarchy to host buffers for inspection (tests):
 *   nodes : (N - 1) x 16 FP32 -- per internal node the boxes of its two
 *           children (lo xyz, hi xyz for left, then for right), the two child
 *           references as int32 bit patterns (>= 0 internal node, < 0 leaf
 *           slot ~ref), then two words of traversal hints;
 *   perm  : N int32, the input triangle index stored in each leaf slot;
 *   codes : N uint32, the sorted Morton codes.
 * Any pointer may be NULL.  Synchronises hip_stream. */
uvc_status uvc_scene_export_bvh(const uvc_scene* scene, float* nodes_host,
                                int32_t* perm_host, uint32_t* codes_host,
                                void* hip_stream);

/* Release a scene (NULL is allowed).  Waits for the device to be idle. */
void uvc_destroy_scene(uvc_scene* scene);

/* ------------------------------------------------------------------------
 * Irradiance matrix (Sec. IV-C).
 * ------------------------------------------------------------------------ */

/* A lamp is n_src point sources mounted dz[j] metres above the pose base
 * point, each emitting power_w[j] watts (Sec. IV-C: an extended lamp as
 * point sources of equal power; each source may have its own emission
 * pattern).  Host arrays, copied by the call.  1 <= n_src <= 32,
 * power_w[j] > 0, dz[j] finite.
 * Emission pattern (optional; zero-initialised fields = uniform emission):
 *   n_prof, profile: 0 (uniform, weight 1) or 2..33 finite weights >= 0, not
 *     all 0, at cos(theta) = -1 + 2 q / (n_prof - 1), q = 0 .. n_prof - 1,
 *     interpolated linearly; theta is the angle between the upward vertical
 *     through the source and the direction from the source to the element.
 *     The source's term P_j / (4 pi) <d, n> / |d|^3 is multiplied by the
 *     weight.
 *   up_mask / down_mask: bit j set = source j emits only into the open
 *     half-space above (element centroid z > source z) / below its own
 *     height (a shield); a source may not be in both.  Where a source does
 *     not emit, no segment is cast and its visibility bit is 0.
 * The many-room batch (uvc_batch_*) takes uniform lamps only. */
typedef struct {
    int32_t n_src;
    const float* dz;
    const float* power_w;
    int32_t n_prof;
    const float* profile;
    uint32_t up_mask;
    uint32_t down_mask;
} uvc_lamp;

enum { UVC_PATH_AUTO = 0, UVC_PATH_LBVH = 1, UVC_PATH_BRUTE = 2 };

/* UVC_FLAG_NO_NEAR: the hierarchy path walks every segment to its target
 * instead of stopping short and testing the element's near list (same
 * results, slower; for testing).
 * UVC_FLAG_NO_CACHE: the hierarchy path does not test each lane's last
 * occluding triangle before walking the next source's segment (same
 * results; for testing and measurement). */
enum { UVC_FLAG_NO_NEAR = 1, UVC_FLAG_NO_CACHE = 2 };

/* Counters accumulated by an instrumented launch (opts.stats_dev). */
enum {
    UVC_STAT_RAYS = 0,       /* occlusion segments cast (front-facing triples) */
    UVC_STAT_NODES = 1,      /* per-ray hierarchy node visits (2 child boxes)  */
    UVC_STAT_TRIS = 2,       /* per-ray segment/triangle tests                 */
    UVC_STAT_RECHECK = 3,    /* triangle decisions re-taken in FP64            */
    UVC_STAT_FRONT64 = 4,    /* front-facing decisions re-taken in FP64        */
    UVC_STAT_VISIBLE = 5,    /* visible (pose, source, element) triples        */
    UVC_STAT_STEPS = 6,      /* wavefront traversal steps (one node each)      */
    UVC_STAT_NEAR = 7,       /* per-ray near-list segment/triangle tests       */
    UVC_STAT_CACHE = 8,      /* per-ray tests of the lane's last occluder      */
    UVC_STAT_CACHE_HIT = 9,  /* ... of which found the segment blocked         */
    UVC_STAT_LEAF_STEPS = 10,/* wavefront leaf tests (one triangle each)       */
    UVC_STAT_N = 11
};

typedef struct {
    int32_t path;        /* UVC_PATH_*; AUTO picks the brute-force path for
                            small meshes and the hierarchy otherwise          */
    int32_t packet_poses; /* hierarchy path: poses per wavefront packet, a
                            power of two in [1, 64] (0 = 16); the 64 lanes
                            hold packet_poses poses x 64/packet_poses
                            elements                                          */
    float band_scale;    /* multiplies the FP32 decision bands: 1 = default;
                            +inf re-takes every decision in FP64 (slow);
                            0 leaves only exact ties to FP64 (unsafe: FP32
                            may then disagree with the exact predicate)       */
    int32_t tile_tris;   /* brute-force path: triangles per LDS tile (0 = default) */
    int32_t flags;       /* UVC_FLAG_* bits                                   */
    int32_t waves;       /* hierarchy path: kernel variant compiled for this
                            many waves per SIMD: 5 (no register cap), 6 or
                            8 (0 = 6)                                         */
    uint64_t* stats_dev; /* NULL, or UVC_STAT_N device counters that an
                            instrumented (slower) kernel adds to              */
    float* kernel_ms;    /* NULL, or host float: HIP events are recorded on
                            hip_stream around the irradiance kernel launches,
                            the call synchronises and stores their elapsed
                            milliseconds here (for measurement)              */
} uvc_opts;

/* Dense irradiance matrix.
 *   poses_dev : K x pose_dim FP32 lamp base points, (x, y) with base height 0
 *               or (x, y, z).  Source j of pose k sits at
 *               (x_k, y_k, fl32(z_k + dz[j])).  Every source point must lie
 *               within 2 * max_abs_coord of the origin (UVC_EINVAL otherwise).
 *               The poses are copied to the host once for validation.
 *   E_dev     : K x N FP32, caller-owned, fully overwritten:
 *               E[k*N + i] = sum over j ascending (FP32 adds) of
 *                 V_kji * P_j * <p_kj - c_i, n_i> / (4 pi |p_kj - c_i|^3),
 *               where V_kji = 1 iff <p_kj - c_i, n_i> > 0 and no triangle
 *               other than i meets the open segment p_kj -> c_i (closed
 *               triangles; the paper's visibility condition after its
 *               inverse-square law).  A visible term is never below
 *               FLT_MIN, so E[k*N+i] != 0 exactly when some V_kji = 1.
 *   vis_dev   : NULL, or K x N uint32 with bit j = V_kji.
 * Visibility is decided in FP32 where the FP32 value is provably on the same
 * side of zero as the exact one, and re-decided in FP64 otherwise, so every
 * bit equals the FP64 segment/triangle predicate.  Synchronises hip_stream
 * before the main launch (pose validation); the launch itself is async. */
uvc_status uvc_compute_irradiance_dense(const uvc_scene* scene,
                                        const float* poses_dev, int64_t K,
                                        int32_t pose_dim, const uvc_lamp* lamp,
                                        const uvc_opts* opts, float* E_dev,
                                        uint32_t* vis_dev, void* hip_stream);

/* The dense call for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, same validation and the same bits in E_dev and vis_dev as
 * uvc_compute_irradiance_dense, but no hipMalloc, hipFree or other
 * allocation.  Its scratch (8 work counters, the pose check word and the
 * pose visiting order) lives in a file-scope device array of 4 MiB + 256 B
 * that each GPU holds until the process ends; poses are checked on the
 * device and visited in the caller's order.  Limits: K <= 1,048,576 poses
 * (UVC_EINVAL beyond), and opts->kernel_ms must be NULL (timing needs HIP
 * events; UVC_EINVAL otherwise).  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams or host threads) race
 * and must be serialised by the caller.  Synchronises hip_stream once
 * (pose check) before the launch. */
uvc_status uvc_compute_irradiance_dense_noalloc(const uvc_scene* scene,
                                                const float* poses_dev,
                                                int64_t K, int32_t pose_dim,
                                                const uvc_lamp* lamp,
                                                const uvc_opts* opts,
                                                float* E_dev, uint32_t* vis_dev,
                                                void* hip_stream);

/* Area-integrated irradiance (Sec. IV-C, the visibility-cube procedure): the
 * paper's own entry, the power a triangle receives over its area, with
 * partial occlusion.  Each source emits through a cube of face_res x
 * face_res pixels per face (0: 512, the paper's resolution; at most 1024):
 * face f has axis f / 2 and outward sign + for even f, pixel (a, b) spans
 * u in [-1 + 2a/R, -1 + 2(a+1)/R] along axis (f/2 + 1) mod 3 and v likewise
 * along (f/2 + 2) mod 3, carries the power P_j w_j dOmega / (4 pi) (dOmega
 * the pixel's exact solid angle, w_j the lamp's emission weight at the
 * pixel centre direction; hemisphere masks drop pixels whose centre
 * direction points into the masked half) and sends it along the ray
 * through its centre to the closest triangle, which collects it if the ray
 * reaches its front side.  E_dev[k * N + i] (K x N FP32, caller-owned,
 * input element order) = collected power / triangle area (W/m^2);
 * power_dev: NULL or K FP64 values, the power collected per pose.
 * Closest hits are decided in FP32, with a ray within ~1e-6 (relative) of
 * a triangle edge counted as inside so that no ray slips between triangles
 * that share an edge (such pixels, and rays meeting two triangles at nearly
 * the same distance, may go to a neighbour of the FP64 choice); collection
 * is in 2^-40 W fixed point
 * with integer atomics, so results do not depend on scheduling.  Requires
 * total lamp power <= 2^22 W.  Non-finite poses return UVC_EINVAL (poses
 * are copied to the host for the check).  Synchronises hip_stream. */
uvc_status uvc_compute_irradiance_area(const uvc_scene* scene,
                                       const float* poses_dev, int64_t K,
                                       int32_t pose_dim, const uvc_lamp* lamp,
                                       int32_t face_res, float* E_dev,
                                       double* power_dev, void* hip_stream);

/* Irradiance of a subset of the elements: targets_dev holds n_targets input
 * element indices (device int32); E_dev (K x n_targets FP32, device) gets
 * column j = element targets_dev[j], bit-identical to that column of the
 * dense matrix.  vis_dev: NULL or K x n_targets uint32.  Same options,
 * validation and synchronisation as the dense call. */
uvc_status uvc_compute_irradiance_targets(const uvc_scene* scene,
                                          const float* poses_dev, int64_t K,
                                          int32_t pose_dim, const uvc_lamp* lamp,
                                          const uvc_opts* opts,
                                          const int32_t* targets_dev,
                                          int64_t n_targets, float* E_dev,
                                          uint32_t* vis_dev, void* hip_stream);

/* CSR irradiance matrix (rows = poses, ascending columns, only entries with
 * some V_kji = 1 stored), in two phases so that the caller owns the output.
 * begin computes everything, keeps the compacted entries in library memory,
 * returns the nonzero count and synchronises hip_stream.  finish writes
 * row_ptr (K+1 int64), col (nnz int32) and val (nnz FP32, bit-identical to
 * the dense values) into caller device buffers and releases the job.
 * uvc_csr_job_destroy releases a job without finishing it. */
typedef struct uvc_csr_job uvc_csr_job;

uvc_status uvc_compute_irradiance_csr_begin(const uvc_scene* scene,
                                            const float* poses_dev, int64_t K,
                                            int32_t pose_dim,
                                            const uvc_lamp* lamp,
                                            const uvc_opts* opts,
                                            void* hip_stream,
                                            uvc_csr_job** job, int64_t* nnz);
uvc_status uvc_compute_irradiance_csr_finish(uvc_csr_job* job,
                                             int64_t* row_ptr_dev,
                                             int32_t* col_dev, float* val_dev,
                                             void* hip_stream);
void uvc_csr_job_destroy(uvc_csr_job* job);

/* ------------------------------------------------------------------------
 * Autotuning of the launch options.
 * ------------------------------------------------------------------------ */

/* Pick the fastest launch options for this scene's size class: the first
 * max(probe_poses (<= 0: 256), 2^23 / N) poses, at most K (a probe large
 * enough for the persistent loop's steady state), are computed with every
 * hierarchy variant (packet_poses 4/8/16/32/64 x waves 5/6/8) and, for
 * meshes of up to 16,384 triangles, every brute-force LDS tile (256..2048);
 * each is timed with HIP events and scored in occlusion rays per second.  The winner is stored in
 * the JSON table at table_path (NULL: no table) under the key
 * "n<floor(log2 N)>_s<n_src>" and returned in *best.  When the table already
 * holds the key and force == 0, no probe runs.  Synchronises hip_stream. */
uvc_status uvc_autotune(const uvc_scene* scene, const float* poses_dev,
                        int64_t K, int32_t pose_dim, const uvc_lamp* lamp,
                        int32_t probe_poses, const char* table_path,
                        int32_t force, uvc_opts* best, void* hip_stream);

/* Register a tuning table for the whole library (json: the text of a table
 * written by uvc_autotune; NULL clears it).  While one is registered, calls
 * with opts->path = UVC_PATH_AUTO (dense, CSR, targets and the batch) take
 * the path, packet shape, occupancy and LDS tile of the scene's size class
 * from it (options the caller set to nonzero values stay the caller's);
 * size classes the table lacks keep the built-in rule (brute force up to
 * 2,048 triangles).  UVC_EINVAL for an entry with invalid options. */
uvc_status uvc_set_tune_table(const char* json);

/* ------------------------------------------------------------------------
 * Many rooms in one launch.
 * ------------------------------------------------------------------------ */
typedef struct uvc_batch uvc_batch;

enum { UVC_BATCH_PERSISTENT = 0, UVC_BATCH_GRAPH = 1, UVC_BATCH_PER_ROOM = 2 };

/* Prepare the dense irradiance matrices of n_rooms rooms (same lamp; hierarchy
 * path) for repeated runs.  scenes[r], the device poses poses_dev[r]
 * (K[r] x pose_dim) and the caller-owned device outputs E_dev[r] (K[r] x N_r
 * FP32) must stay valid while the batch exists.  Launch options per room:
 * with tune_table_json (the text of a table written by uvc_autotune), or
 * with opts->path = UVC_PATH_AUTO and a table registered by
 * uvc_set_tune_table, each room takes the packet shape and occupancy of its
 * size class's hierarchy entry (the persistent launch honours the packet
 * shape per room and runs at 6 waves per SIMD; one launch per room honours
 * both); rooms without an entry, and every room otherwise, take opts.  The
 * results are the same bits whatever the options.  Poses are validated here
 * (synchronises hip_stream).  The work queue lists the rooms by estimated
 * cost per work item, longest first. */
uvc_status uvc_batch_create(const uvc_scene* const* scenes, int32_t n_rooms,
                            const float* const* poses_dev, const int64_t* K,
                            int32_t pose_dim, const uvc_lamp* lamp,
                            const uvc_opts* opts, const char* tune_table_json,
                            float* const* E_dev, void* hip_stream,
                            uvc_batch** out);

/* Compute every room's E.  mode UVC_BATCH_PERSISTENT: one persistent launch
 * whose workgroups drain the queue through an atomic counter;
 * UVC_BATCH_GRAPH: the same work (a counter-reset kernel and the launch)
 * captured once into a hipGraph on a library-owned stream and replayed on
 * hip_stream; UVC_BATCH_PER_ROOM: one launch per
 * room.  All modes write identical bits.  kernel_ms: NULL or host float that
 * receives the HIP-event time of the launches (the call then synchronises).
 * Runs on one batch must not overlap (they share the queue counter). */
uvc_status uvc_batch_run(uvc_batch* batch, int32_t mode, float* kernel_ms,
                         void* hip_stream);

void uvc_batch_destroy(uvc_batch* batch);

/* ------------------------------------------------------------------------
 * Dosage LP (Sec. IV-D, relaxed LP), the consumer of E.
 * ------------------------------------------------------------------------ */
typedef struct {
    double objective;        /* sum_k t_k + sum_i p_i sigma_i over visible elements */
    double primal_residual;  /* relative KKT residuals of the returned point     */
    double dual_residual;
    double gap;
    int32_t iterations;
    int64_t n_visible;       /* elements with some E[k,i] > 0                     */
    double penalty;          /* p_0 (the default penalty when penalty_dev = NULL) */
    int64_t working_poses;   /* column generation (large CSR input): poses in the
                                final working set; 0 for a direct solve           */
    int32_t rounds;          /* column generation: working LPs solved; 0 direct  */
} uvc_lp_info;

/* Solve  min sum_k t_k + sum_i p_i sigma_i
 *        s.t. sum_k E[k,i] t_k + sigma_i >= mu_min (every visible element),
 *             sum_k t_k <= t_max, t >= 0, sigma >= 0
 * (Sec. IV-D, relaxed LP) for the pose-major K x N matrix E on the device,
 * given either dense (row_ptr_dev = NULL: E_dev holds K x N FP32, row k =
 * pose k) or as CSR (row_ptr_dev: K + 1 int64 offsets starting at 0;
 * col_dev: nnz = row_ptr[K] int32 element indices, strictly ascending within
 * each row, in [0, N); E_dev: the nnz FP32 values), e.g. the output of
 * uvc_compute_irradiance_csr_*.  A CSR input is validated on the device (a
 * bad row is named in the error).  Up to 8,192 poses it is expanded once
 * into a library-owned dense copy of K N 4 bytes for the normal-matrix
 * products; with more poses the LP is solved by column generation: the
 * method below over a working set of poses (initially the ceil(K/10)
 * poses with the largest row sums of E), every other pose priced against the working
 * duals (reduced cost 1 + y_b - sum_i E[k,i] y_i from its sparse row) and
 * those below -1e-6 added (the most negative first, at most
 * max(64, ceil(K/10)/4) per round; working poses without dwell whose
 * reduced cost exceeds 1e-2 (1 + y_b) leave the set, each at most once)
 * until none is left, which makes the working solution optimal over
 * all K poses (info->working_poses, info->rounds; the dual residual
 * reported covers the pricing; an element no working pose sees keeps
 * sigma_i = mu_min and dual p_i, and counts in the objective when some
 * pose sees it).  Elements with
 * E[k,i] = 0 for every k are dropped (sigma_i = mu_min, excluded from the
 * objective).  penalty_dev: N FP64 device values or NULL for
 * p_i = 1.001 * ||E||_F (the paper asks for p_i > ||I||_F).  Mehrotra
 * predictor-corrector interior point method; its K x K normal matrix is
 * formed and Cholesky-factored on the GPU in FP64 (8 K^2 bytes of scratch).
 * Stops when the relative primal residual, dual residual and duality gap are
 * all <= tol.  Outputs (device FP64, each may be NULL): t_out_dev (K),
 * sigma_out_dev (N) and y_out_dev (N + 1): the duals of the N coverage rows
 * (for a dropped element, its penalty p_i: its sigma_i = mu_min lies inside
 * its bound) followed by the dual of the time-budget row.  With them the
 * reduced cost of any further pose k is 1 + y_N - sum_i E[k,i] y_i.
 * K = 0 or N = 0: UVC_OK with t = 0, sigma = mu_min, coverage duals equal
 * to the penalties (0 for the default penalty of an empty matrix), budget
 * dual 0 and objective 0.  Returns UVC_ENOTCONV with the last point when
 * max_iter is reached.  Synchronises hip_stream. */
uvc_status uvc_solve_dosage_lp(const float* E_dev, const int64_t* row_ptr_dev,
                               const int32_t* col_dev, int64_t K, int64_t N,
                               const double* penalty_dev, double mu_min,
                               double t_max, double tol, int32_t max_iter,
                               double* t_out_dev, double* sigma_out_dev,
                               double* y_out_dev, uvc_lp_info* info,
                               void* hip_stream);

/* ------------------------------------------------------------------------
 * Learned pose ranker.  Not part of the paper: a pruning step in front of
 * E assembly whose result is always checked against the paper's LP (Sec. IV-D)
 * on the full candidate set when pruning could have cost coverage.
 * ------------------------------------------------------------------------ */

/* Number of FP32 parameters of the ranker MLP (64 -> 128 -> 128 -> 1, ReLU):
 * W1[128][64], b1[128], W2[128][128], b2[128], W3[128], b3, in this order
 * (24,961 floats). */
int64_t uvc_ranker_param_count(void);

/* Per-pose visibility features, feat_dev[k * 64 + b] (K x 64 FP32, device).
 * From the point (x_k, y_k, z_k + src_height) (z_k = 0 for 2-D poses), 256
 * rays in an equal-area direction set (16 azimuths x 16 bands uniform in the
 * vertical direction cosine, cell centres) find their closest triangle; each
 * hit adds the area its ray stands for, (4 pi / 256) r^2 / max(|cos|, 0.05)
 * with r the hit distance and cos the cosine between ray and triangle
 * normal, to bin 8 * d + c, d = distance bin with edges
 * 0.5, 1, 1.5, 2, 3, 4, 6 m and c = min(7, floor(8 |cos|)); the features are
 * log1p of the bin sums (summed in ray order).  Misses add nothing.
 * Non-finite poses or height return UVC_EINVAL (the poses are copied to the
 * host for the check, which synchronises hip_stream). */
uvc_status uvc_ranker_features(const uvc_scene* scene, const float* poses_dev,
                               int64_t K, int32_t pose_dim, float src_height,
                               float* feat_dev, void* hip_stream);

/* Scores score_dev[b] (B FP32, device) of the MLP with parameters
 * params_dev on features feat_dev (B x 64).  bf16 != 0 rounds every weight
 * and layer input to bfloat16 (nearest even) before its FP32 product and
 * accumulation. */
uvc_status uvc_ranker_forward(const float* params_dev, const float* feat_dev,
                              int64_t B, int32_t bf16, float* score_dev,
                              void* hip_stream);

/* Non-learned baseline score: the visible area sum_b expm1(feat[k,b]). */
uvc_status uvc_ranker_area_score(const float* feat_dev, int64_t K,
                                 float* score_dev, void* hip_stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with the
 * 1-based step count) on the mean binary cross-entropy with logits of the
 * batch: rows idx_dev[0..B) of feat_dev / label_dev (idx_dev NULL: rows
 * 0..B).  params_dev, adam_m, adam_v: uvc_ranker_param_count() FP32 each,
 * device, updated in place.  grad_out_dev: NULL or a device buffer of the
 * same size that receives the batch gradient.  *loss_out (host, may be NULL)
 * receives the batch's mean loss before the update.  Synchronises
 * hip_stream. */
uvc_status uvc_ranker_train_step(float* params_dev, float* adam_m,
                                 float* adam_v, const float* feat_dev,
                                 const float* label_dev,
                                 const int32_t* idx_dev, int64_t B, float lr,
                                 int64_t step, float* grad_out_dev,
                                 float* loss_out, void* hip_stream);

enum { UVC_RANK_MLP = 0, UVC_RANK_AREA = 1, UVC_RANK_NONE = 2 };

typedef struct {
    double objective;        /* LP objective of the returned plan (over the elements
                                some candidate pose sees)                            */
    double penalty;          /* the LP penalty p used                                */
    double min_reduced_cost; /* smallest reduced cost of a pruned pose at the end    */
    int64_t n_kept;          /* poses in the LP that produced the plan               */
    int64_t n_added;         /* poses added by pricing                               */
    int64_t n_priced;        /* element columns computed for pricing (all rounds)    */
    int32_t rounds;          /* restricted LPs solved                                */
    int32_t rounds_added;    /* pricing rounds that added poses                      */
    int32_t fell_back;       /* 1: the full candidate set produced the plan          */
    int32_t lp_iterations;   /* summed over every LP solved                          */
    int32_t lp_converged;
    float ms_features, ms_score, ms_E, ms_lp, ms_price, ms_fallback, ms_total;
    int64_t n_dropped;       /* kept poses without dwell that left the set (each at
                                most once; reduced cost above 1e-2 (1 + y_b))        */
} uvc_plan_info;

/* Dwell-time plan with pose pruning and column generation.
 *
 * score_mode UVC_RANK_MLP scores the K poses with the MLP (params_dev, bf16
 * as in uvc_ranker_forward) on features taken at feature_height;
 * UVC_RANK_AREA scores them by visible area; UVC_RANK_NONE solves the LP
 * over all K poses directly.  The ceil(keep_frac K) best-scoring poses
 * (ties: lower index) form the restricted set.  Each round assembles E on
 * the restricted set (opts as for the dense call) and solves the relaxed LP
 * (tol, max_iter as for uvc_solve_dosage_lp) with the penalty p for every
 * element (penalty <= 0: the LP's default 1.001 ||E||_F over all K poses,
 * from one pass of the dense kernel over pose blocks that keeps only the
 * norm, so that the restricted LPs and the pricing solve the LP over all
 * K poses; the fallback passes the caller's penalty on, so that it is
 * exactly the full plan, whose default is the same p up to the order of
 * the norm's sum).  With its
 * duals y, every pruned pose k gets the reduced cost
 * 1 + y_b - sum_i E[k,i] y_i, summed over the elements with y_i > 1e-9
 * max y (their E columns over all K poses come from the targets kernel;
 * elements no candidate sees are skipped afterwards).  If none is below
 * -1e-6 the restricted plan is optimal for the LP over all K poses and is
 * returned; otherwise up to max(16, |R_0|) poses with the most negative
 * reduced costs join (kept poses without dwell whose reduced cost exceeds
 * 1e-2 (1 + y_b) leave first, each at most once) and the next round
 * starts; every restricted LP is solved to tol (one that stops at max_iter
 * with relative residuals and gap within 1e-6 is used as it is, and
 * lp_converged = 0 reports it).  After max_rounds rounds that added poses with pricing still
 * negative, or if an LP stops farther from convergence, the
 * plan is recomputed from all K poses (fell_back = 1).  Outputs: t_out_dev
 * (K FP64, zero for pruned poses), sigma_out_dev (N FP64), kept_host (NULL
 * or K int32: the first n_kept entries list the poses of the final LP,
 * ascending) and *info with HIP-event stage times.  Synchronises
 * hip_stream. */
uvc_status uvc_plan_ranked(const uvc_scene* scene, const float* poses_dev,
                           int64_t K, int32_t pose_dim, const uvc_lamp* lamp,
                           const uvc_opts* opts, int32_t score_mode,
                           const float* params_dev, int32_t bf16,
                           float keep_frac, float feature_height,
                           double penalty, double mu_min, double t_max,
                           double tol, int32_t max_iter, int32_t max_rounds,
                           double* t_out_dev, double* sigma_out_dev,
                           int32_t* kept_host, uvc_plan_info* info,
                           void* hip_stream);

/* Objective of a dwell-time plan t_dev (K FP64, device) on the dense E_dev
 * (K x N FP32, device): sum_k t_k + p * sum_i max(0, mu_min - sum_k E[k,i] t_k)
 * over the visible elements (some E[k,i] > 0), i.e. the relaxed LP objective
 * with sigma at its smallest feasible value.  penalty <= 0 selects the LP's
 * default p = 1.001 ||E||_F.  Optional outputs: the shortfall sum, the number
 * of visible elements short by more than 1e-6 mu_min, the number of visible
 * elements.  Used to compare plans from different pose subsets on the same
 * matrix.  Synchronises hip_stream. */
uvc_status uvc_plan_evaluate(const float* E_dev, int64_t K, int64_t N,
                             const double* t_dev, double mu_min,
                             double penalty, double* objective,
                             double* shortfall, int64_t* n_short,
                             int64_t* n_visible, void* hip_stream);

/* ------------------------------------------------------------------------
 * Route stage (Sec. IV-D second stage; roadmap distances Sec. IV-B): a
 * closed tour over the poses the LP gives a dwell time.
 * ------------------------------------------------------------------------ */

/* Free space is an H x W grid of cells of side `cell` (free_dev: H * W
 * uint8, row-major, row = y index, nonzero = free; cell (r, c) covers
 * [x0 + c cell, x0 + (c + 1) cell) x [y0 + r cell, y0 + (r + 1) cell)).  A
 * stop lies in cell (floor((y - y0) / cell), floor((x - x0) / cell)),
 * evaluated in FP64.  Paths step between 8-connected free cells at cost
 * cell (orthogonal) or cell * sqrt(2) (diagonal, allowed only when both
 * orthogonal neighbours are free); the distance between two stops is the
 * smallest FP64 sum of a path's steps between their cells, symmetrised as
 * min(d(a, b), d(b, a)) (the paper uses roadmap distances; a grid stands in
 * for the roadmap).
 * uvc_route_geodesics: the m x m matrix dist_dev (FP64, device) for the m
 * stops stops_dev (m x 2 FP32, device; m <= 4096, H W m <= 2^31).
 * UVC_EINVAL if a stop lies outside the grid or in a blocked cell, or if
 * two stops are not connected.  Synchronises hip_stream. */
uvc_status uvc_route_geodesics(const uint8_t* free_dev, int32_t H, int32_t W,
                               float x0, float y0, float cell,
                               const float* stops_dev, int32_t m,
                               double* dist_dev, void* hip_stream);

/* Closed tour over m stops (m <= 4096) with the distance matrix dist_dev
 * (m x m FP64, device, symmetric): nearest neighbour from stop 0 (ties: the
 * lowest index), then best-improvement 2-opt (move (i, j), 0 <= i <= m-3,
 * i+2 <= j <= m-1, not (0, m-1): reverse stops i+1 .. j; index i m + j) and,
 * when no 2-opt move improves, best-improvement Or-opt (move (s, i, p):
 * stops i .. i+s-1, 1 <= s <= 3, 1 <= i <= m-s, reinserted in the same
 * orientation after the stop at position p outside [i-1, i+s-1]; index
 * ((s-1) m + i) m + p); the best move has the smallest FP64 delta, ties
 * the lowest index; stop when no move improves by more than 1e-12 of the
 * tour length or after max_moves moves (<= 0: 100 m).  The paper uses LKH;
 * this is a local search.  Outputs: tour_host (m int32, stop 0 first), the
 * tour length (FP64 sum in tour order) and the number of moves.
 * Synchronises hip_stream. */
uvc_status uvc_route_tour(const double* dist_dev, int32_t m, int32_t max_moves,
                          int32_t* tour_host, double* length, int32_t* moves,
                          void* hip_stream);

/* The plan after the LP: the stops are the poses with
 * t_k > rel_threshold * sum t (t_dev: K FP64, device; poses_dev K x
 * pose_dim FP32, device), ascending; their geodesics and tour as above.
 * Outputs: stops_host (K int32 capacity; the first *m_out entries are the
 * pose indices in tour order), the tour length (m) and the plan time
 * sum_k t_k + length / v_max (s).  Synchronises hip_stream. */
uvc_status uvc_plan_route(const float* poses_dev, int64_t K, int32_t pose_dim,
                          const double* t_dev, double rel_threshold,
                          const uint8_t* free_dev, int32_t H, int32_t W,
                          float x0, float y0, float cell, double v_max,
                          int32_t* stops_host, int32_t* m_out,
                          double* length, double* plan_time,
                          void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* UVC_H */
