/*
 * slimvdb.h -- C ABI of the MI355X (gfx950) semantic TSDF integrator.
 *
 * The library fuses posed, semantically labelled point clouds into a sparse
 * voxel map of 8x8x8-voxel leaves, as the SLIM-VDB method does (arXiv
 * 2512.12945): per point, a voxel walk over the truncation band around the
 * point along its sensor ray (Sec. III-A), the running weighted TSDF mean and
 * weight (Eq. (1)-(2), weight 1), and the conjugate Bayesian semantic update,
 * closed set (Dirichlet concentrations, Thm. 1 / Eq. (6)) or open set
 * (Normal-Inverse-Gamma statistics with lambda = 2 nu = W and a diagonal beta,
 * Thm. 2 / Eqs. (11)-(14) and Sec. III-D).  All compute runs in HIP kernels on
 * the map's GPU; this header needs no HIP or torch include.
 *
 * Conventions shared by every call
 *   - Every function returns a slim_status: SLIM_OK (0) or a negative error.
 *     A failing call leaves a message for slim_last_error() (thread-local)
 *     and never throws.
 *   - "dev" pointers are device memory on the map's GPU; "host" pointers are
 *     ordinary CPU memory.  The caller owns every buffer it passes and keeps
 *     it valid until the work queued on `stream` has finished.  The library
 *     owns the map's own device memory.
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *     Work is queued asynchronously unless the description says the call
 *     synchronises.  One map must be used from one stream at a time.
 *   - Voxel keys are integer voxel coordinates k = floor(x / voxel_size) per
 *     axis, valid for |k| < 2^20.  A voxel's centre is (k + 1/2) voxel_size.
 *     Its leaf is floor(k / 8) per axis; its offset in the leaf is k mod 8.
 */
#ifndef SLIMVDB_H
#define SLIMVDB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t slim_status;
#define SLIM_OK 0
#define SLIM_ERR_INVALID (-1)     /* bad argument or configuration; nothing queued */
#define SLIM_ERR_CAPACITY (-2)    /* a frame needed more leaves or voxels than configured */
#define SLIM_ERR_DEVICE (-3)      /* a HIP runtime call failed */
#define SLIM_ERR_UNSUPPORTED (-4) /* valid request this build does not handle */

/* semantic model of a map */
#define SLIM_SEM_NONE 0   /* geometry only: D and W */
#define SLIM_SEM_CLOSED 1 /* K Dirichlet class counts per voxel (Sec. III-C) */
#define SLIM_SEM_OPEN 2   /* L-dim NIG mean m and diagonal beta per voxel (Sec. III-D) */
/* Non-Bayesian ablation (SLIM-VDB* of Sec. IV): a voxel keeps the semantics of
 * its most recent measurement -- the observing point with the highest index in
 * the latest frame that observed it.  D and W follow Eq. (1)-(2) as above. */
#define SLIM_SEM_CLOSED_LAST 3 /* 1 float per voxel: the class index (label, or first argmax of the row) */
#define SLIM_SEM_OPEN_LAST 4   /* L floats per voxel: the embedding */

/* layout of the per-point semantic input of slim_integrate */
#define SLIM_IN_NONE 0      /* no semantics (SLIM_SEM_NONE maps) */
#define SLIM_IN_LABEL_I32 1 /* int32[N]: class index; a one-hot observation (Eq. (6)) */
#define SLIM_IN_PROB_F32 2  /* float[N x K] row-major: class probabilities, added as expected counts */
#define SLIM_IN_LOGIT_F32 3 /* float[N x K] row-major: logits, softmax taken per point (K <= 64) */
#define SLIM_IN_EMB_BF16 4  /* uint16[N x L] row-major bfloat16 embedding (open set) */
#define SLIM_IN_EMB_F32 5   /* float[N x L] row-major embedding (open set) */

typedef struct slim_map slim_map; /* opaque */

typedef struct slim_map_config {
    float voxel_size;   /* edge of a voxel in metres, > 0 */
    float sdf_trunc;    /* truncation distance tau in metres, >= voxel_size */
    float min_range;    /* points closer than this to the sensor are rejected, >= 0 */
    float max_range;    /* points farther than this are rejected, > min_range */
    int32_t sem_mode;   /* SLIM_SEM_* */
    int32_t num_classes;/* K, 1..256, closed set only */
    int32_t embed_dim;  /* L, 1..1024, open set only */
    int32_t device;     /* HIP device ordinal that holds the map */
    int64_t max_leaves; /* capacity in 8^3 leaves, 1 .. 2^26 */
    int64_t max_voxels; /* capacity in voxel records, 1 .. 2^31 - 1; records are allocated per
                           8 x 8-voxel slab of a leaf, so this rounds up to a multiple of 64 and
                           a slab holds 64 records once any of its voxels is observed */
} slim_map_config;

typedef struct slim_stats {
    int64_t leaves;              /* leaves allocated */
    int64_t voxels;              /* voxels with W > 0 */
    int64_t points_last;         /* points passed to the last slim_integrate */
    int64_t rejected_last;       /* of those, rejected (non-finite, out of range, bad label, key range) */
    int64_t pairs_last;          /* voxel updates (point, voxel) of the last frame */
    int64_t touched_leaves_last; /* leaves the last frame touched */
    int64_t new_leaves_last;     /* leaves it created */
    int64_t voxels_old_last;     /* voxels it updated that already existed */
    int64_t voxels_new_last;     /* voxels it created */
    int32_t status_last;         /* SLIM_OK, or the error the last frame hit on the GPU */
    int32_t reserved;
} slim_stats;

/* Creates an empty map on config->device: the sparse voxel store of Sec. III-A
 * (voxels near the surface holding signed distance, weight and semantic
 * parameters; the role of OpenVDB's tree, Sec. II-C, with O(1) lookup and
 * insertion and no preset bounds), here 8^3-voxel leaves found by a hashed
 * leaf table, with D and W per voxel and the semantic state of Sec. III-C or
 * III-D.  Allocates every device buffer the configured
 * capacity needs (leaf table, leaf index, voxel records).  *out receives the
 * handle.  SLIM_ERR_INVALID on a bad configuration, SLIM_ERR_DEVICE if
 * allocation fails. */
slim_status slim_map_create(const slim_map_config *config, slim_map **out);

/* Frees the map after waiting for all work on its device.  NULL is a no-op.
 * (Lifetime of the voxel store of Sec. III-A; no paper equation.) */
slim_status slim_map_destroy(slim_map *map);

/* Empties the map (no leaves, no voxels) and keeps its capacity: the empty
 * store a sequence of frames starts from (Sec. III-A).  Queued on `stream`. */
slim_status slim_map_reset(slim_map *map, void *stream);

/* Integrates one frame (Sec. III-A to III-D): for each of the n points,
 * points_dev[3 i .. 3 i + 2] (float, sensor frame, metres), the band walk of
 * the ray from the sensor origin, the TSDF update of every voxel on it whose
 * signed distance exceeds -sdf_trunc, and the semantic update of the same
 * voxels with the same unit weight.  pose_host is map_T_sensor, 4x4 row-major
 * double; the sensor origin is its translation.  Geometry is computed in
 * binary32 relative to the origin's voxel (the anchor, floor(t / voxel_size)
 * in double); an origin 2^20 or more voxels out is anchored at +2^20, and each
 * point whose walk then leaves |k| < 2^20 is rejected.  sem_dev holds the
 * per-point semantics in the layout sem_kind names (NULL for SLIM_IN_NONE).
 * Per-voxel results equal one batch update per voxel with all of the frame's
 * observations of that voxel, which is what the paper's per-point recursion
 * reaches (Thm. 1 and 2 are stated for sets); observations are combined in
 * point order, so repeated runs are bitwise identical.
 * Rejected points (non-finite, range outside [min_range, max_range], label
 * outside [0, K), a walk leaving |k| < 2^20) contribute nothing and are
 * counted.  Requires n < 2^23.  Queued on `stream`; the frame is applied
 * entirely or not at all: if it needs more leaves or voxels than configured,
 * the map is left unchanged and the next slim_map_stats reports
 * SLIM_ERR_CAPACITY.  Synchronous validation errors return SLIM_ERR_INVALID
 * with nothing queued. */
slim_status slim_integrate(slim_map *map, const float *points_dev, int64_t n, const double *pose_host,
                           const void *sem_dev, int32_t sem_kind, void *stream);

/* As slim_integrate, with the points back-projected from a depth image (the
 * RGB-D input of Sec. III-A): depth_dev is float [height x width] row-major,
 * metres along the optical axis; intrinsics_host = {fx, fy, cx, cy}.  Pixel
 * (u, v) is point i = v * width + u at (((u - cx) / fx) d, ((v - cy) / fy) d,
 * d), each operation rounded to binary32 in that order; a depth that is not
 * finite and positive rejects the pixel.  sem_dev holds one row per pixel in
 * the same order.  Requires width * height < 2^23. */
slim_status slim_integrate_depth(slim_map *map, const float *depth_dev, int32_t width, int32_t height,
                                 const float *intrinsics_host, const double *pose_host, const void *sem_dev,
                                 int32_t sem_kind, void *stream);

/* Synchronises `stream` and copies the map's counters to *out_host: leaves and
 * voxels of the store (Sec. III-A), and the last frame's points, rejections,
 * voxel updates and touched/new leaves and voxels (the quantities the
 * integration of Sec. III-A to III-D produces per frame).  Returns the first
 * asynchronous error since the previous call (then cleared), else SLIM_OK. */
slim_status slim_map_stats(slim_map *map, slim_stats *out_host, void *stream);

/* Exports every voxel with W > 0, ordered by leaf coordinate (x, then y, then
 * z) and, inside a leaf, by offset (x, then y, then z).  Synchronises
 * `stream`.  *count_host receives the voxel count M.  With capacity == 0 only
 * the count is returned.  Otherwise capacity must be >= M, and the call
 * writes keys_dev (int32 [M x 3] voxel coordinates), d_dev and w_dev (float
 * [M] TSDF and weight) and, unless NULL, sem_dev (float [M x S]: the K class
 * counts, or the L means followed by the L betas; for the most-recent modes
 * the class index (S = 1) or the embedding (S = L); S = 0 for geometry-only
 * maps).  Counts c are stored without prior: the Dirichlet posterior is
 * alpha0 + c and its predictive is (alpha0 + c_i) / (K alpha0 + sum c)
 * (Eq. (7)).  Any async error pending on the map is returned first. */
slim_status slim_extract(slim_map *map, int64_t capacity, int32_t *keys_dev, float *d_dev, float *w_dev,
                         float *sem_dev, int64_t *count_host, void *stream);

/* Maximum leaves of a map that slim_extract_noalloc exports. */
#define SLIM_EXTRACT_NOALLOC_MAX_LEAVES (1LL << 20)

/* As slim_extract, for callers that cannot allocate device memory (code around
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, outputs and errors, and it calls no hipMalloc, hipFree or
 * other allocating routine.  Its per-leaf scratch (16 bytes a leaf) is a
 * fixed device array of the library of 16 MiB, one per GPU, held until the
 * process ends; a map with more than SLIM_EXTRACT_NOALLOC_MAX_LEAVES leaves is
 * refused with SLIM_ERR_CAPACITY before anything is queued.  Every call on one
 * GPU shares that array: calls that overlap on one GPU (several host threads,
 * or streams not synchronised with each other) race and must not be made.
 * Synchronises `stream` before returning, as slim_extract does. */
slim_status slim_extract_noalloc(slim_map *map, int64_t capacity, int32_t *keys_dev, float *d_dev, float *w_dev,
                                 float *sem_dev, int64_t *count_host, void *stream);

/* Sparse querying of the map (Sec. III-A: the store gives fast querying; O(1)
 * lookup, Sec. II-C): looks up the voxels holding m world points xyz_dev (float [m x 3]),
 * voxel floor(x / voxel_size) in binary32, and writes their state: d_dev,
 * w_dev (float [m]) and, unless NULL, sem_dev (float [m x S], as
 * slim_extract).  Unobserved voxels, and points with non-finite or
 * out-of-range coordinates, read as all zeros (W = 0).  Queued on `stream`. */
slim_status slim_query(slim_map *map, const float *xyz_dev, int64_t m, float *d_dev, float *w_dev, float *sem_dev,
                       void *stream);

/* Parameters of slim_predict (host struct; the prototypes live on the device). */
typedef struct slim_predict_params {
    float alpha0;                /* closed set: symmetric Dirichlet prior added to the counts, > 0 */
    float temperature;           /* open set: softmax temperature over cosine similarities, > 0 */
    float threshold;             /* largest class probability below this -> label -1 (T_p, Sec. III-D) */
    int32_t num_prototypes;      /* open set: class prototypes, 1..1024 */
    const float *prototypes_dev; /* open set: float [num_prototypes x L] row-major */
} slim_predict_params;

/* Semantic read-out at m world points xyz_dev (float [m x 3]), one voxel each
 * (floor(x / voxel_size), binary32).  Closed set: prob_dev (float [m x K],
 * unless NULL) receives the Dirichlet predictive (alpha0 + c_i) /
 * (K alpha0 + sum c) of Eq. (7) -- the prior's 1/K for unobserved voxels.
 * Open set: prob_dev (float [m x num_prototypes], unless NULL) receives the
 * softmax over cos(mean, prototype_j) / temperature (0 for unobserved
 * voxels), the mean being the location of the Student-t predictive of
 * Eq. (15); var_dev (float [m x L], unless NULL) receives that Student-t's
 * variance with lambda = 2 nu = W, 2 beta (W + 1) / (W (W - 2)), NaN for
 * W <= 2.  label_dev (int32 [m], unless NULL): the first index of the largest
 * probability, or -1 if the voxel is unobserved or that probability is below
 * threshold.  Most-recent modes: closed -> the stored class, one-hot; open ->
 * the prototype softmax of the stored embedding; var_dev must be NULL.
 * Geometry-only maps: SLIM_ERR_UNSUPPORTED.  Queued on `stream`. */
slim_status slim_predict(slim_map *map, const float *xyz_dev, int64_t m, const slim_predict_params *params,
                         float *prob_dev, int32_t *label_dev, float *var_dev, void *stream);

/* Renders the map from a pinhole camera: pose_host is map_T_camera (4 x 4
 * row-major FP64), intrinsics_host {fx, fy, cx, cy}.  Pixel (u, v) casts the
 * ray through ((u - cx) / fx, (v - cy) / fy, 1) (binary32, formed as a sensor
 * point at unit depth is), walked cell by cell as in integration over
 * distances [near, far] along the ray.  The surface is the first pair of
 * consecutive observed cells with D > 0 followed by D <= 0; depth_dev
 * (float [height x width]) receives the distance along the ray where D,
 * interpolated linearly between the two cells' centre projections onto the
 * ray, is zero (NaN: no surface); key_dev (int32 [height x width x 3], unless
 * NULL) the voxel behind the surface; label_dev (int32 [height x width],
 * unless NULL) its class (closed set: first largest count; most-recent closed
 * set: the stored class; otherwise, or without a surface, -1).  The map-
 * viewing role NanoVDB plays in Sec. III-E.  Queued on `stream`. */
slim_status slim_render(slim_map *map, const double *pose_host, const float *intrinsics_host, int32_t width,
                        int32_t height, float near_dist, float far_dist, float *depth_dev, int32_t *key_dev,
                        int32_t *label_dev, void *stream);

/* As slim_integrate, with each point given as a range along a direction:
 * point i is ranges_dev[i] * dirs_dev[3 i .. 3 i + 2] (one binary32 product per
 * component; dirs are unit vectors in the sensor frame).  A non-finite range
 * rejects the point. */
slim_status slim_integrate_rays(slim_map *map, const float *ranges_dev, const float *dirs_dev, int64_t n,
                                const double *pose_host, const void *sem_dev, int32_t sem_kind, void *stream);

/* Map loss of a closed-set map (differentiation workload):
 *   L = (1/m) sum_v -log p_v(labels_v)  +  (1/M') sum_s |D(v_s)|
 * where p_v(i) = (alpha0 + c_vi) / (K alpha0 + sum_i c_vi) is the Dirichlet
 * posterior predictive (Eq. (7)), the first sum runs over the m voxels listed in
 * keys_dev (int32 [m x 3]; they must be all voxels of the map, e.g. from
 * slim_extract) with ground-truth classes labels_dev (int32 [m]), and the second
 * over the M' of the s world points samples_dev (float [s x 3]) whose voxel
 * (floor(x / voxel_size), binary32 division) is in the map.  Writes
 * loss_dev[0..2] = (L, first term, second term) on the device and keeps the
 * per-voxel adjoints dL/dc and dL/dD for slim_backward_rays.  A voxel whose label
 * is outside [0, K) adds no cross-entropy term and gets dL/dc = 0 (it still
 * counts in m, and its surface samples count); voxels not listed get zero
 * adjoints.  Sums are formed in a fixed order (bitwise repeatable).  Queued on `stream`; the first call on a
 * map allocates the adjoint buffers (synchronising).  SLIM_ERR_UNSUPPORTED for
 * open-set or geometry-only maps. */
slim_status slim_map_loss(slim_map *map, const int32_t *keys_dev, const int32_t *labels_dev, int64_t m,
                          const float *samples_dev, int64_t s, float alpha0, float *loss_dev, void *stream);

/* Gradient of the last slim_map_loss with respect to the logits and ranges of
 * one frame that was integrated with slim_integrate_rays(SLIM_IN_LOGIT_F32) into
 * the map (same arguments; the map must not have changed since the loss).  For
 * each point, the band walk is recomputed and
 *   dL/dlogit_k = p_k (G_k - sum_i p_i G_i),  G = sum over its voxels of dL/dc_v,
 *   dL/drange   = sum over its voxels with sdf < tau of dL/dD_v / W_v
 * (p the softmax of the point's logits; d sdf / d range = 1 along the ray).
 * Writes grad_logits_dev (float [n x K]) and grad_ranges_dev (float [n]);
 * rejected points get zeros.  grad_scale_dev (float [1], may be NULL = 1)
 * multiplies both.  K <= 32.  Queued on `stream`. */
slim_status slim_backward_rays(slim_map *map, const float *ranges_dev, const float *dirs_dev, int64_t n,
                               const double *pose_host, const float *logits_dev, const float *grad_scale_dev,
                               float *grad_logits_dev, float *grad_ranges_dev, void *stream);

/* One frame of a batched integration: either points (points != NULL) or
 * ranges and directions, as for slim_integrate / slim_integrate_rays. */
typedef struct slim_frame {
    const float *points; /* dev, n x 3 sensor frame, or NULL */
    const float *ranges; /* dev, n, with dirs */
    const float *dirs;   /* dev, n x 3 unit sensor-frame directions */
    int64_t n;
    double pose[16];     /* map_T_sensor, row-major */
    const void *sem;     /* dev, layout per sem_kind */
    int32_t sem_kind;    /* SLIM_IN_* */
    int32_t reserved;
} slim_frame;

/* Integrates frames[i] into maps[i] for i < nmaps, for maps of any mix of
 * modes, classes and embedding sizes on one device, as one persistent launch
 * for all maps (or, by slim_launch_shape.batch_mode, one launch per kernel
 * stage for all maps) instead of six per map.  Results are identical to nmaps
 * calls of slim_integrate.  With use_graph != 0 the work is captured once into
 * a HIP graph (the descriptor copy and the launch), which later calls with the
 * same maps, the same per-map walk grid (ceil(n_i / 256) blocks) and the same
 * launch shape replay; point counts, poses and buffers may change between
 * replays.
 * Maps must be distinct.  The launch resources belong to maps[0] (the first
 * call allocates them, synchronising).  Queued on `stream`. */
slim_status slim_integrate_batched(slim_map *const *maps, int32_t nmaps, const slim_frame *frames, int32_t use_graph,
                                   void *stream);

/* Integrates `count` frames into one map, in order: the map and the per-frame
 * statistics afterwards are the same as after count calls of slim_integrate /
 * slim_integrate_rays (bit for bit).  Geometry-only and label maps (int32
 * labels, at most 32 classes, Bayesian mode) take consecutive frames in
 * multi-frame passes (up to slim_launch_shape.pass_frames, at most 8,
 * default 8; the last frame alone): one ray walk over all their rays, one
 * plan, bucketing, leaf kernel and commit, each voxel applying its frames'
 * observations frame by frame, Eq. (1)-(2) and Eq. (6) as for a frame alone.  This form returns after
 * the GPU has finished the call's work: a pass that exceeds the map's
 * capacity or staging table is not applied, and its frames and the later ones
 * are then integrated again one at a time, as per-frame calls would.  Other
 * maps return at once, with the ray walk of frame t + 1 on an internal stream
 * beside the rest of frame t (a second staging buffer makes them independent;
 * the walk reads no map state).  Every frame's inputs must be ready in
 * `stream` order when the call is made; at most 2^23 points in a frame.
 * frames[i] as for slim_integrate_batched.  Queued on `stream`; kernel timing
 * (slim_profile_enable) covers the pass form (one launch set per pass) and
 * single-frame calls, not the overlapped form. */
slim_status slim_integrate_sequence(slim_map *map, const slim_frame *frames_host, int32_t count, void *stream);

/* Grid sizes of the grid-stride kernels of integration: leaf planning and pair
 * bucketing blocks, and leaf-kernel blocks per compute unit (1 .. 32; default 16); and
 * pass_frames, the most frames slim_integrate_sequence takes in one pass
 * (0: the default 8, 1: one at a time, at most 8).
 * batch_mode picks the form of slim_integrate_batched: 1 one persistent launch
 * whose workgroups take ray-chunk, planning, bucketing, leaf-tile, combine and
 * commit items of every map from a queue, 2 one launch per stage, 0 the
 * default (1).  In the persistent launch the three grid sizes are the numbers
 * of planning, bucketing and leaf-tile (and combine) items of the whole batch,
 * shared between the maps in proportion to their rays, and walk_chunk is the
 * size of a ray-chunk item in blocks of 256 rays (1 .. 64, 0: the default 4).
 * Leaf tiles: a touched leaf with at most wave_pairs pairs is one wave's work
 * (16 .. 256, capped at 128 for accumulated frames; 0: the cap), and a sorted
 * leaf with more than slab_pairs pairs is split into one item per x-slab
 * (512 .. 2048; 0: 2048, what the leaf kernel's LDS holds).
 * Results do not depend on any of them (each voxel's sums are exact integers
 * or formed in frame and point order); they only move time.  NULL restores
 * the defaults.  Batched calls use the shape of maps[0]. */
typedef struct slim_launch_shape {
    int32_t plan_blocks, bucket_blocks, leaf_blocks_per_cu, pass_frames;
    int32_t batch_mode, walk_chunk, wave_pairs, slab_pairs;
} slim_launch_shape;
slim_status slim_set_launch_shape(slim_map *map, const slim_launch_shape *shape);

/* Kernel timing (measurement support, not part of the method).  While
 * enabled, slim_integrate (and each pass or single frame of
 * slim_integrate_sequence) brackets each stage of integration with HIP events
 * on the stream it launches on: index 0 ray walk and pair emission, 1 leaf
 * planning, 2 pair bucketing, 3 leaf kernel (accumulation, or sort and
 * combine), 4 wave-per-voxel combine (no kernel, and about zero time, for
 * frames whose leaf kernel combines its voxels itself), 5 commit.
 * slim_profile_read returns the accumulated per-stage time in milliseconds
 * and launch counts and resets them; n_kernels is the length of ms_host and
 * launches_host, and the call writes min(n_kernels, 6) entries.  Reading
 * synchronises `stream`. */
slim_status slim_profile_enable(slim_map *map, int32_t enable);
slim_status slim_profile_read(slim_map *map, double *ms_host, int64_t *launches_host, int32_t n_kernels,
                              void *stream);

/* The same timing per launch set (one slim_integrate call, or one pass or
 * single frame of slim_integrate_sequence), oldest first, for the sets
 * recorded since the previous call (at most 65536 are kept): frames_host[i]
 * frames in set i, ms_host[6 i + k] the time of its stage k (indexed as
 * slim_profile_read), span_ms_host[i] the time from the start of its first
 * stage to the end of its last.  Writes min(capacity, *count_host) sets,
 * *count_host receives the number recorded; clears the record.  Synchronises
 * `stream`. */
slim_status slim_profile_sets(slim_map *map, int32_t capacity, int32_t *frames_host, double *ms_host,
                              double *span_ms_host, int32_t *count_host, void *stream);

/* Message of the last failing call on this thread ("" if none). */
const char *slim_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SLIMVDB_H */
