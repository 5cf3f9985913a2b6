/*
 * gsr.h -- C ABI of the MI355X (gfx950) differentiable tile-based Gaussian
 * splat rasterizer.
 *
 * The operation.  The paper optimises its Gaussians (and, jointly, the camera
 * poses) for 30 iterations per keyframe with its own differentiable renderer,
 * derived from Taming 3DGS (Sec. 5.2; joint pose/Gaussian optimisation: Sec. 1,
 * Sec. 3, Sec. 7; a node holds position, opacity, rotation, scale and SH
 * coefficients: Sec. 7).  The renderer is the 3DGS rasterizer of that lineage:
 *
 *   projection  per Gaussian and view: camera-space mean p = R_cw mu + t_cw;
 *               EWA 2D covariance J R_cw Sigma R_cw^T J^T + 0.3 I with
 *               Sigma = R(q) diag(exp(2 s)) R(q)^T; conic = its inverse;
 *               centre (fx x/z + cx, fy y/z + cy); colour
 *               max(0, sum_k sh_k Y_k(d) + 1/2) with d the unit direction from
 *               the camera centre; the exact axis-aligned box of the
 *               alpha >= 1/255 ellipse, in pixels and 16x16 tiles.
 *   binning     one (tile, depth) pair per covered tile, sorted by tile, then
 *               float32 bits of camera-space depth, then Gaussian index.
 *   compositing per pixel (centre at i + 1/2), front to back over its tile's
 *               list: alpha = min(0.99, o exp(-sigma)); skip alpha < 1/255;
 *               stop, without adding, where T (1 - alpha) < 1e-4;
 *               C = sum c_k alpha_k T_k + T_final bg.
 *   backward    exact derivatives of the above with respect to every
 *               Gaussian parameter and to each view's world->camera matrix
 *               (and its 6-DoF left-perturbation twist).
 *
 * Conventions.  All floats are IEEE binary32.  Quaternions are (w, x, y, z),
 * need not be unit length, and gradients are with respect to the raw values.
 * Opacities are activated values in [0, 1].  Scales are natural logarithms.
 * SH coefficients are laid out [n][K][3], K = (degree + 1)^2, degree <= 3, in
 * the real-SH order m = -l..l of the 3DGS basis.  world_to_cam is a row-major
 * 4x4 rigid transform with OpenCV axes (x right, y down, z forward) whose last
 * row is (0, 0, 0, 1).  Images are planar: view v occupies 3 * H_v * W_v floats
 * laid out [3][H_v][W_v], views concatenated in order.
 *
 * Memory and ownership.  Every buffer passed in is owned by the caller.  The
 * library never allocates or frees device memory, and holds no host buffers,
 * events or other state between calls apart from each thread's last-error
 * message (and the host plans of the bundle adjustment, owned by the caller
 * through gsr_ba_plan_destroy); the one exception is the device scratch of
 * gsr_hierarchy_cut_static, a fixed array in the library's code object, and
 * the per-device addresses of it that that entry point looks up once.
 * Device pointers must be 16-byte aligned.  The workspace carries the
 * forward pass's state to the backward pass: do not reuse it for another
 * forward between a forward and its backward.  One workspace per in-flight
 * iteration; calls on different workspaces and streams are independent.
 *
 * Errors.  Every entry point returns a status code; no C++ exception crosses
 * the ABI.  gsr_last_error() returns a thread-local description of the last
 * failure.  Argument checks are host-side and O(1); per-element preconditions
 * (finite values, opacity in [0, 1]) are documented, not checked.  A Gaussian
 * behind the near plane, with a zero quaternion, a degenerate 2D covariance,
 * opacity below 1/255 or no pixel centre in its box is culled.
 *
 * Pair capacity.  The number of (tile, Gaussian) pairs M is data dependent.
 * The workspace is sized for a caller-chosen pair capacity.  Without
 * GSR_FLAG_SYNC the forward never waits for the device: if M exceeds the
 * capacity the kernels skip the binning, the image is background only, the
 * overflow is recorded in the workspace header, and gsr_query_pairs (after a
 * stream synchronisation) reports it with the M needed.  With GSR_FLAG_SYNC
 * the forward synchronises once, after grouping the pairs by tile, and
 * returns GSR_ERR_CAPACITY (with nothing rendered) when M exceeds the
 * capacity; it also reads the longest tile list there and sizes the
 * multi-workgroup sort of lists longer than 4096 entries from it.
 * Without GSR_FLAG_SYNC both passes are free of host synchronisation and of
 * memset nodes, so they can be captured in a HIP graph.
 */
#ifndef GSR_H
#define GSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSR_ABI_VERSION 3

/* Status codes. */
#define GSR_OK 0
#define GSR_ERR_INVALID_ARGUMENT 1
#define GSR_ERR_WORKSPACE_TOO_SMALL 2
#define GSR_ERR_CAPACITY 3
#define GSR_ERR_HIP 4
#define GSR_ERR_UNSUPPORTED 5

/* Most views one call can render. */
#define GSR_MAX_VIEWS 32

/* Flags. */
#define GSR_FLAG_SYNC 1u        /* forward: synchronise once (pair capacity, long tile lists) */
#define GSR_FLAG_PERSISTENT 2u  /* compositing as persistent work-queue launches */
#define GSR_FLAG_STATS 4u       /* forward: also count the work (gsr_query_stats); slower */

/* Intrinsics of one view (host struct).  The pose is passed separately, as a
   device array, so that it can be optimised on the device. */
typedef struct gsr_camera {
    int32_t width, height;  /* pixels, 1..65535 */
    float fx, fy, cx, cy;   /* pinhole intrinsics, pixels */
    float near_plane;       /* cull camera-space z <= near_plane (0.2 typical) */
} gsr_camera;

/* Gaussian parameters: device pointers, float32, C-contiguous. */
typedef struct gsr_gaussians {
    int64_t n;               /* number of Gaussians, 0..2^31-1 */
    int32_t sh_degree;       /* 0..3 */
    const float *means;      /* [n][3] */
    const float *log_scales; /* [n][3] */
    const float *quats;      /* [n][4], (w, x, y, z) */
    const float *opacities;  /* [n], in [0, 1] */
    const float *sh;         /* [n][K][3] */
} gsr_gaussians;

/* Gradient outputs, same shapes as gsr_gaussians; overwritten (not
   accumulated); summed over views. */
typedef struct gsr_gaussian_grads {
    float *means;
    float *log_scales;
    float *quats;
    float *opacities;
    float *sh;
} gsr_gaussian_grads;

/* Stages of the two passes, for the optional per-stage timing events. */
#define GSR_STAGE_PROJECT 0        /* forward: per-Gaussian projection */
#define GSR_STAGE_COMPACT 1        /* forward: visible-item compaction and pair offsets */
#define GSR_STAGE_EMIT 2           /* forward: pair emission */
#define GSR_STAGE_TILE_SORT 3      /* forward: tile sort, tile ranges, per-tile depth sort */
#define GSR_STAGE_COMPOSITE_FWD 4  /* forward: compositing */
#define GSR_STAGE_COMPOSITE_BWD 5  /* backward: compositing */
#define GSR_STAGE_PROJECT_BWD 6    /* backward: per-Gaussian reduction, chain rule, pose */
#define GSR_NUM_STAGES 7

/* Launch parameters.  Zero fields take defaults.  None of them changes any
   result: tile membership is the exact alpha >= 1/255 box, so the image and
   the gradients are independent of the tile shape. */
typedef struct gsr_launch_config {
    int32_t tile_h;          /* tile height in pixels: 4, 8, 16 (default) or 32; width is 16 */
    int32_t persistent_ctas; /* workgroups of a persistent launch; 0 = as many as can be resident at once */
    /* NULL, or a host array of 2 * GSR_NUM_STAGES hipEvent_t owned by the
       caller: events[2 s] / events[2 s + 1] are recorded on the stream just
       before / after stage s of the pass being enqueued. */
    void *stage_events;
    /* Tile lists longer than 4096 entries: a forward with GSR_FLAG_SYNC sizes
       their multi-workgroup sort itself (from the longest list it measured).
       Without it, this many merge passes are enqueued (covering lists up to
       4096 * 2^long_list_passes entries, e.g. from an earlier forward's
       gsr_stats.longest_list); a list no pass covers is sorted by one
       workgroup, which is exact but slow for very long lists. */
    int32_t long_list_passes;
    int32_t reserved0;
    /* NULL, or a device int64: only Gaussians i < *active_count take part in
       the call (i < n always); the others are treated as culled (no pairs,
       zero gradients) and their parameters are never read.  It lets a size
       computed on the device, such as the count gsr_hierarchy_cut writes,
       drive the rasterizer without a host round trip (n is then the capacity
       of the parameter arrays and sizes the workspace).  Must be the same
       for a forward and its backward. */
    const int64_t *active_count;
} gsr_launch_config;

/* Work counters of the last forward (see gsr_query_stats). */
typedef struct gsr_stats {
    int64_t visible;      /* (view, Gaussian) items with at least one tile */
    int64_t pairs;        /* (tile, Gaussian) pairs M needed */
    int64_t evaluations;  /* sum over pixels of list entries evaluated up to the stop */
    int64_t contributors; /* sum over pixels of Gaussians composited */
    int64_t replays;      /* sum over pixels of list positions the backward replays */
    int64_t long_lists;   /* tiles whose list is longer than 4096 entries */
    int64_t longest_list; /* length of the longest of those (0 if none) */
} gsr_stats;

/* Library version (GSR_ABI_VERSION) and status names. */
int gsr_version(void);
const char *gsr_status_string(int status);
/* Thread-local description of this thread's last failure ("" if none). */
const char *gsr_last_error(void);

/*
 * Workspace size (host only, no device work) for n Gaussians rendered into
 * n_views views (host array cams[n_views]) with room for pair_capacity
 * (tile, Gaussian) pairs, 0 < pair_capacity < 2^31.  Returns 0 on invalid
 * arguments (see gsr_last_error).  cfg may be NULL.
 */
size_t gsr_workspace_bytes(int64_t n, int32_t n_views, const gsr_camera *cams, int64_t pair_capacity,
                           const gsr_launch_config *cfg);

/*
 * Forward pass.  ws: device workspace of ws_bytes (>= gsr_workspace_bytes with
 * the same n, views, capacity and cfg).  g: Gaussians (host struct of device
 * pointers).  cams: host array [n_views].  world_to_cam: device [n_views][16].
 * bg: host float[3] background colour.  out_rgb: device, planar images of all
 * views.  out_T: device [sum H_v W_v] final transmittance, may be NULL.
 * stream: hipStream_t (NULL = default stream).  Enqueued asynchronously
 * unless GSR_FLAG_SYNC.
 */
int gsr_rasterize_forward(void *ws, size_t ws_bytes, const gsr_gaussians *g, int32_t n_views,
                          const gsr_camera *cams, const float *world_to_cam, const float *bg,
                          const gsr_launch_config *cfg, float *out_rgb, float *out_T, uint32_t flags,
                          void *stream);

/*
 * Backward pass of the most recent forward on this workspace (same g, views,
 * cams, world_to_cam, bg, cfg).  out_rgb: the forward's output image, unchanged.
 * dL_drgb: device, same layout as out_rgb.  grads: device outputs, overwritten.
 * dL_dworld_to_cam: device [n_views][16] (row-major, last row zero), may be
 * NULL.  dL_dtwist: device [n_views][6], gradient of a left perturbation
 * exp(xi^) T with xi = (rho, phi), translation first, may be NULL.
 * Enqueued asynchronously on stream; never synchronises.
 */
int gsr_rasterize_backward(void *ws, size_t ws_bytes, const gsr_gaussians *g, int32_t n_views,
                           const gsr_camera *cams, const float *world_to_cam, const float *bg,
                           const gsr_launch_config *cfg, const float *out_rgb, const float *dL_drgb,
                           const gsr_gaussian_grads *grads, float *dL_dworld_to_cam, float *dL_dtwist,
                           uint32_t flags, void *stream);

/*
 * The same backward for the photometric loss itself: the mean absolute error
 * L = sum |C - target| / (3 sum H_v W_v) over every channel and pixel of all
 * views (the rendering loss of the optimisation, Sec. 5.2, read as L1), so
 * that dL/dC = sign(C - target) / (3 sum H_v W_v) is formed inside the
 * backward compositing instead of being passed in.  target_rgb: device, same
 * layout as out_rgb.  Other arguments, outputs and errors as for
 * gsr_rasterize_backward.
 */
int gsr_rasterize_backward_l1(void *ws, size_t ws_bytes, const gsr_gaussians *g, int32_t n_views,
                              const gsr_camera *cams, const float *world_to_cam, const float *bg,
                              const gsr_launch_config *cfg, const float *out_rgb, const float *target_rgb,
                              const gsr_gaussian_grads *grads, float *dL_dworld_to_cam, float *dL_dtwist,
                              uint32_t flags, void *stream);

/*
 * Forward and the backward of the mean absolute error (as
 * gsr_rasterize_backward_l1) in one call: the compositing forward and
 * backward run fused per tile (Sec. 5.2's rendering loss, whose gradient at a
 * pixel needs only that pixel's own colour), so the backward's replay of a
 * tile follows its forward in the same workgroup.  Outputs: out_rgb and out_T
 * as gsr_rasterize_forward, grads, dL_dworld_to_cam and dL_dtwist as
 * gsr_rasterize_backward; bitwise the same values as the two calls, and the
 * same workspace state afterwards (a later gsr_rasterize_backward on ws is
 * valid).  target_rgb: device, layout of out_rgb.  Flags as for the forward;
 * with GSR_FLAG_STATS the two passes run separately (the work counters come
 * from the forward's kernel).  Errors: those of both passes.
 */
int gsr_rasterize_step_l1(void *ws, size_t ws_bytes, const gsr_gaussians *g, int32_t n_views,
                          const gsr_camera *cams, const float *world_to_cam, const float *bg,
                          const gsr_launch_config *cfg, const float *target_rgb, float *out_rgb, float *out_T,
                          const gsr_gaussian_grads *grads, float *dL_dworld_to_cam, float *dL_dtwist, uint32_t flags,
                          void *stream);

/*
 * Pair count of the last forward on ws.  Reads the workspace header with a
 * blocking device->host copy on stream (so it waits for the forward).
 * needed: M required; capacity: M the workspace holds; overflowed: 1 if the
 * last forward skipped binning for lack of capacity.  Any output may be NULL.
 */
int gsr_query_pairs(const void *ws, size_t ws_bytes, int64_t *needed, int64_t *capacity,
                    int32_t *overflowed, void *stream);

/*
 * Work counters of the last forward on ws (for measurement).  visible and
 * pairs are always counted; evaluations, contributors and replays only by a
 * forward run with GSR_FLAG_STATS (zero otherwise).  Blocking, like
 * gsr_query_pairs.
 */
int gsr_query_stats(const void *ws, size_t ws_bytes, gsr_stats *out, void *stream);

/*
 * Introspection of the last forward's intermediate state, for stage-by-stage
 * tests and measurement (device-to-device copies enqueued on stream; call
 * gsr_query_pairs first to size the pair buffers).  Arguments as for the
 * forward that produced the workspace.  Every output may be NULL:
 *   pair_tiles, pair_items [min(M, capacity)]: the sorted pairs (global tile
 *     id = tile offset of the view + ty * tiles_x + tx; item = v n + i);
 *   ranges [2 * total tiles]: [start, end) of each tile in the sorted pairs;
 *   records [n_views n][12]: per item (u_hi, v_hi, A, B, C, opacity, r, g, b,
 *     bits(x0 | x1 << 16), bits(y0 | y1 << 16), bits(pair offset)), meaningful
 *     only where tile_counts > 0; centre_lo [n_views n][2]: (u_lo, v_lo);
 *   depth_keys [n_views n]: float32 bits of camera-space depth (culled:
 *     0xffffffff); tile_counts [n_views n]: tiles touched (0 = culled).
 */
int gsr_export_state(const void *ws, size_t ws_bytes, const gsr_gaussians *g, int32_t n_views,
                     const gsr_camera *cams, const gsr_launch_config *cfg, uint32_t *pair_tiles,
                     uint32_t *pair_items, uint32_t *ranges, float *records, float *centre_lo,
                     uint32_t *depth_keys, uint32_t *tile_counts, void *stream);

/* ------------------------------------------------------------------------
 * Parameter updates around the rasterizer.  All arrays are device memory,
 * caller-owned, 16-byte aligned, and updated in place on `stream`; no entry
 * point allocates.  Status codes and gsr_last_error() as above.
 * ------------------------------------------------------------------------ */

/* Mutable views of the five Gaussian arrays (shapes and layout of
   gsr_gaussians); also used for the optimiser's two moment arrays. */
typedef struct gsr_param_set {
    float *means;
    float *log_scales;
    float *quats;
    float *opacities;
    float *sh;
} gsr_param_set;

typedef struct gsr_adam_config {
    float lr_means, lr_log_scales, lr_quats, lr_opacities;
    float lr_sh_dc;    /* SH coefficient k = 0 */
    float lr_sh_rest;  /* SH coefficients k >= 1 */
    float beta1, beta2, eps;
    int32_t sparse;    /* 1: only Gaussians that some view of the last forward on ws saw are
                          updated (parameters and moments); the others are left untouched */
    int32_t reserved[4];
} gsr_adam_config;

/*
 * One Adam step of the joint optimisation (each keyframe trains the model for
 * 30 iterations of render, loss and update: Sec. 5.2; the renderer's lineage
 * optimises with Adam) from gradients such as gsr_rasterize_backward writes.
 * For every array element, with t = step >= 1:
 *   m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
 *   p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * Opacities are activated values in (0, 1): their step is taken on the logit
 * l = ln(o / (1 - o)), with g = o (1 - o) dL/do, and o <- 1 / (1 + e^-l); their
 * moments therefore refer to the logit.  Opacities are first clamped to
 * [1e-7, 1 - 1e-7].  ws/ws_bytes/n_views/cams/cfg are those of the last
 * forward (read only when acfg->sparse is set; ws may then not be NULL).
 * exp_avg and exp_avg_sq start at zero and are owned by the caller.
 */
int gsr_adam_step(void *ws, size_t ws_bytes, int64_t n, int32_t sh_degree, int32_t n_views,
                  const gsr_camera *cams, const gsr_launch_config *cfg, const gsr_param_set *params,
                  const gsr_gaussian_grads *grads, const gsr_param_set *exp_avg,
                  const gsr_param_set *exp_avg_sq, int64_t step, const gsr_adam_config *acfg, void *stream);

/*
 * Pose update of the joint optimisation: one Adam step on each view's 6-DoF
 * twist gradient (translation first, the convention of dL_dtwist in
 * gsr_rasterize_backward), then the SE(3) retraction
 *   world_to_cam <- exp(xi^) world_to_cam,  xi = -lr m_hat / (sqrt(v_hat) + eps),
 * with exp the closed-form SE(3) exponential (Rodrigues' rotation and its
 * left Jacobian for the translation), evaluated in double precision.
 * world_to_cam [n_views][16] row-major; dL_dtwist, exp_avg, exp_avg_sq
 * [n_views][6]; step >= 1; 1 <= n_views <= GSR_MAX_VIEWS.
 */
int gsr_pose_step(float *world_to_cam, const float *dL_dtwist, float *exp_avg, float *exp_avg_sq,
                  int32_t n_views, int64_t step, float lr, float beta1, float beta2, float eps, void *stream);

/*
 * Loop-closure relocation (Sec. 6.3: every Gaussian follows the Sim(3)
 * correction of the keyframe that spawned it, with its scale and rotation
 * updated accordingly).  For Gaussian i with k = keyframe_of[i] in
 * [0, n_keyframes) and sim3[k] = (s, qw, qx, qy, qz, tx, ty, tz) (unit q):
 *   mean <- s R(q) mean + t,  quat <- q * quat (Hamilton product),
 *   log-scales <- log-scales + ln s;  opacity and SH are unchanged.
 * Gaussians with k outside [0, n_keyframes) are left as they are.  The same
 * call moves hierarchy nodes (pass each node's keyframe).  keyframe_of [n]
 * and sim3 [n_keyframes][8] are device arrays.
 */
int gsr_sim3_relocate(const gsr_param_set *params, int64_t n, const int32_t *keyframe_of, const float *sim3,
                      int32_t n_keyframes, void *stream);

/* ------------------------------------------------------------------------
 * Level of detail (Sec. 7).
 * ------------------------------------------------------------------------ */

/* Bytes of device scratch memory gsr_hierarchy_cut needs for n_nodes nodes
   (0 with gsr_last_error() set for a bad n_nodes). */
size_t gsr_hierarchy_cut_scratch_bytes(int64_t n_nodes);

/*
 * Per-view cut of a Gaussian hierarchy (Sec. 7.2: rendering starts at the
 * roots and descends until a node is finer than a screen-size threshold or
 * is a leaf).  nodes: every node's parameters (only means and log_scales are
 * read; n = nodes->n); parent [n] (negative for roots), child_count [n] (0 for
 * leaves), device int32.  With S(i) = max(fx, fy) exp(max_a log_scale_a(i)) /
 * |mean(i) - camera centre| (double precision), node i is in the cut when it
 * is a leaf or S(i) < tau, and every ancestor has children and S >= tau.
 * cut_nodes [n] (device) receives the cut in ascending node order.  Its size
 * goes to n_cut_device (device int64, written on `stream`, so that a gather
 * and a rasterization enqueued after it can read it without a host round
 * trip: see gsr_gather_gaussians and gsr_launch_config.active_count) and/or
 * to *n_cut (host); at least one of the two must be given, and with n_cut the
 * call blocks until the count has been read back.  world_to_cam: device [16]
 * of the view.  scratch: device memory of gsr_hierarchy_cut_scratch_bytes(n)
 * bytes, 256-byte aligned, used only during the call's kernels.  Without
 * n_cut the call neither allocates nor synchronises, so it can be captured in
 * a HIP graph.  Ancestor chains longer than 64 (or cyclic parent links) end
 * the chain: such a node is not in the cut.
 */
int gsr_hierarchy_cut(const gsr_gaussians *nodes, const int32_t *parent, const int32_t *child_count,
                      const gsr_camera *cam, const float *world_to_cam, float tau, void *scratch,
                      size_t scratch_bytes, int32_t *cut_nodes, int64_t *n_cut_device, int64_t *n_cut,
                      void *stream);

/*
 * Scratch-free form of gsr_hierarchy_cut, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation.  Same arguments, results and errors as
 * gsr_hierarchy_cut, without scratch/scratch_bytes: the scratch comes from a
 * 16 MiB array the library keeps in device memory (one per device, from the
 * library's load until the process ends).  At most 2^23 nodes (8,388,608);
 * larger hierarchies fail with GSR_ERR_UNSUPPORTED.  It calls no allocating
 * routine; with n_cut NULL it does not synchronise either.  Every call on one
 * device shares that array: calls that overlap on a device (on different
 * streams or threads) race and must be ordered by the caller.  Each call
 * writes every scratch word it reads before reading it, so nothing carries
 * over from the previous call.
 */
int gsr_hierarchy_cut_static(const gsr_gaussians *nodes, const int32_t *parent, const int32_t *child_count,
                             const gsr_camera *cam, const float *world_to_cam, float tau, int32_t *cut_nodes,
                             int64_t *n_cut_device, int64_t *n_cut, void *stream);

/* Most merge levels gsr_hierarchy_build builds. */
#define GSR_MAX_HIERARCHY_LEVELS 30

/*
 * Node layout of a hierarchy built by gsr_hierarchy_build (host only): level 0
 * holds the n_leaves leaves, level l + 1 one node per run of `branching`
 * consecutive level-l nodes (the last run may be shorter), for `levels`
 * merge levels or until a level has a single node.  *n_levels receives the
 * number of levels including the leaves; level_start [levels + 2] (may be
 * NULL) receives the first node of each level and, after the last, the node
 * count.  1 <= n_leaves < 2^31, 0 <= levels <= GSR_MAX_HIERARCHY_LEVELS,
 * 2 <= branching <= 64.
 */
int gsr_hierarchy_layout(int64_t n_leaves, int32_t levels, int32_t branching, int64_t *level_start,
                         int32_t *n_levels);

/*
 * Builds (or refreshes, after the leaves changed) every inner node of a
 * hierarchy on the device (Sec. 7.1: groups of Gaussians are merged into one
 * node by a KL-divergence criterion).  nodes: parameter arrays holding every
 * node in the layout of gsr_hierarchy_layout; rows [0, n_leaves) are the
 * leaves, already in their grouping order (e.g. along a space-filling curve),
 * and are only read; the rows of the inner nodes are overwritten.  A parent
 * is the Gaussian that minimises KL(mixture || single) for the mixture of its
 * children weighted by opacity w_i = o_i / sum o (the mixture's mean and
 * covariance, computed in double precision), with opacity 1 - prod(1 - o_i)
 * and the w-weighted mean of the children's SH coefficients; its covariance
 * is stored as log-scales (eigenvalues ascending, variances below 1e-12
 * raised to it) and a unit quaternion with w >= 0 (eigenvectors, determinant
 * +1).  The children of a node must not all have zero opacity.  parent [n]
 * (-1 for roots) and child_count [n] (0 for leaves), device int32, receive
 * the links the level-of-detail cut reads.  Asynchronous on `stream`; no
 * allocation.
 */
int gsr_hierarchy_build(const gsr_param_set *nodes, int32_t sh_degree, int64_t n_leaves, int32_t levels,
                        int32_t branching, int32_t *parent, int32_t *child_count, void *stream);

/* Copies rows index[0 .. m) of src into rows 0 .. m of dst (all five arrays;
   src->sh_degree gives the SH row length), e.g. to rasterize a cut.  index:
   device int32, each in [0, src->n).  m = n_index, or, when count (a device
   int64, e.g. the n_cut_device of gsr_hierarchy_cut on the same stream) is
   given, min(*count, n_index) read on the device; rows of dst from m on are
   left untouched.  Never synchronises. */
int gsr_gather_gaussians(const gsr_gaussians *src, const int32_t *index, int64_t n_index, const int64_t *count,
                         const gsr_param_set *dst, void *stream);

/* ------------------------------------------------------------------------
 * Local bundle adjustment (Sec. 5.1, "Local Bundle Adjustment" and "Solver
 * efficiency"; appendix "Details on Local Pose Reconstruction", paragraph
 * "Fast Bundle Adjustment"): keyframe poses, one shared focal length and a
 * fixed set of landmarks, each seen by a fixed subset of the keyframes,
 * refined by Levenberg-Marquardt steps solved through a dense
 * Schur complement over the camera unknowns.  All arithmetic is FP64.
 *
 * Model: the observation of landmark j in keyframe i predicts
 *   f (X / Z, Y / Z) + (cx, cy),  X = R_i p_j + t_i  (world-to-camera pose);
 * residual = prediction - observation; cost = 1/2 sum |residual|^2.  A step
 * solves (H + lambda diag H) delta = -g with H = J^T J, g = J^T r over the free
 * poses (left twists exp(xi^) T, xi = (rho, phi), translation first), f and
 * the landmarks, and is always taken.  Fixed keyframes (free_slot -1) enter
 * the cost but never move.
 * ------------------------------------------------------------------------ */

/* Opaque solver plan: the problem's structure, uploaded into the caller's
   workspace.  Host object, owned by the caller through gsr_ba_plan_destroy. */
typedef struct gsr_ba_plan gsr_ba_plan;

/* Device workspace bytes for a problem with n_cams keyframes of which n_free
   are optimised (at most 20), n_landmarks landmarks (1 .. 2^24) and max_obs
   observation slots per landmark (2 .. 8).  0 with gsr_last_error() set when a
   size is out of range. */
size_t gsr_ba_workspace_bytes(int32_t n_cams, int32_t n_free, int32_t n_landmarks, int32_t max_obs);

/*
 * Checks the structure and uploads it.  free_slot [n_cams] (host): the index of
 * each optimised keyframe among the optimised ones (a one-to-one map onto
 * 0 .. n_free-1), -1 for a fixed keyframe.  obs_cam [n_landmarks][max_obs]
 * (host): the keyframes that see each landmark, valid entries first, -1 after;
 * every landmark needs at least 2 distinct keyframes.  workspace: device
 * memory of gsr_ba_workspace_bytes(...) bytes, 256-byte aligned; it must stay
 * alive, and be used by no other call, while the plan is used.  Blocking:
 * returns when the upload on `stream` has finished.  *plan receives the plan
 * (NULL on error).  Fails with GSR_ERR_UNSUPPORTED when the device cannot hold
 * the reduced system in one workgroup's LDS.
 */
int gsr_ba_plan_create(int32_t n_cams, const int32_t *free_slot, int32_t n_landmarks, int32_t max_obs,
                       const int32_t *obs_cam, void *workspace, size_t workspace_bytes, void *stream, gsr_ba_plan **plan);

/* Frees the host plan (not the workspace).  NULL is accepted. */
int gsr_ba_plan_destroy(gsr_ba_plan *plan);

/*
 * Runs `iterations` steps on `stream` (asynchronous; no allocation, no host
 * synchronisation, so a caller may capture it in a graph).  Device arrays,
 * updated in place: poses [n_cams][3][4] (row-major R | t), focal [1],
 * landmarks [n_landmarks][3].  obs_uv [n_landmarks][max_obs][2] (device): the
 * observed pixel of each valid slot (unused slots are not read).  (cx, cy):
 * principal point.  lambda >= 0: damping.  costs: NULL, or device
 * [iterations + 1] receiving the cost before each step and after the last.
 * Every observed point must stay in front of its camera (Z > 0).  A landmark
 * whose damped 3x3 block is exactly singular (in practice only with
 * lambda = 0) is not eliminated: its inverse is taken as zero, so it keeps its
 * position and its observations enter the camera system without the Schur
 * correction.  Calls that share a plan must not overlap.
 */
int gsr_ba_solve(const gsr_ba_plan *plan, double *poses, double *focal, double cx, double cy, double *landmarks,
                 const double *obs_uv, int32_t iterations, double lambda, double *costs, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GSR_H */
