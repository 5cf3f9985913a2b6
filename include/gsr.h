/*
 * gsr.h -- C ABI of the MI355X (gfx950) differentiable tile-based Gaussian
 * splat rasterizer.
 *
 * The operation.  The paper optimises its Gaussians (and, jointly, the camera
 * poses) for 30 iterations per keyframe with "a custom differentiable renderer
 * based on Taming 3DGS" (Sec. 5.2; joint pose/Gaussian optimisation: Sec. 1,
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
 * library never allocates or frees device memory and keeps no mutable global
 * state.  Device pointers must be 16-byte aligned.  The workspace carries the
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
 * the forward synchronises once, after counting pairs, and returns
 * GSR_ERR_CAPACITY (with nothing rendered) when M exceeds the capacity.
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

#define GSR_ABI_VERSION 1

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
#define GSR_FLAG_SYNC 1u        /* forward: synchronise once to check the pair capacity */
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
#define GSR_STAGE_DEPTH_SORT 1     /* forward: visible compaction + depth sort */
#define GSR_STAGE_EMIT 2           /* forward: pair offsets + pair emission */
#define GSR_STAGE_TILE_SORT 3      /* forward: tile sort + tile ranges */
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
    int32_t reserved[4];
} gsr_launch_config;

/* Work counters of the last forward (see gsr_query_stats). */
typedef struct gsr_stats {
    int64_t visible;      /* (view, Gaussian) items with at least one tile */
    int64_t pairs;        /* (tile, Gaussian) pairs M needed */
    int64_t evaluations;  /* sum over pixels of list entries evaluated up to the stop */
    int64_t contributors; /* sum over pixels of Gaussians composited */
    int64_t replays;      /* sum over pixels of list positions the backward replays */
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

#ifdef __cplusplus
}
#endif
#endif /* GSR_H */
