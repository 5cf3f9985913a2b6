// gsr_api.hip -- host side of the C ABI declared in include/gsr.h: argument
// checks, workspace layout and the launch sequence of each pass.  The library
// never allocates device memory; all state of a pass lives in the caller's
// workspace.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gsr_ba.h"
#include "gsr_internal.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return GSR_OK;
    return fail(GSR_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

int build_views(int32_t n_views, const gsr_camera *cams, const gsr_launch_config *cfg, gsr::ViewTable &vt) {
    if (n_views < 1 || n_views > GSR_MAX_VIEWS)
        return fail(GSR_ERR_INVALID_ARGUMENT, "n_views=%d outside 1..%d", n_views, GSR_MAX_VIEWS);
    if (!cams) return fail(GSR_ERR_INVALID_ARGUMENT, "cams is NULL");
    int tile_h = cfg && cfg->tile_h ? cfg->tile_h : 16;
    if (tile_h != 4 && tile_h != 8 && tile_h != 16 && tile_h != 32)
        return fail(GSR_ERR_UNSUPPORTED, "tile_h=%d (supported: 4, 8, 16, 32)", tile_h);
    std::memset(&vt, 0, sizeof(vt));
    vt.n_views = n_views;
    vt.tile_h = tile_h;
    uint64_t tiles = 0, pixels = 0;
    for (int v = 0; v < n_views; ++v) {
        const gsr_camera &c = cams[v];
        if (c.width < 1 || c.height < 1 || c.width > 65535 || c.height > 65535)
            return fail(GSR_ERR_INVALID_ARGUMENT, "view %d: size %dx%d outside 1..65535", v, c.width, c.height);
        if (!(c.fx > 0.f) || !(c.fy > 0.f))
            return fail(GSR_ERR_INVALID_ARGUMENT, "view %d: focal lengths must be positive", v);
        if (!(c.near_plane >= 0.f)) return fail(GSR_ERR_INVALID_ARGUMENT, "view %d: near_plane < 0", v);
        gsr::ViewInfo &vi = vt.v[v];
        vi.width = c.width;
        vi.height = c.height;
        vi.tiles_x = (c.width + gsr::kTileW - 1) / gsr::kTileW;
        vi.tiles_y = (c.height + tile_h - 1) / tile_h;
        vi.fx = c.fx;
        vi.fy = c.fy;
        vi.cx = c.cx;
        vi.cy = c.cy;
        vi.near_plane = c.near_plane;
        // Jacobian evaluated at x/z, y/z clamped to 1.3 x the half-FOV tangent
        vi.limx = 1.3f * ((float)c.width / (2.0f * c.fx));
        vi.limy = 1.3f * ((float)c.height / (2.0f * c.fy));
        vi.tile_off = (uint32_t)tiles;
        vi.pix_off = (uint32_t)pixels;
        tiles += (uint64_t)vi.tiles_x * vi.tiles_y;
        pixels += (uint64_t)c.width * c.height;
    }
    if (tiles >= 0xffffffffull || pixels >= 0xffffffffull)
        return fail(GSR_ERR_INVALID_ARGUMENT, "too many tiles or pixels in one call");
    vt.total_tiles = (uint32_t)tiles;
    vt.total_pixels = (uint32_t)pixels;
    return GSR_OK;
}

int tile_bits(uint32_t total_tiles) {
    int b = 1;
    while ((1ull << b) < total_tiles) ++b;
    return b;
}

gsr::WsLayout make_layout(uint64_t n, const gsr::ViewTable &vt, uint64_t cap) {
    using namespace gsr;
    WsLayout L{};
    const uint64_t items = n * (uint64_t)vt.n_views;
    L.items = items;
    L.cap = cap;
    L.chunks = chunk_count(cap);
    L.hist_blocks = (uint32_t)std::max<uint64_t>(1, (cap + kSortTile - 1) / kSortTile);
    L.pose_blocks = (uint32_t)std::max<uint64_t>(1, (n + kProjThreads - 1) / kProjThreads);
    const uint64_t scan_blocks = std::max<uint64_t>(1, (items + kScanTile - 1) / kScanTile);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.header = take(sizeof(WsHeader));
    L.rec = take(sizeof(Rec) * items);
    L.ulo = take(sizeof(float2) * items);
    L.zkey = take(4 * items);
    L.count = take(4 * items);
    L.scan_tmp = take(8 * scan_blocks);
    L.vis = take(4 * items);
    L.poff = take(4 * items);
    L.chunk_item = take(4 * (L.chunks + 1));
    L.item_box = take(16 * items);
    L.carry = take(4ull * 2 * kPartialStride * L.chunks);
    L.screen = take(48 * items);
    L.pkey[0] = take(4 * cap);
    L.pkey[1] = take(4 * cap);
    L.pval[0] = take(4 * cap);
    L.pval[1] = take(4 * cap);
    L.pflag = take((cap + 3) & ~uint64_t(3));
    L.hist = take(4ull * 256 * L.hist_blocks);
    L.digit_total = take(4 * 256);
    L.ranges = take(8ull * vt.total_tiles);
    L.tile_cut = take(4ull * vt.total_tiles);
    L.tile_order = take(4ull * kCostBuckets * (1 + vt.total_tiles));
    L.long_tiles = take(4ull * (3 * kMaxLongTiles + 2));
    L.pix_T = take(4ull * vt.total_pixels);
    L.pix_n = take(4ull * vt.total_pixels);
    L.partial = take(4ull * kPartialStride * cap);
    L.pose_part = take(4ull * 12 * vt.n_views * L.pose_blocks);
    L.view_seg = take(4ull * (GSR_MAX_VIEWS + 1));
    L.total = o;
    return L;
}

int check_gaussians(const gsr_gaussians *g) {
    if (!g) return fail(GSR_ERR_INVALID_ARGUMENT, "gaussians is NULL");
    if (g->n < 0 || g->n > 0x7fffffffll) return fail(GSR_ERR_INVALID_ARGUMENT, "n=%lld outside 0..2^31-1", (long long)g->n);
    if (g->sh_degree < 0 || g->sh_degree > 3)
        return fail(GSR_ERR_UNSUPPORTED, "sh_degree=%d (supported: 0..3)", g->sh_degree);
    if (g->n > 0) {
        const void *ptrs[5] = {g->means, g->log_scales, g->quats, g->opacities, g->sh};
        for (int k = 0; k < 5; ++k) {
            if (!ptrs[k]) return fail(GSR_ERR_INVALID_ARGUMENT, "Gaussian parameter pointer %d is NULL", k);
            if (reinterpret_cast<uintptr_t>(ptrs[k]) & 15u)
                return fail(GSR_ERR_INVALID_ARGUMENT, "Gaussian parameter pointer %d is not 16-byte aligned", k);
        }
    }
    return GSR_OK;
}

struct Ptrs {
    gsr::WsHeader *hdr;
    gsr::Rec *rec;
    float2 *ulo;
    uint32_t *zkey, *count, *scan_tmp, *vis, *poff, *chunk_item, *pkey[2], *pval[2], *hist, *digit_total, *pflag;
    float4 *screen;
    float *carry;
    uint4 *item_box;
    uint2 *ranges;
    uint32_t *tile_cut;
    uint32_t *tile_order;
    uint32_t *long_tiles, *view_seg;
    float *pix_T;
    uint32_t *pix_n;
    float *partial, *pose_part;
};

Ptrs carve(void *ws, const gsr::WsLayout &L) {
    char *b = static_cast<char *>(ws);
    Ptrs p;
    p.hdr = reinterpret_cast<gsr::WsHeader *>(b + L.header);
    p.rec = reinterpret_cast<gsr::Rec *>(b + L.rec);
    p.ulo = reinterpret_cast<float2 *>(b + L.ulo);
    p.zkey = reinterpret_cast<uint32_t *>(b + L.zkey);
    p.count = reinterpret_cast<uint32_t *>(b + L.count);
    p.scan_tmp = reinterpret_cast<uint32_t *>(b + L.scan_tmp);
    for (int k = 0; k < 2; ++k) {
        p.pkey[k] = reinterpret_cast<uint32_t *>(b + L.pkey[k]);
        p.pval[k] = reinterpret_cast<uint32_t *>(b + L.pval[k]);
    }
    p.pflag = reinterpret_cast<uint32_t *>(b + L.pflag);
    p.vis = reinterpret_cast<uint32_t *>(b + L.vis);
    p.poff = reinterpret_cast<uint32_t *>(b + L.poff);
    p.chunk_item = reinterpret_cast<uint32_t *>(b + L.chunk_item);
    p.carry = reinterpret_cast<float *>(b + L.carry);
    p.item_box = reinterpret_cast<uint4 *>(b + L.item_box);
    p.screen = reinterpret_cast<float4 *>(b + L.screen);
    p.tile_cut = reinterpret_cast<uint32_t *>(b + L.tile_cut);
    p.tile_order = reinterpret_cast<uint32_t *>(b + L.tile_order);
    p.long_tiles = reinterpret_cast<uint32_t *>(b + L.long_tiles);
    p.hist = reinterpret_cast<uint32_t *>(b + L.hist);
    p.digit_total = reinterpret_cast<uint32_t *>(b + L.digit_total);
    p.ranges = reinterpret_cast<uint2 *>(b + L.ranges);
    p.pix_T = reinterpret_cast<float *>(b + L.pix_T);
    p.pix_n = reinterpret_cast<uint32_t *>(b + L.pix_n);
    p.partial = reinterpret_cast<float *>(b + L.partial);
    p.pose_part = reinterpret_cast<float *>(b + L.pose_part);
    p.view_seg = reinterpret_cast<uint32_t *>(b + L.view_seg);
    return p;
}

// Caller-fixed workgroup count for persistent launches (0: as many as fit).
int persistent_ctas(const gsr_launch_config *cfg) { return cfg && cfg->persistent_ctas > 0 ? cfg->persistent_ctas : 0; }

// The pair capacity is whatever the workspace holds beyond the fixed regions;
// forward, backward and introspection all derive it the same way.
int layout_from_bytes(uint64_t n, const gsr::ViewTable &vt, size_t ws_bytes, gsr::WsLayout &L, uint64_t &cap) {
    const gsr::WsLayout L0 = make_layout(n, vt, 1);
    if (ws_bytes < L0.total) return fail(GSR_ERR_WORKSPACE_TOO_SMALL, "workspace %zu < %zu bytes", ws_bytes, L0.total);
    // largest capacity whose layout fits (the layout size grows with it);
    // per pair the workspace holds 4 key/value words and 9 moment floats
    uint64_t lo = 1, hi = (ws_bytes - L0.total) / (16 + 4 * gsr::kPartialStride) + 2;
    if (hi > 0x7ffffffeull) hi = 0x7ffffffeull;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo + 1) / 2;
        if (make_layout(n, vt, mid).total <= ws_bytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    cap = lo;
    L = make_layout(n, vt, cap);
    if (L.total > ws_bytes) return fail(GSR_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
    return GSR_OK;
}

// Optional per-stage timing events (caller-owned hipEvent_t array).
struct StageMark {
    hipEvent_t *ev;
    hipStream_t st;
    void begin(int s) const {
        if (ev) (void)hipEventRecord(ev[2 * s], st);
    }
    void end(int s) const {
        if (ev) (void)hipEventRecord(ev[2 * s + 1], st);
    }
};

// The synchronous forward's header readback: a copy into the caller's stack
// frame on the forward's stream, then a wait for that stream.  The library
// keeps no host buffers or events of its own.
int read_header_now(const gsr::WsHeader *dev_hdr, gsr::WsHeader &out, hipStream_t st) {
    int rc = check_hip(hipMemcpyAsync(&out, dev_hdr, sizeof(out), hipMemcpyDeviceToHost, st), "header copy");
    if (rc) return rc;
    return check_hip(hipStreamSynchronize(st), "stream sync");
}

// Number of tile-sort passes decides which ping-pong buffer holds the result.
int pair_result_buffer(uint32_t total_tiles) { return ((tile_bits(total_tiles) + 7) / 8) & 1; }

}  // namespace

namespace {

// Checks of the backward's arguments (those of the forward are checked by it).
int check_backward_args(const gsr_gaussians *g, const void *ws, const float *world_to_cam, const float *out_rgb,
                        const float *upstream, const gsr_gaussian_grads *grads) {
    if (!ws || !world_to_cam || !out_rgb || !upstream || !grads)
        return fail(GSR_ERR_INVALID_ARGUMENT,
                    "ws, world_to_cam, out_rgb, the upstream gradient (or target) and grads must not be NULL");
    if (g->n > 0 && (!grads->means || !grads->log_scales || !grads->quats || !grads->opacities || !grads->sh))
        return fail(GSR_ERR_INVALID_ARGUMENT, "a gradient output pointer is NULL");
    if (g->n > 0 && ((reinterpret_cast<uintptr_t>(grads->quats) | reinterpret_cast<uintptr_t>(grads->sh)) & 15u))
        return fail(GSR_ERR_INVALID_ARGUMENT, "grads->quats and grads->sh must be 16-byte aligned");
    return GSR_OK;
}

// The backward compositing's rows of unseen Gaussians to zero (see ZeroRows).
gsr::ZeroRows zero_rows(const gsr_gaussians *g, const gsr::ViewTable &vt, const gsr_gaussian_grads *grads,
                        const Ptrs &p) {
    gsr::ZeroRows zr{};
    zr.g = *grads;
    zr.count = p.count;
    zr.n = (uint64_t)g->n;
    zr.n_views = vt.n_views;
    zr.sh_k = (g->sh_degree + 1) * (g->sh_degree + 1);
    zr.per_tile = vt.total_tiles ? (zr.n + vt.total_tiles - 1) / vt.total_tiles : 0;
    return zr;
}

float l1_scale_of(const gsr::ViewTable &vt) { return 1.0f / (float)(3.0 * (double)vt.total_pixels); }

// A8, A9 and the pose gradient, after the backward compositing.
int backward_tail(const gsr_gaussians *g, const gsr::ViewTable &vt, const float *world_to_cam,
                  const gsr::WsLayout &L, uint64_t cap, const Ptrs &p, const gsr_gaussian_grads *grads,
                  float *dL_dworld_to_cam, float *dL_dtwist, const StageMark &mark, hipStream_t st) {
    using namespace gsr;
    mark.begin(GSR_STAGE_PROJECT_BWD);
    launch_pair_reduce(p.poff, p.chunk_item, cap, p.vis, p.pflag, p.partial, p.screen, p.carry, p.hdr, st);
    launch_project_bwd(*g, vt, world_to_cam, (uint64_t)g->n, p.rec, p.count, p.vis, p.hdr, p.screen, p.carry, *grads,
                       p.pose_part, L.pose_blocks, p.view_seg, vt.total_tiles == 0, st);
    if (g->n == 0)  // no Gaussian wrote a partial: the pose gradient is zero
        launch_fill_u32(reinterpret_cast<uint32_t *>(p.pose_part), 0u, 12ull * vt.n_views * L.pose_blocks, st);
    launch_pose_finalize(vt, world_to_cam, p.pose_part, L.pose_blocks, p.hdr, p.view_seg, vt.total_tiles != 0,
                         dL_dworld_to_cam, dL_dtwist, st);
    mark.end(GSR_STAGE_PROJECT_BWD);
    return check_hip(hipGetLastError(), "backward launch");
}

int backward_impl(void *ws, size_t ws_bytes, const gsr_gaussians *g, int32_t n_views, const gsr_camera *cams,
                         const float *world_to_cam, const gsr_launch_config *cfg, const float *out_rgb,
                         const float *dL_drgb, const float *target_rgb, const gsr_gaussian_grads *grads,
                         float *dL_dworld_to_cam, float *dL_dtwist, uint32_t flags, void *stream) {
    using namespace gsr;
    int rc = check_gaussians(g);
    if (rc) return rc;
    ViewTable vt;
    if ((rc = build_views(n_views, cams, cfg, vt))) return rc;
    if ((rc = check_backward_args(g, ws, world_to_cam, out_rgb, dL_drgb ? dL_drgb : target_rgb, grads))) return rc;
    WsLayout L;
    uint64_t cap = 0;
    if ((rc = layout_from_bytes((uint64_t)g->n, vt, ws_bytes, L, cap))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Ptrs p = carve(ws, L);
    const int pc = pair_result_buffer(vt.total_tiles);
    const bool pers = (flags & GSR_FLAG_PERSISTENT) != 0;
    const StageMark mark{cfg ? static_cast<hipEvent_t *>(cfg->stage_events) : nullptr, st};
    mark.begin(GSR_STAGE_COMPOSITE_BWD);
    if (pers) launch_reset_queue(p.hdr, 1, st);
    const ZeroRows zr = zero_rows(g, vt, grads, p);
    Upstream up{dL_drgb, target_rgb, 0.f};
    if (target_rgb) up.l1_scale = l1_scale_of(vt);
    launch_composite_bwd(vt, p.ranges, p.pval[pc], p.rec, p.ulo, out_rgb, up, p.pix_n, p.tile_cut, p.tile_order, p.partial,
                         reinterpret_cast<uint8_t *>(p.pflag), zr, p.hdr, pers, persistent_ctas(cfg), st);
    mark.end(GSR_STAGE_COMPOSITE_BWD);
    return backward_tail(g, vt, world_to_cam, L, cap, p, grads, dL_dworld_to_cam, dL_dtwist, mark, st);
}

// Checks of the forward's arguments; on success vt, L, cap and p describe the
// workspace.
int forward_setup(void *ws, size_t ws_bytes, const gsr_gaussians *g, int32_t n_views, const gsr_camera *cams,
                  const float *world_to_cam, const float *bg, const gsr_launch_config *cfg, const float *out_rgb,
                  gsr::ViewTable &vt, gsr::WsLayout &L, uint64_t &cap, Ptrs &p) {
    using namespace gsr;
    int rc = check_gaussians(g);
    if (rc) return rc;
    if ((rc = build_views(n_views, cams, cfg, vt))) return rc;
    if (!ws || !world_to_cam || !bg || !out_rgb)
        return fail(GSR_ERR_INVALID_ARGUMENT, "ws, world_to_cam, bg and out_rgb must not be NULL");
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return fail(GSR_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
    if ((uint64_t)g->n * (uint64_t)n_views >= 0x7fffffffull)
        return fail(GSR_ERR_INVALID_ARGUMENT, "n * n_views must stay below 2^31");
    if ((rc = layout_from_bytes((uint64_t)g->n, vt, ws_bytes, L, cap))) return rc;
    p = carve(ws, L);
    return GSR_OK;
}

// A1-A5 of a forward (projection, compaction, emission, tile sort, ranges,
// per-tile depth sort); pc: the pair buffer holding the sorted lists.  With
// schedule, every tile is also filed in tile_order by min(list length, the
// replay count tile_cut holds from the previous step): the fused
// compositing's schedule.
int forward_binning(const gsr_gaussians *g, const gsr::ViewTable &vt, const float *world_to_cam,
                    const gsr_launch_config *cfg, const gsr::WsLayout &L, uint64_t cap, const Ptrs &p, uint32_t flags,
                    bool schedule, const StageMark &mark, hipStream_t st, int &pc) {
    using namespace gsr;
    int rc = GSR_OK;
    const uint64_t n = (uint64_t)g->n;
    mark.begin(GSR_STAGE_PROJECT);
    launch_project_fwd(*g, vt, world_to_cam, n, p.rec, p.ulo, p.zkey, p.count, p.hdr, (uint32_t)cap,
                       cfg ? cfg->active_count : nullptr, st);
    mark.end(GSR_STAGE_PROJECT);
    mark.begin(GSR_STAGE_COMPACT);
    launch_visible_offsets(vt, n, p.count, p.rec, p.zkey, L.items, p.vis, p.poff, p.item_box, p.chunk_item, L.chunks,
                           p.scan_tmp, p.hdr, st);
    mark.end(GSR_STAGE_COMPACT);
    mark.begin(GSR_STAGE_EMIT);
    const uint64_t pair_grid = cap;  // every kernel reads the pair count from the header
    launch_emit_pairs(p.poff, p.chunk_item, p.item_box, pair_grid, p.pkey[0], p.pval[0], p.pflag, p.hdr, st);
    mark.end(GSR_STAGE_EMIT);
    mark.begin(GSR_STAGE_TILE_SORT);
    pc = 0;
    {
        uint32_t *k2[2] = {p.pkey[0], p.pkey[1]}, *v2[2] = {p.pval[0], p.pval[1]};
        // unstable: the per-tile depth sort fixes the order within a tile
        radix_sort_u32(k2, v2, SortCount{nullptr, p.hdr}, pair_grid, 0, tile_bits(vt.total_tiles), p.hist,
                       L.hist_blocks, p.digit_total, pc, false, st);
    }
    launch_tile_ranges(p.pkey[pc], pair_grid, p.ranges, vt.total_tiles, p.long_tiles, p.tile_order, p.hdr, st);
    // lists longer than one workgroup sorts: runs of kLongWindow, then merge passes
    int passes = cfg ? std::max(0, std::min(cfg->long_list_passes, kMaxLongPasses)) : 0;
    uint64_t long_pairs = cap, n_long = kMaxLongTiles;
    if (flags & GSR_FLAG_SYNC) {
        WsHeader h;
        if ((rc = read_header_now(p.hdr, h, st))) return rc;
        if (h.overflow)
            return fail(GSR_ERR_CAPACITY, "needs %u pairs, workspace holds %llu", h.n_pairs, (unsigned long long)cap);
        passes = 0;
        if (h.n_long > 0 && h.n_long <= kMaxLongTiles) {
            const uint32_t runs = (h.max_long + kLongWindow - 1) / kLongWindow;
            while ((1u << passes) < runs && passes < kMaxLongPasses) ++passes;
        }
        long_pairs = h.long_pairs;
        n_long = h.n_long;
    }
    const uint32_t chunk_wgs = passes > 0 ? (uint32_t)((long_pairs + kLongWindow - 1) / kLongWindow + n_long) : 0u;
    const uint32_t merge_wgs = passes > 0 ? (uint32_t)((long_pairs + kMergeWindow - 1) / kMergeWindow + n_long) : 0u;
    uint32_t *xh = p.pkey[pc ^ 1], *xl = p.pval[pc ^ 1], *yh = p.pkey[pc], *yl = p.pval[pc];
    if (passes > 0) launch_long_windows(p.ranges, p.long_tiles, passes, p.hdr, st);
    launch_tile_depth_sort(p.ranges, vt.total_tiles, p.pval[pc], p.zkey, xh, xl, yh, yl, p.long_tiles, passes,
                           chunk_wgs, schedule ? p.tile_order : nullptr, p.tile_cut, p.hdr, st);
    for (int q = 0; q < passes; ++q) {
        // the runs start in x when the pass count is odd, so that the last pass reads x
        const bool from_x = ((passes - q) & 1) != 0;
        launch_long_merge(p.ranges, p.long_tiles, p.hdr, q, passes, from_x ? xh : yh, from_x ? xl : yl,
                          from_x ? yh : xh, from_x ? yl : xl, p.pval[pc], merge_wgs, st);
    }
    mark.end(GSR_STAGE_TILE_SORT);
    return GSR_OK;
}

}  // namespace

extern "C" {

int gsr_version(void) { return GSR_ABI_VERSION; }

const char *gsr_status_string(int status) {
    switch (status) {
        case GSR_OK: return "GSR_OK";
        case GSR_ERR_INVALID_ARGUMENT: return "GSR_ERR_INVALID_ARGUMENT";
        case GSR_ERR_WORKSPACE_TOO_SMALL: return "GSR_ERR_WORKSPACE_TOO_SMALL";
        case GSR_ERR_CAPACITY: return "GSR_ERR_CAPACITY";
        case GSR_ERR_HIP: return "GSR_ERR_HIP";
        case GSR_ERR_UNSUPPORTED: return "GSR_ERR_UNSUPPORTED";
        default: return "GSR_ERR_UNKNOWN";
    }
}

const char *gsr_last_error(void) { return g_last_error.c_str(); }

size_t gsr_workspace_bytes(int64_t n, int32_t n_views, const gsr_camera *cams, int64_t pair_capacity,
                           const gsr_launch_config *cfg) {
    gsr::ViewTable vt;
    if (n < 0 || n > 0x7fffffffll) return (size_t)fail(0, "n=%lld outside 0..2^31-1", (long long)n);
    if (pair_capacity < 1 || pair_capacity >= 0x7fffffffll)
        return (size_t)fail(0, "pair_capacity=%lld outside 1..2^31-2", (long long)pair_capacity);
    if (build_views(n_views, cams, cfg, vt) != GSR_OK) return 0;
    if ((uint64_t)n * (uint64_t)n_views >= 0x7fffffffull)
        return (size_t)fail(0, "n * n_views must stay below 2^31");
    return make_layout((uint64_t)n, vt, (uint64_t)pair_capacity).total;
}

int gsr_rasterize_forward(void *ws, size_t ws_bytes, const gsr_gaussians *g, int32_t n_views,
                          const gsr_camera *cams, const float *world_to_cam, const float *bg,
                          const gsr_launch_config *cfg, float *out_rgb, float *out_T, uint32_t flags, void *stream) {
    using namespace gsr;
    ViewTable vt;
    WsLayout L;
    uint64_t cap = 0;
    Ptrs p;
    int rc = forward_setup(ws, ws_bytes, g, n_views, cams, world_to_cam, bg, cfg, out_rgb, vt, L, cap, p);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const StageMark mark{cfg ? static_cast<hipEvent_t *>(cfg->stage_events) : nullptr, st};
    int pc = 0;
    if ((rc = forward_binning(g, vt, world_to_cam, cfg, L, cap, p, flags, false, mark, st, pc))) return rc;
    const bool pers = (flags & GSR_FLAG_PERSISTENT) != 0;
    mark.begin(GSR_STAGE_COMPOSITE_FWD);
    launch_composite_fwd(vt, p.ranges, p.pval[pc], p.rec, p.ulo, make_float3(bg[0], bg[1], bg[2]), out_rgb, out_T,
                         p.pix_T, p.pix_n, p.tile_cut, p.tile_order, p.hdr, pers, persistent_ctas(cfg),
                         (flags & GSR_FLAG_STATS) != 0, st);
    mark.end(GSR_STAGE_COMPOSITE_FWD);
    return check_hip(hipGetLastError(), "forward launch");
}

int gsr_rasterize_backward(void *ws, size_t ws_bytes, const gsr_gaussians *g, int32_t n_views,
                           const gsr_camera *cams, const float *world_to_cam, const float *bg,
                           const gsr_launch_config *cfg, const float *out_rgb, const float *dL_drgb,
                           const gsr_gaussian_grads *grads, float *dL_dworld_to_cam, float *dL_dtwist, uint32_t flags,
                           void *stream) {
    (void)bg;
    if (!dL_drgb) return fail(GSR_ERR_INVALID_ARGUMENT, "dL_drgb must not be NULL");
    return backward_impl(ws, ws_bytes, g, n_views, cams, world_to_cam, cfg, out_rgb, dL_drgb, nullptr, grads,
                         dL_dworld_to_cam, dL_dtwist, flags, stream);
}

int gsr_rasterize_backward_l1(void *ws, size_t ws_bytes, const gsr_gaussians *g, int32_t n_views,
                              const gsr_camera *cams, const float *world_to_cam, const float *bg,
                              const gsr_launch_config *cfg, const float *out_rgb, const float *target_rgb,
                              const gsr_gaussian_grads *grads, float *dL_dworld_to_cam, float *dL_dtwist,
                              uint32_t flags, void *stream) {
    (void)bg;
    if (!target_rgb) return fail(GSR_ERR_INVALID_ARGUMENT, "target_rgb must not be NULL");
    return backward_impl(ws, ws_bytes, g, n_views, cams, world_to_cam, cfg, out_rgb, nullptr, target_rgb, grads,
                         dL_dworld_to_cam, dL_dtwist, flags, stream);
}

int gsr_rasterize_step_l1(void *ws, size_t ws_bytes, const gsr_gaussians *g, int32_t n_views,
                          const gsr_camera *cams, const float *world_to_cam, const float *bg,
                          const gsr_launch_config *cfg, const float *target_rgb, float *out_rgb, float *out_T,
                          const gsr_gaussian_grads *grads, float *dL_dworld_to_cam, float *dL_dtwist, uint32_t flags,
                          void *stream) {
    using namespace gsr;
    if (!target_rgb) return fail(GSR_ERR_INVALID_ARGUMENT, "target_rgb must not be NULL");
    if (flags & GSR_FLAG_STATS) {
        // the work counters come from the forward kernel: run the two passes
        int rc = gsr_rasterize_forward(ws, ws_bytes, g, n_views, cams, world_to_cam, bg, cfg, out_rgb, out_T, flags,
                                       stream);
        if (rc) return rc;
        return gsr_rasterize_backward_l1(ws, ws_bytes, g, n_views, cams, world_to_cam, bg, cfg, out_rgb, target_rgb,
                                         grads, dL_dworld_to_cam, dL_dtwist, flags, stream);
    }
    ViewTable vt;
    WsLayout L;
    uint64_t cap = 0;
    Ptrs p;
    int rc = forward_setup(ws, ws_bytes, g, n_views, cams, world_to_cam, bg, cfg, out_rgb, vt, L, cap, p);
    if (rc) return rc;
    if ((rc = check_backward_args(g, ws, world_to_cam, out_rgb, target_rgb, grads))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const StageMark mark{cfg ? static_cast<hipEvent_t *>(cfg->stage_events) : nullptr, st};
    int pc = 0;
    if ((rc = forward_binning(g, vt, world_to_cam, cfg, L, cap, p, flags, true, mark, st, pc))) return rc;
    const bool pers = (flags & GSR_FLAG_PERSISTENT) != 0;
    // the fused compositing is timed as the forward compositing stage; the
    // backward compositing stage is empty
    mark.begin(GSR_STAGE_COMPOSITE_FWD);
    launch_composite_step(vt, p.ranges, p.pval[pc], p.rec, p.ulo, make_float3(bg[0], bg[1], bg[2]), target_rgb,
                          l1_scale_of(vt), out_rgb, out_T, p.pix_T, p.pix_n, p.tile_cut, p.tile_order, p.partial,
                          reinterpret_cast<uint8_t *>(p.pflag), zero_rows(g, vt, grads, p), p.hdr, pers,
                          persistent_ctas(cfg), st);
    mark.end(GSR_STAGE_COMPOSITE_FWD);
    mark.begin(GSR_STAGE_COMPOSITE_BWD);
    mark.end(GSR_STAGE_COMPOSITE_BWD);
    return backward_tail(g, vt, world_to_cam, L, cap, p, grads, dL_dworld_to_cam, dL_dtwist, mark, st);
}

int gsr_query_pairs(const void *ws, size_t ws_bytes, int64_t *needed, int64_t *capacity, int32_t *overflowed,
                    void *stream) {
    if (!ws || ws_bytes < sizeof(gsr::WsHeader)) return fail(GSR_ERR_INVALID_ARGUMENT, "bad workspace");
    gsr::WsHeader h;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = check_hip(hipMemcpyAsync(&h, ws, sizeof(h), hipMemcpyDeviceToHost, st), "header copy");
    if (rc) return rc;
    if ((rc = check_hip(hipStreamSynchronize(st), "stream sync"))) return rc;
    if (needed) *needed = h.n_pairs;
    if (capacity) *capacity = h.pair_capacity;
    if (overflowed) *overflowed = (int32_t)h.overflow;
    return GSR_OK;
}

int gsr_query_stats(const void *ws, size_t ws_bytes, gsr_stats *out, void *stream) {
    if (!ws || ws_bytes < sizeof(gsr::WsHeader) || !out) return fail(GSR_ERR_INVALID_ARGUMENT, "bad arguments");
    gsr::WsHeader h;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = check_hip(hipMemcpyAsync(&h, ws, sizeof(h), hipMemcpyDeviceToHost, st), "header copy");
    if (rc) return rc;
    if ((rc = check_hip(hipStreamSynchronize(st), "stream sync"))) return rc;
    out->visible = h.n_visible;
    out->pairs = h.n_pairs;
    out->evaluations = (int64_t)h.evaluations;
    out->contributors = (int64_t)h.contributors;
    out->replays = (int64_t)h.replays;
    out->long_lists = h.n_long;
    out->longest_list = h.max_long;
    return GSR_OK;
}

int gsr_export_state(const void *ws, size_t ws_bytes, const gsr_gaussians *g, int32_t n_views, const gsr_camera *cams,
                     const gsr_launch_config *cfg, uint32_t *pair_tiles, uint32_t *pair_items, uint32_t *ranges,
                     float *records, float *centre_lo, uint32_t *depth_keys, uint32_t *tile_counts, void *stream) {
    using namespace gsr;
    int rc = check_gaussians(g);
    if (rc) return rc;
    ViewTable vt;
    if ((rc = build_views(n_views, cams, cfg, vt))) return rc;
    if (!ws) return fail(GSR_ERR_INVALID_ARGUMENT, "ws is NULL");
    WsLayout L;
    uint64_t cap = 0;
    if ((rc = layout_from_bytes((uint64_t)g->n, vt, ws_bytes, L, cap))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Ptrs p = carve(const_cast<void *>(ws), L);
    WsHeader h;
    if ((rc = check_hip(hipMemcpyAsync(&h, p.hdr, sizeof(h), hipMemcpyDeviceToHost, st), "header copy"))) return rc;
    if ((rc = check_hip(hipStreamSynchronize(st), "stream sync"))) return rc;
    const uint64_t m = h.overflow ? 0 : std::min<uint64_t>(h.n_pairs, cap);
    const int pc = pair_result_buffer(vt.total_tiles);
    struct Copy {
        void *dst;
        const void *src;
        size_t bytes;
    } copies[] = {
        {pair_items, p.pval[pc], 4 * m},
        {ranges, p.ranges, 8ull * vt.total_tiles},
        {records, p.rec, sizeof(Rec) * L.items},
        {centre_lo, p.ulo, sizeof(float2) * L.items},
        {depth_keys, p.zkey, 4 * L.items},
        {tile_counts, p.count, 4 * L.items},
    };
    if (pair_tiles && m > 0) launch_expand_ranges(p.ranges, vt.total_tiles, pair_tiles, p.hdr, st);
    for (const Copy &c : copies) {
        if (!c.dst || c.bytes == 0) continue;
        if ((rc = check_hip(hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyDeviceToDevice, st), "export copy"))) return rc;
    }
    return GSR_OK;
}

}  // extern "C"

namespace {

gsr::AdamScalars adam_scalars(float beta1, float beta2, float eps, int64_t step, double &bc1) {
    gsr::AdamScalars a;
    a.b1 = beta1;
    a.b2 = beta2;
    a.one_m_b1 = 1.f - beta1;
    a.one_m_b2 = 1.f - beta2;
    a.eps = eps;
    bc1 = 1.0 - std::pow((double)beta1, (double)step);
    a.inv_sqrt_bc2 = (float)(1.0 / std::sqrt(1.0 - std::pow((double)beta2, (double)step)));
    return a;
}

int check_adam_hyper(float beta1, float beta2, float eps, int64_t step) {
    if (step < 1) return fail(GSR_ERR_INVALID_ARGUMENT, "step=%lld must be >= 1", (long long)step);
    if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(GSR_ERR_INVALID_ARGUMENT, "need 0 <= beta1, beta2 < 1 and eps > 0");
    return GSR_OK;
}

int check_param_set(const float *const ptrs[5], bool sh_vec, const char *what) {
    for (int k = 0; k < 5; ++k)
        if (!ptrs[k]) return fail(GSR_ERR_INVALID_ARGUMENT, "%s: array %d is NULL", what, k);
    if (reinterpret_cast<uintptr_t>(ptrs[2]) & 15u) return fail(GSR_ERR_INVALID_ARGUMENT, "%s: quats not 16-byte aligned", what);
    if (sh_vec && (reinterpret_cast<uintptr_t>(ptrs[4]) & 15u))
        return fail(GSR_ERR_INVALID_ARGUMENT, "%s: sh not 16-byte aligned", what);
    return GSR_OK;
}

}  // namespace

extern "C" {

int gsr_adam_step(void *ws, size_t ws_bytes, int64_t n, int32_t sh_degree, int32_t n_views, const gsr_camera *cams,
                  const gsr_launch_config *cfg, const gsr_param_set *params, const gsr_gaussian_grads *grads,
                  const gsr_param_set *exp_avg, const gsr_param_set *exp_avg_sq, int64_t step,
                  const gsr_adam_config *acfg, void *stream) {
    using namespace gsr;
    if (n < 0 || n > 0x7fffffffll) return fail(GSR_ERR_INVALID_ARGUMENT, "n=%lld outside 0..2^31-1", (long long)n);
    if (sh_degree < 0 || sh_degree > 3) return fail(GSR_ERR_UNSUPPORTED, "sh_degree=%d (supported: 0..3)", sh_degree);
    if (!params || !grads || !exp_avg || !exp_avg_sq || !acfg)
        return fail(GSR_ERR_INVALID_ARGUMENT, "params, grads, exp_avg, exp_avg_sq and acfg must not be NULL");
    int rc = check_adam_hyper(acfg->beta1, acfg->beta2, acfg->eps, step);
    if (rc) return rc;
    const int K = (sh_degree + 1) * (sh_degree + 1);
    const bool sh_vec = (3 * K) % 4 == 0;
    if (n > 0) {
        const float *const sets[4][5] = {
            {params->means, params->log_scales, params->quats, params->opacities, params->sh},
            {grads->means, grads->log_scales, grads->quats, grads->opacities, grads->sh},
            {exp_avg->means, exp_avg->log_scales, exp_avg->quats, exp_avg->opacities, exp_avg->sh},
            {exp_avg_sq->means, exp_avg_sq->log_scales, exp_avg_sq->quats, exp_avg_sq->opacities, exp_avg_sq->sh}};
        const char *names[4] = {"params", "grads", "exp_avg", "exp_avg_sq"};
        for (int s = 0; s < 4; ++s)
            if ((rc = check_param_set(sets[s], sh_vec, names[s]))) return rc;
    }
    AdamArgs A{};
    A.p = *params;
    A.g = *grads;
    A.m = *exp_avg;
    A.v = *exp_avg_sq;
    A.n = (uint64_t)n;
    A.sh_k = K;
    A.n_views = n_views;
    A.count = nullptr;
    if (acfg->sparse) {
        ViewTable vt;
        if (!ws) return fail(GSR_ERR_INVALID_ARGUMENT, "sparse Adam needs the workspace of the last forward");
        if ((rc = build_views(n_views, cams, cfg, vt))) return rc;
        WsLayout L;
        uint64_t cap = 0;
        if ((rc = layout_from_bytes((uint64_t)n, vt, ws_bytes, L, cap))) return rc;
        A.count = reinterpret_cast<const uint32_t *>(static_cast<const char *>(ws) + L.count);
    }
    double bc1 = 0.0;
    A.a = adam_scalars(acfg->beta1, acfg->beta2, acfg->eps, step, bc1);
    const float lrs[6] = {acfg->lr_means, acfg->lr_log_scales, acfg->lr_quats, acfg->lr_opacities, acfg->lr_sh_dc,
                          acfg->lr_sh_rest};
    for (int k = 0; k < 6; ++k) A.step_size[k] = (float)((double)lrs[k] / bc1);
    launch_adam_step(A, static_cast<hipStream_t>(stream));
    return check_hip(hipGetLastError(), "adam launch");
}

int gsr_pose_step(float *world_to_cam, const float *dL_dtwist, float *exp_avg, float *exp_avg_sq, int32_t n_views,
                  int64_t step, float lr, float beta1, float beta2, float eps, void *stream) {
    using namespace gsr;
    if (n_views < 1 || n_views > GSR_MAX_VIEWS)
        return fail(GSR_ERR_INVALID_ARGUMENT, "n_views=%d outside 1..%d", n_views, GSR_MAX_VIEWS);
    if (!world_to_cam || !dL_dtwist || !exp_avg || !exp_avg_sq)
        return fail(GSR_ERR_INVALID_ARGUMENT, "world_to_cam, dL_dtwist, exp_avg and exp_avg_sq must not be NULL");
    int rc = check_adam_hyper(beta1, beta2, eps, step);
    if (rc) return rc;
    double bc1 = 0.0;
    const AdamScalars a = adam_scalars(beta1, beta2, eps, step, bc1);
    launch_pose_step(world_to_cam, dL_dtwist, exp_avg, exp_avg_sq, n_views, a, (float)((double)lr / bc1),
                     static_cast<hipStream_t>(stream));
    return check_hip(hipGetLastError(), "pose step launch");
}

int gsr_sim3_relocate(const gsr_param_set *params, int64_t n, const int32_t *keyframe_of, const float *sim3,
                      int32_t n_keyframes, void *stream) {
    using namespace gsr;
    if (n < 0 || n > 0x7fffffffll) return fail(GSR_ERR_INVALID_ARGUMENT, "n=%lld outside 0..2^31-1", (long long)n);
    if (n_keyframes < 0) return fail(GSR_ERR_INVALID_ARGUMENT, "n_keyframes=%d is negative", n_keyframes);
    if (!params) return fail(GSR_ERR_INVALID_ARGUMENT, "params must not be NULL");
    if (n == 0) return GSR_OK;
    if (!params->means || !params->quats || !params->log_scales || !keyframe_of || (n_keyframes > 0 && !sim3))
        return fail(GSR_ERR_INVALID_ARGUMENT, "means, quats, log_scales, keyframe_of and sim3 must not be NULL");
    if (reinterpret_cast<uintptr_t>(params->quats) & 15u)
        return fail(GSR_ERR_INVALID_ARGUMENT, "quats must be 16-byte aligned");
    launch_sim3_relocate(params->means, params->quats, params->log_scales, (uint64_t)n, keyframe_of, sim3, n_keyframes,
                         static_cast<hipStream_t>(stream));
    return check_hip(hipGetLastError(), "relocation launch");
}

}  // extern "C"

namespace {

struct CutScratch {
    size_t descend, in_cut, block_tmp, count, total;
};

constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// descend flags [n], in-cut flags [n], one word per scan block, the count
constexpr CutScratch cut_scratch_layout(uint64_t n) {
    CutScratch c{};
    c.descend = 0;
    c.in_cut = align256(n);
    c.block_tmp = c.in_cut + align256(n);
    const uint64_t blocks = (n + gsr::kScanTile - 1) / gsr::kScanTile;
    c.count = c.block_tmp + align256(4 * (blocks > 0 ? blocks : 1));
    c.total = c.count + align256(4);
    return c;
}

// The scratch-free cut takes its scratch from this device array (each device
// holds its own copy from module load until the process ends): hierarchies
// of up to 2^23 nodes, 16.0 MiB.
constexpr uint64_t kCutStaticMaxNodes = 1ull << 23;
constexpr size_t kCutStaticBytes = cut_scratch_layout(kCutStaticMaxNodes).total;
static __device__ __align__(256) uint8_t scratch[kCutStaticBytes];

constexpr int kMaxDevices = 64;

// Device address of `scratch` on the current device, looked up once per
// device with that device current.  Host code never uses the array's name
// as an address: on the host it names a stand-in, not device memory.
int static_cut_scratch(void **out) {
    static std::once_flag once[kMaxDevices];
    static void *ptr[kMaxDevices];
    static hipError_t err[kMaxDevices];
    int dev = 0;
    int rc = check_hip(hipGetDevice(&dev), "current device");
    if (rc) return rc;
    if (dev < 0 || dev >= kMaxDevices) return fail(GSR_ERR_UNSUPPORTED, "device %d beyond the first %d", dev, kMaxDevices);
    std::call_once(once[dev], [dev] { err[dev] = hipGetSymbolAddress(&ptr[dev], HIP_SYMBOL(scratch)); });
    if (err[dev] != hipSuccess)
        return fail(GSR_ERR_HIP, "address of the static cut scratch: %s", hipGetErrorString(err[dev]));
    *out = ptr[dev];
    return GSR_OK;
}

int cut_impl(const gsr_gaussians *nodes, const int32_t *parent, const int32_t *child_count, const gsr_camera *cam,
             const float *world_to_cam, float tau, void *scratch_buf, size_t scratch_bytes, int32_t *cut_nodes,
             int64_t *n_cut_device, int64_t *n_cut, void *stream);

}  // namespace

extern "C" {

size_t gsr_hierarchy_cut_scratch_bytes(int64_t n_nodes) {
    if (n_nodes < 0 || n_nodes > 0x7fffffffll) return (size_t)fail(0, "n_nodes=%lld outside 0..2^31-1", (long long)n_nodes);
    return cut_scratch_layout((uint64_t)n_nodes).total;
}

int gsr_hierarchy_cut(const gsr_gaussians *nodes, const int32_t *parent, const int32_t *child_count,
                      const gsr_camera *cam, const float *world_to_cam, float tau, void *scratch_buf,
                      size_t scratch_bytes, int32_t *cut_nodes, int64_t *n_cut_device, int64_t *n_cut, void *stream) {
    return cut_impl(nodes, parent, child_count, cam, world_to_cam, tau, scratch_buf, scratch_bytes, cut_nodes,
                    n_cut_device, n_cut, stream);
}

int gsr_hierarchy_cut_static(const gsr_gaussians *nodes, const int32_t *parent, const int32_t *child_count,
                             const gsr_camera *cam, const float *world_to_cam, float tau, int32_t *cut_nodes,
                             int64_t *n_cut_device, int64_t *n_cut, void *stream) {
    if (!nodes) return fail(GSR_ERR_INVALID_ARGUMENT, "nodes must not be NULL");
    if (nodes->n > (int64_t)kCutStaticMaxNodes)
        return fail(GSR_ERR_UNSUPPORTED, "n=%lld nodes exceeds the %llu the static scratch holds (use gsr_hierarchy_cut)",
                    (long long)nodes->n, (unsigned long long)kCutStaticMaxNodes);
    void *buf = nullptr;
    if (nodes->n > 0) {
        const int rc = static_cut_scratch(&buf);
        if (rc) return rc;
    }
    return cut_impl(nodes, parent, child_count, cam, world_to_cam, tau, buf, kCutStaticBytes, cut_nodes, n_cut_device,
                    n_cut, stream);
}

}  // extern "C"

namespace {

int cut_impl(const gsr_gaussians *nodes, const int32_t *parent, const int32_t *child_count, const gsr_camera *cam,
             const float *world_to_cam, float tau, void *scratch_buf, size_t scratch_bytes, int32_t *cut_nodes,
             int64_t *n_cut_device, int64_t *n_cut, void *stream) {
    using namespace gsr;
    if (!nodes || !cam) return fail(GSR_ERR_INVALID_ARGUMENT, "nodes and cam must not be NULL");
    if (!n_cut && !n_cut_device) return fail(GSR_ERR_INVALID_ARGUMENT, "n_cut and n_cut_device are both NULL");
    if (nodes->n < 0 || nodes->n > 0x7fffffffll)
        return fail(GSR_ERR_INVALID_ARGUMENT, "n=%lld outside 0..2^31-1", (long long)nodes->n);
    if (!(tau > 0.f)) return fail(GSR_ERR_INVALID_ARGUMENT, "tau must be positive");
    const uint64_t n = (uint64_t)nodes->n;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n_cut) *n_cut = 0;
    if (n == 0) {
        if (!n_cut_device) return GSR_OK;
        launch_store_count_i64(nullptr, n_cut_device, st);
        return check_hip(hipGetLastError(), "cut count launch");
    }
    if (!nodes->means || !nodes->log_scales || !parent || !child_count || !world_to_cam || !scratch_buf || !cut_nodes)
        return fail(GSR_ERR_INVALID_ARGUMENT, "a device pointer is NULL");
    if (reinterpret_cast<uintptr_t>(scratch_buf) & 255u)
        return fail(GSR_ERR_INVALID_ARGUMENT, "scratch must be 256-byte aligned");
    const CutScratch L = cut_scratch_layout(n);
    if (scratch_bytes < L.total) return fail(GSR_ERR_WORKSPACE_TOO_SMALL, "scratch %zu < %zu bytes", scratch_bytes, L.total);
    char *b = static_cast<char *>(scratch_buf);
    uint8_t *descend = reinterpret_cast<uint8_t *>(b + L.descend), *in_cut = reinterpret_cast<uint8_t *>(b + L.in_cut);
    uint32_t *count = reinterpret_cast<uint32_t *>(b + L.count);
    launch_hierarchy_cut_flags(nodes->means, nodes->log_scales, parent, child_count, n, world_to_cam,
                               std::max(cam->fx, cam->fy), tau, descend, in_cut, st);
    launch_compact_flags(in_cut, n, reinterpret_cast<uint32_t *>(cut_nodes), reinterpret_cast<uint32_t *>(b + L.block_tmp),
                         count, st);
    if (n_cut_device) launch_store_count_i64(count, n_cut_device, st);
    int rc = check_hip(hipGetLastError(), "cut launch");
    if (rc || !n_cut) return rc;
    uint32_t h = 0;
    if ((rc = check_hip(hipMemcpyAsync(&h, count, 4, hipMemcpyDeviceToHost, st), "cut count copy"))) return rc;
    if ((rc = check_hip(hipStreamSynchronize(st), "stream sync"))) return rc;
    *n_cut = h;
    return GSR_OK;
}

}  // namespace

extern "C" {

int gsr_hierarchy_layout(int64_t n_leaves, int32_t levels, int32_t branching, int64_t *level_start,
                         int32_t *n_levels) {
    if (n_leaves < 1 || n_leaves > 0x7fffffffll)
        return fail(GSR_ERR_INVALID_ARGUMENT, "n_leaves=%lld outside 1..2^31-1", (long long)n_leaves);
    if (levels < 0 || levels > GSR_MAX_HIERARCHY_LEVELS)
        return fail(GSR_ERR_INVALID_ARGUMENT, "levels=%d outside 0..%d", levels, GSR_MAX_HIERARCHY_LEVELS);
    if (branching < 2 || branching > 64) return fail(GSR_ERR_INVALID_ARGUMENT, "branching=%d outside 2..64", branching);
    if (!n_levels) return fail(GSR_ERR_INVALID_ARGUMENT, "n_levels must not be NULL");
    int64_t at = 0, n = n_leaves;
    int32_t l = 0;
    if (level_start) level_start[0] = 0;
    for (;;) {
        at += n;
        ++l;
        if (level_start) level_start[l] = at;
        if (l - 1 == levels || n <= 1) break;
        n = (n + branching - 1) / branching;
        if (at + n > 0x7fffffffll) return fail(GSR_ERR_INVALID_ARGUMENT, "more than 2^31-1 nodes");
    }
    *n_levels = l;
    return GSR_OK;
}

int gsr_hierarchy_build(const gsr_param_set *nodes, int32_t sh_degree, int64_t n_leaves, int32_t levels,
                        int32_t branching, int32_t *parent, int32_t *child_count, void *stream) {
    using namespace gsr;
    int64_t ls[GSR_MAX_HIERARCHY_LEVELS + 2];
    int32_t nl = 0;
    int rc = gsr_hierarchy_layout(n_leaves, levels, branching, ls, &nl);
    if (rc) return rc;
    if (sh_degree < 0 || sh_degree > 3) return fail(GSR_ERR_UNSUPPORTED, "sh_degree=%d (supported: 0..3)", sh_degree);
    if (!nodes || !parent || !child_count) return fail(GSR_ERR_INVALID_ARGUMENT, "nodes, parent and child_count must not be NULL");
    const float *const ptrs[5] = {nodes->means, nodes->log_scales, nodes->quats, nodes->opacities, nodes->sh};
    if ((rc = check_param_set(ptrs, ((sh_degree + 1) * (sh_degree + 1) * 3) % 4 == 0, "nodes"))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    launch_fill_i32(child_count, 0, (uint64_t)n_leaves, st);                          // leaves
    launch_fill_i32(parent + ls[nl - 1], -1, (uint64_t)(ls[nl] - ls[nl - 1]), st);  // roots
    for (int32_t l = 0; l + 1 < nl; ++l)
        launch_hierarchy_level(*nodes, sh_degree, (uint64_t)ls[l], (uint64_t)(ls[l + 1] - ls[l]), (uint64_t)ls[l + 1],
                               (uint32_t)branching, parent, child_count, st);
    return check_hip(hipGetLastError(), "hierarchy build launch");
}

int gsr_gather_gaussians(const gsr_gaussians *src, const int32_t *index, int64_t n_index, const int64_t *count,
                         const gsr_param_set *dst, void *stream) {
    using namespace gsr;
    int rc = check_gaussians(src);
    if (rc) return rc;
    if (!dst || n_index < 0) return fail(GSR_ERR_INVALID_ARGUMENT, "dst is NULL or n_index < 0");
    if (n_index == 0) return GSR_OK;
    if (!index || !dst->means || !dst->log_scales || !dst->quats || !dst->opacities || !dst->sh)
        return fail(GSR_ERR_INVALID_ARGUMENT, "index or a destination array is NULL");
    if ((reinterpret_cast<uintptr_t>(dst->quats) | reinterpret_cast<uintptr_t>(dst->sh)) & 15u)
        return fail(GSR_ERR_INVALID_ARGUMENT, "dst quats and sh must be 16-byte aligned");
    launch_gather_gaussians(*src, index, (uint64_t)n_index, count, *dst, static_cast<hipStream_t>(stream));
    return check_hip(hipGetLastError(), "gather launch");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Local bundle adjustment.
// ---------------------------------------------------------------------------
namespace {

struct BaLayout {
    size_t obs_rec, lm_rec, S, dc, obs_cam, free_slot, slot_cam, block_ab, block_off, pairs, rec_pos, total;
};

BaLayout ba_layout(int n_cams, int n_free, int K, int M) {
    BaLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t D = 6 * (size_t)n_free + 1, nblk = (size_t)n_free * (n_free + 1) / 2;
    const size_t max_pairs = (size_t)K * ((size_t)M + (size_t)M * (M - 1) / 2);
    L.obs_rec = take((size_t)K * M * gsr::kBaRecStride * sizeof(double));
    L.lm_rec = take((size_t)K * gsr::kBaLmStride * sizeof(double));
    L.S = take(gsr::kBaAsmSplit * (D + 1) * (D + 1) * sizeof(double));   // partial systems (pitch D + 1) + rhs + cost
    L.dc = take(D * sizeof(double));
    L.obs_cam = take((size_t)K * M * sizeof(int32_t));
    L.free_slot = take((size_t)n_cams * sizeof(int32_t));
    L.slot_cam = take((size_t)(n_free > 0 ? n_free : 1) * sizeof(int32_t));
    L.block_ab = take((nblk > 0 ? nblk : 1) * sizeof(int2));
    L.block_off = take((nblk + 1) * sizeof(uint32_t));
    L.pairs = take((max_pairs > 0 ? max_pairs : 1) * sizeof(int2));
    L.rec_pos = take((size_t)K * M * sizeof(int32_t));
    L.total = off;
    return L;
}

bool ba_sizes_ok(int32_t n_cams, int32_t n_free, int32_t K, int32_t M) {
    return n_cams >= 1 && n_cams <= 65535 && n_free >= 0 && n_free <= n_cams && n_free <= gsr::kBaMaxFree && K >= 1 &&
           K <= (1 << 24) && M >= 2 && M <= gsr::kBaMaxObs;
}

}  // namespace

struct gsr_ba_plan {
    char *ws;
    BaLayout L;
    int n_cams, F, K, M, D, nblk;
};

extern "C" {

size_t gsr_ba_workspace_bytes(int32_t n_cams, int32_t n_free, int32_t n_landmarks, int32_t max_obs) {
    if (!ba_sizes_ok(n_cams, n_free, n_landmarks, max_obs)) {
        fail(GSR_ERR_INVALID_ARGUMENT, "sizes outside n_cams 1..65535, n_free 0..min(n_cams, %d), n_landmarks 1..2^24, "
                                       "max_obs 2..%d", gsr::kBaMaxFree, gsr::kBaMaxObs);
        return 0;
    }
    return ba_layout(n_cams, n_free, n_landmarks, max_obs).total;
}

int gsr_ba_plan_create(int32_t n_cams, const int32_t *free_slot, int32_t n_landmarks, int32_t max_obs,
                       const int32_t *obs_cam, void *workspace, size_t workspace_bytes, void *stream, gsr_ba_plan **plan) {
    using namespace gsr;
    if (!plan) return fail(GSR_ERR_INVALID_ARGUMENT, "plan is NULL");
    *plan = nullptr;
    if (!free_slot || !obs_cam || !workspace) return fail(GSR_ERR_INVALID_ARGUMENT, "a pointer is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) & 255u) return fail(GSR_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
    if (n_cams < 1 || n_cams > 65535) return fail(GSR_ERR_INVALID_ARGUMENT, "n_cams=%d outside 1..65535", n_cams);
    int F = 0;
    for (int i = 0; i < n_cams; ++i) F += free_slot[i] >= 0;
    if (F > kBaMaxFree) return fail(GSR_ERR_UNSUPPORTED, "%d free keyframes (at most %d)", F, kBaMaxFree);
    if (!ba_sizes_ok(n_cams, F, n_landmarks, max_obs))
        return fail(GSR_ERR_INVALID_ARGUMENT, "n_landmarks=%d or max_obs=%d out of range (1..2^24, 2..%d)", n_landmarks,
                    max_obs, kBaMaxObs);
    std::vector<int32_t> slot_cam(F > 0 ? F : 1, -1);
    for (int i = 0; i < n_cams; ++i) {
        const int s = free_slot[i];
        if (s < -1 || s >= F || (s >= 0 && slot_cam[s] >= 0))
            return fail(GSR_ERR_INVALID_ARGUMENT, "free_slot must map the free keyframes one-to-one onto 0..%d", F - 1);
        if (s >= 0) slot_cam[s] = i;
    }
    const int K = n_landmarks, M = max_obs;
    for (int j = 0; j < K; ++j) {
        int cnt = 0;
        for (int k = 0; k < M; ++k) {
            const int c = obs_cam[(size_t)j * M + k];
            if (c < 0) continue;
            if (c >= n_cams || k != cnt)
                return fail(GSR_ERR_INVALID_ARGUMENT, "landmark %d: keyframe indices must be in 0..%d and come first", j,
                            n_cams - 1);
            for (int q = 0; q < k; ++q)
                if (obs_cam[(size_t)j * M + q] == c)
                    return fail(GSR_ERR_INVALID_ARGUMENT, "landmark %d: keyframe %d observed twice", j, c);
            ++cnt;
        }
        if (cnt < 2) return fail(GSR_ERR_INVALID_ARGUMENT, "landmark %d has %d observations (at least 2)", j, cnt);
    }
    const BaLayout L = ba_layout(n_cams, F, K, M);
    if (workspace_bytes < L.total) return fail(GSR_ERR_WORKSPACE_TOO_SMALL, "workspace %zu < %zu bytes", workspace_bytes, L.total);
    const int D = 6 * F + 1, nblk = F * (F + 1) / 2;
    int dev = 0, lds_max = 0;
    int rc = check_hip(hipGetDevice(&dev), "current device");
    if (rc) return rc;
    if ((rc = check_hip(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "LDS limit")))
        return rc;
    const size_t lds = ba_lds_bytes(D);
    if (lds > (size_t)lds_max) return fail(GSR_ERR_UNSUPPORTED, "reduced system needs %zu bytes of LDS (%d available)", lds, lds_max);
    if ((rc = check_hip(ba_allow_lds(D), "LDS attribute"))) return rc;
    // observation-pair lists of the reduced system's blocks (a <= b), each in landmark order
    std::vector<std::vector<int2>> lists((size_t)nblk);
    auto block_of = [F](int a, int b) { return a * F - a * (a - 1) / 2 + (b - a); };
    int slot[kBaMaxObs];
    for (int j = 0; j < K; ++j) {
        for (int k = 0; k < M; ++k) {
            const int c = obs_cam[(size_t)j * M + k];
            slot[k] = c >= 0 ? free_slot[c] : -1;
        }
        for (int k1 = 0; k1 < M; ++k1) {
            if (slot[k1] < 0) continue;
            const int o1 = j * M + k1;
            lists[block_of(slot[k1], slot[k1])].push_back(make_int2(o1, o1));
            for (int k2 = k1 + 1; k2 < M; ++k2) {
                if (slot[k2] < 0) continue;
                const int o2 = j * M + k2;
                if (slot[k1] < slot[k2]) lists[block_of(slot[k1], slot[k2])].push_back(make_int2(o1, o2));
                else lists[block_of(slot[k2], slot[k1])].push_back(make_int2(o2, o1));
            }
        }
    }
    // records are stored keyframe-major (free slot, then landmark): a diagonal
    // block's list is then one contiguous run of records, and the two sides of
    // an off-diagonal block's pairs advance through two runs
    std::vector<int32_t> rec_pos((size_t)K * M, -1);
    int32_t next_rec = 0;
    for (int a = 0; a < F; ++a)
        for (const int2 &e : lists[block_of(a, a)]) rec_pos[e.x] = next_rec++;
    for (auto &l : lists)
        for (int2 &e : l) e = make_int2(rec_pos[e.x], rec_pos[e.y]);
    std::vector<int2> block_ab(nblk > 0 ? nblk : 1), pairs;
    std::vector<uint32_t> block_off(nblk + 1, 0);
    for (int a = 0, b = 0; a < F; ++a)
        for (int q = a; q < F; ++q, ++b) {
            block_ab[b] = make_int2(a, q);
            block_off[b] = (uint32_t)pairs.size();
            pairs.insert(pairs.end(), lists[b].begin(), lists[b].end());
        }
    block_off[nblk] = (uint32_t)pairs.size();
    if (pairs.empty()) pairs.push_back(make_int2(0, 0));
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(workspace);
    const struct {
        size_t off;
        const void *src;
        size_t bytes;
    } up[] = {{L.obs_cam, obs_cam, (size_t)K * M * 4},
              {L.free_slot, free_slot, (size_t)n_cams * 4},
              {L.slot_cam, slot_cam.data(), slot_cam.size() * 4},
              {L.block_ab, block_ab.data(), block_ab.size() * sizeof(int2)},
              {L.block_off, block_off.data(), block_off.size() * 4},
              {L.pairs, pairs.data(), pairs.size() * sizeof(int2)},
              {L.rec_pos, rec_pos.data(), rec_pos.size() * 4}};
    for (const auto &u : up)
        if ((rc = check_hip(hipMemcpyAsync(ws + u.off, u.src, u.bytes, hipMemcpyHostToDevice, st), "structure upload")))
            return rc;
    if ((rc = check_hip(hipStreamSynchronize(st), "stream sync"))) return rc;
    gsr_ba_plan *p = static_cast<gsr_ba_plan *>(std::malloc(sizeof(gsr_ba_plan)));
    if (!p) return fail(GSR_ERR_CAPACITY, "out of host memory");
    *p = gsr_ba_plan{ws, L, n_cams, F, K, M, D, nblk};
    *plan = p;
    return GSR_OK;
}

int gsr_ba_plan_destroy(gsr_ba_plan *plan) {
    std::free(plan);
    return GSR_OK;
}

int gsr_ba_solve(const gsr_ba_plan *plan, double *poses, double *focal, double cx, double cy, double *landmarks,
                 const double *obs_uv, int32_t iterations, double lambda, double *costs, void *stream) {
    using namespace gsr;
    if (!plan) return fail(GSR_ERR_INVALID_ARGUMENT, "plan is NULL");
    if (!poses || !focal || !landmarks || !obs_uv) return fail(GSR_ERR_INVALID_ARGUMENT, "a device pointer is NULL");
    if (iterations < 0 || iterations > 1000000) return fail(GSR_ERR_INVALID_ARGUMENT, "iterations=%d outside 0..10^6", iterations);
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(GSR_ERR_INVALID_ARGUMENT, "lambda must be finite and >= 0");
    if (!std::isfinite(cx) || !std::isfinite(cy)) return fail(GSR_ERR_INVALID_ARGUMENT, "principal point must be finite");
    const BaLayout &L = plan->L;
    char *ws = plan->ws;
    BaArgs A{};
    A.poses = poses;
    A.focal = focal;
    A.landmarks = landmarks;
    A.obs_uv = obs_uv;
    A.obs_cam = reinterpret_cast<const int32_t *>(ws + L.obs_cam);
    A.free_slot = reinterpret_cast<const int32_t *>(ws + L.free_slot);
    A.slot_cam = reinterpret_cast<const int32_t *>(ws + L.slot_cam);
    A.block_ab = reinterpret_cast<const int2 *>(ws + L.block_ab);
    A.pairs = reinterpret_cast<const int2 *>(ws + L.pairs);
    A.rec_pos = reinterpret_cast<const int32_t *>(ws + L.rec_pos);
    A.block_off = reinterpret_cast<const uint32_t *>(ws + L.block_off);
    A.obs_rec = reinterpret_cast<double *>(ws + L.obs_rec);
    A.lm_rec = reinterpret_cast<double *>(ws + L.lm_rec);
    A.S = reinterpret_cast<double *>(ws + L.S);
    A.dc = reinterpret_cast<double *>(ws + L.dc);
    A.costs = costs;
    A.cx = cx;
    A.cy = cy;
    A.lambda = lambda;
    A.K = plan->K;
    A.M = plan->M;
    A.F = plan->F;
    A.D = plan->D;
    A.nblk = plan->nblk;
    launch_ba_iterations(A, iterations, static_cast<hipStream_t>(stream));
    return check_hip(hipGetLastError(), "bundle adjustment launch");
}

}  // extern "C"
