// gsr_internal.h -- definitions shared by the HIP translation units of the
// rasterizer library (gfx950, wave64).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gsr.h"

namespace gsr {

constexpr int kWave = 64;
constexpr int kTileW = 16;           // tile width in pixels (one row of a wave's 16 lanes)
constexpr float kAlphaMax = 0.99f;   // alpha clamp
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;       // stop before transmittance falls below this
constexpr float kLowPass = 0.3f;     // added to the 2D covariance diagonal
constexpr float kLog2e = 1.4426950408889634f;
constexpr uint32_t kCulledKey = 0xffffffffu;

// Per-view constants passed by value in kernel arguments.
struct ViewInfo {
    int32_t width, height, tiles_x, tiles_y;
    float fx, fy, cx, cy, near_plane, limx, limy;
    uint32_t tile_off;   // first global tile id of the view
    uint32_t pix_off;    // first pixel of the view in the concatenated images
};

struct ViewTable {
    int32_t n_views;
    int32_t tile_h;        // tile height in pixels (4, 8, 16 or 32)
    uint32_t total_tiles;
    uint32_t total_pixels;
    ViewInfo v[GSR_MAX_VIEWS];
};

// Workspace header (first 256 bytes of the workspace, device memory).
struct WsHeader {
    uint32_t n_visible;      // visible (view, Gaussian) items
    uint32_t n_pairs;        // pairs needed (saturates at 0xffffffff)
    uint32_t overflow;       // 1 if n_pairs > capacity: binning was skipped
    uint32_t pair_capacity;
    unsigned long long evaluations;   // sum over pixels of list entries evaluated
    unsigned long long replays;       // sum over pixels of n_contrib
    unsigned long long contributors;  // sum over pixels of Gaussians composited
    uint32_t queue[4];       // persistent-launch work counters
    uint32_t n_long;         // tiles whose list is longer than kGroupSortMax
    uint32_t long_pairs;     // entries in those lists
    uint32_t max_long;       // the longest of them
    uint32_t pad[47];
};
static_assert(sizeof(WsHeader) == 256, "header is 256 bytes");

// Projected record of one (view, Gaussian) item, three float4:
//   r0 = (u_hi, v_hi, A, B)      conic (A, B, C) = inverse 2D covariance
//   r1 = (C, opacity, red, green)
//   r2 = (blue, bits(x0 | x1 << 16), bits(y0 | y1 << 16), bits(pair_offset))
// The inclusive pixel box (x0..x1, y0..y1) is that of the alpha >= 1/255
// ellipse.  The centre is stored as u = u_hi + u_lo (double-float) so that
// tile-relative offsets keep ~1e-6 px accuracy; the low parts live in `ulo`.
struct Rec {
    float4 r0, r1, r2;
};

// Offsets of the workspace regions, all 256-byte aligned.
struct WsLayout {
    size_t header;
    size_t rec;         // Rec[items]
    size_t ulo;         // float2[items] low parts of (u, v)
    size_t zkey;        // u32[items] depth key (float bits) or kCulledKey
    size_t count;       // u32[items] tiles touched
    size_t scan_tmp;    // u32 scratch for scans (block sums)
    size_t vis;         // u32[items] visible item ids in ascending order
    size_t poff;        // u32[items] pair offset of the k-th visible item
    size_t chunk_item;  // u32[chunks + 1] index (into vis) of the item holding each chunk's first pair
    size_t item_box;    // uint4[items] per visible index: (first tile of the box, width | tiles_x << 16, depth key, item)
    size_t carry;       // float[chunks * 2 * 9] chunk-boundary partial sums of the pair moments
    size_t screen;      // float4[items * 3] per-item sums of the pair moments
    size_t pkey[2];     // u32[cap] tile keys ping-pong
    size_t pval[2];     // u32[cap] item ids ping-pong
    size_t pflag;       // u8[cap] per pair slot (emission order): 1 once the backward compositing wrote its moments
    size_t hist;        // u32[256 * max_blocks] radix histograms
    size_t digit_total; // u32[256] radix digit totals
    size_t ranges;      // uint2[total_tiles]
    size_t tile_cut;    // u32[total_tiles]: list positions any pixel of the tile used (the backward replays those)
    size_t tile_order;  // u32[kCostBuckets] bucket counts, then u32[kCostBuckets][tiles] tile ids per bucket
    size_t long_tiles;  // u32[kMaxLongTiles] tiles whose list is longer than kGroupSortMax (any order), then
                        // u32[2][kMaxLongTiles + 1] their first window of kLongWindow / kMergeWindow entries
    size_t pix_T;       // float[total_pixels] final transmittance
    size_t pix_n;       // u32[total_pixels] last contributor + 1
    size_t partial;     // float[cap * 9] per-pair moments of the pixel gradients
    size_t pose_part;   // float[views * pose_blocks * 12]
    size_t view_seg;    // u32[GSR_MAX_VIEWS + 1] first visible index of each view
    size_t total;
    uint64_t items, cap, chunks;
    uint32_t hist_blocks, pose_blocks;
};

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;     // 1024
constexpr int kSortThreads = 256;
constexpr int kSortTile = 3072;                           // elements per sort block
constexpr int kGroupSortMax = 4096;                       // longest list one workgroup sorts in registers
constexpr uint32_t kMaxLongTiles = 1024;                  // longer lists the multi-workgroup path takes
constexpr uint32_t kLongWindow = 4096;                    // entries per sorted run of a long list
constexpr uint32_t kMergeWindow = 2048;                   // outputs per workgroup of a merge pass
constexpr int kMaxLongPasses = 16;                        // merge passes at most (lists up to 2^28 entries)
constexpr int kProjThreads = 256;
constexpr int kPartialStride = 9;                         // floats per pair gradient
// Backward tile schedule: tiles in descending buckets of their replay count
// (16 buckets per octave), so that the heaviest start first.
constexpr uint32_t kCostBuckets = 128;
// Bucket of a tile's cost (its replay count, or its list length): 16 per
// octave, floor(16 log2(n + 1)), the top bucket taking everything above 255.
__device__ __forceinline__ uint32_t cost_bucket(uint32_t n) {
    return min(kCostBuckets - 1, (uint32_t)(16.f * __log2f((float)n + 1.f)));
}
// Pairs are also processed in fixed chunks of consecutive emission-order
// slots (A3 emission, A8 reduction): 256 threads x 4 pairs.
constexpr uint32_t kChunkPairs = 1024;
constexpr uint32_t kChunkThreads = 256;
constexpr uint32_t kChunkPerThread = kChunkPairs / kChunkThreads;
__host__ __device__ constexpr uint64_t chunk_count(uint64_t pairs) { return (pairs + kChunkPairs - 1) / kChunkPairs; }

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).  All enqueue on `st`.
// ---------------------------------------------------------------------------
void launch_fill_u32(uint32_t *p, uint32_t value, uint64_t n, hipStream_t st);
void launch_reset_header(WsHeader *h, uint32_t cap, hipStream_t st);

// Also resets the workspace header (pair capacity cap) for this forward.
void launch_project_fwd(const gsr_gaussians &g, const ViewTable &vt, const float *w2c, uint64_t n,
                        Rec *rec, float2 *ulo, uint32_t *zkey, uint32_t *count, WsHeader *hdr, uint32_t cap,
                        const int64_t *active, hipStream_t st);

// Exclusive scans / compaction / sorting / binning.
// Visible items (ascending ids), their pair offsets (also into each record's
// r2.w), their box words (by visible index) and each chunk's first item;
// header: visible and pair counts, overflow.  block_tmp: 2 u32 per block of
// kScanTile items.
void launch_visible_offsets(const ViewTable &vt, uint64_t n, const uint32_t *count, Rec *rec,
                            const uint32_t *zkey, uint64_t items, uint32_t *vis, uint32_t *poff, uint4 *item_box,
                            uint32_t *chunk_item, uint64_t chunks_cap, uint32_t *block_tmp, WsHeader *hdr,
                            hipStream_t st);
// Element count of a sort, read on the device: *n_dev, or (hdr set) the pair
// count, 0 if the binning overflowed.
struct SortCount {
    const uint32_t *n_dev;
    const WsHeader *hdr;
    __device__ uint64_t operator()() const {
        if (hdr) return hdr->overflow ? 0ull : (uint64_t)hdr->n_pairs;
        return (uint64_t)*n_dev;
    }
};
// LSD sort of (key, value) on bits [begin_bit, end_bit), at most 8 per pass,
// ping-ponging between keys[cur]/keys[cur ^ 1]; `cur` ends at the result.
// Stable when `stable`; otherwise equal keys come out in an unspecified order.
void radix_sort_u32(uint32_t *keys[2], uint32_t *vals[2], SortCount sc, uint64_t n_cap, int begin_bit, int end_bit,
                    uint32_t *hist, uint32_t hist_blocks, uint32_t *digit_total, int &cur, bool stable,
                    hipStream_t st);
// Each tile's list (grouped by the tile sort, in no particular order)
// sorted by (depth key, item).  Lists longer than kGroupSortMax: with
// long_passes > 0 (and at most kMaxLongTiles of them), `chunk_wgs` extra
// workgroups sort them in runs of kLongWindow into the key buffer the first
// merge pass reads (x when long_passes is odd, else y; hi = depth key,
// lo = item); lists longer than kLongWindow << long_passes, or all long lists
// when long_passes == 0, are sorted by one workgroup in global memory
// (x_hi/x_lo as scratch).  sched (or NULL): one more workgroup files the
// fused compositing's schedule there (layout of WsLayout::tile_order): every
// tile in the bucket of min(its list length, cost_hint[t]), cost_hint being
// the previous step's replay count per tile (any values: only the order of
// the tiles depends on them).
void launch_tile_depth_sort(const uint2 *ranges, uint32_t total_tiles, uint32_t *pval, const uint32_t *zkey,
                            uint32_t *x_hi, uint32_t *x_lo, uint32_t *y_hi, uint32_t *y_lo,
                            const uint32_t *long_tiles, int long_passes, uint32_t chunk_wgs, uint32_t *sched,
                            const uint32_t *cost_hint, const WsHeader *hdr, hipStream_t st);
// Merge pass p of long_passes over the long lists' runs (run length
// kLongWindow << p); the last pass writes the item ids into pval.
// Window offsets of the long lists the multi-workgroup path takes: first
// window of each of kLongWindow entries (long_tiles + kMaxLongTiles) and of
// kMergeWindow entries (after those), with the totals at index n_long.
void launch_long_windows(const uint2 *ranges, uint32_t *long_tiles, int long_passes, const WsHeader *hdr,
                         hipStream_t st);
void launch_long_merge(const uint2 *ranges, const uint32_t *long_tiles, const WsHeader *hdr, int p, int long_passes,
                       const uint32_t *src_hi, const uint32_t *src_lo, uint32_t *dst_hi, uint32_t *dst_lo,
                       uint32_t *pval, uint32_t merge_wgs, hipStream_t st);
// Tile id of every position of the sorted pairs, from the ranges.
void launch_expand_ranges(const uint2 *ranges, uint32_t total_tiles, uint32_t *pair_tiles, const WsHeader *hdr,
                          hipStream_t st);
void launch_reset_queue(WsHeader *h, int which, hipStream_t st);
void launch_emit_pairs(const uint32_t *poff, const uint32_t *chunk_item, const uint4 *item_box, uint64_t pair_grid,
                       uint32_t *pkey, uint32_t *pval, uint32_t *pflag, const WsHeader *hdr, hipStream_t st);
// Also clears the backward schedule's bucket counts (tile_order).
void launch_tile_ranges(const uint32_t *pkey, uint64_t cap, uint2 *ranges, uint32_t total_tiles,
                        uint32_t *long_tiles, uint32_t *tile_order, WsHeader *hdr, hipStream_t st);

void launch_composite_fwd(const ViewTable &vt, const uint2 *ranges, const uint32_t *pval, const Rec *rec,
                          const float2 *ulo, float3 bg, float *out_rgb, float *out_T, float *pix_T,
                          uint32_t *pix_n, uint32_t *tile_cut, uint32_t *tile_order, WsHeader *hdr,
                          bool persistent, int persistent_ctas, bool stats, hipStream_t st);
// Gradient rows of the Gaussians no view saw are zeroed by the backward
// compositing (memory work hidden under its ALU work): tile t takes Gaussians
// [t * per_tile, (t + 1) * per_tile).
struct ZeroRows {
    gsr_gaussian_grads g;
    const uint32_t *count;  // tiles touched per (view, Gaussian)
    uint64_t n, per_tile;
    int32_t n_views, sh_k;
};
// The upstream image gradient: given (grad), or the mean absolute error
// against a target image, dL/dC = sign(C - target) * l1_scale.
struct Upstream {
    const float *grad;
    const float *target;
    float l1_scale;
};
void launch_composite_bwd(const ViewTable &vt, const uint2 *ranges, const uint32_t *pval, const Rec *rec,
                          const float2 *ulo, const float *out_rgb, const Upstream &up, const uint32_t *pix_n,
                          const uint32_t *tile_cut, const uint32_t *tile_order, float *partial, uint8_t *pflag,
                          const ZeroRows &zr, WsHeader *hdr, bool persistent, int persistent_ctas, hipStream_t st);
// A6 and A7 fused for the mean absolute error against `target` (dL/dC =
// sign(C - target) * l1_scale): the forward's outputs and workspace state
// (image, out_T, pix_T, pix_n, tile_cut) and the backward's (moments, slot
// flags, zeroed rows) in one launch; tiles in the order of `tile_order` as
// filed by launch_tile_depth_sort's sched.
void launch_composite_step(const ViewTable &vt, const uint2 *ranges, const uint32_t *pval, const Rec *rec,
                           const float2 *ulo, float3 bg, const float *target, float l1_scale, float *out_rgb,
                           float *out_T, float *pix_T, uint32_t *pix_n, uint32_t *tile_cut,
                           const uint32_t *tile_order, float *partial, uint8_t *pflag, const ZeroRows &zr,
                           WsHeader *hdr, bool persistent, int persistent_ctas, hipStream_t st);
void launch_pair_reduce(const uint32_t *poff, const uint32_t *chunk_item, uint64_t pair_grid, const uint32_t *vis,
                        const uint32_t *pflag, const float *partial, float4 *screen, float *carry, const WsHeader *hdr,
                        hipStream_t st);

// zero_unseen: also write the zero rows of the Gaussians no view saw (when the
// backward compositing did not).  seg: u32[GSR_MAX_VIEWS + 1] scratch.
void launch_project_bwd(const gsr_gaussians &g, const ViewTable &vt, const float *w2c, uint64_t n,
                        const Rec *rec, const uint32_t *count, const uint32_t *vis, const WsHeader *hdr,
                        const float4 *screen, const float *carry, const gsr_gaussian_grads &gr, float *pose_part,
                        uint32_t pose_blocks, uint32_t *seg, bool zero_unseen, hipStream_t st);
// dense: the partials come from the per-view launches over the visible items
// (only the blocks with items are summed; seg as for launch_project_bwd).
void launch_pose_finalize(const ViewTable &vt, const float *w2c, const float *pose_part, uint32_t pose_blocks,
                          const WsHeader *hdr, const uint32_t *seg, bool dense, float *dL_dw2c, float *dL_dtwist,
                          hipStream_t st);

// Ordered compaction of byte flags (gsr_sort.hip).
void launch_compact_flags(const uint8_t *flags, uint64_t n, uint32_t *out_idx, uint32_t *block_tmp,
                          uint32_t *out_count, hipStream_t st);
inline uint64_t scan_blocks_for(uint64_t n) { return (n + kScanTile - 1) / kScanTile; }

// Level-of-detail cut and row gather (gsr_hierarchy.hip).
void launch_hierarchy_cut_flags(const float *means, const float *log_scales, const int32_t *parent,
                                const int32_t *child_count, uint64_t n, const float *w2c, float focal, float tau,
                                uint8_t *descend, uint8_t *in_cut, hipStream_t st);
void launch_gather_gaussians(const gsr_gaussians &src, const int32_t *index, uint64_t n_out, const int64_t *count,
                             const gsr_param_set &dst, hipStream_t st);
void launch_store_count_i64(const uint32_t *count, int64_t *out, hipStream_t st);
void launch_hierarchy_level(const gsr_param_set &nodes, int sh_degree, uint64_t child_base, uint64_t n_child,
                            uint64_t parent_base, uint32_t branching, int32_t *parent, int32_t *child_count,
                            hipStream_t st);
void launch_fill_i32(int32_t *p, int32_t value, uint64_t n, hipStream_t st);

// Parameter updates (gsr_update.hip).
struct AdamScalars {
    float b1, b2, one_m_b1, one_m_b2, eps;
    float inv_sqrt_bc2;  // 1 / sqrt(1 - b2^t)
};
struct AdamArgs {
    gsr_param_set p, m, v;
    gsr_gaussian_grads g;
    const uint32_t *count;  // tiles touched per (view, Gaussian) of the last forward; NULL = update all
    uint64_t n;
    int32_t n_views, sh_k;  // sh_k = (degree + 1)^2
    AdamScalars a;
    float step_size[6];     // lr / (1 - b1^t): means, log-scales, quats, opacities, SH DC, SH rest
};
void launch_adam_step(const AdamArgs &A, hipStream_t st);
void launch_pose_step(float *w2c, const float *g, float *m, float *v, int n_views, const AdamScalars &a,
                      float step_size, hipStream_t st);
void launch_sim3_relocate(float *means, float *quats, float *log_scales, uint64_t n, const int32_t *keyframe_of,
                          const float *sim3, int32_t n_keyframes, hipStream_t st);

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
// One DPP step: v + (v moved across lanes by `ctrl`), only in the rows enabled
// by `row_mask` (other rows add 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v) {
    // every lane reads a source lane of its row (the controls used here have
    // no out-of-range source), so no "old" value is needed; with bound_ctrl
    // set the compiler folds the move into the add (v_add_f32_dpp)
    if constexpr (ROW_MASK == 0xf)
        return v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
    else
        return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

// Sum over the 64 lanes of a wave, with VALU data-parallel-primitive moves
// (no LDS round trips): swaps within quads, mirrors within half-rows and rows
// leave every lane with its 16-lane row's sum; two row broadcasts then
// accumulate rows 0..3 into row 3.  The total is read from lane 63 and
// returned to every lane.  Fixed order, so the result is deterministic.
__device__ __forceinline__ float wave_sum(float v) {
    v = dpp_add<0xB1, 0xf>(v);   // quad_perm [1, 0, 3, 2]
    v = dpp_add<0x4E, 0xf>(v);   // quad_perm [2, 3, 0, 1]
    v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
    v = dpp_add<0x140, 0xf>(v);  // row_mirror
    v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Inclusive prefix sum over the 64 lanes of a wave, `add` combining, with DPP
// moves that stay in the VALU: Hillis-Steele row shifts by 1, 2, 4 and 8
// within each row of 16 lanes, then the row totals by two row broadcasts
// (lane 15 into rows 1 and 3, lane 31 into rows 2 and 3).  Lanes without a
// source lane, and rows a broadcast skips, combine with 0.
template <class Add>
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x, Add add) {
    x = add(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false));  // row_shr:1
    x = add(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false));  // row_shr:2
    x = add(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false));  // row_shr:4
    x = add(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false));  // row_shr:8
    x = add(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false));  // row_bcast:15
    x = add(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return x;
}

// Reduction over the 64 lanes of a wave with `op` (associative and
// commutative, `identity` its neutral value), by the DPP pattern of wave_sum;
// every lane gets the result.
template <class Op>
__device__ __forceinline__ uint32_t wave_reduce(uint32_t x, uint32_t identity, Op op) {
    const int id = (int)identity;
    x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0xB1, 0xf, 0xf, false));   // quad_perm [1, 0, 3, 2]
    x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x4E, 0xf, 0xf, false));   // quad_perm [2, 3, 0, 1]
    x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x141, 0xf, 0xf, false));  // row_half_mirror
    x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x140, 0xf, 0xf, false));  // row_mirror
    x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x142, 0xa, 0xf, false));  // row_bcast:15
    x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

__device__ __forceinline__ uint32_t pack_u16(uint32_t lo, uint32_t hi) { return lo | (hi << 16); }

// The chip's 8 XCDs (each with its own L2) take a grid's workgroups in turn:
// workgroup b runs on XCD b % 8.  This maps b to a work index so that each XCD
// gets one contiguous range of [0, count) (a bijection for b < count), and
// neighbouring work items, which touch neighbouring data, share an L2.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t count) {
    const uint32_t q = count / kXcds, r = count % kXcds, x = b % kXcds;
    return x * q + min(x, r) + b / kXcds;
}


// ---------------------------------------------------------------------------
// The items whose pairs fall in one chunk of emission-order slots.  The k-th
// visible item (ascending item id) owns the contiguous pair range
// [poff[k], poff[k + 1]), so a chunk meets the visible indices
// chunk_item[c] .. chunk_item[c + 1] (the last one only if it starts before
// the chunk's end).  Each local item gets its first pair, the global id of its
// box's first tile, its box width in tiles (low 16 bits) with its view's tiles
// per row (high 16 bits), its depth key and its item id; p0[nloc] is the end of
// the last one.
// ---------------------------------------------------------------------------
struct ChunkItems {
    uint32_t p0[kChunkPairs + 2];
    uint32_t tile0[kChunkPairs + 1];
    uint32_t wx[kChunkPairs + 1];
    uint32_t item[kChunkPairs + 1];
    uint32_t zkey[kChunkPairs + 1];
};

// Box word of a visible item: (first tile, box width | tiles per row << 16,
// depth key, item), from the pixel box in its record's third word (r2).
__device__ __forceinline__ uint4 item_box_word(const ViewTable &vt, uint64_t n, uint32_t item, const float4 &r2,
                                               uint32_t z) {
    const uint32_t bx = __float_as_uint(r2.y), by = __float_as_uint(r2.z);
    const uint32_t tx0 = (bx & 0xffffu) / kTileW, tx1 = (bx >> 16) / kTileW;
    const uint32_t ty0 = (by & 0xffffu) / (uint32_t)vt.tile_h;
    const int v = (int)(item / n);
    const uint32_t tiles_x = (uint32_t)vt.v[v].tiles_x;
    return make_uint4(vt.v[v].tile_off + ty0 * tiles_x + tx0, (tx1 - tx0 + 1) | (tiles_x << 16), z, item);
}

// The chunk's item range, from the box words by visible index (one coalesced
// 16-byte load per item); every thread of the workgroup calls it (it ends
// with a barrier).
__device__ __forceinline__ uint32_t load_chunk_items(const uint32_t *__restrict__ poff,
                                                     const uint32_t *__restrict__ chunk_item,
                                                     const uint4 *__restrict__ boxes, uint32_t c, uint32_t m,
                                                     uint32_t nvis, ChunkItems &ci, uint32_t &i_lo) {
    const uint32_t c0 = c * kChunkPairs;
    i_lo = chunk_item[c];
    const uint32_t i_hi = c0 + kChunkPairs < m ? chunk_item[c + 1] : nvis - 1;
    const uint32_t nloc = i_hi - i_lo + 1;
    for (uint32_t k = threadIdx.x; k <= nloc; k += kChunkThreads) {
        const uint32_t i = i_lo + k;
        if (k == nloc) {
            ci.p0[k] = i < nvis ? poff[i] : m;
            continue;
        }
        ci.p0[k] = poff[i];
        const uint4 bw = boxes[i];
        ci.tile0[k] = bw.x;
        ci.wx[k] = bw.y;
        ci.zkey[k] = bw.z;
        ci.item[k] = bw.w;
    }
    __syncthreads();
    return nloc;
}

// largest local index k < nloc with p0[k] <= p (p0[0] <= p holds)
__device__ __forceinline__ uint32_t find_chunk_item(const ChunkItems &ci, uint32_t nloc, uint32_t p) {
    uint32_t lo = 0, hi = nloc - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (ci.p0[mid] <= p)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Global tiles of consecutive pairs p, p + 1, ...: the walker keeps the
// (row, column) of the current pair in its item's box, so only the first pair
// needs a division.
struct PairWalker {
    uint32_t k, row, col;
    __device__ __forceinline__ void start(const ChunkItems &ci, uint32_t nloc, uint32_t p) {
        k = find_chunk_item(ci, nloc, p);
        const uint32_t q = p - ci.p0[k], w = ci.wx[k] & 0xffffu;
        row = q / w;
        col = q - row * w;
    }
    // move to pair p (the pair after the previous one)
    __device__ __forceinline__ void next(const ChunkItems &ci, uint32_t nloc, uint32_t p) {
        if (k + 1 < nloc && ci.p0[k + 1] <= p) {
            ++k;
            while (k + 1 < nloc && ci.p0[k + 1] <= p) ++k;  // (items own at least one pair: not taken)
            row = col = 0;
        } else if (++col == (ci.wx[k] & 0xffffu)) {
            col = 0;
            ++row;
        }
    }
    __device__ __forceinline__ uint32_t tile(const ChunkItems &ci) const {
        return ci.tile0[k] + row * (ci.wx[k] >> 16) + col;
    }
};

}  // namespace gsr
