// gsr_composite.hip -- per-tile compositing on gfx950 (A6 forward, A7 backward).
//
// Mapping.  One wave64 per tile of 16 x (4 RPL) pixels: lane l owns column
// l % 16 and rows l / 16 + 4 k, k < RPL, of the tile.  A tile's sorted list is
// consumed in batches of 64 records: each lane stages one record in LDS
// (pre-scaled conic, tile-relative centre) and the whole wave then reads them
// back as broadcasts.  With a single wave per tile there is no cross-wave
// synchronisation in the inner loop, and a row "slab" (the 16 x 4 pixels of
// one k) is skipped as a whole when the Gaussian's alpha >= 1/255 box misses
// it.  Both passes take every decision (slab skip, alpha < 1/255, the stop)
// with the same instructions on the same values, so the backward replays
// exactly the forward's contributors.  The per-pixel updates
// are branch-free (selects), so the only branches are wave-uniform.
//
// Early stop.  Dense scenes saturate long before the end of a tile's list:
// the forward records per tile the number of list positions any of its
// pixels used (nmax).  The backward replays only [start, start + nmax) and
// flags the pair slots of those positions as it stages their records; the
// per-Gaussian reduction reads the moments of flagged slots only, so unused
// pairs cost neither a replay nor a write nor a read.
//
// Backward.  Front to back again (nothing per (pixel, Gaussian) is stored):
// from the forward's output C_out and the running accumulation, the colour
// behind contributor k is B_k = C_out - sum_{j<=k} c_j a_j T_j; only its
// projection on the upstream gradient g is needed, kept as one running value
// g.B = g.C_out - sum, from which alpha dL/dalpha = w g.c - g.B alpha / (1 - alpha)
// (w = alpha T); with g.B taken after the Gaussian's own term and
// T' = T (1 - alpha) that is w (g.c - g.B / T'), one reciprocal per row and
// one fused multiply-add for the update of g.B.  A Gaussian that no lane
// reaches in any row skips the
// reduction: its moments are zero and the finalising lanes write zeros.
// Per pair the kernel produces nine moments over the tile's pixels: with
// w = dL/dsigma, the sums of w dx, w dy, w dx^2, w dx dy, w dy^2, of
// alpha dL/dalpha and of the colour gradient; they are linear in the per-pixel
// terms, so the conversion to (u, v, conic, opacity) gradients happens once
// per Gaussian after the reduction over its tiles.  Each lane sums its pixels'
// terms in registers; the lanes of each quad are added with two DPP swaps,
// and the 16 quad sums are transposed through LDS in groups of seven
// Gaussians (63 values per row), after which lane r < 63 adds the 16 values
// of one (Gaussian, moment) in a fixed order (no atomics, deterministic) and
// the pair's slot in emission order is written once.  (Quads rather than lane
// pairs halve the transpose buffer, which had held the kernel to 3.5 waves
// per SIMD.)
//
// Schedule.  The forward files every tile in a bucket of its replay count
// (nmax), and the backward's workgroups take the tiles heaviest first: in
// tile order the dense centre tiles, dispatched late, left a tail.  Which
// workgroup takes which tile changes no result.
//
// Fused step.  For the mean absolute error the upstream gradient of a pixel
// is a function of that pixel's colour alone, so k_composite_step runs a
// tile's forward and, in the same workgroup, its backward: the two tile
// passes are the functions the separate kernels call, so the results are
// theirs bit for bit, but a SIMD then holds waves in both phases (the
// backward's arithmetic fills the forward's latency) and the forward's
// per-pixel state never leaves registers.  Its schedule cannot use this
// step's replay counts, which exist only after the forward; it takes the
// tile's list length, capped by the replay count the workspace holds from the
// previous step.
#include "gsr_internal.h"

namespace gsr {

struct TileCtx {
    int v;
    uint32_t ox, oy;          // tile origin in pixels
    uint32_t width, height;   // view size
    uint32_t pix_off;         // first pixel of the view
    uint32_t tx, ty;          // tile coordinates
};

__device__ __forceinline__ TileCtx tile_ctx(const ViewTable &vt, uint32_t t) {
    int v = 0;
    while (v + 1 < vt.n_views && t >= vt.v[v + 1].tile_off) ++v;
    TileCtx c;
    c.v = v;
    const uint32_t lt = t - vt.v[v].tile_off;
    const uint32_t tx_n = (uint32_t)vt.v[v].tiles_x;
    c.tx = lt % tx_n;
    c.ty = lt / tx_n;
    c.ox = c.tx * kTileW;
    c.oy = c.ty * (uint32_t)vt.tile_h;
    c.width = (uint32_t)vt.v[v].width;
    c.height = (uint32_t)vt.v[v].height;
    c.pix_off = vt.v[v].pix_off;
    return c;
}

// Rows [y0, y1] of the tile (tile-relative pixel rows) narrowed to those that
// the Gaussian's alpha >= 1/255 ellipse reaches within the tile's columns.
// With (dx, dy) = pixel - centre and sigma = A dx^2 / 2 + B dx dy + C dy^2 / 2,
// the ellipse sigma <= s over the column band dx in [lo, hi] spans
// dy in [min h, max g] with g, h = (-B dx +- sqrt(2 C s - det dx^2)) / C,
// det = A C - B^2: g is concave with its peak at dx = -B sqrt(2 s / (A det)),
// h convex with its trough at the opposite dx, so each extreme is at that
// point clamped to the band.  FP32 with slack: s = 1.001 (ln(255 o) + 0.01)
// + 0.01 (the 1.001 grows the extents by far more than the evaluation's
// rounding, about 1e-6 relative, at any scale) and 0.01 px more on each
// side; a row left out then has alpha below 0.99 / 255 at every pixel, which
// the compositing's own FP32 evaluation cannot round up to 1/255, so leaving
// it out changes nothing but the work.  Degenerate conics keep the box's rows.
__device__ __forceinline__ void ellipse_rows_in_band(float A, float B, float C, float opacity, float ut, float vt,
                                                     int &y0, int &y1) {
    if (y0 > y1) return;
    const float det = A * C - B * B;
    const float s = 1.001f * (__logf(255.f * opacity) + 0.01f) + 0.01f;
    if (!(det > 0.f) || !(A > 0.f) || !(C > 0.f) || !(s > 0.f)) return;
    const float idet = __builtin_amdgcn_rcpf(det), iC = __builtin_amdgcn_rcpf(C);
    const float X = __builtin_sqrtf(2.f * C * s * idet);  // half-width of the ellipse
    const float lo = fmaxf(0.5f - ut - 0.01f, -X), hi = fminf((float)kTileW - 0.5f - ut + 0.01f, X);
    if (lo > hi) {  // the ellipse misses the tile's columns
        y1 = y0 - 1;
        return;
    }
    const float xs = -B * __builtin_sqrtf(2.f * s * idet * __builtin_amdgcn_rcpf(A));
    const float xt = fminf(fmaxf(xs, lo), hi), xb = fminf(fmaxf(-xs, lo), hi);
    const float top = (-B * xt + __builtin_sqrtf(fmaxf(0.f, 2.f * C * s - det * xt * xt))) * iC;
    const float bot = (-B * xb - __builtin_sqrtf(fmaxf(0.f, 2.f * C * s - det * xb * xb))) * iC;
    // pixel row r (centre r + 0.5) lies in [vt + bot, vt + top]
    const float r0 = ceilf(vt + bot - 0.51f), r1 = floorf(vt + top - 0.49f);
    y0 = max(y0, (int)fmaxf(r0, -1.f));
    y1 = min(y1, (int)fminf(r1, 65536.f));
}

// Staged record (LDS): three float4 per Gaussian.
//   a = (u - ox, v - oy, -A log2e / 2, -B log2e)
//   b = (-C log2e / 2, log2(opacity), red, green)
//   d = (blue, bits(slab mask), bits(pair index), opacity)
// so that sigma * log2e = -(a.z dx^2 + a.w dx dy + b.x dy^2) and
// alpha = min(0.99, exp2(-sigma log2e + b.y)).  Bit k of the slab mask is set
// when the Gaussian's alpha >= 1/255 ellipse (with slack) reaches rows
// [4k, 4k + 3] of the tile within its columns.
__device__ __forceinline__ void stage_record(const Rec &r, const float2 lo, const TileCtx &c, uint32_t tile_h,
                                             float4 &a, float4 &b, float4 &d) {
    const float ut = (r.r0.x - (float)c.ox) + lo.x;
    const float vt = (r.r0.y - (float)c.oy) + lo.y;
    a = make_float4(ut, vt, -0.5f * kLog2e * r.r0.z, -kLog2e * r.r0.w);
    b = make_float4(-0.5f * kLog2e * r.r1.x, __log2f(r.r1.y), r.r1.z, r.r1.w);
    const uint32_t by = __float_as_uint(r.r2.z);
    int y0 = max((int)(by & 0xffffu) - (int)c.oy, 0), y1 = min((int)(by >> 16) - (int)c.oy, (int)tile_h - 1);
    ellipse_rows_in_band(r.r0.z, r.r0.w, r.r1.x, r.r1.y, ut, vt, y0, y1);
    const uint32_t smask = y0 <= y1 ? ((2u << (y1 >> 2)) - 1u) & ~((1u << (y0 >> 2)) - 1u) : 0u;
    // pair index in emission order: offset + row-major position in the tile box
    const uint32_t bx = __float_as_uint(r.r2.y);
    const uint32_t tx0 = (bx & 0xffffu) / kTileW, tx1 = (bx >> 16) / kTileW;
    const uint32_t ty0 = (by & 0xffffu) / tile_h;
    const uint32_t p = __float_as_uint(r.r2.w) + (c.ty - ty0) * (tx1 - tx0 + 1) + (c.tx - tx0);
    d = make_float4(r.r2.x, __uint_as_float(smask), __uint_as_float(p), r.r1.y);
}

// The slab mask of a staged record, as a scalar (the record is an LDS broadcast).
__device__ __forceinline__ uint32_t slab_mask(float packed) {
    return __builtin_amdgcn_readfirstlane(__float_as_uint(packed));
}

// A slab whose every pixel has exponent below this (log2 of alpha before the
// clamp) cannot reach alpha >= 1/255: skipping it changes no decision (the
// margin dwarfs the exponential's rounding).
constexpr float kLog2AlphaSkip = -7.9943534f - 0.01f;  // log2(1/255) - 0.01

// The r-th tile of the backward's schedule: tiles in descending cost buckets
// (any order within a bucket: tiles are independent, so results do not
// depend on it), or tile r when the buckets do not hold every tile (a forward
// that skipped compositing).  One whole wave calls it.  Not inlined: its
// loop-invariant loads would otherwise be hoisted and held in registers
// through the tile's loops (13 more VGPRs, one wave fewer per SIMD).
__device__ __noinline__ uint32_t tile_by_cost(const uint32_t *__restrict__ order, uint32_t total_tiles,
                                                 uint32_t r) {
    const int lane = threadIdx.x & 63;
    static_assert(kCostBuckets == 2 * kWave, "two buckets per lane");
    // lane l: buckets 127 - 2l and 126 - 2l (descending cost)
    const uint32_t b0 = kCostBuckets - 1 - 2 * lane, c0 = order[b0], c1 = order[b0 - 1];
    const uint32_t incl = wave_inclusive_scan(c0 + c1, [](uint32_t a, uint32_t b) { return a + b; });
    if ((uint32_t)__shfl((int)incl, 63, 64) != total_tiles) return r;
    const unsigned long long past = __ballot(r < incl);  // lanes whose buckets end beyond r
    const int L = __ffsll((long long)past) - 1;
    const uint32_t before = (uint32_t)__shfl((int)(incl - c0 - c1), L, 64);
    const uint32_t cL0 = (uint32_t)__shfl((int)c0, L, 64);
    const uint32_t k = r - before;
    const uint32_t b = k < cL0 ? kCostBuckets - 1 - 2 * (uint32_t)L : kCostBuckets - 2 - 2 * (uint32_t)L;
    return order[kCostBuckets + (size_t)b * total_tiles + (k < cL0 ? k : k - cL0)];
}

__device__ __forceinline__ uint32_t next_tile(bool persistent, uint32_t *queue, uint32_t first, uint32_t &iter) {
    if (!persistent) return iter++ == 0 ? first : 0xffffffffu;
    uint32_t t = 0;
    if (threadIdx.x == 0) t = atomicAdd(queue, 1u);
    return __shfl(t, 0, kWave);
}

// Exponent of alpha before the clamp, ex = log2(opacity) - sigma log2e
// = b.y + a.z dx^2 + a.w dx dy + b.x dy^2, for the pixel at (dx, dy) from the
// centre.  A lane's pixels share dx, so the dx terms and b.y are formed once
// per Gaussian (RowQuad) and each row evaluates (b.x dy + a.w dx) dy +
// (a.z dx^2 + b.y) by two fused multiply-adds.  sigma is a positive definite
// quadratic form (the conic inverts a covariance with the 0.3 I low-pass
// added), so there is no sign test: an FP32 exponent above b.y is rounding
// near the centre, where the exact sigma is >= 0 and the Gaussian counts.
struct RowQuad {
    float p, q;  // a.z dx^2 + b.y, a.w dx
};
__device__ __forceinline__ RowQuad row_quad(const float4 &a, const float4 &b, float dx) {
    return RowQuad{fmaf(a.z * dx, dx, b.y), a.w * dx};
}
__device__ __forceinline__ float alpha_exponent(const RowQuad &rq, const float4 &b, float dy) {
    return fmaf(fmaf(b.x, dy, rq.q), dy, rq.p);
}

// ---------------------------------------------------------------------------
// A6: forward
// ---------------------------------------------------------------------------
// One tile's forward pass over its sorted list, from the per-pixel state
// (T > 0: the pixel is still compositing; T < 0: it stopped, or lies outside
// the image, and -T is its final transmittance) to the accumulated colours
// and, per pixel, the list position after its last contributor (last).  With
// STATS also the contributor count and the position of the stop.
template <int RPL, bool STATS>
__device__ __forceinline__ void tile_forward(const ViewTable &vt, const TileCtx &c, uint2 rg,
                                             const uint32_t *__restrict__ pval, const Rec *__restrict__ rec,
                                             const float2 *__restrict__ ulo, float4 *sa, float4 *sb, float4 *sd,
                                             int lane, int ly, float pxl, float (&T)[RPL], float (&C0)[RPL],
                                             float (&C1)[RPL], float (&C2)[RPL], uint32_t (&last)[RPL],
                                             uint32_t (&ncontrib)[RPL], uint32_t (&stop_at)[RPL]) {
    for (uint32_t b0 = rg.x; b0 < rg.y; b0 += kWave) {
        bool any_live = false;
#pragma unroll
        for (int k = 0; k < RPL; ++k) any_live |= T[k] > 0.f;
        if (__ballot(any_live) == 0ull) break;
        const uint32_t idx = b0 + lane;
        if (idx < rg.y) {
            const uint32_t item = pval[idx];
            float4 a, b, d;
            stage_record(rec[item], ulo[item], c, (uint32_t)vt.tile_h, a, b, d);
            sa[lane] = a;
            sb[lane] = b;
            sd[lane] = d;
        }
        __syncthreads();
        const int cnt = (int)min((uint32_t)kWave, rg.y - b0);
        for (int j = 0; j < cnt; ++j) {
            if ((j & 15) == 15) {  // leave the batch once every pixel of the tile has stopped
                bool any = false;
#pragma unroll
                for (int k = 0; k < RPL; ++k) any |= T[k] > 0.f;
                if (__ballot(any) == 0ull) break;
            }
            const float4 a = sa[j], b = sb[j], d = sd[j];
            const uint32_t pos = b0 - rg.x + (uint32_t)j;
            const float dx = a.x - pxl;
            const uint32_t smask = slab_mask(d.y);
            const RowQuad rq = row_quad(a, b, dx);
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                if (!(smask & (1u << k))) continue;
                const float dy = a.y - ((float)(ly + 4 * k) + 0.5f);
                const float ex = alpha_exponent(rq, b, dy);
                if (__ballot(T[k] > 0.f && ex >= kLog2AlphaSkip) == 0ull) continue;
                const float alpha = fminf(kAlphaMax, __builtin_amdgcn_exp2f(ex));
                const bool ok = alpha >= kAlphaMin;
                const float wa = alpha * T[k];
                const float Tn = T[k] - wa;  // T (1 - alpha)
                // a stopped pixel has Tn <= 0 < kTMin, so it never adds again; the
                // pixel stops where ok holds and add does not
                const bool add = ok & (Tn >= kTMin);
                const float w = add ? wa : 0.f;
                C0[k] = fmaf(b.z, w, C0[k]);
                C1[k] = fmaf(b.w, w, C1[k]);
                C2[k] = fmaf(d.x, w, C2[k]);
                last[k] = add ? pos + 1 : last[k];
                if constexpr (STATS) {
                    ncontrib[k] += add ? 1u : 0u;
                    stop_at[k] = (ok && !add && T[k] > 0.f) ? pos : stop_at[k];
                }
                // (two selects: written as one nested select, the compiler branched on it)
                const float Ts = ok ? -fabsf(T[k]) : T[k];
                T[k] = add ? Tn : Ts;
            }
        }
        __syncthreads();
    }
}

template <int RPL, bool STATS>
__global__ __launch_bounds__(kWave) void k_composite_fwd(ViewTable vt, const uint2 *__restrict__ ranges,
                                                         const uint32_t *__restrict__ pval,
                                                         const Rec *__restrict__ rec, const float2 *__restrict__ ulo,
                                                         float3 bg,
                                                         float *__restrict__ out_rgb, float *__restrict__ out_T,
                                                         float *__restrict__ pix_T, uint32_t *__restrict__ pix_n,
                                                         uint32_t *__restrict__ tile_cut, uint32_t *__restrict__ tile_order,
                                                         WsHeader *hdr, int persistent) {
    __shared__ float4 sa[kWave], sb[kWave], sd[kWave];
    const int lane = threadIdx.x;
    const int lx = lane & 15, ly = lane >> 4;
    const float pxl = (float)lx + 0.5f;
    uint32_t iter = 0;
    for (;;) {
        const uint32_t t = next_tile(persistent != 0, &hdr->queue[0], blockIdx.x, iter);
        if (t >= vt.total_tiles) break;
        const TileCtx c = tile_ctx(vt, t);
        const uint32_t px = c.ox + lx;
        float T[RPL], C0[RPL], C1[RPL], C2[RPL];
        uint32_t last[RPL], stop_at[RPL], ncontrib[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const uint32_t py = c.oy + ly + 4 * k;
            T[k] = (px < c.width && py < c.height) ? 1.f : -1.f;
            C0[k] = C1[k] = C2[k] = 0.f;
            last[k] = 0;
            ncontrib[k] = 0;
            stop_at[k] = 0xffffffffu;
        }
        const uint2 rg = ranges[t];
        tile_forward<RPL, STATS>(vt, c, rg, pval, rec, ulo, sa, sb, sd, lane, ly, pxl, T, C0, C1, C2, last, ncontrib,
                                 stop_at);
        // outputs
        const uint32_t len = rg.y - rg.x;
        uint32_t evals = 0, replays = 0, contrib = 0, nmax = 0;
        const size_t plane = (size_t)c.width * c.height;
        float *img = out_rgb + 3 * (size_t)c.pix_off;
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const uint32_t py = c.oy + ly + 4 * k;
            if (px < c.width && py < c.height) {
                const size_t pix = (size_t)py * c.width + px;
                const float Tf = fabsf(T[k]);
                img[pix] = C0[k] + Tf * bg.x;
                img[plane + pix] = C1[k] + Tf * bg.y;
                img[2 * plane + pix] = C2[k] + Tf * bg.z;
                pix_T[c.pix_off + pix] = Tf;
                pix_n[c.pix_off + pix] = last[k];
                if (out_T) out_T[c.pix_off + pix] = Tf;
                evals += stop_at[k] != 0xffffffffu ? stop_at[k] + 1 : len;
                replays += last[k];
                contrib += ncontrib[k];
                nmax = max(nmax, last[k]);
            }
        }
        nmax = wave_reduce(nmax, 0u, [](uint32_t a, uint32_t b) { return max(a, b); });
        if constexpr (STATS) {
            // work counters for the measurement harness (integer adds: order independent)
            unsigned long long e = evals, rp = replays, cc = contrib;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                e += __shfl_xor(e, o, kWave);
                rp += __shfl_xor(rp, o, kWave);
                cc += __shfl_xor(cc, o, kWave);
            }
            if (lane == 0) {
                atomicAdd(&hdr->evaluations, e);
                atomicAdd(&hdr->replays, rp);
                atomicAdd(&hdr->contributors, cc);
            }
        }
        if (lane == 0) {
            tile_cut[t] = nmax;  // positions the backward replays
            // the backward's schedule: this tile in the bucket of its replay count
            const uint32_t b = cost_bucket(nmax);
            const uint32_t slot = atomicAdd(&tile_order[b], 1u);
            tile_order[kCostBuckets + (size_t)b * vt.total_tiles + slot] = t;
        }
    }
}

// ---------------------------------------------------------------------------
// A7: backward
// ---------------------------------------------------------------------------
constexpr int kGroup = 7;                          // Gaussians per LDS transpose
constexpr int kRedCols = kGroup * kPartialStride;  // 63 values per row
constexpr int kRedRows = kWave / 4;                // lane quads are summed first
constexpr int kRedStride = kRedCols + 2;           // odd row stride: conflict-free rows and columns

// Zero gradient rows of the Gaussians of tile t's slice that no view saw, one
// row per lane (fire-and-forget stores that overlap the tile's ALU work).
__device__ __forceinline__ void zero_unseen_rows(const ZeroRows &z, uint32_t t, bool overflow, int lane) {
    const uint64_t g0 = (uint64_t)t * z.per_tile, g1 = min(z.n, g0 + z.per_tile);
    const int K3 = 3 * z.sh_k;
    for (uint64_t i = g0 + (uint64_t)lane; i < g1; i += kWave) {
        bool seen = false;
        if (!overflow)
            for (int v = 0; v < z.n_views; ++v) seen |= z.count[(uint64_t)v * z.n + i] > 0u;
        if (seen) continue;
        for (int a = 0; a < 3; ++a) z.g.means[3 * i + a] = 0.f, z.g.log_scales[3 * i + a] = 0.f;
        reinterpret_cast<float4 *>(z.g.quats)[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        z.g.opacities[i] = 0.f;
        if ((K3 & 3) == 0) {
            float4 *row = reinterpret_cast<float4 *>(z.g.sh + (uint64_t)K3 * i);
            for (int k = 0; k < K3 / 4; ++k) row[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
            float *row = z.g.sh + (uint64_t)K3 * i;
            for (int k = 0; k < K3; ++k) row[k] = 0.f;
        }
    }
}

__device__ __forceinline__ float l1_grad(float c, float target, float scale) {
    return c > target ? scale : (c < target ? -scale : 0.f);
}

// One tile's backward pass over list positions [rg.x, end): the per-pixel
// state starts at T = 1, the upstream gradient g = dL/dC (g0, g1, g2), gB =
// g . C_out and the contributor count ncon; the pass writes the nine moments
// of every replayed pair to `partial` (at its slot in emission order) and
// flags the slot.
template <int RPL>
__device__ __forceinline__ void tile_backward(const ViewTable &vt, const TileCtx &c, uint2 rg, uint32_t end,
                                              const uint32_t *__restrict__ pval, const Rec *__restrict__ rec,
                                              const float2 *__restrict__ ulo, float4 *sa, float4 *sb, float4 *sd,
                                              float *red, int lane, int ly, float pxl, int fq, int fc,
                                              float (&T)[RPL], const float (&g0)[RPL], const float (&g1)[RPL],
                                              const float (&g2)[RPL], float (&gB)[RPL], const uint32_t (&ncon)[RPL],
                                              float *__restrict__ partial, uint8_t *__restrict__ pflag) {
    // per-lane sums over one Gaussian's rows: colour-gradient weights w,
    // sa = alpha dL/dalpha, sa dy and sa dy^2 (the rows share dx); zero
    // between Gaussians (a Gaussian no lane reaches leaves them so, and the
    // reduction of one that some lane reaches resets them)
    float a_c0 = 0.f, a_c1 = 0.f, a_c2 = 0.f, a_sa = 0.f, a_say = 0.f, a_sayy = 0.f;
    for (uint32_t b0 = rg.x; b0 < end; b0 += kWave) {
        const uint32_t idx = b0 + lane;
        if (idx < end) {
            const uint32_t item = pval[idx];
            float4 a, b, d;
            stage_record(rec[item], ulo[item], c, (uint32_t)vt.tile_h, a, b, d);
            sa[lane] = a;
            sb[lane] = b;
            sd[lane] = d;
            pflag[__float_as_uint(d.z)] = 1;  // this pair's moments get written: the reduction reads them
        }
        __syncthreads();
        const int cnt = (int)min((uint32_t)kWave, end - b0);
        for (int j0 = 0; j0 < cnt; j0 += kGroup) {
            uint32_t zq = 0;  // Gaussians of the group with all moments zero
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                const int j = j0 + q;
                float dx = 0.f;
                bool live = false;  // wave-uniform: some lane reached some row of this Gaussian
                if (j < cnt) {
                    const uint32_t pos = b0 - rg.x + (uint32_t)j;
                    const float4 a = sa[j], b = sb[j], d = sd[j];
                    dx = a.x - pxl;
                    const uint32_t smask = slab_mask(d.y);
                    const RowQuad rq = row_quad(a, b, dx);
#pragma unroll
                    for (int k = 0; k < RPL; ++k) {
                        if (!(smask & (1u << k))) continue;
                        const float dy = a.y - ((float)(ly + 4 * k) + 0.5f);
                        const float ex = alpha_exponent(rq, b, dy);
                        if (__ballot(pos < ncon[k] && ex >= kLog2AlphaSkip) == 0ull) continue;
                        live = true;
                        const float araw = __builtin_amdgcn_exp2f(ex);
                        const float alpha = fminf(kAlphaMax, araw);
                        const bool ok = pos < ncon[k] && alpha >= kAlphaMin;
                        const float w = ok ? alpha * T[k] : 0.f;
                        a_c0 = fmaf(w, g0[k], a_c0);
                        a_c1 = fmaf(w, g1[k], a_c1);
                        a_c2 = fmaf(w, g2[k], a_c2);
                        const float grgb = fmaf(g0[k], b.z, fmaf(g1[k], b.w, g2[k] * d.x));
                        // alpha dL/dalpha = alpha T g.c - alpha g.B / (1 - alpha), with
                        // B the colour behind this Gaussian; with w = alpha T and
                        // T' = T (1 - alpha) that is w (g.c - g.B / T') (w = 0 where
                        // the Gaussian does not contribute)
                        gB[k] = fmaf(-w, grgb, gB[k]);
                        T[k] -= w;  // T (1 - alpha) where the Gaussian contributed
                        const float h = fmaf(-gB[k], __builtin_amdgcn_rcpf(T[k]), grgb);
                        // dL/dsigma = -sa, alpha dL/dalpha = sa (zero through the 0.99 clamp)
                        const float sa_ = (araw < kAlphaMax ? w : 0.f) * h;
                        a_sa += sa_;
                        const float say = sa_ * dy;
                        a_say += say;
                        a_sayy = fmaf(say, dy, a_sayy);
                    }
                }
                if (!live) zq |= 1u << q;  // every moment is zero: the finaliser writes 0
                if (live) {
                    // (no contraction: a product contracted into the first DPP add
                    // costs a separate lane move, and its four quad lanes would no
                    // longer add a and b as b and a)
#pragma clang fp contract(off)
                    // the moments of sa (= -dL/dsigma): sums of sa dx, sa dy, sa dx^2,
                    // sa dx dy, sa dy^2 (the negated S_x .. S_yy of the projection
                    // backward), then S_o = sum sa and the colour gradient
                    float s[kPartialStride];
                    s[0] = dx * a_sa;
                    s[1] = a_say;
                    s[2] = dx * s[0];
                    s[3] = dx * a_say;
                    s[4] = a_sayy;
                    s[5] = a_sa;
                    s[6] = a_c0;
                    s[7] = a_c1;
                    s[8] = a_c2;
                    // add the lanes of each quad (quad_perm [1, 0, 3, 2], then [2, 3, 0, 1]):
                    // all four lanes hold the same sum (each step adds a and b as b and a,
                    // exactly equal) and store it to the same place, so no lane is masked
                    // off and each move folds into its add
#pragma unroll
                    for (int cc = 0; cc < kPartialStride; ++cc)
                        s[cc] = dpp_add<0x4E, 0xf>(dpp_add<0xB1, 0xf>(s[cc]));
#pragma unroll
                    for (int cc = 0; cc < kPartialStride; ++cc)
                        red[(lane >> 2) * kRedStride + q * kPartialStride + cc] = s[cc];
                    a_c0 = a_c1 = a_c2 = a_sa = a_say = a_sayy = 0.f;
                }
            }
            __syncthreads();
            if (lane < kRedCols && j0 + fq < cnt) {
                float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
                if (!((zq >> fq) & 1u)) {
#pragma unroll
                    for (int r = 0; r < kRedRows; r += 4) {
                        p0 += red[(r + 0) * kRedStride + lane];
                        p1 += red[(r + 1) * kRedStride + lane];
                        p2 += red[(r + 2) * kRedStride + lane];
                        p3 += red[(r + 3) * kRedStride + lane];
                    }
                }
                const uint32_t p = __float_as_uint(sd[j0 + fq].z);
                partial[(size_t)p * kPartialStride + fc] = (p0 + p1) + (p2 + p3);
            }
            __syncthreads();
        }
    }
}

template <int RPL>
__global__ __launch_bounds__(kWave) void k_composite_bwd(ViewTable vt, const uint2 *__restrict__ ranges,
                                                         const uint32_t *__restrict__ pval,
                                                         const Rec *__restrict__ rec, const float2 *__restrict__ ulo,
                                                         const float *__restrict__ out_rgb, Upstream up,
                                                         const uint32_t *__restrict__ pix_n,
                                                         const uint32_t *__restrict__ tile_cut,
                                                         const uint32_t *__restrict__ tile_order,
                                                         float *__restrict__ partial, uint8_t *__restrict__ pflag,
                                                         ZeroRows zr, WsHeader *hdr, int persistent) {
    __shared__ float4 sa[kWave], sb[kWave], sd[kWave];
    __shared__ float red[kRedRows * kRedStride];
    const int lane = threadIdx.x;
    const int lx = lane & 15, ly = lane >> 4;
    const float pxl = (float)lx + 0.5f;
    // the (Gaussian of the group, moment) this lane finalises
    const int fq = lane / kPartialStride, fc = lane - fq * kPartialStride;
    uint32_t iter = 0;
    for (;;) {
        const uint32_t r = next_tile(persistent != 0, &hdr->queue[1], blockIdx.x, iter);
        if (r >= vt.total_tiles) break;
        const uint32_t t = tile_by_cost(tile_order, vt.total_tiles, r);  // heaviest tiles first
        zero_unseen_rows(zr, t, hdr->overflow != 0u, lane);
        const TileCtx c = tile_ctx(vt, t);
        const uint32_t px = c.ox + lx;
        const size_t plane = (size_t)c.width * c.height;
        const float *img = out_rgb + 3 * (size_t)c.pix_off;
        const float *gimg = (up.target ? up.target : up.grad) + 3 * (size_t)c.pix_off;
        // gB = g . (colour still to come behind the current position): g . C_out
        // before the first contributor, reduced by each contribution
        float T[RPL], g0[RPL], g1[RPL], g2[RPL], gB[RPL];
        uint32_t ncon[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const uint32_t py = c.oy + ly + 4 * k;
            T[k] = 1.f;
            if (px < c.width && py < c.height) {
                const size_t pix = (size_t)py * c.width + px;
                ncon[k] = pix_n[c.pix_off + pix];
                const float i0 = img[pix], i1 = img[plane + pix], i2 = img[2 * plane + pix];
                g0[k] = gimg[pix];
                g1[k] = gimg[plane + pix];
                g2[k] = gimg[2 * plane + pix];
                if (up.target) {  // mean absolute error: dL/dC = sign(C - target) / count
                    g0[k] = l1_grad(i0, g0[k], up.l1_scale);
                    g1[k] = l1_grad(i1, g1[k], up.l1_scale);
                    g2[k] = l1_grad(i2, g2[k], up.l1_scale);
                }
                gB[k] = fmaf(g2[k], i2, fmaf(g1[k], i1, g0[k] * i0));
            } else {
                ncon[k] = 0;
                g0[k] = g1[k] = g2[k] = gB[k] = 0.f;
            }
        }
        const uint2 rg = ranges[t];
        const uint32_t end = rg.x + tile_cut[t];  // positions any pixel of the tile used
        tile_backward<RPL>(vt, c, rg, end, pval, rec, ulo, sa, sb, sd, red, lane, ly, pxl, fq, fc, T, g0, g1, g2, gB,
                           ncon, partial, pflag);
    }
}

// ---------------------------------------------------------------------------
// A6 + A7 for the photometric loss in one pass over the tiles: a workgroup
// composites its tile forward, forms dL/dC = sign(C - target) * l1_scale of
// the tile's pixels from the colours it has just accumulated (the gradient of
// a pixel depends on its own colour only), and replays the tile backward,
// with the same two tile passes as the kernels above, so that the image, the
// workspace state and the moments are theirs bit for bit.  What changes is the
// schedule: a SIMD holds waves in both phases, so the backward's arithmetic
// fills the forward's latency, and the forward's per-pixel state stays in
// registers.  A fused tile lasts both passes, so a heavy tile dispatched late
// leaves a long tail: the tiles are taken in descending buckets of min(list
// length, the replay count the workspace holds from its previous step),
// filed by a workgroup of the per-tile depth sort (exact for a repeated step,
// the list length on a fresh workspace; any order gives the same results).
// ---------------------------------------------------------------------------
template <int RPL>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(5))) void k_composite_step(
    ViewTable vt, const uint2 *__restrict__ ranges, const uint32_t *__restrict__ pval, const Rec *__restrict__ rec,
    const float2 *__restrict__ ulo, float3 bg, const float *__restrict__ target, float l1_scale,
    float *__restrict__ out_rgb, float *__restrict__ out_T, float *__restrict__ pix_T, uint32_t *__restrict__ pix_n,
    uint32_t *__restrict__ tile_cut, const uint32_t *__restrict__ tile_order, float *__restrict__ partial,
    uint8_t *__restrict__ pflag, ZeroRows zr, WsHeader *hdr, int persistent) {
    __shared__ float4 sa[kWave], sb[kWave], sd[kWave];
    __shared__ float red[kRedRows * kRedStride];
    const int lane = threadIdx.x;
    const int lx = lane & 15, ly = lane >> 4;
    const float pxl = (float)lx + 0.5f;
    const int fq = lane / kPartialStride, fc = lane - fq * kPartialStride;
    uint32_t iter = 0;
    for (;;) {
        const uint32_t r = next_tile(persistent != 0, &hdr->queue[0], blockIdx.x, iter);
        if (r >= vt.total_tiles) break;
        const uint32_t t = tile_by_cost(tile_order, vt.total_tiles, r);
        zero_unseen_rows(zr, t, hdr->overflow != 0u, lane);
        const TileCtx c = tile_ctx(vt, t);
        const uint32_t px = c.ox + lx;
        const uint2 rg = ranges[t];
        float T[RPL], C0[RPL], C1[RPL], C2[RPL];
        uint32_t last[RPL], unused0[RPL], unused1[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const uint32_t py = c.oy + ly + 4 * k;
            T[k] = (px < c.width && py < c.height) ? 1.f : -1.f;
            C0[k] = C1[k] = C2[k] = 0.f;
            last[k] = 0;
        }
        tile_forward<RPL, false>(vt, c, rg, pval, rec, ulo, sa, sb, sd, lane, ly, pxl, T, C0, C1, C2, last, unused0,
                                 unused1);
        // outputs, and the backward's start: g = dL/dC, gB = g . C_out
        const size_t plane = (size_t)c.width * c.height;
        float *img = out_rgb + 3 * (size_t)c.pix_off;
        const float *tgt = target + 3 * (size_t)c.pix_off;
        float g0[RPL], g1[RPL], g2[RPL], gB[RPL];
        uint32_t ncon[RPL], nmax = 0;
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const uint32_t py = c.oy + ly + 4 * k;
            if (px < c.width && py < c.height) {
                const size_t pix = (size_t)py * c.width + px;
                const float Tf = fabsf(T[k]);
                const float i0 = C0[k] + Tf * bg.x, i1 = C1[k] + Tf * bg.y, i2 = C2[k] + Tf * bg.z;
                img[pix] = i0;
                img[plane + pix] = i1;
                img[2 * plane + pix] = i2;
                pix_T[c.pix_off + pix] = Tf;
                pix_n[c.pix_off + pix] = last[k];
                if (out_T) out_T[c.pix_off + pix] = Tf;
                nmax = max(nmax, last[k]);
                ncon[k] = last[k];
                g0[k] = l1_grad(i0, tgt[pix], l1_scale);
                g1[k] = l1_grad(i1, tgt[plane + pix], l1_scale);
                g2[k] = l1_grad(i2, tgt[2 * plane + pix], l1_scale);
                gB[k] = fmaf(g2[k], i2, fmaf(g1[k], i1, g0[k] * i0));
            } else {
                ncon[k] = 0;
                g0[k] = g1[k] = g2[k] = gB[k] = 0.f;
            }
            T[k] = 1.f;
        }
        nmax = wave_reduce(nmax, 0u, [](uint32_t a, uint32_t b) { return max(a, b); });
        if (lane == 0) tile_cut[t] = nmax;
        tile_backward<RPL>(vt, c, rg, rg.x + nmax, pval, rec, ulo, sa, sb, sd, red, lane, ly, pxl, fq, fc, T, g0, g1,
                           g2, gB, ncon, partial, pflag);
    }
}

// Workgroups of a persistent launch: as many as can be resident at once
// (occupancy of this kernel x compute units of the current device, queried at
// each launch: nothing is cached between calls), unless the caller fixed it.
template <typename Kernel>
static int resident_ctas(Kernel kernel, int requested) {
    if (requested > 0) return requested;
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kWave, 0) != hipSuccess || per <= 0) per = 8;
    return cus * per;
}

void launch_composite_fwd(const ViewTable &vt, const uint2 *ranges, const uint32_t *pval, const Rec *rec,
                          const float2 *ulo, float3 bg, float *out_rgb, float *out_T, float *pix_T,
                          uint32_t *pix_n, uint32_t *tile_cut, uint32_t *tile_order, WsHeader *hdr,
                          bool persistent, int persistent_ctas, bool stats, hipStream_t st) {
    if (vt.total_tiles == 0) return;
    const int p = persistent ? 1 : 0;
#define GSR_FWD(R, S)                                                                                               \
    hipLaunchKernelGGL((k_composite_fwd<R, S>),                                                                     \
                       dim3(persistent ? (unsigned)resident_ctas(k_composite_fwd<R, S>, persistent_ctas)            \
                                       : vt.total_tiles),                                                           \
                       dim3(kWave), 0, st, vt, ranges, pval, rec, ulo, bg, out_rgb, out_T, pix_T, pix_n,            \
                       tile_cut, tile_order, hdr, p)
#define GSR_FWD_RPL(R) \
    if (stats) GSR_FWD(R, true); else GSR_FWD(R, false)
    switch (vt.tile_h) {
        case 4: GSR_FWD_RPL(1); break;
        case 8: GSR_FWD_RPL(2); break;
        case 32: GSR_FWD_RPL(8); break;
        default: GSR_FWD_RPL(4); break;
    }
#undef GSR_FWD_RPL
#undef GSR_FWD
}

void launch_composite_bwd(const ViewTable &vt, const uint2 *ranges, const uint32_t *pval, const Rec *rec,
                          const float2 *ulo, const float *out_rgb, const Upstream &up, const uint32_t *pix_n,
                          const uint32_t *tile_cut, const uint32_t *tile_order, float *partial, uint8_t *pflag,
                          const ZeroRows &zr, WsHeader *hdr, bool persistent, int persistent_ctas, hipStream_t st) {
    if (vt.total_tiles == 0) return;
    const int p = persistent ? 1 : 0;
#define GSR_BWD(R)                                                                                                  \
    hipLaunchKernelGGL(k_composite_bwd<R>,                                                                          \
                       dim3(persistent ? (unsigned)resident_ctas(k_composite_bwd<R>, persistent_ctas)               \
                                       : vt.total_tiles),                                                           \
                       dim3(kWave), 0, st, vt, ranges, pval, rec, ulo, out_rgb, up, pix_n, tile_cut, tile_order,    \
                       partial, pflag, zr, hdr, p)
    switch (vt.tile_h) {
        case 4: GSR_BWD(1); break;
        case 8: GSR_BWD(2); break;
        case 32: GSR_BWD(8); break;
        default: GSR_BWD(4); break;
    }
#undef GSR_BWD
}


void launch_composite_step(const ViewTable &vt, const uint2 *ranges, const uint32_t *pval, const Rec *rec,
                           const float2 *ulo, float3 bg, const float *target, float l1_scale, float *out_rgb,
                           float *out_T, float *pix_T, uint32_t *pix_n, uint32_t *tile_cut,
                           const uint32_t *tile_order, float *partial, uint8_t *pflag, const ZeroRows &zr,
                           WsHeader *hdr, bool persistent, int persistent_ctas, hipStream_t st) {
    if (vt.total_tiles == 0) return;
    const int p = persistent ? 1 : 0;
#define GSR_STEP(R)                                                                                                 \
    hipLaunchKernelGGL(k_composite_step<R>,                                                                         \
                       dim3(persistent ? (unsigned)resident_ctas(k_composite_step<R>, persistent_ctas)              \
                                       : vt.total_tiles),                                                           \
                       dim3(kWave), 0, st, vt, ranges, pval, rec, ulo, bg, target, l1_scale, out_rgb, out_T, pix_T, \
                       pix_n, tile_cut, tile_order, partial, pflag, zr, hdr, p)
    switch (vt.tile_h) {
        case 4: GSR_STEP(1); break;
        case 8: GSR_STEP(2); break;
        case 32: GSR_STEP(8); break;
        default: GSR_STEP(4); break;
    }
#undef GSR_STEP
}

}  // namespace gsr
