// gsr_composite.hip -- per-tile compositing on gfx950 (A6 forward, A7 backward).
//
// Mapping.  One wave64 per tile of 16 x (4 RPL) pixels: lane l owns column
// l % 16 and rows l / 16 + 4 k, k < RPL, of the tile.  A tile's sorted list is
// consumed in batches of 64 records: each lane stages one record in LDS
// (pre-scaled conic, tile-relative centre) and the whole wave then reads them
// back as broadcasts.  With a single wave per tile there is no cross-wave
// synchronisation in the inner loop, and a row "slab" (the 16 x 4 pixels of
// one k) is skipped as a whole when the Gaussian's alpha >= 1/255 box misses
// it.  Both passes take every decision (box slab skip, sigma < 0, alpha <
// 1/255, the stop) with the same instructions on the same values, so the
// backward replays exactly the forward's contributors.
//
// Backward.  Front to back again (nothing per (pixel, Gaussian) is stored):
// from the forward's output C_out and the running accumulation, the colour
// behind contributor k is B_k = C_out - sum_{j<=k} c_j a_j T_j; only its
// projection on the upstream gradient g is needed, g.B_k = g.C_out - sum.
// Each lane sums its pixels' contributions in registers; the wave then reduces
// the nine screen-space gradient components and writes them once to the pair's
// slot in emission order (no atomics, deterministic).
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

// Staged record (LDS): three float4 per Gaussian.
//   a = (u - ox, v - oy, -A log2e / 2, -B log2e)
//   b = (-C log2e / 2, log2(opacity), red, green)
//   c = (blue, bits(y0 - oy | (y1 - oy) << 16), bits(pair index), opacity)
// so that sigma * log2e = -(a.z dx^2 + a.w dx dy + b.x dy^2) and
// alpha = min(0.99, exp2(-sigma log2e + b.y)).
__device__ __forceinline__ void stage_record(const Rec &r, const float2 lo, const TileCtx &c, uint32_t tile_h,
                                             float4 &a, float4 &b, float4 &d) {
    const float ut = (r.r0.x - (float)c.ox) + lo.x;
    const float vt = (r.r0.y - (float)c.oy) + lo.y;
    a = make_float4(ut, vt, -0.5f * kLog2e * r.r0.z, -kLog2e * r.r0.w);
    b = make_float4(-0.5f * kLog2e * r.r1.x, __log2f(r.r1.y), r.r1.z, r.r1.w);
    const uint32_t by = __float_as_uint(r.r2.z);
    const int y0 = (int)(by & 0xffffu) - (int)c.oy, y1 = (int)(by >> 16) - (int)c.oy;
    // clamp into [-1, tile_h] so the packed fields stay non-negative 16-bit values
    const uint32_t y0c = (uint32_t)(max(y0, -1) + 1), y1c = (uint32_t)(min(y1, (int)tile_h) + 1);
    // pair index in emission order: offset + row-major position in the tile box
    const uint32_t bx = __float_as_uint(r.r2.y);
    const uint32_t tx0 = (bx & 0xffffu) / kTileW, tx1 = (bx >> 16) / kTileW;
    const uint32_t ty0 = (by & 0xffffu) / tile_h;
    const uint32_t p = __float_as_uint(r.r2.w) + (c.ty - ty0) * (tx1 - tx0 + 1) + (c.tx - tx0);
    d = make_float4(r.r2.x, __uint_as_float(y0c | (y1c << 16)), __uint_as_float(p), r.r1.y);
}

// Does the record's box (rows y0..y1 relative to the tile, stored +1) touch
// rows [r0, r0 + 3] of the tile?
__device__ __forceinline__ bool slab_hit(float packed, int r0) {
    const uint32_t u = __float_as_uint(packed);
    const int y0 = (int)(u & 0xffffu) - 1, y1 = (int)(u >> 16) - 1;
    return y0 <= r0 + 3 && y1 >= r0;
}

__device__ __forceinline__ uint32_t next_tile(bool persistent, uint32_t *queue, uint32_t first, uint32_t &iter) {
    if (!persistent) return iter++ == 0 ? first : 0xffffffffu;
    uint32_t t = 0;
    if (threadIdx.x == 0) t = atomicAdd(queue, 1u);
    return __shfl(t, 0, kWave);
}

// ---------------------------------------------------------------------------
// A6: forward
// ---------------------------------------------------------------------------
template <int RPL>
__global__ __launch_bounds__(kWave) void k_composite_fwd(ViewTable vt, const uint2 *__restrict__ ranges,
                                                         const uint32_t *__restrict__ pval,
                                                         const Rec *__restrict__ rec, const float2 *__restrict__ ulo,
                                                         float3 bg, float *__restrict__ out_rgb,
                                                         float *__restrict__ out_T, float *__restrict__ pix_T,
                                                         uint32_t *__restrict__ pix_n, WsHeader *hdr, int persistent) {
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
        bool live[RPL];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const uint32_t py = c.oy + ly + 4 * k;
            live[k] = px < c.width && py < c.height;
            T[k] = 1.f;
            C0[k] = C1[k] = C2[k] = 0.f;
            last[k] = 0;
            ncontrib[k] = 0;
            stop_at[k] = 0xffffffffu;
        }
        const uint2 rg = ranges[t];
        for (uint32_t b0 = rg.x; b0 < rg.y; b0 += kWave) {
            bool any_live = false;
#pragma unroll
            for (int k = 0; k < RPL; ++k) any_live |= live[k];
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
                const float4 a = sa[j], b = sb[j], d = sd[j];
                const float dx = a.x - pxl;
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
                    if (!slab_hit(d.y, 4 * k)) continue;  // uniform across the wave
                    const float dy = a.y - ((float)(ly + 4 * k) + 0.5f);
                    const float e2 = a.z * dx * dx + a.w * dx * dy + b.x * dy * dy;
                    const float alpha = fminf(kAlphaMax, exp2f(e2 + b.y));
                    if (live[k] && e2 <= 0.f && alpha >= kAlphaMin) {
                        const float Tn = T[k] * (1.f - alpha);
                        if (Tn < kTMin) {
                            live[k] = false;
                            stop_at[k] = b0 - rg.x + (uint32_t)j;
                        } else {
                            const float w = alpha * T[k];
                            C0[k] += b.z * w;
                            C1[k] += b.w * w;
                            C2[k] += d.x * w;
                            T[k] = Tn;
                            last[k] = b0 - rg.x + (uint32_t)j + 1;
                            ++ncontrib[k];
                        }
                    }
                }
            }
            __syncthreads();
        }
        // outputs
        const uint32_t len = rg.y - rg.x;
        uint32_t evals = 0, replays = 0, contrib = 0;
        const size_t plane = (size_t)c.width * c.height;
        float *img = out_rgb + 3 * (size_t)c.pix_off;
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const uint32_t py = c.oy + ly + 4 * k;
            if (px < c.width && py < c.height) {
                const size_t pix = (size_t)py * c.width + px;
                img[pix] = C0[k] + T[k] * bg.x;
                img[plane + pix] = C1[k] + T[k] * bg.y;
                img[2 * plane + pix] = C2[k] + T[k] * bg.z;
                pix_T[c.pix_off + pix] = T[k];
                pix_n[c.pix_off + pix] = last[k];
                if (out_T) out_T[c.pix_off + pix] = T[k];
                evals += stop_at[k] != 0xffffffffu ? stop_at[k] + 1 : len;
                replays += last[k];
                contrib += ncontrib[k];
            }
        }
        // per-tile work counters for the measurement harness (integer adds:
        // order independent)
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
}

// ---------------------------------------------------------------------------
// A7: backward
// ---------------------------------------------------------------------------
template <int RPL>
__global__ __launch_bounds__(kWave) void k_composite_bwd(ViewTable vt, const uint2 *__restrict__ ranges,
                                                         const uint32_t *__restrict__ pval,
                                                         const Rec *__restrict__ rec, const float2 *__restrict__ ulo,
                                                         const float *__restrict__ out_rgb,
                                                         const float *__restrict__ dL_drgb,
                                                         const uint32_t *__restrict__ pix_n,
                                                         float *__restrict__ partial, WsHeader *hdr, int persistent) {
    __shared__ float4 sa[kWave], sb[kWave], sd[kWave];
    const int lane = threadIdx.x;
    const int lx = lane & 15, ly = lane >> 4;
    const float pxl = (float)lx + 0.5f;
    uint32_t iter = 0;
    for (;;) {
        const uint32_t t = next_tile(persistent != 0, &hdr->queue[1], blockIdx.x, iter);
        if (t >= vt.total_tiles) break;
        const TileCtx c = tile_ctx(vt, t);
        const uint32_t px = c.ox + lx;
        const size_t plane = (size_t)c.width * c.height;
        const float *img = out_rgb + 3 * (size_t)c.pix_off;
        const float *gimg = dL_drgb + 3 * (size_t)c.pix_off;
        float T[RPL], g0[RPL], g1[RPL], g2[RPL], gout[RPL], gacc[RPL];
        uint32_t ncon[RPL];
        uint32_t nmax = 0;
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const uint32_t py = c.oy + ly + 4 * k;
            T[k] = 1.f;
            gacc[k] = 0.f;
            if (px < c.width && py < c.height) {
                const size_t pix = (size_t)py * c.width + px;
                ncon[k] = pix_n[c.pix_off + pix];
                g0[k] = gimg[pix];
                g1[k] = gimg[plane + pix];
                g2[k] = gimg[2 * plane + pix];
                gout[k] = g0[k] * img[pix] + g1[k] * img[plane + pix] + g2[k] * img[2 * plane + pix];
            } else {
                ncon[k] = 0;
                g0[k] = g1[k] = g2[k] = gout[k] = 0.f;
            }
            nmax = max(nmax, ncon[k]);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) nmax = max(nmax, (uint32_t)__shfl_xor((int)nmax, o, kWave));
        const uint2 rg = ranges[t];
        for (uint32_t b0 = rg.x; b0 < rg.y; b0 += kWave) {
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
                const uint32_t pos = b0 - rg.x + (uint32_t)j;
                const float4 a = sa[j], b = sb[j], d = sd[j];
                float s[kPartialStride] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // Swx Swy Sxx Sxy Syy So gr gg gb
                bool any = false;
                if (pos < nmax) {
                    const float dx = a.x - pxl;
#pragma unroll
                    for (int k = 0; k < RPL; ++k) {
                        if (!slab_hit(d.y, 4 * k)) continue;
                        const float dy = a.y - ((float)(ly + 4 * k) + 0.5f);
                        const float e2 = a.z * dx * dx + a.w * dx * dy + b.x * dy * dy;
                        const float araw = exp2f(e2 + b.y);
                        const float alpha = fminf(kAlphaMax, araw);
                        if (pos < ncon[k] && e2 <= 0.f && alpha >= kAlphaMin) {
                            any = true;
                            const float w = alpha * T[k];
                            s[6] += w * g0[k];
                            s[7] += w * g1[k];
                            s[8] += w * g2[k];
                            const float grgb = g0[k] * b.z + g1[k] * b.w + g2[k] * d.x;
                            gacc[k] += w * grgb;
                            const float one_m = 1.f - alpha;
                            const float dalpha = T[k] * grgb - (gout[k] - gacc[k]) / one_m;
                            T[k] *= one_m;
                            if (araw < kAlphaMax) {
                                const float sa_ = dalpha * alpha;  // dL/dsigma = -sa_, dL/do = sa_ / o
                                s[5] += sa_;
                                const float wx = -sa_ * dx, wy = -sa_ * dy;
                                s[0] += wx;
                                s[1] += wy;
                                s[2] += wx * dx;
                                s[3] += wx * dy;
                                s[4] += wy * dy;
                            }
                        }
                    }
                }
                const uint32_t p = __float_as_uint(d.z);
                float *dst = partial + (size_t)p * kPartialStride;
                if (__ballot(any) != 0ull) {
#pragma unroll
                    for (int q = 0; q < kPartialStride; ++q) s[q] = wave_sum(s[q]);
                    // screen-space gradient of (u, v, A, B, C, o, r, g, b)
                    const float A = -2.f * a.z / kLog2e, B = -a.w / kLog2e, Cc = -2.f * b.x / kLog2e;
                    float outv = 0.f;
                    switch (lane) {
                        case 0: outv = A * s[0] + B * s[1]; break;
                        case 1: outv = Cc * s[1] + B * s[0]; break;
                        case 2: outv = 0.5f * s[2]; break;
                        case 3: outv = s[3]; break;
                        case 4: outv = 0.5f * s[4]; break;
                        case 5: outv = s[5] / d.w; break;
                        case 6: outv = s[6]; break;
                        case 7: outv = s[7]; break;
                        case 8: outv = s[8]; break;
                        default: break;
                    }
                    if (lane < kPartialStride) dst[lane] = outv;
                } else if (lane < kPartialStride) {
                    dst[lane] = 0.f;
                }
            }
            __syncthreads();
        }
    }
}

void launch_composite_fwd(const ViewTable &vt, const uint2 *ranges, const uint32_t *pval, const Rec *rec,
                          const float2 *ulo, float3 bg, float *out_rgb, float *out_T, float *pix_T, uint32_t *pix_n,
                          WsHeader *hdr, bool persistent, int persistent_ctas, hipStream_t st) {
    if (vt.total_tiles == 0) return;
    const dim3 grid(persistent ? (unsigned)persistent_ctas : vt.total_tiles);
    const int p = persistent ? 1 : 0;
    switch (vt.tile_h) {
        case 4: hipLaunchKernelGGL(k_composite_fwd<1>, grid, dim3(kWave), 0, st, vt, ranges, pval, rec, ulo, bg, out_rgb, out_T, pix_T, pix_n, hdr, p); break;
        case 8: hipLaunchKernelGGL(k_composite_fwd<2>, grid, dim3(kWave), 0, st, vt, ranges, pval, rec, ulo, bg, out_rgb, out_T, pix_T, pix_n, hdr, p); break;
        case 32: hipLaunchKernelGGL(k_composite_fwd<8>, grid, dim3(kWave), 0, st, vt, ranges, pval, rec, ulo, bg, out_rgb, out_T, pix_T, pix_n, hdr, p); break;
        default: hipLaunchKernelGGL(k_composite_fwd<4>, grid, dim3(kWave), 0, st, vt, ranges, pval, rec, ulo, bg, out_rgb, out_T, pix_T, pix_n, hdr, p); break;
    }
}

void launch_composite_bwd(const ViewTable &vt, const uint2 *ranges, const uint32_t *pval, const Rec *rec,
                          const float2 *ulo, const float *out_rgb, const float *dL_drgb, const float *pix_T,
                          const uint32_t *pix_n, float *partial, WsHeader *hdr, bool persistent, int persistent_ctas,
                          hipStream_t st) {
    (void)pix_T;
    if (vt.total_tiles == 0) return;
    const dim3 grid(persistent ? (unsigned)persistent_ctas : vt.total_tiles);
    const int p = persistent ? 1 : 0;
    switch (vt.tile_h) {
        case 4: hipLaunchKernelGGL(k_composite_bwd<1>, grid, dim3(kWave), 0, st, vt, ranges, pval, rec, ulo, out_rgb, dL_drgb, pix_n, partial, hdr, p); break;
        case 8: hipLaunchKernelGGL(k_composite_bwd<2>, grid, dim3(kWave), 0, st, vt, ranges, pval, rec, ulo, out_rgb, dL_drgb, pix_n, partial, hdr, p); break;
        case 32: hipLaunchKernelGGL(k_composite_bwd<8>, grid, dim3(kWave), 0, st, vt, ranges, pval, rec, ulo, out_rgb, dL_drgb, pix_n, partial, hdr, p); break;
        default: hipLaunchKernelGGL(k_composite_bwd<4>, grid, dim3(kWave), 0, st, vt, ranges, pval, rec, ulo, out_rgb, dL_drgb, pix_n, partial, hdr, p); break;
    }
}

}  // namespace gsr
