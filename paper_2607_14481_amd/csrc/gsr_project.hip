// gsr_project.hip -- per-Gaussian stages of the rasterizer on gfx950:
//   A1 k_project_fwd  : EWA projection, SH colour, alpha >= 1/255 box, tile count
//   A8+A9 k_project_bwd: per-Gaussian sum of the per-pair screen-space
//                        gradients, chain rule to every parameter, per-block
//                        partial sums of each view's pose gradient
//   k_pose_finalize    : fixed-order sum of those partials, 4x4 and 6-DoF twist
//
// The geometric part of A1 runs in FP64: it is HBM-bound (~100-300 bytes per
// Gaussian against a few hundred flops), so double precision costs nothing
// measurable and keeps the centre, box and depth key within an ulp of the exact
// values (world coordinates of tens of metres otherwise cost ~1e-4 px).
#include "gsr_internal.h"

namespace gsr {

// Real SH basis of degree <= 3 in the 3DGS order and signs (real harmonics with
// the Condon-Shortley phase, m = -l..l).  Normalisations: c0 = 1/(2 sqrt(pi)),
// c1 = sqrt(3/(4 pi)), c2a = sqrt(15/pi)/2, c2b = sqrt(5/pi)/4,
// c2c = sqrt(15/pi)/4, c3a = sqrt(35/(2 pi))/4, c3b = sqrt(105/pi)/2,
// c3c = sqrt(21/(2 pi))/4, c3d = sqrt(7/pi)/4, c3e = sqrt(105/pi)/4.
struct ShC {
    static constexpr double c0 = 0.28209479177387814, c1 = 0.4886025119029199;
    static constexpr double c2a = 1.0925484305920792, c2b = 0.31539156525252005, c2c = 0.5462742152960396;
    static constexpr double c3a = 0.5900435899266435, c3b = 2.890611442640554, c3c = 0.4570457994644658;
    static constexpr double c3d = 0.3731763325901154, c3e = 1.445305721320277;
};

template <int DEG, typename T>
__device__ __forceinline__ void sh_eval(T x, T y, T z, T *Y) {
    Y[0] = T(ShC::c0);
    if constexpr (DEG >= 1) {
        Y[1] = -T(ShC::c1) * y;
        Y[2] = T(ShC::c1) * z;
        Y[3] = -T(ShC::c1) * x;
    }
    if constexpr (DEG >= 2) {
        const T xx = x * x, yy = y * y, zz = z * z;
        Y[4] = T(ShC::c2a) * x * y;
        Y[5] = -T(ShC::c2a) * y * z;
        Y[6] = T(ShC::c2b) * (T(2) * zz - xx - yy);
        Y[7] = -T(ShC::c2a) * x * z;
        Y[8] = T(ShC::c2c) * (xx - yy);
        if constexpr (DEG >= 3) {
            Y[9] = -T(ShC::c3a) * y * (T(3) * xx - yy);
            Y[10] = T(ShC::c3b) * x * y * z;
            Y[11] = -T(ShC::c3c) * y * (T(4) * zz - xx - yy);
            Y[12] = T(ShC::c3d) * z * (T(2) * zz - T(3) * xx - T(3) * yy);
            Y[13] = -T(ShC::c3c) * x * (T(4) * zz - xx - yy);
            Y[14] = T(ShC::c3e) * z * (xx - yy);
            Y[15] = -T(ShC::c3a) * x * (xx - T(3) * yy);
        }
    }
}

// Gradient of sum_k w_k Y_k(x, y, z) with respect to (x, y, z), for weights w.
template <int DEG>
__device__ __forceinline__ void sh_grad_dir(float x, float y, float z, const float *w, float &gx, float &gy,
                                            float &gz) {
    gx = gy = gz = 0.f;
    if constexpr (DEG >= 1) {
        const float c1 = float(ShC::c1);
        gy -= c1 * w[1];
        gz += c1 * w[2];
        gx -= c1 * w[3];
    }
    if constexpr (DEG >= 2) {
        const float a = float(ShC::c2a), b = float(ShC::c2b), c = float(ShC::c2c);
        gx += a * y * w[4];
        gy += a * x * w[4];
        gy -= a * z * w[5];
        gz -= a * y * w[5];
        gx -= 2.f * b * x * w[6];
        gy -= 2.f * b * y * w[6];
        gz += 4.f * b * z * w[6];
        gx -= a * z * w[7];
        gz -= a * x * w[7];
        gx += 2.f * c * x * w[8];
        gy -= 2.f * c * y * w[8];
    }
    if constexpr (DEG >= 3) {
        const float a = float(ShC::c3a), b = float(ShC::c3b), c = float(ShC::c3c);
        const float d = float(ShC::c3d), e = float(ShC::c3e);
        const float xx = x * x, yy = y * y, zz = z * z;
        // y(3x^2 - y^2)
        gx -= a * 6.f * x * y * w[9];
        gy -= a * (3.f * xx - 3.f * yy) * w[9];
        // xyz
        gx += b * y * z * w[10];
        gy += b * x * z * w[10];
        gz += b * x * y * w[10];
        // y(4z^2 - x^2 - y^2)
        gx += c * 2.f * x * y * w[11];
        gy -= c * (4.f * zz - xx - 3.f * yy) * w[11];
        gz -= c * 8.f * y * z * w[11];
        // z(2z^2 - 3x^2 - 3y^2)
        gx -= d * 6.f * x * z * w[12];
        gy -= d * 6.f * y * z * w[12];
        gz += d * (6.f * zz - 3.f * xx - 3.f * yy) * w[12];
        // x(4z^2 - x^2 - y^2)
        gx -= c * (4.f * zz - 3.f * xx - yy) * w[13];
        gy += c * 2.f * x * y * w[13];
        gz -= c * 8.f * x * z * w[13];
        // z(x^2 - y^2)
        gx += e * 2.f * x * z * w[14];
        gy -= e * 2.f * y * z * w[14];
        gz += e * (xx - yy) * w[14];
        // x(x^2 - 3y^2)
        gx -= a * (3.f * xx - 3.f * yy) * w[15];
        gy += a * 6.f * x * y * w[15];
    }
}

// Rotation matrix of a unit quaternion (w, x, y, z).
template <typename T>
__device__ __forceinline__ void quat_rot(T w, T x, T y, T z, T R[9]) {
    R[0] = T(1) - T(2) * (y * y + z * z);
    R[1] = T(2) * (x * y - w * z);
    R[2] = T(2) * (x * z + w * y);
    R[3] = T(2) * (x * y + w * z);
    R[4] = T(1) - T(2) * (x * x + z * z);
    R[5] = T(2) * (y * z - w * x);
    R[6] = T(2) * (x * z - w * y);
    R[7] = T(2) * (y * z + w * x);
    R[8] = T(1) - T(2) * (x * x + y * y);
}

__device__ __forceinline__ void load_pose(const float *__restrict__ w2c, int v, float W[9], float t[3]) {
    const float *m = w2c + 16 * v;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        W[3 * r + 0] = m[4 * r + 0];
        W[3 * r + 1] = m[4 * r + 1];
        W[3 * r + 2] = m[4 * r + 2];
        t[r] = m[4 * r + 3];
    }
}

// ---------------------------------------------------------------------------
// A1: projection forward.  One thread per (view, Gaussian) item, item = v n + i.
// ---------------------------------------------------------------------------
template <int DEG>
__global__ __launch_bounds__(kProjThreads) void k_project_fwd(gsr_gaussians g, ViewTable vt,
                                                              const float *__restrict__ w2c, uint64_t n,
                                                              Rec *__restrict__ rec, float2 *__restrict__ ulo,
                                                              uint32_t *__restrict__ zkey,
                                                              uint32_t *__restrict__ count,
                                                              WsHeader *__restrict__ hdr, uint32_t cap,
                                                              const int64_t *__restrict__ active) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    if (blockIdx.x == 0 && threadIdx.x < sizeof(WsHeader) / 4) {
        // a fresh header for this forward (read first by the visible-item scan)
        reinterpret_cast<uint32_t *>(hdr)[threadIdx.x] = threadIdx.x == offsetof(WsHeader, pair_capacity) / 4 ? cap : 0u;
    }
    const uint64_t item = (uint64_t)blockIdx.x * kProjThreads + threadIdx.x;
    if (item >= n * (uint64_t)vt.n_views) return;
    const int v = (int)(item / n);
    const uint64_t i = item - (uint64_t)v * n;
    if (active && (int64_t)i >= *active) {  // beyond the device-given count: culled, nothing read
        zkey[item] = kCulledKey;
        count[item] = 0;
        return;
    }
    const ViewInfo cam = vt.v[v];

    float Wf[9], tf[3];
    load_pose(w2c, v, Wf, tf);
    const double mx = g.means[3 * i + 0], my = g.means[3 * i + 1], mz = g.means[3 * i + 2];
    const double px = (double)Wf[0] * mx + (double)Wf[1] * my + (double)Wf[2] * mz + (double)tf[0];
    const double py = (double)Wf[3] * mx + (double)Wf[4] * my + (double)Wf[5] * mz + (double)tf[1];
    const double pz = (double)Wf[6] * mx + (double)Wf[7] * my + (double)Wf[8] * mz + (double)tf[2];

    uint32_t cnt = 0;
    uint32_t key = kCulledKey;
    do {
        if (!(pz > (double)cam.near_plane)) break;
        const float4 qf = reinterpret_cast<const float4 *>(g.quats)[i];
        const double qn = sqrt((double)qf.x * qf.x + (double)qf.y * qf.y + (double)qf.z * qf.z + (double)qf.w * qf.w);
        if (!(qn > 0.0)) break;
        double R[9];
        quat_rot<double>(qf.x / qn, qf.y / qn, qf.z / qn, qf.w / qn, R);
        const double s0 = exp((double)g.log_scales[3 * i + 0]);
        const double s1 = exp((double)g.log_scales[3 * i + 1]);
        const double s2 = exp((double)g.log_scales[3 * i + 2]);
        // M = R diag(s); Sigma = M M^T (symmetric, 6 entries)
        const double M[9] = {R[0] * s0, R[1] * s1, R[2] * s2, R[3] * s0, R[4] * s1,
                             R[5] * s2, R[6] * s0, R[7] * s1, R[8] * s2};
        double Sg[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                Sg[3 * a + b] = M[3 * a] * M[3 * b] + M[3 * a + 1] * M[3 * b + 1] + M[3 * a + 2] * M[3 * b + 2];
        const double rx = px / pz, ry = py / pz;
        const double rxc = fmin(fmax(rx, -(double)cam.limx), (double)cam.limx);
        const double ryc = fmin(fmax(ry, -(double)cam.limy), (double)cam.limy);
        const double j00 = cam.fx / pz, j02 = -cam.fx * rxc / pz;
        const double j11 = cam.fy / pz, j12 = -cam.fy * ryc / pz;
        // T = J W (2x3)
        double T0[3], T1[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            T0[b] = j00 * Wf[b] + j02 * Wf[6 + b];
            T1[b] = j11 * Wf[3 + b] + j12 * Wf[6 + b];
        }
        double TS0[3], TS1[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            TS0[b] = T0[0] * Sg[b] + T0[1] * Sg[3 + b] + T0[2] * Sg[6 + b];
            TS1[b] = T1[0] * Sg[b] + T1[1] * Sg[3 + b] + T1[2] * Sg[6 + b];
        }
        const double ca = TS0[0] * T0[0] + TS0[1] * T0[1] + TS0[2] * T0[2] + (double)kLowPass;
        const double cb = TS0[0] * T1[0] + TS0[1] * T1[1] + TS0[2] * T1[2];
        const double cc = TS1[0] * T1[0] + TS1[1] * T1[1] + TS1[2] * T1[2] + (double)kLowPass;
        const double det = ca * cc - cb * cb;
        if (!(det > 0.0)) break;
        const float op = g.opacities[i];
        if (!(op >= kAlphaMin)) break;
        const double u = cam.fx * rx + cam.cx, vv = cam.fy * ry + cam.cy;
        // exact box of the alpha >= 1/255 ellipse, pixel centres at i + 1/2
        const double k2 = 2.0 * log(255.0 * (double)op);
        const double ex = sqrt(k2 * ca), ey = sqrt(k2 * cc);
        double x0 = ceil(u - ex - 0.5), x1 = floor(u + ex - 0.5);
        double y0 = ceil(vv - ey - 0.5), y1 = floor(vv + ey - 0.5);
        x0 = fmax(x0, 0.0);
        y0 = fmax(y0, 0.0);
        x1 = fmin(x1, (double)(cam.width - 1));
        y1 = fmin(y1, (double)(cam.height - 1));
        if (!(x0 <= x1) || !(y0 <= y1)) break;
        const uint32_t ix0 = (uint32_t)x0, ix1 = (uint32_t)x1, iy0 = (uint32_t)y0, iy1 = (uint32_t)y1;
        cnt = (ix1 / kTileW - ix0 / kTileW + 1) * (iy1 / vt.tile_h - iy0 / vt.tile_h + 1);
        key = __float_as_uint((float)pz);

        // colour: direction from the camera centre c = -W^T t, world frame
        const double cx = -((double)Wf[0] * tf[0] + (double)Wf[3] * tf[1] + (double)Wf[6] * tf[2]);
        const double cy = -((double)Wf[1] * tf[0] + (double)Wf[4] * tf[1] + (double)Wf[7] * tf[2]);
        const double cz = -((double)Wf[2] * tf[0] + (double)Wf[5] * tf[1] + (double)Wf[8] * tf[2]);
        double dx = mx - cx, dy = my - cy, dz = mz - cz;
        const double dn = sqrt(dx * dx + dy * dy + dz * dz);
        dx /= dn;
        dy /= dn;
        dz /= dn;
        double Y[K];
        sh_eval<DEG, double>(dx, dy, dz, Y);
        double col[3] = {0.5, 0.5, 0.5};
        const float *shp = g.sh + (size_t)i * K * 3;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            col[0] += (double)shp[3 * k + 0] * Y[k];
            col[1] += (double)shp[3 * k + 1] * Y[k];
            col[2] += (double)shp[3 * k + 2] * Y[k];
        }
        const float uh = (float)u, vh = (float)vv;
        Rec r;
        r.r0 = make_float4(uh, vh, (float)(cc / det), (float)(-cb / det));
        r.r1 = make_float4((float)(ca / det), op, (float)fmax(col[0], 0.0), (float)fmax(col[1], 0.0));
        r.r2 = make_float4((float)fmax(col[2], 0.0), __uint_as_float(pack_u16(ix0, ix1)),
                           __uint_as_float(pack_u16(iy0, iy1)), 0.f);
        rec[item] = r;
        ulo[item] = make_float2((float)(u - (double)uh), (float)(vv - (double)vh));
    } while (0);
    zkey[item] = key;
    count[item] = cnt;
}

void launch_project_fwd(const gsr_gaussians &g, const ViewTable &vt, const float *w2c, uint64_t n, Rec *rec,
                        float2 *ulo, uint32_t *zkey, uint32_t *count, WsHeader *hdr, uint32_t cap,
                        const int64_t *active, hipStream_t st) {
    const uint64_t items = n * (uint64_t)vt.n_views;
    if (items == 0) {
        launch_reset_header(hdr, cap, st);
        return;
    }
    const dim3 grid((unsigned)((items + kProjThreads - 1) / kProjThreads));
    switch (g.sh_degree) {
        case 0: hipLaunchKernelGGL(k_project_fwd<0>, grid, dim3(kProjThreads), 0, st, g, vt, w2c, n, rec, ulo, zkey, count, hdr, cap, active); break;
        case 1: hipLaunchKernelGGL(k_project_fwd<1>, grid, dim3(kProjThreads), 0, st, g, vt, w2c, n, rec, ulo, zkey, count, hdr, cap, active); break;
        case 2: hipLaunchKernelGGL(k_project_fwd<2>, grid, dim3(kProjThreads), 0, st, g, vt, w2c, n, rec, ulo, zkey, count, hdr, cap, active); break;
        default: hipLaunchKernelGGL(k_project_fwd<3>, grid, dim3(kProjThreads), 0, st, g, vt, w2c, n, rec, ulo, zkey, count, hdr, cap, active); break;
    }
}

// ---------------------------------------------------------------------------
// A8: per-item sums of the per-pair moments, in a fixed order.
//
// An item's pairs are contiguous in emission order, but their number ranges
// from one to thousands (splats near the camera), so the work is split by
// pairs, not by items: a workgroup takes one chunk of 1024 consecutive pair
// slots, 4 per thread (nine float4 loads per thread, coalesced).  Pairs whose
// tile stopped before reaching the item were never written by the backward
// compositing and count as zero: the emission clears one flag byte per slot
// and the backward compositing sets the flags of the slots it replays, so the
// flags (4 per thread, one 32-bit load) tell which moments to load without
// finding each pair's tile first.
//
// Within the chunk a segmented inclusive scan over the threads (keys = local
// item index; in each wave DPP row shifts and row broadcasts, which stay in
// the VALU, then a carry across the four waves) gives each item's sum at the
// thread holding its last pair.  Items that lie wholly
// in the chunk are written to `screen`; an item that starts before the chunk
// leaves its part of this chunk in carry[c][0], one that ends after it in
// carry[c][1], and A9 adds an item's parts from its first chunk to its last
// in chunk order.  Every sum is a fixed function of the layout, so two runs
// agree bit for bit.
// ---------------------------------------------------------------------------
constexpr uint32_t kNoKey = 0xffffffffu;

// The chunk's items as the reduction needs them: first pair slot and item id
// (p0[nloc] is the end of the last one).  Item ids come from the visible list.
struct ChunkSlots {
    uint32_t p0[kChunkPairs + 2];
    uint32_t item[kChunkPairs + 1];
};

__device__ __forceinline__ uint32_t load_chunk_slots(const uint32_t *__restrict__ poff,
                                                     const uint32_t *__restrict__ chunk_item,
                                                     const uint32_t *__restrict__ vis, uint32_t c, uint32_t m,
                                                     uint32_t nvis, ChunkSlots &cs) {
    const uint32_t c0 = c * kChunkPairs;
    const uint32_t i_lo = chunk_item[c];
    const uint32_t i_hi = c0 + kChunkPairs < m ? chunk_item[c + 1] : nvis - 1;
    const uint32_t nloc = i_hi - i_lo + 1;
    for (uint32_t k = threadIdx.x; k <= nloc; k += kChunkThreads) {
        const uint32_t i = i_lo + k;
        if (k == nloc) {
            cs.p0[k] = i < nvis ? poff[i] : m;
            continue;
        }
        cs.p0[k] = poff[i];
        cs.item[k] = vis[i];
    }
    __syncthreads();
    return nloc;
}

// largest local index k < nloc with p0[k] <= p (p0[0] <= p holds)
__device__ __forceinline__ uint32_t find_chunk_slot(const ChunkSlots &cs, uint32_t nloc, uint32_t p) {
    uint32_t lo = 0, hi = nloc - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (cs.p0[mid] <= p)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// One step of a segmented inclusive scan over the wave: (v, f) takes the
// (value, segment-start) pair of the lane `CTRL` names (rows outside ROW_MASK,
// and lanes without a source, take (0, false)) and combines
// (v_src, f_src) + (v, f) = (f ? v : v_src + v, f_src | f).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void seg_scan_step(float (&v)[kPartialStride], bool &f) {
    const bool fs = __builtin_amdgcn_update_dpp(0, f ? 1 : 0, CTRL, ROW_MASK, 0xf, false) != 0;
#pragma unroll
    for (int j = 0; j < kPartialStride; ++j) {
        const float o = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v[j]), CTRL, ROW_MASK, 0xf, false));
        v[j] = f ? v[j] : o + v[j];
    }
    f = f || fs;
}

__device__ __forceinline__ void write_item_sum(const ChunkSlots &ci, uint32_t k, uint32_t c0, uint32_t cend,
                                               uint32_t c, const float v[kPartialStride], float4 *__restrict__ screen,
                                               float *__restrict__ carry) {
    const bool before = ci.p0[k] < c0, after = ci.p0[k + 1] > cend;
    if (!before && !after) {
        float4 *o = screen + 3 * (size_t)ci.item[k];
        o[0] = make_float4(v[0], v[1], v[2], v[3]);
        o[1] = make_float4(v[4], v[5], v[6], v[7]);
        o[2] = make_float4(v[8], 0.f, 0.f, 0.f);
        return;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        if (q == 0 ? before : after) {
            float *o = carry + ((size_t)c * 2 + q) * kPartialStride;
#pragma unroll
            for (int j = 0; j < kPartialStride; ++j) o[j] = v[j];
        }
    }
}

__global__ __launch_bounds__(kChunkThreads) void k_pair_reduce(const uint32_t *__restrict__ poff,
                                                               const uint32_t *__restrict__ chunk_item,
                                                               const uint32_t *__restrict__ vis,
                                                               const uint32_t *__restrict__ pflag,
                                                               const float *__restrict__ partial,
                                                               float4 *__restrict__ screen, float *__restrict__ carry,
                                                               const WsHeader *__restrict__ hdr) {
    __shared__ ChunkSlots ci;
    __shared__ uint32_t s_kf[kChunkThreads], s_kl[kChunkThreads];
    __shared__ float s_wv[4][kPartialStride];
    __shared__ uint32_t s_wf[4];
    if (hdr->overflow) return;
    const uint32_t m = hdr->n_pairs, nvis = hdr->n_visible;
    const uint32_t c = blockIdx.x, c0 = c * kChunkPairs;
    if (c0 >= m) return;  // uniform per workgroup
    const uint32_t cend = min(c0 + kChunkPairs, m);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

    // ---- this thread's pairs and whether the backward compositing wrote
    // their moments (pairs past the positions their tile replayed were never
    // reached: most of a dense scene's pairs, so their values are not read).
    // The flags and the moments are loaded before the chunk's items, so their
    // latency overlaps.
    const uint32_t pb = c0 + (uint32_t)tid * kChunkPerThread;
    bool valid[kChunkPerThread];
    {
        const uint32_t f4 = pb < cend ? pflag[pb / 4] : 0u;
#pragma unroll
        for (uint32_t u = 0; u < kChunkPerThread; ++u) valid[u] = pb + u < cend && ((f4 >> (8 * u)) & 0xffu) != 0;
    }
    float x[kChunkPerThread][kPartialStride];
#pragma unroll
    for (uint32_t u = 0; u < kChunkPerThread; ++u)
#pragma unroll
        for (int j = 0; j < kPartialStride; ++j) x[u][j] = 0.f;
    bool any = false;
#pragma unroll
    for (uint32_t u = 0; u < kChunkPerThread; ++u) any |= valid[u];
    if (any && pb + kChunkPerThread <= cend) {
        const float4 *src = reinterpret_cast<const float4 *>(partial + (size_t)pb * kPartialStride);
        float4 f[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) f[j] = src[j];
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            x[(4 * j + 0) / 9][(4 * j + 0) % 9] = f[j].x;
            x[(4 * j + 1) / 9][(4 * j + 1) % 9] = f[j].y;
            x[(4 * j + 2) / 9][(4 * j + 2) % 9] = f[j].z;
            x[(4 * j + 3) / 9][(4 * j + 3) % 9] = f[j].w;
        }
#pragma unroll
        for (uint32_t u = 0; u < kChunkPerThread; ++u)
#pragma unroll
            for (int j = 0; j < kPartialStride; ++j) x[u][j] = valid[u] ? x[u][j] : 0.f;
    } else if (any) {
#pragma unroll
        for (uint32_t u = 0; u < kChunkPerThread; ++u)
#pragma unroll
            for (int j = 0; j < kPartialStride; ++j)
                x[u][j] = valid[u] ? partial[(size_t)(pb + u) * kPartialStride + j] : 0.f;
    }
    const uint32_t nloc = load_chunk_slots(poff, chunk_item, vis, c, m, nvis, ci);
    uint32_t key[kChunkPerThread];
#pragma unroll
    for (uint32_t u = 0; u < kChunkPerThread; ++u) key[u] = kNoKey;
    if (pb < cend) {
        uint32_t k = find_chunk_slot(ci, nloc, pb);
#pragma unroll
        for (uint32_t u = 0; u < kChunkPerThread; ++u) {
            const uint32_t p = pb + u;
            if (p < cend) {
                while (k + 1 < nloc && ci.p0[k + 1] <= p) ++k;
                key[u] = k;
            }
        }
    }

    // ---- segments inside the thread: head (first), complete middles, tail (last)
    float head[kPartialStride], v[kPartialStride];
    bool multi = false;
    uint32_t kc = key[0];
#pragma unroll
    for (int j = 0; j < kPartialStride; ++j) v[j] = x[0][j], head[j] = 0.f;
#pragma unroll
    for (uint32_t u = 1; u < kChunkPerThread; ++u) {
        if (key[u] == kc) {
#pragma unroll
            for (int j = 0; j < kPartialStride; ++j) v[j] += x[u][j];
        } else {
            if (!multi) {
#pragma unroll
                for (int j = 0; j < kPartialStride; ++j) head[j] = v[j];
                multi = true;
            } else if (kc != kNoKey) {
                write_item_sum(ci, kc, c0, cend, c, v, screen, carry);  // started and ended in this thread
            }
            kc = key[u];
#pragma unroll
            for (int j = 0; j < kPartialStride; ++j) v[j] = x[u][j];
        }
    }
    const uint32_t kf = key[0], kl = kc;
    s_kf[tid] = kf;
    s_kl[tid] = kl;
    __syncthreads();
    const uint32_t kl_prev = tid > 0 ? s_kl[tid - 1] : kNoKey;
    const uint32_t kf_next = tid + 1 < (int)kChunkThreads ? s_kf[tid + 1] : kNoKey;

    // ---- segmented inclusive scan of the tails: (v, f) with f = "a segment starts in range"
    bool f = multi || kl_prev != kf;
    // Hillis-Steele within each row of 16 lanes, then the row totals by two
    // row broadcasts (lane 15 into rows 1 and 3, lane 31 into rows 2 and 3)
    seg_scan_step<0x111, 0xf>(v, f);  // row_shr:1
    seg_scan_step<0x112, 0xf>(v, f);  // row_shr:2
    seg_scan_step<0x114, 0xf>(v, f);  // row_shr:4
    seg_scan_step<0x118, 0xf>(v, f);  // row_shr:8
    seg_scan_step<0x142, 0xa>(v, f);  // row_bcast:15
    seg_scan_step<0x143, 0xc>(v, f);  // row_bcast:31
    if (lane == kWave - 1) {
#pragma unroll
        for (int j = 0; j < kPartialStride; ++j) s_wv[wv][j] = v[j];
        s_wf[wv] = f ? 1u : 0u;
    }
    __syncthreads();
    // running value of the segment open at the end of the previous waves
    float cin[kPartialStride];
#pragma unroll
    for (int j = 0; j < kPartialStride; ++j) cin[j] = 0.f;
    for (int w = 0; w < wv; ++w) {
#pragma unroll
        for (int j = 0; j < kPartialStride; ++j) cin[j] = s_wf[w] ? s_wv[w][j] : cin[j] + s_wv[w][j];
    }
    if (!f) {
#pragma unroll
        for (int j = 0; j < kPartialStride; ++j) v[j] = cin[j] + v[j];
    }
    // inclusive value of the previous thread's tail segment
    float prev[kPartialStride];
#pragma unroll
    for (int j = 0; j < kPartialStride; ++j)  // wave_shr:1, lane 0 keeps cin
        prev[j] = __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(cin[j]), __float_as_int(v[j]), 0x138, 0xf, 0xf, false));

    // ---- finished segments
    if (multi && kf != kNoKey) {  // the head segment ends in this thread
        float tot[kPartialStride];
#pragma unroll
        for (int j = 0; j < kPartialStride; ++j) tot[j] = kl_prev == kf ? prev[j] + head[j] : head[j];
        write_item_sum(ci, kf, c0, cend, c, tot, screen, carry);
    }
    if (kl != kNoKey && kf_next != kl) write_item_sum(ci, kl, c0, cend, c, v, screen, carry);
}

void launch_pair_reduce(const uint32_t *poff, const uint32_t *chunk_item, uint64_t pair_grid, const uint32_t *vis,
                        const uint32_t *pflag, const float *partial, float4 *screen, float *carry, const WsHeader *hdr,
                        hipStream_t st) {
    const uint64_t chunks = chunk_count(pair_grid);
    if (chunks == 0) return;
    hipLaunchKernelGGL(k_pair_reduce, dim3((unsigned)chunks), dim3(kChunkThreads), 0, st, poff, chunk_item, vis,
                       pflag, partial, screen, carry, hdr);
}

// ---------------------------------------------------------------------------
// A9: projection backward.  One thread per Gaussian; loops over views and
// chains each visible item's screen-space gradient back to the parameters and
// to the view's pose.  The item's pair moments come from A8 (or, when its
// pairs span several chunks, from their chunk-boundary parts added in chunk
// order) and turn into the gradient of (u, v, A, B, C, opacity, colour) with
// the item's own conic and opacity: sigma = A dx^2 / 2 + B dx dy + C dy^2 / 2
// with (dx, dy) = (u, v) - pixel, so dL/du = A S_x + B S_y,
// dL/dv = B S_x + C S_y, dL/d(A, B, C) = (S_xx / 2, S_xy, S_yy / 2) and
// dL/do = S_o / o, where S_x = sum w dx, S_xx = sum w dx^2, ... over the
// item's pixels with w = dL/dsigma and S_o = sum alpha dL/dalpha.  The pair
// moments hold S_x .. S_yy negated (sums of -w dx, ...: the compositing forms
// them without a sign change per pair).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void item_moments(const float4 *__restrict__ screen, const float *__restrict__ carry,
                                             uint64_t item, uint32_t p0, uint32_t cnt, float S[kPartialStride]) {
    const uint32_t cf = p0 / kChunkPairs, cl = (p0 + cnt - 1) / kChunkPairs;
    if (cf == cl) {
        const float4 s0 = screen[3 * item], s1 = screen[3 * item + 1], s2 = screen[3 * item + 2];
        S[0] = s0.x, S[1] = s0.y, S[2] = s0.z, S[3] = s0.w;
        S[4] = s1.x, S[5] = s1.y, S[6] = s1.z, S[7] = s1.w, S[8] = s2.x;
        return;
    }
    const float *t = carry + ((size_t)cf * 2 + 1) * kPartialStride;  // its part of the first chunk
#pragma unroll
    for (int j = 0; j < kPartialStride; ++j) S[j] = t[j];
    for (uint32_t c = cf + 1; c <= cl; ++c) {
        const float *h = carry + (size_t)c * 2 * kPartialStride;  // the chunk's first item is this one
#pragma unroll
        for (int j = 0; j < kPartialStride; ++j) S[j] += h[j];
    }
}

// Chain rule of one visible (view, Gaussian) item: its screen-space gradient
// (from the pair moments) back to the Gaussian's parameters (added to gmu, gls,
// gq, gop and to the SH row gsh: stored by the first view, added to by later
// ones) and to the view's pose (added to gW, gt).
template <int DEG>
__device__ __forceinline__ void item_backward(const gsr_gaussians &g, const ViewInfo &cam, const float *__restrict__ w2c,
                                              int v, uint64_t i, uint64_t item, uint32_t cnt,
                                              const Rec *__restrict__ rec, const float4 *__restrict__ screen,
                                              const float *__restrict__ carry, const float *sh_row, float *gsh,
                                              bool &sh_written, float (&gmu)[3], float (&gls)[3], float (&gq)[4],
                                              float &gop, float (&gW)[9], float (&gt)[3]) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const float4 r0 = rec[item].r0, r1 = rec[item].r1;
    float S[kPartialStride];
    item_moments(screen, carry, item, __float_as_uint(rec[item].r2.w), cnt, S);
    // S[0..4] hold the moments of sa = -dL/dsigma: S_x = -S[0], ..., S_yy = -S[4]
    const float gu = -fmaf(r0.z, S[0], r0.w * S[1]), gv = -fmaf(r0.w, S[0], r1.x * S[1]);
    const float gA = -0.5f * S[2], gB = -S[3], gC = -0.5f * S[4], go = S[5] / r1.y;
    const float grgb[3] = {S[6], S[7], S[8]};

    float W[9], t[3];
    load_pose(w2c, v, W, t);
    const float mu[3] = {g.means[3 * i], g.means[3 * i + 1], g.means[3 * i + 2]};
    const double pxd = (double)W[0] * mu[0] + (double)W[1] * mu[1] + (double)W[2] * mu[2] + (double)t[0];
    const double pyd = (double)W[3] * mu[0] + (double)W[4] * mu[1] + (double)W[5] * mu[2] + (double)t[1];
    const double pzd = (double)W[6] * mu[0] + (double)W[7] * mu[1] + (double)W[8] * mu[2] + (double)t[2];
    const float p[3] = {(float)pxd, (float)pyd, (float)pzd};

    gop += go;

    // ---- colour -> SH coefficients and direction
    const float cxw = -(W[0] * t[0] + W[3] * t[1] + W[6] * t[2]);
    const float cyw = -(W[1] * t[0] + W[4] * t[1] + W[7] * t[2]);
    const float czw = -(W[2] * t[0] + W[5] * t[1] + W[8] * t[2]);
    float dvec[3] = {mu[0] - cxw, mu[1] - cyw, mu[2] - czw};
    const float dn = sqrtf(dvec[0] * dvec[0] + dvec[1] * dvec[1] + dvec[2] * dvec[2]);
    const float dir[3] = {dvec[0] / dn, dvec[1] / dn, dvec[2] / dn};
    float Y[K];
    sh_eval<DEG, float>(dir[0], dir[1], dir[2], Y);
    // colour, to know which channels the forward clamped at 0 (the row is read
    // twice rather than held in registers)
    float col[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
    for (int k = 0; k < K; ++k) {
        col[0] = fmaf(sh_row[3 * k], Y[k], col[0]);
        col[1] = fmaf(sh_row[3 * k + 1], Y[k], col[1]);
        col[2] = fmaf(sh_row[3 * k + 2], Y[k], col[2]);
    }
    float gc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) gc[c] = col[c] < 0.f ? 0.f : grgb[c];
    // coefficient gradients (added to an earlier view's) and the weights of
    // dRGB/ddir; gsh may be sh_row itself: each coefficient is read before it
    // is overwritten
    float wdir[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float s0 = sh_row[3 * k], s1 = sh_row[3 * k + 1], s2 = sh_row[3 * k + 2];
        wdir[k] = fmaf(gc[0], s0, fmaf(gc[1], s1, gc[2] * s2));
        float o0 = gc[0] * Y[k], o1 = gc[1] * Y[k], o2 = gc[2] * Y[k];
        if (sh_written) o0 += gsh[3 * k], o1 += gsh[3 * k + 1], o2 += gsh[3 * k + 2];
        gsh[3 * k] = o0;
        gsh[3 * k + 1] = o1;
        gsh[3 * k + 2] = o2;
    }
    sh_written = true;
    float gdx, gdy, gdz;
    sh_grad_dir<DEG>(dir[0], dir[1], dir[2], wdir, gdx, gdy, gdz);
    const float dd = gdx * dir[0] + gdy * dir[1] + gdz * dir[2];
    const float gd[3] = {(gdx - dir[0] * dd) / dn, (gdy - dir[1] * dd) / dn, (gdz - dir[2] * dd) / dn};
    // mean gets +gd, camera centre gets -gd; c_a = -sum_b W[b][a] t_b
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        gmu[a] += gd[a];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            gW[3 * b + a] += t[b] * gd[a];
            gt[b] += W[3 * b + a] * gd[a];
        }
    }

    // ---- recompute the covariance chain
    const float4 qf = reinterpret_cast<const float4 *>(g.quats)[i];
    const float qn = sqrtf(qf.x * qf.x + qf.y * qf.y + qf.z * qf.z + qf.w * qf.w);
    const float q[4] = {qf.x / qn, qf.y / qn, qf.z / qn, qf.w / qn};
    float R[9];
    quat_rot<float>(q[0], q[1], q[2], q[3], R);
    const float sc[3] = {expf(g.log_scales[3 * i]), expf(g.log_scales[3 * i + 1]),
                         expf(g.log_scales[3 * i + 2])};
    float M[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) M[3 * a + b] = R[3 * a + b] * sc[b];
    float Sg[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            Sg[3 * a + b] = M[3 * a] * M[3 * b] + M[3 * a + 1] * M[3 * b + 1] + M[3 * a + 2] * M[3 * b + 2];
    const float rx = (float)(pxd / pzd), ry = (float)(pyd / pzd);
    const float rxc = fminf(fmaxf(rx, -cam.limx), cam.limx);
    const float ryc = fminf(fmaxf(ry, -cam.limy), cam.limy);
    const float iz = 1.f / p[2];
    float J[6] = {cam.fx * iz, 0.f, -cam.fx * rxc * iz, 0.f, cam.fy * iz, -cam.fy * ryc * iz};
    float T[6];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            T[3 * a + b] = J[3 * a] * W[b] + J[3 * a + 1] * W[3 + b] + J[3 * a + 2] * W[6 + b];
    float TS[6];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            TS[3 * a + b] = T[3 * a] * Sg[b] + T[3 * a + 1] * Sg[3 + b] + T[3 * a + 2] * Sg[6 + b];
    const double ca = (double)(TS[0] * T[0] + TS[1] * T[1] + TS[2] * T[2]) + (double)kLowPass;
    const double cb = (double)(TS[0] * T[3] + TS[1] * T[4] + TS[2] * T[5]);
    const double cc = (double)(TS[3] * T[3] + TS[4] * T[4] + TS[5] * T[5]) + (double)kLowPass;
    // ---- conic (A, B, C) -> covariance (a, b, c)
    const double D = ca * cc - cb * cb;
    const double iD2 = 1.0 / (D * D);
    const float ga = (float)((-cc * cc * gA + cb * cc * gB - cb * cb * gC) * iD2);
    const float gb = (float)((2.0 * cb * cc * gA - (ca * cc + cb * cb) * gB + 2.0 * ca * cb * gC) * iD2);
    const float gcv = (float)((-cb * cb * gA + ca * cb * gB - ca * ca * gC) * iD2);
    const float G2[4] = {ga, 0.5f * gb, 0.5f * gb, gcv};
    // gSigma = T^T G2 T (3x3), gT = 2 G2 T Sigma (2x3)
    float gS[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            gS[3 * a + b] = T[a] * (G2[0] * T[b] + G2[1] * T[3 + b]) + T[3 + a] * (G2[2] * T[b] + G2[3] * T[3 + b]);
    float gT[6];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            gT[3 * a + b] = 2.f * (G2[2 * a] * TS[b] + G2[2 * a + 1] * TS[3 + b]);
    // T = J W: gJ = gT W^T, gW += J^T gT
    float gJ[6];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            gJ[3 * a + b] = gT[3 * a] * W[3 * b] + gT[3 * a + 1] * W[3 * b + 1] + gT[3 * a + 2] * W[3 * b + 2];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) gW[3 * a + b] += J[a] * gT[b] + J[3 + a] * gT[3 + b];
    // J entries -> camera-space mean
    float gp[3] = {0.f, 0.f, 0.f};
    const float iz2 = iz * iz;
    gp[2] += -cam.fx * iz2 * gJ[0] - cam.fy * iz2 * gJ[4];
    const float grxc = -cam.fx * iz * gJ[2];
    const float gryc = -cam.fy * iz * gJ[5];
    gp[2] += cam.fx * rxc * iz2 * gJ[2] + cam.fy * ryc * iz2 * gJ[5];
    if (rx >= -cam.limx && rx <= cam.limx) {
        gp[0] += grxc * iz;
        gp[2] -= grxc * p[0] * iz2;
    }
    if (ry >= -cam.limy && ry <= cam.limy) {
        gp[1] += gryc * iz;
        gp[2] -= gryc * p[1] * iz2;
    }
    // centre (u, v)
    gp[0] += gu * cam.fx * iz;
    gp[1] += gv * cam.fy * iz;
    gp[2] -= (gu * cam.fx * p[0] + gv * cam.fy * p[1]) * iz2;
    // p = W mu + t
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        gmu[a] += W[a] * gp[0] + W[3 + a] * gp[1] + W[6 + a] * gp[2];
        gt[a] += gp[a];
#pragma unroll
        for (int b = 0; b < 3; ++b) gW[3 * a + b] += gp[a] * mu[b];
    }
    // Sigma = M M^T, M = R diag(s): gM = 2 gSigma M
    float gR[9];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        float gsb = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float gM = 2.f * (gS[3 * a] * M[b] + gS[3 * a + 1] * M[3 + b] + gS[3 * a + 2] * M[6 + b]);
            gR[3 * a + b] = gM * sc[b];
            gsb += gM * R[3 * a + b];
        }
        gls[b] += gsb * sc[b];
    }
    // R(q_hat) -> q_hat
    const float w = q[0], x = q[1], y = q[2], z = q[3];
    float gqh[4];
    gqh[0] = 2.f * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
    gqh[1] = 2.f * (y * gR[1] + z * gR[2] + y * gR[3] - w * gR[5] + z * gR[6] + w * gR[7]) -
             4.f * x * (gR[4] + gR[8]);
    gqh[2] = 2.f * (x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] + z * gR[7]) -
             4.f * y * (gR[0] + gR[8]);
    gqh[3] = 2.f * (-w * gR[1] + x * gR[2] + w * gR[3] + y * gR[5] + x * gR[6] + y * gR[7]) -
             4.f * z * (gR[0] + gR[4]);
    const float qd = gqh[0] * q[0] + gqh[1] * q[1] + gqh[2] * q[2] + gqh[3] * q[3];
#pragma unroll
    for (int k = 0; k < 4; ++k) gq[k] += (gqh[k] - q[k] * qd) / qn;
}

// Per-block partial of one view's pose gradient (every thread of the block
// takes part): wave sums, then the four waves in a fixed order; layout
// [view][entry of the 3x4 block][workgroup].
__device__ __forceinline__ void pose_block_partial(const float (&gW)[9], const float (&gt)[3], float *red,
                                                   float *__restrict__ pose_part, int v, uint32_t pose_blocks) {
    float pv[12];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        pv[4 * r] = gW[3 * r];
        pv[4 * r + 1] = gW[3 * r + 1];
        pv[4 * r + 2] = gW[3 * r + 2];
        pv[4 * r + 3] = gt[r];
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) pv[k] = wave_sum(pv[k]);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) red[wv * 12 + k] = pv[k];
    }
    __syncthreads();
    if (threadIdx.x < 12) {
        const int k = threadIdx.x;
        pose_part[((size_t)v * 12 + k) * pose_blocks + blockIdx.x] = (red[k] + red[12 + k]) + (red[24 + k] + red[36 + k]);
    }
    __syncthreads();
}

template <int DEG>
__global__ __launch_bounds__(kProjThreads) void k_project_bwd(
    gsr_gaussians g, ViewTable vt, const float *__restrict__ w2c, uint64_t n, const Rec *__restrict__ rec,
    const uint32_t *__restrict__ count, const WsHeader *__restrict__ hdr, const float4 *__restrict__ screen,
    const float *__restrict__ carry, gsr_gaussian_grads gr, float *__restrict__ pose_part, uint32_t pose_blocks,
    int zero_unseen) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr bool kVecSH = (3 * K) % 4 == 0;  // SH rows of 16-byte multiples: float4 loads and stores
    __shared__ float red[4 * 12];
    __shared__ uint32_t s_list[kProjThreads];  // block-local indices of the Gaussians seen by some view
    __shared__ uint32_t s_wcnt[4];
    __shared__ uint8_t s_vis[kProjThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kProjThreads;
    const uint32_t nb = (uint32_t)min((uint64_t)kProjThreads, n - base);
    // after a pair overflow no pair gradient exists: every Gaussian gets zero
    const bool ovf = hdr->overflow != 0u;

    // ---- the block's Gaussians that some view sees, compacted so that the
    // chain rule below runs on full waves (most Gaussians are off-screen)
    {
        bool vis = false;
        if (!ovf && threadIdx.x < nb)
            for (int v = 0; v < vt.n_views; ++v) vis |= count[(uint64_t)v * n + base + threadIdx.x] > 0u;
        const unsigned long long bal = __ballot(vis);
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        if (lane == 0) s_wcnt[wv] = (uint32_t)__popcll(bal);
        s_vis[threadIdx.x] = vis ? 1 : 0;
        __syncthreads();
        uint32_t off = 0;
        for (int w = 0; w < wv; ++w) off += s_wcnt[w];
        if (vis) s_list[off + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull))] = threadIdx.x;
        __syncthreads();
    }
    const uint32_t nlist = s_wcnt[0] + s_wcnt[1] + s_wcnt[2] + s_wcnt[3];
    // ---- zero rows of the others, block-wide and coalesced (unless the backward
    // compositing already did)
    if (zero_unseen) {
        float *zm = gr.means + 3 * base, *zl = gr.log_scales + 3 * base;
        for (uint32_t f = threadIdx.x; f < 3 * nb; f += kProjThreads)
            if (!s_vis[f / 3]) zm[f] = 0.f, zl[f] = 0.f;
        for (uint32_t f = threadIdx.x; f < nb; f += kProjThreads)
            if (!s_vis[f]) {
                reinterpret_cast<float4 *>(gr.quats)[base + f] = make_float4(0.f, 0.f, 0.f, 0.f);
                gr.opacities[base + f] = 0.f;
            }
        if constexpr (kVecSH) {
            constexpr uint32_t R4 = 3 * K / 4;  // float4 per SH row
            float4 *zs = reinterpret_cast<float4 *>(gr.sh) + base * R4;
            for (uint32_t f = threadIdx.x; f < R4 * nb; f += kProjThreads)
                if (!s_vis[f / R4]) zs[f] = make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
            float *zs = gr.sh + base * 3 * K;
            for (uint32_t f = threadIdx.x; f < 3 * K * nb; f += kProjThreads)
                if (!s_vis[f / (3 * K)]) zs[f] = 0.f;
        }
    }
    const bool live = threadIdx.x < nlist;
    const uint64_t i = base + (live ? s_list[threadIdx.x] : 0u);

    float gmu[3] = {0, 0, 0}, gls[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gop = 0.f;
    bool sh_written = false;  // SH gradient rows are stored by the first visible view, added to by later ones
    float *gsh = gr.sh + (size_t)i * K * 3;

    for (int v = 0; v < vt.n_views; ++v) {
        float gW[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, gt[3] = {0, 0, 0};
        const uint64_t item = (uint64_t)v * n + i;
        const uint32_t cnt = live ? count[item] : 0u;
        if (cnt > 0)
            item_backward<DEG>(g, vt.v[v], w2c, v, i, item, cnt, rec, screen, carry, g.sh + (size_t)i * K * 3, gsh,
                               sh_written, gmu, gls, gq, gop, gW, gt);
        pose_block_partial(gW, gt, red, pose_part, v, pose_blocks);
    }
    if (!live) return;  // its rows were zeroed above (or it is one of the zeroed ones)
    gr.means[3 * i] = gmu[0];
    gr.means[3 * i + 1] = gmu[1];
    gr.means[3 * i + 2] = gmu[2];
    gr.log_scales[3 * i] = gls[0];
    gr.log_scales[3 * i + 1] = gls[1];
    gr.log_scales[3 * i + 2] = gls[2];
    reinterpret_cast<float4 *>(gr.quats)[i] = make_float4(gq[0], gq[1], gq[2], gq[3]);
    gr.opacities[i] = gop;
}

// The same for one view, over its segment of the visible-item list instead of
// over all Gaussians: every thread of a block has a seen Gaussian (the list is
// dense), where the per-block compaction above leaves two of every three
// threads idle when a third of the Gaussians is seen.  Several views run one
// launch each, in view order: a Gaussian's gradient rows are stored by the
// first view that sees it and added to by the later ones (the order of the
// sums above), and rows no view sees were zeroed by the backward compositing.
// seg (several views): first visible index of each view, and the total.
template <int DEG>
__global__ __launch_bounds__(kProjThreads) void k_project_bwd_vis(
    gsr_gaussians g, ViewTable vt, const float *__restrict__ w2c, uint64_t n, int v, const uint32_t *__restrict__ seg,
    const uint32_t *__restrict__ vis, const Rec *__restrict__ rec, const uint32_t *__restrict__ count,
    const WsHeader *__restrict__ hdr, const float4 *__restrict__ screen, const float *__restrict__ carry,
    gsr_gaussian_grads gr, float *__restrict__ pose_part, uint32_t pose_blocks) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr bool kVec = (3 * K) % 4 == 0;
    constexpr int kUnit = kVec ? 4 : 1;              // floats per cooperative access
    constexpr int kUnits = 3 * K / kUnit;            // accesses per SH row
    constexpr int kStride = kVec ? 3 * K + 4 : 3 * K;  // LDS row stride in floats (16-B aligned when vectorised)
    __shared__ float red[4 * 12];
    __shared__ __align__(16) float s_sh[4][64 * kStride];
    const uint32_t nvis = hdr->overflow ? 0u : hdr->n_visible;
    const uint32_t lo = seg ? min(seg[v], nvis) : 0u, hi = seg ? min(seg[v + 1], nvis) : nvis;
    if (lo + blockIdx.x * kProjThreads >= hi) {  // uniform: no item, a zero partial
        if (threadIdx.x < 12) pose_part[((size_t)v * 12 + threadIdx.x) * pose_blocks + blockIdx.x] = 0.f;
        return;
    }
    const uint32_t k = lo + blockIdx.x * kProjThreads + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t wave_first = lo + blockIdx.x * kProjThreads + (uint32_t)wave * 64;
    const bool live = k < hi;
    const uint64_t item = live ? vis[k] : (uint64_t)v * n;
    const uint64_t i = item - (uint64_t)v * n;  // the Gaussian
    // stored by this view (no earlier view saw the Gaussian) or added to
    bool first = true;
    for (int u = 0; u < v && live; ++u) first &= count[(uint64_t)u * n + i] == 0u;
    float *rows = s_sh[wave];
    // the wave's SH rows, staged through LDS with row-contiguous (coalesced)
    // accesses instead of one 3K-float row per lane
#pragma unroll 4
    for (int u = lane; u < 64 * kUnits; u += 64) {
        const int r = u / kUnits, c = u - r * kUnits;
        const uint64_t ir = (uint64_t)__shfl((long long)i, r, 64);
        if (wave_first + (uint32_t)r < hi) {
            if constexpr (kVec)
                *reinterpret_cast<float4 *>(rows + r * kStride + 4 * c) =
                    reinterpret_cast<const float4 *>(g.sh)[ir * kUnits + c];
            else
                rows[r * kStride + c] = g.sh[ir * kUnits + c];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    float gW[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, gt[3] = {0, 0, 0};
    if (live) {
        float gmu[3] = {0, 0, 0}, gls[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gop = 0.f;
        bool sh_written = false;
        float *row = rows + lane * kStride;  // read, then overwritten with this view's SH gradient
        item_backward<DEG>(g, vt.v[v], w2c, v, i, item, count[item], rec, screen, carry, row, row, sh_written, gmu,
                           gls, gq, gop, gW, gt);
        if (!first) {
#pragma unroll
            for (int c = 0; c < 3; ++c) gmu[c] += gr.means[3 * i + c], gls[c] += gr.log_scales[3 * i + c];
            const float4 q = reinterpret_cast<const float4 *>(gr.quats)[i];
            gq[0] += q.x, gq[1] += q.y, gq[2] += q.z, gq[3] += q.w;
            gop += gr.opacities[i];
        }
        gr.means[3 * i] = gmu[0];
        gr.means[3 * i + 1] = gmu[1];
        gr.means[3 * i + 2] = gmu[2];
        gr.log_scales[3 * i] = gls[0];
        gr.log_scales[3 * i + 1] = gls[1];
        gr.log_scales[3 * i + 2] = gls[2];
        reinterpret_cast<float4 *>(gr.quats)[i] = make_float4(gq[0], gq[1], gq[2], gq[3]);
        gr.opacities[i] = gop;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll 4
    for (int u = lane; u < 64 * kUnits; u += 64) {
        const int r = u / kUnits, c = u - r * kUnits;
        const uint64_t ir = (uint64_t)__shfl((long long)i, r, 64);
        const bool add = __shfl((int)!first, r, 64) != 0;
        if (wave_first + (uint32_t)r < hi) {
            if constexpr (kVec) {
                float4 o = *reinterpret_cast<const float4 *>(rows + r * kStride + 4 * c);
                float4 *dst = reinterpret_cast<float4 *>(gr.sh) + ir * kUnits + c;
                if (add) {
                    const float4 e = *dst;
                    o.x += e.x, o.y += e.y, o.z += e.z, o.w += e.w;
                }
                *dst = o;
            } else {
                float o = rows[r * kStride + c];
                if (add) o += gr.sh[ir * kUnits + c];
                gr.sh[ir * kUnits + c] = o;
            }
        }
    }
    pose_block_partial(gW, gt, red, pose_part, v, pose_blocks);
}

// First visible index of each view (the list is in ascending item order and
// item = view * n + Gaussian), and the visible count at index n_views; one
// thread per entry.
static_assert(GSR_MAX_VIEWS < 64, "one wave computes the view segments");
__global__ void k_view_segments(const uint32_t *__restrict__ vis, uint64_t n, int n_views,
                                const WsHeader *__restrict__ hdr, uint32_t *__restrict__ seg) {
    const int v = threadIdx.x;
    if (v > n_views) return;
    const uint32_t nvis = hdr->overflow ? 0u : hdr->n_visible;
    const uint64_t key = (uint64_t)v * n;
    uint32_t a = 0, b = nvis;  // first index whose item is >= key
    while (a < b) {
        const uint32_t mid = (a + b) >> 1;
        if ((uint64_t)vis[mid] < key)
            a = mid + 1;
        else
            b = mid;
    }
    seg[v] = a;
}

void launch_project_bwd(const gsr_gaussians &g, const ViewTable &vt, const float *w2c, uint64_t n, const Rec *rec,
                        const uint32_t *count, const uint32_t *vis, const WsHeader *hdr, const float4 *screen,
                        const float *carry, const gsr_gaussian_grads &gr, float *pose_part, uint32_t pose_blocks,
                        uint32_t *seg, bool zero_unseen, hipStream_t st) {
    if (n == 0) return;
    const dim3 grid(pose_blocks);
    const int z = zero_unseen ? 1 : 0;
    if (!zero_unseen) {
        // one dense launch per view, in view order
        if (vt.n_views > 1)
            hipLaunchKernelGGL(k_view_segments, dim3(1), dim3(64), 0, st, vis, n, vt.n_views, hdr, seg);
        const uint32_t *sg = vt.n_views > 1 ? seg : nullptr;
        for (int v = 0; v < vt.n_views; ++v) {
            switch (g.sh_degree) {
                case 0: hipLaunchKernelGGL(k_project_bwd_vis<0>, grid, dim3(kProjThreads), 0, st, g, vt, w2c, n, v, sg, vis, rec, count, hdr, screen, carry, gr, pose_part, pose_blocks); break;
                case 1: hipLaunchKernelGGL(k_project_bwd_vis<1>, grid, dim3(kProjThreads), 0, st, g, vt, w2c, n, v, sg, vis, rec, count, hdr, screen, carry, gr, pose_part, pose_blocks); break;
                case 2: hipLaunchKernelGGL(k_project_bwd_vis<2>, grid, dim3(kProjThreads), 0, st, g, vt, w2c, n, v, sg, vis, rec, count, hdr, screen, carry, gr, pose_part, pose_blocks); break;
                default: hipLaunchKernelGGL(k_project_bwd_vis<3>, grid, dim3(kProjThreads), 0, st, g, vt, w2c, n, v, sg, vis, rec, count, hdr, screen, carry, gr, pose_part, pose_blocks); break;
            }
        }
        return;
    }
    switch (g.sh_degree) {
        case 0: hipLaunchKernelGGL(k_project_bwd<0>, grid, dim3(kProjThreads), 0, st, g, vt, w2c, n, rec, count, hdr, screen, carry, gr, pose_part, pose_blocks, z); break;
        case 1: hipLaunchKernelGGL(k_project_bwd<1>, grid, dim3(kProjThreads), 0, st, g, vt, w2c, n, rec, count, hdr, screen, carry, gr, pose_part, pose_blocks, z); break;
        case 2: hipLaunchKernelGGL(k_project_bwd<2>, grid, dim3(kProjThreads), 0, st, g, vt, w2c, n, rec, count, hdr, screen, carry, gr, pose_part, pose_blocks, z); break;
        default: hipLaunchKernelGGL(k_project_bwd<3>, grid, dim3(kProjThreads), 0, st, g, vt, w2c, n, rec, count, hdr, screen, carry, gr, pose_part, pose_blocks, z); break;
    }
}

// ---------------------------------------------------------------------------
// Pose gradient: one workgroup per view sums the per-block partials in a fixed
// order, writes the 4x4 gradient (last row zero) and the left-perturbation
// twist: M = G T^T, d/drho = M[0:3, 3], d/dphi = (M21 - M12, M02 - M20, M10 - M01).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(768) void k_pose_finalize(const float *__restrict__ w2c,
                                                       const float *__restrict__ pose_part, uint32_t pose_blocks,
                                                       const WsHeader *__restrict__ hdr,
                                                       const uint32_t *__restrict__ seg, int dense,
                                                       float *__restrict__ dL_dw2c, float *__restrict__ dL_dtwist) {
    // one workgroup per view, one wave per entry of the top 3x4 block
    __shared__ float G[16];
    const int v = blockIdx.x;
    const int k = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // the dense backward's grid is sized by capacity: only the blocks that had
    // items of this view's segment wrote a nonzero partial
    uint32_t used = pose_blocks;
    if (dense) {
        const uint32_t nvis = hdr->overflow ? 0u : hdr->n_visible;
        const uint32_t lo = seg ? min(seg[v], nvis) : 0u, hi = seg ? min(seg[v + 1], nvis) : nvis;
        used = min(pose_blocks, (hi - lo + (uint32_t)kProjThreads - 1u) / (uint32_t)kProjThreads);
    }
    const float *src = pose_part + ((size_t)v * 12 + k) * pose_blocks;
    float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, acc3 = 0.f;  // independent loads in flight
    uint32_t b = lane;
    for (; b + 192 < used; b += 256) {
        acc0 += src[b];
        acc1 += src[b + 64];
        acc2 += src[b + 128];
        acc3 += src[b + 192];
    }
    for (; b < used; b += 64) acc0 += src[b];
    const float acc = wave_sum((acc0 + acc1) + (acc2 + acc3));
    if (lane == 0) G[k] = acc;
    if (threadIdx.x == 0) G[12] = G[13] = G[14] = G[15] = 0.f;
    __syncthreads();
    if (threadIdx.x < 16 && dL_dw2c) dL_dw2c[16 * v + threadIdx.x] = G[threadIdx.x];
    if (threadIdx.x == 0 && dL_dtwist) {
        const float *T = w2c + 16 * v;
        float M[16];
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                M[4 * a + b] = G[4 * a] * T[4 * b] + G[4 * a + 1] * T[4 * b + 1] + G[4 * a + 2] * T[4 * b + 2] +
                               G[4 * a + 3] * T[4 * b + 3];
        float *o = dL_dtwist + 6 * v;
        o[0] = M[3];
        o[1] = M[7];
        o[2] = M[11];
        o[3] = M[9] - M[6];
        o[4] = M[2] - M[8];
        o[5] = M[4] - M[1];
    }
}

void launch_pose_finalize(const ViewTable &vt, const float *w2c, const float *pose_part, uint32_t pose_blocks,
                          const WsHeader *hdr, const uint32_t *seg, bool dense, float *dL_dw2c, float *dL_dtwist,
                          hipStream_t st) {
    if (!dL_dw2c && !dL_dtwist) return;
    hipLaunchKernelGGL(k_pose_finalize, dim3(vt.n_views), dim3(768), 0, st, w2c, pose_part, pose_blocks, hdr,
                       vt.n_views > 1 ? seg : nullptr, dense ? 1 : 0, dL_dw2c, dL_dtwist);
}

}  // namespace gsr
