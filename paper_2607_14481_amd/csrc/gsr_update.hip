// gsr_update.hip -- parameter updates around the rasterizer on gfx950:
//   * the fused Adam step of the joint optimisation over the five Gaussian
//     arrays (optionally only for the Gaussians the last forward saw),
//   * the pose step: Adam on each view's 6-DoF twist, then the SE(3)
//     retraction of its world-to-camera transform,
//   * the loop-closure Sim(3) relocation of Gaussians (or hierarchy nodes).
// The first and last are elementwise and HBM-bound: every array is walked as
// one flat sequence of float4 (or float) units, so loads and stores are
// coalesced whatever the row length of an array.
#include "gsr_internal.h"

namespace gsr {

constexpr float kOpacityLo = 1e-7f, kOpacityHi = 1.f - 1e-7f;

// Did some view of the last forward see Gaussian i?  (count = tiles touched)
__device__ __forceinline__ bool seen(const uint32_t *__restrict__ count, uint64_t n, int n_views, uint64_t i) {
    bool s = false;
    for (int v = 0; v < n_views; ++v) s |= count[(uint64_t)v * n + i] > 0u;
    return s;
}

__device__ __forceinline__ void adam_elem(float &p, float g, float &m, float &v, const AdamScalars &a, float step_size) {
    m = fmaf(a.b1, m, a.one_m_b1 * g);
    v = fmaf(a.b2, v, a.one_m_b2 * g * g);
    const float denom = fmaf(sqrtf(v), a.inv_sqrt_bc2, a.eps);
    p -= step_size * (m / denom);
}

// One array of the parameter set, as flat float (W = 1) or float4 (W = 4) units.
template <int W>
__device__ __forceinline__ void adam_units(float *p, const float *g, float *m, float *v, uint64_t unit,
                                           const AdamScalars &a, float step_size) {
    if constexpr (W == 4) {
        float4 P = reinterpret_cast<float4 *>(p)[unit], G = reinterpret_cast<const float4 *>(g)[unit];
        float4 M = reinterpret_cast<float4 *>(m)[unit], V = reinterpret_cast<float4 *>(v)[unit];
        adam_elem(P.x, G.x, M.x, V.x, a, step_size);
        adam_elem(P.y, G.y, M.y, V.y, a, step_size);
        adam_elem(P.z, G.z, M.z, V.z, a, step_size);
        adam_elem(P.w, G.w, M.w, V.w, a, step_size);
        reinterpret_cast<float4 *>(p)[unit] = P;
        reinterpret_cast<float4 *>(m)[unit] = M;
        reinterpret_cast<float4 *>(v)[unit] = V;
    } else {
        float P = p[unit], M = m[unit], V = v[unit];
        adam_elem(P, g[unit], M, V, a, step_size);
        p[unit] = P;
        m[unit] = M;
        v[unit] = V;
    }
}

// Segments of the flat walk: means (3n floats), log-scales (3n floats),
// quaternions (n float4), opacities (n floats, on the logit), SH (n 3K/4
// float4 when 3K is a multiple of 4, else n 3K floats).
template <bool VEC_SH>
__global__ __launch_bounds__(256) void k_adam_step(AdamArgs A) {
    const uint64_t n = A.n;
    const uint64_t K3 = 3ull * (uint64_t)A.sh_k;
    const uint64_t s0 = 3 * n, s1 = s0 + 3 * n, s2 = s1 + n, s3 = s2 + n;
    const uint64_t sh_units = VEC_SH ? n * K3 / 4 : n * K3;
    const uint64_t total = s3 + sh_units;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < total; u += stride) {
        uint64_t gi;  // Gaussian of this unit
        if (u < s0) gi = u / 3;
        else if (u < s1) gi = (u - s0) / 3;
        else if (u < s2) gi = u - s1;
        else if (u < s3) gi = u - s2;
        else gi = VEC_SH ? (u - s3) * 4 / K3 : (u - s3) / K3;
        if (A.count && !seen(A.count, n, A.n_views, gi)) continue;
        if (u < s0) {
            adam_units<1>(A.p.means, A.g.means, A.m.means, A.v.means, u, A.a, A.step_size[0]);
        } else if (u < s1) {
            adam_units<1>(A.p.log_scales, A.g.log_scales, A.m.log_scales, A.v.log_scales, u - s0, A.a,
                          A.step_size[1]);
        } else if (u < s2) {
            adam_units<4>(A.p.quats, A.g.quats, A.m.quats, A.v.quats, u - s1, A.a, A.step_size[2]);
        } else if (u < s3) {
            // opacity: the step is on l = ln(o / (1 - o)), with dL/dl = o (1 - o) dL/do
            const uint64_t i = u - s2;
            const float o = fminf(fmaxf(A.p.opacities[i], kOpacityLo), kOpacityHi);
            float l = logf(o) - log1pf(-o);
            float m = A.m.opacities[i], v = A.v.opacities[i];
            adam_elem(l, o * (1.f - o) * A.g.opacities[i], m, v, A.a, A.step_size[3]);
            A.p.opacities[i] = 1.f / (1.f + expf(-l));
            A.m.opacities[i] = m;
            A.v.opacities[i] = v;
        } else if constexpr (VEC_SH) {
            const uint64_t w = u - s3;
            // a row is a whole number of units, but its first unit holds the three
            // DC floats and one float of k = 1: the rate is chosen per float
            const uint64_t e0 = w * 4;
            float4 P = reinterpret_cast<float4 *>(A.p.sh)[w], G = reinterpret_cast<const float4 *>(A.g.sh)[w];
            float4 M = reinterpret_cast<float4 *>(A.m.sh)[w], V = reinterpret_cast<float4 *>(A.v.sh)[w];
            float *pp = &P.x, *gg = &G.x, *mm = &M.x, *vv = &V.x;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const bool dc = (e0 + c) % K3 < 3;
                adam_elem(pp[c], gg[c], mm[c], vv[c], A.a, dc ? A.step_size[4] : A.step_size[5]);
            }
            reinterpret_cast<float4 *>(A.p.sh)[w] = P;
            reinterpret_cast<float4 *>(A.m.sh)[w] = M;
            reinterpret_cast<float4 *>(A.v.sh)[w] = V;
        } else {
            const uint64_t e = u - s3;
            const bool dc = e % K3 < 3;
            adam_units<1>(A.p.sh, A.g.sh, A.m.sh, A.v.sh, e, A.a, dc ? A.step_size[4] : A.step_size[5]);
        }
    }
}

void launch_adam_step(const AdamArgs &A, hipStream_t st) {
    if (A.n == 0) return;
    const uint64_t K3 = 3ull * (uint64_t)A.sh_k;
    const bool vec = K3 % 4 == 0;
    const uint64_t total = 8 * A.n + (vec ? A.n * K3 / 4 : A.n * K3);
    uint64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (vec)
        hipLaunchKernelGGL(k_adam_step<true>, dim3((unsigned)blocks), dim3(256), 0, st, A);
    else
        hipLaunchKernelGGL(k_adam_step<false>, dim3((unsigned)blocks), dim3(256), 0, st, A);
}

// ---------------------------------------------------------------------------
// Pose step: one thread per view.  xi = -lr m_hat / (sqrt(v_hat) + eps), then
// T <- exp(xi^) T with the closed-form SE(3) exponential: for phi = xi[3:6],
// theta = |phi|, R = I + a [phi]x + b [phi]x^2 and t = (I + b [phi]x + c [phi]x^2) rho
// with a = sin(theta)/theta, b = (1 - cos(theta))/theta^2,
// c = (theta - sin(theta))/theta^3 (series near theta = 0).
// ---------------------------------------------------------------------------
__global__ void k_pose_step(float *__restrict__ w2c, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, int n_views, AdamScalars a, float step_size) {
    const int k = threadIdx.x;
    if (k >= n_views) return;
    double xi[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        float p = 0.f, mj = m[6 * k + j], vj = v[6 * k + j];
        adam_elem(p, g[6 * k + j], mj, vj, a, step_size);
        m[6 * k + j] = mj;
        v[6 * k + j] = vj;
        xi[j] = (double)p;
    }
    const double px = xi[3], py = xi[4], pz = xi[5];
    const double th2 = px * px + py * py + pz * pz, th = sqrt(th2);
    double ca, cb, cc;
    if (th < 1e-4) {
        ca = 1.0 - th2 / 6.0;
        cb = 0.5 - th2 / 24.0;
        cc = 1.0 / 6.0 - th2 / 120.0;
    } else {
        ca = sin(th) / th;
        cb = (1.0 - cos(th)) / th2;
        cc = (th - sin(th)) / (th2 * th);
    }
    const double W[9] = {0, -pz, py, pz, 0, -px, -py, px, 0};
    double W2[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) W2[3 * r + c] = W[3 * r] * W[c] + W[3 * r + 1] * W[3 + c] + W[3 * r + 2] * W[6 + c];
    double E[16];
    for (int r = 0; r < 3; ++r) {
        double t = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double id = r == c ? 1.0 : 0.0;
            E[4 * r + c] = id + ca * W[3 * r + c] + cb * W2[3 * r + c];
            t += (id + cb * W[3 * r + c] + cc * W2[3 * r + c]) * xi[c];
        }
        E[4 * r + 3] = t;
    }
    E[12] = E[13] = E[14] = 0.0;
    E[15] = 1.0;
    float *T = w2c + 16 * k;
    double Tin[16];
    for (int j = 0; j < 16; ++j) Tin[j] = (double)T[j];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double s = 0.0;
            for (int j = 0; j < 4; ++j) s += E[4 * r + j] * Tin[4 * j + c];
            T[4 * r + c] = (float)s;
        }
}

void launch_pose_step(float *w2c, const float *g, float *m, float *v, int n_views, const AdamScalars &a,
                      float step_size, hipStream_t st) {
    hipLaunchKernelGGL(k_pose_step, dim3(1), dim3(64), 0, st, w2c, g, m, v, n_views, a, step_size);
}

// ---------------------------------------------------------------------------
// Sim(3) relocation: one thread per Gaussian.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sim3_relocate(float *__restrict__ means, float *__restrict__ quats,
                                                       float *__restrict__ log_scales, uint64_t n,
                                                       const int32_t *__restrict__ keyframe_of,
                                                       const float *__restrict__ sim3, int32_t n_keyframes) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int32_t k = keyframe_of[i];
    if (k < 0 || k >= n_keyframes) return;
    const float *S = sim3 + 8 * (size_t)k;
    const float s = S[0], qw = S[1], qx = S[2], qy = S[3], qz = S[4];
    // R(q) of the unit quaternion (w, x, y, z)
    const float R[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy),
                        2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                        2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)};
    const float mx = means[3 * i], my = means[3 * i + 1], mz = means[3 * i + 2];
    means[3 * i] = fmaf(s, R[0] * mx + R[1] * my + R[2] * mz, S[5]);
    means[3 * i + 1] = fmaf(s, R[3] * mx + R[4] * my + R[5] * mz, S[6]);
    means[3 * i + 2] = fmaf(s, R[6] * mx + R[7] * my + R[8] * mz, S[7]);
    const float4 g = reinterpret_cast<const float4 *>(quats)[i];  // (w, x, y, z)
    reinterpret_cast<float4 *>(quats)[i] =
        make_float4(qw * g.x - qx * g.y - qy * g.z - qz * g.w, qw * g.y + qx * g.x + qy * g.w - qz * g.z,
                    qw * g.z - qx * g.w + qy * g.x + qz * g.y, qw * g.w + qx * g.z - qy * g.y + qz * g.x);
    const float ls = logf(s);
    log_scales[3 * i] += ls;
    log_scales[3 * i + 1] += ls;
    log_scales[3 * i + 2] += ls;
}

void launch_sim3_relocate(float *means, float *quats, float *log_scales, uint64_t n, const int32_t *keyframe_of,
                          const float *sim3, int32_t n_keyframes, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_sim3_relocate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, means, quats,
                       log_scales, n, keyframe_of, sim3, n_keyframes);
}

}  // namespace gsr
