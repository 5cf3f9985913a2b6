// gsr_hierarchy.hip -- per-view level-of-detail cut of a Gaussian hierarchy
// and the gather of the cut's rows, on gfx950.
//
// Rendering a hierarchy starts from its roots and descends until a node is
// finer than a screen-size threshold or is a leaf (Sec. 7.2); with the screen
// size S = f * (largest axis scale) / (distance to the camera centre), a node
// is in the cut exactly when it does not descend (it is a leaf or S < tau)
// while every one of its ancestors does.  That makes the cut a per-node test:
// one kernel marks the nodes that descend, a second one walks each node's
// ancestor chain (a few levels), and an ordered compaction lists the cut in
// ascending node order.  S is evaluated in double precision so that the
// decision agrees with the FP64 reference away from ties.
#include "gsr_internal.h"

namespace gsr {

constexpr int kMaxDepth = 64;  // longer ancestor chains (or cycles) are cut off

__global__ __launch_bounds__(256) void k_cut_descend(const float *__restrict__ means,
                                                     const float *__restrict__ log_scales,
                                                     const int32_t *__restrict__ child_count, uint64_t n,
                                                     const float *__restrict__ w2c, double focal, double tau,
                                                     uint8_t *__restrict__ descend) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    if (child_count[i] <= 0) {
        descend[i] = 0;
        return;
    }
    // camera centre c = -R^T t of the row-major world-to-camera transform
    double c[3];
    for (int a = 0; a < 3; ++a)
        c[a] = -((double)w2c[a] * w2c[3] + (double)w2c[4 + a] * w2c[7] + (double)w2c[8 + a] * w2c[11]);
    const double dx = (double)means[3 * i] - c[0], dy = (double)means[3 * i + 1] - c[1],
                 dz = (double)means[3 * i + 2] - c[2];
    const double dist = fmax(sqrt(dx * dx + dy * dy + dz * dz), 1e-9);
    const float lmax = fmaxf(fmaxf(log_scales[3 * i], log_scales[3 * i + 1]), log_scales[3 * i + 2]);
    const double s = focal * exp((double)lmax) / dist;
    descend[i] = s >= tau ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_cut_select(const int32_t *__restrict__ parent, uint64_t n,
                                                    const uint8_t *__restrict__ descend, uint8_t *__restrict__ in_cut) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    bool in = descend[i] == 0;
    int64_t a = parent[i];
    for (int hop = 0; in && a >= 0 && (uint64_t)a < n; ++hop) {
        if (hop == kMaxDepth || !descend[a]) {
            in = false;
            break;
        }
        a = parent[a];
    }
    in_cut[i] = in ? 1 : 0;
}

void launch_hierarchy_cut_flags(const float *means, const float *log_scales, const int32_t *parent,
                                const int32_t *child_count, uint64_t n, const float *w2c, float focal, float tau,
                                uint8_t *descend, uint8_t *in_cut, hipStream_t st) {
    if (n == 0) return;
    const dim3 grid((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(k_cut_descend, grid, dim3(256), 0, st, means, log_scales, child_count, n, w2c, (double)focal,
                       (double)tau, descend);
    hipLaunchKernelGGL(k_cut_select, grid, dim3(256), 0, st, parent, n, descend, in_cut);
}

// Row gather as one flat walk over output units (consecutive lanes copy
// consecutive units, so stores are coalesced and, for the ascending runs a cut
// mostly consists of, so are loads): means and log-scales as floats (3 per
// row), quaternions as float4, opacities as floats, SH as float4 when a row is
// a multiple of 16 bytes, else as floats.
template <int K>
__global__ __launch_bounds__(256) void k_gather(gsr_gaussians src, const int32_t *__restrict__ index, uint64_t n_max,
                                                const int64_t *__restrict__ count, gsr_param_set dst) {
    const uint64_t n_out = count ? (uint64_t)min((int64_t)n_max, max(*count, (int64_t)0)) : n_max;
    constexpr bool kVec = (3 * K) % 4 == 0;
    constexpr uint64_t kShUnits = kVec ? 3 * K / 4 : 3 * K;  // SH units per row
    const uint64_t s0 = 3 * n_out, s1 = s0 + 3 * n_out, s2 = s1 + n_out, s3 = s2 + n_out;
    const uint64_t total = s3 + kShUnits * n_out;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < total; u += stride) {
        if (u < s0) {
            const uint64_t r = u / 3, c = u - 3 * r;
            dst.means[u] = src.means[3 * (uint64_t)index[r] + c];
        } else if (u < s1) {
            const uint64_t w = u - s0, r = w / 3, c = w - 3 * r;
            dst.log_scales[w] = src.log_scales[3 * (uint64_t)index[r] + c];
        } else if (u < s2) {
            const uint64_t r = u - s1;
            reinterpret_cast<float4 *>(dst.quats)[r] = reinterpret_cast<const float4 *>(src.quats)[index[r]];
        } else if (u < s3) {
            const uint64_t r = u - s2;
            dst.opacities[r] = src.opacities[index[r]];
        } else {
            const uint64_t w = u - s3, r = w / kShUnits, c = w - kShUnits * r;
            const uint64_t from = (uint64_t)index[r] * kShUnits + c;
            if constexpr (kVec)
                reinterpret_cast<float4 *>(dst.sh)[w] = reinterpret_cast<const float4 *>(src.sh)[from];
            else
                dst.sh[w] = src.sh[from];
        }
    }
}

void launch_gather_gaussians(const gsr_gaussians &src, const int32_t *index, uint64_t n_out, const int64_t *count,
                             const gsr_param_set &dst, hipStream_t st) {
    if (n_out == 0) return;
    const dim3 grid(4096);  // grid-stride walk
    switch (src.sh_degree) {
        case 0: hipLaunchKernelGGL(k_gather<1>, grid, dim3(256), 0, st, src, index, n_out, count, dst); break;
        case 1: hipLaunchKernelGGL(k_gather<4>, grid, dim3(256), 0, st, src, index, n_out, count, dst); break;
        case 2: hipLaunchKernelGGL(k_gather<9>, grid, dim3(256), 0, st, src, index, n_out, count, dst); break;
        default: hipLaunchKernelGGL(k_gather<16>, grid, dim3(256), 0, st, src, index, n_out, count, dst); break;
    }
}

// The cut's size as the device int64 that gathers and rasterizations read.
__global__ void k_store_count_i64(const uint32_t *__restrict__ count, int64_t *__restrict__ out) {
    if (threadIdx.x == 0) *out = count ? (int64_t)*count : 0;
}

void launch_store_count_i64(const uint32_t *count, int64_t *out, hipStream_t st) {
    hipLaunchKernelGGL(k_store_count_i64, dim3(1), dim3(64), 0, st, count, out);
}


// ---------------------------------------------------------------------------
// Hierarchy build (Sec. 7.1: groups of Gaussians merged into one node by a
// KL-divergence criterion).  Level l + 1 merges runs of `branching`
// consecutive level-l nodes; a parent is the single Gaussian that minimises
// KL(mixture || single) for the opacity-weighted mixture of its children,
// i.e. the mixture's mean and covariance:
//   w_i = o_i / sum o,  mu = sum w_i mu_i,
//   Sigma = sum w_i (Sigma_i + (mu_i - mu)(mu_i - mu)^T),
// with opacity 1 - prod (1 - o_i) and the w-weighted mean of the SH rows.
// The covariance is stored factored: eigenvalues ascending -> log-scales,
// eigenvectors (determinant +1) -> quaternion with w >= 0.
//
// k_merge_geometry: one thread per parent, FP64.  Moments are accumulated
// about the first child's mean, so the spread term does not cancel against
// the coordinates' magnitude (a street 2 km long).  The 3x3 eigenproblem is
// solved by cyclic Jacobi rotations (quadratic convergence; a sweep limit of
// 12 is never reached).  The thread also writes its node's child count and its
// children's parent index.  k_merge_sh: one thread per float4 (or float) of
// a parent's SH row, coalesced over consecutive parents.
// ---------------------------------------------------------------------------
constexpr double kMergeMinVar = 1e-12;

__device__ inline void quat_to_rot_d(double w, double x, double y, double z, double R[9]) {
    const double n = sqrt(w * w + x * x + y * y + z * z);
    w /= n, x /= n, y /= n, z /= n;
    R[0] = 1 - 2 * (y * y + z * z), R[1] = 2 * (x * y - w * z), R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z), R[4] = 1 - 2 * (x * x + z * z), R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y), R[7] = 2 * (y * z + w * x), R[8] = 1 - 2 * (x * x + y * y);
}

// Symmetric 3x3 eigendecomposition, a (row-major) overwritten; eigenvalues in
// lam (ascending), eigenvectors in the columns of V (determinant +1).
__device__ inline void sym3_eig(double a[9], double lam[3], double V[9]) {
    for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 12; ++sweep) {
        const double off = a[1] * a[1] + a[2] * a[2] + a[5] * a[5];
        const double dia = a[0] * a[0] + a[4] * a[4] + a[8] * a[8];
        if (!(off > 1e-34 * dia)) break;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int p = r == 2 ? 1 : 0, q = r == 0 ? 1 : 2;
            const double apq = a[3 * p + q];
            if (apq == 0.0) continue;
            const double theta = (a[3 * q + q] - a[3 * p + p]) / (2.0 * apq);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
            // A <- J^T A J with J the rotation in the (p, q) plane
            for (int k = 0; k < 3; ++k) {  // columns p, q
                const double akp = a[3 * k + p], akq = a[3 * k + q];
                a[3 * k + p] = c * akp - s * akq;
                a[3 * k + q] = s * akp + c * akq;
            }
            for (int k = 0; k < 3; ++k) {  // rows p, q
                const double apk = a[3 * p + k], aqk = a[3 * q + k];
                a[3 * p + k] = c * apk - s * aqk;
                a[3 * q + k] = s * apk + c * aqk;
            }
            a[3 * p + q] = a[3 * q + p] = 0.0;
            for (int k = 0; k < 3; ++k) {  // V <- V J
                const double vkp = V[3 * k + p], vkq = V[3 * k + q];
                V[3 * k + p] = c * vkp - s * vkq;
                V[3 * k + q] = s * vkp + c * vkq;
            }
        }
    }
    lam[0] = a[0], lam[1] = a[4], lam[2] = a[8];
    // ascending, columns along
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2 - i; ++j)
            if (lam[j] > lam[j + 1]) {
                const double tl = lam[j];
                lam[j] = lam[j + 1], lam[j + 1] = tl;
                for (int k = 0; k < 3; ++k) {
                    const double tv = V[3 * k + j];
                    V[3 * k + j] = V[3 * k + j + 1], V[3 * k + j + 1] = tv;
                }
            }
    const double det = V[0] * (V[4] * V[8] - V[5] * V[7]) - V[1] * (V[3] * V[8] - V[5] * V[6]) +
                       V[2] * (V[3] * V[7] - V[4] * V[6]);
    if (det < 0.0)
        for (int k = 0; k < 3; ++k) V[3 * k + 2] = -V[3 * k + 2];
}

// Unit quaternion (w, x, y, z), w >= 0, of a proper rotation matrix: the
// largest of the four squared components is taken from the diagonal, the
// others from sums and differences of the off-diagonal entries over it.
__device__ inline void rot_to_quat_d(const double R[9], double q[4]) {
    const double tr = R[0] + R[4] + R[8];
    const double sq[4] = {1.0 + tr, 1.0 + 2.0 * R[0] - tr, 1.0 + 2.0 * R[4] - tr, 1.0 + 2.0 * R[8] - tr};
    int k = 0;
    for (int i = 1; i < 4; ++i)
        if (sq[i] > sq[k]) k = i;
    const double s = sqrt(fmax(sq[k], 1e-300));  // 2 |q_k|
    const double d = 2.0 * s;
    if (k == 0) {
        q[0] = s / 2, q[1] = (R[7] - R[5]) / d, q[2] = (R[2] - R[6]) / d, q[3] = (R[3] - R[1]) / d;
    } else if (k == 1) {
        q[0] = (R[7] - R[5]) / d, q[1] = s / 2, q[2] = (R[1] + R[3]) / d, q[3] = (R[2] + R[6]) / d;
    } else if (k == 2) {
        q[0] = (R[2] - R[6]) / d, q[1] = (R[1] + R[3]) / d, q[2] = s / 2, q[3] = (R[5] + R[7]) / d;
    } else {
        q[0] = (R[3] - R[1]) / d, q[1] = (R[2] + R[6]) / d, q[2] = (R[5] + R[7]) / d, q[3] = s / 2;
    }
    const double sg = q[0] < 0.0 ? -1.0 : 1.0;
    const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int i = 0; i < 4; ++i) q[i] *= sg / n;
}

__global__ __launch_bounds__(256) void k_merge_geometry(gsr_param_set nodes, uint64_t child_base, uint64_t n_child,
                                                        uint64_t parent_base, uint32_t branching,
                                                        int32_t *__restrict__ parent, int32_t *__restrict__ child_count) {
    const uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x;  // parent within its level
    const uint64_t first = (uint64_t)j * branching;
    if (first >= n_child) return;
    const uint32_t k = (uint32_t)min((uint64_t)branching, n_child - first);
    const uint64_t c0 = child_base + first, p = parent_base + j;
    const double ox = nodes.means[3 * c0], oy = nodes.means[3 * c0 + 1], oz = nodes.means[3 * c0 + 2];
    double wsum = 0.0, keep = 1.0, d[3] = {0.0, 0.0, 0.0}, S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (uint32_t i = 0; i < k; ++i) {
        const uint64_t c = c0 + i;
        parent[c] = (int32_t)p;
        const double o = nodes.opacities[c];
        const float4 qf = reinterpret_cast<const float4 *>(nodes.quats)[c];
        double R[9];
        quat_to_rot_d(qf.x, qf.y, qf.z, qf.w, R);
        const double e0 = exp(2.0 * (double)nodes.log_scales[3 * c]), e1 = exp(2.0 * (double)nodes.log_scales[3 * c + 1]),
                     e2 = exp(2.0 * (double)nodes.log_scales[3 * c + 2]);
        const double dx = (double)nodes.means[3 * c] - ox, dy = (double)nodes.means[3 * c + 1] - oy,
                     dz = (double)nodes.means[3 * c + 2] - oz;
        // o (Sigma_c + d d^T), upper triangle: 00 01 02 11 12 22
        const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
        const double dd[3] = {dx, dy, dz};
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            const int a = ia[t], b = ib[t];
            const double sig = R[3 * a] * R[3 * b] * e0 + R[3 * a + 1] * R[3 * b + 1] * e1 + R[3 * a + 2] * R[3 * b + 2] * e2;
            S[t] += o * (sig + dd[a] * dd[b]);
        }
        d[0] += o * dx, d[1] += o * dy, d[2] += o * dz;
        wsum += o;
        keep *= 1.0 - o;
    }
    child_count[p] = (int32_t)k;
    const double inv = 1.0 / wsum;
    const double m[3] = {d[0] * inv, d[1] * inv, d[2] * inv};  // mean about the first child
    double A[9];
    A[0] = S[0] * inv - m[0] * m[0], A[1] = A[3] = S[1] * inv - m[0] * m[1], A[2] = A[6] = S[2] * inv - m[0] * m[2];
    A[4] = S[3] * inv - m[1] * m[1], A[5] = A[7] = S[4] * inv - m[1] * m[2], A[8] = S[5] * inv - m[2] * m[2];
    double lam[3], V[9], q[4];
    sym3_eig(A, lam, V);
    rot_to_quat_d(V, q);
    nodes.means[3 * p] = (float)(ox + m[0]);
    nodes.means[3 * p + 1] = (float)(oy + m[1]);
    nodes.means[3 * p + 2] = (float)(oz + m[2]);
    for (int a = 0; a < 3; ++a) nodes.log_scales[3 * p + a] = (float)(0.5 * log(fmax(lam[a], kMergeMinVar)));
    reinterpret_cast<float4 *>(nodes.quats)[p] = make_float4((float)q[0], (float)q[1], (float)q[2], (float)q[3]);
    nodes.opacities[p] = (float)(1.0 - keep);
}

// SH rows of the parents: unit u of parent j (K3 / 4 float4 units, or K3
// floats when a row is not a whole number of float4).
template <int K3, bool VEC>
__global__ __launch_bounds__(256) void k_merge_sh(gsr_param_set nodes, uint64_t child_base, uint64_t n_child,
                                                  uint64_t parent_base, uint64_t n_parent, uint32_t branching) {
    constexpr uint32_t kUnits = VEC ? K3 / 4 : K3;
    const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_parent * kUnits) return;
    const uint64_t j = t / kUnits, u = t - j * kUnits;
    const uint64_t first = j * branching, c0 = child_base + first, p = parent_base + j;
    const uint32_t k = (uint32_t)min((uint64_t)branching, n_child - first);
    float wsum = 0.f;
    for (uint32_t i = 0; i < k; ++i) wsum += nodes.opacities[c0 + i];
    const float inv = 1.f / wsum;
    if constexpr (VEC) {
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        for (uint32_t i = 0; i < k; ++i) {
            const float w = nodes.opacities[c0 + i] * inv;
            const float4 v = reinterpret_cast<const float4 *>(nodes.sh)[(c0 + i) * kUnits + u];
            acc.x = fmaf(w, v.x, acc.x), acc.y = fmaf(w, v.y, acc.y), acc.z = fmaf(w, v.z, acc.z),
            acc.w = fmaf(w, v.w, acc.w);
        }
        reinterpret_cast<float4 *>(nodes.sh)[p * kUnits + u] = acc;
    } else {
        float acc = 0.f;
        for (uint32_t i = 0; i < k; ++i) acc = fmaf(nodes.opacities[c0 + i] * inv, nodes.sh[(c0 + i) * kUnits + u], acc);
        nodes.sh[p * kUnits + u] = acc;
    }
}

__global__ __launch_bounds__(256) void k_fill_i32(int32_t *__restrict__ p, int32_t value, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = value;
}

void launch_hierarchy_level(const gsr_param_set &nodes, int sh_degree, uint64_t child_base, uint64_t n_child,
                            uint64_t parent_base, uint32_t branching, int32_t *parent, int32_t *child_count,
                            hipStream_t st) {
    const uint64_t n_parent = (n_child + branching - 1) / branching;
    if (n_parent == 0) return;
    hipLaunchKernelGGL(k_merge_geometry, dim3((unsigned)((n_parent + 255) / 256)), dim3(256), 0, st, nodes, child_base,
                       n_child, parent_base, branching, parent, child_count);
    auto sh = [&](auto kernel, uint64_t units) {
        hipLaunchKernelGGL(kernel, dim3((unsigned)((n_parent * units + 255) / 256)), dim3(256), 0, st, nodes,
                           child_base, n_child, parent_base, n_parent, branching);
    };
    switch (sh_degree) {
        case 0: sh(k_merge_sh<3, false>, 3); break;
        case 1: sh(k_merge_sh<12, true>, 3); break;
        case 2: sh(k_merge_sh<27, false>, 27); break;
        default: sh(k_merge_sh<48, true>, 12); break;
    }
}

void launch_fill_i32(int32_t *p, int32_t value, uint64_t n, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, value, n);
}

}  // namespace gsr
