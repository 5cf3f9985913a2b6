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

}  // namespace gsr
