// gsr_ba.hip -- local bundle adjustment with a dense Schur complement on
// gfx950, in FP64 (Sec. 5.1, "Local Bundle Adjustment" and "Solver
// efficiency"; appendix "Details on Local Pose Reconstruction", paragraph
// "Fast Bundle Adjustment").
//
// Unknowns: the free keyframe poses (a left twist (rho, phi) each, translation
// first), one shared focal length f, and the landmarks.  Residual of the
// observation of landmark j in keyframe i: f (X / Z, Y / Z) + c - z_ij with
// X = R_i p_j + t_i.  One iteration is a Levenberg-Marquardt step with
// Marquardt damping (every diagonal of the normal matrix scaled by 1 + lambda)
// taken unconditionally:
//
//   k_ba_landmark   one 8-lane group per landmark, one lane per observation
//                   slot: residual and Jacobians, the landmark's 3x3 block
//                   (damped, inverted in closed form), and for every
//                   observation in a free keyframe the pieces of the Schur
//                   complement it contributes (below);
//   k_ba_assemble   workgroups per block (a, b) of the reduced camera
//                   system, each walking its part of a host-built list of
//                   observation pairs in a fixed order (deterministic, no
//                   atomics) into a partial system, plus workgroups for the
//                   focal-length entry and the cost; the records are stored
//                   keyframe-major, so a diagonal block reads one contiguous
//                   run of them;
//   k_ba_solve      one workgroup: adds the partial systems, then a blocked
//                   Cholesky in LDS with the forward solve riding along, and
//                   the backward solve in one wave;
//   k_ba_update     landmark back-substitution and update, and the SE(3)
//                   retraction of the free poses and the focal step.
//
// The pieces per observation o (landmark j, free keyframe a), with
// B_o = Jx^T Jp (6x3), Hinv the inverse of the damped landmark block,
// Y_o = B_o Hinv, b_f = sum over the landmark's observations of Jf^T Jp and
// g_p the landmark gradient:
//   D_o = Jx^T Jx - Y_o B_o^T   (diagonal block, damping added from dg_o),
//   dg_o = diag(Jx^T Jx),  c_o = Jx^T Jf - Y_o b_f,  s_o = Jx^T r - Y_o g_p;
// and per landmark y_f = Hinv b_f, h_g = Hinv g_p, Jf^T Jf, y_f . b_f,
// Jf^T r - y_f . g_p and its share of the cost.  Off-diagonal blocks are
// -sum over shared landmarks of Y_{o_a} B_{o_b}^T.
#include "gsr_ba.h"

namespace gsr {

namespace {

constexpr int kLanesPerLm = kBaMaxObs;   // 8
constexpr int kBaThreads = 256;
constexpr int kSolveThreads = 512;    // the solve: 2 waves per SIMD to overlap its dependent chains

// offsets inside an observation record
constexpr int kRB = 0, kRY = 18, kRD = 36, kRDg = 57, kRC = 63, kRS = 69;
// offsets inside a landmark record
constexpr int kLYf = 0, kLHg = 3, kLFf = 6, kLFs = 7, kLSf = 8, kLCost = 9;

// One DPP step on a double (both 32-bit halves moved alike): v + v moved
// across lanes by `ctrl`, only in the rows enabled by `row_mask` (others add 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add_d(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    int lo = (int)(unsigned)b, hi = (int)(unsigned)(b >> 32);
    if constexpr (ROW_MASK == 0xf) {
        lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xf, 0xf, true);
        hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xf, 0xf, true);
    } else {
        lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, false);
        hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, false);
    }
    return v + __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double readlane_d(double v, int l) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over an 8-lane group (one landmark's observation slots): two quad swaps
// give each lane its quad's sum, the half-row mirror adds the other quad's.
// Additions pair the same operands on every lane, so all 8 lanes hold the
// bit-identical total.
__device__ __forceinline__ double group_sum(double v) {
    v = dpp_add_d<0xB1, 0xf>(v);   // quad_perm [1, 0, 3, 2]
    v = dpp_add_d<0x4E, 0xf>(v);   // quad_perm [2, 3, 0, 1]
    return dpp_add_d<0x141, 0xf>(v);  // row_half_mirror
}

// Sum over the 64 lanes of a wave in a fixed order: quad swaps, half-row and
// row mirrors leave each lane with its 16-lane row's sum, two row broadcasts
// gather the rows into row 3; lane 63's total is returned to every lane.
__device__ __forceinline__ double wave_sum_d(double v) {
    v = dpp_add_d<0xB1, 0xf>(v);   // quad_perm [1, 0, 3, 2]
    v = dpp_add_d<0x4E, 0xf>(v);   // quad_perm [2, 3, 0, 1]
    v = dpp_add_d<0x141, 0xf>(v);  // row_half_mirror
    v = dpp_add_d<0x140, 0xf>(v);  // row_mirror
    v = dpp_add_d<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_add_d<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return readlane_d(v, 63);
}

// Sum of N per-thread accumulators over the 256-thread block in a fixed
// order (deterministic): wave sums, then thread t adds the four waves' value
// t in wave order.  red: 5 N doubles of LDS; returns the N sums (in LDS,
// valid for every thread).
template <int N>
__device__ __forceinline__ const double *block_sum(const double (&acc)[N], double *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < N; ++t) {
        const double v = wave_sum_d(acc[t]);
        if (lane == 0) red[w * N + t] = v;
    }
    __syncthreads();
    if (threadIdx.x < N) {
        const int t = threadIdx.x;
        red[4 * N + t] = ((red[t] + red[N + t]) + red[2 * N + t]) + red[3 * N + t];
    }
    __syncthreads();
    return red + 4 * N;
}

// A partial system: D rows of pitch D + 1 (even, as D = 6F + 1 is odd, so rows
// are 16-byte aligned), then the right-hand side (D), the cost and a pad.
__device__ __forceinline__ size_t part_stride(int D) { return (size_t)(D + 1) * (D + 1); }

struct ObsGeom {
    double r[2], jx[2][6], jf[2], jp[2][3];
};

// Residual and Jacobians of one observation.
__device__ __forceinline__ ObsGeom observe(const double *__restrict__ T, const double p[3], double f, double cx, double cy,
                                           const double uv[2]) {
    ObsGeom o;
    const double x = fma(T[0], p[0], fma(T[1], p[1], fma(T[2], p[2], T[3])));
    const double y = fma(T[4], p[0], fma(T[5], p[1], fma(T[6], p[2], T[7])));
    const double z = fma(T[8], p[0], fma(T[9], p[1], fma(T[10], p[2], T[11])));
    const double iz = 1.0 / z, xn = x * iz, yn = y * iz;
    o.r[0] = fma(f, xn, cx) - uv[0];
    o.r[1] = fma(f, yn, cy) - uv[1];
    const double a = f * iz, b = -a * xn, c = -a * yn;   // d pi / dX = [[a, 0, b], [0, a, c]]
    // dX/drho = I, dX/dphi = -[X]x (left perturbation)
    o.jx[0][0] = a;   o.jx[0][1] = 0.0; o.jx[0][2] = b;
    o.jx[0][3] = b * y; o.jx[0][4] = a * z - b * x; o.jx[0][5] = -a * y;
    o.jx[1][0] = 0.0; o.jx[1][1] = a;   o.jx[1][2] = c;
    o.jx[1][3] = c * y - a * z; o.jx[1][4] = -c * x; o.jx[1][5] = a * x;
    o.jf[0] = xn;
    o.jf[1] = yn;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        o.jp[0][k] = fma(a, T[k], b * T[8 + k]);
        o.jp[1][k] = fma(a, T[4 + k], c * T[8 + k]);
    }
    return o;
}

__global__ void __launch_bounds__(kBaThreads) k_ba_landmark(BaArgs A, int cost_only) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t j = gid / kLanesPerLm;
    const int k = (int)(gid % kLanesPerLm);
    const bool lm_ok = j < (uint32_t)A.K;          // whole groups share j: shuffles stay in the group
    const uint64_t o = (uint64_t)j * A.M + k;
    const int cam = (lm_ok && k < A.M) ? A.obs_cam[o] : -1;
    const double f = A.focal[0];
    ObsGeom g = {};
    if (cam >= 0) {
        double p[3] = {A.landmarks[3 * j], A.landmarks[3 * j + 1], A.landmarks[3 * j + 2]};
        double uv[2] = {A.obs_uv[2 * o], A.obs_uv[2 * o + 1]};
        g = observe(A.poses + 12 * cam, p, f, A.cx, A.cy, uv);
    }
    const double cost = group_sum(0.5 * (g.r[0] * g.r[0] + g.r[1] * g.r[1]));
    if (cost_only) {
        if (lm_ok && k == 0) A.lm_rec[(uint64_t)j * kBaLmStride + kLCost] = cost;
        return;
    }
    // landmark block, gradient and focal coupling, summed over the group
    double H[6], gp[3], bf[3];
    {
        int t = 0;
#pragma unroll
        for (int u = 0; u < 3; ++u)
#pragma unroll
            for (int v = u; v < 3; ++v) H[t++] = group_sum(fma(g.jp[0][u], g.jp[0][v], g.jp[1][u] * g.jp[1][v]));
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            gp[u] = group_sum(fma(g.jp[0][u], g.r[0], g.jp[1][u] * g.r[1]));
            bf[u] = group_sum(fma(g.jf[0], g.jp[0][u], g.jf[1] * g.jp[1][u]));
        }
    }
    const double ff = group_sum(fma(g.jf[0], g.jf[0], g.jf[1] * g.jf[1]));
    const double sfj = group_sum(fma(g.jf[0], g.r[0], g.jf[1] * g.r[1]));
    // H = [[H0 H1 H2], [H1 H3 H4], [H2 H4 H5]], damped; inverse by cofactors
    const double d0 = H[0] * (1.0 + A.lambda), d1 = H[3] * (1.0 + A.lambda), d2 = H[5] * (1.0 + A.lambda);
    const double c00 = d1 * d2 - H[4] * H[4], c01 = H[2] * H[4] - H[1] * d2, c02 = H[1] * H[4] - H[2] * d1;
    const double c11 = d0 * d2 - H[2] * H[2], c12 = H[1] * H[2] - d0 * H[4], c22 = d0 * d1 - H[1] * H[1];
    const double det = d0 * c00 + H[1] * c01 + H[2] * c02;
    const double id = det != 0.0 ? 1.0 / det : 0.0;
    const double Hi[3][3] = {{c00 * id, c01 * id, c02 * id}, {c01 * id, c11 * id, c12 * id}, {c02 * id, c12 * id, c22 * id}};
    double yf[3], hg[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
        yf[u] = fma(Hi[u][0], bf[0], fma(Hi[u][1], bf[1], Hi[u][2] * bf[2]));
        hg[u] = fma(Hi[u][0], gp[0], fma(Hi[u][1], gp[1], Hi[u][2] * gp[2]));
    }
    if (lm_ok && k == 0) {
        double *L = A.lm_rec + (uint64_t)j * kBaLmStride;
        L[kLYf] = yf[0]; L[kLYf + 1] = yf[1]; L[kLYf + 2] = yf[2];
        L[kLHg] = hg[0]; L[kLHg + 1] = hg[1]; L[kLHg + 2] = hg[2];
        L[kLFf] = ff;
        L[kLFs] = fma(yf[0], bf[0], fma(yf[1], bf[1], yf[2] * bf[2]));
        L[kLSf] = sfj - fma(yf[0], gp[0], fma(yf[1], gp[1], yf[2] * gp[2]));
        L[kLCost] = cost;
    }
    if (cam < 0 || A.free_slot[cam] < 0) return;
    double B[6][3], Y[6][3], rec[kBaRecStride];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int u = 0; u < 3; ++u) B[i][u] = fma(g.jx[0][i], g.jp[0][u], g.jx[1][i] * g.jp[1][u]);
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int u = 0; u < 3; ++u) Y[i][u] = fma(B[i][0], Hi[0][u], fma(B[i][1], Hi[1][u], B[i][2] * Hi[2][u]));
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            rec[kRB + 3 * i + u] = B[i][u];
            rec[kRY + 3 * i + u] = Y[i][u];
        }
    int t = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int q = i; q < 6; ++q) {
            const double jj = fma(g.jx[0][i], g.jx[0][q], g.jx[1][i] * g.jx[1][q]);
            const double yb = fma(Y[i][0], B[q][0], fma(Y[i][1], B[q][1], Y[i][2] * B[q][2]));
            rec[kRD + t++] = jj - yb;
            if (q == i) rec[kRDg + i] = jj;
        }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        rec[kRC + i] = fma(g.jx[0][i], g.jf[0], g.jx[1][i] * g.jf[1]) -
                       fma(Y[i][0], bf[0], fma(Y[i][1], bf[1], Y[i][2] * bf[2]));
        rec[kRS + i] = fma(g.jx[0][i], g.r[0], g.jx[1][i] * g.r[1]) -
                       fma(Y[i][0], gp[0], fma(Y[i][1], gp[1], Y[i][2] * gp[2]));
    }
    rec[kBaRecStride - 1] = 0.0;
    // records (keyframe-major, see the pair lists) are 608 bytes from a
    // 256-byte aligned base: 16-byte stores
    double2 *R = reinterpret_cast<double2 *>(A.obs_rec + (uint64_t)A.rec_pos[o] * kBaRecStride);
#pragma unroll
    for (int q = 0; q < kBaRecStride / 2; ++q) R[q] = make_double2(rec[2 * q], rec[2 * q + 1]);
}

// Blocks x = 0 .. nblk-1: block (a, b) of the reduced system from its pair
// list; block x = nblk: the focal-length diagonal entry, its right-hand side
// and the cost.  Each is split over kBaAsmSplit workgroups (y) that take
// consecutive parts of the list (of the landmarks) and write a partial system
// of their own; the solve adds the partials in order.
__global__ void __launch_bounds__(kBaThreads) k_ba_assemble(BaArgs A) {
    __shared__ double red[5 * 39];
    const int D = A.D, SP = D + 1, fcol = D - 1;
    const int part = blockIdx.y;
    double *S = A.S + part * part_stride(D), *s = S + (uint64_t)D * SP;
    if ((int)blockIdx.x == A.nblk) {
        const int j0 = (int)((int64_t)A.K * part / kBaAsmSplit), j1 = (int)((int64_t)A.K * (part + 1) / kBaAsmSplit);
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int jb = j0 + threadIdx.x; jb < j1; jb += 4 * kBaThreads) {   // 4 landmarks' loads in flight
            double v[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = jb + u * kBaThreads;
                const double *L = A.lm_rec + (uint64_t)j * kBaLmStride;
                const bool ok = j < j1;
                v[u][0] = ok ? L[kLFf] : 0.0;
                v[u][1] = ok ? L[kLFs] : 0.0;
                v[u][2] = ok ? L[kLSf] : 0.0;
                v[u][3] = ok ? L[kLCost] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[t] += v[u][t];
        }
        const double *sum = block_sum(acc, red);
        if (threadIdx.x == 0) {
            S[(uint64_t)fcol * SP + fcol] = sum[0] * (1.0 + A.lambda) - sum[1];
            s[fcol] = sum[2];
            s[D] = sum[3];   // the cost slot after the right-hand side
        }
        return;
    }
    const int2 ab = A.block_ab[blockIdx.x];
    const uint32_t b0 = A.block_off[blockIdx.x], len = A.block_off[blockIdx.x + 1] - b0;
    const uint32_t e0 = b0 + (uint32_t)((uint64_t)len * part / kBaAsmSplit);
    const uint32_t e1 = b0 + (uint32_t)((uint64_t)len * (part + 1) / kBaAsmSplit);
    const int ra = 6 * ab.x, rb = 6 * ab.y;
    if (ab.x == ab.y) {
        double acc[39];
#pragma unroll
        for (int t = 0; t < 39; ++t) acc[t] = 0.0;
        for (uint32_t e = e0 + threadIdx.x; e < e1; e += kBaThreads) {
            const double *R = A.obs_rec + (uint64_t)A.pairs[e].x * kBaRecStride + kRD;
#pragma unroll
            for (int t = 0; t < 39; ++t) acc[t] += R[t];
        }
        const double *sum = block_sum(acc, red);
        for (int t = threadIdx.x; t < 36; t += kBaThreads) {
            const int i = t / 6, q = t % 6;
            const int lo = i < q ? i : q, hi = i < q ? q : i;
            const int tri = lo * 6 - lo * (lo - 1) / 2 + (hi - lo);   // packed upper-triangle index
            double v = sum[tri];
            if (i == q) v += A.lambda * sum[21 + i];
            S[(uint64_t)(ra + i) * SP + ra + q] = v;
        }
        if (threadIdx.x < 6) {
            const int i = threadIdx.x;
            S[(uint64_t)(ra + i) * SP + fcol] = sum[27 + i];
            S[(uint64_t)fcol * SP + ra + i] = sum[27 + i];
            s[ra + i] = sum[33 + i];
        }
        return;
    }
    double acc[36];
#pragma unroll
    for (int t = 0; t < 36; ++t) acc[t] = 0.0;
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += kBaThreads) {
        const int2 pr = A.pairs[e];
        const double *Ya = A.obs_rec + (uint64_t)pr.x * kBaRecStride + kRY;
        const double *Bb = A.obs_rec + (uint64_t)pr.y * kBaRecStride + kRB;
        double y[18], b[18];
#pragma unroll
        for (int t = 0; t < 18; ++t) {
            y[t] = Ya[t];
            b[t] = Bb[t];
        }
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int q = 0; q < 6; ++q)
                acc[6 * i + q] += fma(y[3 * i], b[3 * q], fma(y[3 * i + 1], b[3 * q + 1], y[3 * i + 2] * b[3 * q + 2]));
    }
    const double *sum = block_sum(acc, red);
    for (int t = threadIdx.x; t < 36; t += kBaThreads) {
        const int i = t / 6, q = t % 6;
        S[(uint64_t)(ra + i) * SP + rb + q] = -sum[t];
        S[(uint64_t)(rb + q) * SP + ra + i] = -sum[t];
    }
}

// Cholesky S = L L^T of the reduced system (D x D, symmetric positive definite
// after damping) in LDS, right-looking in column blocks of 8, then
// dc = -S^-1 s.  Per block: wave 0 factors the 8 x 8 diagonal block in
// registers (lane = row * 8 + column) and solves its part of L z = s while the
// other waves file the previous block's panel; then 2 x 2 tiles of the
// trailing lower triangle each solve the panel rows they need against the
// block and take the rank-8 update, the first tile of each row band keeping
// its rows' panel and folding them into z.  Two barriers per block.  Finally
// wave 0 solves L^T x = z a column at a time.
__global__ void __launch_bounds__(kSolveThreads) k_ba_solve(BaArgs A, int iter) {
    extern __shared__ double lds[];
    // odd row pitch: column walks (one row per lane) hit distinct LDS banks
    const int D = A.D, P = D | 1;
    double *M = lds, *rhs = lds + (uint64_t)D * P, *dinv = rhs + D, *pan = dinv + D;   // pan: [D][8]
    const int tid = threadIdx.x, lane = tid & 63;
    const size_t ps = part_stride(D);
    // lower triangle of the sum of the partial systems, as column pairs of
    // 16-byte loads, 2 pairs x kBaAsmSplit partials in flight per thread
    {
        const int SP = D + 1, half = SP / 2, items = D * half;
        for (int base = tid; base < items; base += 2 * kSolveThreads) {
            double2 v[2][kBaAsmSplit];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int it = base + u * kSolveThreads, r = it / half, cp = it - r * half;
                const bool ok = it < items && 2 * cp <= r;
#pragma unroll
                for (int q = 0; q < kBaAsmSplit; ++q)
                    v[u][q] = ok ? *reinterpret_cast<const double2 *>(A.S + q * ps + (size_t)r * SP + 2 * cp)
                                 : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int it = base + u * kSolveThreads, r = it / half, cp = it - r * half;
                if (it < items && 2 * cp <= r) {
                    double2 w = v[u][0];
#pragma unroll
                    for (int q = 1; q < kBaAsmSplit; ++q) {
                        w.x += v[u][q].x;
                        w.y += v[u][q].y;
                    }
                    M[r * P + 2 * cp] = w.x;
                    if (2 * cp + 1 <= r) M[r * P + 2 * cp + 1] = w.y;
                }
            }
        }
    }
    for (int t = tid; t <= D; t += kSolveThreads) {   // right-hand side and (t = D) the cost
        const size_t at = (size_t)D * (D + 1) + t;
        double v = A.S[at];
#pragma unroll
        for (int q = 1; q < kBaAsmSplit; ++q) v += A.S[q * ps + at];
        if (t < D) rhs[t] = v;
        else if (A.costs) A.costs[iter] = v;
    }
    __syncthreads();
    for (int k0 = 0; k0 < D; k0 += 8) {
        const int nb = D - k0 < 8 ? D - k0 : 8, k1 = k0 + nb;
        if (tid < 64) {
            // rows/columns past the block's end are padded with the identity
            const int r = lane >> 3, c = lane & 7;
            const bool in = r < nb && c <= r;
            double a = in ? M[(k0 + r) * P + k0 + c] : (r == c ? 1.0 : 0.0);
            double y = (c == 0 && r < nb) ? rhs[k0 + r] : 0.0;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const double inv = rsqrt(readlane_d(a, j * 9)), ljj = readlane_d(a, j * 9) * inv;
                if (c == j) a = r == j ? ljj : (r > j ? a * inv : a);
                const double lrj = __shfl(a, r * 8 + j, 64), lcj = __shfl(a, c * 8 + j, 64);
                if (c > j && r >= c) a = fma(-lrj, lcj, a);
                const double zj = readlane_d(y, j * 8) * inv;
                if (c == 0) y = r == j ? zj : (r > j ? fma(-lrj, zj, y) : y);
            }
            if (in) M[(k0 + r) * P + k0 + c] = a;
            if (r == c && r < nb) dinv[k0 + r] = 1.0 / a;
            if (c == 0 && r < nb) rhs[k0 + r] = y;
        } else if (k0 > 0) {
            // meanwhile the other waves file the previous block's panel (rows
            // k0.., columns k0 - 8 .. k0 - 1) into the factor
            for (int e = tid - 64; e < (D - k0) * 8; e += kSolveThreads - 64)
                M[(k0 + (e >> 3)) * P + k0 - 8 + (e & 7)] = pan[(k0 + (e >> 3)) * 8 + (e & 7)];
        }
        __syncthreads();
        const int n = D - k1;   // n > 0 implies a full block (nb = 8)
        if (n > 0) {
            // the factor's 8 x 8 block, its reciprocal diagonal and z entries are
            // the same for every thread: read from LDS where used (broadcasts)
            const double *lb = M + k0 * P + k0, *di = dinv + k0, *zb = rhs + k0;
            const int T = (n + 1) >> 1, ntiles = T * (T + 1) / 2;
            for (int t = tid; t < ntiles; t += kSolveThreads) {
                int ti = (int)((sqrtf(8.f * (float)t + 1.f) - 1.f) * 0.5f);
                while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
                while (ti * (ti + 1) / 2 > t) --ti;
                const int tj = t - ti * (ti + 1) / 2;
                const int i0 = k1 + 2 * ti, j0 = k1 + 2 * tj;
                // the panel rows of this tile (L[row][k0..k1) = A[row][k0..k1) L_blk^-T),
                // recomputed by every tile that needs them: no panel phase, no barrier
                double li[2][8], lj[2][8];
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int m = 0; m < 8; ++m) {
                        li[u][m] = i0 + u < D ? M[(i0 + u) * P + k0 + m] : 0.0;
                        lj[u][m] = j0 + u < D ? M[(j0 + u) * P + k0 + m] : 0.0;
                    }
                double acc[2][2];
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int v = 0; v < 2; ++v) {
                        const int i = i0 + u, j = j0 + v;
                        acc[u][v] = (i < D && j <= i) ? M[i * P + j] : 0.0;
                    }
#pragma unroll
                for (int m = 0; m < 8; ++m) {
#pragma unroll
                    for (int q = 0; q < m; ++q) {
                        const double l = lb[m * P + q];
#pragma unroll
                        for (int u = 0; u < 2; ++u) {
                            li[u][m] = fma(-li[u][q], l, li[u][m]);
                            lj[u][m] = fma(-lj[u][q], l, lj[u][m]);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        li[u][m] *= di[m];
                        lj[u][m] *= di[m];
                    }
                }
                if (tj == 0) {
                    // the first tile of each row band files its rows' panel and
                    // folds them into z (one owner per row)
#pragma unroll
                    for (int u = 0; u < 2; ++u)
                        if (i0 + u < D) {
                            double rr = rhs[i0 + u];
#pragma unroll
                            for (int m = 0; m < 8; ++m) {
                                pan[(i0 + u) * 8 + m] = li[u][m];
                                rr = fma(-li[u][m], zb[m], rr);
                            }
                            rhs[i0 + u] = rr;
                        }
                }
#pragma unroll
                for (int m = 0; m < 8; ++m)
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int v = 0; v < 2; ++v) acc[u][v] = fma(-li[u][m], lj[v][m], acc[u][v]);
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int v = 0; v < 2; ++v) {
                        const int i = i0 + u, j = j0 + v;
                        if (i < D && j <= i) M[i * P + j] = acc[u][v];
                    }
            }
        }
        __syncthreads();
    }
    // L^T x = z by wave 0: lane owns entries lane and lane + 64; x_q is final
    // once every row below q has been folded in.
    if (tid >= 64) return;
    const double di0 = lane < D ? dinv[lane] : 0.0, di1 = lane + 64 < D ? dinv[lane + 64] : 0.0;
    double y0 = lane < D ? rhs[lane] : 0.0, y1 = lane + 64 < D ? rhs[lane + 64] : 0.0;
    // rows of L read four at a time ahead of the dependent steps that use them
    int q = D - 1;
    for (; q >= 4; q -= 4) {
        double m0[4], m1[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            m0[u] = lane < q - u ? M[(q - u) * P + lane] : 0.0;
            m1[u] = lane + 64 < q - u ? M[(q - u) * P + lane + 64] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = q - u;
            const double xr = r < 64 ? readlane_d(y0 * di0, r) : readlane_d(y1 * di1, r - 64);
            y0 = fma(-m0[u], xr, y0);
            y1 = fma(-m1[u], xr, y1);
        }
    }
    for (; q > 0; --q) {
        const double xq = q < 64 ? readlane_d(y0 * di0, q) : readlane_d(y1 * di1, q - 64);
        if (lane < q) y0 = fma(-M[q * P + lane], xq, y0);
        if (lane + 64 < q) y1 = fma(-M[q * P + lane + 64], xq, y1);
    }
    if (lane < D) A.dc[lane] = -y0 * di0;
    if (lane + 64 < D) A.dc[lane + 64] = -y1 * di1;
}

// SE(3) exponential of (rho, phi): R = I + a [phi]x + b [phi]x^2,
// V = I + b [phi]x + c [phi]x^2 with a = sin t / t, b = (1 - cos t) / t^2,
// c = (t - sin t) / t^3, t = |phi| (series below t = 1e-2, error < 1e-15).
__device__ void se3_exp(const double xi[6], double Rm[3][3], double tv[3]) {
    const double w0 = xi[3], w1 = xi[4], w2 = xi[5];
    const double t2 = w0 * w0 + w1 * w1 + w2 * w2, t = sqrt(t2);
    double a, b, c;
    if (t < 1e-2) {
        a = 1.0 - t2 / 6.0 * (1.0 - t2 / 20.0);
        b = 0.5 - t2 / 24.0 * (1.0 - t2 / 30.0);
        c = 1.0 / 6.0 - t2 / 120.0 * (1.0 - t2 / 42.0);
    } else {
        const double sn = sin(t), cs = cos(t);
        a = sn / t;
        b = (1.0 - cs) / t2;
        c = (t - sn) / (t2 * t);
    }
    const double W[3][3] = {{0.0, -w2, w1}, {w2, 0.0, -w0}, {-w1, w0, 0.0}};
    double W2[3][3];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) W2[r][q] = W[r][0] * W[0][q] + W[r][1] * W[1][q] + W[r][2] * W[2][q];
    double V[3][3];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) {
            const double id = r == q ? 1.0 : 0.0;
            Rm[r][q] = id + a * W[r][q] + b * W2[r][q];
            V[r][q] = id + b * W[r][q] + c * W2[r][q];
        }
    for (int r = 0; r < 3; ++r) tv[r] = V[r][0] * xi[0] + V[r][1] * xi[1] + V[r][2] * xi[2];
}

// Landmark back-substitution p_j -= h_g + sum_o Y_o^T dc_a + y_f df, and (the
// last block) the pose retraction T_a <- exp(dc_a) T_a and f += df.
__global__ void __launch_bounds__(kBaThreads) k_ba_update(BaArgs A) {
    const double df = A.dc[A.D - 1];
    if (blockIdx.x == gridDim.x - 1) {
        const int a = threadIdx.x;
        if (a < A.F) {
            double xi[6], Rm[3][3], tv[3];
            for (int q = 0; q < 6; ++q) xi[q] = A.dc[6 * a + q];
            se3_exp(xi, Rm, tv);
            double *T = A.poses + 12 * A.slot_cam[a];
            double N[12];
            for (int r = 0; r < 3; ++r) {
                for (int q = 0; q < 4; ++q) N[4 * r + q] = Rm[r][0] * T[q] + Rm[r][1] * T[4 + q] + Rm[r][2] * T[8 + q];
                N[4 * r + 3] += tv[r];
            }
            for (int q = 0; q < 12; ++q) T[q] = N[q];
        }
        if (a == 0) A.focal[0] += df;
        return;
    }
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t j = gid / kLanesPerLm;
    const int k = (int)(gid % kLanesPerLm);
    const bool lm_ok = j < (uint32_t)A.K;
    const uint64_t o = (uint64_t)j * A.M + k;
    const int cam = (lm_ok && k < A.M) ? A.obs_cam[o] : -1;
    const int slot = cam >= 0 ? A.free_slot[cam] : -1;
    double v[3] = {0.0, 0.0, 0.0};
    if (slot >= 0) {
        const double *Y = A.obs_rec + (uint64_t)A.rec_pos[o] * kBaRecStride + kRY;
        const double *dc = A.dc + 6 * slot;
        for (int i = 0; i < 6; ++i)
            for (int u = 0; u < 3; ++u) v[u] = fma(Y[3 * i + u], dc[i], v[u]);
    }
    for (int u = 0; u < 3; ++u) v[u] = group_sum(v[u]);
    if (lm_ok && k == 0) {
        const double *L = A.lm_rec + (uint64_t)j * kBaLmStride;
        for (int u = 0; u < 3; ++u) A.landmarks[3 * j + u] -= L[kLHg + u] + v[u] + L[kLYf + u] * df;
    }
}

__global__ void __launch_bounds__(kBaThreads) k_ba_cost(BaArgs A, int iter) {
    __shared__ double red[5];
    double acc[1] = {0.0};
    for (int j0 = threadIdx.x; j0 < A.K; j0 += 8 * kBaThreads) {   // 8 loads in flight per thread
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = j0 + u * kBaThreads;
            v[u] = j < A.K ? A.lm_rec[(uint64_t)j * kBaLmStride + kLCost] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[0] += v[u];
    }
    const double *sum = block_sum(acc, red);
    if (threadIdx.x == 0 && A.costs) A.costs[iter] = sum[0];
}

}  // namespace

size_t ba_solve_lds_bytes(int D) { return ((size_t)D * (D | 1) + 10 * (size_t)D) * sizeof(double); }

size_t ba_lds_bytes(int D) { return ba_solve_lds_bytes(D); }

hipError_t ba_allow_lds(int D) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ba_solve), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)ba_solve_lds_bytes(D));
}

void launch_ba_iterations(const BaArgs &A, int iterations, hipStream_t st) {
    const unsigned lm_blocks = (unsigned)(((uint64_t)A.K * kLanesPerLm + kBaThreads - 1) / kBaThreads);
    const size_t solve_lds = ba_solve_lds_bytes(A.D);
    for (int it = 0; it < iterations; ++it) {
        hipLaunchKernelGGL(k_ba_landmark, dim3(lm_blocks), dim3(kBaThreads), 0, st, A, 0);
        hipLaunchKernelGGL(k_ba_assemble, dim3((unsigned)A.nblk + 1, kBaAsmSplit), dim3(kBaThreads), 0, st, A);
        hipLaunchKernelGGL(k_ba_solve, dim3(1), dim3(kSolveThreads), solve_lds, st, A, it);
        hipLaunchKernelGGL(k_ba_update, dim3(lm_blocks + 1), dim3(kBaThreads), 0, st, A);
    }
    hipLaunchKernelGGL(k_ba_landmark, dim3(lm_blocks), dim3(kBaThreads), 0, st, A, 1);
    hipLaunchKernelGGL(k_ba_cost, dim3(1), dim3(kBaThreads), 0, st, A, iterations);
}

}  // namespace gsr
