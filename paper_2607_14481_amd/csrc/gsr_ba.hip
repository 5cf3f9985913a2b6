// gsr_ba.hip -- local bundle adjustment with a dense Schur complement on
// gfx950, in FP64 (Sec. 4.3, "Local Bundle Adjustment" and "Solver
// efficiency"; appendix "Fast Bundle Adjustment").
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
//   k_ba_assemble   one workgroup per block (a, b) of the reduced camera
//                   system, walking a host-built list of observation pairs
//                   in a fixed order (deterministic, no atomics), plus one
//                   workgroup for the focal-length entry and the cost;
//   k_ba_solve      one workgroup: LDL^T of the reduced system in LDS, one
//                   barrier per column, the forward solve riding along as
//                   an extra column; the backward solve in one wave;
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
#include "gsr_internal.h"

namespace gsr {

namespace {

constexpr int kLanesPerLm = kBaMaxObs;   // 8
constexpr int kBaThreads = 256;

// offsets inside an observation record
constexpr int kRB = 0, kRY = 18, kRD = 36, kRDg = 57, kRC = 63, kRS = 69;
// offsets inside a landmark record
constexpr int kLYf = 0, kLHg = 3, kLFf = 6, kLFs = 7, kLSf = 8, kLCost = 9;

__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int m = 1; m < kLanesPerLm; m <<= 1) v += __shfl_xor(v, m, kLanesPerLm);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Sum of N per-thread accumulators over a 256-thread block, in a fixed
// order: every wave reduces by butterfly, then thread t < N adds the four
// wave sums of value t in wave order.  Result valid in red[t] (all threads
// may read it after the trailing barrier).
template <int N>
__device__ __forceinline__ void block_sum(double (&acc)[N], double *red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < N; ++t) {
        const double s = wave_sum(acc[t]);
        if (lane == 0) red[w * N + t] = s;
    }
    __syncthreads();
    if (threadIdx.x < N) {
        const int t = threadIdx.x;
        red[4 * N + t] = ((red[t] + red[N + t]) + red[2 * N + t]) + red[3 * N + t];
    }
    __syncthreads();
}

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
    double *R = A.obs_rec + o * kBaRecStride;
    double B[6][3], Y[6][3];
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
            R[kRB + 3 * i + u] = B[i][u];
            R[kRY + 3 * i + u] = Y[i][u];
        }
    int t = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int q = i; q < 6; ++q) {
            const double jj = fma(g.jx[0][i], g.jx[0][q], g.jx[1][i] * g.jx[1][q]);
            const double yb = fma(Y[i][0], B[q][0], fma(Y[i][1], B[q][1], Y[i][2] * B[q][2]));
            R[kRD + t++] = jj - yb;
            if (q == i) R[kRDg + i] = jj;
        }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        R[kRC + i] = fma(g.jx[0][i], g.jf[0], g.jx[1][i] * g.jf[1]) -
                     fma(Y[i][0], bf[0], fma(Y[i][1], bf[1], Y[i][2] * bf[2]));
        R[kRS + i] = fma(g.jx[0][i], g.r[0], g.jx[1][i] * g.r[1]) -
                     fma(Y[i][0], gp[0], fma(Y[i][1], gp[1], Y[i][2] * gp[2]));
    }
}

// Blocks 0 .. nblk-1: block (a, b) of the reduced system from its pair list;
// block nblk: the focal-length diagonal entry, its right-hand side and the cost.
__global__ void __launch_bounds__(kBaThreads) k_ba_assemble(BaArgs A, int iter) {
    __shared__ double red[5 * 39];
    const int D = A.D, fcol = D - 1;
    double *S = A.S, *s = A.S + (uint64_t)D * D;
    if ((int)blockIdx.x == A.nblk) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int j = threadIdx.x; j < A.K; j += kBaThreads) {
            const double *L = A.lm_rec + (uint64_t)j * kBaLmStride;
            acc[0] += L[kLFf];
            acc[1] += L[kLFs];
            acc[2] += L[kLSf];
            acc[3] += L[kLCost];
        }
        block_sum<4>(acc, red);
        if (threadIdx.x == 0) {
            S[(uint64_t)fcol * D + fcol] = red[16] * (1.0 + A.lambda) - red[17];
            s[fcol] = red[18];
            if (A.costs) A.costs[iter] = red[19];
        }
        return;
    }
    const int2 ab = A.block_ab[blockIdx.x];
    const uint32_t e0 = A.block_off[blockIdx.x], e1 = A.block_off[blockIdx.x + 1];
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
        block_sum<39>(acc, red);
        const double *sum = red + 4 * 39;
        for (int t = threadIdx.x; t < 36; t += kBaThreads) {
            const int i = t / 6, q = t % 6;
            const int lo = i < q ? i : q, hi = i < q ? q : i;
            const int tri = lo * 6 - lo * (lo - 1) / 2 + (hi - lo);   // packed upper-triangle index
            double v = sum[tri];
            if (i == q) v += A.lambda * sum[21 + i];
            S[(uint64_t)(ra + i) * D + ra + q] = v;
        }
        if (threadIdx.x < 6) {
            const int i = threadIdx.x;
            S[(uint64_t)(ra + i) * D + fcol] = sum[27 + i];
            S[(uint64_t)fcol * D + ra + i] = sum[27 + i];
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
    block_sum<36>(acc, red);
    const double *sum = red + 4 * 36;
    for (int t = threadIdx.x; t < 36; t += kBaThreads) {
        const int i = t / 6, q = t % 6;
        S[(uint64_t)(ra + i) * D + rb + q] = -sum[t];
        S[(uint64_t)(rb + q) * D + ra + i] = -sum[t];
    }
}

// LDL^T of the reduced system S (D x D, symmetric positive definite after
// damping) without pivoting, then dc = -S^-1 s.  Thread (i, h) owns row i and
// the columns of parity h; step k folds column k into the trailing lower
// triangle, A[i][q] -= A[i][k] A[q][k] / A[k][k] for k < q <= i, and does the
// same to the right-hand side.  Afterwards d_k = A[k][k], L_ik = A[i][k] / d_k.
__global__ void __launch_bounds__(kBaThreads) k_ba_solve(BaArgs A) {
    extern __shared__ double lds[];
    // odd row pitch: the column walks of the update (one row per lane) then hit
    // distinct LDS banks
    const int D = A.D, P = D | 1;
    double *M = lds, *rhs = lds + (uint64_t)D * P;
    const double *S = A.S, *s = A.S + (uint64_t)D * D;
    for (int t = threadIdx.x; t < D * D; t += kBaThreads) {
        const int r = t / D, c = t % D;
        if (c <= r) M[r * P + c] = S[t];
    }
    for (int t = threadIdx.x; t < D; t += kBaThreads) rhs[t] = s[t];
    __syncthreads();
    const int i = threadIdx.x & 127, h = threadIdx.x >> 7;
    for (int k = 0; k < D - 1; ++k) {
        if (i > k && i < D) {
            const double l = M[i * P + k] / M[k * P + k];
            for (int q = k + 1 + h; q <= i; q += 2) M[i * P + q] = fma(-l, M[q * P + k], M[i * P + q]);
            if (h == 0) rhs[i] = fma(-l, rhs[k], rhs[i]);
        }
        __syncthreads();
    }
    // rhs now holds z with L z = s; x solves D L^T x = z, done by wave 0:
    // lane owns entries lane, lane + 64; x_q final once all rows below q folded in.
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    double y0 = lane < D ? rhs[lane] / M[lane * P + lane] : 0.0;
    double y1 = lane + 64 < D ? rhs[lane + 64] / M[(lane + 64) * P + lane + 64] : 0.0;
    for (int q = D - 1; q > 0; --q) {
        const double xq = __shfl(q < 64 ? y0 : y1, q & 63, 64);
        if (lane < q) y0 = fma(-M[q * P + lane] / M[lane * P + lane], xq, y0);
        if (lane + 64 < q) y1 = fma(-M[q * P + lane + 64] / M[(lane + 64) * P + lane + 64], xq, y1);
    }
    if (lane < D) A.dc[lane] = -y0;
    if (lane + 64 < D) A.dc[lane + 64] = -y1;
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
        const double *Y = A.obs_rec + o * kBaRecStride + kRY;
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
    for (int j = threadIdx.x; j < A.K; j += kBaThreads) acc[0] += A.lm_rec[(uint64_t)j * kBaLmStride + kLCost];
    block_sum<1>(acc, red);
    if (threadIdx.x == 0 && A.costs) A.costs[iter] = red[4];
}

}  // namespace

size_t ba_solve_lds_bytes(int D) { return ((size_t)D * (D | 1) + D) * sizeof(double); }

hipError_t ba_allow_lds(size_t bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ba_solve), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

void launch_ba_iterations(const BaArgs &A, int iterations, hipStream_t st) {
    const unsigned lm_blocks = (unsigned)(((uint64_t)A.K * kLanesPerLm + kBaThreads - 1) / kBaThreads);
    const size_t lds = ba_solve_lds_bytes(A.D);
    for (int it = 0; it < iterations; ++it) {
        hipLaunchKernelGGL(k_ba_landmark, dim3(lm_blocks), dim3(kBaThreads), 0, st, A, 0);
        hipLaunchKernelGGL(k_ba_assemble, dim3((unsigned)A.nblk + 1), dim3(kBaThreads), 0, st, A, it);
        hipLaunchKernelGGL(k_ba_solve, dim3(1), dim3(kBaThreads), lds, st, A);
        hipLaunchKernelGGL(k_ba_update, dim3(lm_blocks + 1), dim3(kBaThreads), 0, st, A);
    }
    hipLaunchKernelGGL(k_ba_landmark, dim3(lm_blocks), dim3(kBaThreads), 0, st, A, 1);
    hipLaunchKernelGGL(k_ba_cost, dim3(1), dim3(kBaThreads), 0, st, A, iterations);
}

}  // namespace gsr
