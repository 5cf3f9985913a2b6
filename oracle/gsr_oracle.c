/*
 * gsr_oracle.c -- plain FP64 CPU oracle of the differentiable tile-based
 * Gaussian-splat rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code, header, table or constant with the GPU library, and the GPU library
 * never calls it.
 *
 * What it computes.  The paper trains its Gaussians with its own
 * differentiable renderer, derived from Taming 3DGS (Sec. 5.2, Gaussian
 * placement and optimisation); poses and Gaussians are optimised jointly (Sec. 1, Sec. 3,
 * Sec. 7).  The paper does not write the renderer down, so this oracle follows
 * the 3DGS rasterizer that both cited works define (EWA splatting with a
 * +0.3 I low-pass, 16x16 tiles, alpha <= 0.99, skip alpha < 1/255, stop when
 * transmittance would fall below 1e-4) in the plainest form that reaches the
 * same numbers:
 *
 *   or_project_one  -- per Gaussian and view: camera-space mean, EWA 2D
 *                      covariance and conic, SH colour, pixel/tile rectangle.
 *   or_bin          -- (tile, depth-bits, index) pair list, sorted with qsort,
 *                      and per-tile [start, end) ranges.
 *   or_render       -- per tile, per pixel, front-to-back compositing; then,
 *                      if an upstream image gradient is given, the exact
 *                      derivative of that forward by a hand-derived chain rule,
 *                      accumulated serially (one thread, fixed order).
 *
 * Readings of the paper that the oracle fixes (all listed in the design notes):
 *   quaternion (w,x,y,z), normalised inside, gradient w.r.t. the raw value;
 *   opacity given already activated; scale = exp(log-scale); world->camera
 *   4x4 row-major, OpenCV axes; pixel centre at (i + 1/2); near plane cull
 *   z <= near; Jacobian evaluated at x/z, y/z clamped to 1.3x the half-FOV
 *   tangent (no gradient through a clamped coordinate); tile membership is the
 *   exact axis-aligned box of the alpha >= 1/255 ellipse; depth key is the
 *   float32 bit pattern of camera-space z, ties broken by Gaussian index;
 *   gradients are true derivatives (zero through alpha's 0.99 clamp).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct or_camera {
    int32_t width, height;
    double fx, fy, cx, cy, near_plane;
    double w2c[16]; /* row-major world->camera; last row (0,0,0,1) */
} or_camera;

/* Per-Gaussian projected record (one view). */
typedef struct or_proj {
    int32_t visible;
    double p[3];              /* camera-space mean */
    double u, v;              /* pixel-space centre */
    double cov[3];            /* 2D covariance incl. low-pass: a, b, c */
    double conic[3];          /* inverse covariance: A, B, C */
    double opacity;
    double rgb[3];
    int32_t rgb_clamped[3];   /* colour was clamped at 0 */
    int32_t rect[4];          /* inclusive pixel box x0, y0, x1, y1 */
    int32_t trect[4];         /* inclusive tile box */
    uint32_t zbits;           /* float32 bit pattern of p[2] */
} or_proj;

/* ---------------------------------------------------------------------------
 * Real spherical harmonics up to degree 3 (the 3DGS basis: real SH with the
 * Condon-Shortley phase, in the order m = -l..l).  Constants are the textbook
 * normalisations written as expressions.
 * ------------------------------------------------------------------------- */
static void sh_basis(int degree, const double d[3], double *Y, double (*dY)[3])
{
    const double x = d[0], y = d[1], z = d[2];
    const double PI = 3.14159265358979323846;
    const double c0 = 0.5 * sqrt(1.0 / PI);
    const double c1 = sqrt(3.0 / (4.0 * PI));
    const double c2a = 0.5 * sqrt(15.0 / PI);   /* xy, yz, xz terms */
    const double c2b = 0.25 * sqrt(5.0 / PI);   /* 2z^2 - x^2 - y^2 */
    const double c2c = 0.25 * sqrt(15.0 / PI);  /* x^2 - y^2 */
    const double c3a = 0.25 * sqrt(35.0 / (2.0 * PI));
    const double c3b = 0.5 * sqrt(105.0 / PI);
    const double c3c = 0.25 * sqrt(21.0 / (2.0 * PI));
    const double c3d = 0.25 * sqrt(7.0 / PI);
    const double c3e = 0.25 * sqrt(105.0 / PI);
    int k;
    for (k = 0; k < 16; ++k) {
        Y[k] = 0.0;
        if (dY) dY[k][0] = dY[k][1] = dY[k][2] = 0.0;
    }
    Y[0] = c0;
    if (degree < 1) return;
    Y[1] = -c1 * y;  Y[2] = c1 * z;  Y[3] = -c1 * x;
    if (dY) { dY[1][1] = -c1; dY[2][2] = c1; dY[3][0] = -c1; }
    if (degree < 2) return;
    Y[4] = c2a * x * y;
    Y[5] = -c2a * y * z;
    Y[6] = c2b * (2.0 * z * z - x * x - y * y);
    Y[7] = -c2a * x * z;
    Y[8] = c2c * (x * x - y * y);
    if (dY) {
        dY[4][0] = c2a * y;          dY[4][1] = c2a * x;
        dY[5][1] = -c2a * z;         dY[5][2] = -c2a * y;
        dY[6][0] = -2.0 * c2b * x;   dY[6][1] = -2.0 * c2b * y;  dY[6][2] = 4.0 * c2b * z;
        dY[7][0] = -c2a * z;         dY[7][2] = -c2a * x;
        dY[8][0] = 2.0 * c2c * x;    dY[8][1] = -2.0 * c2c * y;
    }
    if (degree < 3) return;
    Y[9]  = -c3a * y * (3.0 * x * x - y * y);
    Y[10] = c3b * x * y * z;
    Y[11] = -c3c * y * (4.0 * z * z - x * x - y * y);
    Y[12] = c3d * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
    Y[13] = -c3c * x * (4.0 * z * z - x * x - y * y);
    Y[14] = c3e * z * (x * x - y * y);
    Y[15] = -c3a * x * (x * x - 3.0 * y * y);
    if (dY) {
        dY[9][0] = -c3a * 6.0 * x * y;
        dY[9][1] = -c3a * (3.0 * x * x - 3.0 * y * y);
        dY[10][0] = c3b * y * z;  dY[10][1] = c3b * x * z;  dY[10][2] = c3b * x * y;
        dY[11][0] = -c3c * (-2.0 * x * y);
        dY[11][1] = -c3c * (4.0 * z * z - x * x - 3.0 * y * y);
        dY[11][2] = -c3c * (8.0 * y * z);
        dY[12][0] = c3d * (-6.0 * x * z);
        dY[12][1] = c3d * (-6.0 * y * z);
        dY[12][2] = c3d * (6.0 * z * z - 3.0 * x * x - 3.0 * y * y);
        dY[13][0] = -c3c * (4.0 * z * z - 3.0 * x * x - y * y);
        dY[13][1] = -c3c * (-2.0 * x * y);
        dY[13][2] = -c3c * (8.0 * x * z);
        dY[14][0] = c3e * 2.0 * x * z;  dY[14][1] = -c3e * 2.0 * y * z;
        dY[14][2] = c3e * (x * x - y * y);
        dY[15][0] = -c3a * (3.0 * x * x - 3.0 * y * y);
        dY[15][1] = -c3a * (-6.0 * x * y);
    }
}

/* Exported for the basis pin (orthonormality / comparison with a library SH). */
void or_sh_basis(int degree, const double *dir, double *Y)
{
    sh_basis(degree, dir, Y, 0);
}

/* Unit-quaternion rotation matrix, q = (w, x, y, z), already normalised. */
static void quat_to_rot(const double q[4], double R[3][3])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1.0 - 2.0 * (y * y + z * z);
    R[0][1] = 2.0 * (x * y - w * z);
    R[0][2] = 2.0 * (x * z + w * y);
    R[1][0] = 2.0 * (x * y + w * z);
    R[1][1] = 1.0 - 2.0 * (x * x + z * z);
    R[1][2] = 2.0 * (y * z - w * x);
    R[2][0] = 2.0 * (x * z - w * y);
    R[2][1] = 2.0 * (y * z + w * x);
    R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

/* Exported for the rotation pin: normalises q first, like the renderer. */
void or_quat_to_rot(const double *q, double *R9)
{
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double qn[4] = {q[0] / n, q[1] / n, q[2] / n, q[3] / n};
    double R[3][3];
    int i, j;
    quat_to_rot(qn, R);
    for (i = 0; i < 3; ++i)
        for (j = 0; j < 3; ++j) R9[3 * i + j] = R[i][j];
}

static double clampd(double v, double lo, double hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

static uint32_t f32_bits(double v)
{
    float f = (float)v;
    uint32_t b;
    memcpy(&b, &f, 4);
    return b;
}

/*
 * Projection of Gaussian i into one view.  Returns the record; invisible
 * Gaussians (behind the near plane, zero quaternion, degenerate 2D covariance,
 * opacity < 1/255 or no pixel centre inside the alpha >= 1/255 box) get
 * visible = 0 and nothing else is meaningful.
 */
static void or_project_one(int64_t i, int sh_degree, const double *means, const double *log_scales,
                           const double *quats, const double *opac, const double *sh,
                           const or_camera *cam, int tile_w, int tile_h, or_proj *r)
{
    const int K = (sh_degree + 1) * (sh_degree + 1);
    const double *mu = means + 3 * i;
    const double *qr = quats + 4 * i;
    double W[3][3], t[3], q[4], R[3][3], s[3], Sig[3][3], T[2][3];
    double qn, rx, ry, limx, limy, rxc, ryc, J[2][3], camc[3], dvec[3], dn, dir[3];
    double Y[16], a, b, c, det, k2, ex, ey, o;
    int a_, b_, k, ch;

    memset(r, 0, sizeof(*r));
    for (a_ = 0; a_ < 3; ++a_) {
        for (b_ = 0; b_ < 3; ++b_) W[a_][b_] = cam->w2c[4 * a_ + b_];
        t[a_] = cam->w2c[4 * a_ + 3];
    }
    for (a_ = 0; a_ < 3; ++a_)
        r->p[a_] = W[a_][0] * mu[0] + W[a_][1] * mu[1] + W[a_][2] * mu[2] + t[a_];
    r->zbits = f32_bits(r->p[2]);
    if (!(r->p[2] > cam->near_plane)) return;

    qn = sqrt(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
    if (!(qn > 0.0)) return;
    for (k = 0; k < 4; ++k) q[k] = qr[k] / qn;
    quat_to_rot(q, R);
    for (k = 0; k < 3; ++k) s[k] = exp(log_scales[3 * i + k]);
    /* Sigma = R diag(s^2) R^T */
    for (a_ = 0; a_ < 3; ++a_)
        for (b_ = 0; b_ < 3; ++b_) {
            double acc = 0.0;
            for (k = 0; k < 3; ++k) acc += R[a_][k] * s[k] * s[k] * R[b_][k];
            Sig[a_][b_] = acc;
        }

    /* EWA: Jacobian of the pinhole map at the (clamped) camera-space mean. */
    rx = r->p[0] / r->p[2];
    ry = r->p[1] / r->p[2];
    limx = 1.3 * (cam->width / (2.0 * cam->fx));
    limy = 1.3 * (cam->height / (2.0 * cam->fy));
    rxc = clampd(rx, -limx, limx);
    ryc = clampd(ry, -limy, limy);
    J[0][0] = cam->fx / r->p[2]; J[0][1] = 0.0; J[0][2] = -cam->fx * rxc / r->p[2];
    J[1][0] = 0.0; J[1][1] = cam->fy / r->p[2]; J[1][2] = -cam->fy * ryc / r->p[2];
    /* T = J W ; Sigma' = T Sigma T^T + 0.3 I */
    for (a_ = 0; a_ < 2; ++a_)
        for (b_ = 0; b_ < 3; ++b_)
            T[a_][b_] = J[a_][0] * W[0][b_] + J[a_][1] * W[1][b_] + J[a_][2] * W[2][b_];
    {
        double TS[2][3];
        for (a_ = 0; a_ < 2; ++a_)
            for (b_ = 0; b_ < 3; ++b_)
                TS[a_][b_] = T[a_][0] * Sig[0][b_] + T[a_][1] * Sig[1][b_] + T[a_][2] * Sig[2][b_];
        a = TS[0][0] * T[0][0] + TS[0][1] * T[0][1] + TS[0][2] * T[0][2] + 0.3;
        b = TS[0][0] * T[1][0] + TS[0][1] * T[1][1] + TS[0][2] * T[1][2];
        c = TS[1][0] * T[1][0] + TS[1][1] * T[1][1] + TS[1][2] * T[1][2] + 0.3;
    }
    r->cov[0] = a; r->cov[1] = b; r->cov[2] = c;
    det = a * c - b * b;
    if (!(det > 0.0)) return;
    r->conic[0] = c / det;
    r->conic[1] = -b / det;
    r->conic[2] = a / det;
    r->u = cam->fx * rx + cam->cx;
    r->v = cam->fy * ry + cam->cy;

    /* View-dependent colour: direction from the camera centre, world frame. */
    for (a_ = 0; a_ < 3; ++a_) camc[a_] = -(W[0][a_] * t[0] + W[1][a_] * t[1] + W[2][a_] * t[2]);
    for (a_ = 0; a_ < 3; ++a_) dvec[a_] = mu[a_] - camc[a_];
    dn = sqrt(dvec[0] * dvec[0] + dvec[1] * dvec[1] + dvec[2] * dvec[2]);
    for (a_ = 0; a_ < 3; ++a_) dir[a_] = dvec[a_] / dn;
    sh_basis(sh_degree, dir, Y, 0);
    for (ch = 0; ch < 3; ++ch) {
        double acc = 0.5;
        for (k = 0; k < K; ++k) acc += sh[(i * K + k) * 3 + ch] * Y[k];
        r->rgb_clamped[ch] = acc < 0.0;
        r->rgb[ch] = acc < 0.0 ? 0.0 : acc;
    }

    /* Extent: exact bounding box of the alpha >= 1/255 ellipse. */
    o = opac[i];
    r->opacity = o;
    if (!(o >= 1.0 / 255.0)) return;
    k2 = 2.0 * log(255.0 * o);
    ex = sqrt(k2 * a);
    ey = sqrt(k2 * c);
    {
        /* pixel centres px + 1/2 with |px + 1/2 - u| <= ex, clipped to the image */
        double x0 = ceil(r->u - ex - 0.5), x1 = floor(r->u + ex - 0.5);
        double y0 = ceil(r->v - ey - 0.5), y1 = floor(r->v + ey - 0.5);
        if (x0 < 0.0) x0 = 0.0;
        if (y0 < 0.0) y0 = 0.0;
        if (x1 > cam->width - 1.0) x1 = cam->width - 1.0;
        if (y1 > cam->height - 1.0) y1 = cam->height - 1.0;
        if (!(x0 <= x1) || !(y0 <= y1)) return;
        r->rect[0] = (int32_t)x0; r->rect[1] = (int32_t)y0;
        r->rect[2] = (int32_t)x1; r->rect[3] = (int32_t)y1;
    }
    r->trect[0] = r->rect[0] / tile_w;
    r->trect[1] = r->rect[1] / tile_h;
    r->trect[2] = r->rect[2] / tile_w;
    r->trect[3] = r->rect[3] / tile_h;
    r->visible = 1;
}

/* ---------------------------------------------------------------------------
 * Binning: pairs (tile, zbits, gaussian) for every tile of every visible
 * Gaussian's tile box, in lexicographic order.
 * ------------------------------------------------------------------------- */
typedef struct or_pair {
    uint32_t tile, zbits, gid;
} or_pair;

static int pair_cmp(const void *pa, const void *pb)
{
    const or_pair *a = (const or_pair *)pa, *b = (const or_pair *)pb;
    if (a->tile != b->tile) return a->tile < b->tile ? -1 : 1;
    if (a->zbits != b->zbits) return a->zbits < b->zbits ? -1 : 1;
    if (a->gid != b->gid) return a->gid < b->gid ? -1 : 1;
    return 0;
}

/*
 * or_bin: n items with inclusive tile boxes trect[4n] (ignored when
 * visible[i] == 0) and depth keys zbits[n]; tiles_x * tiles_y tiles.
 * Writes up to cap sorted pairs into out_tile/out_gid and the per-tile
 * [start, end) into ranges[2 * n_tiles].  Returns the pair count M; when M
 * exceeds cap or an output pointer is NULL, only M is computed.
 */
int64_t or_bin(int64_t n, const int32_t *visible, const int32_t *trect, const uint32_t *zbits,
               int32_t tiles_x, int32_t tiles_y, int64_t cap, uint32_t *out_tile, uint32_t *out_gid,
               uint32_t *ranges)
{
    int64_t m = 0, i, j;
    or_pair *pairs;
    for (i = 0; i < n; ++i)
        if (visible[i])
            m += (int64_t)(trect[4 * i + 2] - trect[4 * i] + 1) * (trect[4 * i + 3] - trect[4 * i + 1] + 1);
    if (m > cap || !out_tile || !out_gid) return m;
    pairs = (or_pair *)malloc(sizeof(or_pair) * (size_t)(m > 0 ? m : 1));
    j = 0;
    for (i = 0; i < n; ++i) {
        int32_t tx, ty;
        if (!visible[i]) continue;
        for (ty = trect[4 * i + 1]; ty <= trect[4 * i + 3]; ++ty)
            for (tx = trect[4 * i]; tx <= trect[4 * i + 2]; ++tx) {
                pairs[j].tile = (uint32_t)(ty * tiles_x + tx);
                pairs[j].zbits = zbits[i];
                pairs[j].gid = (uint32_t)i;
                ++j;
            }
    }
    qsort(pairs, (size_t)m, sizeof(or_pair), pair_cmp);
    for (i = 0; i < 2 * (int64_t)tiles_x * tiles_y; ++i) ranges[i] = 0;
    for (i = 0; i < m; ++i) {
        out_tile[i] = pairs[i].tile;
        out_gid[i] = pairs[i].gid;
        if (i == 0 || pairs[i].tile != pairs[i - 1].tile) ranges[2 * pairs[i].tile] = (uint32_t)i;
        if (i == m - 1 || pairs[i].tile != pairs[i + 1].tile) ranges[2 * pairs[i].tile + 1] = (uint32_t)(i + 1);
    }
    free(pairs);
    return m;
}

/* ---------------------------------------------------------------------------
 * Projection-stage export for the stage tests (records of every Gaussian).
 * rec[n][16] = u, v, z, a, b, c, A, B, C, opacity, r, g, b, visible, (2 unused)
 * rect[n][4] pixel box, trect[n][4] tile box, zbits[n].
 * ------------------------------------------------------------------------- */
void or_project(int64_t n, int sh_degree, const double *means, const double *log_scales,
                const double *quats, const double *opac, const double *sh, const or_camera *cam,
                int tile_w, int tile_h, double *rec, int32_t *rect, int32_t *trect, uint32_t *zbits)
{
    int64_t i;
    or_proj r;
    for (i = 0; i < n; ++i) {
        or_project_one(i, sh_degree, means, log_scales, quats, opac, sh, cam, tile_w, tile_h, &r);
        double *o = rec + 16 * i;
        o[0] = r.u; o[1] = r.v; o[2] = r.p[2];
        o[3] = r.cov[0]; o[4] = r.cov[1]; o[5] = r.cov[2];
        o[6] = r.conic[0]; o[7] = r.conic[1]; o[8] = r.conic[2];
        o[9] = r.opacity; o[10] = r.rgb[0]; o[11] = r.rgb[1]; o[12] = r.rgb[2];
        o[13] = r.visible; o[14] = 0.0; o[15] = 0.0;
        memcpy(rect + 4 * i, r.rect, sizeof(r.rect));
        memcpy(trect + 4 * i, r.trect, sizeof(r.trect));
        zbits[i] = r.zbits;
    }
}

/* ---------------------------------------------------------------------------
 * Rendering (forward + optional backward) of one view.
 * ------------------------------------------------------------------------- */

/* Screen-space gradient accumulator per Gaussian: u, v, A, B, C, o, r, g, b. */
enum { G_U, G_V, G_A, G_B, G_C, G_O, G_R, G_G, G_BL, G_N };

typedef struct or_opts {
    int32_t tile_w, tile_h;
    /* thresholds (the renderer's decision rules) */
    double alpha_max, alpha_min, t_min;
    /* ambiguity margins for flagging pixels whose result is decided by a
       rounding-sensitive comparison */
    double eps_alpha, eps_t, eps_z_rel;
} or_opts;

void or_default_opts(or_opts *o)
{
    o->tile_w = 16; o->tile_h = 16;
    o->alpha_max = 0.99; o->alpha_min = 1.0 / 255.0; o->t_min = 1e-4;
    /* margins sized to an FP32 compositing path: alpha carries ~1e-7 relative
       rounding (5e-6 relative margin at 1/255), the transmittance product ~1e-6
       relative after a few hundred factors (2e-5 relative margin at 1e-4),
       depth keys come from an FP64 projection (near-exact ties only) */
    o->eps_alpha = 2e-8; o->eps_t = 2e-9; o->eps_z_rel = 1e-9;
}

/*
 * Projection backward for one Gaussian in one view: from screen-space
 * gradients gs[G_N] to parameter gradients (accumulated) and to the pose
 * gradient gW (3x3, accumulated) and gt (3, accumulated).
 */
static void or_project_backward(int64_t i, int sh_degree, const double *means, const double *log_scales,
                                const double *quats, const double *sh, const or_camera *cam,
                                const or_proj *r, const double *gs, double *g_means, double *g_log_scales,
                                double *g_quats, double *g_opac, double *g_sh, double gW[3][3], double gt[3])
{
    const int K = (sh_degree + 1) * (sh_degree + 1);
    const double *mu = means + 3 * i;
    const double *qr = quats + 4 * i;
    double W[3][3], t[3], qn, q[4], R[3][3], s[3], Sig[3][3];
    double p[3], rx, ry, limx, limy, rxc, ryc, J[2][3], T[2][3];
    double a = r->cov[0], b = r->cov[1], c = r->cov[2], D, ga, gb, gc, G2[2][2];
    double gSig[3][3], gT[2][3], gJ[2][3], gp[3] = {0, 0, 0};
    double camc[3], dvec[3], dn, dir[3], Y[16], dY[16][3], gdir[3] = {0, 0, 0}, gd[3], gcam[3];
    double grgb[3], gM[3][3], gR[3][3], gq[4] = {0, 0, 0, 0}, gqn[4], dot;
    int a_, b_, k, ch;

    for (a_ = 0; a_ < 3; ++a_) {
        for (b_ = 0; b_ < 3; ++b_) W[a_][b_] = cam->w2c[4 * a_ + b_];
        t[a_] = cam->w2c[4 * a_ + 3];
    }
    for (a_ = 0; a_ < 3; ++a_) p[a_] = r->p[a_];

    /* opacity */
    g_opac[i] += gs[G_O];

    /* colour -> SH coefficients and view direction */
    for (a_ = 0; a_ < 3; ++a_) camc[a_] = -(W[0][a_] * t[0] + W[1][a_] * t[1] + W[2][a_] * t[2]);
    for (a_ = 0; a_ < 3; ++a_) dvec[a_] = mu[a_] - camc[a_];
    dn = sqrt(dvec[0] * dvec[0] + dvec[1] * dvec[1] + dvec[2] * dvec[2]);
    for (a_ = 0; a_ < 3; ++a_) dir[a_] = dvec[a_] / dn;
    sh_basis(sh_degree, dir, Y, dY);
    for (ch = 0; ch < 3; ++ch) grgb[ch] = r->rgb_clamped[ch] ? 0.0 : gs[G_R + ch];
    for (k = 0; k < K; ++k)
        for (ch = 0; ch < 3; ++ch) {
            g_sh[(i * K + k) * 3 + ch] += grgb[ch] * Y[k];
            for (a_ = 0; a_ < 3; ++a_) gdir[a_] += grgb[ch] * sh[(i * K + k) * 3 + ch] * dY[k][a_];
        }
    dot = gdir[0] * dir[0] + gdir[1] * dir[1] + gdir[2] * dir[2];
    for (a_ = 0; a_ < 3; ++a_) gd[a_] = (gdir[a_] - dir[a_] * dot) / dn;
    for (a_ = 0; a_ < 3; ++a_) {
        g_means[3 * i + a_] += gd[a_];
        gcam[a_] = -gd[a_];
    }
    /* camc_a = -sum_j W[j][a] t[j] */
    for (a_ = 0; a_ < 3; ++a_)
        for (b_ = 0; b_ < 3; ++b_) {
            gW[b_][a_] += -t[b_] * gcam[a_];
            gt[b_] += -W[b_][a_] * gcam[a_];
        }

    /* conic (A, B, C) -> 2D covariance (a, b, c) */
    D = a * c - b * b;
    ga = (-c * c * gs[G_A] + b * c * gs[G_B] - b * b * gs[G_C]) / (D * D);
    gb = (2.0 * b * c * gs[G_A] - (a * c + b * b) * gs[G_B] + 2.0 * a * b * gs[G_C]) / (D * D);
    gc = (-b * b * gs[G_A] + a * b * gs[G_B] - a * a * gs[G_C]) / (D * D);
    G2[0][0] = ga; G2[0][1] = G2[1][0] = 0.5 * gb; G2[1][1] = gc;

    /* recompute Sigma, J, T */
    qn = sqrt(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
    for (k = 0; k < 4; ++k) q[k] = qr[k] / qn;
    quat_to_rot(q, R);
    for (k = 0; k < 3; ++k) s[k] = exp(log_scales[3 * i + k]);
    for (a_ = 0; a_ < 3; ++a_)
        for (b_ = 0; b_ < 3; ++b_) {
            double acc = 0.0;
            for (k = 0; k < 3; ++k) acc += R[a_][k] * s[k] * s[k] * R[b_][k];
            Sig[a_][b_] = acc;
        }
    rx = p[0] / p[2];
    ry = p[1] / p[2];
    limx = 1.3 * (cam->width / (2.0 * cam->fx));
    limy = 1.3 * (cam->height / (2.0 * cam->fy));
    rxc = clampd(rx, -limx, limx);
    ryc = clampd(ry, -limy, limy);
    J[0][0] = cam->fx / p[2]; J[0][1] = 0.0; J[0][2] = -cam->fx * rxc / p[2];
    J[1][0] = 0.0; J[1][1] = cam->fy / p[2]; J[1][2] = -cam->fy * ryc / p[2];
    for (a_ = 0; a_ < 2; ++a_)
        for (b_ = 0; b_ < 3; ++b_)
            T[a_][b_] = J[a_][0] * W[0][b_] + J[a_][1] * W[1][b_] + J[a_][2] * W[2][b_];

    /* Sigma' = T Sigma T^T: gSigma = T^T G2 T, gT = 2 G2 T Sigma */
    for (a_ = 0; a_ < 3; ++a_)
        for (b_ = 0; b_ < 3; ++b_) {
            double acc = 0.0;
            int m1, m2;
            for (m1 = 0; m1 < 2; ++m1)
                for (m2 = 0; m2 < 2; ++m2) acc += T[m1][a_] * G2[m1][m2] * T[m2][b_];
            gSig[a_][b_] = acc;
        }
    for (a_ = 0; a_ < 2; ++a_)
        for (b_ = 0; b_ < 3; ++b_) {
            double acc = 0.0;
            int m1, m2;
            for (m1 = 0; m1 < 2; ++m1)
                for (m2 = 0; m2 < 3; ++m2) acc += G2[a_][m1] * T[m1][m2] * Sig[m2][b_];
            gT[a_][b_] = 2.0 * acc;
        }
    /* T = J W: gJ = gT W^T, gW += J^T gT */
    for (a_ = 0; a_ < 2; ++a_)
        for (b_ = 0; b_ < 3; ++b_)
            gJ[a_][b_] = gT[a_][0] * W[b_][0] + gT[a_][1] * W[b_][1] + gT[a_][2] * W[b_][2];
    for (a_ = 0; a_ < 3; ++a_)
        for (b_ = 0; b_ < 3; ++b_) gW[a_][b_] += J[0][a_] * gT[0][b_] + J[1][a_] * gT[1][b_];

    /* J entries -> camera-space mean (true derivative, clamp passes nothing) */
    gp[2] += -cam->fx / (p[2] * p[2]) * gJ[0][0] - cam->fy / (p[2] * p[2]) * gJ[1][1];
    {
        double grxc = gJ[0][2] * (-cam->fx / p[2]);
        double gryc = gJ[1][2] * (-cam->fy / p[2]);
        gp[2] += gJ[0][2] * cam->fx * rxc / (p[2] * p[2]) + gJ[1][2] * cam->fy * ryc / (p[2] * p[2]);
        if (rx >= -limx && rx <= limx) {
            gp[0] += grxc / p[2];
            gp[2] += grxc * (-p[0] / (p[2] * p[2]));
        }
        if (ry >= -limy && ry <= limy) {
            gp[1] += gryc / p[2];
            gp[2] += gryc * (-p[1] / (p[2] * p[2]));
        }
    }
    /* pixel centre */
    gp[0] += gs[G_U] * cam->fx / p[2];
    gp[2] += -gs[G_U] * cam->fx * p[0] / (p[2] * p[2]);
    gp[1] += gs[G_V] * cam->fy / p[2];
    gp[2] += -gs[G_V] * cam->fy * p[1] / (p[2] * p[2]);

    /* p = W mu + t */
    for (a_ = 0; a_ < 3; ++a_) {
        g_means[3 * i + a_] += W[0][a_] * gp[0] + W[1][a_] * gp[1] + W[2][a_] * gp[2];
        gt[a_] += gp[a_];
        for (b_ = 0; b_ < 3; ++b_) gW[a_][b_] += gp[a_] * mu[b_];
    }

    /* Sigma = M M^T with M = R diag(s): gM = 2 gSigma M */
    for (a_ = 0; a_ < 3; ++a_)
        for (b_ = 0; b_ < 3; ++b_) {
            double acc = 0.0;
            for (k = 0; k < 3; ++k) acc += gSig[a_][k] * R[k][b_] * s[b_];
            gM[a_][b_] = 2.0 * acc;
        }
    for (b_ = 0; b_ < 3; ++b_) {
        double gsj = 0.0;
        for (a_ = 0; a_ < 3; ++a_) {
            gR[a_][b_] = gM[a_][b_] * s[b_];
            gsj += gM[a_][b_] * R[a_][b_];
        }
        g_log_scales[3 * i + b_] += gsj * s[b_];
    }
    /* rotation matrix entries -> normalised quaternion */
    {
        const double w = q[0], x = q[1], y = q[2], z = q[3];
        gq[0] = 2.0 * (-z * gR[0][1] + y * gR[0][2] + z * gR[1][0] - x * gR[1][2] - y * gR[2][0] + x * gR[2][1]);
        gq[1] = 2.0 * (y * gR[0][1] + z * gR[0][2] + y * gR[1][0] - w * gR[1][2] + z * gR[2][0] + w * gR[2][1])
              - 4.0 * x * (gR[1][1] + gR[2][2]);
        gq[2] = 2.0 * (x * gR[0][1] + w * gR[0][2] + x * gR[1][0] + z * gR[1][2] - w * gR[2][0] + z * gR[2][1])
              - 4.0 * y * (gR[0][0] + gR[2][2]);
        gq[3] = 2.0 * (-w * gR[0][1] + x * gR[0][2] + w * gR[1][0] + y * gR[1][2] + x * gR[2][0] + y * gR[2][1])
              - 4.0 * z * (gR[0][0] + gR[1][1]);
    }
    /* normalisation q_hat = q / |q| */
    dot = gq[0] * q[0] + gq[1] * q[1] + gq[2] * q[2] + gq[3] * q[3];
    for (k = 0; k < 4; ++k) gqn[k] = (gq[k] - q[k] * dot) / qn;
    for (k = 0; k < 4; ++k) g_quats[4 * i + k] += gqn[k];
}

/*
 * or_render: one view.
 *   out_img [H*W*3], out_T [H*W], out_n [H*W] (last contributor position + 1
 *   within the pixel's tile list), out_ambig [H*W] (nullable): 0, or the
 *   reasons the pixel's result is decided by a rounding-sensitive comparison
 *   (bit 0: an alpha near 1/255, bit 1: near the 0.99 clamp, bit 2: a
 *   transmittance near the stop threshold, bit 3: two consecutive
 *   contributors with equal float32 depth).
 *   tile_mask [n_tiles] (nullable): only listed tiles are rendered and
 *   differentiated; other pixels are left untouched.
 *   dL_dimg (nullable): upstream gradient [H*W*3].  When given, parameter
 *   gradients are ACCUMULATED into g_* (caller zeroes them) and the pose
 *   gradient is accumulated into g_w2c[16] (row-major, last row stays 0).
 *   g_screen [n*G_N] (nullable) receives the screen-space gradients.
 * Returns the pair count M.
 */
int64_t or_render(int64_t n, int sh_degree, const double *means, const double *log_scales,
                  const double *quats, const double *opac, const double *sh, const or_camera *cam,
                  const double *bg, const or_opts *opts, const uint8_t *tile_mask,
                  double *out_img, double *out_T, int32_t *out_n, uint8_t *out_ambig,
                  const double *dL_dimg, double *g_means, double *g_log_scales, double *g_quats,
                  double *g_opac, double *g_sh, double *g_w2c, double *g_screen)
{
    const int tw = opts->tile_w, th = opts->tile_h;
    const int tiles_x = (cam->width + tw - 1) / tw, tiles_y = (cam->height + th - 1) / th;
    const int64_t n_tiles = (int64_t)tiles_x * tiles_y;
    or_proj *proj = (or_proj *)malloc(sizeof(or_proj) * (size_t)(n > 0 ? n : 1));
    int32_t *vis = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *trect = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)(n > 0 ? n : 1));
    uint32_t *zb = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    uint32_t *ranges = (uint32_t *)malloc(sizeof(uint32_t) * 2 * (size_t)n_tiles);
    double *gscr = 0;
    uint32_t *ptile, *pgid;
    int64_t i, m, tile;
    /* per-pixel scratch of one pixel's contributors */
    int64_t list_cap = 1024;
    int64_t *c_gid = (int64_t *)malloc(sizeof(int64_t) * (size_t)list_cap);
    double *c_alpha = (double *)malloc(sizeof(double) * (size_t)list_cap);
    double *c_T = (double *)malloc(sizeof(double) * (size_t)list_cap);
    double *c_e = (double *)malloc(sizeof(double) * (size_t)list_cap);
    double *c_dx = (double *)malloc(sizeof(double) * (size_t)list_cap);
    double *c_dy = (double *)malloc(sizeof(double) * (size_t)list_cap);
    int32_t *c_clamp = (int32_t *)malloc(sizeof(int32_t) * (size_t)list_cap);

    for (i = 0; i < n; ++i) {
        or_project_one(i, sh_degree, means, log_scales, quats, opac, sh, cam, tw, th, &proj[i]);
        vis[i] = proj[i].visible;
        memcpy(trect + 4 * i, proj[i].trect, sizeof(proj[i].trect));
        zb[i] = proj[i].zbits;
        if (tile_mask && vis[i]) {
            /* keep only Gaussians touching a selected tile (the lists of the
               selected tiles are unchanged by this) */
            int32_t tx, ty, hit = 0;
            for (ty = trect[4 * i + 1]; ty <= trect[4 * i + 3] && !hit; ++ty)
                for (tx = trect[4 * i]; tx <= trect[4 * i + 2]; ++tx)
                    if (tile_mask[(int64_t)ty * tiles_x + tx]) { hit = 1; break; }
            vis[i] = hit;
        }
    }
    m = or_bin(n, vis, trect, zb, tiles_x, tiles_y, INT64_MAX, 0, 0, ranges);
    ptile = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(m > 0 ? m : 1));
    pgid = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(m > 0 ? m : 1));
    or_bin(n, vis, trect, zb, tiles_x, tiles_y, m, ptile, pgid, ranges);

    if (dL_dimg) gscr = (double *)calloc((size_t)(n > 0 ? n : 1) * G_N, sizeof(double));

    for (tile = 0; tile < n_tiles; ++tile) {
        const int txi = (int)(tile % tiles_x), tyi = (int)(tile / tiles_x);
        const uint32_t s0 = ranges[2 * tile], s1 = ranges[2 * tile + 1];
        int px, py;
        if (tile_mask && !tile_mask[tile]) continue;
        for (py = tyi * th; py < (tyi + 1) * th && py < cam->height; ++py)
            for (px = txi * tw; px < (txi + 1) * tw && px < cam->width; ++px) {
                const int64_t pix = (int64_t)py * cam->width + px;
                double T = 1.0, C[3] = {0, 0, 0};
                int32_t last = 0, ambig = 0;
                int64_t nc = 0;
                uint32_t j;
                float zprev = 0.0f;
                int have_prev = 0;
                for (j = s0; j < s1; ++j) {
                    const or_proj *g = &proj[pgid[j]];
                    const double dx = g->u - (px + 0.5), dy = g->v - (py + 0.5);
                    const double sig = 0.5 * (g->conic[0] * dx * dx + g->conic[2] * dy * dy) + g->conic[1] * dx * dy;
                    double e, araw, alpha, Tn;
                    if (sig < 0.0) continue;
                    e = exp(-sig);
                    araw = g->opacity * e;
                    if (fabs(araw - opts->alpha_min) < opts->eps_alpha) ambig |= 1;
                    if (fabs(araw - opts->alpha_max) < opts->eps_alpha) ambig |= 2;
                    alpha = araw < opts->alpha_max ? araw : opts->alpha_max;
                    if (alpha < opts->alpha_min) continue;
                    Tn = T * (1.0 - alpha);
                    if (fabs(Tn - opts->t_min) < opts->eps_t) ambig |= 4;
                    {
                        float zf;
                        memcpy(&zf, &g->zbits, 4);
                        if (have_prev && fabsf(zf - zprev) <= (float)opts->eps_z_rel * zf) ambig |= 8;
                        zprev = zf;
                        have_prev = 1;
                    }
                    if (Tn < opts->t_min) break;
                    if (nc == list_cap) {
                        list_cap *= 2;
                        c_gid = (int64_t *)realloc(c_gid, sizeof(int64_t) * (size_t)list_cap);
                        c_alpha = (double *)realloc(c_alpha, sizeof(double) * (size_t)list_cap);
                        c_T = (double *)realloc(c_T, sizeof(double) * (size_t)list_cap);
                        c_e = (double *)realloc(c_e, sizeof(double) * (size_t)list_cap);
                        c_dx = (double *)realloc(c_dx, sizeof(double) * (size_t)list_cap);
                        c_dy = (double *)realloc(c_dy, sizeof(double) * (size_t)list_cap);
                        c_clamp = (int32_t *)realloc(c_clamp, sizeof(int32_t) * (size_t)list_cap);
                    }
                    c_gid[nc] = pgid[j]; c_alpha[nc] = alpha; c_T[nc] = T; c_e[nc] = e;
                    c_dx[nc] = dx; c_dy[nc] = dy; c_clamp[nc] = araw > opts->alpha_max;
                    ++nc;
                    C[0] += g->rgb[0] * alpha * T;
                    C[1] += g->rgb[1] * alpha * T;
                    C[2] += g->rgb[2] * alpha * T;
                    T = Tn;
                    last = (int32_t)(j - s0 + 1);
                }
                out_img[3 * pix + 0] = C[0] + T * bg[0];
                out_img[3 * pix + 1] = C[1] + T * bg[1];
                out_img[3 * pix + 2] = C[2] + T * bg[2];
                out_T[pix] = T;
                out_n[pix] = last;
                if (out_ambig) out_ambig[pix] = (uint8_t)ambig;

                if (dL_dimg) {
                    /* back to front: Bk = sum_{j>k} c_j a_j T_j + T_final bg */
                    const double *g = dL_dimg + 3 * pix;
                    double Bacc[3] = {T * bg[0], T * bg[1], T * bg[2]};
                    int64_t k;
                    for (k = nc - 1; k >= 0; --k) {
                        const or_proj *G = &proj[c_gid[k]];
                        double *gs = gscr + G_N * c_gid[k];
                        const double a = c_alpha[k], Tk = c_T[k];
                        double dalpha = 0.0, dsig;
                        int ch;
                        for (ch = 0; ch < 3; ++ch) {
                            gs[G_R + ch] += a * Tk * g[ch];
                            dalpha += g[ch] * (G->rgb[ch] * Tk - Bacc[ch] / (1.0 - a));
                            Bacc[ch] += G->rgb[ch] * a * Tk;
                        }
                        if (c_clamp[k]) continue;
                        gs[G_O] += dalpha * c_e[k];
                        dsig = -dalpha * a;
                        gs[G_A] += dsig * 0.5 * c_dx[k] * c_dx[k];
                        gs[G_B] += dsig * c_dx[k] * c_dy[k];
                        gs[G_C] += dsig * 0.5 * c_dy[k] * c_dy[k];
                        gs[G_U] += dsig * (G->conic[0] * c_dx[k] + G->conic[1] * c_dy[k]);
                        gs[G_V] += dsig * (G->conic[2] * c_dy[k] + G->conic[1] * c_dx[k]);
                    }
                }
            }
    }

    if (dL_dimg) {
        double gW[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, gt[3] = {0, 0, 0};
        int a_, b_;
        for (i = 0; i < n; ++i) {
            if (!vis[i]) continue;
            or_project_backward(i, sh_degree, means, log_scales, quats, sh, cam, &proj[i], gscr + G_N * i,
                                g_means, g_log_scales, g_quats, g_opac, g_sh, gW, gt);
        }
        for (a_ = 0; a_ < 3; ++a_) {
            for (b_ = 0; b_ < 3; ++b_) g_w2c[4 * a_ + b_] += gW[a_][b_];
            g_w2c[4 * a_ + 3] += gt[a_];
        }
        if (g_screen) memcpy(g_screen, gscr, sizeof(double) * (size_t)n * G_N);
        free(gscr);
    }

    free(proj); free(vis); free(trect); free(zb); free(ranges); free(ptile); free(pgid);
    free(c_gid); free(c_alpha); free(c_T); free(c_e); free(c_dx); free(c_dy); free(c_clamp);
    return m;
}

/* 6-DoF gradient of a left perturbation exp(xi^) T, xi = (rho, phi), from the
   gradient G of the 4x4 world->camera matrix: M = G T^T. */
void or_pose_twist(const double *G, const double *T, double *twist)
{
    double M[4][4];
    int i, j, k;
    for (i = 0; i < 4; ++i)
        for (j = 0; j < 4; ++j) {
            double acc = 0.0;
            for (k = 0; k < 4; ++k) acc += G[4 * i + k] * T[4 * j + k];
            M[i][j] = acc;
        }
    twist[0] = M[0][3]; twist[1] = M[1][3]; twist[2] = M[2][3];
    twist[3] = M[2][1] - M[1][2];
    twist[4] = M[0][2] - M[2][0];
    twist[5] = M[1][0] - M[0][1];
}
