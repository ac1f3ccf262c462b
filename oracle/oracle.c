/*
 * CPU oracle for the 3D Gaussian Splatting training hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The GPU path never links,
 * imports or calls it, and it shares no code with the GPU path.
 *
 * What it computes, step by step, in the order of the training pipeline the
 * paper describes (Sec. 2 and Sec. 4): EWA projection with degree-3 SH colour
 * and a 3-sigma tile rectangle (Sec. 4.1 counts tiles during projection),
 * exclusive scan of tile counts ("Index Offset"), key generation with 32-bit
 * (tile, depth) keys and the depth map z -> (2z+1)/(z+1) (Sec. 4.4), a stable
 * sort, per-tile ranges, front-to-back alpha compositing, the L1 loss
 * gradient, the exact piecewise derivative of compositing (the rasterisation
 * backward of Sec. 4.2, here as a plain per-pixel loop), the projection
 * backward, and Adam applied to log-scales and opacity logits as stored
 * (Sec. 4.3).
 *
 * Two builds of this file:
 *   liboracle_f32.so  (default)     forward values in float32, the paper's
 *                                   precision (48 FP32 SH coefficients,
 *                                   Sec. 4.6).  Every float step that decides
 *                                   an integer (tile rectangle, sort key,
 *                                   compositing skip/stop) is taken in float32
 *                                   with a fixed operation order and no
 *                                   contraction.  Reductions, the backward and
 *                                   Adam are evaluated in float64.
 *   liboracle_f64.so  (-DOR_DOUBLE) everything in float64; used only by the
 *                                   finite-difference and closed-form checks.
 *
 * Constants the paper does not print (0.3 dilation, 0.99 alpha clamp, 1/255
 * skip, 1e-4 stop, 3 sigma, Adam beta/eps) follow the classic 3DGS rule.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -fPIC -shared
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef OR_DOUBLE
typedef double real;
#define RSQRT(x) sqrt(x)
#define RFLOOR(x) floor(x)
#define RCEIL(x) ceil(x)
#define RMIN(a, b) fmin(a, b)
#define RMAX(a, b) fmax(a, b)
#define REXP(x) exp(x)
#else
typedef float real;
#define RSQRT(x) sqrtf(x)
#define RFLOOR(x) floorf(x)
#define RCEIL(x) ceilf(x)
#define RMIN(a, b) fminf(a, b)
#define RMAX(a, b) fmaxf(a, b)
#define REXP(x) expf(x)
#endif
typedef double acc;

/* One camera view, 128 bytes, the same byte layout as the Python view record. */
typedef struct {
    float R[9];      /* world -> camera rotation, row major */
    float t[3];      /* world -> camera translation */
    float campos[3]; /* camera centre, world space */
    float fx, fy, cx, cy;
    float lim_x, lim_y; /* 1.3 * tan(half fov): clamp of x/z, y/z in J */
    float znear, zfar;
    float bg[3];
    int32_t width, height;
    int32_t pad[4];
} or_view;

/* ------------------------------------------------------------------------- */
/* Scalar helpers                                                             */
/* ------------------------------------------------------------------------- */

/* e^x for the parameter activations (scale, sigmoid).  Float build: the
 * Cody & Waite (1980) argument reduction x = n ln2 + r with a two-part ln2
 * whose high part has trailing zero bits (so n*ln2_hi is exact), e^r by the
 * Taylor polynomial of degree 7 in Horner form, then an exact scaling by 2^n.
 * Every operation is a single IEEE float operation, so any implementation of
 * the same steps gives the same bits. */
static real exp_param(real x)
{
#ifdef OR_DOUBLE
    return exp(x);
#else
    if (x != x) return x;
    if (x > 100.0f) x = 100.0f;
    if (x < -100.0f) x = -100.0f;
    const float log2e = (float)1.4426950408889634074;
    const float ln2_hi = 0.693145751953125f;            /* 0x3F317200 */
    const float ln2_lo = (float)(0.6931471805599453094 - 0.693145751953125);
    float n = rintf(x * log2e);
    float r = (x - n * ln2_hi) - n * ln2_lo;
    float p = (float)(1.0 / 5040.0);
    p = p * r + (float)(1.0 / 720.0);
    p = p * r + (float)(1.0 / 120.0);
    p = p * r + (float)(1.0 / 24.0);
    p = p * r + (float)(1.0 / 6.0);
    p = p * r + 0.5f;
    p = p * r + 1.0f;
    p = p * r + 1.0f;
    return ldexpf(p, (int)n);
#endif
}

static real sigmoid_param(real x) { return (real)1 / ((real)1 + exp_param(-x)); }

/* ln x for x > 0, for the opacity threshold of exact tile culling.  Float
 * build: x = m 2^k with m in [1/sqrt 2, sqrt 2) (exact), then
 * ln m = 2 atanh(s) with s = (m - 1)/(m + 1), summed as the odd series
 * s (2 + z (2/3 + z (2/5 + ... + z 2/13))), z = s^2, in Horner form, and
 * ln x = k ln2_hi + (k ln2_lo + ln m); every step one IEEE float operation,
 * coefficients the float32 values nearest 2/(2j+1). */
static real log_spec(real x)
{
#ifdef OR_DOUBLE
    return log(x);
#else
    int k;
    float m = frexpf(x, &k);                       /* x = m 2^k, m in [0.5, 1) */
    if (m < 0.70710676908493042f) { m = m * 2.0f; k = k - 1; }
    const float s = (m - 1.0f) / (m + 1.0f);
    const float z = s * s;
    float p = 0.15384615957736969f;                /* 2/13 */
    p = p * z + 0.18181818723678589f;              /* 2/11 */
    p = p * z + 0.22222222387790680f;              /* 2/9 */
    p = p * z + 0.28571429848670959f;              /* 2/7 */
    p = p * z + 0.40000000596046448f;              /* 2/5 */
    p = p * z + 0.66666668653488159f;              /* 2/3 */
    p = p * z + 2.0f;
    const float lm = s * p;
    const float fk = (float)k;
    return fk * 0.693145751953125f + (fk * 1.4286067653301870e-06f + lm);
#endif
}

/* ------------------------------------------------------------------------- */
/* Tile sets (Sec. 4.1)                                                       */
/* ------------------------------------------------------------------------- */

/* Exact culling: the tiles of a Gaussian are those whose square meets the
 * ellipse where it can reach alpha >= 1/255, i.e. the points d (offset from
 * the 2D mean) with A dx^2 + 2 B dx dy + C dy^2 <= tau, tau = 2 ln(255 o).
 * Tile rows are those meeting [v - hy, v + hy]; in each row band
 * [ya, yb] (clipped to the ellipse) the ellipse's x-extent is either its
 * global extreme (when the extreme point's y lies in the band) or the
 * boundary at one of the band's edges, and the column range is that extent
 * rounded outwards to tile boundaries.  Everything is float arithmetic in a
 * fixed order. */
typedef struct {
    real u, v, A, B, C, tau, dQ, hx, hy, ys;
} or_ellipse;

static int ellipse_setup(real u, real v, real A, real B, real C, real o, or_ellipse* e)
{
    const real x = (real)255 * o;
    if (!(x > (real)1)) return 0;                   /* alpha never reaches 1/255 */
    e->u = u; e->v = v; e->A = A; e->B = B; e->C = C;
    e->tau = (real)2 * log_spec(x);
    e->dQ = A * C - B * B;
    if (!(e->dQ > 0) || !(A > 0) || !(C > 0)) return 0;
    e->hx = RSQRT((e->tau * C) / e->dQ);
    e->hy = RSQRT((e->tau * A) / e->dQ);
    e->ys = -((B * e->hx) / C);                     /* dy of the rightmost point */
    return 1;
}

/* boundary x-offsets of the ellipse at height dy: (-B dy +- sqrt(A tau - dQ dy^2)) / A */
static real ellipse_xp(const or_ellipse* e, real dy)
{
    real w = e->A * e->tau - e->dQ * (dy * dy);
    w = RMAX(w, (real)0);
    return (RSQRT(w) - e->B * dy) / e->A;
}
static real ellipse_xm(const or_ellipse* e, real dy)
{
    real w = e->A * e->tau - e->dQ * (dy * dy);
    w = RMAX(w, (real)0);
    return (-RSQRT(w) - e->B * dy) / e->A;
}

/* rows [*y0, *y1) of tiles that meet the ellipse */
static void ellipse_rows(const or_ellipse* e, int tile, int gy, int* y0, int* y1)
{
    const real invT = (real)1 / (real)tile;
    const real fgy = (real)gy;
    *y0 = (int)RMIN(RMAX(RFLOOR((e->v - e->hy) * invT), (real)0), fgy);
    *y1 = (int)RMIN(RMAX(RFLOOR((e->v + e->hy) * invT) + (real)1, (real)0), fgy);
}

/* column range [*xa, *xb) of tile row ty (empty if *xb <= *xa) */
static void ellipse_span(const or_ellipse* e, int tile, int gx, int ty, int* xa, int* xb)
{
    const real invT = (real)1 / (real)tile;
    const real fgx = (real)gx;
    real ya = (real)(ty * tile) - e->v;
    real yb = (real)((ty + 1) * tile) - e->v;
    ya = RMAX(ya, -e->hy);
    yb = RMIN(yb, e->hy);
    const real xmax = (ya <= e->ys && e->ys <= yb) ? e->hx
                                                   : RMAX(ellipse_xp(e, ya), ellipse_xp(e, yb));
    const real xmin = (ya <= -e->ys && -e->ys <= yb) ? -e->hx
                                                     : RMIN(ellipse_xm(e, ya), ellipse_xm(e, yb));
    *xa = (int)RMIN(RMAX(RFLOOR((e->u + xmin) * invT), (real)0), fgx);
    *xb = (int)RMIN(RMAX(RFLOOR((e->u + xmax) * invT) + (real)1, (real)0), fgx);
}

/* Real spherical harmonics up to degree 3, orthonormal on the unit sphere,
 * in the sign convention common to 3DGS trainers. */
static const double SH_C0 = 0.28209479177387814;  /* 1/(2 sqrt(pi)) */
static const double SH_C1 = 0.4886025119029199;   /* sqrt(3/(4 pi)) */
static const double SH_C2[5] = {1.0925484305920792, -1.0925484305920792, 0.31539156525252005,
                                -1.0925484305920792, 0.5462742152960396};
static const double SH_C3[7] = {-0.5900435899266435, 2.890611442640554, -0.4570457994644658,
                                0.3731763325901154, -0.4570457994644658, 1.445305721320277,
                                -0.5900435899266435};

static void sh_basis(real x, real y, real z, real Y[16])
{
    const real xx = x * x, yy = y * y, zz = z * z;
    const real xy = x * y, yz = y * z, xz = x * z;
    Y[0] = (real)SH_C0;
    Y[1] = -((real)SH_C1 * y);
    Y[2] = (real)SH_C1 * z;
    Y[3] = -((real)SH_C1 * x);
    Y[4] = (real)SH_C2[0] * xy;
    Y[5] = (real)SH_C2[1] * yz;
    Y[6] = (real)SH_C2[2] * (((real)2 * zz - xx) - yy);
    Y[7] = (real)SH_C2[3] * xz;
    Y[8] = (real)SH_C2[4] * (xx - yy);
    Y[9] = ((real)SH_C3[0] * y) * ((real)3 * xx - yy);
    Y[10] = ((real)SH_C3[1] * xy) * z;
    Y[11] = ((real)SH_C3[2] * y) * (((real)4 * zz - xx) - yy);
    Y[12] = ((real)SH_C3[3] * z) * (((real)2 * zz - (real)3 * xx) - (real)3 * yy);
    Y[13] = ((real)SH_C3[4] * x) * (((real)4 * zz - xx) - yy);
    Y[14] = ((real)SH_C3[5] * z) * (xx - yy);
    Y[15] = ((real)SH_C3[6] * x) * (xx - (real)3 * yy);
}

/* d Y_m / d(x, y, z), the direction components taken as free variables. */
static void sh_basis_grad(acc x, acc y, acc z, acc dY[16][3])
{
    const acc xx = x * x, yy = y * y, zz = z * z;
    memset(dY, 0, sizeof(acc) * 48);
    dY[1][1] = -SH_C1;
    dY[2][2] = SH_C1;
    dY[3][0] = -SH_C1;
    dY[4][0] = SH_C2[0] * y; dY[4][1] = SH_C2[0] * x;
    dY[5][1] = SH_C2[1] * z; dY[5][2] = SH_C2[1] * y;
    dY[6][0] = -2 * SH_C2[2] * x; dY[6][1] = -2 * SH_C2[2] * y; dY[6][2] = 4 * SH_C2[2] * z;
    dY[7][0] = SH_C2[3] * z; dY[7][2] = SH_C2[3] * x;
    dY[8][0] = 2 * SH_C2[4] * x; dY[8][1] = -2 * SH_C2[4] * y;
    dY[9][0] = SH_C3[0] * 6 * x * y; dY[9][1] = SH_C3[0] * (3 * xx - 3 * yy);
    dY[10][0] = SH_C3[1] * y * z; dY[10][1] = SH_C3[1] * x * z; dY[10][2] = SH_C3[1] * x * y;
    dY[11][0] = -2 * SH_C3[2] * x * y; dY[11][1] = SH_C3[2] * (4 * zz - xx - 3 * yy);
    dY[11][2] = 8 * SH_C3[2] * y * z;
    dY[12][0] = -6 * SH_C3[3] * x * z; dY[12][1] = -6 * SH_C3[3] * y * z;
    dY[12][2] = SH_C3[3] * (6 * zz - 3 * xx - 3 * yy);
    dY[13][0] = SH_C3[4] * (4 * zz - 3 * xx - yy); dY[13][1] = -2 * SH_C3[4] * x * y;
    dY[13][2] = 8 * SH_C3[4] * x * z;
    dY[14][0] = 2 * SH_C3[5] * x * z; dY[14][1] = -2 * SH_C3[5] * y * z;
    dY[14][2] = SH_C3[5] * (xx - yy);
    dY[15][0] = SH_C3[6] * (3 * xx - 3 * yy); dY[15][1] = -6 * SH_C3[6] * x * y;
}

/* ------------------------------------------------------------------------- */
/* Projection (EWA splatting, Zwicker et al.; 3DGS Sec. 4 of Kerbl et al.)    */
/* ------------------------------------------------------------------------- */

typedef struct {
    int valid;
    /* outputs */
    real u, v, z;
    real a, b, c;       /* 2D covariance with the 0.3 dilation */
    real A, B, C;       /* conic = inverse 2D covariance */
    real o;
    real col[3];
    real raw[3];        /* SH sum before the +0.5 and the clamp */
    real radius;
    int32_t x0, y0, x1, y1;
    uint32_t tiles;
    /* intermediates kept for the backward */
    real qn[4], qnorm;
    real Rq[9];
    real s[3];
    real M[9];
    real Sig[9];
    real p[3];
    real tx, ty, txc, tyc;
    real J00, J02, J11, J12;
    real Am[6];
    real dir[3], dlen;
    real Y[16];
} or_proj;

static int finite_all(const real* p, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(p[i])) return 0;
    return 1;
}

/* Rotation R of the normalised quaternion (w, x, y, z), scales s = exp(log-scale),
 * M = R diag(s) and Sigma = M M^T.  Returns 0 for a zero quaternion. */
static int covariance3d(const real* lsc, const real* quat, or_proj* P)
{
    real w = quat[0], x = quat[1], y = quat[2], z = quat[3];
    real n2 = w * w + x * x;
    n2 = n2 + y * y;
    n2 = n2 + z * z;
    real nrm = RSQRT(n2);
    if (!(nrm > 0)) return 0;
    w = w / nrm; x = x / nrm; y = y / nrm; z = z / nrm;
    P->qn[0] = w; P->qn[1] = x; P->qn[2] = y; P->qn[3] = z; P->qnorm = nrm;
    {
        const real xx = x * x, yy = y * y, zz = z * z;
        const real xy = x * y, xz = x * z, yz = y * z;
        const real wx = w * x, wy = w * y, wz = w * z;
        real* R = P->Rq;
        R[0] = (real)1 - (real)2 * (yy + zz);
        R[1] = (real)2 * (xy - wz);
        R[2] = (real)2 * (xz + wy);
        R[3] = (real)2 * (xy + wz);
        R[4] = (real)1 - (real)2 * (xx + zz);
        R[5] = (real)2 * (yz - wx);
        R[6] = (real)2 * (xz - wy);
        R[7] = (real)2 * (yz + wx);
        R[8] = (real)1 - (real)2 * (xx + yy);
    }
    /* Sigma = R S S^T R^T with S = diag(exp(log-scale)) */
    for (int j = 0; j < 3; ++j) P->s[j] = exp_param(lsc[j]);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) P->M[i * 3 + j] = P->Rq[i * 3 + j] * P->s[j];
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) {
            const real* Mi = P->M + i * 3;
            const real* Mj = P->M + j * 3;
            real sij = Mi[0] * Mj[0] + Mi[1] * Mj[1];
            sij = sij + Mi[2] * Mj[2];
            P->Sig[i * 3 + j] = sij;
            P->Sig[j * 3 + i] = sij;
        }
    return 1;
}

static void project_one(const real* mean, const real* lsc, const real* quat, real logit,
                        const real* sh, const or_view* vw, int tile, int cull, or_proj* P)
{
    memset(P, 0, sizeof(*P));
    if (!finite_all(mean, 3) || !finite_all(lsc, 3) || !finite_all(quat, 4) || !isfinite(logit) ||
        !finite_all(sh, 48))
        return;
    if (!covariance3d(lsc, quat, P)) return;

    /* camera-space mean */
    const real W[9] = {vw->R[0], vw->R[1], vw->R[2], vw->R[3], vw->R[4],
                       vw->R[5], vw->R[6], vw->R[7], vw->R[8]};
    for (int i = 0; i < 3; ++i) {
        real pi = W[i * 3 + 0] * (real)mean[0] + W[i * 3 + 1] * (real)mean[1];
        pi = pi + W[i * 3 + 2] * (real)mean[2];
        P->p[i] = pi + (real)vw->t[i];
    }
    const real pz = P->p[2];
    if (!(pz > (real)vw->znear && pz < (real)vw->zfar)) return;
    P->z = pz;

    /* pinhole projection of the mean; pixel (col j, row i) has centre (j+.5, i+.5) */
    const real fx = vw->fx, fy = vw->fy;
    P->tx = P->p[0] / pz;
    P->ty = P->p[1] / pz;
    P->u = fx * P->tx + (real)vw->cx;
    P->v = fy * P->ty + (real)vw->cy;

    /* Jacobian of the pinhole map at the (frustum-clamped) mean */
    P->txc = RMIN((real)vw->lim_x, RMAX(-(real)vw->lim_x, P->tx));
    P->tyc = RMIN((real)vw->lim_y, RMAX(-(real)vw->lim_y, P->ty));
    P->J00 = fx / pz;
    P->J02 = -((fx * P->txc) / pz);
    P->J11 = fy / pz;
    P->J12 = -((fy * P->tyc) / pz);
    for (int j = 0; j < 3; ++j) {
        P->Am[0 * 3 + j] = P->J00 * W[0 * 3 + j] + P->J02 * W[2 * 3 + j];
        P->Am[1 * 3 + j] = P->J11 * W[1 * 3 + j] + P->J12 * W[2 * 3 + j];
    }
    /* Sigma' = Am Sigma Am^T, then the 0.3 low-pass dilation */
    real Tm[6];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) {
            real t = P->Am[i * 3 + 0] * P->Sig[0 * 3 + j] + P->Am[i * 3 + 1] * P->Sig[1 * 3 + j];
            Tm[i * 3 + j] = t + P->Am[i * 3 + 2] * P->Sig[2 * 3 + j];
        }
    real s00 = Tm[0] * P->Am[0] + Tm[1] * P->Am[1];
    s00 = s00 + Tm[2] * P->Am[2];
    real s01 = Tm[0] * P->Am[3] + Tm[1] * P->Am[4];
    s01 = s01 + Tm[2] * P->Am[5];
    real s11 = Tm[3] * P->Am[3] + Tm[4] * P->Am[4];
    s11 = s11 + Tm[5] * P->Am[5];
    const real a = s00 + (real)0.3, b = s01, c = s11 + (real)0.3;
    P->a = a; P->b = b; P->c = c;
    const real det = a * c - b * b;
    if (!(det > 0)) return;
    P->A = c / det;
    P->B = -(b / det);
    P->C = a / det;

    /* 3-sigma radius from the larger eigenvalue, then the tile rectangle:
     * tiles whose span [t*T, (t+1)*T) meets [mean - r, mean + r] on each axis. */
    const real mid = (real)0.5 * (a + c);
    const real dd = a - c;
    real disc = (real)0.25 * (dd * dd) + b * b;
    const real lam = mid + RSQRT(RMAX(disc, (real)0));
    const real r = RCEIL((real)3 * RSQRT(lam));
    P->radius = r;
    const int gx = (vw->width + tile - 1) / tile;
    const int gy = (vw->height + tile - 1) / tile;
    const real invT = (real)1 / (real)tile;
    const real fgx = (real)gx, fgy = (real)gy;
    const real fx0 = RMIN(RMAX(RFLOOR((P->u - r) * invT), (real)0), fgx);
    const real fx1 = RMIN(RMAX(RFLOOR((P->u + r) * invT) + (real)1, (real)0), fgx);
    const real fy0 = RMIN(RMAX(RFLOOR((P->v - r) * invT), (real)0), fgy);
    const real fy1 = RMIN(RMAX(RFLOOR((P->v + r) * invT) + (real)1, (real)0), fgy);
    P->x0 = (int32_t)fx0; P->x1 = (int32_t)fx1;
    P->y0 = (int32_t)fy0; P->y1 = (int32_t)fy1;
    uint32_t count = (uint32_t)((P->x1 - P->x0) * (P->y1 - P->y0));

    /* opacity */
    P->o = sigmoid_param((real)logit);

    if (cull == 1) {
        /* exact culling: rows of the opacity-threshold ellipse, column spans per row;
         * the rectangle becomes the ellipse's bounding tile box */
        or_ellipse e;
        if (!ellipse_setup(P->u, P->v, P->A, P->B, P->C, P->o, &e)) return;
        ellipse_rows(&e, tile, gy, &P->y0, &P->y1);
        P->x0 = (int32_t)RMIN(RMAX(RFLOOR((e.u - e.hx) * invT), (real)0), fgx);
        P->x1 = (int32_t)RMIN(RMAX(RFLOOR((e.u + e.hx) * invT) + (real)1, (real)0), fgx);
        count = 0;
        for (int ty = P->y0; ty < P->y1; ++ty) {
            int xa, xb;
            ellipse_span(&e, tile, gx, ty, &xa, &xb);
            if (xb > xa) count += (uint32_t)(xb - xa);
        }
    }
    if (!(P->x1 > P->x0 && P->y1 > P->y0) || count == 0) return;

    /* view-dependent colour: SH degree 3 along the camera-to-mean direction */
    real dv[3];
    for (int i = 0; i < 3; ++i) dv[i] = (real)mean[i] - (real)vw->campos[i];
    real l2 = dv[0] * dv[0] + dv[1] * dv[1];
    l2 = l2 + dv[2] * dv[2];
    P->dlen = RSQRT(l2);
    if (!(P->dlen > 0)) return;
    for (int i = 0; i < 3; ++i) P->dir[i] = dv[i] / P->dlen;
    sh_basis(P->dir[0], P->dir[1], P->dir[2], P->Y);
    for (int k = 0; k < 3; ++k) {
        real s = (real)sh[0 * 3 + k] * P->Y[0];
        for (int m = 1; m < 16; ++m) s = s + (real)sh[m * 3 + k] * P->Y[m];
        P->raw[k] = s;
        P->col[k] = RMAX(s + (real)0.5, (real)0);
    }

    P->tiles = count;
    P->valid = 1;
}

/* Projection of every Gaussian into every view.  Outputs are indexed
 * [view][gaussian]; float outputs are widened to double for the caller. */
void or_project(const real* means, const real* log_scales, const real* quats,
                const real* logits, const real* sh, int64_t n, const or_view* views, int n_views,
                int tile, int cull, double* xy, double* conic, double* opac, double* rgb,
                double* depth, double* radius, double* cov2d, int32_t* rect, uint32_t* tiles)
{
    for (int vi = 0; vi < n_views; ++vi) {
#pragma omp parallel for schedule(static)
        for (int64_t g = 0; g < n; ++g) {
            or_proj P;
            project_one(means + 3 * g, log_scales + 3 * g, quats + 4 * g, logits[g], sh + 48 * g,
                        views + vi, tile, cull, &P);
            const int64_t o = (int64_t)vi * n + g;
            xy[2 * o + 0] = P.u; xy[2 * o + 1] = P.v;
            conic[3 * o + 0] = P.A; conic[3 * o + 1] = P.B; conic[3 * o + 2] = P.C;
            opac[o] = P.o;
            for (int k = 0; k < 3; ++k) rgb[3 * o + k] = P.col[k];
            depth[o] = P.z;
            radius[o] = P.radius;
            cov2d[3 * o + 0] = P.a; cov2d[3 * o + 1] = P.b; cov2d[3 * o + 2] = P.c;
            rect[4 * o + 0] = P.x0; rect[4 * o + 1] = P.y0;
            rect[4 * o + 2] = P.x1; rect[4 * o + 3] = P.y1;
            tiles[o] = P.valid ? P.tiles : 0u;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Binning: scan, keys, sort, ranges (Sec. 4.1 count-then-fill; Sec. 4.4)     */
/* ------------------------------------------------------------------------- */

/* Exclusive prefix sum of counts[0..m) into offsets[0..m]; returns -1 if the
 * total does not fit in 32 bits. */
int or_scan(const uint32_t* counts, int64_t m, uint32_t* offsets)
{
    uint64_t run = 0;
    for (int64_t i = 0; i < m; ++i) {
        offsets[i] = (uint32_t)run;
        run += counts[i];
        if (run > 0xFFFFFFFFull) return -1;
    }
    offsets[m] = (uint32_t)run;
    return 0;
}

/* Smallest B >= 1 with 2^B >= ntiles, and depth bits D = min(23, 32 - B). */
int or_tile_bits(int ntiles)
{
    int b = 1;
    while ((1 << b) < ntiles) ++b;
    return b;
}
int or_depth_bits(int ntiles)
{
    int b = or_tile_bits(ntiles);
    return (32 - b) < 23 ? (32 - b) : 23;
}

/* Depth key: z > 0 maps to f = (2z+1)/(z+1) in (1, 2); the top D of its 23
 * mantissa bits order depths within a tile. */
uint32_t or_depth_key(float z, int D)
{
    real zr = (real)z;
    real num = (real)2 * zr + (real)1;
    real den = zr + (real)1;
    float f = (float)(num / den);
    uint32_t bits;
    memcpy(&bits, &f, 4);
    return (bits & 0x7FFFFFu) >> (23 - D);
}

/* For each view v and Gaussian g, write one (key, value) per touched tile:
 * rows y0..y1-1 outer, columns inner (x0..x1-1 for the 3-sigma rectangle,
 * the row's span for exact culling), at positions starting at offsets[v*n+g].
 * key = (tile << D) | depth bits; value = the position itself (the unsorted
 * intersection index); gid = g. */
void or_emit_keys(const int32_t* rect, const uint32_t* tiles, const double* depth,
                  const double* xy, const double* conic, const double* opac, int cull,
                  const uint32_t* offsets, int64_t n, const or_view* views, int n_views, int tile,
                  uint32_t* keys, uint32_t* vals, uint32_t* gid)
{
    for (int vi = 0; vi < n_views; ++vi) {
        const int gx = (views[vi].width + tile - 1) / tile;
        const int gy = (views[vi].height + tile - 1) / tile;
        const int D = or_depth_bits(gx * gy);
#pragma omp parallel for schedule(static)
        for (int64_t g = 0; g < n; ++g) {
            const int64_t o = (int64_t)vi * n + g;
            if (tiles[o] == 0) continue;
            uint32_t pos = offsets[o];
            const uint32_t dk = or_depth_key((float)depth[o], D);
            or_ellipse e;
            if (cull == 1)
                ellipse_setup((real)xy[2 * o], (real)xy[2 * o + 1], (real)conic[3 * o],
                              (real)conic[3 * o + 1], (real)conic[3 * o + 2], (real)opac[o], &e);
            for (int ty = rect[4 * o + 1]; ty < rect[4 * o + 3]; ++ty) {
                int xa = rect[4 * o + 0], xb = rect[4 * o + 2];
                if (cull == 1) ellipse_span(&e, tile, gx, ty, &xa, &xb);
                for (int tx = xa; tx < xb; ++tx) {
                    const uint32_t t = (uint32_t)(ty * gx + tx);
                    keys[pos] = (t << D) | dk;
                    vals[pos] = pos;
                    gid[pos] = (uint32_t)g;
                    ++pos;
                }
            }
        }
    }
}

static int cmp_u64(const void* a, const void* b)
{
    const uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

/* Stable ascending sort of (key, value) within each segment
 * [seg_begin[s], seg_begin[s+1]).  Values are distinct and increasing in
 * input order, so ordering by (key, value) is exactly the stable order. */
void or_sort_segments(uint32_t* keys, uint32_t* vals, const uint32_t* seg_begin, int n_seg)
{
    for (int s = 0; s < n_seg; ++s) {
        const uint32_t b = seg_begin[s], e = seg_begin[s + 1];
        const uint32_t len = e - b;
        if (len == 0) continue;
        uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * len);
        for (uint32_t i = 0; i < len; ++i) tmp[i] = ((uint64_t)keys[b + i] << 32) | vals[b + i];
        qsort(tmp, len, sizeof(uint64_t), cmp_u64);
        for (uint32_t i = 0; i < len; ++i) {
            keys[b + i] = (uint32_t)(tmp[i] >> 32);
            vals[b + i] = (uint32_t)tmp[i];
        }
        free(tmp);
    }
}

static uint32_t lower_bound_u64(const uint32_t* k, uint32_t len, uint64_t x)
{
    uint32_t lo = 0, hi = len;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if ((uint64_t)k[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* Per view, per tile t: [start, end) = [lower_bound(t<<D), lower_bound((t+1)<<D))
 * within the view's sorted segment, as global positions. ranges[2*(tile_base+t)]. */
void or_tile_ranges(const uint32_t* keys, const uint32_t* seg_begin, const or_view* views,
                    int n_views, int tile, uint32_t* ranges)
{
    int64_t tb = 0;
    for (int vi = 0; vi < n_views; ++vi) {
        const int gx = (views[vi].width + tile - 1) / tile;
        const int gy = (views[vi].height + tile - 1) / tile;
        const int nt = gx * gy;
        const int D = or_depth_bits(nt);
        const uint32_t b = seg_begin[vi], len = seg_begin[vi + 1] - b;
        for (int t = 0; t < nt; ++t) {
            ranges[2 * (tb + t) + 0] = b + lower_bound_u64(keys + b, len, (uint64_t)t << D);
            ranges[2 * (tb + t) + 1] = b + lower_bound_u64(keys + b, len, (uint64_t)(t + 1) << D);
        }
        tb += nt;
    }
}

/* ------------------------------------------------------------------------- */
/* Rasterisation: front-to-back compositing per pixel over its tile's list    */
/* ------------------------------------------------------------------------- */

typedef struct {
    const double* xy;
    const double* conic;
    const double* opac;
    const double* rgb;
} or_splats;

typedef struct {
    double margin_alpha;  /* relative distance of o*G to 1/255 */
    double margin_clamp;  /* relative distance of o*G to 0.99 */
    double margin_stop;   /* relative distance of T(1-alpha) to 1e-4 */
    double margin_power;  /* |quadratic form| relative to its terms */
    double form_eps;      /* float32 error of the quadratic form per unit of its
                             absolute terms (rounding of products and sums) */
} or_margins;

/* One compositing step, float precision (the paper's).  Returns 0 = skipped,
 * 1 = composited, 2 = stop (not composited).  Sets *fragile when a decision
 * lies within reach of its threshold for a different but equally valid
 * float32 evaluation: the quadratic form d^T Q d carries an absolute rounding
 * error proportional to the sum of its absolute terms (large for elongated
 * Gaussians, where the terms cancel), which moves alpha by that much
 * relatively; transmittance accumulates the alpha errors of the pairs
 * composited before (*terr, relative, in/out). */
static int composite_step(real px, real py, real u, real v, real A, real B, real C, real o,
                          real T, real* alpha_out, real* G_out, real* ag_out, real* dx_out,
                          real* dy_out, const or_margins* mg, int* fragile, double* terr)
{
    const real dx = px - u, dy = py - v;
    const real qa = (A * dx) * dx, qc = (C * dy) * dy, qb = (B * dx) * dy;
    const real power = (real)(-0.5) * (qa + qc) - qb;
    *dx_out = dx; *dy_out = dy;
    double ea = 0.0;
    if (mg) {
        const double form = (double)qa + (double)qc + 2.0 * (double)qb;
        const double mag = fabs((double)qa) + fabs((double)qc) + 2.0 * fabs((double)qb);
        if (fabs(form) <= mg->margin_power * mag) *fragile = 1;
        ea = 0.5 * mg->form_eps * mag;   /* relative error of alpha */
    }
    if (power > (real)0) return 0;
    const real G = REXP(power);
    const real ag = o * G;
    const real alpha = RMIN((real)0.99, ag);
    if (mg) {
        if (fabs((double)ag - 1.0 / 255.0) <= (mg->margin_alpha + ea) * (1.0 / 255.0)) *fragile = 1;
        if (fabs((double)ag - 0.99) <= (mg->margin_clamp + ea) * 0.99) *fragile = 1;
    }
    *G_out = G; *ag_out = ag; *alpha_out = alpha;
    if (alpha < (real)(1.0 / 255.0)) return 0;
    const real test_T = T * ((real)1 - alpha);
    if (mg) {
        const double et = *terr + (ea + mg->margin_alpha) * (double)alpha / (1.0 - (double)alpha);
        if (fabs((double)test_T - 1e-4) <= (mg->margin_stop + et) * 1e-4) *fragile = 1;
        *terr = et;
    }
    if (test_T < (real)1e-4) return 2;
    return 1;
}

static int view_of_tile(const or_view* views, int n_views, int tile, int64_t gtile, int* local,
                        int64_t* pixbase)
{
    int64_t tb = 0, pb = 0;
    for (int vi = 0; vi < n_views; ++vi) {
        const int gx = (views[vi].width + tile - 1) / tile;
        const int gy = (views[vi].height + tile - 1) / tile;
        if (gtile < tb + (int64_t)gx * gy) {
            *local = (int)(gtile - tb);
            *pixbase = pb;
            return vi;
        }
        tb += (int64_t)gx * gy;
        pb += (int64_t)views[vi].width * views[vi].height;
    }
    return -1;
}

/* Forward: image [pixels][3] (views concatenated), T_final, last (entries
 * composited, as list index + 1 of the last composited entry), fragile flag per
 * pixel, and per tile: traversal count (max over pixels of the entries a pixel
 * examined) and the evaluated-pair count. */
void or_raster_fwd(const double* xy, const double* conic, const double* opac, const double* rgb,
                   const uint32_t* ranges, const uint32_t* vals, const uint32_t* gid, int64_t n,
                   const or_view* views, int n_views, int tile, const double* margins,
                   const uint8_t* tile_mask, double* image, double* Tfinal, uint32_t* last,
                   uint8_t* fragile, uint32_t* tile_traversed, uint64_t* tile_evaluated)
{
    int64_t ntiles = 0;
    for (int vi = 0; vi < n_views; ++vi)
        ntiles += (int64_t)((views[vi].width + tile - 1) / tile) *
                  ((views[vi].height + tile - 1) / tile);
    or_margins mg;
    const or_margins* pm = NULL;
    if (margins) {
        mg.margin_alpha = margins[0]; mg.margin_clamp = margins[1];
        mg.margin_stop = margins[2]; mg.margin_power = margins[3];
        mg.form_eps = margins[4];
        pm = &mg;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t gt = 0; gt < ntiles; ++gt) {
        if (tile_mask && !tile_mask[gt]) continue;
        int lt = 0;
        int64_t pixbase = 0;
        const int vi = view_of_tile(views, n_views, tile, gt, &lt, &pixbase);
        const or_view* vw = views + vi;
        const int gx = (vw->width + tile - 1) / tile;
        const int tx = lt % gx, ty = lt / gx;
        const uint32_t start = ranges[2 * gt], end = ranges[2 * gt + 1];
        uint32_t trav = 0;
        uint64_t evals = 0;
        for (int iy = ty * tile; iy < (ty + 1) * tile && iy < vw->height; ++iy)
            for (int ix = tx * tile; ix < (tx + 1) * tile && ix < vw->width; ++ix) {
                const real px = (real)ix + (real)0.5, py = (real)iy + (real)0.5;
                real T = 1;
                acc Cacc[3] = {0, 0, 0};
                uint32_t lst = 0, examined = 0;
                int frag = 0;
                double terr = 0.0;
                for (uint32_t e = start; e < end; ++e) {
                    const int64_t g = (int64_t)vi * n + gid[vals[e]];
                    real alpha = 0, G = 0, ag = 0, dx, dy;
                    ++examined;
                    const int st = composite_step(px, py, (real)xy[2 * g], (real)xy[2 * g + 1],
                                                  (real)conic[3 * g], (real)conic[3 * g + 1],
                                                  (real)conic[3 * g + 2], (real)opac[g], T, &alpha,
                                                  &G, &ag, &dx, &dy, pm, &frag, &terr);
                    if (st == 2) break;
                    if (st == 0) continue;
                    for (int k = 0; k < 3; ++k)
                        Cacc[k] += (acc)alpha * (acc)T * (acc)rgb[3 * g + k];
                    T = T * ((real)1 - alpha);
                    lst = e - start + 1;
                }
                const int64_t pix = pixbase + (int64_t)iy * vw->width + ix;
                for (int k = 0; k < 3; ++k) image[3 * pix + k] = Cacc[k] + (acc)T * (acc)vw->bg[k];
                Tfinal[pix] = T;
                last[pix] = lst;
                if (fragile) fragile[pix] = (uint8_t)frag;
                if (examined > trav) trav = examined;
                evals += examined;
            }
        if (tile_traversed) tile_traversed[gt] = trav;
        if (tile_evaluated) tile_evaluated[gt] = evals;
    }
}

/* L1 loss mean|C - C^| over all channels of all pixels and its gradient
 * sign(C - C^)/count (sign(0) = 0).  Pixels where |C - C^| is within
 * sign_margin of max(|C|, |C^|) in any channel are marked in fragile (if
 * given): there the sign may differ between two float32 implementations.
 * Where last (nullable) says the pixel composited nothing, its colour is the
 * background itself, which every implementation that composites nothing
 * there (the compositing decisions are flagged on their own) reproduces
 * exactly, so its sign is not flagged. */
double or_l1(const double* image, const float* target, int64_t npix, double sign_margin,
             const uint32_t* last, double* dLdC, uint8_t* fragile)
{
    const double inv = 1.0 / (3.0 * (double)npix);
    double loss = 0;
    for (int64_t i = 0; i < 3 * npix; ++i) {
        const double d = image[i] - (double)target[i];
        loss += fabs(d);
        dLdC[i] = d > 0 ? inv : (d < 0 ? -inv : 0.0);
        const double mag = fmax(fabs(image[i]), fabs((double)target[i]));
        const int exact = last && last[i / 3] == 0;
        if (fragile && !exact && mag > 0 && fabs(d) <= sign_margin * mag) fragile[i / 3] = 1;
    }
    return loss * inv;
}

/* Marks in support[view * n + g] every (view, Gaussian) whose compositing at
 * a pixel flagged in pixmask could differ, through a decision taken at a
 * near-tie there, between two float32 implementations.  A pixel adds to a
 * Gaussian's gradient only where it composites that Gaussian (Sec. 4.2), so
 * these are the only gradients a flagged pixel can move.  The pixel's list is
 * walked front to back in float64 with every decision loosened by rel_margin
 * (plus the quadratic form's float32 error, form_eps per unit of its absolute
 * terms) in the direction that keeps more entries: an entry is marked when its
 * alpha reaches (1/255)(1 - margin), transmittance falls by the smallest alpha
 * the margin allows, and the walk stops only where T (1 - alpha) is below
 * 1e-4 (1 - rel_margin) even then. */
void or_pixel_support(const double* xy, const double* conic, const double* opac,
                      const uint32_t* ranges, const uint32_t* vals, const uint32_t* gid, int64_t n,
                      const or_view* views, int n_views, int tile, const uint8_t* pixmask,
                      double rel_margin, double form_eps, uint8_t* support)
{
    int64_t tb = 0, pb = 0;
    for (int vi = 0; vi < n_views; ++vi) {
        const or_view* vw = views + vi;
        const int gx = (vw->width + tile - 1) / tile;
        const int gy = (vw->height + tile - 1) / tile;
        for (int iy = 0; iy < vw->height; ++iy)
            for (int ix = 0; ix < vw->width; ++ix) {
                if (!pixmask[pb + (int64_t)iy * vw->width + ix]) continue;
                const int64_t gt = tb + (int64_t)(iy / tile) * gx + ix / tile;
                const double px = ix + 0.5, py = iy + 0.5;
                double T = 1.0;
                for (uint32_t e = ranges[2 * gt]; e < ranges[2 * gt + 1]; ++e) {
                    const int64_t g = (int64_t)vi * n + gid[vals[e]];
                    const double dx = px - xy[2 * g], dy = py - xy[2 * g + 1];
                    const double qa = conic[3 * g] * dx * dx, qc = conic[3 * g + 2] * dy * dy;
                    const double qb = conic[3 * g + 1] * dx * dy;
                    const double slack = 0.5 * form_eps * (fabs(qa) + fabs(qc) + 2.0 * fabs(qb));
                    const double power = -0.5 * (qa + qc) - qb;
                    const double hi = opac[g] * exp(fmin(0.0, power + slack));
                    const double lo = power - slack > 0.0 ? 0.0 : opac[g] * exp(power - slack);
                    const double m = rel_margin + slack;
                    if (hi < (1.0 / 255.0) * (1.0 - m)) continue;
                    support[g] = 1;
                    const double alpha_lo = lo < (1.0 / 255.0) * (1.0 + m) ? 0.0 : fmin(0.99, lo) * (1.0 - m);
                    if (T * (1.0 - fmin(0.99, hi)) < 1e-4 * (1.0 - rel_margin)) break;
                    T *= 1.0 - alpha_lo;
                }
            }
        tb += (int64_t)gx * gy;
        pb += (int64_t)vw->width * vw->height;
    }
}

/* Backward of compositing.  For each tile and pixel the included entries are
 * found again exactly as in the forward; with S_i the colour composited behind
 * entry i plus T_final * bg:
 *   dL/dc_i     = alpha_i T_i g
 *   dL/dalpha_i = g . (T_i c_i - S_i / (1 - alpha_i))
 * then through alpha = min(0.99, o G), G = exp(power), power = -1/2 d^T Q d
 * (zero through the clamp).  Per-intersection partials (9 values: d mean2d x,y;
 * d conic A,B,C; d opacity; d colour r,g,b) accumulate at the entry's unsorted
 * index; grads2d[view][g][9] sums each Gaussian's intersections in index order.
 * mag2d (nullable, same shape as grads2d) receives, per component, a
 * running error bound in units of the float32 rounding unit (Wilkinson's
 * running error analysis): the sum over pixels of each pixel's term with
 * every factor and every difference inside it taken in absolute value (for
 * dL/dalpha: sum_k |g_k| (T_i |c_ik| + S_ik / (1 - alpha_i))), weighted by
 * the relative error a float32 evaluation of that term can carry: the
 * quadratic form's (twice the sum of its absolute terms, which exp carries
 * into alpha), that of the pixel's final transmittance (each composited
 * entry before adds two roundings and its alpha's error scaled by
 * alpha / (1 - alpha)), and a few roundings more. */
void or_raster_bwd(const double* xy, const double* conic, const double* opac, const double* rgb,
                   const uint32_t* ranges, const uint32_t* vals, const uint32_t* gid,
                   const uint32_t* offsets, int64_t n, const or_view* views, int n_views, int tile,
                   const uint8_t* tile_mask, const double* dLdC, double* partials, double* grads2d,
                   double* mag2d)
{
    int64_t ntiles = 0;
    for (int vi = 0; vi < n_views; ++vi)
        ntiles += (int64_t)((views[vi].width + tile - 1) / tile) *
                  ((views[vi].height + tile - 1) / tile);
    const uint64_t K = offsets[(int64_t)n_views * n];
    memset(partials, 0, sizeof(double) * 9 * K);
    double* pmag = mag2d ? (double*)calloc(9 * (K ? K : 1), sizeof(double)) : NULL;
#pragma omp parallel
    {
        uint32_t cap = 0;
        uint32_t* e_idx = NULL;
        real* e_alpha = NULL;
        real* e_T = NULL;
        real* e_G = NULL;
        real* e_ag = NULL;
        real* e_dx = NULL;
        real* e_dy = NULL;
        double* e_fm = NULL;
#pragma omp for schedule(dynamic, 4)
        for (int64_t gt = 0; gt < ntiles; ++gt) {
            if (tile_mask && !tile_mask[gt]) continue;
            int lt = 0;
            int64_t pixbase = 0;
            const int vi = view_of_tile(views, n_views, tile, gt, &lt, &pixbase);
            const or_view* vw = views + vi;
            const int gx = (vw->width + tile - 1) / tile;
            const int tx = lt % gx, ty = lt / gx;
            const uint32_t start = ranges[2 * gt], end = ranges[2 * gt + 1];
            if (end - start > cap) {
                cap = end - start;
                e_idx = (uint32_t*)realloc(e_idx, sizeof(uint32_t) * cap);
                e_alpha = (real*)realloc(e_alpha, sizeof(real) * cap);
                e_T = (real*)realloc(e_T, sizeof(real) * cap);
                e_G = (real*)realloc(e_G, sizeof(real) * cap);
                e_ag = (real*)realloc(e_ag, sizeof(real) * cap);
                e_dx = (real*)realloc(e_dx, sizeof(real) * cap);
                e_dy = (real*)realloc(e_dy, sizeof(real) * cap);
                e_fm = (double*)realloc(e_fm, sizeof(double) * cap);
            }
            for (int iy = ty * tile; iy < (ty + 1) * tile && iy < vw->height; ++iy)
                for (int ix = tx * tile; ix < (tx + 1) * tile && ix < vw->width; ++ix) {
                    const real px = (real)ix + (real)0.5, py = (real)iy + (real)0.5;
                    real T = 1;
                    uint32_t m = 0;
                    int frag = 0;
                    double rT = 0.0;   /* error bound of T, in rounding units */
                    for (uint32_t e = start; e < end; ++e) {
                        const int64_t g = (int64_t)vi * n + gid[vals[e]];
                        real alpha = 0, G = 0, ag = 0, dx, dy;
                        const int st = composite_step(px, py, (real)xy[2 * g], (real)xy[2 * g + 1],
                                                      (real)conic[3 * g], (real)conic[3 * g + 1],
                                                      (real)conic[3 * g + 2], (real)opac[g], T,
                                                      &alpha, &G, &ag, &dx, &dy, NULL, &frag, NULL);
                        if (st == 2) break;
                        if (st == 0) continue;
                        e_idx[m] = e; e_alpha[m] = alpha; e_T[m] = T; e_G[m] = G; e_ag[m] = ag;
                        e_dx[m] = dx; e_dy[m] = dy;
                        if (pmag) {
                            const double qa = fabs((double)conic[3 * g] * dx * dx);
                            const double qc = fabs((double)conic[3 * g + 2] * dy * dy);
                            const double qb = fabs((double)conic[3 * g + 1] * dx * dy);
                            e_fm[m] = 2.0 * (qa + qc + 2.0 * qb) + 4.0;
                            rT += 2.0 + e_fm[m] * (double)alpha / (1.0 - (double)alpha);
                        }
                        ++m;
                        T = T * ((real)1 - alpha);
                    }
                    const int64_t pix = pixbase + (int64_t)iy * vw->width + ix;
                    const acc gk[3] = {dLdC[3 * pix], dLdC[3 * pix + 1], dLdC[3 * pix + 2]};
                    acc S[3];
                    for (int k = 0; k < 3; ++k) S[k] = (acc)T * (acc)vw->bg[k];
                    for (uint32_t jj = m; jj-- > 0;) {
                        const uint32_t e = e_idx[jj];
                        const int64_t g = (int64_t)vi * n + gid[vals[e]];
                        const acc al = e_alpha[jj], Ti = e_T[jj];
                        const acc c[3] = {rgb[3 * g], rgb[3 * g + 1], rgb[3 * g + 2]};
                        acc* pp = partials + 9 * (uint64_t)vals[e];
                        acc* pm = pmag ? pmag + 9 * (uint64_t)vals[e] : NULL;
                        acc dalpha = 0, dmag = 0;
                        for (int k = 0; k < 3; ++k) {
                            pp[6 + k] += al * Ti * gk[k];
                            dalpha += gk[k] * (Ti * c[k] - S[k] / (1.0 - al));
                            if (pm) {
                                pm[6 + k] += al * Ti * fabs(gk[k]) * (rT + e_fm[jj] + 8.0);
                                dmag += fabs(gk[k]) * (Ti * fabs(c[k]) + fabs(S[k]) / (1.0 - al));
                            }
                        }
                        for (int k = 0; k < 3; ++k) S[k] += al * Ti * c[k];
                        if (e_ag[jj] > (real)0.99) continue; /* clamped: no gradient to o, G */
                        const acc G = e_G[jj];
                        const acc dpow = (acc)e_ag[jj] * dalpha;
                        const acc dx = e_dx[jj], dy = e_dy[jj];
                        const acc A = conic[3 * g], B = conic[3 * g + 1], C = conic[3 * g + 2];
                        pp[5] += G * dalpha;
                        pp[2] += -0.5 * dx * dx * dpow;
                        pp[3] += -dx * dy * dpow;
                        pp[4] += -0.5 * dy * dy * dpow;
                        pp[0] += dpow * (A * dx + B * dy);
                        pp[1] += dpow * (B * dx + C * dy);
                        const double wgt = pm ? rT + e_fm[jj] + 8.0 : 0.0;
                        if (pm) {
                            const acc dpm = (acc)e_ag[jj] * dmag * wgt;
                            pm[5] += G * dmag * wgt;
                            pm[2] += 0.5 * dx * dx * dpm;
                            pm[3] += fabs(dx * dy) * dpm;
                            pm[4] += 0.5 * dy * dy * dpm;
                            pm[0] += dpm * (fabs(A * dx) + fabs(B * dy));
                            pm[1] += dpm * (fabs(B * dx) + fabs(C * dy));
                        }
                    }
                }
        }
        free(e_idx); free(e_alpha); free(e_T); free(e_G); free(e_ag); free(e_dx); free(e_dy);
        free(e_fm);
    }
    /* sum each Gaussian's intersections, in index order */
#pragma omp parallel for schedule(static)
    for (int64_t o = 0; o < (int64_t)n_views * n; ++o) {
        acc s[9] = {0};
        for (uint32_t i = offsets[o]; i < offsets[o + 1]; ++i)
            for (int k = 0; k < 9; ++k) s[k] += partials[9 * (uint64_t)i + k];
        for (int k = 0; k < 9; ++k) grads2d[9 * o + k] = s[k];
        if (pmag) {
            acc sm[9] = {0};
            for (uint32_t i = offsets[o]; i < offsets[o + 1]; ++i)
                for (int k = 0; k < 9; ++k) sm[k] += pmag[9 * (uint64_t)i + k];
            for (int k = 0; k < 9; ++k) mag2d[9 * o + k] = sm[k];
        }
    }
    free(pmag);
}

/* ------------------------------------------------------------------------- */
/* Projection backward: chain rule from the 2D quantities to the parameters   */
/* ------------------------------------------------------------------------- */

/* grads[g][59] in the canonical order: mean(3), log-scale(3), quaternion(4),
 * opacity logit(1), SH coefficient m*3+k (48).  Sums over views. */
void or_project_bwd(const real* means, const real* log_scales, const real* quats,
                    const real* logits, const real* sh, int64_t n, const or_view* views,
                    int n_views, int tile, int cull, const double* grads2d, double* grads)
{
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
        acc G[59];
        memset(G, 0, sizeof(G));
        for (int vi = 0; vi < n_views; ++vi) {
            or_proj P;
            project_one(means + 3 * g, log_scales + 3 * g, quats + 4 * g, logits[g], sh + 48 * g,
                        views + vi, tile, cull, &P);
            if (!P.valid) continue;
            const acc* d2 = grads2d + 9 * ((int64_t)vi * n + g);
            const acc du = d2[0], dv = d2[1], dA = d2[2], dB = d2[3], dC = d2[4], dop = d2[5];
            const or_view* vw = views + vi;
            const acc W[9] = {vw->R[0], vw->R[1], vw->R[2], vw->R[3], vw->R[4],
                              vw->R[5], vw->R[6], vw->R[7], vw->R[8]};
            acc dmean[3] = {0, 0, 0};

            /* colour: c = max(0, raw + 1/2), raw = sum_m sh[m] Y_m(dir) */
            acc draw[3];
            for (int k = 0; k < 3; ++k)
                draw[k] = ((acc)P.raw[k] + 0.5 >= 0.0) ? d2[6 + k] : 0.0;
            for (int m = 0; m < 16; ++m)
                for (int k = 0; k < 3; ++k) G[11 + m * 3 + k] += (acc)P.Y[m] * draw[k];
            {
                acc dY[16][3];
                sh_basis_grad(P.dir[0], P.dir[1], P.dir[2], dY);
                acc ddir[3] = {0, 0, 0};
                for (int m = 1; m < 16; ++m) {
                    acc w = 0;
                    for (int k = 0; k < 3; ++k) w += (acc)sh[48 * g + m * 3 + k] * draw[k];
                    for (int i = 0; i < 3; ++i) ddir[i] += w * dY[m][i];
                }
                const acc d0 = P.dir[0], d1 = P.dir[1], d2d = P.dir[2];
                const acc dd = d0 * ddir[0] + d1 * ddir[1] + d2d * ddir[2];
                const acc L = P.dlen;
                dmean[0] += (ddir[0] - d0 * dd) / L;
                dmean[1] += (ddir[1] - d1 * dd) / L;
                dmean[2] += (ddir[2] - d2d * dd) / L;
            }

            /* opacity: o = sigmoid(logit) */
            G[10] += dop * (acc)P.o * (1.0 - (acc)P.o);

            /* conic -> 2D covariance: dSigma' = -Q Gbar Q with Q = [[A,B],[B,C]] and
             * Gbar = [[dA, dB/2],[dB/2, dC]] (B occupies both off-diagonal slots). */
            const acc A = P.A, B = P.B, C = P.C;
            const acc g11 = dA, g12 = 0.5 * dB, g22 = dC;
            const acc q00 = A * g11 + B * g12, q01 = A * g12 + B * g22;
            const acc q10 = B * g11 + C * g12, q11 = B * g12 + C * g22;
            const acc dS00 = -(q00 * A + q01 * B);
            const acc dS01 = -(q00 * B + q01 * C);
            const acc dS11 = -(q10 * B + q11 * C);
            const acc dS[4] = {dS00, dS01, dS01, dS11};

            /* Sigma' = Am Sigma Am^T: dSigma = Am^T dS Am, dAm = 2 dS Am Sigma */
            acc Am[6], Sig[9];
            for (int i = 0; i < 6; ++i) Am[i] = P.Am[i];
            for (int i = 0; i < 9; ++i) Sig[i] = P.Sig[i];
            acc dSig[9];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    acc s = 0;
                    for (int k = 0; k < 2; ++k)
                        for (int l = 0; l < 2; ++l) s += Am[k * 3 + i] * dS[k * 2 + l] * Am[l * 3 + j];
                    dSig[i * 3 + j] = s;
                }
            acc dAm[6];
            for (int k = 0; k < 2; ++k)
                for (int j = 0; j < 3; ++j) {
                    acc s = 0;
                    for (int l = 0; l < 2; ++l)
                        for (int m = 0; m < 3; ++m) s += dS[k * 2 + l] * Am[l * 3 + m] * Sig[m * 3 + j];
                    dAm[k * 3 + j] = 2.0 * s;
                }

            /* Sigma = M M^T, M = R diag(s): dM = 2 dSigma M */
            acc dM[9];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    acc s = 0;
                    for (int k = 0; k < 3; ++k) s += dSig[i * 3 + k] * (acc)P.M[k * 3 + j];
                    dM[i * 3 + j] = 2.0 * s;
                }
            acc dR[9];
            for (int j = 0; j < 3; ++j) {
                acc ds = 0;
                for (int i = 0; i < 3; ++i) {
                    ds += dM[i * 3 + j] * (acc)P.Rq[i * 3 + j];
                    dR[i * 3 + j] = dM[i * 3 + j] * (acc)P.s[j];
                }
                G[3 + j] += ds * (acc)P.s[j]; /* d log-scale = ds * s */
            }
            /* rotation matrix of the unit quaternion (w, x, y, z) */
            {
                const acc w = P.qn[0], x = P.qn[1], y = P.qn[2], z = P.qn[3];
                acc dq[4];
                dq[0] = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
                dq[1] = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] +
                               z * dR[6] + w * dR[7] - 2.0 * x * dR[8]);
                dq[2] = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] -
                               w * dR[6] + z * dR[7] - 2.0 * y * dR[8]);
                dq[3] = 2.0 * (-2.0 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] -
                               2.0 * z * dR[4] + y * dR[5] + x * dR[6] + y * dR[7]);
                /* through the normalisation q^ = q / |q| */
                const acc qh[4] = {w, x, y, z};
                const acc dot = qh[0] * dq[0] + qh[1] * dq[1] + qh[2] * dq[2] + qh[3] * dq[3];
                for (int i = 0; i < 4; ++i) G[6 + i] += (dq[i] - qh[i] * dot) / (acc)P.qnorm;
            }

            /* Am = J W: dJ = dAm W^T; J depends on the camera-space mean p */
            const acc z = P.z, x = P.p[0], y = P.p[1];
            const acc fx = vw->fx, fy = vw->fy;
            const acc dJ00 = dAm[0] * W[0] + dAm[1] * W[1] + dAm[2] * W[2];
            const acc dJ02 = dAm[0] * W[6] + dAm[1] * W[7] + dAm[2] * W[8];
            const acc dJ11 = dAm[3] * W[3] + dAm[4] * W[4] + dAm[5] * W[5];
            const acc dJ12 = dAm[3] * W[6] + dAm[4] * W[7] + dAm[5] * W[8];
            acc dp[3] = {0, 0, 0};
            dp[2] += dJ00 * (-fx / (z * z));
            dp[2] += dJ11 * (-fy / (z * z));
            /* J02 = -fx txc / z, txc = clamp(x / z) */
            dp[2] += dJ02 * (fx * (acc)P.txc / (z * z));
            if (P.tx == P.txc) {
                const acc dtxc = dJ02 * (-fx / z);
                dp[0] += dtxc / z;
                dp[2] += dtxc * (-x / (z * z));
            }
            dp[2] += dJ12 * (fy * (acc)P.tyc / (z * z));
            if (P.ty == P.tyc) {
                const acc dtyc = dJ12 * (-fy / z);
                dp[1] += dtyc / z;
                dp[2] += dtyc * (-y / (z * z));
            }
            /* mean 2D: u = fx x/z + cx, v = fy y/z + cy */
            dp[0] += du * fx / z;
            dp[2] += du * (-fx * x / (z * z));
            dp[1] += dv * fy / z;
            dp[2] += dv * (-fy * y / (z * z));
            /* p = W mean + t */
            for (int i = 0; i < 3; ++i)
                dmean[i] += W[0 * 3 + i] * dp[0] + W[1 * 3 + i] * dp[1] + W[2 * 3 + i] * dp[2];
            for (int i = 0; i < 3; ++i) G[i] += dmean[i];
        }
        for (int k = 0; k < 59; ++k) grads[59 * g + k] = G[k];
    }
}

/* ------------------------------------------------------------------------- */
/* Adam (Kingma & Ba; the bias-corrected form of torch.optim.Adam)            */
/* ------------------------------------------------------------------------- */

/* Parameter groups by canonical index: 0-2 means, 3-5 log-scales, 6-9
 * quaternion, 10 opacity logit, 11-13 SH DC, 14-58 SH rest. */
static int param_group(int k)
{
    if (k < 3) return 0;
    if (k < 6) return 1;
    if (k < 10) return 2;
    if (k < 11) return 3;
    if (k < 14) return 4;
    return 5;
}

void or_adam(float* params, float* m, float* v, const double* grads, int64_t n, const double* lr,
             double beta1, double beta2, double eps, int step)
{
    const double bc1 = 1.0 - pow(beta1, step);
    const double bc2 = 1.0 - pow(beta2, step);
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g)
        for (int k = 0; k < 59; ++k) {
            const int64_t i = 59 * g + k;
            const double gr = grads[i];
            const double mm = beta1 * (double)m[i] + (1.0 - beta1) * gr;
            const double vv = beta2 * (double)v[i] + (1.0 - beta2) * gr * gr;
            const double denom = sqrt(vv) / sqrt(bc2) + eps;
            params[i] = (float)((double)params[i] - (lr[param_group(k)] / bc1) * mm / denom);
            m[i] = (float)mm;
            v[i] = (float)vv;
        }
}

/* ------------------------------------------------------------------------- */
/* Small entry points for the checks                                          */
/* ------------------------------------------------------------------------- */

/* R (row major) and Sigma of one Gaussian; returns 0 for a zero quaternion. */
int or_cov3d(const real* log_scale, const real* quat, double* R, double* Sig)
{
    or_proj P;
    memset(&P, 0, sizeof(P));
    if (!covariance3d(log_scale, quat, &P)) return 0;
    for (int i = 0; i < 9; ++i) { R[i] = P.Rq[i]; Sig[i] = P.Sig[i]; }
    return 1;
}

void or_sh_basis(const double* dir, double* Y)
{
    real y16[16];
    sh_basis((real)dir[0], (real)dir[1], (real)dir[2], y16);
    for (int i = 0; i < 16; ++i) Y[i] = y16[i];
}

double or_exp_param(double x) { return (double)exp_param((real)x); }
double or_log_spec(double x) { return (double)log_spec((real)x); }

/* Tile set of one screen-space Gaussian under exact culling, for tests:
 * writes 1 into mask[ty * gx + tx] for each listed tile; returns the count
 * (0 if the Gaussian is culled). */
int or_ellipse_tiles(double u, double v, double A, double B, double C, double o, int tile, int gx,
                     int gy, uint8_t* mask)
{
    or_ellipse e;
    if (!ellipse_setup((real)u, (real)v, (real)A, (real)B, (real)C, (real)o, &e)) return 0;
    int y0, y1, count = 0;
    ellipse_rows(&e, tile, gy, &y0, &y1);
    for (int ty = y0; ty < y1; ++ty) {
        int xa, xb;
        ellipse_span(&e, tile, gx, ty, &xa, &xb);
        for (int tx = xa; tx < xb; ++tx) { mask[ty * gx + tx] = 1; ++count; }
    }
    return count;
}
double or_sigmoid(double x) { return (double)sigmoid_param((real)x); }

int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int or_is_double(void)
{
#ifdef OR_DOUBLE
    return 1;
#else
    return 0;
#endif
}
