// EWA projection of one Gaussian into one view, float32, no contraction.
//
// Every float step that decides the tile rectangle (and therefore the sort
// keys and tile lists) is written as a fixed sequence of IEEE single
// operations, so the rectangle is a deterministic function of the inputs:
// the translation unit is compiled with -ffp-contract=off and the only
// transcendental, e^x for the scale and opacity activations, is evaluated by
// Cody & Waite's argument reduction with a degree-7 Taylor polynomial and an
// exact power-of-two scaling (each step one IEEE operation), not by a
// hardware approximation.  Division and square root are correctly rounded
// (the HIP default on gfx950).
#pragma once

#include "cull_math.h"
#include "gs_internal.h"

#pragma clang fp contract(off)

namespace gs {

// e^x: x = n ln2 + r, ln2 split in a high part with trailing zero bits (so
// n*ln2_hi is exact for |n| < 512) and a low part; e^r by Horner; 2^n exactly.
GS_DEV float exp_cw(float x) {
    if (x != x) return x;
    if (x > 100.0f) x = 100.0f;
    if (x < -100.0f) x = -100.0f;
    const float log2e = 0x1.715476p+0f;
    const float ln2_hi = 0x1.62e4p-1f;
    const float ln2_lo = 0x1.7f7d1cp-20f;
    const float n = __builtin_rintf(x * log2e);
    const float r = (x - n * ln2_hi) - n * ln2_lo;
    float p = 0x1.a01a02p-13f;   // 1/7!
    p = p * r + 0x1.6c16c2p-10f; // 1/6!
    p = p * r + 0x1.111112p-7f;  // 1/5!
    p = p * r + 0x1.555556p-5f;  // 1/4!
    p = p * r + 0x1.555556p-3f;  // 1/3!
    p = p * r + 0.5f;
    p = p * r + 1.0f;
    p = p * r + 1.0f;
    return __builtin_ldexpf(p, (int)n);
}

// Real spherical harmonics, degree <= 3, orthonormal on the sphere.
constexpr float kSH0 = 0x1.20dd76p-2f;    // 1/(2 sqrt(pi))
constexpr float kSH1 = 0x1.f45438p-2f;    // sqrt(3/(4 pi))
constexpr float kSH2a = 0x1.17b142p+0f;   // sqrt(15/pi)/2
constexpr float kSH2c = 0x1.42f602p-2f;   // sqrt(5/pi)/4
constexpr float kSH2e = 0x1.17b142p-1f;   // sqrt(15/pi)/4
constexpr float kSH3a = -0x1.2e1a32p-1f;  // -sqrt(35/(2 pi))/4
constexpr float kSH3b = 0x1.71ff8ep+1f;   // sqrt(105/pi)/2
constexpr float kSH3c = -0x1.d403d0p-2f;  // -sqrt(21/(2 pi))/4
constexpr float kSH3d = 0x1.7e21f0p-2f;   // sqrt(7/pi)/4
constexpr float kSH3f = 0x1.71ff8ep+0f;   // sqrt(105/pi)/4

GS_DEV void sh_eval(float x, float y, float z, float Y[16]) {
    const float xx = x * x, yy = y * y, zz = z * z;
    const float xy = x * y, yz = y * z, xz = x * z;
    Y[0] = kSH0;
    Y[1] = -(kSH1 * y);
    Y[2] = kSH1 * z;
    Y[3] = -(kSH1 * x);
    Y[4] = kSH2a * xy;
    Y[5] = (-kSH2a) * yz;
    Y[6] = kSH2c * ((2.0f * zz - xx) - yy);
    Y[7] = (-kSH2a) * xz;
    Y[8] = kSH2e * (xx - yy);
    Y[9] = (kSH3a * y) * (3.0f * xx - yy);
    Y[10] = (kSH3b * xy) * z;
    Y[11] = (kSH3c * y) * ((4.0f * zz - xx) - yy);
    Y[12] = (kSH3d * z) * ((2.0f * zz - 3.0f * xx) - 3.0f * yy);
    Y[13] = (kSH3c * x) * ((4.0f * zz - xx) - yy);
    Y[14] = (kSH3f * z) * (xx - yy);
    Y[15] = (kSH3a * x) * (xx - 3.0f * yy);
}

struct Proj {
    bool valid;
    float u, v, z;
    float a, b, c;     // 2D covariance incl. 0.3 dilation
    float A, B, C;     // conic
    float o;
    float col[3], raw[3];
    float radius;
    int x0, y0, x1, y1;   // bounding tile box of the tile set
    uint32_t count;       // tiles in the set
    // kept for the backward
    float qn[4], qnorm;
    float Rq[9];
    float s[3];
    float M[9];
    float Sig[6];      // 00 01 02 11 12 22
    float p[3];
    float tx, ty, txc, tyc;
    float J00, J02, J11, J12;
    float Am[6];
    float dir[3], dlen;
    float Y[16];
};

GS_DEV bool finite4(float4 a) {
    return __builtin_isfinite(a.x) && __builtin_isfinite(a.y) && __builtin_isfinite(a.z) &&
           __builtin_isfinite(a.w);
}

GS_DEV float sig_at(const float S[6], int i, int j) {
    // symmetric 3x3 stored 00 01 02 11 12 22
    const int a = i < j ? i : j, b = i < j ? j : i;
    return a == 0 ? S[b] : (a == 1 ? S[2 + b] : S[5]);
}

// Projects Gaussian (p0 = mean xyz + logit, p1 = log-scales, p2 = quaternion
// wxyz, sh = 48 coefficients) into view vw with tile edge T.  With
// want_colour = false the SH colour is skipped (binning only needs geometry).
// cull selects the tile set (GS_CULL_RECT / GS_CULL_ELLIPSE); with kCount the
// set is counted into P.count and an empty set culls the Gaussian (callers
// that already know the Gaussian has tiles pass kCount = false).
template <bool kColour, bool kCount = true>
GS_DEV void project_gaussian(float4 p0, float4 p1, float4 p2, const float4* sh, const gs_view& vw,
                             int tile, int gx, int gy, int cull, Proj& P) {
    P.valid = false;
    // quaternion -> rotation
    float w = p2.x, x = p2.y, y = p2.z, z = p2.w;
    float n2 = w * w + x * x;
    n2 = n2 + y * y;
    n2 = n2 + z * z;
    const float nrm = __builtin_sqrtf(n2);
    if (!(nrm > 0.0f)) return;
    w = w / nrm; x = x / nrm; y = y / nrm; z = z / nrm;
    P.qn[0] = w; P.qn[1] = x; P.qn[2] = y; P.qn[3] = z; P.qnorm = nrm;
    {
        const float xx = x * x, yy = y * y, zz = z * z;
        const float xy = x * y, xz = x * z, yz = y * z;
        const float wx = w * x, wy = w * y, wz = w * z;
        P.Rq[0] = 1.0f - 2.0f * (yy + zz);
        P.Rq[1] = 2.0f * (xy - wz);
        P.Rq[2] = 2.0f * (xz + wy);
        P.Rq[3] = 2.0f * (xy + wz);
        P.Rq[4] = 1.0f - 2.0f * (xx + zz);
        P.Rq[5] = 2.0f * (yz - wx);
        P.Rq[6] = 2.0f * (xz - wy);
        P.Rq[7] = 2.0f * (yz + wx);
        P.Rq[8] = 1.0f - 2.0f * (xx + yy);
    }
    P.s[0] = exp_cw(p1.x);
    P.s[1] = exp_cw(p1.y);
    P.s[2] = exp_cw(p1.z);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) P.M[i * 3 + j] = P.Rq[i * 3 + j] * P.s[j];
    {
        int k = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) {
                float sij = P.M[i * 3 + 0] * P.M[j * 3 + 0] + P.M[i * 3 + 1] * P.M[j * 3 + 1];
                sij = sij + P.M[i * 3 + 2] * P.M[j * 3 + 2];
                P.Sig[k++] = sij;
            }
    }
    // camera-space mean
    const float mu[3] = {p0.x, p0.y, p0.z};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        float pi = vw.R[i * 3 + 0] * mu[0] + vw.R[i * 3 + 1] * mu[1];
        pi = pi + vw.R[i * 3 + 2] * mu[2];
        P.p[i] = pi + vw.t[i];
    }
    const float pz = P.p[2];
    if (!(pz > vw.znear && pz < vw.zfar)) return;
    P.z = pz;
    const float fx = vw.fx, fy = vw.fy;
    P.tx = P.p[0] / pz;
    P.ty = P.p[1] / pz;
    P.u = fx * P.tx + vw.cx;
    P.v = fy * P.ty + vw.cy;
    P.txc = fminf(vw.lim_x, fmaxf(-vw.lim_x, P.tx));
    P.tyc = fminf(vw.lim_y, fmaxf(-vw.lim_y, P.ty));
    P.J00 = fx / pz;
    P.J02 = -((fx * P.txc) / pz);
    P.J11 = fy / pz;
    P.J12 = -((fy * P.tyc) / pz);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        P.Am[j] = P.J00 * vw.R[j] + P.J02 * vw.R[6 + j];
        P.Am[3 + j] = P.J11 * vw.R[3 + j] + P.J12 * vw.R[6 + j];
    }
    float Tm[6];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            float t = P.Am[i * 3 + 0] * sig_at(P.Sig, 0, j) + P.Am[i * 3 + 1] * sig_at(P.Sig, 1, j);
            Tm[i * 3 + j] = t + P.Am[i * 3 + 2] * sig_at(P.Sig, 2, j);
        }
    float s00 = Tm[0] * P.Am[0] + Tm[1] * P.Am[1];
    s00 = s00 + Tm[2] * P.Am[2];
    float s01 = Tm[0] * P.Am[3] + Tm[1] * P.Am[4];
    s01 = s01 + Tm[2] * P.Am[5];
    float s11 = Tm[3] * P.Am[3] + Tm[4] * P.Am[4];
    s11 = s11 + Tm[5] * P.Am[5];
    const float a = s00 + 0.3f, b = s01, c = s11 + 0.3f;
    P.a = a; P.b = b; P.c = c;
    const float det = a * c - b * b;
    if (!(det > 0.0f)) return;
    P.A = c / det;
    P.B = -(b / det);
    P.C = a / det;
    const float mid = 0.5f * (a + c);
    const float dd = a - c;
    const float disc = 0.25f * (dd * dd) + b * b;
    const float lam = mid + __builtin_sqrtf(fmaxf(disc, 0.0f));
    const float r = __builtin_ceilf(3.0f * __builtin_sqrtf(lam));
    P.radius = r;
    const float invT = 1.0f / (float)tile;
    const float fgx = (float)gx, fgy = (float)gy;
    const float fx0 = fminf(fmaxf(__builtin_floorf((P.u - r) * invT), 0.0f), fgx);
    const float fx1 = fminf(fmaxf(__builtin_floorf((P.u + r) * invT) + 1.0f, 0.0f), fgx);
    const float fy0 = fminf(fmaxf(__builtin_floorf((P.v - r) * invT), 0.0f), fgy);
    const float fy1 = fminf(fmaxf(__builtin_floorf((P.v + r) * invT) + 1.0f, 0.0f), fgy);
    P.x0 = (int)fx0; P.x1 = (int)fx1; P.y0 = (int)fy0; P.y1 = (int)fy1;
    P.o = 1.0f / (1.0f + exp_cw(-p0.w));
    uint32_t count = (uint32_t)((P.x1 - P.x0) * (P.y1 - P.y0));
    if (cull == GS_CULL_ELLIPSE) {
        Ellipse e;
        if (!ellipse_setup(P.u, P.v, P.A, P.B, P.C, P.o, e)) return;
        ellipse_rows(e, tile, gy, P.y0, P.y1);
        ellipse_cols(e, tile, gx, P.x0, P.x1);
        count = 0;
        if (kCount) {
            for (int ty = P.y0; ty < P.y1; ++ty) {
                int xa, xb;
                ellipse_span(e, tile, gx, ty, xa, xb);
                count += xb > xa ? (uint32_t)(xb - xa) : 0u;
            }
        }
    }
    if (!(P.x1 > P.x0 && P.y1 > P.y0) || (kCount && count == 0)) return;
    P.count = count;
    // view direction and colour
    float dv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) dv[i] = mu[i] - vw.campos[i];
    float l2 = dv[0] * dv[0] + dv[1] * dv[1];
    l2 = l2 + dv[2] * dv[2];
    P.dlen = __builtin_sqrtf(l2);
    if (!(P.dlen > 0.0f)) return;
#pragma unroll
    for (int i = 0; i < 3; ++i) P.dir[i] = dv[i] / P.dlen;
    if (kColour) {
        sh_eval(P.dir[0], P.dir[1], P.dir[2], P.Y);
        float c[48];
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            const float4 f = sh[q];
            c[4 * q + 0] = f.x; c[4 * q + 1] = f.y; c[4 * q + 2] = f.z; c[4 * q + 3] = f.w;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float s = c[k] * P.Y[0];
#pragma unroll
            for (int m = 1; m < 16; ++m) s = s + c[m * 3 + k] * P.Y[m];
            P.raw[k] = s;
            P.col[k] = fmaxf(s + 0.5f, 0.0f);
        }
    }
    P.valid = true;
}

}  // namespace gs
