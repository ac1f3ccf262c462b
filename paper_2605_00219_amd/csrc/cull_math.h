// Tile sets of a projected Gaussian (Sec. 4.1).
//
// 3-sigma rectangle: the tiles whose span meets [mean - r, mean + r] on both
// axes, r = ceil(3 sqrt(lambda_max)).
//
// Exact culling: the tiles whose square meets the ellipse where the Gaussian
// can still reach alpha >= 1/255, i.e. the offsets d from the 2D mean with
// A dx^2 + 2 B dx dy + C dy^2 <= tau, tau = 2 ln(255 o).  The tile rows are
// those meeting [v - hy, v + hy]; within a row band [ya, yb] the ellipse's
// x-extent is its global extreme when the extreme point's height lies in the
// band, else the boundary at one of the band's edges, and the column span is
// that extent rounded outwards to tile boundaries.  Every step is one IEEE
// float operation in a fixed order (the translation units that include this
// are built without contraction), so the tile set is reproducible bit for
// bit wherever it is evaluated: projection counts it, binning enumerates it.
#pragma once

#include "gs_internal.h"

#pragma clang fp contract(off)

namespace gs {

// ln x for finite x >= 1: x = m 2^k with m in [1/sqrt 2, sqrt 2), ln m =
// 2 atanh(s), s = (m - 1)/(m + 1), by the odd series to s^13 in Horner form
// (coefficients: the float32 values nearest 2/(2j+1)), then k ln 2 with ln 2
// split in two parts.
GS_DEV float log_cull(float x) {
    const uint32_t bits = __float_as_uint(x);
    int k = (int)((bits >> 23) & 0xFFu) - 126;
    float m = __uint_as_float((bits & 0x7FFFFFu) | 0x3F000000u);   // [0.5, 1)
    if (m < 0.70710676908493042f) { m = m * 2.0f; k = k - 1; }
    const float s = (m - 1.0f) / (m + 1.0f);
    const float z = s * s;
    float p = 0.15384615957736969f;
    p = p * z + 0.18181818723678589f;
    p = p * z + 0.22222222387790680f;
    p = p * z + 0.28571429848670959f;
    p = p * z + 0.40000000596046448f;
    p = p * z + 0.66666668653488159f;
    p = p * z + 2.0f;
    const float lm = s * p;
    const float fk = (float)k;
    return fk * 0.693145751953125f + (fk * 1.4286067653301870e-06f + lm);
}

struct Ellipse {
    float u, v, A, B, C, tau, dQ, hx, hy, ys;
};

// false: the Gaussian cannot reach alpha 1/255 anywhere (or its conic is degenerate)
GS_DEV bool ellipse_setup(float u, float v, float A, float B, float C, float o, Ellipse& e) {
    const float x = 255.0f * o;
    if (!(x > 1.0f)) return false;
    e.u = u; e.v = v; e.A = A; e.B = B; e.C = C;
    e.tau = 2.0f * log_cull(x);
    e.dQ = A * C - B * B;
    if (!(e.dQ > 0.0f) || !(A > 0.0f) || !(C > 0.0f)) return false;
    e.hx = __builtin_sqrtf((e.tau * C) / e.dQ);
    e.hy = __builtin_sqrtf((e.tau * A) / e.dQ);
    e.ys = -((B * e.hx) / C);   // height of the rightmost point
    return true;
}

// right / left boundary offset at height dy
GS_DEV float ellipse_xp(const Ellipse& e, float dy) {
    float w = e.A * e.tau - e.dQ * (dy * dy);
    w = fmaxf(w, 0.0f);
    return (__builtin_sqrtf(w) - e.B * dy) / e.A;
}
GS_DEV float ellipse_xm(const Ellipse& e, float dy) {
    float w = e.A * e.tau - e.dQ * (dy * dy);
    w = fmaxf(w, 0.0f);
    return (-__builtin_sqrtf(w) - e.B * dy) / e.A;
}

GS_DEV void ellipse_rows(const Ellipse& e, int tile, int gy, int& y0, int& y1) {
    const float invT = 1.0f / (float)tile;
    const float fgy = (float)gy;
    y0 = (int)fminf(fmaxf(__builtin_floorf((e.v - e.hy) * invT), 0.0f), fgy);
    y1 = (int)fminf(fmaxf(__builtin_floorf((e.v + e.hy) * invT) + 1.0f, 0.0f), fgy);
}

GS_DEV void ellipse_cols(const Ellipse& e, int tile, int gx, int& x0, int& x1) {
    const float invT = 1.0f / (float)tile;
    const float fgx = (float)gx;
    x0 = (int)fminf(fmaxf(__builtin_floorf((e.u - e.hx) * invT), 0.0f), fgx);
    x1 = (int)fminf(fmaxf(__builtin_floorf((e.u + e.hx) * invT) + 1.0f, 0.0f), fgx);
}

// column span [xa, xb) of tile row ty (empty if xb <= xa)
GS_DEV void ellipse_span(const Ellipse& e, int tile, int gx, int ty, int& xa, int& xb) {
    const float invT = 1.0f / (float)tile;
    const float fgx = (float)gx;
    float ya = (float)(ty * tile) - e.v;
    float yb = (float)((ty + 1) * tile) - e.v;
    ya = fmaxf(ya, -e.hy);
    yb = fminf(yb, e.hy);
    const float xmax = (ya <= e.ys && e.ys <= yb) ? e.hx : fmaxf(ellipse_xp(e, ya), ellipse_xp(e, yb));
    const float xmin = (ya <= -e.ys && -e.ys <= yb) ? -e.hx
                                                     : fminf(ellipse_xm(e, ya), ellipse_xm(e, yb));
    xa = (int)fminf(fmaxf(__builtin_floorf((e.u + xmin) * invT), 0.0f), fgx);
    xb = (int)fminf(fmaxf(__builtin_floorf((e.u + xmax) * invT) + 1.0f, 0.0f), fgx);
}

}  // namespace gs
