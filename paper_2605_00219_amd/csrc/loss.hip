// Fused L1 + D-SSIM loss gradient against an RGBA8 reference (Sec. 4.5):
// L = (1 - lam)/(3P) sum m |x - y| + lam/(3P) sum m (1 - S), per colour
// channel, x the render, y = rgb / 255, m = alpha / 255 (or 1).  S is the SSIM
// map of each channel with an 11 x 11 Gaussian window (sigma 1.5), zero
// outside each view's image.
//
// Two kernels over 16 x 16 output blocks of each view, each staging its block
// plus a 5-pixel halo in LDS and summing the window separably (rows, then
// columns):
//   k_ssim_fwd  window moments of x, y, x^2, y^2, xy -> S and the coefficient
//               maps a = m dS/dmu_x, b = m dS/dE[x^2], c = m dS/dE[xy]
//               (9 floats per pixel in the workspace), per-block loss sums;
//   k_ssim_bwd  window sums of a, b, c -> dL/dx = (1 - lam)/(3P) m sign(x - y)
//               - lam/(3P) (G*a + 2 x G*b + y G*c).
// The reference stays 4 x uint8 per pixel; the render stays channel-last.
#include <cmath>

#include "gs_internal.h"

namespace gs {

constexpr int kLB = 16;              // output block edge
constexpr int kHalo = 5;             // window radius
constexpr int kLR = kLB + 2 * kHalo; // staged region edge (26)
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct LossGeo {
    int32_t width[GS_MAX_VIEWS], height[GS_MAX_VIEWS];
    int64_t pixel_base[GS_MAX_VIEWS];
    int32_t block_base[GS_MAX_VIEWS + 1];   // first 16 x 16 block of each view
    int32_t blocks_x[GS_MAX_VIEWS];
    int n_views;
    float win[2 * kHalo + 1];               // normalised 1-D Gaussian window
    float l1_scale, ssim_scale;             // (1 - lam)/(3P), lam/(3P)
    int use_mask;
};

struct BlockPos {
    int view, x0, y0, W, H;
    int64_t base;
};

GS_DEV BlockPos block_pos(const LossGeo& g, int blk) {
    BlockPos p;
    int v = 0;
    for (int i = 1; i < g.n_views; ++i)
        if (blk >= g.block_base[i]) v = i;
    const int lb = blk - g.block_base[v];
    p.view = v;
    p.x0 = (lb % g.blocks_x[v]) * kLB;
    p.y0 = (lb / g.blocks_x[v]) * kLB;
    p.W = g.width[v];
    p.H = g.height[v];
    p.base = g.pixel_base[v];
    return p;
}

GS_DEV float u8f(uint32_t v) { return (float)v * (1.0f / 255.0f); }

__global__ __launch_bounds__(kLB * kLB) void k_ssim_fwd(const float* __restrict__ rgb,
                                                        const uint32_t* __restrict__ target, LossGeo g,
                                                        float* __restrict__ coef, float* __restrict__ loss_blocks) {
    // staged x and y, 3 channels each, over the 26 x 26 region
    __shared__ float s_x[3][kLR][kLR];
    __shared__ float s_y[3][kLR][kLR];
    // row sums of the 5 moments x 3 channels over 26 rows x 16 columns
    __shared__ float s_h[15][kLR][kLB];
    __shared__ float s_red[2][kLB * kLB / kWave];
    const BlockPos p = block_pos(g, blockIdx.x);
    const int t = threadIdx.x;
    for (int i = t; i < kLR * kLR; i += kLB * kLB) {
        const int ry = i / kLR, rx = i % kLR;
        const int ix = p.x0 - kHalo + rx, iy = p.y0 - kHalo + ry;
        float x0 = 0.f, x1 = 0.f, x2 = 0.f, y0 = 0.f, y1 = 0.f, y2 = 0.f;
        if (ix >= 0 && ix < p.W && iy >= 0 && iy < p.H) {
            const int64_t pix = p.base + (int64_t)iy * p.W + ix;
            x0 = rgb[3 * pix + 0]; x1 = rgb[3 * pix + 1]; x2 = rgb[3 * pix + 2];
            const uint32_t r = target[pix];
            y0 = u8f(r & 0xFF); y1 = u8f((r >> 8) & 0xFF); y2 = u8f((r >> 16) & 0xFF);
        }
        s_x[0][ry][rx] = x0; s_x[1][ry][rx] = x1; s_x[2][ry][rx] = x2;
        s_y[0][ry][rx] = y0; s_y[1][ry][rx] = y1; s_y[2][ry][rx] = y2;
    }
    __syncthreads();
    // horizontal window sums: (row, output column) positions, 15 moments each
    for (int i = t; i < kLR * kLB; i += kLB * kLB) {
        const int ry = i / kLB, cx = i % kLB;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float mx = 0.f, my = 0.f, xx = 0.f, yy = 0.f, xy = 0.f;
#pragma unroll
            for (int d = 0; d < 2 * kHalo + 1; ++d) {
                const float w = g.win[d];
                const float xv = s_x[k][ry][cx + d], yv = s_y[k][ry][cx + d];
                mx = fmaf(w, xv, mx);
                my = fmaf(w, yv, my);
                xx = fmaf(w, xv * xv, xx);
                yy = fmaf(w, yv * yv, yy);
                xy = fmaf(w, xv * yv, xy);
            }
            s_h[5 * k + 0][ry][cx] = mx;
            s_h[5 * k + 1][ry][cx] = my;
            s_h[5 * k + 2][ry][cx] = xx;
            s_h[5 * k + 3][ry][cx] = yy;
            s_h[5 * k + 4][ry][cx] = xy;
        }
    }
    __syncthreads();
    // vertical window sums at this thread's output pixel
    const int ox = t % kLB, oy = t / kLB;
    const int ix = p.x0 + ox, iy = p.y0 + oy;
    const bool inside = ix < p.W && iy < p.H;
    float l1 = 0.f, ls = 0.f;
    if (inside) {
        const int64_t pix = p.base + (int64_t)iy * p.W + ix;
        const float m = g.use_mask ? u8f(target[pix] >> 24) : 1.0f;
        float out[9];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float mom[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                float acc = 0.f;
#pragma unroll
                for (int d = 0; d < 2 * kHalo + 1; ++d) acc = fmaf(g.win[d], s_h[5 * k + q][oy + d][ox], acc);
                mom[q] = acc;
            }
            const float mx = mom[0], my = mom[1];
            const float sxx = mom[2] - mx * mx, syy = mom[3] - my * my, sxy = mom[4] - mx * my;
            const float a1 = 2.f * mx * my + kC1, a2 = 2.f * sxy + kC2;
            const float b1 = mx * mx + my * my + kC1, b2 = sxx + syy + kC2;
            const float inv = 1.0f / (b1 * b2);
            const float s = a1 * a2 * inv;
            const float ds_dmx = 2.f * my * (a2 - a1) * inv - 2.f * mx * s / b1 + 2.f * mx * s / b2;
            const float ds_dexx = -s / b2;
            const float ds_dexy = 2.f * a1 * inv;
            out[3 * k + 0] = m * ds_dmx;
            out[3 * k + 1] = m * ds_dexx;
            out[3 * k + 2] = m * ds_dexy;
            const float xv = s_x[k][oy + kHalo][ox + kHalo], yv = s_y[k][oy + kHalo][ox + kHalo];
            l1 += m * fabsf(xv - yv);
            ls += m * (1.0f - s);
        }
#pragma unroll
        for (int c = 0; c < 9; ++c) coef[9 * pix + c] = out[c];
    }
    if (loss_blocks) {
        // fixed-order block sums
        for (int off = 32; off > 0; off >>= 1) {
            l1 += __shfl_xor(l1, off);
            ls += __shfl_xor(ls, off);
        }
        if (t % kWave == 0) {
            s_red[0][t / kWave] = l1;
            s_red[1][t / kWave] = ls;
        }
        __syncthreads();
        if (t == 0) {
            float a = 0.f, b = 0.f;
            for (int i = 0; i < kLB * kLB / kWave; ++i) {
                a += s_red[0][i];
                b += s_red[1][i];
            }
            loss_blocks[2 * blockIdx.x + 0] = a;
            loss_blocks[2 * blockIdx.x + 1] = b;
        }
    }
}

__global__ __launch_bounds__(kLB * kLB) void k_ssim_bwd(const float* __restrict__ rgb,
                                                        const uint32_t* __restrict__ target, LossGeo g,
                                                        const float* __restrict__ coef, float* __restrict__ dLdC) {
    __shared__ float s_c[9][kLR][kLR];
    __shared__ float s_h[9][kLR][kLB];
    const BlockPos p = block_pos(g, blockIdx.x);
    const int t = threadIdx.x;
    for (int i = t; i < kLR * kLR; i += kLB * kLB) {
        const int ry = i / kLR, rx = i % kLR;
        const int ix = p.x0 - kHalo + rx, iy = p.y0 - kHalo + ry;
        const bool in = ix >= 0 && ix < p.W && iy >= 0 && iy < p.H;
        const int64_t pix = p.base + (int64_t)iy * p.W + ix;
#pragma unroll
        for (int c = 0; c < 9; ++c) s_c[c][ry][rx] = in ? coef[9 * pix + c] : 0.f;
    }
    __syncthreads();
    for (int i = t; i < kLR * kLB; i += kLB * kLB) {
        const int ry = i / kLB, cx = i % kLB;
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            float acc = 0.f;
#pragma unroll
            for (int d = 0; d < 2 * kHalo + 1; ++d) acc = fmaf(g.win[d], s_c[c][ry][cx + d], acc);
            s_h[c][ry][cx] = acc;
        }
    }
    __syncthreads();
    const int ox = t % kLB, oy = t / kLB;
    const int ix = p.x0 + ox, iy = p.y0 + oy;
    if (ix >= p.W || iy >= p.H) return;
    const int64_t pix = p.base + (int64_t)iy * p.W + ix;
    const uint32_t r = target[pix];
    const float m = g.use_mask ? u8f(r >> 24) : 1.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float gs[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            float acc = 0.f;
#pragma unroll
            for (int d = 0; d < 2 * kHalo + 1; ++d) acc = fmaf(g.win[d], s_h[3 * k + q][oy + d][ox], acc);
            gs[q] = acc;
        }
        const float xv = rgb[3 * pix + k], yv = u8f((r >> (8 * k)) & 0xFF);
        const float d = xv - yv;
        const float sgn = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
        dLdC[3 * pix + k] = g.l1_scale * m * sgn - g.ssim_scale * (gs[0] + 2.f * xv * gs[1] + yv * gs[2]);
    }
}

static LossGeo loss_geo(const gs_layout& L, float lam, int use_mask, int64_t* blocks) {
    LossGeo g;
    memset(&g, 0, sizeof(g));
    g.n_views = L.n_views;
    int32_t nb = 0;
    for (int v = 0; v < L.n_views; ++v) {
        g.width[v] = L.width[v];
        g.height[v] = L.height[v];
        g.pixel_base[v] = L.pixel_base[v];
        g.blocks_x[v] = (L.width[v] + kLB - 1) / kLB;
        g.block_base[v] = nb;
        nb += g.blocks_x[v] * ((L.height[v] + kLB - 1) / kLB);
    }
    for (int v = L.n_views; v <= GS_MAX_VIEWS; ++v) g.block_base[v] = nb;
    double w[2 * kHalo + 1], sum = 0.0;
    for (int i = 0; i < 2 * kHalo + 1; ++i) {
        const double d = (double)(i - kHalo);
        w[i] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
        sum += w[i];
    }
    for (int i = 0; i < 2 * kHalo + 1; ++i) g.win[i] = (float)(w[i] / sum);
    const double P = (double)L.pixel_base[L.n_views];
    g.l1_scale = (float)((1.0 - lam) / (3.0 * P));
    g.ssim_scale = (float)(lam / (3.0 * P));
    g.use_mask = use_mask;
    *blocks = nb;
    return g;
}

int64_t loss_blocks(const gs_layout& L) {
    int64_t nb = 0;
    loss_geo(L, 0.f, 0, &nb);
    return nb;
}

int launch_loss_l1_ssim(const float* rgb, const uint8_t* target, const gs_layout& L, float lam, int use_mask,
                        float* dLdC, float* loss_blocks_out, void* ws, hipStream_t s) {
    int64_t nb = 0;
    const LossGeo g = loss_geo(L, lam, use_mask, &nb);
    if (nb == 0) return GS_OK;
    float* coef = static_cast<float*>(ws);
    const uint32_t* tgt = reinterpret_cast<const uint32_t*>(target);
    hipLaunchKernelGGL(k_ssim_fwd, dim3((unsigned)nb), dim3(kLB * kLB), 0, s, rgb, tgt, g, coef, loss_blocks_out);
    int rc = check_launch("ssim_fwd");
    if (rc != GS_OK) return rc;
    hipLaunchKernelGGL(k_ssim_bwd, dim3((unsigned)nb), dim3(kLB * kLB), 0, s, rgb, tgt, g, coef, dLdC);
    return check_launch("ssim_bwd");
}

}  // namespace gs
