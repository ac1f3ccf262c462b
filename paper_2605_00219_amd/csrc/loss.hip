// Fused L1 + D-SSIM loss gradient against an RGBA8 reference (Sec. 4.5):
// L = (1 - lam)/(3P) sum m |x - y| + lam/(3P) sum m (1 - S), per colour
// channel, x the render, y = rgb / 255, m = alpha / 255 (or 1).  S is the SSIM
// map of each channel with an 11 x 11 Gaussian window (sigma 1.5), zero
// outside each view's image.
//
// Two kernels, each over (64 x 16 output block, colour channel) units (the
// channels are independent in both terms), each staging its block plus a
// 5-pixel halo of one channel in LDS and summing the window separably,
// columns first (16 x 74 partial sums instead of 26 x 64 rows first):
//   k_ssim_moments  window moments of x, y, x^2, y^2, xy -> S and the
//                   coefficient maps a = m dS/dmu_x, b = m dS/dE[x^2],
//                   c = m dS/dE[xy] (plane-major in the workspace), and the
//                   unit's loss sums;
//   k_ssim_grad     window sums of a, b, c -> dL/dx = (1 - lam)/(3P) m sign(x - y)
//                   - lam/(3P) (G*a + 2 x G*b + y G*c).
// Both are bound by vector ALU issue, so the arithmetic around the window sums
// is kept small: a staging thread owns one staged column and steps 3 rows at
// a time, indices are 32-bit, the SSIM derivatives take one reciprocal, and
// the row pass of a thread yields exactly its 4
// output pixels (four 16-byte LDS reads per plane cover the 14 inputs), whose
// SSIM terms or gradients it then computes in registers.  Each XCD takes a
// contiguous band of blocks, so the halos that neighbouring blocks share, and
// the render lines that a block's three channels share, are read through one
// L2.  Both kernels are persistent (four workgroups per CU) and load
// the next unit's inputs into registers while the current unit is summed.
// The reference stays 4 x uint8 per pixel; the render stays channel-last.
#include <atomic>
#include <climits>
#include <cmath>

#include "gs_internal.h"

namespace gs {

constexpr int kBW = 64;                   // output block width
constexpr int kBH = 16;                   // output block height
constexpr int kHalo = 5;                  // window radius
constexpr int kTaps = 2 * kHalo + 1;
constexpr int kSW = kBW + 2 * kHalo;      // staged columns (74)
constexpr int kSH = kBH + 2 * kHalo;      // staged rows (26)
constexpr int kP = 76;                    // row pitch of the column sums in LDS (16-byte rows)
constexpr int kLT = 256;                  // threads per workgroup
constexpr int kCR = 4;                    // output rows per column-pass item
constexpr int kCItems = kSW * (kBH / kCR);            // column-pass items (296)
// staging: thread t < 222 owns staged column t % 74 and rows t / 74 + 3 s,
// the pixel at LDS index t + 222 s (row pitch kSW)
constexpr int kSRows = 3;
constexpr int kSThreads = kSRows * kSW;                // 222
constexpr int kStage = (kSH + kSRows - 1) / kSRows;    // staged pixels per thread (9)
static_assert(kSThreads <= kLT, "staging threads");
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;
static_assert(kBW * kBH == 4 * kLT, "row pass: one 4-pixel item per thread");
static_assert(kP % 4 == 0 && kP >= kBW + 12, "16-byte rows hold every 4-column window");

struct LossGeo {
    int32_t width[GS_MAX_VIEWS], height[GS_MAX_VIEWS];
    int32_t pixel_base[GS_MAX_VIEWS];       // first pixel of each view
    int32_t cbase[GS_MAX_VIEWS];            // first workspace index of each view
    int32_t cpitch[GS_MAX_VIEWS];           // workspace row pitch (whole blocks)
    int32_t block_base[GS_MAX_VIEWS + 1];   // first 64 x 16 block of each view
    int32_t blocks_x[GS_MAX_VIEWS];
    int32_t n_views, n_blocks;
    int32_t cplane;                         // workspace plane stride (views padded to whole blocks)
    float win[kTaps];                       // normalised 1-D Gaussian window
    float l1_scale, ssim_scale;             // (1 - lam)/(3P), lam/(3P)
    int use_mask;
};

struct BlockPos {
    int x0, y0, W, H, base, cbase, cpitch;
};

// workgroup -> (block, channel).  Workgroups are dealt to the 8 XCDs in
// turn, so XCD x = wg % 8 runs units m = wg / 8 = 0, 1, ... of its own band
// of blocks [x nb / 8, (x + 1) nb / 8) (row-major, so neighbouring blocks and
// their shared halos stay in one L2), the three channels of a block in
// succession; false past the end of the band
GS_DEV bool unit_of(const LossGeo& g, int wg, int* blk, int* ch) {
    const int x = wg % 8, m = wg / 8;
    *ch = m % 3;
    *blk = x * g.n_blocks / 8 + m / 3;
    return *blk < (x + 1) * g.n_blocks / 8;
}

GS_DEV BlockPos block_pos(const LossGeo& g, int blk) {
    int v = 0;
    for (int i = 1; i < g.n_views; ++i)
        if (blk >= g.block_base[i]) v = i;
    const int lb = blk - g.block_base[v];
    BlockPos p;
    p.x0 = (lb % g.blocks_x[v]) * kBW;
    p.y0 = (lb / g.blocks_x[v]) * kBH;
    p.W = g.width[v];
    p.H = g.height[v];
    p.base = g.pixel_base[v];
    p.cbase = g.cbase[v];
    p.cpitch = g.cpitch[v];
    return p;
}

GS_DEV float u8f(uint32_t v) { return (float)v * (1.0f / 255.0f); }
GS_DEV bool inside(int ix, int iy, const BlockPos& p) { return (unsigned)ix < (unsigned)p.W && (unsigned)iy < (unsigned)p.H; }

// 16 consecutive floats from a 16-byte aligned LDS row
GS_DEV void ld16(const float* row, int c0, float (&v)[16]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float4 q = *reinterpret_cast<const float4*>(row + c0 + 4 * i);
        v[4 * i + 0] = q.x; v[4 * i + 1] = q.y; v[4 * i + 2] = q.z; v[4 * i + 3] = q.w;
    }
}

// window sums at 4 consecutive positions from their 14 inputs
GS_DEV void wsum4(const float* win, const float (&v)[16], float (&o)[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float a = 0.f;
#pragma unroll
        for (int d = 0; d < kTaps; ++d) a = fmaf(win[d], v[j + d], a);
        o[j] = a;
    }
}

// The thread index, opaque to the compiler, so that addresses derived from it
// are recomputed per unit rather than held in registers across the loop.
GS_DEV int opaque_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// ---- k_ssim_moments -----------------------------------------------------

struct MomIn {
    float x[kStage];       // render channel over the staged region
    uint32_t y[kStage];    // reference words over the staged region
    uint32_t o[4];         // reference words of the thread's 4 output pixels
};

GS_DEV void mom_load(const LossGeo& g, int blk, int k, const float* __restrict__ rgb,
                     const uint32_t* __restrict__ target, int t, MomIn& in) {
    const BlockPos p = block_pos(g, blk);
    const int ro = t / kSW, ix = p.x0 - kHalo + t % kSW, iy0 = p.y0 - kHalo + ro;
    const bool col_ok = t < kSThreads && (unsigned)ix < (unsigned)p.W;
    const int pix0 = p.base + iy0 * p.W + ix;
#pragma unroll
    for (int s = 0; s < kStage; ++s) {
        in.x[s] = 0.f;
        in.y[s] = 0u;
        if (col_ok && ro + kSRows * s < kSH && (unsigned)(iy0 + kSRows * s) < (unsigned)p.H) {
            const int pix = pix0 + kSRows * s * p.W;
            in.x[s] = rgb[3 * pix + k];
            in.y[s] = target[pix];
        }
    }
    const int iy = p.y0 + t / 16, ix0 = p.x0 + 4 * (t % 16);
    const uint32_t* to = target + (p.base + iy * p.W + ix0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        in.o[j] = 0u;
        if (iy < p.H && ix0 + j < p.W) in.o[j] = to[j];
    }
}

__global__ __launch_bounds__(kLT) __attribute__((amdgpu_waves_per_eu(4))) void k_ssim_moments(
    const float* __restrict__ rgb, const uint32_t* __restrict__ target, LossGeo g, float* __restrict__ coef,
    float* __restrict__ loss_units) {
    __shared__ float s_x[kSH * kSW];
    __shared__ float s_y[kSH * kSW];
    __shared__ __align__(16) float s_v[5][kBH][kP];   // column sums of x, y, x^2, y^2, xy
    __shared__ float s_red[2][kLT / kWave];
    int wg = blockIdx.x, blk, k;
    if (!unit_of(g, wg, &blk, &k)) return;
    MomIn in;
    mom_load(g, blk, k, rgb, target, opaque_tid(), in);
    for (;;) {
        const int t = opaque_tid();
        const BlockPos p = block_pos(g, blk);
#pragma unroll
        for (int s = 0; s < kStage; ++s) {
            if (t < kSThreads && t / kSW + kSRows * s < kSH) {
                s_x[t + kSThreads * s] = in.x[s];
                s_y[t + kSThreads * s] = u8f((in.y[s] >> (8 * k)) & 0xFF);
            }
        }
        uint32_t ow[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) ow[j] = in.o[j];
        __syncthreads();
        // column pass: (staged column, 4 output rows) items
        for (int it = t; it < kCItems; it += kLT) {
            const int c = it % kSW, r0 = (it / kSW) * kCR;
            float a[5][kCR];
#pragma unroll
            for (int q = 0; q < 5; ++q)
#pragma unroll
                for (int j = 0; j < kCR; ++j) a[q][j] = 0.f;
#pragma unroll
            for (int i = 0; i < kCR + 2 * kHalo; ++i) {
                const float xv = s_x[(r0 + i) * kSW + c], yv = s_y[(r0 + i) * kSW + c];
                const float v[5] = {xv, yv, xv * xv, yv * yv, xv * yv};
#pragma unroll
                for (int j = 0; j < kCR; ++j) {
                    const int d = i - j;
                    if (d >= 0 && d < kTaps) {
#pragma unroll
                        for (int q = 0; q < 5; ++q) a[q][j] = fmaf(g.win[d], v[q], a[q][j]);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < 5; ++q)
#pragma unroll
                for (int j = 0; j < kCR; ++j) s_v[q][r0 + j][c] = a[q][j];
        }
        __syncthreads();
        // the next unit's loads are in flight during the row pass
        const int wg_next = wg + (int)gridDim.x;
        int blk_next, k_next;
        const bool more = unit_of(g, wg_next, &blk_next, &k_next);
        if (more) mom_load(g, blk_next, k_next, rgb, target, t, in);
        // row pass: this thread's 4 output pixels
        const int r = t / 16, c0 = 4 * (t % 16);
        float mom[5][4];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            float v[16];
            ld16(&s_v[q][r][0], c0, v);
            wsum4(g.win, v, mom[q]);
        }
        float l1 = 0.f, ls = 0.f;
        float ca[4], cb[4], cc[4];
        const int iy = p.y0 + r;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            ca[j] = 0.f;
            cb[j] = 0.f;
            cc[j] = 0.f;
            if (inside(p.x0 + c0 + j, iy, p)) {
                const float m = g.use_mask ? u8f(ow[j] >> 24) : 1.0f;
                const float mx = mom[0][j], my = mom[1][j];
                const float sxx = mom[2][j] - mx * mx, syy = mom[3][j] - my * my, sxy = mom[4][j] - mx * my;
                const float a1 = 2.f * mx * my + kC1, a2 = 2.f * sxy + kC2;
                const float b1 = mx * mx + my * my + kC1, b2 = sxx + syy + kC2;
                // one reciprocal: 1/b1 = b2 inv, 1/b2 = b1 inv
                const float inv = __builtin_amdgcn_rcpf(b1 * b2);
                const float sv = a1 * a2 * inv;
                const float m2i = 2.f * m * inv;
                ca[j] = m2i * (my * (a2 - a1) + mx * sv * (b1 - b2));   // m dS/dmu_x
                cb[j] = -m * sv * b1 * inv;                              // m dS/dE[x^2]
                cc[j] = m2i * a1;                                        // m dS/dE[xy]
                const int si = (r + kHalo) * kSW + c0 + j + kHalo;
                const float xv = s_x[si], yv = s_y[si];
                l1 += m * fabsf(xv - yv);
                ls += m * (1.0f - sv);
            }
        }
        // the block's rows lie inside the padded workspace view
        const int ci = p.cbase + iy * p.cpitch + p.x0 + c0;
        st4(coef, (g.cplane * (3 * k + 0) + ci) / 4, make_float4(ca[0], ca[1], ca[2], ca[3]));
        st4(coef, (g.cplane * (3 * k + 1) + ci) / 4, make_float4(cb[0], cb[1], cb[2], cb[3]));
        st4(coef, (g.cplane * (3 * k + 2) + ci) / 4, make_float4(cc[0], cc[1], cc[2], cc[3]));
        if (loss_units) {
            // fixed-order sums over the unit
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
                for (int i = 0; i < kLT / kWave; ++i) {
                    a += s_red[0][i];
                    b += s_red[1][i];
                }
                const int u = 3 * blk + k;
                loss_units[2 * u + 0] = a;
                loss_units[2 * u + 1] = b;
            }
        }
        if (!more) break;
        __syncthreads();   // LDS reads of this unit end before the next unit's writes
        wg = wg_next;
        blk = blk_next;
        k = k_next;
    }
}

// ---- k_ssim_grad ---------------------------------------------------------

struct GradIn {
    float c[3][kStage];    // the channel's coefficient planes over the staged region
    float x[4];            // render channel at the thread's 4 output pixels
    uint32_t y[4];         // reference words there
};

GS_DEV void grad_load(const LossGeo& g, int blk, int k, const float* __restrict__ rgb,
                      const uint32_t* __restrict__ target, const float* __restrict__ coef, int t,
                      GradIn& in) {
    const BlockPos p = block_pos(g, blk);
    const int ro = t / kSW, ix = p.x0 - kHalo + t % kSW, iy0 = p.y0 - kHalo + ro;
    const bool col_ok = t < kSThreads && (unsigned)ix < (unsigned)p.W;
    const int ci0 = g.cplane * 3 * k + p.cbase + iy0 * p.cpitch + ix;
#pragma unroll
    for (int s = 0; s < kStage; ++s) {
        in.c[0][s] = 0.f;
        in.c[1][s] = 0.f;
        in.c[2][s] = 0.f;
        if (col_ok && ro + kSRows * s < kSH && (unsigned)(iy0 + kSRows * s) < (unsigned)p.H) {
            const int ci = ci0 + kSRows * s * p.cpitch;
#pragma unroll
            for (int q = 0; q < 3; ++q) in.c[q][s] = coef[ci + q * g.cplane];
        }
    }
    const int iy = p.y0 + t / 16, ix0 = p.x0 + 4 * (t % 16);
    const int pix = p.base + iy * p.W + ix0;
    const float* xo = rgb + (3 * pix + k);
    const uint32_t* to = target + pix;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        in.x[j] = 0.f;
        in.y[j] = 0u;
        if (iy < p.H && ix0 + j < p.W) {
            in.x[j] = xo[3 * j];
            in.y[j] = to[j];
        }
    }
}

__global__ __launch_bounds__(kLT) __attribute__((amdgpu_waves_per_eu(4))) void k_ssim_grad(
    const float* __restrict__ rgb, const uint32_t* __restrict__ target, LossGeo g,
    const float* __restrict__ coef, float* __restrict__ dLdC) {
    __shared__ float s_c[3][kSH * kSW];
    __shared__ __align__(16) float s_v[3][kBH][kP];
    int wg = blockIdx.x, blk, k;
    if (!unit_of(g, wg, &blk, &k)) return;
    GradIn in;
    grad_load(g, blk, k, rgb, target, coef, opaque_tid(), in);
    for (;;) {
        const int t = opaque_tid();
        const BlockPos p = block_pos(g, blk);
#pragma unroll
        for (int s = 0; s < kStage; ++s) {
            if (t < kSThreads && t / kSW + kSRows * s < kSH) {
#pragma unroll
                for (int q = 0; q < 3; ++q) s_c[q][t + kSThreads * s] = in.c[q][s];
            }
        }
        float xo[4];
        uint32_t yo[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            xo[j] = in.x[j];
            yo[j] = in.y[j];
        }
        __syncthreads();
        const int wg_next = wg + (int)gridDim.x;
        int blk_next, k_next;
        const bool more = unit_of(g, wg_next, &blk_next, &k_next);
        if (more) grad_load(g, blk_next, k_next, rgb, target, coef, t, in);
        for (int it = t; it < kCItems; it += kLT) {
            const int c = it % kSW, r0 = (it / kSW) * kCR;
            float a[3][kCR];
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int j = 0; j < kCR; ++j) a[q][j] = 0.f;
#pragma unroll
            for (int i = 0; i < kCR + 2 * kHalo; ++i) {
                float v[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) v[q] = s_c[q][(r0 + i) * kSW + c];
#pragma unroll
                for (int j = 0; j < kCR; ++j) {
                    const int d = i - j;
                    if (d >= 0 && d < kTaps) {
#pragma unroll
                        for (int q = 0; q < 3; ++q) a[q][j] = fmaf(g.win[d], v[q], a[q][j]);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int j = 0; j < kCR; ++j) s_v[q][r0 + j][c] = a[q][j];
        }
        __syncthreads();
        const int r = t / 16, c0 = 4 * (t % 16);
        float gs[3][4];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            float v[16];
            ld16(&s_v[q][r][0], c0, v);
            wsum4(g.win, v, gs[q]);
        }
        const int iy = p.y0 + r, ix0 = p.x0 + c0;
        float* out = dLdC + (3 * (p.base + iy * p.W + ix0) + k);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (iy < p.H && ix0 + j < p.W) {
                const float m = g.use_mask ? u8f(yo[j] >> 24) : 1.0f;
                const float xv = xo[j], yv = u8f((yo[j] >> (8 * k)) & 0xFF);
                const float d = xv - yv;
                const float sgn = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
                out[3 * j] = g.l1_scale * m * sgn - g.ssim_scale * (gs[0][j] + 2.f * xv * gs[1][j] + yv * gs[2][j]);
            }
        }
        if (!more) break;
        __syncthreads();   // LDS reads of this unit end before the next unit's writes
        wg = wg_next;
        blk = blk_next;
        k = k_next;
    }
}

// ---- host ------------------------------------------------------------------

// compute units of the current device (asked on every call: nothing is kept)
static int cu_count() {
    int dev = 0, c = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
        return 256;
    return c;
}

// false when the views are too large for 32-bit pixel and workspace indices
static bool loss_geo(const gs_layout& L, float lam, int use_mask, LossGeo* out) {
    LossGeo g;
    memset(&g, 0, sizeof(g));
    g.n_views = L.n_views;
    int64_t nb = 0, cb = 0;
    for (int v = 0; v < L.n_views; ++v) {
        const int64_t bx = (L.width[v] + kBW - 1) / kBW, by = (L.height[v] + kBH - 1) / kBH;
        g.width[v] = L.width[v];
        g.height[v] = L.height[v];
        g.pixel_base[v] = (int32_t)L.pixel_base[v];
        g.blocks_x[v] = (int32_t)bx;
        g.block_base[v] = (int32_t)nb;
        g.cbase[v] = (int32_t)cb;
        g.cpitch[v] = (int32_t)(bx * kBW);
        nb += bx * by;
        cb += bx * kBW * by * kBH;
        if (nb > INT_MAX / 24 || 9 * cb > INT_MAX) return false;
    }
    if (3 * L.pixel_base[L.n_views] > INT_MAX) return false;
    for (int v = L.n_views; v <= GS_MAX_VIEWS; ++v) g.block_base[v] = (int32_t)nb;
    g.n_blocks = (int32_t)nb;
    g.cplane = (int32_t)cb;
    double w[kTaps], sum = 0.0;
    for (int i = 0; i < kTaps; ++i) {
        const double d = (double)(i - kHalo);
        w[i] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
        sum += w[i];
    }
    for (int i = 0; i < kTaps; ++i) g.win[i] = (float)(w[i] / sum);
    const double P = (double)L.pixel_base[L.n_views];
    g.l1_scale = (float)((1.0 - lam) / (3.0 * P));
    g.ssim_scale = (float)(lam / (3.0 * P));
    g.use_mask = use_mask;
    *out = g;
    return true;
}

int64_t loss_blocks(const gs_layout& L) {
    LossGeo g;
    return loss_geo(L, 0.f, 0, &g) ? 3 * (int64_t)g.n_blocks : 0;
}

size_t loss_workspace(const gs_layout& L) {
    LossGeo g;
    return loss_geo(L, 0.f, 0, &g) ? (size_t)9 * sizeof(float) * (size_t)std::max(g.cplane, 1) : 0;
}

int launch_loss_l1_ssim(const float* rgb, const uint8_t* target, const gs_layout& L, float lam, int use_mask,
                        float* dLdC, float* loss_units, void* ws, hipStream_t s) {
    LossGeo g;
    if (!loss_geo(L, lam, use_mask, &g)) {
        set_error("gs_loss_l1_ssim: views too large for 32-bit pixel indices");
        return GS_ERR_INVALID_ARG;
    }
    if (g.n_blocks == 0) return GS_OK;
    // every XCD's band has at most ceil(nb / 8) blocks of three units; a
    // persistent grid of four workgroups per CU (their LDS fills a CU), a
    // multiple of 8 so that each workgroup keeps to one XCD's band
    const unsigned units = 24u * (unsigned)((g.n_blocks + 7) / 8);
    const unsigned resident = std::max(8u, (unsigned)(4 * cu_count()) / 8u * 8u);
    const unsigned grid = std::min(units, resident);
    float* coef = static_cast<float*>(ws);
    const uint32_t* tgt = reinterpret_cast<const uint32_t*>(target);
    hipLaunchKernelGGL(k_ssim_moments, dim3(grid), dim3(kLT), 0, s, rgb, tgt, g, coef, loss_units);
    int rc = check_launch("ssim_moments");
    if (rc != GS_OK) return rc;
    hipLaunchKernelGGL(k_ssim_grad, dim3(grid), dim3(kLT), 0, s, rgb, tgt, g, coef, dLdC);
    return check_launch("ssim_grad");
}

}  // namespace gs
