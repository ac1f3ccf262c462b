// Learned tile schedule: per-tile features, a small fp32 MLP (8 -> 32 -> 32 -> 1,
// ReLU) that predicts the cost of rasterising a tile, its training step (full
// batch, Adam), and the ordering of tiles by descending predicted cost for the
// persistent rasteriser.  Everything is deterministic: sums run in a fixed
// order, no floating-point atomics.
#include "gs_internal.h"

namespace gs {

constexpr int kIn = 8, kH = 32;
constexpr int kNorm = 4 * kIn;   // mean, std, low and high of each feature
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kH * kIn, kOffW2 = kOffB1 + kH,
              kOffB2 = kOffW2 + kH * kH, kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH;
static_assert(kOffB3 + 1 == GS_MLP_PARAMS, "weight layout");

// ---------------------------------------------------------------------------
// tile features
// ---------------------------------------------------------------------------

// Opacity, depth and radius statistics cover the front of the list only (the
// entries a pixel reaches before it saturates), so the cost of the features
// does not grow with the length of the list.
constexpr uint32_t kFeatEntries = 512;

__global__ __launch_bounds__(64) void k_tile_features(const float4* __restrict__ rec,
                                                      const uint32_t* __restrict__ vals,
                                                      const uint2* __restrict__ ranges, int64_t n,
                                                      gs_layout L, float* __restrict__ feat) {
    const int gt = blockIdx.x;
    const int v = view_of_tile(L, gt);
    const uint2 r = ranges[gt];
    const uint32_t fe = min(r.y, r.x + kFeatEntries);
    float so = 0.f, mo = 0.f, sz = 0.f, mz = 3.4e38f, sr = 0.f;
    for (uint32_t j = r.x + threadIdx.x; j < fe; j += 64) {
        const float4* r = rec + 4 * ((int64_t)v * n + vals[j]);
        const float o = r[1].y;
        const float4 q2 = r[2];
        so += o;
        mo = fmaxf(mo, o);
        sz += q2.y;
        mz = fminf(mz, q2.y);
        sr += q2.z;
    }
    for (int off = 32; off > 0; off >>= 1) {
        so += __shfl_xor(so, off);
        mo = fmaxf(mo, __shfl_xor(mo, off));
        sz += __shfl_xor(sz, off);
        mz = fminf(mz, __shfl_xor(mz, off));
        sr += __shfl_xor(sr, off);
    }
    if (threadIdx.x == 0) {
        const uint32_t len = r.y - r.x;
        const uint32_t flen = fe - r.x;
        const float inv = flen ? 1.0f / (float)flen : 0.0f;
        const int lt = gt - L.tile_base[v];
        const int gx = L.tiles_x[v], gy = L.tiles_y[v];
        float* f = feat + 8 * (int64_t)gt;
        f[0] = log1pf((float)len);
        f[1] = so * inv;
        f[2] = len ? mo : 0.f;
        f[3] = sz * inv;
        f[4] = len ? mz : 0.f;
        f[5] = sr * inv;
        f[6] = ((float)(lt % gx) + 0.5f) / (float)gx;
        f[7] = ((float)(lt / gx) + 0.5f) / (float)gy;
    }
}

int launch_tile_features(const gs_splats& sp, int64_t n, const gs_layout& L, const gs_bins& b,
                         float* features, hipStream_t s) {
    const int total = L.tile_base[L.n_views];
    if (total == 0) return GS_OK;
    hipLaunchKernelGGL(k_tile_features, dim3(total), dim3(64), 0, s,
                       reinterpret_cast<const float4*>(sp.rec), b.vals,
                       reinterpret_cast<const uint2*>(b.ranges), n, L, features);
    return check_launch("tile_features");
}

// ---------------------------------------------------------------------------
// MLP forward
// ---------------------------------------------------------------------------

GS_DEV void mlp_row(const float* w, const float* norm, const float* x, float xn[kIn], float h1[kH],
                    float h2[kH], float* y) {
#pragma unroll
    for (int i = 0; i < kIn; ++i)
        xn[i] = (fminf(fmaxf(x[i], norm[2 * kIn + i]), norm[3 * kIn + i]) - norm[i]) / norm[kIn + i];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float s = w[kOffB1 + j];
#pragma unroll
        for (int i = 0; i < kIn; ++i) s = __builtin_fmaf(w[kOffW1 + j * kIn + i], xn[i], s);
        h1[j] = fmaxf(s, 0.0f);
    }
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        float s = w[kOffB2 + j];
#pragma unroll
        for (int i = 0; i < kH; ++i) s = __builtin_fmaf(w[kOffW2 + j * kH + i], h1[i], s);
        h2[j] = fmaxf(s, 0.0f);
    }
    float s = w[kOffB3];
#pragma unroll
    for (int j = 0; j < kH; ++j) s = __builtin_fmaf(w[kOffW3 + j], h2[j], s);
    *y = s;
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ w,
                                                     const float* __restrict__ norm,
                                                     const float* __restrict__ x, int64_t rows,
                                                     float* __restrict__ out) {
    __shared__ float sw[GS_MLP_PARAMS];
    __shared__ float sn[kNorm];
    for (int i = threadIdx.x; i < GS_MLP_PARAMS; i += blockDim.x) sw[i] = w[i];
    if (threadIdx.x < kNorm) sn[threadIdx.x] = norm[threadIdx.x];
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    float xi[kIn], xn[kIn], h1[kH], h2[kH], y;
#pragma unroll
    for (int i = 0; i < kIn; ++i) xi[i] = x[r * kIn + i];
    mlp_row(sw, sn, xi, xn, h1, h2, &y);
    out[r] = y;
}

int launch_mlp_forward(const float* w, const float* norm, const float* x, int64_t rows, float* out,
                       hipStream_t s) {
    if (rows == 0) return GS_OK;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, w, norm,
                       x, rows, out);
    return check_launch("mlp_forward");
}

// ---------------------------------------------------------------------------
// MLP training step (MSE, Adam)
// ---------------------------------------------------------------------------

constexpr int kRowsPerChunk = 64;
constexpr int kStride = 2 * kH + 2 * kH + kIn + 1;  // h1, h2, dh1, dh2, xn, dy per row
constexpr int kSlots = (GS_MLP_PARAMS + 63) / 64;

// One wavefront per workgroup; workgroup b handles chunks b, b + G, b + 2G, ...
// and writes its partial gradient (and squared-error sum) to scratch row b.
__global__ __launch_bounds__(64) void k_mlp_grad(const float* __restrict__ w,
                                                 const float* __restrict__ norm,
                                                 const float* __restrict__ x,
                                                 const float* __restrict__ t, int64_t rows,
                                                 float* __restrict__ scratch) {
    __shared__ float sw[GS_MLP_PARAMS];
    __shared__ float sn[kNorm];
    __shared__ float rowbuf[kRowsPerChunk][kStride];
    for (int i = threadIdx.x; i < GS_MLP_PARAMS; i += 64) sw[i] = w[i];
    if (threadIdx.x < kNorm) sn[threadIdx.x] = norm[threadIdx.x];
    __syncthreads();
    float acc[kSlots];
#pragma unroll
    for (int k = 0; k < kSlots; ++k) acc[k] = 0.f;
    float sq = 0.f;
    const float scale = 2.0f / (float)rows;
    const int64_t nchunks = (rows + kRowsPerChunk - 1) / kRowsPerChunk;
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int64_t r = c * kRowsPerChunk + threadIdx.x;
        float* rb = rowbuf[threadIdx.x];
        if (r < rows) {
            float xi[kIn], xn[kIn], h1[kH], h2[kH], y;
#pragma unroll
            for (int i = 0; i < kIn; ++i) xi[i] = x[r * kIn + i];
            mlp_row(sw, sn, xi, xn, h1, h2, &y);
            const float e = y - t[r];
            sq = __builtin_fmaf(e, e, sq);
            const float dy = scale * e;
            float dh2[kH];
#pragma unroll
            for (int j = 0; j < kH; ++j) dh2[j] = h2[j] > 0.0f ? dy * sw[kOffW3 + j] : 0.0f;
#pragma unroll
            for (int i = 0; i < kH; ++i) {
                float s = 0.f;
#pragma unroll
                for (int j = 0; j < kH; ++j) s = __builtin_fmaf(sw[kOffW2 + j * kH + i], dh2[j], s);
                rb[2 * kH + i] = h1[i] > 0.0f ? s : 0.0f;  // dh1
            }
#pragma unroll
            for (int j = 0; j < kH; ++j) {
                rb[j] = h1[j];
                rb[kH + j] = h2[j];
                rb[3 * kH + j] = dh2[j];
            }
#pragma unroll
            for (int i = 0; i < kIn; ++i) rb[4 * kH + i] = xn[i];
            rb[4 * kH + kIn] = dy;
        } else {
            for (int i = 0; i < kStride; ++i) rb[i] = 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            const int p = threadIdx.x + 64 * k;
            if (p >= GS_MLP_PARAMS) break;
            float s = acc[k];
            for (int rr = 0; rr < kRowsPerChunk; ++rr) {
                const float* q = rowbuf[rr];
                float gval;
                if (p < kOffB1) gval = q[2 * kH + p / kIn] * q[4 * kH + p % kIn];
                else if (p < kOffW2) gval = q[2 * kH + (p - kOffB1)];
                else if (p < kOffB2) gval = q[3 * kH + (p - kOffW2) / kH] * q[(p - kOffW2) % kH];
                else if (p < kOffW3) gval = q[3 * kH + (p - kOffB2)];
                else if (p < kOffB3) gval = q[4 * kH + kIn] * q[kH + (p - kOffW3)];
                else gval = q[4 * kH + kIn];
                s += gval;
            }
            acc[k] = s;
        }
        __syncthreads();
    }
    float* out = scratch + (int64_t)blockIdx.x * (GS_MLP_PARAMS + 1);
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
        const int p = threadIdx.x + 64 * k;
        if (p < GS_MLP_PARAMS) out[p] = acc[k];
    }
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
    if (threadIdx.x == 0) out[GS_MLP_PARAMS] = sq;
}

__global__ void k_mlp_tick(int32_t* step, float* bias) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int t = *step + 1;
    *step = t;
    bias[0] = (float)(1.0 - pow(0.9, (double)t));
    bias[1] = (float)sqrt(1.0 - pow(0.999, (double)t));
}

__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ w, const float* __restrict__ part,
                                                  int groups, int64_t rows, float* __restrict__ m,
                                                  float* __restrict__ v, const float* __restrict__ bias,
                                                  float lr, float* __restrict__ loss_out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > GS_MLP_PARAMS) return;
    float g = 0.f;
    for (int b = 0; b < groups; ++b) g += part[(int64_t)b * (GS_MLP_PARAMS + 1) + p];
    if (p == GS_MLP_PARAMS) {
        if (loss_out) *loss_out = g / (float)rows;
        return;
    }
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mm = b1 * m[p] + (1.0f - b1) * g;
    const float vv = b2 * v[p] + (1.0f - b2) * (g * g);
    m[p] = mm;
    v[p] = vv;
    w[p] = w[p] - (lr / bias[0]) * (mm / (__builtin_sqrtf(vv) / bias[1] + eps));
}

int launch_mlp_train_step(float* w, const float* norm, const float* x, const float* y,
                          int64_t rows, float* grad, float* m, float* v, int32_t* step, float lr,
                          float* loss_out, hipStream_t s) {
    const int groups = GS_MLP_GROUPS;
    hipLaunchKernelGGL(k_mlp_grad, dim3(groups), dim3(64), 0, s, w, norm, x, y, rows, grad);
    int rc = check_launch("mlp_grad");
    if (rc != GS_OK) return rc;
    float* bias = grad + (int64_t)groups * (GS_MLP_PARAMS + 1);
    hipLaunchKernelGGL(k_mlp_tick, dim3(1), dim3(64), 0, s, step, bias);
    if ((rc = check_launch("mlp_tick")) != GS_OK) return rc;
    hipLaunchKernelGGL(k_mlp_adam, dim3((GS_MLP_PARAMS + 1 + 255) / 256), dim3(256), 0, s, w, grad,
                       groups, rows, m, v, bias, lr, loss_out);
    return check_launch("mlp_adam");
}

// ---------------------------------------------------------------------------
// ordering by predicted cost
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_cost_keys(const float* __restrict__ pred, int32_t total,
                                                   uint32_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals,
                                                   uint32_t* __restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const float p = pred[i];
    if (!__builtin_isfinite(p)) atomicOr(bad, 1u);
    const uint32_t u = __float_as_uint(p);
    const uint32_t asc = (u & 0x80000000u) ? ~u : (u | 0x80000000u);  // ascending float order
    keys[i] = ~asc;                                                    // descending
    vals[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k_cost_finish(uint32_t* __restrict__ order, int32_t total,
                                                     const uint32_t* __restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    if (*bad) order[i] = (uint32_t)i;  // static schedule fallback
}

int launch_order_by_cost(const float* pred, int32_t total, uint32_t* order, void* scratch,
                         hipStream_t s) {
    uint32_t* keys = (uint32_t*)scratch;
    uint32_t* bad = keys + total;
    void* sort_scratch = (char*)scratch + 4 * ((size_t)total + 64);
    int rc = launch_fill_u32(bad, 0u, 1, s);
    if (rc != GS_OK) return rc;
    const unsigned grid = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(k_cost_keys, dim3(grid), dim3(256), 0, s, pred, total, keys, order, bad);
    if ((rc = check_launch("cost_keys")) != GS_OK) return rc;
    if ((rc = sort_pairs(keys, order, total, sort_scratch, s)) != GS_OK) return rc;
    hipLaunchKernelGGL(k_cost_finish, dim3(grid), dim3(256), 0, s, order, total, bad);
    return check_launch("cost_finish");
}

}  // namespace gs
