// Projection backward fused with Adam: one thread per Gaussian streams its
// parameter record and both Adam moments once, gathers the screen-space
// gradient records of the intersections the rasteriser traversed (through the
// inverse sort permutation), and writes parameters and moments once.  No per-parameter gradient buffer exists
// unless the caller asks for one (grads_out).  Log-scales and opacity logits
// are optimised as stored: the chain rule through exp and the sigmoid is part
// of this kernel.
//
// The forward quantities needed by the chain rule are recomputed with the same
// float32 code as the projection kernel, so every branch decision (culling,
// Jacobian clamp, colour clamp) matches the forward pass bitwise.
#include "project_math.h"

namespace gs {

struct AdamArgs {
    float4* params;
    int64_t n;
    const gs_view* views;
    int n_views;
    int tile;
    int32_t gx[GS_MAX_VIEWS], gy[GS_MAX_VIEWS];
    int32_t tile_base[GS_MAX_VIEWS];
    const uint32_t* offsets;
    const uint32_t* inv;
    const float4* grec;
    const uint32_t* tile_stop;
    int64_t capacity;
    float4* m;
    float4* v;
    const float* bias;  // [0] = 1 - beta1^t, [1] = sqrt(1 - beta2^t)
    float lr[6];
    float beta1, beta2, eps;
    float4* grads_out;
};

// d Y_m / d(x, y, z) contracted with w[m]: returns sum_m w[m] dY_m/d(dir)
GS_DEV void sh_dir_grad(float x, float y, float z, const float w[16], float out[3]) {
    const float xx = x * x, yy = y * y, zz = z * z;
    float gx = 0.f, gy = 0.f, gz = 0.f;
    gy += w[1] * (-kSH1);
    gz += w[2] * kSH1;
    gx += w[3] * (-kSH1);
    gx += w[4] * (kSH2a * y); gy += w[4] * (kSH2a * x);
    gy += w[5] * (-kSH2a * z); gz += w[5] * (-kSH2a * y);
    gx += w[6] * (-2.f * kSH2c * x); gy += w[6] * (-2.f * kSH2c * y); gz += w[6] * (4.f * kSH2c * z);
    gx += w[7] * (-kSH2a * z); gz += w[7] * (-kSH2a * x);
    gx += w[8] * (2.f * kSH2e * x); gy += w[8] * (-2.f * kSH2e * y);
    gx += w[9] * (kSH3a * 6.f * x * y); gy += w[9] * (kSH3a * (3.f * xx - 3.f * yy));
    gx += w[10] * (kSH3b * y * z); gy += w[10] * (kSH3b * x * z); gz += w[10] * (kSH3b * x * y);
    gx += w[11] * (-2.f * kSH3c * x * y); gy += w[11] * (kSH3c * (4.f * zz - xx - 3.f * yy));
    gz += w[11] * (8.f * kSH3c * y * z);
    gx += w[12] * (-6.f * kSH3d * x * z); gy += w[12] * (-6.f * kSH3d * y * z);
    gz += w[12] * (kSH3d * (6.f * zz - 3.f * xx - 3.f * yy));
    gx += w[13] * (kSH3c * (4.f * zz - 3.f * xx - yy)); gy += w[13] * (-2.f * kSH3c * x * y);
    gz += w[13] * (8.f * kSH3c * x * z);
    gx += w[14] * (2.f * kSH3f * x * z); gy += w[14] * (-2.f * kSH3f * y * z);
    gz += w[14] * (kSH3f * (xx - yy));
    gx += w[15] * (kSH3a * (3.f * xx - 3.f * yy)); gy += w[15] * (-6.f * kSH3a * x * y);
    out[0] = gx; out[1] = gy; out[2] = gz;
}

GS_DEV float adam_one(float p, float g, float& m, float& v, float lr, float beta1, float beta2,
                      float eps, float bc1, float bc2s) {
    m = beta1 * m + (1.0f - beta1) * g;
    v = beta2 * v + (1.0f - beta2) * (g * g);
    const float denom = __builtin_sqrtf(v) / bc2s + eps;
    return p - (lr / bc1) * (m / denom);
}

__global__ __launch_bounds__(256) void k_project_bwd_adam(AdamArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    const int64_t n = a.n;
    const float4 p0 = a.params[0 * n + g];
    const float4 p1 = a.params[1 * n + g];
    const float4 p2 = a.params[2 * n + g];
    float4 sh[12];
    bool finite = finite4(p0) && finite4(make_float4(p1.x, p1.y, p1.z, 0.0f)) && finite4(p2);
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        sh[q] = a.params[(3 + q) * n + g];
        finite = finite && finite4(sh[q]);
    }
    float gm[3] = {0.f, 0.f, 0.f}, gls[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f};
    float glo = 0.f;
    float gsh[48];
#pragma unroll
    for (int i = 0; i < 48; ++i) gsh[i] = 0.f;

    for (int vi = 0; vi < a.n_views && finite; ++vi) {
        const int64_t o = (int64_t)vi * n + g;
        const uint64_t b = a.offsets[o];
        uint64_t e = a.offsets[o + 1];
        if (e == b) continue;
        if (e > (uint64_t)a.capacity) e = (uint64_t)a.capacity;
        const gs_view vw = a.views[vi];
        Proj P;
        project_gaussian<true>(p0, p1, p2, sh, vw, a.tile, a.gx[vi], a.gy[vi], P);
        if (!P.valid) continue;
        // sum the records of this Gaussian's traversed intersections, in
        // unsorted-index order (tile = its rectangle, row major)
        float d[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        const uint32_t w = (uint32_t)(P.x1 - P.x0);
        const int tbase = a.tile_base[vi] + P.y0 * a.gx[vi] + P.x0;
        uint32_t kx = 0, ky = 0;
        for (uint64_t i = b; i < e; ++i) {
            const uint32_t j = a.inv[i];
            if (j < a.tile_stop[tbase + (int)(ky * (uint32_t)a.gx[vi] + kx)]) {
                const float4 r0 = a.grec[3 * (int64_t)j + 0];
                const float4 r1 = a.grec[3 * (int64_t)j + 1];
                const float4 r2 = a.grec[3 * (int64_t)j + 2];
                d[0] += r0.x; d[1] += r0.y; d[2] += r0.z; d[3] += r0.w;
                d[4] += r1.x; d[5] += r1.y; d[6] += r1.z; d[7] += r1.w; d[8] += r2.x;
            }
            if (++kx == w) { kx = 0; ++ky; }
        }

        float dmean[3] = {0.f, 0.f, 0.f};
        // colour: c = max(0, raw + 1/2), raw = sum_m sh[m] Y_m(dir)
        float draw[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) draw[k] = (P.raw[k] + 0.5f >= 0.0f) ? d[6 + k] : 0.0f;
        float c[48];
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            c[4 * q + 0] = sh[q].x; c[4 * q + 1] = sh[q].y; c[4 * q + 2] = sh[q].z; c[4 * q + 3] = sh[q].w;
        }
        float wY[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
#pragma unroll
            for (int k = 0; k < 3; ++k) gsh[m * 3 + k] += P.Y[m] * draw[k];
            wY[m] = c[m * 3 + 0] * draw[0] + c[m * 3 + 1] * draw[1] + c[m * 3 + 2] * draw[2];
        }
        {
            float ddir[3];
            sh_dir_grad(P.dir[0], P.dir[1], P.dir[2], wY, ddir);
            const float dd = P.dir[0] * ddir[0] + P.dir[1] * ddir[1] + P.dir[2] * ddir[2];
#pragma unroll
            for (int i = 0; i < 3; ++i) dmean[i] += (ddir[i] - P.dir[i] * dd) / P.dlen;
        }
        // opacity
        glo += d[5] * P.o * (1.0f - P.o);
        // conic -> 2D covariance
        const float A = P.A, B = P.B, C = P.C;
        const float g11 = d[2], g12 = 0.5f * d[3], g22 = d[4];
        const float q00 = A * g11 + B * g12, q01 = A * g12 + B * g22;
        const float q10 = B * g11 + C * g12, q11 = B * g12 + C * g22;
        const float dS[4] = {-(q00 * A + q01 * B), -(q00 * B + q01 * C), -(q00 * B + q01 * C),
                             -(q10 * B + q11 * C)};
        // 2D covariance = Am Sigma Am^T
        float Sig[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Sig[i * 3 + j] = sig_at(P.Sig, i, j);
        float dSig[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                float s = 0.f;
#pragma unroll
                for (int k = 0; k < 2; ++k)
#pragma unroll
                    for (int l = 0; l < 2; ++l) s += P.Am[k * 3 + i] * dS[k * 2 + l] * P.Am[l * 3 + j];
                dSig[i * 3 + j] = s;
            }
        float dAm[6];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            float t[3];
#pragma unroll
            for (int mm = 0; mm < 3; ++mm) t[mm] = dS[k * 2 + 0] * P.Am[mm] + dS[k * 2 + 1] * P.Am[3 + mm];
#pragma unroll
            for (int j = 0; j < 3; ++j)
                dAm[k * 3 + j] = 2.0f * (t[0] * Sig[0 * 3 + j] + t[1] * Sig[1 * 3 + j] + t[2] * Sig[2 * 3 + j]);
        }
        // Sigma = M M^T, M = R diag(s)
        float dR[9];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            float ds = 0.f;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const float dM = 2.0f * (dSig[i * 3 + 0] * P.M[0 * 3 + j] + dSig[i * 3 + 1] * P.M[1 * 3 + j] +
                                         dSig[i * 3 + 2] * P.M[2 * 3 + j]);
                ds += dM * P.Rq[i * 3 + j];
                dR[i * 3 + j] = dM * P.s[j];
            }
            gls[j] += ds * P.s[j];
        }
        {
            const float w = P.qn[0], x = P.qn[1], y = P.qn[2], z = P.qn[3];
            float dq[4];
            dq[0] = 2.f * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
            dq[1] = 2.f * (y * dR[1] + z * dR[2] + y * dR[3] - 2.f * x * dR[4] - w * dR[5] + z * dR[6] +
                           w * dR[7] - 2.f * x * dR[8]);
            dq[2] = 2.f * (-2.f * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                           z * dR[7] - 2.f * y * dR[8]);
            dq[3] = 2.f * (-2.f * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.f * z * dR[4] +
                           y * dR[5] + x * dR[6] + y * dR[7]);
            const float dot = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
            gq[0] += (dq[0] - w * dot) / P.qnorm;
            gq[1] += (dq[1] - x * dot) / P.qnorm;
            gq[2] += (dq[2] - y * dot) / P.qnorm;
            gq[3] += (dq[3] - z * dot) / P.qnorm;
        }
        // Am = J W; J depends on the camera-space mean
        const float* W = vw.R;
        const float z = P.z, x = P.p[0], y = P.p[1];
        const float fx = vw.fx, fy = vw.fy;
        const float dJ00 = dAm[0] * W[0] + dAm[1] * W[1] + dAm[2] * W[2];
        const float dJ02 = dAm[0] * W[6] + dAm[1] * W[7] + dAm[2] * W[8];
        const float dJ11 = dAm[3] * W[3] + dAm[4] * W[4] + dAm[5] * W[5];
        const float dJ12 = dAm[3] * W[6] + dAm[4] * W[7] + dAm[5] * W[8];
        const float iz = 1.0f / z, iz2 = iz * iz;
        float dp[3] = {0.f, 0.f, 0.f};
        dp[2] += dJ00 * (-fx * iz2) + dJ11 * (-fy * iz2);
        dp[2] += dJ02 * (fx * P.txc * iz2) + dJ12 * (fy * P.tyc * iz2);
        if (P.tx == P.txc) {
            const float dt = dJ02 * (-fx * iz);
            dp[0] += dt * iz;
            dp[2] += dt * (-x * iz2);
        }
        if (P.ty == P.tyc) {
            const float dt = dJ12 * (-fy * iz);
            dp[1] += dt * iz;
            dp[2] += dt * (-y * iz2);
        }
        dp[0] += d[0] * fx * iz;
        dp[2] += d[0] * (-fx * x * iz2);
        dp[1] += d[1] * fy * iz;
        dp[2] += d[1] * (-fy * y * iz2);
#pragma unroll
        for (int i = 0; i < 3; ++i) dmean[i] += W[0 * 3 + i] * dp[0] + W[1 * 3 + i] * dp[1] + W[2 * 3 + i] * dp[2];
#pragma unroll
        for (int i = 0; i < 3; ++i) gm[i] += dmean[i];
    }

    // gradients in parameter-block layout
    float4 G[15];
    G[0] = make_float4(gm[0], gm[1], gm[2], glo);
    G[1] = make_float4(gls[0], gls[1], gls[2], 0.f);
    G[2] = make_float4(gq[0], gq[1], gq[2], gq[3]);
#pragma unroll
    for (int q = 0; q < 12; ++q) G[3 + q] = make_float4(gsh[4 * q], gsh[4 * q + 1], gsh[4 * q + 2], gsh[4 * q + 3]);
    if (a.grads_out) {
#pragma unroll
        for (int q = 0; q < 15; ++q) a.grads_out[q * n + g] = G[q];
    }
    if (a.m) {
        const float bc1 = a.bias[0], bc2s = a.bias[1];
        const float b1 = a.beta1, b2 = a.beta2, eps = a.eps;
        float4 P4[15];
        P4[0] = p0; P4[1] = p1; P4[2] = p2;
#pragma unroll
        for (int q = 0; q < 12; ++q) P4[3 + q] = sh[q];
#pragma unroll
        for (int q = 0; q < 15; ++q) {
            float4 mm = a.m[q * n + g], vv = a.v[q * n + g], pp = P4[q];
            const float4 gg = G[q];
            // parameter group of each component
            int gr[4];
            if (q == 0) { gr[0] = gr[1] = gr[2] = 0; gr[3] = 3; }
            else if (q == 1) { gr[0] = gr[1] = gr[2] = 1; gr[3] = -1; }
            else if (q == 2) { gr[0] = gr[1] = gr[2] = gr[3] = 2; }
            else if (q == 3) { gr[0] = gr[1] = gr[2] = 4; gr[3] = 5; }
            else { gr[0] = gr[1] = gr[2] = gr[3] = 5; }
            if (gr[0] >= 0) pp.x = adam_one(pp.x, gg.x, mm.x, vv.x, a.lr[gr[0]], b1, b2, eps, bc1, bc2s);
            if (gr[1] >= 0) pp.y = adam_one(pp.y, gg.y, mm.y, vv.y, a.lr[gr[1]], b1, b2, eps, bc1, bc2s);
            if (gr[2] >= 0) pp.z = adam_one(pp.z, gg.z, mm.z, vv.z, a.lr[gr[2]], b1, b2, eps, bc1, bc2s);
            if (gr[3] >= 0) pp.w = adam_one(pp.w, gg.w, mm.w, vv.w, a.lr[gr[3]], b1, b2, eps, bc1, bc2s);
            a.params[q * n + g] = pp;
            a.m[q * n + g] = mm;
            a.v[q * n + g] = vv;
        }
    }
}

// step += 1; bias[0] = 1 - beta1^t, bias[1] = sqrt(1 - beta2^t)
__global__ void k_adam_tick(int32_t* step, float* bias, float beta1, float beta2) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int t = *step + 1;
    *step = t;
    bias[0] = (float)(1.0 - pow((double)beta1, (double)t));
    bias[1] = (float)sqrt(1.0 - pow((double)beta2, (double)t));
}

int launch_project_bwd_adam(float* params, int64_t n, const gs_view* views, const gs_layout& L,
                            const gs_bins& b, const gs_grads2d& grads, const gs_adam* adam,
                            float* grads_out, hipStream_t s) {
    if (n == 0) return GS_OK;
    AdamArgs a;
    memset(&a, 0, sizeof(a));
    a.params = reinterpret_cast<float4*>(params);
    a.n = n;
    a.views = views;
    a.n_views = L.n_views;
    a.tile = L.tile;
    for (int v = 0; v < GS_MAX_VIEWS; ++v) {
        a.gx[v] = v < L.n_views ? L.tiles_x[v] : 0;
        a.gy[v] = v < L.n_views ? L.tiles_y[v] : 0;
        a.tile_base[v] = v < L.n_views ? L.tile_base[v] : 0;
    }
    a.offsets = b.offsets;
    a.inv = b.inv;
    a.grec = reinterpret_cast<const float4*>(grads.rec);
    a.tile_stop = grads.tile_stop;
    a.capacity = b.capacity;
    a.grads_out = reinterpret_cast<float4*>(grads_out);
    if (adam) {
        a.m = reinterpret_cast<float4*>(adam->m);
        a.v = reinterpret_cast<float4*>(adam->v);
        a.bias = adam->scratch;
        for (int i = 0; i < 6; ++i) a.lr[i] = adam->lr[i];
        a.beta1 = adam->beta1;
        a.beta2 = adam->beta2;
        a.eps = adam->eps;
        hipLaunchKernelGGL(k_adam_tick, dim3(1), dim3(64), 0, s, adam->step, adam->scratch, adam->beta1,
                           adam->beta2);
        int rc = check_launch("adam_tick");
        if (rc != GS_OK) return rc;
    }
    hipLaunchKernelGGL(k_project_bwd_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return check_launch("project_bwd_adam");
}

}  // namespace gs
