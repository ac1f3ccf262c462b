// Projection backward fused with Adam, in two kernels.
//
// Record sums: the backward rasteriser wrote one screen-space gradient record
// per composited intersection at its unsorted index and flagged it in a bit
// mask, so a (view, Gaussian)'s records lie in its own contiguous index range
// and the 64 Gaussians of a wavefront own one contiguous range.  The
// wavefront walks that range 64 indices at a time, compacts the flagged
// indices into LDS, and sums each batch of 64 flagged records per owner with
// a segmented scan across lanes (owners ascend with the index); each run's
// total is added to its owner's accumulator in LDS, batch after batch, so the
// order of every sum is fixed.  The sums go to a dense [9][views * n] array,
// which the chain-rule kernel reads (and the caller may).
//
// Chain rule + Adam: one thread per Gaussian streams its parameter record and
// both Adam moments once, and writes parameters and moments once.  No
// per-parameter gradient buffer exists unless the caller asks for one
// (grads_out).  Log-scales and opacity logits are optimised as stored: the
// chain rule through exp and the sigmoid is part of this kernel.
//
// The forward quantities needed by the chain rule are recomputed with the same
// float32 code as the projection kernel, so every branch decision (culling,
// Jacobian clamp, colour clamp) matches the forward pass bitwise.
#include "project_math.h"

namespace gs {

struct RecArgs {
    const uint32_t* offsets;   // exclusive scan of the tile counts per (view, Gaussian)
    const uint32_t* rec_mask;
    const float4* grec;
    int64_t capacity;
    float* sums;
};

// No scratch: the record sums live in LDS.
size_t gather_workspace(int64_t) { return 0; }

constexpr int kAdamThreads = 256;
constexpr int kAdamWaves = kAdamThreads / kWave;

// Sums over the flagged records of (view, Gaussian own0 + lane) for the
// wavefront's 64 Gaussians, whose records occupy the index range [R0, R1)
// (lanes past n own nothing); `mine` is the range's mask word R0 / 32 + lane,
// loaded by the caller together with the other views' (a range of more than
// 64 words loads the rest here).  s_idx: 128 words, s_acc: 9 x 64 floats,
// both this wavefront's own.
GS_DEV void wave_record_sums(const RecArgs& r, uint32_t own0, uint32_t R0, uint32_t R1, uint32_t mine,
                             int lane, uint32_t* s_idx, float* s_acc, float d[9]) {
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int c = 0; c < 9; ++c) s_acc[c * kWave + lane] = 0.0f;
    // sum one batch of k <= 64 compacted indices s_idx[0, k) into s_acc
    auto batch = [&](int k) {
        __builtin_amdgcn_wave_barrier();
        const bool act = lane < k;
        float v[9];
        uint32_t own = 0xFFFFFFFFu;
#pragma unroll
        for (int c = 0; c < 9; ++c) v[c] = 0.0f;
        if (act) {
            const float4* q = r.grec + 3 * (int64_t)s_idx[lane];
            const float4 q0 = q[0], q1 = q[1], q2 = q[2];
            v[0] = q0.x; v[1] = q0.y; v[2] = q0.z; v[3] = q0.w;
            v[4] = q1.x; v[5] = q1.y; v[6] = q1.z; v[7] = q1.w; v[8] = q2.x;
            own = __float_as_uint(q2.y) - own0;
        }
        const uint32_t prev = (uint32_t)__shfl_up((int)own, 1);
        uint32_t head = (act && (lane == 0 || prev != own)) ? 1u : 0u;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            float y[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) y[c] = __shfl_up(v[c], off);
            const uint32_t hy = (uint32_t)__shfl_up((int)head, off);
            if (lane >= off && !head) {
#pragma unroll
                for (int c = 0; c < 9; ++c) v[c] = y[c] + v[c];
                head = hy;
            }
        }
        const uint32_t next = (uint32_t)__shfl_down((int)own, 1);
        const bool tail = act && (lane == k - 1 || next != own);
        if (tail && own < (uint32_t)kWave) {
#pragma unroll
            for (int c = 0; c < 9; ++c) s_acc[c * kWave + own] += v[c];
        }
        __builtin_amdgcn_wave_barrier();
    };
    int cnt = 0;
    if (R1 > R0) {
        // 64 mask words at a time (one per lane), then 64 indices (two words)
        // per step
        const uint32_t wlast = (R1 - 1) >> 5;
        for (uint32_t wb = R0 >> 5; wb <= wlast; wb += kWave) {
            if (wb != (R0 >> 5)) mine = wb + (uint32_t)lane <= wlast ? r.rec_mask[wb + lane] : 0u;
            const uint32_t nw = min((uint32_t)kWave, wlast - wb + 1);
            for (uint32_t k = 0; k < nw; k += 2) {
                const uint32_t idx = (wb + k) * 32u + (uint32_t)lane;
                const uint32_t word = (uint32_t)__shfl((int)mine, (int)k + (lane >> 5));
                const bool f = idx >= R0 && idx < R1 && ((word >> (lane & 31)) & 1u);
                const uint64_t m = __ballot(f);
                if (m == 0ull) continue;
                if (f) s_idx[cnt + __popcll(m & lt)] = idx;
                cnt += __popcll(m);
                if (cnt >= kWave) {
                    batch(kWave);
                    cnt -= kWave;
                    if (lane < cnt) s_idx[lane] = s_idx[kWave + lane];
                }
            }
        }
    }
    if (cnt > 0) batch(cnt);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int c = 0; c < 9; ++c) d[c] = s_acc[c * kWave + lane];
}

// views whose index ranges and first mask words are loaded together
constexpr int kViewGroup = 4;

// One wavefront per 64 consecutive Gaussians: their record sums in every view,
// to sums (every (view, Gaussian), zero where nothing was flagged).  A kernel
// of its own: beside the float64 chain rule (256 VGPRs, two wavefronts per
// SIMD) the walks and scans run with too little latency hiding at 8 views.
// Its first thread also advances the Adam step (when `step` is set): step +=
// 1, bias[0] = 1 - beta1^t, bias[1] = sqrt(1 - beta2^t), for the chain-rule
// kernel that follows.
__global__ __launch_bounds__(kAdamThreads) void k_record_sums(RecArgs r, int64_t n, int n_views, int32_t* step,
                                                              float* bias, float beta1, float beta2) {
    __shared__ uint32_t s_idx[kAdamWaves][2 * kWave];
    __shared__ float s_acc[kAdamWaves][9 * kWave];
    if (step && blockIdx.x == 0 && threadIdx.x == 0) {
        const int t = *step + 1;
        *step = t;
        bias[0] = (float)(1.0 - pow((double)beta1, (double)t));
        bias[1] = (float)sqrt(1.0 - pow((double)beta2, (double)t));
    }
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    const int64_t g0 = (int64_t)blockIdx.x * kAdamThreads + wv * kWave;
    if (g0 >= n) return;                    // whole wavefronts only
    const int64_t g = g0 + lane;
    const bool live = g < n;
    const int64_t vn = (int64_t)n_views * n;
    const int nlive = __popcll(__ballot(live));
    const uint64_t cap = (uint64_t)r.capacity;
    for (int v0 = 0; v0 < n_views; v0 += kViewGroup) {
        // the ranges and first mask words of kViewGroup views, loaded together
        uint32_t R0[kViewGroup], R1[kViewGroup], mine[kViewGroup];
#pragma unroll
        for (int j = 0; j < kViewGroup; ++j) {
            uint32_t ob = 0, oe = 0;
            if (live && v0 + j < n_views) {
                const int64_t o = (int64_t)(v0 + j) * n + g;
                ob = (uint32_t)min((uint64_t)r.offsets[o], cap);
                oe = (uint32_t)min((uint64_t)r.offsets[o + 1], cap);
            }
            // offsets ascend with the Gaussian: lane 0's start to the last
            // live lane's end
            R0[j] = (uint32_t)__shfl((int)ob, 0);
            R1[j] = (uint32_t)__shfl((int)oe, nlive - 1);
        }
#pragma unroll
        for (int j = 0; j < kViewGroup; ++j) {
            const uint32_t w0 = R0[j] >> 5;
            mine[j] = R1[j] > R0[j] && w0 + (uint32_t)lane <= ((R1[j] - 1) >> 5) ? r.rec_mask[w0 + lane] : 0u;
        }
#pragma unroll 1
        for (int j = 0; j < kViewGroup && v0 + j < n_views; ++j) {
            uint32_t r0 = R0[0], r1 = R1[0], mw = mine[0];
#pragma unroll
            for (int q = 1; q < kViewGroup; ++q)
                if (j == q) { r0 = R0[q]; r1 = R1[q]; mw = mine[q]; }
            float d[9];
            wave_record_sums(r, (uint32_t)((int64_t)(v0 + j) * n + g0), r0, r1, mw, lane, s_idx[wv], s_acc[wv], d);
            if (live) {
#pragma unroll
                for (int c = 0; c < 9; ++c) r.sums[c * vn + (int64_t)(v0 + j) * n + g] = d[c];
            }
        }
    }
}

struct AdamArgs {
    float4* params;
    int64_t n;
    const gs_view* views;
    int n_views;
    int tile;
    int cull;
    int32_t gx[GS_MAX_VIEWS], gy[GS_MAX_VIEWS];
    RecArgs rec;
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

// One Adam update (Kingma & Ba; the bias-corrected form of torch.optim.Adam):
// step = lr / (1 - beta1^t), inv_bc2s = 1 / sqrt(1 - beta2^t), both computed
// once per thread; the per-component square root and reciprocal are the
// hardware's (about 1 ulp), which moves the update by a relative 1e-7.
GS_DEV float adam_one(float p, float g, float& m, float& v, float step, float beta1, float beta2,
                      float eps, float inv_bc2s) {
    m = beta1 * m + (1.0f - beta1) * g;
    v = beta2 * v + (1.0f - beta2) * (g * g);
    const float denom = __builtin_amdgcn_sqrtf(v) * inv_bc2s + eps;
    return p - step * (m * __builtin_amdgcn_rcpf(denom));
}

__global__ __launch_bounds__(kAdamThreads, 2) void k_project_bwd_adam(AdamArgs a) {
    const int64_t n = a.n;
    const int64_t g = (int64_t)blockIdx.x * kAdamThreads + threadIdx.x;
    if (g >= n) return;
    const int64_t vn = (int64_t)a.n_views * n;
    const float4 p0 = a.params[0 * n + g];
    const float4 p1 = a.params[1 * n + g];
    const float4 p2 = a.params[2 * n + g];
    const bool finite = finite4(p0) && finite4(make_float4(p1.x, p1.y, p1.z, 0.0f)) && finite4(p2);
    float gm[3] = {0.f, 0.f, 0.f}, gls[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f};
    float glo = 0.f;
    float gsh[48];
#pragma unroll
    for (int i = 0; i < 48; ++i) gsh[i] = 0.f;

    for (int vi = 0; vi < a.n_views; ++vi) {
        const int64_t o = (int64_t)vi * n + g;
        if (!finite || a.rec.offsets[o + 1] == a.rec.offsets[o]) continue;
        float d[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) d[c] = a.rec.sums[c * vn + o];
        // SH coefficients are loaded per view and not kept: the Adam update
        // below reads them again, which keeps them out of the registers the
        // float64 chain rule needs
        float4 sh[12];
        bool sh_finite = true;
#pragma unroll
        for (int q = 0; q < 12; ++q) {
            sh[q] = a.params[(3 + q) * n + g];
            sh_finite = sh_finite && finite4(sh[q]);
        }
        if (!sh_finite) continue;
        const gs_view vw = a.views[vi];
        Proj P;
        project_gaussian<true, false>(p0, p1, p2, sh, vw, a.tile, a.gx[vi], a.gy[vi], a.cull, P);
        if (!P.valid) continue;

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
        // conic -> 2D covariance -> 3D covariance -> scales, rotation, and the
        // Jacobian's dependence on the mean.  These steps run in float64 from
        // the forward's float32 values: for elongated Gaussians the conic
        // gradients are orders of magnitude larger than the parameter
        // gradients they cancel down to, and float32 would lose most digits.
        const double A = P.A, B = P.B, C = P.C;
        const double g11 = d[2], g12 = 0.5 * (double)d[3], g22 = d[4];
        const double q00 = A * g11 + B * g12, q01 = A * g12 + B * g22;
        const double q10 = B * g11 + C * g12, q11 = B * g12 + C * g22;
        const double dS[4] = {-(q00 * A + q01 * B), -(q00 * B + q01 * C), -(q00 * B + q01 * C),
                              -(q10 * B + q11 * C)};
        double Am[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) Am[i] = P.Am[i];
        // 2D covariance = Am Sigma Am^T
        double dSig[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                double sacc = 0.0;
#pragma unroll
                for (int k = 0; k < 2; ++k)
#pragma unroll
                    for (int l = 0; l < 2; ++l) sacc += Am[k * 3 + i] * dS[k * 2 + l] * Am[l * 3 + j];
                dSig[i * 3 + j] = sacc;
            }
        double dAm[6];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            double t[3];
#pragma unroll
            for (int mm = 0; mm < 3; ++mm) t[mm] = dS[k * 2 + 0] * Am[mm] + dS[k * 2 + 1] * Am[3 + mm];
#pragma unroll
            for (int j = 0; j < 3; ++j)
                dAm[k * 3 + j] = 2.0 * (t[0] * (double)sig_at(P.Sig, 0, j) + t[1] * (double)sig_at(P.Sig, 1, j) +
                                        t[2] * (double)sig_at(P.Sig, 2, j));
        }
        // Sigma = M M^T, M = R diag(s)
        double dR[9];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double ds = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double dM = 2.0 * (dSig[i * 3 + 0] * (double)P.M[0 * 3 + j] +
                                         dSig[i * 3 + 1] * (double)P.M[1 * 3 + j] +
                                         dSig[i * 3 + 2] * (double)P.M[2 * 3 + j]);
                ds += dM * (double)P.Rq[i * 3 + j];
                dR[i * 3 + j] = dM * (double)P.s[j];
            }
            gls[j] += (float)(ds * (double)P.s[j]);
        }
        {
            const double w = P.qn[0], x = P.qn[1], y = P.qn[2], z = P.qn[3];
            double dq[4];
            dq[0] = 2.0 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
            dq[1] = 2.0 * (y * dR[1] + z * dR[2] + y * dR[3] - 2.0 * x * dR[4] - w * dR[5] + z * dR[6] +
                           w * dR[7] - 2.0 * x * dR[8]);
            dq[2] = 2.0 * (-2.0 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6] +
                           z * dR[7] - 2.0 * y * dR[8]);
            dq[3] = 2.0 * (-2.0 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2.0 * z * dR[4] +
                           y * dR[5] + x * dR[6] + y * dR[7]);
            const double dot = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
            const double iq = 1.0 / (double)P.qnorm;
            gq[0] += (float)((dq[0] - w * dot) * iq);
            gq[1] += (float)((dq[1] - x * dot) * iq);
            gq[2] += (float)((dq[2] - y * dot) * iq);
            gq[3] += (float)((dq[3] - z * dot) * iq);
        }
        // Am = J W; J depends on the camera-space mean
        const float* W = vw.R;
        const double z = P.z, x = P.p[0], y = P.p[1];
        const double fx = vw.fx, fy = vw.fy;
        const double dJ00 = dAm[0] * W[0] + dAm[1] * W[1] + dAm[2] * W[2];
        const double dJ02 = dAm[0] * W[6] + dAm[1] * W[7] + dAm[2] * W[8];
        const double dJ11 = dAm[3] * W[3] + dAm[4] * W[4] + dAm[5] * W[5];
        const double dJ12 = dAm[3] * W[6] + dAm[4] * W[7] + dAm[5] * W[8];
        const double iz = 1.0 / z, iz2 = iz * iz;
        double dp[3] = {0.0, 0.0, 0.0};
        dp[2] += dJ00 * (-fx * iz2) + dJ11 * (-fy * iz2);
        dp[2] += dJ02 * (fx * (double)P.txc * iz2) + dJ12 * (fy * (double)P.tyc * iz2);
        if (P.tx == P.txc) {
            const double dt = dJ02 * (-fx * iz);
            dp[0] += dt * iz;
            dp[2] += dt * (-x * iz2);
        }
        if (P.ty == P.tyc) {
            const double dt = dJ12 * (-fy * iz);
            dp[1] += dt * iz;
            dp[2] += dt * (-y * iz2);
        }
        dp[0] += (double)d[0] * fx * iz;
        dp[2] += (double)d[0] * (-fx * x * iz2);
        dp[1] += (double)d[1] * fy * iz;
        dp[2] += (double)d[1] * (-fy * y * iz2);
#pragma unroll
        for (int i = 0; i < 3; ++i)
            dmean[i] += (float)(W[0 * 3 + i] * dp[0] + W[1 * 3 + i] * dp[1] + W[2 * 3 + i] * dp[2]);
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
        const float inv_bc2s = 1.0f / bc2s;
        float step[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) step[k] = a.lr[k] / bc1;
        // the moments (and SH coefficients) of kAdamBatch planes are loaded
        // together, so a thread waits on memory twice rather than fifteen
        // times (eight planes fit in the registers; all fifteen spill)
        constexpr int kAdamBatch = 8;
#pragma unroll
        for (int q0 = 0; q0 < 15; q0 += kAdamBatch) {
            float4 mm[kAdamBatch], vv[kAdamBatch], pq[kAdamBatch];
#pragma unroll
            for (int j = 0; j < kAdamBatch; ++j) {
                if (q0 + j >= 15) break;
                mm[j] = a.m[(q0 + j) * n + g];
                vv[j] = a.v[(q0 + j) * n + g];
                const int q = q0 + j;
                pq[j] = q == 0 ? p0 : (q == 1 ? p1 : (q == 2 ? p2 : a.params[q * n + g]));
            }
#pragma unroll
            for (int j = 0; j < kAdamBatch; ++j) {
                const int q = q0 + j;
                if (q >= 15) break;
                float4 pp = pq[j];
                const float4 gg = G[q];
                // parameter group of each component
                int gr[4];
                if (q == 0) { gr[0] = gr[1] = gr[2] = 0; gr[3] = 3; }
                else if (q == 1) { gr[0] = gr[1] = gr[2] = 1; gr[3] = -1; }
                else if (q == 2) { gr[0] = gr[1] = gr[2] = gr[3] = 2; }
                else if (q == 3) { gr[0] = gr[1] = gr[2] = 4; gr[3] = 5; }
                else { gr[0] = gr[1] = gr[2] = gr[3] = 5; }
                if (gr[0] >= 0) pp.x = adam_one(pp.x, gg.x, mm[j].x, vv[j].x, step[gr[0]], b1, b2, eps, inv_bc2s);
                if (gr[1] >= 0) pp.y = adam_one(pp.y, gg.y, mm[j].y, vv[j].y, step[gr[1]], b1, b2, eps, inv_bc2s);
                if (gr[2] >= 0) pp.z = adam_one(pp.z, gg.z, mm[j].z, vv[j].z, step[gr[2]], b1, b2, eps, inv_bc2s);
                if (gr[3] >= 0) pp.w = adam_one(pp.w, gg.w, mm[j].w, vv[j].w, step[gr[3]], b1, b2, eps, inv_bc2s);
                a.params[q * n + g] = pp;
                a.m[q * n + g] = mm[j];
                a.v[q * n + g] = vv[j];
            }
        }
    }
}

// The no-allocation entry point: the projection backward needs no scratch at
// all (the record sums live in LDS), so it is the same launch.
int launch_project_bwd_adam_noalloc(float* params, int64_t n, const gs_view* views, const gs_layout& L,
                                    const gs_splats& splats, const gs_bins& b, const gs_grads2d& grads,
                                    const gs_adam* adam, float* grads_out, hipStream_t s) {
    return launch_project_bwd_adam(params, n, views, L, splats, b, grads, adam, grads_out, s);
}

int launch_project_bwd_adam(float* params, int64_t n, const gs_view* views, const gs_layout& L,
                            const gs_splats& splats, const gs_bins& b, const gs_grads2d& grads,
                            const gs_adam* adam, float* grads_out, hipStream_t s) {
    if (n == 0) return GS_OK;
    int rc = GS_OK;
    RecArgs ra;
    ra.offsets = b.offsets;
    ra.rec_mask = grads.rec_mask;
    ra.grec = reinterpret_cast<const float4*>(grads.rec);
    ra.capacity = b.capacity;
    ra.sums = grads.sums;
    AdamArgs a;
    memset(&a, 0, sizeof(a));
    a.params = reinterpret_cast<float4*>(params);
    a.n = n;
    a.views = views;
    a.n_views = L.n_views;
    a.tile = L.tile;
    a.cull = L.cull;
    for (int v = 0; v < GS_MAX_VIEWS; ++v) {
        a.gx[v] = v < L.n_views ? L.tiles_x[v] : 0;
        a.gy[v] = v < L.n_views ? L.tiles_y[v] : 0;
    }
    a.grads_out = reinterpret_cast<float4*>(grads_out);
    if (adam) {
        a.m = reinterpret_cast<float4*>(adam->m);
        a.v = reinterpret_cast<float4*>(adam->v);
        a.bias = adam->scratch;
        for (int i = 0; i < 6; ++i) a.lr[i] = adam->lr[i];
        a.beta1 = adam->beta1;
        a.beta2 = adam->beta2;
        a.eps = adam->eps;
    }
    a.rec = ra;
    hipLaunchKernelGGL(k_record_sums, dim3((unsigned)((n + kAdamThreads - 1) / kAdamThreads)), dim3(kAdamThreads),
                       0, s, ra, n, L.n_views, adam ? adam->step : nullptr, adam ? adam->scratch : nullptr,
                       adam ? adam->beta1 : 0.0f, adam ? adam->beta2 : 0.0f);
    rc = check_launch("record_sums");
    if (rc != GS_OK) return rc;
    hipLaunchKernelGGL(k_project_bwd_adam, dim3((unsigned)((n + kAdamThreads - 1) / kAdamThreads)),
                       dim3(kAdamThreads), 0, s, a);
    return check_launch("project_bwd_adam");
}

}  // namespace gs
