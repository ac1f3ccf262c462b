// Projection backward fused with Adam, in two passes.
//
// Gather: per (view, Gaussian), the sum of the screen-space gradient records
// the backward rasteriser flagged.  It wrote them at their unsorted indices,
// so a Gaussian's records are one contiguous range.  The sums go to a dense
// [9][views * n] array.
//
// Chain rule + Adam: one thread per Gaussian streams its parameter record and
// both Adam moments once, reads its per-view sums (coalesced), and writes
// parameters and moments once.  No per-parameter gradient buffer exists
// unless the caller asks for one (grads_out).  Log-scales and opacity logits
// are optimised as stored: the chain rule through exp and the sigmoid is part
// of this kernel.
//
// The forward quantities needed by the chain rule are recomputed with the same
// float32 code as the projection kernel, so every branch decision (culling,
// Jacobian clamp, colour clamp) matches the forward pass bitwise.
#include <mutex>

#include "project_math.h"

namespace gs {

struct GatherArgs {
    const uint32_t* offsets;
    const uint32_t* rec_mask;
    const float4* grec;
    int64_t n;
    int64_t capacity;
    int n_views;
    float* sums;
    float* part_first;      // per unit, kPart floats: owner bits, then the sum of the
                            // unit's first run (owner 0xFFFFFFFF: no run)
    float* part_last;       // per unit, kPart floats: the same for its last run, if it
                            // is not also the first
};

constexpr int kPart = 10;   // floats per partial slot

constexpr int kGatherThreads = 256;
constexpr int kGatherE = 512;                           // intersection indices per unit
constexpr int kGatherPer = kGatherE / kGatherThreads;   // indices per thread
static_assert(kGatherPer == 2, "two compacted records per thread in the segmented scan");

size_t gather_workspace(int64_t capacity) {
    const size_t nb = (size_t)((capacity + kGatherE - 1) / kGatherE) + 1;
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    return 2 * up(4 * kPart * nb);
}

static void carve_gather(void* ws, int64_t capacity, GatherArgs& g) {
    const size_t nb = (size_t)((capacity + kGatherE - 1) / kGatherE) + 1;
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    char* p = static_cast<char*>(ws);
    g.part_first = reinterpret_cast<float*>(p);
    p += up(4 * kPart * nb);
    g.part_last = reinterpret_cast<float*>(p);
}

// Number of valid intersections (clamped to the capacity).
GS_DEV uint64_t entries_valid(const GatherArgs& a, int64_t vn) {
    return min((uint64_t)a.offsets[vn], (uint64_t)a.capacity);
}

// Gather, one workgroup per unit of E intersection indices.  Each thread
// reads the record-mask bits of its indices; a workgroup scan of the flag
// counts gives every flagged record a slot, and the flagged records (9
// gradient components and the owner (view, Gaussian) the backward stored in
// the record) are compacted into LDS in index order.  A Gaussian's indices
// are one contiguous range, so its flagged records in the unit are one run of
// equal owner, summed by a segmented scan over the compacted records.
// A run with runs on both sides lies wholly inside the unit, so its sum is the
// Gaussian's and goes to sums; the unit's first run goes to its first partial
// slot and its last run (if there are two or more) to its last partial slot,
// each tagged with the owner, for the chain-rule kernel to add up.  Every unit
// writes the tags of both slots; sums of Gaussians without a middle run keep
// the zeros filled beforehand.
__global__ __launch_bounds__(kGatherThreads) void k_gather2d(GatherArgs a) {
    constexpr int NW = kGatherThreads / kWave;
    __shared__ float s_val[9][kGatherE];
    __shared__ uint32_t s_own[kGatherE];
    __shared__ uint32_t s_flag[kGatherThreads];
    __shared__ uint32_t s_wsum[NW];
    const int64_t vn = (int64_t)a.n_views * a.n;
    const uint64_t kc = entries_valid(a, vn);
    const uint32_t unit = blockIdx.x;
    const uint64_t e0 = (uint64_t)unit * kGatherE;
    if (e0 >= kc) return;
    const uint64_t e1 = min(e0 + (uint64_t)kGatherE, kc);
    const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
    const uint64_t i0 = e0 + (uint64_t)kGatherPer * t;
    uint32_t bits = 0;
    if (i0 < e1) {
        bits = (a.rec_mask[i0 >> 5] >> (uint32_t)(i0 & 31)) & ((1u << kGatherPer) - 1u);
        const uint64_t left = e1 - i0;
        if (left < (uint64_t)kGatherPer) bits &= (1u << left) - 1u;
    }
    const uint32_t cnt = (uint32_t)__popc(bits);
    uint32_t incl = cnt;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    if (lane == kWave - 1) s_wsum[w] = incl;
    if (t == 0) {
        a.part_first[kPart * (int64_t)unit] = __uint_as_float(0xFFFFFFFFu);
        a.part_last[kPart * (int64_t)unit] = __uint_as_float(0xFFFFFFFFu);
    }
    __syncthreads();
    uint32_t pos = incl - cnt, nf = 0;
#pragma unroll
    for (int j = 0; j < NW; ++j) {
        if (j < w) pos += s_wsum[j];
        nf += s_wsum[j];
    }
    if (nf == 0) return;
#pragma unroll
    for (int q = 0; q < kGatherPer; ++q) {
        if ((bits >> q) & 1u) {
            const float4* g = a.grec + 3 * (int64_t)(i0 + (uint64_t)q);
            const float4 r0 = g[0], r1 = g[1], r2 = g[2];
            s_val[0][pos] = r0.x; s_val[1][pos] = r0.y; s_val[2][pos] = r0.z; s_val[3][pos] = r0.w;
            s_val[4][pos] = r1.x; s_val[5][pos] = r1.y; s_val[6][pos] = r1.z; s_val[7][pos] = r1.w;
            s_val[8][pos] = r2.x;
            s_own[pos] = __float_as_uint(r2.y);
            ++pos;
        }
    }
    __syncthreads();
    // segmented inclusive scan over the compacted records, two per thread
    // (records 2t and 2t + 1): the last record of each run ends up with the
    // run's sum.  Per thread: the pair's aggregate; across threads: a
    // Hillis-Steele scan of (aggregate, run-start flag); then each record adds
    // the running sum before it unless a run starts at it.
    const uint32_t p0 = 2 * (uint32_t)t, p1 = p0 + 1;
    const bool act0 = p0 < nf, act1 = p1 < nf;
    const uint32_t own0 = act0 ? s_own[p0] : 0xFFFFFFFFu;
    const uint32_t own1 = act1 ? s_own[p1] : 0xFFFFFFFFu;
    const bool head0 = act0 && (p0 == 0 || s_own[p0 - 1] != own0);
    const bool head1 = act1 && own1 != own0;
    const bool tail0 = act0 && (!act1 || own1 != own0);
    const bool tail1 = act1 && (p1 == nf - 1 || s_own[p1 + 1] != own1);
    float v0[9], v1[9], agg[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        v0[c] = act0 ? s_val[c][p0] : 0.f;
        v1[c] = act1 ? s_val[c][p1] : 0.f;
        agg[c] = head1 ? v1[c] : v0[c] + v1[c];
    }
    uint32_t f = (head0 || head1) ? 1u : 0u;
    const uint32_t nt = (nf + 1) / 2;   // threads holding records
    for (uint32_t off = 1; off < nt; off <<= 1) {
        __syncthreads();
        s_flag[t] = f;
#pragma unroll
        for (int c = 0; c < 9; ++c) s_val[c][t] = agg[c];
        __syncthreads();
        if ((uint32_t)t >= off && !f) {
#pragma unroll
            for (int c = 0; c < 9; ++c) agg[c] = s_val[c][t - off] + agg[c];
            f = s_flag[t - off];
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 9; ++c) s_val[c][t] = agg[c];   // inclusive, per thread
    __syncthreads();
    if (!head0 && t > 0) {
#pragma unroll
        for (int c = 0; c < 9; ++c) v0[c] = s_val[c][t - 1] + v0[c];
    }
    if (!head1) {
#pragma unroll
        for (int c = 0; c < 9; ++c) v1[c] = v0[c] + v1[c];
    }
    // the unit's first run goes to the first slot, its last run (if not also
    // the first) to the last slot, every other run to sums
    const uint32_t first_own = s_own[0];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const bool tl = h == 0 ? tail0 : tail1;
        const uint32_t own = h == 0 ? own0 : own1;
        const uint32_t p = h == 0 ? p0 : p1;
        if (!tl || (int64_t)own >= vn) continue;
        float* dst;
        int64_t stride;
        if (own == first_own) { dst = a.part_first + kPart * (int64_t)unit; stride = 1; }
        else if (p == nf - 1) { dst = a.part_last + kPart * (int64_t)unit; stride = 1; }
        else { dst = a.sums + own; stride = vn; }
        if (stride == 1) {
            dst[0] = __uint_as_float(own);
            ++dst;
        }
#pragma unroll
        for (int c = 0; c < 9; ++c) dst[c * stride] = h == 0 ? v0[c] : v1[c];
    }
}

// Sum of the flagged records of (view, Gaussian) o: its middle run if it had
// one (sums, zero otherwise), then, unit by unit over the units its index
// range covers, the first and last partial slots tagged with o.  The result
// is also stored to sums when a partial slot contributed.
GS_DEV void gather_total(const GatherArgs& a, int64_t o, int64_t vn, float d[9]) {
    const uint64_t b = min((uint64_t)a.offsets[o], (uint64_t)a.capacity);
    const uint64_t e = min((uint64_t)a.offsets[o + 1], (uint64_t)a.capacity);
#pragma unroll
    for (int c = 0; c < 9; ++c) d[c] = a.sums[c * vn + o];
    if (e <= b) return;
    const uint32_t tag = (uint32_t)o;
    bool added = false;
    for (uint64_t u = b / kGatherE; u <= (e - 1) / kGatherE; ++u) {
        const float* pf = a.part_first + kPart * u;
        if (__float_as_uint(pf[0]) == tag) {
#pragma unroll
            for (int c = 0; c < 9; ++c) d[c] += pf[1 + c];
            added = true;
        }
        const float* pl = a.part_last + kPart * u;
        if (__float_as_uint(pl[0]) == tag) {
#pragma unroll
            for (int c = 0; c < 9; ++c) d[c] += pl[1 + c];
            added = true;
        }
    }
    if (added) {
#pragma unroll
        for (int c = 0; c < 9; ++c) a.sums[c * vn + o] = d[c];
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
    GatherArgs ga;
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

__global__ __launch_bounds__(256, 2) void k_project_bwd_adam(AdamArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.n) return;
    const int64_t n = a.n;
    const float4 p0 = a.params[0 * n + g];
    const float4 p1 = a.params[1 * n + g];
    const float4 p2 = a.params[2 * n + g];
    const bool finite = finite4(p0) && finite4(make_float4(p1.x, p1.y, p1.z, 0.0f)) && finite4(p2);
    float gm[3] = {0.f, 0.f, 0.f}, gls[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f};
    float glo = 0.f;
    float gsh[48];
#pragma unroll
    for (int i = 0; i < 48; ++i) gsh[i] = 0.f;

    const int64_t vn = (int64_t)a.n_views * n;
    for (int vi = 0; vi < a.n_views; ++vi) {
        const int64_t o = (int64_t)vi * n + g;
        float d[9];
        gather_total(a.ga, o, vn, d);
        if (!finite || a.ga.offsets[o + 1] == a.ga.offsets[o]) continue;
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
        // together, so a thread waits on memory three times rather than fifteen
        constexpr int kAdamBatch = 5;
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

// step += 1; bias[0] = 1 - beta1^t, bias[1] = sqrt(1 - beta2^t)
__global__ void k_adam_tick(int32_t* step, float* bias, float beta1, float beta2) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int t = *step + 1;
    *step = t;
    bias[0] = (float)(1.0 - pow((double)beta1, (double)t));
    bias[1] = (float)sqrt(1.0 - pow((double)beta2, (double)t));
}

// Device scratch of gs_project_bwd_adam_noalloc: the gather's partial slots.
// Host code never uses the array's name as an address: each device's copy is
// found once with hipGetSymbolAddress (with that device current) and that
// pointer is what the kernels receive.
static __device__ __align__(256) unsigned char scratch[GS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

static int noalloc_scratch(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error("gs_project_bwd_adam_noalloc: hipGetDevice: %s", hipGetErrorString(e));
        return GS_ERR_HIP;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("gs_project_bwd_adam_noalloc: device %d beyond %d", dev, kMaxDevices);
        return GS_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("gs_project_bwd_adam_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
            return GS_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GS_OK;
}

int launch_project_bwd_adam_noalloc(float* params, int64_t n, const gs_view* views, const gs_layout& L,
                                    const gs_splats& splats, const gs_bins& b, const gs_grads2d& grads,
                                    const gs_adam* adam, float* grads_out, hipStream_t s) {
    const size_t need = gather_workspace(b.capacity);
    if (need > (size_t)GS_NOALLOC_SCRATCH_BYTES) {
        set_error("gs_project_bwd_adam_noalloc: capacity %lld needs %zu bytes of scratch, more than the "
                  "%zu the library holds",
                  (long long)b.capacity, need, (size_t)GS_NOALLOC_SCRATCH_BYTES);
        return GS_ERR_WORKSPACE;
    }
    void* ws = nullptr;
    const int rc = noalloc_scratch(&ws);
    if (rc != GS_OK) return rc;
    gs_grads2d g = grads;
    g.workspace = ws;
    return launch_project_bwd_adam(params, n, views, L, splats, b, g, adam, grads_out, s);
}

int launch_project_bwd_adam(float* params, int64_t n, const gs_view* views, const gs_layout& L,
                            const gs_splats& splats, const gs_bins& b, const gs_grads2d& grads,
                            const gs_adam* adam, float* grads_out, hipStream_t s) {
    if (n == 0) return GS_OK;
    int rc = GS_OK;
    GatherArgs ga;
    memset(&ga, 0, sizeof(ga));
    ga.offsets = b.offsets;
    ga.rec_mask = grads.rec_mask;
    ga.grec = reinterpret_cast<const float4*>(grads.rec);
    ga.n = n;
    ga.capacity = b.capacity;
    ga.n_views = L.n_views;
    ga.sums = grads.sums;
    carve_gather(grads.workspace, b.capacity, ga);
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
        hipLaunchKernelGGL(k_adam_tick, dim3(1), dim3(64), 0, s, adam->step, adam->scratch, adam->beta1,
                           adam->beta2);
        rc = check_launch("adam_tick");
        if (rc != GS_OK) return rc;
    }
    const int64_t vn = (int64_t)L.n_views * n;
    // sums of Gaussians without any flagged record stay zero
    rc = launch_fill_u32(reinterpret_cast<uint32_t*>(ga.sums), 0u, 9 * vn, s);
    if (rc != GS_OK) return rc;
    if (b.capacity > 0) {
        hipLaunchKernelGGL(k_gather2d, dim3((unsigned)((b.capacity + kGatherE - 1) / kGatherE)),
                           dim3(kGatherThreads), 0, s, ga);
        rc = check_launch("gather2d");
        if (rc != GS_OK) return rc;
    }
    a.ga = ga;
    hipLaunchKernelGGL(k_project_bwd_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return check_launch("project_bwd_adam");
}

}  // namespace gs
