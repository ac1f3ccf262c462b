// Tile rasteriser: forward alpha compositing and its exact backward.
//
// One workgroup renders one T x T tile (T = 8, 16, 32) with T*T/P lanes, each
// lane rendering P pixels (P = 1 for T = 8; 1, 2 or 4 otherwise, default 2).
// The tile's sorted Gaussian list is consumed in
// batches of S records gathered into LDS; every lane then reads the batch
// with broadcast LDS loads.  The conic is staged pre-scaled by -log2(e)/2 so
// that a pair costs one v_exp_f32.
//
// Backward: alpha is recomputed with the forward's own device function
// (explicit FMAs, so bitwise the forward's alpha), and a pair counts as
// composited when the pixel's forward stop (`last`) lies beyond it and alpha
// reaches the 1/255 cut, so the set of composited pairs is the forward's.
// Transmittance is recomputed front to back as T - alpha T (the forward keeps
// T (1 - alpha), which it also tests against the stop threshold): the two
// agree to float rounding and no decision depends on the backward's value.
// Using the forward's output colour, the colour behind entry i is C_out -
// (colour composited up to and including i), so no per-pair state is stored.  Per-pixel gradient terms
// are summed over each wavefront with DPP row/broadcast reductions (no
// atomics), waves whose lanes all skip a Gaussian skip its reduction (ballot),
// and the per-wave sums are added in a fixed order through LDS: one 48-byte
// record per (Gaussian, tile) intersection that some pixel composited,
// written at its unsorted index (so each Gaussian's records are contiguous
// for the gather that follows) and flagged in a bit mask, deterministic.  The
// forward marks, per sorted entry, whether any pixel of the tile composited
// it; the backward stages only those entries (the others have no gradient),
// and stops at the last entry any of its pixels composited.
//
// Scheduling: either one workgroup per tile, or a persistent grid popping
// tiles from a device counter in the order of a permutation (static or
// learned); the choice changes no output bit.
#include "gs_internal.h"

#pragma clang fp contract(off)

namespace gs {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;

struct RasterArgs {
    gs_layout L;
    const float4* rec;      // 4 float4 per (view, Gaussian)
    const uint32_t* vals;   // Gaussian id per sorted position
    const uint2* ranges;
    const gs_view* views;
    int64_t n;
    const uint32_t* order;  // nullable
    uint32_t* counter;      // nullable: non-null selects the persistent schedule
    int32_t total_tiles;
    // forward outputs / backward inputs
    float* out_rgb;
    float* out_T;
    uint32_t* out_last;
    uint32_t* tile_stats;
    uint32_t* comp_mask;    // bit per sorted entry: composited by some pixel of its tile
    uint32_t* rec_mask;     // bit per unsorted index: gradient record written
    // backward
    const float* target;
    const float* dLdC;
    float inv_count;
    float4* grec;           // 3 float4 per unsorted index
    uint32_t* tile_stop;
    const uint32_t* row_offsets;
    const uint4* rows;
    int64_t row_capacity;
    float* loss;
    int64_t capacity;
    int adaptive_batch;     // backward: per-tile batch ceil(sqrt(N P)) to a multiple of 64, capped at S
};

// Staged splat: (u, v, -A log2e / 2, -B log2e), (-C log2e / 2, o, r, g), b
GS_DEV void stage_splat(const RasterArgs& a, int view, uint32_t sorted_pos, float4& sg, float4& sh,
                        float& sb, uint32_t& gid) {
    gid = a.vals[sorted_pos];
    const float4* r = a.rec + 4 * ((int64_t)view * a.n + gid);
    const float4 q0 = r[0];
    const float4 q1 = r[1];
    const float4 q2 = r[2];
    sg = make_float4(q0.x, q0.y, (-0.5f * kLog2e) * q0.z, (-kLog2e) * q0.w);
    sh = make_float4((-0.5f * kLog2e) * q1.x, q1.y, q1.z, q1.w);
    sb = q2.x;
}

// Unsorted index of (tile (tx, ty), Gaussian gid) in view `view`: the first
// index of the Gaussian's tile row ty plus the column offset within the
// row's span; 0xFFFFFFFF if the row slot is missing (row capacity exceeded).
GS_DEV uint32_t unsorted_index(const RasterArgs& a, int view, uint32_t gid, int tx, int ty) {
    const int64_t o = (int64_t)view * a.n + gid;
    const uint32_t y0 = __float_as_uint(a.rec[4 * o + 3].x) >> 16;
    const uint64_t slot = (uint64_t)a.row_offsets[o] + ((uint32_t)ty - y0);
    if (slot >= (uint64_t)a.row_capacity) return 0xFFFFFFFFu;
    const uint4 row = a.rows[slot];
    return row.x + ((uint32_t)tx - (row.z & 0xFFFFu));
}

// Quadratic form (log2-scaled power) at the pixel, G = 2^power and o*G.
// Returns false when the power is positive (the pair is skipped); G and o*G
// are computed either way so callers can select instead of branching.
GS_DEV bool eval_pair(float px, float py, const float4& sg, const float4& sh, float& dx, float& dy,
                      float& G, float& ag) {
    dx = px - sg.x;
    dy = py - sg.y;
    const float p2 = __builtin_fmaf(sg.z * dx, dx, __builtin_fmaf(sh.x * dy, dy, (sg.w * dx) * dy));
    G = __builtin_amdgcn_exp2f(p2);
    ag = sh.y * G;
    return !(p2 > 0.0f);
}

// Without an order, workgroups (dealt to the 8 XCDs in turn) take chunks of
// kXcdChunk consecutive tiles, chunk c on XCD c % 8, so that neighbouring
// tiles, which stage many of the same splats, read them through one L2; the
// grid is padded to whole rounds of 8 chunks.
constexpr uint32_t kXcds = 8, kXcdChunk = 64;
GS_DEV uint32_t chunked_tile(uint32_t b) {
    const uint32_t x = b % kXcds, i = b / kXcds;
    return ((i / kXcdChunk) * kXcds + x) * kXcdChunk + i % kXcdChunk;
}

// Next tile of this workgroup: -1 = no more work, -2 = skip (an order entry
// outside [0, total tiles) is ignored rather than followed out of bounds).
GS_DEV int next_tile(const RasterArgs& a, int* s_tile) {
    if (a.counter == nullptr) {
        const uint32_t t = a.order ? a.order[blockIdx.x] : chunked_tile(blockIdx.x);
        return t < (uint32_t)a.total_tiles ? (int)t : -2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t k = atomicAdd(a.counter, 1u);
        int t = -1;
        if (k < (uint32_t)a.total_tiles) {
            const uint32_t o = a.order ? a.order[k] : k;
            t = o < (uint32_t)a.total_tiles ? (int)o : -2;
        }
        *s_tile = t;
    }
    __syncthreads();
    return *s_tile;
}

// Pixels per lane: a T x T tile is covered by T*T/PPT lanes.  Wavefront w
// holds the 64 PPT consecutive pixels [64 PPT w, 64 PPT (w + 1)) of the tile
// (row major), i.e. whole tile rows, lane l the pixels 64 PPT w + 64 q + l.
// More pixels per lane read each staged Gaussian from LDS once for several
// pixels, give independent transmittance chains to interleave and share the
// backward's per-Gaussian wavefront reduction; fewer give more wavefronts per
// tile to hide latency (with 16x16 tiles, PPT = 4 is one wavefront per tile).
template <int TILE, int PPT_>
struct Geo {
    static constexpr int PPT = PPT_;
    static constexpr int NT = TILE * TILE / PPT;
    static constexpr int NW = NT / kWave;
    static constexpr int ROWS = kWave * PPT / TILE;   // tile rows per wavefront
    static_assert(NT % kWave == 0 && (kWave * PPT) % TILE == 0, "whole rows per wavefront");
    // tile-local pixel index of lane t's q-th pixel
    static GS_DEV int pixel(int t, int q) { return (t / kWave) * (kWave * PPT) + q * kWave + (t % kWave); }
};

// Whether any pixel centre of the rectangle [x0, x1] x [y0, y1] can give the
// staged Gaussian alpha >= 1/255, decided conservatively: the largest
// log2-scaled power over the rectangle (the concave quadratic's maximum, at
// the mean if it lies inside, else on an edge at the clamped 1D maximiser)
// plus a margin for float rounding, against log2(1 / (255 o)).  False only
// when every pixel of the rectangle would skip the pair, so leaving such
// pairs out changes no result.
GS_DEV bool rect_may_composite(const float4& sg, const float4& sh, float x0, float x1, float y0,
                               float y1) {
    const float a = sg.z, b = sg.w, c = sh.x;   // p2 = a dx^2 + b dx dy + c dy^2, a, c < 0
    const float X0 = x0 - sg.x, X1 = x1 - sg.x, Y0 = y0 - sg.y, Y1 = y1 - sg.y;
    float fmax = 0.0f;
    if (!(X0 <= 0.0f && X1 >= 0.0f && Y0 <= 0.0f && Y1 >= 0.0f)) {
        const float ky = -b / (2.0f * c), kx = -b / (2.0f * a);
        float dy = fminf(fmaxf(ky * X0, Y0), Y1);
        const float e0 = a * X0 * X0 + (b * X0) * dy + c * dy * dy;
        dy = fminf(fmaxf(ky * X1, Y0), Y1);
        const float e1 = a * X1 * X1 + (b * X1) * dy + c * dy * dy;
        float dx = fminf(fmaxf(kx * Y0, X0), X1);
        const float e2 = c * Y0 * Y0 + (b * Y0) * dx + a * dx * dx;
        dx = fminf(fmaxf(kx * Y1, X0), X1);
        const float e3 = c * Y1 * Y1 + (b * Y1) * dx + a * dx * dx;
        fmax = fmaxf(fmaxf(e0, e1), fmaxf(e2, e3));
    }
    const float DX = fmaxf(fabsf(X0), fabsf(X1)), DY = fmaxf(fabsf(Y0), fabsf(Y1));
    const float mag = fabsf(a) * DX * DX + fabsf(c) * DY * DY + fabsf(b) * DX * DY;
    const float L = -__log2f(255.0f * sh.y);
    return !(fmax + 1e-5f * (mag + fabsf(L) + 1.0f) < L);
}

struct TileInfo {
    int view, tx, ty, W, H;
    int64_t pix_base;
    uint2 range;
};

GS_DEV TileInfo tile_info(const RasterArgs& a, int gt) {
    TileInfo t;
    t.view = view_of_tile(a.L, gt);
    const int lt = gt - a.L.tile_base[t.view];
    const int gx = a.L.tiles_x[t.view];
    t.tx = lt % gx;
    t.ty = lt / gx;
    t.W = a.L.width[t.view];
    t.H = a.L.height[t.view];
    t.pix_base = a.L.pixel_base[t.view];
    t.range = a.ranges[gt];
    return t;
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------

template <int CTRL, int ROW_MASK>
GS_DEV uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, false);
}

// OR of `bits` over the wavefront (DPP within rows, ds_bpermute across rows),
// added to *word by one lane if non-zero.  addr16/addr32 = 4 (lane ^ 16 / 32).
GS_DEV void flush_comp_bits(uint32_t* word, uint32_t bits, int addr16, int addr32) {
    bits |= dpp_u32<0xB1, 0xF>(bits);
    bits |= dpp_u32<0x4E, 0xF>(bits);
    bits |= dpp_u32<0x141, 0xF>(bits);
    bits |= dpp_u32<0x140, 0xF>(bits);
    bits |= (uint32_t)__builtin_amdgcn_ds_bpermute(addr16, (int)bits);
    bits |= (uint32_t)__builtin_amdgcn_ds_bpermute(addr32, (int)bits);
    if (bits != 0u && (threadIdx.x & (kWave - 1)) == 0) atomicOr(word, bits);
}

template <int TILE, int S, int PPT_, bool STATS>
__global__ __launch_bounds__(TILE * TILE / PPT_) void k_raster_fwd(RasterArgs a) {
    constexpr int PPT = PPT_, NT = Geo<TILE, PPT_>::NT;
    const int lane_ = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int addr16 = (lane_ ^ 16) << 2, addr32 = (lane_ ^ 32) << 2;
    __shared__ float4 s_g[S];
    __shared__ float4 s_h[S];
    __shared__ float s_b[S];
    __shared__ int s_tile;
    __shared__ uint32_t s_max, s_sum, s_comp;
    for (;;) {
        const int gt = next_tile(a, &s_tile);
        if (gt == -1 || (gt == -2 && a.counter == nullptr)) break;
        if (gt == -2) continue;
        const TileInfo ti = tile_info(a, gt);
        const uint32_t start = ti.range.x, end = ti.range.y;
        float px[PPT], py[PPT], T[PPT], C0[PPT], C1[PPT], C2[PPT];
        uint32_t last[PPT], examined[PPT], composited[PPT];
        bool active[PPT], inside[PPT];
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int p = Geo<TILE, PPT_>::pixel((int)threadIdx.x, q);
            const int ix = ti.tx * TILE + p % TILE, iy = ti.ty * TILE + p / TILE;
            px[q] = (float)ix + 0.5f;
            py[q] = (float)iy + 0.5f;
            inside[q] = ix < ti.W && iy < ti.H;
            active[q] = inside[q];
            T[q] = 1.0f; C0[q] = 0.0f; C1[q] = 0.0f; C2[q] = 0.0f;
            last[q] = 0; examined[q] = 0; composited[q] = 0;
        }
        if (STATS && threadIdx.x == 0) { s_max = 0; s_sum = 0; s_comp = 0; }
        for (uint32_t b0 = start; b0 < end; b0 += S) {
            bool any = false;
#pragma unroll
            for (int q = 0; q < PPT; ++q) any = any || active[q];
            if (__syncthreads_count(any) == 0) break;
            for (int i = threadIdx.x; i < S; i += NT) {
                const uint32_t j = b0 + i;
                if (j < end) {
                    uint32_t gid;
                    stage_splat(a, ti.view, j, s_g[i], s_h[i], s_b[i], gid);
                }
            }
            __syncthreads();
            // branch-free inner loop: every lane evaluates every staged Gaussian
            // for each of its pixels and the decisions select what accumulates;
            // a wavefront whose pixels have all stopped leaves the batch
            if (__ballot(any) != 0ull) {
                const int cnt = (int)min((uint32_t)S, end - b0);
                const uint32_t base = b0 - start + 1u;
                // the staged Gaussians some pixel of this wavefront's rows can
                // composite; the others would change nothing and are passed over
                constexpr int NR = (S + kWave - 1) / kWave;
                const float rx0 = (float)(ti.tx * TILE) + 0.5f, rx1 = rx0 + (float)(TILE - 1);
                const float ry0 = (float)(ti.ty * TILE + wv * Geo<TILE, PPT_>::ROWS) + 0.5f;
                const float ry1 = ry0 + (float)(Geo<TILE, PPT_>::ROWS - 1);
                uint64_t rel[NR];
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    const int k = i * kWave + lane_;
                    rel[i] = __ballot(k < cnt && rect_may_composite(s_g[k], s_h[k], rx0, rx1, ry0, ry1));
                }
                // bits of comp_mask for the entries of this batch that this
                // lane's pixels composited, OR-reduced over the wavefront and
                // flushed once per 32-bit word of the mask
                uint32_t lbits = 0, word = b0 >> 5;
                int prev = -1;
                bool done = false;
#pragma unroll
                for (int i = 0; i < NR; ++i) {
                    if (done) break;
                    for (uint64_t m = rel[i]; m != 0ull; m &= m - 1ull) {
                        const int k = i * kWave + (int)__builtin_ctzll(m);
                        const uint32_t j = b0 + (uint32_t)k;
                        if ((j >> 5) != word) {
                            if (__ballot(lbits != 0u) != 0ull)
                                flush_comp_bits(a.comp_mask + word, lbits, addr16, addr32);
                            lbits = 0;
                            word = j >> 5;
                        }
                        const float4 sg = s_g[k];
                        const float4 sh = s_h[k];
                        const float cb = s_b[k];
                        bool still = false, compd = false;
#pragma unroll
                        for (int q = 0; q < PPT; ++q) {
                            float dx, dy, G, ag;
                            const bool in = eval_pair(px[q], py[q], sg, sh, dx, dy, G, ag);
                            const float alpha = fminf(kAlphaMax, ag);
                            const bool ok = active[q] && in && alpha >= kAlphaMin;
                            const float test_T = T[q] * (1.0f - alpha);
                            const bool stop = ok && test_T < kTMin;
                            const bool comp = ok && !stop;
                            // entries passed over since the previous one count as examined
                            if (STATS) examined[q] += active[q] ? (uint32_t)(k - prev) : 0u;
                            active[q] = active[q] && !stop;
                            const float w = comp ? alpha * T[q] : 0.0f;
                            C0[q] = __builtin_fmaf(w, sh.z, C0[q]);
                            C1[q] = __builtin_fmaf(w, sh.w, C1[q]);
                            C2[q] = __builtin_fmaf(w, cb, C2[q]);
                            T[q] = comp ? test_T : T[q];
                            last[q] = comp ? base + (uint32_t)k : last[q];
                            if (STATS) composited[q] += comp ? 1u : 0u;
                            still = still || active[q];
                            compd = compd || comp;
                        }
                        prev = k;
                        lbits |= compd ? 1u << (j & 31u) : 0u;
                        if (__ballot(still) == 0ull) {
                            done = true;
                            break;
                        }
                    }
                }
                if (STATS && !done) {
#pragma unroll
                    for (int q = 0; q < PPT; ++q) examined[q] += active[q] ? (uint32_t)(cnt - 1 - prev) : 0u;
                }
                if (__ballot(lbits != 0u) != 0ull) flush_comp_bits(a.comp_mask + word, lbits, addr16, addr32);
            }
        }
        const float* bg = a.views[ti.view].bg;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            if (!inside[q]) continue;
            const int p = Geo<TILE, PPT_>::pixel((int)threadIdx.x, q);
            const int64_t pix = ti.pix_base + (int64_t)(ti.ty * TILE + p / TILE) * ti.W +
                                ti.tx * TILE + p % TILE;
            a.out_rgb[3 * pix + 0] = __builtin_fmaf(T[q], bg[0], C0[q]);
            a.out_rgb[3 * pix + 1] = __builtin_fmaf(T[q], bg[1], C1[q]);
            a.out_rgb[3 * pix + 2] = __builtin_fmaf(T[q], bg[2], C2[q]);
            a.out_T[pix] = T[q];
            a.out_last[pix] = last[q];
        }
        if (STATS) {
            uint32_t mx = 0, sm = 0, cp = 0;
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                mx = max(mx, examined[q]);
                sm += examined[q];
                cp += composited[q];
            }
            __syncthreads();
            atomicMax(&s_max, mx);
            atomicAdd(&s_sum, sm);
            atomicAdd(&s_comp, cp);
            __syncthreads();
            if (threadIdx.x == 0) {
                a.tile_stats[4 * (int64_t)gt + 0] = s_max;
                a.tile_stats[4 * (int64_t)gt + 1] = s_sum;
                a.tile_stats[4 * (int64_t)gt + 2] = s_comp;
                a.tile_stats[4 * (int64_t)gt + 3] = 0u;
            }
        }
        if (a.counter == nullptr) break;
    }
}

// ---------------------------------------------------------------------------
// wavefront reduction (DPP): lane 63 receives the sum of all 64 lanes
// ---------------------------------------------------------------------------

template <int CTRL, int ROW_MASK>
GS_DEV float dpp(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xF, false));
}

// Sum over the 16 lanes of each DPP row; every lane of the row gets the sum.
GS_DEV float row_sum(float v) {
    v += dpp<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v += dpp<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v += dpp<0x141, 0xF>(v);  // row_half_mirror
    v += dpp<0x140, 0xF>(v);  // row_mirror
    return v;
}

// The two results of a lane swap, kept apart: without the empty asm the
// compiler in use folds r[0] + r[1] of chained swaps into r[0] + r[0].
GS_DEV float swap_sum(uint32_t x, uint32_t y) {
    asm volatile("" : "+v"(x), "+v"(y));
    return __builtin_bit_cast(float, x) + __builtin_bit_cast(float, y);
}

// Lane-pair sums across the wavefront's halves (v_permlane32_swap): lane l of
// the lower half gets a[l] + a[l + 32], lane l of the upper half b[l - 32] + b[l].
GS_DEV float fold32(float a, float b) {
    const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(uint32_t, a), __builtin_bit_cast(uint32_t, b),
                                                    false, false);
    return swap_sum(r[0], r[1]);
}

// Row-pair sums (v_permlane16_swap): rows 0 and 2 get a's sums over rows
// (0, 1) and (2, 3), rows 1 and 3 b's.
GS_DEV float fold16(float a, float b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(uint32_t, a), __builtin_bit_cast(uint32_t, b),
                                                    false, false);
    return swap_sum(r[0], r[1]);
}

// Wavefront sums of nine values: halves folded pairwise, then row pairs, then
// rows.  Lane 16 r of the result holds the sum of v[(0, 2, 1, 3)[r]], lane
// 16 r + 1 that of v[(4, 6, 5, 7)[r]], and every lane that of v[8]; sum9_slot
// gives the component each lane holds (-1: none it should write).
GS_DEV float sum9(float v0, float v1, float v2, float v3, float v4, float v5, float v6, float v7, float v8,
                  int pos16) {
    const float b0 = row_sum(fold16(fold32(v0, v1), fold32(v2, v3)));
    const float b1 = row_sum(fold16(fold32(v4, v5), fold32(v6, v7)));
    const float a8 = fold32(v8, v8);
    const float b8 = row_sum(fold16(a8, a8));
    return pos16 == 0 ? b0 : (pos16 == 1 ? b1 : b8);
}

GS_DEV int sum9_slot(int lane) {
    const int row = lane >> 4, pos16 = lane & 15, c = ((row & 1) << 1) | (row >> 1);
    return pos16 == 0 ? c : (pos16 == 1 ? 4 + c : (lane == 2 ? 8 : -1));
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------

// With one or two pixels per lane the kernel is held to 72 VGPRs, seven
// wavefronts per SIMD: the per-Gaussian chain (LDS read, exp, compare,
// uniform branch) needs that many wavefronts to keep the VALU busy, and the
// compiler then keeps two per-tile values in scratch (reloaded once per tile,
// outside the Gaussian loops).  Six (76 VGPRs) and eight (64) were no faster
// than five.
template <int TILE, int S, int PPT_>
__global__ __launch_bounds__(TILE * TILE / PPT_) __attribute__((amdgpu_waves_per_eu(PPT_ <= 2 ? 7 : 1)))
void k_raster_bwd(RasterArgs a) {
    constexpr int PPT = PPT_, NT = Geo<TILE, PPT_>::NT, NW = Geo<TILE, PPT_>::NW;
    constexpr int SUB = 64;  // Gaussians per reduction sub-batch
    static_assert(SUB == kWave, "one relevance ballot per sub-batch");
    __shared__ float4 s_g[S];
    __shared__ float4 s_h[S];
    __shared__ float s_b[S];
    __shared__ uint32_t s_gid[S];
    __shared__ uint32_t s_idx[S];
    __shared__ uint32_t s_pos[S];
    __shared__ uint32_t s_mw[S / 32 + 2];
    __shared__ float s_red[NW][SUB][9];
    __shared__ uint64_t s_mask[NW];
    __shared__ int s_tile;
    __shared__ uint32_t s_len;
    __shared__ float s_loss[NW];
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (;;) {
        const int gt = next_tile(a, &s_tile);
        if (gt == -1 || (gt == -2 && a.counter == nullptr)) break;
        if (gt == -2) continue;
        const TileInfo ti = tile_info(a, gt);
        const uint32_t start = ti.range.x;
        // per pixel: dL/dC (g), transmittance T and R = g . (colour composited
        // behind the current entry, background included), starting at g . C_out
        float px[PPT], py[PPT], g0[PPT], g1[PPT], g2[PPT], T[PPT], R[PPT];
        uint32_t lastp[PPT];
        float l1 = 0.0f;
        uint32_t mylen = 0;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int p = Geo<TILE, PPT_>::pixel((int)threadIdx.x, q);
            const int ix = ti.tx * TILE + p % TILE, iy = ti.ty * TILE + p / TILE;
            px[q] = (float)ix + 0.5f;
            py[q] = (float)iy + 0.5f;
            g0[q] = g1[q] = g2[q] = 0.0f;
            T[q] = 1.0f; R[q] = 0.0f;
            lastp[q] = 0;
            if (ix < ti.W && iy < ti.H) {
                const int64_t pix = ti.pix_base + (int64_t)iy * ti.W + ix;
                const float Co0 = a.out_rgb[3 * pix + 0];
                const float Co1 = a.out_rgb[3 * pix + 1];
                const float Co2 = a.out_rgb[3 * pix + 2];
                lastp[q] = a.out_last[pix];
                if (a.target) {
                    const float d0 = Co0 - a.target[3 * pix + 0];
                    const float d1 = Co1 - a.target[3 * pix + 1];
                    const float d2 = Co2 - a.target[3 * pix + 2];
                    g0[q] = d0 > 0.0f ? a.inv_count : (d0 < 0.0f ? -a.inv_count : 0.0f);
                    g1[q] = d1 > 0.0f ? a.inv_count : (d1 < 0.0f ? -a.inv_count : 0.0f);
                    g2[q] = d2 > 0.0f ? a.inv_count : (d2 < 0.0f ? -a.inv_count : 0.0f);
                    l1 += (fabsf(d0) + fabsf(d1)) + fabsf(d2);
                } else {
                    g0[q] = a.dLdC[3 * pix + 0];
                    g1[q] = a.dLdC[3 * pix + 1];
                    g2[q] = a.dLdC[3 * pix + 2];
                }
                R[q] = __builtin_fmaf(g2[q], Co2, __builtin_fmaf(g1[q], Co1, g0[q] * Co0));
            }
            mylen = max(mylen, lastp[q]);
        }
        // the reduced component this lane writes (-1: none)
        const int slot = sum9_slot(lane), pos16 = lane & 15;
        __syncthreads();
        if (threadIdx.x == 0) s_len = 0;
        if (a.loss) {
            // per-tile L1 sum, fixed-order reduction
            float sl = l1;
            for (int off = 32; off > 0; off >>= 1) sl += __shfl_xor(sl, off);
            if (lane == 0) s_loss[w] = sl;
        }
        __syncthreads();
        atomicMax(&s_len, mylen);
        if (a.loss && threadIdx.x == 0) {
            float sl = 0.0f;
            for (int i = 0; i < NW; ++i) sl += s_loss[i];
            a.loss[gt] = sl;
        }
        __syncthreads();
        const uint32_t stop = start + s_len;
        // batch size: S, or per tile the S_t minimising (batches) x (entries
        // per batch) for N listed Gaussians and P pixels (Sec. 4.2):
        // sqrt(N P) rounded up to a wavefront multiple, at most S
        uint32_t St = (uint32_t)S;
        if (a.adaptive_batch) {
            const uint64_t np = (uint64_t)(ti.range.y - ti.range.x) * (uint64_t)(TILE * TILE);
            St = kWave;
            while (St < (uint32_t)S && (uint64_t)St * St < np) St += kWave;
        }
        for (uint32_t b0 = start; b0 < stop; b0 += St) {
            __syncthreads();
            // the forward's composite mask for positions [b0, bend): only
            // entries some pixel of the tile composited are staged, in order
            const uint32_t bend = min(b0 + St, stop);
            const uint32_t w0 = b0 >> 5, nwd = ((bend - 1) >> 5) - w0 + 1;
            if (threadIdx.x < nwd) {
                const uint32_t wb = (w0 + threadIdx.x) << 5;
                uint32_t m = a.comp_mask[w0 + threadIdx.x];
                if (wb < b0) m &= ~0u << (b0 - wb);
                if (bend - wb < 32u) m &= (1u << (bend - wb)) - 1u;
                s_mw[threadIdx.x] = m;
            }
            __syncthreads();
            int cnt = 0;
            for (uint32_t q = 0; q < nwd; ++q) cnt += __popc(s_mw[q]);
            for (int i = threadIdx.x; i < (int)St; i += NT) {
                const uint32_t j = b0 + i;
                if (j < bend) {
                    const uint32_t rel = j - (w0 << 5), wq = rel >> 5, bq = rel & 31u;
                    if ((s_mw[wq] >> bq) & 1u) {
                        int slot = __popc(s_mw[wq] & ((1u << bq) - 1u));
                        for (uint32_t q = 0; q < wq; ++q) slot += __popc(s_mw[q]);
                        uint32_t gid;
                        stage_splat(a, ti.view, j, s_g[slot], s_h[slot], s_b[slot], gid);
                        s_gid[slot] = gid;
                        s_idx[slot] = unsorted_index(a, ti.view, gid, ti.tx, ti.ty);
                        s_pos[slot] = j - start;
                    }
                }
            }
            __syncthreads();
            // this wavefront's rectangle of pixel centres, and the list length
            // its pixels need (the largest of their `last`)
            uint32_t wlen = mylen;
            for (int off = 32; off > 0; off >>= 1) wlen = max(wlen, (uint32_t)__shfl_xor((int)wlen, off));
            const float rx0 = (float)(ti.tx * TILE) + 0.5f, rx1 = rx0 + (float)(TILE - 1);
            const float ry0 = (float)(ti.ty * TILE + w * Geo<TILE, PPT_>::ROWS) + 0.5f;
            const float ry1 = ry0 + (float)(Geo<TILE, PPT_>::ROWS - 1);
            for (int sub = 0; sub < cnt; sub += SUB) {
                const int scnt = min(SUB, cnt - sub);
                uint64_t used = 0;
                // staged Gaussians no pixel of this wavefront can composite (past
                // its pixels' last entries, or outside their reach) are passed
                // over: their gradient terms here would all be zero
                const uint64_t rel = __ballot(lane < scnt && s_pos[sub + lane] < wlen &&
                                              rect_may_composite(s_g[sub + lane], s_h[sub + lane], rx0, rx1, ry0,
                                                                 ry1));
                for (uint64_t mrel = rel; mrel != 0ull; mrel &= mrel - 1ull) {
                    const int kk = (int)__builtin_ctzll(mrel);
                    const int k = sub + kk;
                    const uint32_t pos = s_pos[k];
                    const float4 sg = s_g[k];
                    const float4 sh = s_h[k];
                    const float cb = s_b[k];
                    // evaluate the pixels first; a wavefront none of whose pixels
                    // composite this Gaussian skips the gradient terms entirely
                    float dxq[PPT], dyq[PPT], agq[PPT], alq[PPT];
                    bool cq[PPT];
                    bool any = false;
#pragma unroll
                    for (int q = 0; q < PPT; ++q) {
                        float G;
                        const bool in = eval_pair(px[q], py[q], sg, sh, dxq[q], dyq[q], G, agq[q]);
                        alq[q] = fminf(kAlphaMax, agq[q]);
                        cq[q] = pos < lastp[q] && in && alq[q] >= kAlphaMin;
                        any = any || cq[q];
                    }
                    if (__ballot(any) == 0ull) continue;
                    // (-0 + x is x exactly, so the first slot's terms need no add)
                    float v0 = -0.f, v1 = -0.f, v2 = -0.f, v3 = -0.f, v4 = -0.f, v5 = -0.f, v6 = -0.f,
                          v7 = -0.f, v8 = -0.f;
#pragma unroll
                    for (int q = 0; q < PPT; ++q) {
                        // pixels that do not composite this Gaussian use alpha = 0
                        // (a composited alpha is at least 1/255)
                        const float ae = cq[q] ? alq[q] : 0.0f;
                        // a pixel slot where no lane composites this Gaussian
                        // adds nothing (alpha 0: T and R unchanged)
                        if (PPT > 1 && __ballot(ae > 0.0f) == 0ull) continue;
                        const float wgt = ae * T[q];
                        v6 = __builtin_fmaf(wgt, g0[q], v6);
                        v7 = __builtin_fmaf(wgt, g1[q], v7);
                        v8 = __builtin_fmaf(wgt, g2[q], v8);
                        const float gc = __builtin_fmaf(g2[q], cb, __builtin_fmaf(g1[q], sh.w, g0[q] * sh.z));
                        R[q] = __builtin_fmaf(-wgt, gc, R[q]);
                        const float inv1m = __builtin_amdgcn_rcpf(1.0f - alq[q]);
                        const float dalpha = __builtin_fmaf(T[q], gc, -(R[q] * inv1m));
                        // no gradient through the clamp at 0.99
                        const float ag = (agq[q] > kAlphaMax) ? 0.0f : ae;
                        const float dpow = ag * dalpha;
                        const float dx = dxq[q], dy = dyq[q];
                        const float ddx = dpow * dx, ddy = dpow * dy;
                        v0 += dpow;
                        v1 += ddx;
                        v2 += ddy;
                        v3 = __builtin_fmaf(ddx, dx, v3);
                        v4 = __builtin_fmaf(ddx, dy, v4);
                        v5 = __builtin_fmaf(ddy, dy, v5);
                        T[q] = T[q] - wgt;
                    }
                    const float x = sum9(v0, v1, v2, v3, v4, v5, v6, v7, v8, pos16);
                    if (slot >= 0) s_red[w][kk][slot] = x;
                    used |= 1ull << kk;
                }
                if (lane == 0) s_mask[w] = used;
                __syncthreads();
                for (int kk = threadIdx.x; kk < scnt; kk += NT) {
                    float r0 = 0, r1 = 0, r2 = 0, r3 = 0, r4 = 0, r5 = 0, r6 = 0, r7 = 0, r8 = 0;
                    bool anyw = false;
                    for (int ww = 0; ww < NW; ++ww) {
                        if ((s_mask[ww] >> kk) & 1ull) {
                            anyw = true;
                            const float* q = s_red[ww][kk];
                            r0 += q[0]; r1 += q[1]; r2 += q[2]; r3 += q[3]; r4 += q[4];
                            r5 += q[5]; r6 += q[6]; r7 += q[7]; r8 += q[8];
                        }
                    }
                    const uint32_t idx = s_idx[sub + kk];
                    if ((int64_t)idx >= a.capacity) continue;   // only after a capacity overflow
                    atomicOr(a.rec_mask + (idx >> 5), 1u << (idx & 31u));
                    float4* rec = a.grec + 3 * (int64_t)idx;
                    const uint32_t owner = (uint32_t)((int64_t)ti.view * a.n + s_gid[sub + kk]);
                    if (anyw) {
                        // conic and opacity of this Gaussian, unscaled
                        const float4* rr = a.rec + 4 * (int64_t)owner;
                        const float4 q0 = rr[0];
                        const float4 q1 = rr[1];
                        const float A = q0.z, B = q0.w, C = q1.x, op = q1.y;
                        const float du = A * r1 + B * r2;
                        const float dv = B * r1 + C * r2;
                        rec[0] = make_float4(du, dv, -0.5f * r3, -r4);
                        rec[1] = make_float4(-0.5f * r5, r0 / op, r6, r7);
                        rec[2] = make_float4(r8, __uint_as_float(owner), 0.0f, 0.0f);
                    } else {
                        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
                        rec[0] = z; rec[1] = z; rec[2] = make_float4(0.f, __uint_as_float(owner), 0.f, 0.f);
                    }
                }
                __syncthreads();
            }
        }
        if (threadIdx.x == 0) a.tile_stop[gt] = stop;
        if (a.counter == nullptr) break;
    }
}

// ---------------------------------------------------------------------------
// backward, two-phase form (Sec. 4.2, second implementation)
// ---------------------------------------------------------------------------
// Per batch of S staged entries: a pixel-parallel pass runs through the batch
// front to back, recomputing transmittance, and stores per (entry, pixel)
// u = dL/dpower and w = alpha T in LDS (zero where the pixel does not
// composite the entry).  The Gaussian-parallel pass is then a contraction
// over the tile's pixels, on the matrix cores: with tile-local pixel
// coordinates (X, Y), each wavefront multiplies the S x 64 PPT block of u of
// its own pixels by the pixel moments [1, X, Y, X^2, XY, Y^2] and the block
// of w by the pixels' dL/dC (v_mfma_f32_16x16x4f32, four pixels per
// instruction, sixteen entries per matrix tile).  The wavefronts' partial
// moments are added in a fixed order and turned into the record's sums of u
// (1, dx, dy, dx^2, dx dy, dy^2) with dx = X - mx, mx the mean's offset from
// the tile's first pixel centre (tile-local, so the expansion adds no
// cancellation beyond that of the sums themselves).  The pair evaluation is
// the forward's (offsets from the mean), so composite decisions agree with
// it.

template <int TILE, int S, int PPT_>
__global__ __launch_bounds__(TILE * TILE / PPT_, (TILE == 16 && PPT_ == 1) ? (S == 16 ? 3 : S == 32 ? 2 : 1) : 1)
void k_raster_bwd2(RasterArgs a) {
    constexpr int PPT = PPT_, NT = Geo<TILE, PPT_>::NT;
    constexpr int NP = TILE * TILE;
    // row pitch of the per-pair arrays: NP + 4, so that the matrix-operand
    // reads (16 entries x 4 consecutive pixels) fall on distinct banks
    constexpr int UP = NP + 4;
    constexpr int NW = NT / kWave;
    constexpr int KS = kWave * PPT / 4;  // matrix K-steps (4 pixels each) per wavefront
    constexpr int MT = S / 16;           // 16-entry matrix tiles per batch
    static_assert(S % 16 == 0 && S <= kWave, "whole 16-entry matrix tiles");
    __shared__ float4 s_g[S];
    __shared__ float4 s_h[S];
    __shared__ float s_b[S];
    __shared__ uint32_t s_gid[S];
    __shared__ uint32_t s_idx[S];
    __shared__ uint32_t s_pos[S];
    __shared__ uint32_t s_mw[S / 32 + 2];
    __shared__ float s_u[S * UP];        // dL/dpower per (entry, pixel)
    __shared__ float s_w[S * UP];        // alpha T per (entry, pixel)
    __shared__ float s_gp[3][NP];        // dL/dC per pixel
    __shared__ float s_part[NW][S][9];   // per-wavefront moments
    __shared__ int s_tile;
    __shared__ uint32_t s_len;
    __shared__ float s_loss[NT / kWave];
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (;;) {
        const int gt = next_tile(a, &s_tile);
        if (gt == -1 || (gt == -2 && a.counter == nullptr)) break;
        if (gt == -2) continue;
        const TileInfo ti = tile_info(a, gt);
        const uint32_t start = ti.range.x;
        float px[PPT], py[PPT], g0[PPT], g1[PPT], g2[PPT], T[PPT], R[PPT];
        uint32_t lastp[PPT];
        float l1 = 0.0f;
        uint32_t mylen = 0;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int p = Geo<TILE, PPT_>::pixel((int)threadIdx.x, q);
            const int ix = ti.tx * TILE + p % TILE, iy = ti.ty * TILE + p / TILE;
            px[q] = (float)ix + 0.5f;
            py[q] = (float)iy + 0.5f;
            g0[q] = g1[q] = g2[q] = 0.0f;
            T[q] = 1.0f; R[q] = 0.0f;
            lastp[q] = 0;
            if (ix < ti.W && iy < ti.H) {
                const int64_t pix = ti.pix_base + (int64_t)iy * ti.W + ix;
                const float Co0 = a.out_rgb[3 * pix + 0];
                const float Co1 = a.out_rgb[3 * pix + 1];
                const float Co2 = a.out_rgb[3 * pix + 2];
                lastp[q] = a.out_last[pix];
                if (a.target) {
                    const float d0 = Co0 - a.target[3 * pix + 0];
                    const float d1 = Co1 - a.target[3 * pix + 1];
                    const float d2 = Co2 - a.target[3 * pix + 2];
                    g0[q] = d0 > 0.0f ? a.inv_count : (d0 < 0.0f ? -a.inv_count : 0.0f);
                    g1[q] = d1 > 0.0f ? a.inv_count : (d1 < 0.0f ? -a.inv_count : 0.0f);
                    g2[q] = d2 > 0.0f ? a.inv_count : (d2 < 0.0f ? -a.inv_count : 0.0f);
                    l1 += (fabsf(d0) + fabsf(d1)) + fabsf(d2);
                } else {
                    g0[q] = a.dLdC[3 * pix + 0];
                    g1[q] = a.dLdC[3 * pix + 1];
                    g2[q] = a.dLdC[3 * pix + 2];
                }
                R[q] = __builtin_fmaf(g2[q], Co2, __builtin_fmaf(g1[q], Co1, g0[q] * Co0));
            }
            mylen = max(mylen, lastp[q]);
        }
        __syncthreads();
        if (threadIdx.x == 0) s_len = 0;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const int p = Geo<TILE, PPT_>::pixel((int)threadIdx.x, q);
            s_gp[0][p] = g0[q];
            s_gp[1][p] = g1[q];
            s_gp[2][p] = g2[q];
        }
        if (a.loss) {
            float sl = l1;
            for (int off = 32; off > 0; off >>= 1) sl += __shfl_xor(sl, off);
            if (lane == 0) s_loss[w] = sl;
        }
        __syncthreads();
        atomicMax(&s_len, mylen);
        if (a.loss && threadIdx.x == 0) {
            float sl = 0.0f;
            for (int i = 0; i < NT / kWave; ++i) sl += s_loss[i];
            a.loss[gt] = sl;
        }
        // B operands of this wavefront's K-steps (lane l: pixel 4 s + l / 16 of
        // the wavefront, column l % 16): the pixel moments 1, X, Y, X^2, XY,
        // Y^2 (tile-local pixel indices) in columns 0..5, the pixel's dL/dC in
        // columns 6..8, zeros elsewhere
        float bmom[KS], bgrad[KS];
        {
            const int col = lane % 16;
#pragma unroll
            for (int st = 0; st < KS; ++st) {
                const int p = w * (kWave * PPT) + 4 * st + lane / 16;
                const float X = (float)(p % TILE), Y = (float)(p / TILE);
                bmom[st] = col == 0 ? 1.0f : col == 1 ? X : col == 2 ? Y : col == 3 ? X * X
                         : col == 4 ? X * Y : col == 5 ? Y * Y : 0.0f;
                bgrad[st] = (col >= 6 && col < 9) ? s_gp[col - 6][p] : 0.0f;
            }
        }
        __syncthreads();
        const uint32_t stop = start + s_len;
        for (uint32_t b0 = start; b0 < stop; b0 += S) {
            __syncthreads();
            // stage the entries of [b0, bend) some pixel composited, in order
            const uint32_t bend = min(b0 + (uint32_t)S, stop);
            const uint32_t w0 = b0 >> 5, nwd = ((bend - 1) >> 5) - w0 + 1;
            if (threadIdx.x < nwd) {
                const uint32_t wb = (w0 + threadIdx.x) << 5;
                uint32_t m = a.comp_mask[w0 + threadIdx.x];
                if (wb < b0) m &= ~0u << (b0 - wb);
                if (bend - wb < 32u) m &= (1u << (bend - wb)) - 1u;
                s_mw[threadIdx.x] = m;
            }
            __syncthreads();
            int cnt = 0;
            for (uint32_t q = 0; q < nwd; ++q) cnt += __popc(s_mw[q]);
            for (int i = threadIdx.x; i < S; i += NT) {
                const uint32_t j = b0 + i;
                if (j < bend) {
                    const uint32_t rel = j - (w0 << 5), wq = rel >> 5, bq = rel & 31u;
                    if ((s_mw[wq] >> bq) & 1u) {
                        int slot = __popc(s_mw[wq] & ((1u << bq) - 1u));
                        for (uint32_t q = 0; q < wq; ++q) slot += __popc(s_mw[q]);
                        uint32_t gid;
                        stage_splat(a, ti.view, j, s_g[slot], s_h[slot], s_b[slot], gid);
                        s_gid[slot] = gid;
                        s_idx[slot] = unsorted_index(a, ti.view, gid, ti.tx, ti.ty);
                        s_pos[slot] = j - start;
                    }
                }
            }
            __syncthreads();
            // pixel-parallel pass over the staged entries this wavefront's pixels
            // can composite (lane k tests entry k: within the pixels' list
            // lengths and able to reach their rectangle), in order; the other
            // staged entries get zeros at this wavefront's pixels
            uint64_t wlive;
            {
                uint32_t wlen = mylen;
                for (int off = 32; off > 0; off >>= 1) wlen = max(wlen, (uint32_t)__shfl_xor((int)wlen, off));
                const float rx0 = (float)(ti.tx * TILE) + 0.5f, rx1 = rx0 + (float)(TILE - 1);
                const float ry0 = (float)(ti.ty * TILE + w * Geo<TILE, PPT_>::ROWS) + 0.5f;
                const float ry1 = ry0 + (float)(Geo<TILE, PPT_>::ROWS - 1);
                const uint64_t rel = __ballot(lane < cnt && s_pos[lane] < wlen &&
                                              rect_may_composite(s_g[lane], s_h[lane], rx0, rx1, ry0, ry1));
                const uint64_t staged = cnt >= kWave ? ~0ull : ((1ull << cnt) - 1ull);
                // 16-entry matrix tiles with no entry this wavefront composites
                // are skipped by the matrix pass; the others need zeros in the
                // columns of their other entries
                uint64_t live = 0ull;
#pragma unroll
                for (int t = 0; t < MT; ++t)
                    if ((rel >> (16 * t)) & 0xffffull) live |= 0xffffull << (16 * t);
                wlive = live;
                for (uint64_t m = staged & ~rel & live; m != 0ull; m &= m - 1ull) {
                    const int k = (int)__builtin_ctzll(m);
#pragma unroll
                    for (int qq = 0; qq < PPT; ++qq) {
                        const int p = Geo<TILE, PPT_>::pixel((int)threadIdx.x, qq);
                        s_u[k * UP + p] = 0.0f;
                        s_w[k * UP + p] = 0.0f;
                    }
                }
                for (uint64_t m = rel; m != 0ull; m &= m - 1ull) {
                    const int k = (int)__builtin_ctzll(m);
                    const uint32_t pos = s_pos[k];
                    const float4 sg = s_g[k];
                    const float4 sh = s_h[k];
                    const float cb = s_b[k];
#pragma unroll
                    for (int qq = 0; qq < PPT; ++qq) {
                        float dx, dy, G, ag;
                        const bool in = eval_pair(px[qq], py[qq], sg, sh, dx, dy, G, ag);
                        const float al = fminf(kAlphaMax, ag);
                        const bool c = pos < lastp[qq] && in && al >= kAlphaMin;
                        const float ae = c ? al : 0.0f;
                        const float wgt = ae * T[qq];
                        const float gc = __builtin_fmaf(g2[qq], cb, __builtin_fmaf(g1[qq], sh.w, g0[qq] * sh.z));
                        R[qq] = __builtin_fmaf(-wgt, gc, R[qq]);
                        const float inv1m = __builtin_amdgcn_rcpf(1.0f - al);
                        const float dalpha = __builtin_fmaf(T[qq], gc, -(R[qq] * inv1m));
                        const float agc = (ag > kAlphaMax) ? 0.0f : ae;
                        const int p = Geo<TILE, PPT_>::pixel((int)threadIdx.x, qq);
                        s_u[k * UP + p] = agc * dalpha;
                        s_w[k * UP + p] = wgt;
                        T[qq] = T[qq] - wgt;
                    }
                }
            }
            // the matrix pass reads only this wavefront's pixel columns, which
            // this wavefront has just written (LDS operations of one wavefront
            // complete in order): no workgroup barrier
            __builtin_amdgcn_wave_barrier();
            // Gaussian-parallel pass on the matrix cores: this wavefront's
            // pixels [w 64 PPT, (w + 1) 64 PPT), four per K-step (lane l:
            // pixel 4 s + l / 16, entry l % 16 of the matrix tile, output
            // column l % 16); D rows 4 (l / 16) + v, column l % 16
            {
                floatx4 du[MT], dw[MT];
#pragma unroll
                for (int t = 0; t < MT; ++t) {
                    du[t] = floatx4{0.f, 0.f, 0.f, 0.f};
                    dw[t] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
#pragma unroll
                for (int t = 0; t < MT; ++t) {
                    if (((wlive >> (16 * t)) & 1ull) == 0ull) continue;
                    const int e = 16 * t + lane % 16;
#pragma unroll
                    for (int st = 0; st < KS; ++st) {
                        const int p = w * (kWave * PPT) + 4 * st + lane / 16;
                        du[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(s_u[e * UP + p], bmom[st], du[t], 0, 0, 0);
                        dw[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(s_w[e * UP + p], bgrad[st], dw[t], 0, 0, 0);
                    }
                }
                const int col = lane % 16;
#pragma unroll
                for (int t = 0; t < MT; ++t) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int e = 16 * t + 4 * (lane / 16) + v;
                        if (col < 6) s_part[w][e][col] = du[t][v];
                        else if (col < 9) s_part[w][e][col] = dw[t][v];
                    }
                }
            }
            __syncthreads();
            for (int k = threadIdx.x; k < cnt; k += NT) {
                float r[9];
#pragma unroll
                for (int c = 0; c < 9; ++c) r[c] = 0.0f;
                for (int ww = 0; ww < NW; ++ww)
#pragma unroll
                    for (int c = 0; c < 9; ++c) r[c] += s_part[ww][k][c];
                const uint32_t idx = s_idx[k];
                if ((int64_t)idx >= a.capacity) continue;   // only after a capacity overflow
                atomicOr(a.rec_mask + (idx >> 5), 1u << (idx & 31u));
                float4* rec = a.grec + 3 * (int64_t)idx;
                const uint32_t owner = (uint32_t)((int64_t)ti.view * a.n + s_gid[k]);
                const float4* rr = a.rec + 4 * (int64_t)owner;
                const float4 q0 = rr[0];
                const float4 q1 = rr[1];
                const float A = q0.z, B = q0.w, C = q1.x, op = q1.y;
                // moments of u over (1, X, Y, X^2, XY, Y^2) -> sums over (1, dx,
                // dy, dx^2, dx dy, dy^2), dx = X - mx, dy = Y - my
                const float mx = q0.x - ((float)(ti.tx * TILE) + 0.5f);
                const float my = q0.y - ((float)(ti.ty * TILE) + 0.5f);
                const float s0 = r[0];
                const float s1 = r[1] - mx * r[0];
                const float s2 = r[2] - my * r[0];
                const float s3 = r[3] - mx * (2.0f * r[1] - mx * r[0]);
                const float s4 = r[4] - mx * r[2] - my * r[1] + (mx * my) * r[0];
                const float s5 = r[5] - my * (2.0f * r[2] - my * r[0]);
                rec[0] = make_float4(A * s1 + B * s2, B * s1 + C * s2, -0.5f * s3, -s4);
                rec[1] = make_float4(-0.5f * s5, s0 / op, r[6], r[7]);
                rec[2] = make_float4(r[8], __uint_as_float(owner), 0.0f, 0.0f);
            }
        }
        if (threadIdx.x == 0) a.tile_stop[gt] = stop;
        if (a.counter == nullptr) break;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <int TILE, int S, int PPT>
static void launch_fwd_t(const RasterArgs& a, unsigned grid, hipStream_t s) {
    constexpr int NT = Geo<TILE, PPT>::NT;
    if (a.tile_stats)
        hipLaunchKernelGGL((k_raster_fwd<TILE, S, PPT, true>), dim3(grid), dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL((k_raster_fwd<TILE, S, PPT, false>), dim3(grid), dim3(NT), 0, s, a);
}
template <int TILE, int S, int PPT>
static void launch_bwd_t(const RasterArgs& a, unsigned grid, hipStream_t s) {
    hipLaunchKernelGGL((k_raster_bwd<TILE, S, PPT>), dim3(grid), dim3(Geo<TILE, PPT>::NT), 0, s, a);
}

template <bool FWD, int TILE, int PPT>
static int dispatch_s(const RasterArgs& a, int S, unsigned grid, hipStream_t s) {
    switch (S) {
        case 32: FWD ? launch_fwd_t<TILE, 32, PPT>(a, grid, s) : launch_bwd_t<TILE, 32, PPT>(a, grid, s); break;
        case 64: FWD ? launch_fwd_t<TILE, 64, PPT>(a, grid, s) : launch_bwd_t<TILE, 64, PPT>(a, grid, s); break;
        case 128: FWD ? launch_fwd_t<TILE, 128, PPT>(a, grid, s) : launch_bwd_t<TILE, 128, PPT>(a, grid, s); break;
        case 256: FWD ? launch_fwd_t<TILE, 256, PPT>(a, grid, s) : launch_bwd_t<TILE, 256, PPT>(a, grid, s); break;
        default: set_error("lds_batch must be 32, 64, 128 or 256 (got %d)", S); return GS_ERR_INVALID_ARG;
    }
    return check_launch(FWD ? "rasterize_fwd" : "rasterize_bwd");
}

template <bool FWD>
static int dispatch(const RasterArgs& a, int S, unsigned grid, hipStream_t s) {
    const int ppt = a.L.pixels_per_lane;
    switch (a.L.tile) {
        case 8: return dispatch_s<FWD, 8, 1>(a, S, grid, s);
        case 16:
            return ppt == 1 ? dispatch_s<FWD, 16, 1>(a, S, grid, s)
                 : ppt == 2 ? dispatch_s<FWD, 16, 2>(a, S, grid, s)
                            : dispatch_s<FWD, 16, 4>(a, S, grid, s);
        case 32:
            return ppt == 1 ? dispatch_s<FWD, 32, 1>(a, S, grid, s)
                 : ppt == 2 ? dispatch_s<FWD, 32, 2>(a, S, grid, s)
                            : dispatch_s<FWD, 32, 4>(a, S, grid, s);
        default: set_error("tile must be 8, 16 or 32"); return GS_ERR_INVALID_ARG;
    }
}

static RasterArgs base_args(const gs_splats& sp, int64_t n, const gs_layout& L, const gs_bins& b,
                            const gs_view* views, const gs_schedule* sched) {
    RasterArgs a;
    memset(&a, 0, sizeof(a));
    a.L = L;
    a.rec = reinterpret_cast<const float4*>(sp.rec);
    a.vals = b.vals;
    a.ranges = reinterpret_cast<const uint2*>(b.ranges);
    a.views = views;
    a.n = n;
    a.total_tiles = L.tile_base[L.n_views];
    a.capacity = b.capacity;
    if (sched) {
        a.order = sched->order;
        a.counter = sched->counter;
    }
    return a;
}

static unsigned grid_for(const RasterArgs& a, const gs_schedule* sched) {
    if (sched && sched->counter) return (unsigned)std::max(1, std::min(sched->n_groups, a.total_tiles));
    if (sched && sched->order) return (unsigned)a.total_tiles;
    const unsigned round = kXcds * kXcdChunk;
    return ((unsigned)a.total_tiles + round - 1) / round * round;
}

int launch_raster_fwd(const gs_splats& sp, int64_t n, const gs_layout& L, const gs_bins& b,
                      const gs_view* views, const gs_image& out, int lds_batch,
                      const gs_schedule* sched, hipStream_t s) {
    RasterArgs a = base_args(sp, n, L, b, views, sched);
    a.out_rgb = out.rgb;
    a.out_T = out.T;
    a.out_last = out.last;
    a.tile_stats = out.tile_stats;
    a.comp_mask = out.comp_mask;
    if (a.total_tiles == 0) return GS_OK;
    int rc = launch_fill_u32(a.comp_mask, 0u, (b.capacity + 31) / 32, s);
    if (rc != GS_OK) return rc;
    if (a.counter) {
        rc = launch_fill_u32(a.counter, 0u, 1, s);
        if (rc != GS_OK) return rc;
    }
    return dispatch<true>(a, lds_batch, grid_for(a, sched), s);
}

static int bwd_args(const gs_splats& sp, int64_t n, const gs_layout& L, const gs_bins& b,
                    const gs_view* views, const gs_image& fwd, const float* target, const float* dLdC,
                    const gs_grads2d& grads, float* loss, const gs_schedule* sched, hipStream_t s,
                    RasterArgs* out) {
    RasterArgs a = base_args(sp, n, L, b, views, sched);
    a.out_rgb = fwd.rgb;
    a.out_T = fwd.T;
    a.out_last = fwd.last;
    a.target = target;
    a.dLdC = dLdC;
    a.loss = target ? loss : nullptr;
    a.inv_count = 1.0f / (3.0f * (float)L.pixel_base[L.n_views]);
    a.grec = reinterpret_cast<float4*>(grads.rec);
    a.tile_stop = grads.tile_stop;
    a.comp_mask = fwd.comp_mask;
    a.rec_mask = grads.rec_mask;
    a.row_offsets = b.row_offsets;
    a.rows = reinterpret_cast<const uint4*>(b.rows);
    a.row_capacity = b.row_capacity;
    *out = a;
    if (a.total_tiles == 0) return GS_OK;
    int rc = launch_fill_u32(a.rec_mask, 0u, (b.capacity + 31) / 32, s);
    if (rc != GS_OK) return rc;
    if (a.counter) rc = launch_fill_u32(a.counter, 0u, 1, s);
    return rc;
}

int launch_raster_bwd(const gs_splats& sp, int64_t n, const gs_layout& L, const gs_bins& b,
                      const gs_view* views, const gs_image& fwd, const float* target,
                      const float* dLdC, const gs_grads2d& grads, float* loss, int lds_batch,
                      const gs_schedule* sched, hipStream_t s) {
    // a negative batch selects the per-tile batch with cap -lds_batch
    if (lds_batch < 0 && -lds_batch < kWave) {
        set_error("an adaptive lds_batch needs a cap of at least 64 (got %d)", -lds_batch);
        return GS_ERR_INVALID_ARG;
    }
    RasterArgs a;
    int rc = bwd_args(sp, n, L, b, views, fwd, target, dLdC, grads, loss, sched, s, &a);
    if (rc != GS_OK || a.total_tiles == 0) return rc;
    a.adaptive_batch = lds_batch < 0;
    return dispatch<false>(a, lds_batch < 0 ? -lds_batch : lds_batch, grid_for(a, sched), s);
}

template <int TILE, int S, int PPT>
static int launch_bwd2_t(const RasterArgs& a, unsigned grid, hipStream_t s) {
    hipLaunchKernelGGL((k_raster_bwd2<TILE, S, PPT>), dim3(grid), dim3(Geo<TILE, PPT>::NT), 0, s, a);
    return check_launch("raster_bwd2");
}

template <int TILE, int PPT>
static int launch_bwd2_s(const RasterArgs& a, int S, unsigned grid, hipStream_t s) {
    return S == 16 ? launch_bwd2_t<TILE, 16, PPT>(a, grid, s)
         : S == 32 ? launch_bwd2_t<TILE, 32, PPT>(a, grid, s)
                   : launch_bwd2_t<TILE, 64, PPT>(a, grid, s);
}

int launch_raster_bwd2(const gs_splats& sp, int64_t n, const gs_layout& L, const gs_bins& b,
                       const gs_view* views, const gs_image& fwd, const float* target,
                       const float* dLdC, const gs_grads2d& grads, float* loss, int lds_batch,
                       const gs_schedule* sched, hipStream_t s) {
    if (lds_batch != 16 && lds_batch != 32 && lds_batch != 64) {
        set_error("the two-phase backward's lds_batch must be 16, 32 or 64 (got %d)", lds_batch);
        return GS_ERR_INVALID_ARG;
    }
    if (L.tile != 8 && L.tile != 16) {
        set_error("the two-phase backward supports 8x8 and 16x16 tiles (got %d)", L.tile);
        return GS_ERR_INVALID_ARG;
    }
    RasterArgs a;
    int rc = bwd_args(sp, n, L, b, views, fwd, target, dLdC, grads, loss, sched, s, &a);
    if (rc != GS_OK || a.total_tiles == 0) return rc;
    // one pixel per lane whatever the layout asks of the first backward
    // (pixels are addressed by their tile-local index, so the mapping need
    // not be the forward's): with two, the per-pair arrays and the operands
    // of twice the matrix steps leave one wavefront per SIMD, which measured
    // slower at every batch size
    const unsigned grid = grid_for(a, sched);
    if (L.tile == 8) return launch_bwd2_s<8, 1>(a, lds_batch, grid, s);
    return launch_bwd2_s<16, 1>(a, lds_batch, grid, s);
}

}  // namespace gs
