// Projection forward: one thread per Gaussian, looping over the views so the
// 240-byte parameter record is read from HBM once per call.  Loads are float4
// planes (plane-major SoA), so each wavefront reads 1 KiB contiguous per plane.
// Each output entry is one 64-byte record (one cache line), so the tile
// rasteriser gathers everything it needs about a Gaussian with one line fetch.
#include "project_math.h"

namespace gs {

struct ViewGrid {
    int32_t gx[GS_MAX_VIEWS], gy[GS_MAX_VIEWS];
};

__global__ __launch_bounds__(256) void k_project(const float* __restrict__ params, int64_t n,
                                                 const gs_view* __restrict__ views, int n_views,
                                                 int tile, int cull, ViewGrid grid, gs_splats out) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const float4 p0 = ld4(params, 0 * n + g);
    const float4 p1 = ld4(params, 1 * n + g);
    const float4 p2 = ld4(params, 2 * n + g);
    float4 sh[12];
    bool finite = finite4(p0) && finite4(make_float4(p1.x, p1.y, p1.z, 0.0f)) && finite4(p2);
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        sh[q] = ld4(params, (3 + q) * n + g);
        finite = finite && finite4(sh[q]);
    }
    for (int v = 0; v < n_views; ++v) {
        const gs_view vw = views[v];
        Proj P;
        P.valid = false;
        if (finite) project_gaussian<true>(p0, p1, p2, sh, vw, tile, grid.gx[v], grid.gy[v], cull, P);
        const int64_t o = (int64_t)v * n + g;
        float4* rec = reinterpret_cast<float4*>(out.rec) + 4 * o;
        if (P.valid) {
            rec[0] = make_float4(P.u, P.v, P.A, P.B);
            rec[1] = make_float4(P.C, P.o, P.col[0], P.col[1]);
            rec[2] = make_float4(P.col[2], P.z, P.radius, 0.0f);
            // depth map z -> (2z + 1) / (z + 1) in (1, 2): only mantissa bits vary
            const float f = (2.0f * P.z + 1.0f) / (P.z + 1.0f);
            const uint32_t dcode = __float_as_uint(f) & 0x7FFFFFu;
            rec[3] = make_float4(__uint_as_float((uint32_t)P.x0 | ((uint32_t)P.y0 << 16)),
                                 __uint_as_float((uint32_t)P.x1 | ((uint32_t)P.y1 << 16)),
                                 __uint_as_float(dcode), 0.0f);
            out.tiles[o] = P.count;
        } else {
            const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
            rec[0] = z; rec[1] = z; rec[2] = z; rec[3] = z;
            out.tiles[o] = 0u;
        }
    }
}

int launch_project(const float* params, int64_t n, const gs_view* views, const gs_layout& L,
                   const gs_splats& out, hipStream_t s) {
    if (n == 0) return GS_OK;
    ViewGrid grid;
    for (int v = 0; v < GS_MAX_VIEWS; ++v) {
        grid.gx[v] = v < L.n_views ? L.tiles_x[v] : 0;
        grid.gy[v] = v < L.n_views ? L.tiles_y[v] : 0;
    }
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_project, dim3((unsigned)blocks), dim3(256), 0, s, params, n, views,
                       L.n_views, L.tile, L.cull, grid, out);
    return check_launch("project");
}

}  // namespace gs
