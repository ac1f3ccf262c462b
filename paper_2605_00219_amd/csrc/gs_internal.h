// Internal declarations shared by the HIP translation units of libgs.
// Everything here is gfx950 (CDNA4, wave64) device code or host launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>

#include "gs.h"

#define GS_DEV __device__ __forceinline__

namespace gs {

constexpr int kWave = 64;

// ---- error reporting ------------------------------------------------------
void set_error(const char* fmt, ...);
int check_launch(const char* what);

// ---- layout helpers (device) ----------------------------------------------
GS_DEV int view_of_tile(const gs_layout& L, int gt) {
    int v = 0;
#pragma unroll 1
    for (int i = 1; i < L.n_views; ++i)
        if (gt >= L.tile_base[i]) v = i;
    return v;
}

GS_DEV float4 ld4(const float* p, int64_t i) { return reinterpret_cast<const float4*>(p)[i]; }
GS_DEV void st4(float* p, int64_t i, float4 v) { reinterpret_cast<float4*>(p)[i] = v; }

// ---- launchers (host) ---------------------------------------------------------
int launch_project(const float* params, int64_t n, const gs_view* views, const gs_layout& L,
                   const gs_splats& out, hipStream_t s);
int launch_bin_sort(const gs_splats& sp, int64_t n, const gs_layout& L, const gs_bins& b,
                    void* ws, size_t ws_bytes, const gs_side_stream* side, hipStream_t s);
size_t bin_sort_workspace(int64_t n, const gs_layout& L, int64_t capacity);
size_t gather_workspace(int64_t capacity);
int launch_raster_fwd(const gs_splats& sp, int64_t n, const gs_layout& L, const gs_bins& b,
                      const gs_view* views, const gs_image& out, int lds_batch,
                      const gs_schedule* sched, hipStream_t s);
int launch_raster_bwd(const gs_splats& sp, int64_t n, const gs_layout& L, const gs_bins& b,
                      const gs_view* views, const gs_image& fwd, const float* target,
                      const float* dLdC, const gs_grads2d& grads, float* loss, int lds_batch,
                      const gs_schedule* sched, hipStream_t s);
int launch_raster_bwd2(const gs_splats& sp, int64_t n, const gs_layout& L, const gs_bins& b,
                       const gs_view* views, const gs_image& fwd, const float* target,
                       const float* dLdC, const gs_grads2d& grads, float* loss, int lds_batch,
                       const gs_schedule* sched, hipStream_t s);
int launch_project_bwd_adam(float* params, int64_t n, const gs_view* views, const gs_layout& L,
                            const gs_splats& splats, const gs_bins& b, const gs_grads2d& grads,
                            const gs_adam* adam, float* grads_out, hipStream_t s);
int launch_project_bwd_adam_noalloc(float* params, int64_t n, const gs_view* views, const gs_layout& L,
                                    const gs_splats& splats, const gs_bins& b, const gs_grads2d& grads,
                                    const gs_adam* adam, float* grads_out, hipStream_t s);
int launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s);
int launch_tile_features(const gs_splats& sp, int64_t n, const gs_layout& L, const gs_bins& b,
                         float* features, hipStream_t s);
int launch_mlp_forward(const float* w, const float* norm, const float* x, int64_t rows, float* out,
                       hipStream_t s);
int launch_mlp_train_step(float* w, const float* norm, const float* x, const float* y,
                          int64_t rows, float* grad, float* m, float* v, int32_t* step, float lr,
                          float* loss_out, hipStream_t s);
int launch_order_by_cost(const float* pred, int32_t total, uint32_t* order, void* scratch,
                         hipStream_t s);
int64_t loss_blocks(const gs_layout& L);
size_t loss_workspace(const gs_layout& L);
int launch_loss_l1_ssim(const float* rgb, const uint8_t* target, const gs_layout& L, float lam, int use_mask,
                        float* dLdC, float* loss_blocks_out, void* ws, hipStream_t s);
// stable ascending sort of (key, value) pairs in place; scratch of sort_pairs_scratch(count) bytes
size_t sort_pairs_scratch(int64_t count);
int sort_pairs(uint32_t* keys, uint32_t* vals, int64_t count, void* scratch, hipStream_t s);

}  // namespace gs
