// C ABI entry points: argument validation, error strings, launches.
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>

#include "gs_internal.h"

namespace gs {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: %s", what, hipGetErrorString(e));
        return GS_ERR_HIP;
    }
    return GS_OK;
}

static bool layout_ok(const gs_layout* L) {
    if (!L || L->n_views < 1 || L->n_views > GS_MAX_VIEWS) return false;
    if (L->tile != 8 && L->tile != 16 && L->tile != 32) return false;
    if (L->tile == 8 && L->pixels_per_lane != 1) return false;
    if (L->tile != 8 && L->pixels_per_lane != 1 && L->pixels_per_lane != 2 && L->pixels_per_lane != 4)
        return false;
    if (L->cull != GS_CULL_RECT && L->cull != GS_CULL_ELLIPSE) return false;
    return true;
}

}  // namespace gs

using namespace gs;

#define REQUIRE(cond, ...)                 \
    do {                                   \
        if (!(cond)) {                     \
            set_error(__VA_ARGS__);        \
            return GS_ERR_INVALID_ARG;     \
        }                                  \
    } while (0)

extern "C" {

int gs_version(void) { return GS_VERSION; }

const char* gs_last_error(void) { return g_err; }

int gs_layout_init(const int32_t* widths, const int32_t* heights, int n_views, int tile,
                   gs_layout* out) {
    REQUIRE(out && widths && heights, "gs_layout_init: null pointer");
    REQUIRE(n_views >= 1 && n_views <= GS_MAX_VIEWS, "gs_layout_init: n_views %d not in [1, %d]",
            n_views, GS_MAX_VIEWS);
    REQUIRE(tile == 8 || tile == 16 || tile == 32, "gs_layout_init: tile %d not in {8, 16, 32}", tile);
    gs_layout L;
    memset(&L, 0, sizeof(L));
    L.n_views = n_views;
    L.tile = tile;
    L.pixels_per_lane = tile == 8 ? 1 : 2;
    L.cull = GS_CULL_RECT;
    int64_t tb = 0, pb = 0;
    for (int v = 0; v < n_views; ++v) {
        REQUIRE(widths[v] >= 1 && heights[v] >= 1 && widths[v] <= (1 << 20) && heights[v] <= (1 << 20),
                "gs_layout_init: view %d has invalid size %dx%d", v, widths[v], heights[v]);
        const int gx = (widths[v] + tile - 1) / tile, gy = (heights[v] + tile - 1) / tile;
        REQUIRE(gx < 65536 && gy < 65536, "gs_layout_init: view %d has too many tiles", v);
        const int64_t nt = (int64_t)gx * gy;
        int B = 1;
        while ((int64_t(1) << B) < nt) ++B;
        REQUIRE(B <= 31, "gs_layout_init: view %d needs %d tile bits", v, B);
        L.width[v] = widths[v];
        L.height[v] = heights[v];
        L.tiles_x[v] = gx;
        L.tiles_y[v] = gy;
        L.depth_bits[v] = std::min(23, 32 - B);
        L.tile_base[v] = (int32_t)tb;
        L.pixel_base[v] = pb;
        tb += nt;
        pb += (int64_t)widths[v] * heights[v];
        REQUIRE(tb < (int64_t(1) << 31), "gs_layout_init: more than 2^31 tiles");
    }
    for (int v = n_views; v <= GS_MAX_VIEWS; ++v) {
        L.tile_base[v] = (int32_t)tb;
        L.pixel_base[v] = pb;
    }
    *out = L;
    return GS_OK;
}

size_t gs_bin_sort_workspace_size(int64_t n, const gs_layout* layout, int64_t capacity) {
    if (!layout_ok(layout) || n < 0 || capacity < 0) return 0;
    return bin_sort_workspace(n, *layout, capacity);
}

size_t gs_grads2d_workspace_size(int64_t capacity) {
    if (capacity < 0) return 0;
    return gather_workspace(capacity);
}

int gs_project(const float* params, int64_t n, const gs_view* views, const gs_layout* layout,
               const gs_splats* out, void* stream) {
    REQUIRE(layout_ok(layout), "gs_project: invalid layout");
    REQUIRE(n >= 0 && n < (int64_t(1) << 32), "gs_project: n = %lld out of range", (long long)n);
    REQUIRE(out && views && (n == 0 || params), "gs_project: null pointer");
    REQUIRE(n == 0 || (out->rec && out->tiles), "gs_project: null output buffer");
    return launch_project(params, n, views, *layout, *out, (hipStream_t)stream);
}

int gs_bin_sort(const gs_splats* splats, int64_t n, const gs_layout* layout, const gs_bins* bins,
                void* workspace, size_t workspace_bytes, const gs_side_stream* side, void* stream) {
    REQUIRE(layout_ok(layout), "gs_bin_sort: invalid layout");
    REQUIRE(!side || (side->stream && side->fork && side->join), "gs_bin_sort: incomplete side stream");
    REQUIRE(splats && bins, "gs_bin_sort: null pointer");
    REQUIRE(n >= 0 && (int64_t)layout->n_views * n < (int64_t(1) << 32), "gs_bin_sort: n out of range");
    REQUIRE(bins->capacity >= 0 && bins->capacity < (int64_t(1) << 32) - 1,
            "gs_bin_sort: capacity out of range");
    REQUIRE(bins->offsets && bins->row_offsets && bins->ranges && bins->status &&
            (bins->capacity == 0 || (bins->keys && bins->vals)), "gs_bin_sort: null bins buffer");
    REQUIRE(bins->row_capacity >= 0 && bins->row_capacity < (int64_t(1) << 32) - 1 &&
            (bins->row_capacity == 0 || bins->rows), "gs_bin_sort: bad row buffer");
    REQUIRE(workspace || workspace_bytes == 0, "gs_bin_sort: null workspace");
    return launch_bin_sort(*splats, n, *layout, *bins, workspace, workspace_bytes, side, (hipStream_t)stream);
}

static int check_sched(const gs_schedule* sched) {
    if (!sched) return GS_OK;
    REQUIRE(sched->counter == nullptr || sched->n_groups >= 1, "schedule: n_groups must be >= 1");
    return GS_OK;
}

int gs_rasterize_fwd(const gs_splats* splats, int64_t n, const gs_layout* layout,
                     const gs_bins* bins, const gs_view* views, const gs_image* out, int lds_batch,
                     const gs_schedule* sched, void* stream) {
    REQUIRE(layout_ok(layout), "gs_rasterize_fwd: invalid layout");
    REQUIRE(splats && bins && views && out && out->rgb && out->T && out->last &&
            (out->comp_mask || bins->capacity == 0), "gs_rasterize_fwd: null pointer");
    REQUIRE(lds_batch == 32 || lds_batch == 64 || lds_batch == 128 || lds_batch == 256,
            "gs_rasterize_fwd: lds_batch %d not in {32, 64, 128, 256}", lds_batch);
    int rc = check_sched(sched);
    if (rc != GS_OK) return rc;
    return launch_raster_fwd(*splats, n, *layout, *bins, views, *out, lds_batch, sched,
                             (hipStream_t)stream);
}

int gs_rasterize_bwd(const gs_splats* splats, int64_t n, const gs_layout* layout,
                     const gs_bins* bins, const gs_view* views, const gs_image* fwd,
                     const float* target, const float* dL_dC, const gs_grads2d* grads,
                     float* loss, int lds_batch, const gs_schedule* sched, void* stream) {
    REQUIRE(layout_ok(layout), "gs_rasterize_bwd: invalid layout");
    REQUIRE(splats && bins && views && fwd && fwd->rgb && fwd->last &&
            (fwd->comp_mask || bins->capacity == 0), "gs_rasterize_bwd: null pointer");
    REQUIRE((target != nullptr) != (dL_dC != nullptr),
            "gs_rasterize_bwd: give exactly one of target (fused L1) and dL_dC");
    REQUIRE(grads && grads->tile_stop && ((grads->rec && grads->rec_mask) || bins->capacity == 0),
            "gs_rasterize_bwd: null gradient buffers");
    REQUIRE(lds_batch == 32 || lds_batch == 64 || lds_batch == 128 || lds_batch == 256 || lds_batch == -64 ||
                lds_batch == -128 || lds_batch == -256,
            "gs_rasterize_bwd: lds_batch %d not in {32, 64, 128, 256, -64, -128, -256}", lds_batch);
    int rc = check_sched(sched);
    if (rc != GS_OK) return rc;
    return launch_raster_bwd(*splats, n, *layout, *bins, views, *fwd, target, dL_dC, *grads, loss,
                             lds_batch, sched, (hipStream_t)stream);
}

int gs_rasterize_bwd_twophase(const gs_splats* splats, int64_t n, const gs_layout* layout,
                              const gs_bins* bins, const gs_view* views, const gs_image* fwd,
                              const float* target, const float* dL_dC, const gs_grads2d* grads,
                              float* loss, int lds_batch, const gs_schedule* sched, void* stream) {
    REQUIRE(layout_ok(layout), "gs_rasterize_bwd_twophase: invalid layout");
    REQUIRE(splats && bins && views && fwd && fwd->rgb && fwd->last &&
            (fwd->comp_mask || bins->capacity == 0), "gs_rasterize_bwd_twophase: null pointer");
    REQUIRE((target != nullptr) != (dL_dC != nullptr),
            "gs_rasterize_bwd_twophase: give exactly one of target (fused L1) and dL_dC");
    REQUIRE(grads && grads->tile_stop && ((grads->rec && grads->rec_mask) || bins->capacity == 0),
            "gs_rasterize_bwd_twophase: null gradient buffers");
    REQUIRE(lds_batch == 16 || lds_batch == 32 || lds_batch == 64,
            "gs_rasterize_bwd_twophase: lds_batch %d not in {16, 32, 64}",
            lds_batch);
    REQUIRE(layout->tile == 8 || layout->tile == 16, "gs_rasterize_bwd_twophase: tile %d not in {8, 16}",
            layout->tile);
    int rc = check_sched(sched);
    if (rc != GS_OK) return rc;
    return launch_raster_bwd2(*splats, n, *layout, *bins, views, *fwd, target, dL_dC, *grads, loss,
                              lds_batch, sched, (hipStream_t)stream);
}

int gs_project_bwd_adam(float* params, int64_t n, const gs_view* views, const gs_layout* layout,
                        const gs_splats* splats, const gs_bins* bins, const gs_grads2d* grads,
                        const gs_adam* adam, float* grads_out, void* stream) {
    REQUIRE(layout_ok(layout), "gs_project_bwd_adam: invalid layout");
    REQUIRE(views && bins && bins->offsets && (n == 0 || params), "gs_project_bwd_adam: null pointer");
    REQUIRE(adam || grads_out, "gs_project_bwd_adam: need adam state or grads_out");
    REQUIRE(!adam || (adam->m && adam->v && adam->step && adam->scratch),
            "gs_project_bwd_adam: incomplete adam state");
    REQUIRE(splats && (n == 0 || splats->rec), "gs_project_bwd_adam: null splat records");
    REQUIRE(grads && (grads->sums || n == 0) &&
            ((grads->rec && grads->rec_mask) || bins->capacity == 0),
            "gs_project_bwd_adam: null gradient buffers");
    return launch_project_bwd_adam(params, n, views, *layout, *splats, *bins, *grads, adam, grads_out,
                                   (hipStream_t)stream);
}

int gs_project_bwd_adam_noalloc(float* params, int64_t n, const gs_view* views, const gs_layout* layout,
                                const gs_splats* splats, const gs_bins* bins, const gs_grads2d* grads,
                                const gs_adam* adam, float* grads_out, void* stream) {
    REQUIRE(layout_ok(layout), "gs_project_bwd_adam_noalloc: invalid layout");
    REQUIRE(views && bins && bins->offsets && (n == 0 || params), "gs_project_bwd_adam_noalloc: null pointer");
    REQUIRE(adam || grads_out, "gs_project_bwd_adam_noalloc: need adam state or grads_out");
    REQUIRE(!adam || (adam->m && adam->v && adam->step && adam->scratch),
            "gs_project_bwd_adam_noalloc: incomplete adam state");
    REQUIRE(splats && (n == 0 || splats->rec), "gs_project_bwd_adam_noalloc: null splat records");
    REQUIRE(grads && (grads->sums || n == 0) && ((grads->rec && grads->rec_mask) || bins->capacity == 0),
            "gs_project_bwd_adam_noalloc: null gradient buffers");
    if (n == 0) return GS_OK;
    return launch_project_bwd_adam_noalloc(params, n, views, *layout, *splats, *bins, *grads, adam, grads_out,
                                           (hipStream_t)stream);
}

int64_t gs_loss_blocks(const gs_layout* layout) {
    if (!layout_ok(layout)) return 0;
    return loss_blocks(*layout);
}

size_t gs_loss_workspace_size(const gs_layout* layout) {
    if (!layout_ok(layout)) return 0;
    return loss_workspace(*layout);
}

int gs_loss_l1_ssim(const float* rgb, const uint8_t* target, const gs_layout* layout, float lambda,
                    int use_mask, float* dL_dC, float* loss_blocks_out, void* workspace,
                    size_t workspace_bytes, void* stream) {
    REQUIRE(layout_ok(layout), "gs_loss_l1_ssim: invalid layout");
    REQUIRE(rgb && target && dL_dC && workspace, "gs_loss_l1_ssim: null pointer");
    REQUIRE(((uintptr_t)target & 3u) == 0, "gs_loss_l1_ssim: target not 4-byte aligned");
    REQUIRE(((uintptr_t)workspace & 15u) == 0, "gs_loss_l1_ssim: workspace not 16-byte aligned");
    REQUIRE(gs_loss_workspace_size(layout) > 0, "gs_loss_l1_ssim: views too large for 32-bit pixel indices");
    REQUIRE(lambda >= 0.0f && lambda <= 1.0f, "gs_loss_l1_ssim: lambda %g not in [0, 1]", (double)lambda);
    REQUIRE(workspace_bytes >= gs_loss_workspace_size(layout), "gs_loss_l1_ssim: workspace of %zu bytes, %zu needed",
            workspace_bytes, gs_loss_workspace_size(layout));
    return launch_loss_l1_ssim(rgb, target, *layout, lambda, use_mask, dL_dC, loss_blocks_out, workspace,
                               (hipStream_t)stream);
}

int gs_tile_features(const gs_splats* splats, int64_t n, const gs_layout* layout,
                     const gs_bins* bins, float* features, void* stream) {
    REQUIRE(layout_ok(layout), "gs_tile_features: invalid layout");
    REQUIRE(splats && bins && features, "gs_tile_features: null pointer");
    return launch_tile_features(*splats, n, *layout, *bins, features, (hipStream_t)stream);
}

int gs_mlp_forward(const float* weights, const float* norm, const float* features, int64_t rows,
                   float* out, void* stream) {
    REQUIRE(weights && norm && (rows == 0 || (features && out)), "gs_mlp_forward: null pointer");
    REQUIRE(rows >= 0, "gs_mlp_forward: rows < 0");
    return launch_mlp_forward(weights, norm, features, rows, out, (hipStream_t)stream);
}

int gs_mlp_train_step(float* weights, const float* norm, const float* features,
                      const float* targets, int64_t rows, float* grad_scratch, float* m, float* v,
                      int32_t* step, float lr, float* loss_out, void* stream) {
    REQUIRE(weights && norm && features && targets && grad_scratch && m && v && step,
            "gs_mlp_train_step: null pointer");
    REQUIRE(rows >= 1, "gs_mlp_train_step: rows < 1");
    return launch_mlp_train_step(weights, norm, features, targets, rows, grad_scratch, m, v, step, lr,
                                 loss_out, (hipStream_t)stream);
}

size_t gs_order_by_cost_scratch_size(int32_t total_tiles) {
    if (total_tiles < 1) return 0;
    return sort_pairs_scratch(total_tiles) + 4 * ((size_t)total_tiles + 64);
}

int gs_order_by_cost(const float* predicted, int32_t total_tiles, uint32_t* order, void* scratch,
                     void* stream) {
    REQUIRE(predicted && order && scratch, "gs_order_by_cost: null pointer");
    REQUIRE(total_tiles >= 1, "gs_order_by_cost: total_tiles < 1");
    return launch_order_by_cost(predicted, total_tiles, order, scratch, (hipStream_t)stream);
}

}  // extern "C"
