/*
 * gs.h -- C ABI of the MI355X (gfx950) 3D Gaussian Splatting training hot path.
 *
 * One training iteration is five calls, in the stage order of the paper's
 * pipeline (Sec. 2; stages timed separately in its supplementary timing
 * tables): projection forward -> binning and sorting -> rasterisation forward
 * -> rasterisation backward (with the L1 loss gradient fused in) -> projection
 * backward fused with Adam (Sec. 4.3).
 *
 *   gs_project          EWA projection, SH degree-3 colour, tiles touched
 *                       per Gaussian (Sec. 4.1: counts are produced during
 *                       projection, the key buffer is filled in a later pass)
 *   gs_bin_sort         exclusive scan of the counts, 32-bit (tile, depth) key
 *                       generation with depth map z -> (2z+1)/(z+1) and tile id
 *                       in the top bits (Sec. 4.4), stable LSD radix sort per
 *                       view, per-tile ranges
 *   gs_rasterize_fwd    front-to-back alpha compositing per tile
 *   gs_rasterize_bwd    exact derivative of the compositing, transmittance
 *                       recomputed front to back, no pixel-level atomics
 *                       (Sec. 4.2)
 *   gs_project_bwd_adam projection backward and Adam in one pass, scales and
 *                       opacities updated in log/logit space, no per-parameter
 *                       gradient buffer (Sec. 4.3)
 *
 * Conventions for every call:
 *  - Pointers named *_dev or documented as "device" are device (HBM) pointers;
 *    gs_layout and the small gs_* descriptor structs themselves live on the
 *    host and are read before the call returns.
 *  - The caller owns every buffer.  The library allocates no memory and keeps
 *    no state apart from a per-thread error string.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL = the
 *    default stream); no call synchronises with the host, so every call can be
 *    captured into a HIP graph.
 *  - Return value: GS_OK or a negative GS_ERR_*.  Argument errors are reported
 *    synchronously and nothing is enqueued.  Data-dependent failures (more
 *    intersections than the key buffers hold) set bits in the device status
 *    word of gs_bins instead; outputs of that iteration are then undefined but
 *    every access stays in bounds.  gs_last_error() describes the last error
 *    of the calling thread.
 *  - Results are deterministic: identical inputs give bitwise-identical
 *    outputs (no floating-point atomics anywhere).
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GS_VERSION 1
#define GS_MAX_VIEWS 16
#define GS_PARAM_PLANES 15 /* float4 planes per Gaussian in a parameter block */

enum {
    GS_OK = 0,
    GS_ERR_INVALID_ARG = -1,
    GS_ERR_HIP = -2,
    GS_ERR_WORKSPACE = -3,
    GS_ERR_CAPACITY = -4
};

/* bits of the device status word */
#define GS_STATUS_CAPACITY 1u  /* intersections exceeded gs_bins.capacity */
#define GS_STATUS_OVERFLOW 2u  /* intersection count exceeded 2^32 - 1 */
#define GS_STATUS_ROWS 4u      /* tile-row slots exceeded gs_bins.row_capacity */
#define GS_STATUS_SORT 8u      /* a sort pass gave up waiting on an earlier chunk's counts
                                  (never expected; the sorted order is then invalid) */

/* tile-set rules (gs_layout.cull) */
#define GS_CULL_RECT 0     /* tiles meeting the 3-sigma box [mean +- r] */
#define GS_CULL_ELLIPSE 1  /* exact culling (Sec. 4.1): tiles meeting the ellipse
                              A dx^2 + 2 B dx dy + C dy^2 <= 2 ln(255 o), where the
                              Gaussian can reach alpha 1/255 */

/* One camera view, 128 bytes.  OpenCV camera (x right, y down, z forward);
 * pixel (column j, row i) has its centre at (j + 0.5, i + 0.5). */
typedef struct gs_view {
    float R[9];        /* world -> camera rotation, row major */
    float t[3];        /* world -> camera translation */
    float campos[3];   /* camera centre in world space (SH view direction) */
    float fx, fy, cx, cy;
    float lim_x, lim_y; /* clamp of x/z and y/z in the EWA Jacobian (1.3 tan(fov/2)) */
    float znear, zfar; /* Gaussians with depth outside (znear, zfar) are culled */
    float bg[3];       /* background colour */
    int32_t width, height;
    int32_t pad[4];
} gs_view;

/* Geometry of a set of views rendered together, filled by gs_layout_init.
 * Tiles and pixels of all views are numbered consecutively: view v owns global
 * tiles [tile_base[v], tile_base[v+1]) and pixels [pixel_base[v],
 * pixel_base[v+1]); within a view tiles are row major (tile = ty*tiles_x+tx). */
typedef struct gs_layout {
    int32_t n_views;
    int32_t tile;                          /* tile edge T in pixels: 8, 16 or 32 */
    int32_t pixels_per_lane;               /* rasteriser lanes per tile = T*T / this; 1 for
                                              T = 8, 1, 2 or 4 otherwise (default 2) */
    int32_t cull;                          /* GS_CULL_RECT (default) or GS_CULL_ELLIPSE */
    int32_t width[GS_MAX_VIEWS], height[GS_MAX_VIEWS];
    int32_t tiles_x[GS_MAX_VIEWS], tiles_y[GS_MAX_VIEWS];
    int32_t depth_bits[GS_MAX_VIEWS];      /* D = min(23, 32 - B), B = ceil(log2 #tiles), B >= 1 */
    int32_t tile_base[GS_MAX_VIEWS + 1];
    int64_t pixel_base[GS_MAX_VIEWS + 1];
} gs_layout;

/* Parameter block: GS_PARAM_PLANES planes of n float4 each, plane-major
 * (element (p, g) at float offset 4*(p*n + g)).  Plane 0 = (mean x, y, z,
 * opacity logit); plane 1 = (log-scale x, y, z, unused); plane 2 = quaternion
 * (w, x, y, z), not required to be normalised; planes 3..14 = the 48 SH
 * coefficients c[m*3 + k] (basis function m = 0..15, channel k), plane 3+q
 * holding c[4q .. 4q+3].  Adam moments and gradient outputs use the same
 * layout.  (Paper Sec. 4.6: SH split into 12 128-bit values, scale and opacity
 * packed into 128-bit values.) */

/* Per-view projection outputs, each an array of n_views * n entries indexed
 * [view * n + g]. */
typedef struct gs_splats {
    float* rec;       /* 16 floats (64 bytes, one cache line) per entry:
                           (u, v, A, B)   mean in pixels, conic A, B
                           (C, o, r, g)   conic C, opacity, colour r, g
                           (b, z, radius, 0)  colour b, depth, radius in pixels
                           (rect0, rect1, dcode, 0) uint32 bits:
                               rect0 = x0 | y0 << 16, rect1 = x1 | y1 << 16:
                               the bounding box [x0, x1) x [y0, y1) of the
                               tile set (the whole set for GS_CULL_RECT);
                               dcode = the 23 mantissa bits of the float32
                               (2z + 1) / (z + 1) (the depth part of the keys)
                         colour is after the +0.5 shift and the clamp at 0;
                         entries of culled Gaussians are all zero */
    uint32_t* tiles;  /* tiles touched, 0 for culled Gaussians */
} gs_splats;

/* Intersection buffers.  Intersections of view v occupy the contiguous
 * segment [offsets[v*n], offsets[(v+1)*n]); within it Gaussian g owns the
 * "unsorted indices" [offsets[v*n+g], offsets[v*n+g+1]), one per tile of its
 * tile set in emission order: tile rows y0..y1-1 outer, each row's column
 * span inner.  Every (view, Gaussian) with tiles owns the row slots
 * [row_offsets[v*n+g], row_offsets[v*n+g+1]), one per tile row y0..y1-1 of
 * its bounding box (rows whose span is empty included). */
typedef struct gs_bins {
    uint32_t* offsets;   /* n_views*n + 1: exclusive scan of tiles; [n_views*n] = K */
    uint32_t* row_offsets; /* n_views*n + 1: exclusive scan of tile rows; [n_views*n] = R */
    uint32_t* rows;      /* 4 words per row slot: (first unsorted index of the row,
                            (view, Gaussian) index v*n+g, xa | ty << 16, depth bits
                            of the Gaussian's keys): the row's tiles are (xa.., ty),
                            as many as the next slot's first index minus this one */
    int64_t row_capacity; /* row slots in `rows` */
    uint32_t* keys;      /* capacity: (tile << D) | depth bits, sorted per view */
    uint32_t* vals;      /* capacity: Gaussian id of each sorted key */
    uint32_t* ranges;    /* 2 * total tiles: [start, end) of each tile in sorted order */
    uint32_t* status;    /* 1 word, device status bits (GS_STATUS_*), cleared by gs_bin_sort */
    int64_t capacity;    /* entries in keys / vals and records in gs_grads2d */
} gs_bins;

/* Screen-space gradients written by gs_rasterize_bwd and read by
 * gs_project_bwd_adam: one record per intersection that some pixel of its
 * tile composited (the only ones with a non-zero gradient), at its unsorted
 * index, so that each (view, Gaussian) finds its records in its own
 * contiguous index range; rec_mask flags which records the last call wrote. */
typedef struct gs_grads2d {
    float* rec;           /* capacity records of 12 floats: (d u, d v, d A, d B, d C,
                             d opacity, d r, d g, d b, owner, 0, 0), owner = the bits of
                             the uint32 index v*n+g of the record's (view, Gaussian);
                             records not flagged in rec_mask are left as they were */
    uint32_t* rec_mask;   /* ceil(capacity / 32) words: bit i (word i / 32, bit i % 32)
                             set iff record i was written by the last gs_rasterize_bwd */
    uint32_t* tile_stop;  /* total tiles: the backward traversed sorted positions
                             [ranges[t].start, tile_stop[t]) of tile t (up to the last
                             entry any of its pixels composited) */
    float* sums;          /* 9 planes of n_views * n floats, plane c at c * n_views * n:
                             per (view, Gaussian) sum of its records flagged in rec_mask
                             (components 0..8), written by gs_project_bwd_adam */
    void* workspace;      /* unused (gs_grads2d_workspace_size is 0); may be NULL */
} gs_grads2d;

/* Rasterisation outputs, indexed by global pixel (views concatenated). */
typedef struct gs_image {
    float* rgb;           /* pixels * 3, channel last: C + T_final * bg */
    float* T;             /* pixels: final transmittance */
    uint32_t* last;       /* pixels: 1 + list position (within the tile) of the last
                             composited entry, 0 if none */
    uint32_t* tile_stats; /* nullable; 4 * total tiles: (entries traversed by the tile
                             = max over its pixels of the entries examined, pixel-Gaussian
                             pairs evaluated, pairs composited, 0) */
    uint32_t* comp_mask;  /* ceil(capacity / 32) words, written by gs_rasterize_fwd and
                             read by gs_rasterize_bwd: bit j set iff some pixel of the
                             tile composited sorted entry j */
} gs_image;

/* Optional persistent schedule for the rasterisation kernels: a fixed grid of
 * workgroups pops tiles from a device counter, in the order given by `order`. */
typedef struct gs_schedule {
    const uint32_t* order; /* device, total tiles: global tile ids, a permutation;
                              NULL = ascending */
    uint32_t* counter;     /* device, 1 word, scratch for the work queue */
    int32_t n_groups;      /* workgroups in the persistent grid, >= 1 */
} gs_schedule;

/* Adam state (Kingma & Ba; the bias-corrected form of torch.optim.Adam). */
typedef struct gs_adam {
    float* m;            /* parameter-block layout */
    float* v;            /* parameter-block layout */
    int32_t* step;       /* device, 1 word: incremented by each gs_project_bwd_adam call
                            before use, so the first call runs step 1 */
    float* scratch;      /* device, 4 floats: bias corrections of the current step */
    float lr[6];         /* per group: means, log-scales, quaternion, opacity, SH DC, SH rest */
    float beta1, beta2, eps;
} gs_adam;

/* ---- host-side helpers ---------------------------------------------------- */

int gs_version(void);
const char* gs_last_error(void);

/* Fill a layout for n_views (1..GS_MAX_VIEWS) images of the given sizes and
 * tile edge T (8, 16 or 32).  Fails if any view has more than 2^16 tiles per
 * axis or the total number of tiles exceeds 2^31. */
int gs_layout_init(const int32_t* widths, const int32_t* heights, int n_views, int tile,
                   gs_layout* out);

/* Bytes of scratch that gs_bin_sort needs for n Gaussians, the layout and the
 * given intersection capacity. */
size_t gs_bin_sort_workspace_size(int64_t n, const gs_layout* layout, int64_t capacity);

/* Bytes of scratch (gs_grads2d.workspace) that gs_project_bwd_adam needs for
 * the given intersection capacity: none (0); the per-Gaussian record sums are
 * formed in LDS. */
size_t gs_grads2d_workspace_size(int64_t capacity);

/* A second stream a call may run independent work on, with the two events
 * that fork it from and join it back to the call's stream; all three owned by
 * the caller. */
typedef struct gs_side_stream {
    void* stream;   /* hipStream_t, default priority */
    void* fork;     /* hipEvent_t */
    void* join;     /* hipEvent_t */
} gs_side_stream;

/* ---- the five stages ------------------------------------------------------ */

/* Projection forward (paper Sec. 2 parameterisation; Sec. 4.1 tile count).
 * For every Gaussian g and view v: Sigma = R S S^T R^T (R from the normalised
 * quaternion, S = diag(exp(log-scale))); camera-space mean p = R_v mean + t_v,
 * culled unless znear < p.z < zfar; 2D covariance J R_v Sigma R_v^T J^T + 0.3 I
 * (J the pinhole Jacobian at p with x/z, y/z clamped to +-lim), culled if its
 * determinant is not positive; conic = its inverse; radius = ceil(3 sqrt of its
 * larger eigenvalue); tile set = the tiles overlapping [mean2d - r, mean2d + r]
 * clipped to the image (GS_CULL_RECT), or the tiles meeting the opacity
 * ellipse (GS_CULL_ELLIPSE, see the define), culled if empty; opacity = sigmoid(logit); colour =
 * max(0, sum_m sh[m] Y_m(dir) + 0.5) along dir = (mean - campos)/|mean - campos|.
 * Float steps that decide the rectangle are evaluated in float32 without
 * contraction in a fixed order.  Non-finite parameters cull the Gaussian.
 *   params  device parameter block of n Gaussians
 *   views   device array of layout->n_views gs_view
 *   out     device outputs, n_views * n entries each */
int gs_project(const float* params, int64_t n, const gs_view* views, const gs_layout* layout,
               const gs_splats* out, void* stream);

/* Binning and sorting (Sec. 4.1 count-then-fill, Sec. 4.4 32-bit keys).
 * offsets = exclusive scan of splats->tiles over (view, g); K = offsets[V*n];
 * row_offsets and rows describe each Gaussian's tile rows (R = row_offsets[V*n];
 * GS_STATUS_ROWS is set if R > row_capacity).
 * For each Gaussian, one key per touched tile at its unsorted index:
 * key = (tile << D) | (mantissa(f) >> (23 - D)) with f = (2z+1)/(z+1) in
 * float32, value = g.  Keys of each view are sorted ascending by a stable LSD
 * radix sort (ties keep emission order), then ranges[t] =
 * [lower_bound(t << D), lower_bound((t+1) << D)) in the view's segment, as
 * global positions.  Unsorted index of Gaussian g's entry for tile (tx, ty):
 * rows[4 r] + (tx - xa) with r = row_offsets[v*n+g] + (ty - y0).  If K > capacity only the first `capacity`
 * intersections are written and GS_STATUS_CAPACITY is set; the caller reads
 * offsets[V*n] to size a retry.
 * With many intersections per (view, Gaussian) the depth sort of the
 * (view, Gaussian)s can run beside the scans and row slots: if `side` is
 * given, it is enqueued on side->stream after side->fork is recorded on
 * `stream`, and `stream` waits on side->join (recorded on side->stream after
 * it), so the call stays ordered on `stream` and capturable in a graph; with
 * side NULL everything runs on `stream`.  Same results either way.
 *   workspace  device scratch of gs_bin_sort_workspace_size bytes
 *   side       nullable; caller-owned stream (default priority) and two events
 *              (created with hipEventDisableTiming), used only by this call
 *              while it runs */
int gs_bin_sort(const gs_splats* splats, int64_t n, const gs_layout* layout, const gs_bins* bins,
                void* workspace, size_t workspace_bytes, const gs_side_stream* side, void* stream);

/* Rasterisation forward.  Per pixel, front to back over its tile's sorted
 * list: d = pixel centre - mean2d, power = -1/2 (A dx^2 + C dy^2) - B dx dy,
 * skipped if power > 0; alpha = min(0.99, o e^power), skipped if < 1/255; the
 * pixel stops (entry not composited) once T (1 - alpha) < 1e-4; otherwise
 * C += alpha T c and T *= 1 - alpha.  Output C + T bg.
 *   lds_batch  Gaussians staged in LDS per batch: 32, 64, 128 or 256
 *   sched      NULL: one workgroup per tile; else persistent work queue */
int gs_rasterize_fwd(const gs_splats* splats, int64_t n, const gs_layout* layout,
                     const gs_bins* bins, const gs_view* views, const gs_image* out, int lds_batch,
                     const gs_schedule* sched, void* stream);

/* Rasterisation backward (Sec. 4.2), the exact piecewise derivative of the
 * forward: transmittance is recomputed front to back; with S_i the colour
 * composited behind entry i plus T_final bg,
 *   dL/dc_i = alpha_i T_i g,   dL/dalpha_i = g . (T_i c_i - S_i / (1 - alpha_i)),
 * then through alpha = min(0.99, o G) (no gradient through the clamp),
 * G = e^power and the quadratic form.  g = dL/dC comes from `dL_dC`
 * (pixels * 3) or, if `target` (pixels * 3) is given, from the fused L1 loss
 * mean|C - target| over all channels of all pixels: g = sign(C - target) /
 * (3 * pixels).  Per-pixel contributions are summed over each tile with
 * wavefront reductions (no floating-point atomics) into one record per
 * intersection that some pixel of its tile composited (fwd->comp_mask), written
 * at its unsorted index (see gs_grads2d); entries no pixel composited are
 * skipped without being evaluated, and a tile's traversal ends at the last
 * entry any of its pixels composited.
 *   loss      nullable device, total tiles floats: per-tile sum |C - target|
 *             (only with `target`)
 *   lds_batch  Gaussians staged in LDS per batch: 32, 64, 128 or 256; or
 *             -64, -128, -256 for a per-tile batch (Sec. 4.2): for a tile of P
 *             pixels with N listed Gaussians, sqrt(N P) rounded up to a
 *             multiple of 64 and capped at -lds_batch.  The batch size changes
 *             no result, only the schedule. */
int gs_rasterize_bwd(const gs_splats* splats, int64_t n, const gs_layout* layout,
                     const gs_bins* bins, const gs_view* views, const gs_image* fwd,
                     const float* target, const float* dL_dC, const gs_grads2d* grads,
                     float* loss, int lds_batch, const gs_schedule* sched, void* stream);

/* Rasterisation backward, two-phase form (Sec. 4.2, the second
 * implementation): per batch of lds_batch (16, 32 or 64) entries some pixel
 * composited, a pixel-parallel pass recomputes transmittance front to back and
 * stores, per (entry, pixel), dL/dpower and alpha T in LDS; a Gaussian-
 * parallel pass then sums them over the tile's pixels into the entry's record
 * as a contraction on the fp32 matrix cores (per-pair terms against the
 * pixel moments 1, X, Y, X^2, XY, Y^2 and the pixels' dL/dC; no cross-lane
 * reductions).  Same arguments, outputs and record format as
 * gs_rasterize_bwd (the records agree with it up to float summation order);
 * 8x8 and 16x16 tiles only. */
int gs_rasterize_bwd_twophase(const gs_splats* splats, int64_t n, const gs_layout* layout,
                              const gs_bins* bins, const gs_view* views, const gs_image* fwd,
                              const float* target, const float* dL_dC, const gs_grads2d* grads,
                              float* loss, int lds_batch, const gs_schedule* sched, void* stream);

/* Fused L1 + D-SSIM loss gradient against an RGBA8 reference (Sec. 4.5: the
 * weighted sum of the L1 and SSIM losses in one fused evaluation, the reference
 * kept as 4 x uint8, alpha masking fused):
 *   L = (1 - lambda)/(3P) sum_p m_p sum_k |x_pk - y_pk|
 *     + lambda/(3P) sum_p m_p sum_k (1 - S_pk)
 * over the P pixels of all views, x the render, y = rgb / 255, m = alpha / 255
 * if use_mask else 1, S the SSIM map of each colour channel of each view (an
 * 11 x 11 Gaussian window with sigma 1.5, zero outside the view's image,
 * C1 = 0.01^2, C2 = 0.03^2).  The gradient dL/dx goes to dL_dC, the input of
 * gs_rasterize_bwd.
 *   rgb          device, pixels x 3 float: the render (gs_image.rgb)
 *   target       device, pixels x 4 uint8 (R, G, B, A), 4-byte aligned
 *   dL_dC        device, pixels x 3 float, written
 *   loss_blocks  device, 2 x gs_loss_blocks(layout) floats, nullable: per unit
 *                (64 x 16 pixel block of a view, colour channel) -- unit
 *                3 b + k for block b (views in order, blocks row-major) and
 *                channel k -- the sums of m |x - y| and of m (1 - S) over the
 *                block's pixels in that channel;
 *                L = ((1 - lambda) sum of the first + lambda sum of the second) / (3P)
 *   workspace    device scratch of gs_loss_workspace_size(layout) bytes, 16-byte
 *                aligned (9 floats per pixel of each view padded to whole
 *                64 x 16 blocks); gs_loss_workspace_size returns 0, and the call
 *                fails, when 9 x the padded pixels or 3 x the pixels exceed
 *                2^31 - 1
 * Deterministic; no atomics. */
int64_t gs_loss_blocks(const gs_layout* layout);
size_t gs_loss_workspace_size(const gs_layout* layout);
int gs_loss_l1_ssim(const float* rgb, const uint8_t* target, const gs_layout* layout, float lambda,
                    int use_mask, float* dL_dC, float* loss_blocks, void* workspace,
                    size_t workspace_bytes, void* stream);

/* Projection backward fused with Adam (Sec. 4.3).  First pass: for each
 * (view, Gaussian), the sum of its records flagged in grads->rec_mask, in
 * unsorted-index order, into grads->sums.  Second pass, per Gaussian: applies the
 * chain rule back through colour (SH basis, clamp, view direction), opacity
 * (sigmoid), conic (inverse), 2D covariance (J R Sigma R^T J^T), the pinhole
 * Jacobian and mean projection, scales (exp) and the quaternion normalisation,
 * summing over views; then, if `adam` is given, updates params, m and v in
 * place (log-scales and logits updated as stored).  If `grads_out` is given the
 * gradients are also written there (parameter-block layout).  At least one of
 * adam, grads_out must be non-NULL. */
int gs_project_bwd_adam(float* params, int64_t n, const gs_view* views, const gs_layout* layout,
                        const gs_splats* splats, const gs_bins* bins, const gs_grads2d* grads,
                        const gs_adam* adam, float* grads_out, void* stream);

/* gs_project_bwd_adam for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and results.  The projection backward needs no
 * device scratch at all (the per-(view, Gaussian) record sums are formed in
 * LDS), so neither entry point allocates, reads grads->workspace (it may be
 * NULL) or keeps state between calls; calls on one stream are ordered, calls
 * that overlap on one GPU race only through the caller's own buffers.  Calls
 * no allocating routine. */
int gs_project_bwd_adam_noalloc(float* params, int64_t n, const gs_view* views, const gs_layout* layout,
                                const gs_splats* splats, const gs_bins* bins, const gs_grads2d* grads,
                                const gs_adam* adam, float* grads_out, void* stream);

/* ---- learned tile schedule (per-tile cost model) --------------------------- */

/* 8 features per tile of the current bins (float, total tiles x 8): log(1 +
 * list length); mean and max opacity, mean and min depth and mean radius over
 * the first min(length, 512) entries of the sorted list; tile x and y (centre,
 * normalised by the view's tile grid). */
int gs_tile_features(const gs_splats* splats, int64_t n, const gs_layout* layout,
                     const gs_bins* bins, float* features, void* stream);

/* MLP 8 -> 32 -> 32 -> 1 with ReLU, fp32.  Weights (1377 floats) in the order
 * W1[32][8], b1[32], W2[32][32], b2[32], W3[32], b3[1].  norm: 32 floats,
 * per feature its mean, standard deviation, low and high (8 each): a feature
 * is clamped to [low, high] (the range seen in training, so that a scene
 * unlike the training scenes is not extrapolated), then standardised, before
 * the first layer. */
#define GS_MLP_PARAMS 1377
int gs_mlp_forward(const float* weights, const float* norm, const float* features, int64_t rows,
                   float* out, void* stream);
/* One full-batch Adam step on the mean squared error between the MLP output
 * and `targets` over `rows` examples (deterministic: fixed-order partial sums
 * over GS_MLP_GROUPS workgroups).  grad_scratch: GS_MLP_SCRATCH floats;
 * m, v: GS_MLP_PARAMS floats each; step: device int, incremented; loss_out:
 * nullable device float. */
#define GS_MLP_GROUPS 64
#define GS_MLP_SCRATCH ((GS_MLP_GROUPS + 1) * (GS_MLP_PARAMS + 1))
int gs_mlp_train_step(float* weights, const float* norm, const float* features,
                      const float* targets, int64_t rows, float* grad_scratch, float* m, float* v,
                      int32_t* step, float lr, float* loss_out, void* stream);
/* Order tiles by descending predicted cost (ties by ascending tile id) into
 * `order` (total tiles); falls back to ascending order if any prediction is
 * not finite.  scratch: device, gs_order_by_cost_scratch_size bytes. */
size_t gs_order_by_cost_scratch_size(int32_t total_tiles);
int gs_order_by_cost(const float* predicted, int32_t total_tiles, uint32_t* order, void* scratch,
                     void* stream);

/* Thompson-sampling choice among rasterisation-backward variants (Sec. 4.2:
 * a latency belief per implementation, a random choice favouring the faster
 * ones, a belief update from each measured latency).  Host code, no GPU.
 * Each arm's latencies are Normal(mu, 1/tau) under the conjugate Normal-Gamma
 * prior (mu0, kappa0, alpha0, beta0); after n observations with mean xbar and
 * squared deviations m2:
 *   kappa_n = kappa0 + n, mu_n = (kappa0 mu0 + n xbar) / kappa_n,
 *   alpha_n = alpha0 + n/2, beta_n = beta0 + m2/2 + kappa0 n (xbar - mu0)^2 / (2 kappa_n).
 * gs_ts_select draws tau ~ Gamma(alpha_n, rate beta_n) and mu ~ Normal(mu_n,
 * 1/(kappa_n tau)) per arm and returns the arm with the smallest mu (or a
 * negative GS_ERR_*).  Random numbers come from the splitmix64 sequence seeded
 * by `seed`, so a state replays exactly.  The caller owns the state; calls on
 * one state must not overlap.
 *   gs_ts_init       prior: finite mu0, kappa0 > 0, alpha0 >= 1, beta0 > 0;
 *                    1 <= n_arms <= GS_TS_MAX_ARMS
 *   gs_ts_update     folds one measured latency of `arm` into its belief
 *   gs_ts_posterior  out[4] = (mu_n, kappa_n, alpha_n, beta_n) of `arm`
 *   gs_ts_sample     one draw of `arm`'s mean latency (NaN for an invalid arm) */
#define GS_TS_MAX_ARMS 8
typedef struct gs_ts_state {
    int32_t n_arms;
    int32_t reserved;
    uint64_t rng;                              /* splitmix64 state */
    double mu0, kappa0, alpha0, beta0;         /* prior */
    double n[GS_TS_MAX_ARMS];                  /* observations per arm */
    double mean[GS_TS_MAX_ARMS];               /* their running mean */
    double m2[GS_TS_MAX_ARMS];                 /* their sum of squared deviations */
} gs_ts_state;
int gs_ts_init(gs_ts_state* st, int n_arms, uint64_t seed, double mu0, double kappa0, double alpha0,
               double beta0);
int gs_ts_select(gs_ts_state* st);
int gs_ts_update(gs_ts_state* st, int arm, double latency);
int gs_ts_posterior(const gs_ts_state* st, int arm, double* out);
double gs_ts_sample(gs_ts_state* st, int arm);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
