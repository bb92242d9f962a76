/*
 * bgt.h -- C ABI of the BG-Triangle rasterizer for AMD Instinct MI355X (gfx950).
 *
 * BG-Triangle ("Bezier Gaussian Triangle for 3D Vectorization and
 * Rendering", CVPR 2025) renders degree-n Bezier triangles (Sec. 3.1, Eq. 1-2)
 * by tessellating them into flat triangles and rasterizing those into an index
 * map I_id and a coordinate map I_uv with a boundary set B (Sec. 3.2,
 * Tessellation and Rasterization).  It then places one Gaussian per foreground
 * pixel (Sec. 3.2, Sub-Primitive Generation, Eq. 3-5) and alpha-blends them
 * with the boundary-aware coefficient w (Sec. 3.2, Discontinuity-Aware Alpha
 * Blending, Eq. 6-8) using tiles with per-tile boundary lists sorted by
 * primitive id (Sec. 3.2, Rendering Acceleration).  The backward pass follows
 * Supplementary Sec. C.
 *
 * Conventions shared by every entry point
 *  - Pointers are device memory unless marked (host).  Every call only
 *    enqueues work on `stream` (a hipStream_t; NULL = the null stream) and
 *    never synchronizes, except bgt_query.
 *  - The caller owns every input, output and `state` buffer.  The library
 *    allocates nothing per call, so calls are safe under stream capture.
 *  - Errors are return codes.  Argument errors give BGT_E_INVALID before any
 *    work is enqueued; bgt_last_error(ctx) has the text.
 *  - Capacity overflow.  The pair lists live in the caller's state, sized by
 *    pair_factor and bpair_factor; a forward pass that needs more clamps the
 *    lists (its images and gradients are then incomplete) and records the
 *    overflow on the device, also inside a captured graph.  The device
 *    copies the bits into a word of pinned host memory that the context
 *    owns, so the next bgt_render_fwd or bgt_render_bwd on the context that
 *    runs after the device has executed that pass returns BGT_E_OVERFLOW
 *    without waiting for the device and enqueues nothing; bgt_query always
 *    reports it.  Reporting clears the word.  The caller then grows the
 *    capacities (a new context), resizes the state and recomputes.
 *  - A context is not thread-safe; use one context per host thread.
 *
 * Layouts (structure of arrays, float32)
 *  - ncp = (n+1)(n+2)/2 control points, indexed in the order of Eq. 1's
 *    double sum: i = 0..n outer, j = 0..n-i inner, k = n-i-j; u pairs with
 *    i, v with j, w with k.
 *  - ctrl, color_ctrl: [3][ncp][P]; log_scale: [3][T][P]; quat: [4][T][P]
 *    as (w,x,y,z), T = R(R+1)/2 texels of the attribute map (R = attr_res,
 *    1 or 3; texel t enumerates the nodes (a, b), a + b <= R - 1, of the
 *    barycentric lattice of level R - 1 at (u, v) = (a, b) / (R - 1), a
 *    outer); opacity, sharpness: [P]; sh: [3][K][P], K = (D+1)^2 - 1 for
 *    SH degree D = sh_degree (bands 1..D, m = -l..l within a band).
 *  - Camera v: 16 floats = world-to-camera rotation R (row-major 3x3),
 *    translation t (3), fx, fy, cx, cy.  Axes x right, y down, z forward;
 *    pixel (i, j) has its centre at (i + 0.5, j + 0.5).
 *  - Images: packed HWC float32, view v starting at pixel offset
 *    sum_{u<v} W_u H_u, i.e. element 3 * (offset + y W_v + x) + channel.
 */
#ifndef BGT_H
#define BGT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BGT_OK = 0,
    BGT_E_INVALID = 1,     /* bad argument; nothing was enqueued */
    BGT_E_NOMEM = 2,       /* state buffer too small or host allocation failed */
    BGT_E_OVERFLOW = 3,    /* a pair capacity was exceeded (see bgt_query) */
    BGT_E_HIP = 4,         /* a HIP runtime call failed */
    BGT_E_UNSUPPORTED = 5  /* valid request outside what this library implements */
} bgt_status;

#define BGT_MAX_VIEWS 64

/* bgt_config.flags.  BGT_FLAG_NO_BOUNDARY renders the variant without
 * blending coefficients of the ablation study (Sec. 4.3, Table 3, "w/o B"):
 * every Gaussian composites with w = 1 in Eq. 8, whatever primitive the pixel
 * belongs to; no boundary points are extracted (the boundary set and its
 * tile lists are empty) and the sharpness gradient is 0. */
#define BGT_FLAG_NO_BOUNDARY 1
#define BGT_MAX_DEGREE 5

typedef struct bgt_ctx bgt_ctx;

/* BG-Triangle parameters (Sec. 3.1 control points p_ijk; Sec. 3.2 colour
 * control points p^c_ijk and attribute maps M_h; opacity o, Eq. 8).
 * `sharpness` s_g sets the boundary Gaussian scale r_b = r_ref / s_g.
 * Eq. 5's attribute maps: a Gaussian's log-scales and raw quaternion are the
 * linear interpolation, at its I_uv, of the three texels of the lattice
 * triangle that contains it (R = 1: the single texel); the quaternion is then
 * normalised.  SH colour (resolution-1 map): with D = sh_degree > 0 a
 * Gaussian's colour is Eq. 4's diffuse colour plus sum_k Y_k(d) sh_k, Y_k
 * the real spherical harmonics of bands 1..D (Condon-Shortley phase) and d
 * the unit vector from the camera centre to S_q. */
typedef struct {
    int32_t degree;      /* n, 1..BGT_MAX_DEGREE */
    int32_t num_prims;   /* P >= 1 */
    int32_t attr_res;    /* R, 1 or 3 (the implementation details' rotation and scale maps) */
    int32_t sh_degree;   /* D, 0..3 */
    const float *ctrl, *color_ctrl, *log_scale, *quat, *opacity, *sharpness;
    const float *sh;     /* [3][K][P]; may be NULL when D = 0 */
} bgt_prims;

/* Gradients, same layouts as bgt_prims; every array is overwritten (`sh`
 * only when the prims' sh_degree > 0; it may be NULL otherwise). */
typedef struct {
    float *ctrl, *color_ctrl, *log_scale, *quat, *opacity, *sharpness;
    float *sh;
} bgt_grads;

/* A batch of views rendered together in one call. */
typedef struct {
    int32_t n_views;        /* 1..BGT_MAX_VIEWS */
    int32_t reserved;
    const int32_t *wh;      /* (host) [2 n_views]: width, height of each view */
    const float *cams;      /* [n_views][16] cameras, see Layouts */
} bgt_views;

/* Rendering constants.  bgt_default_config fills the values this library
 * documents for each reading of the paper. */
typedef struct {
    int32_t tess_level;    /* L, sub-triangles per patch L^2, 1..8 (default 4) */
    int32_t tile;          /* blending tile side: 8, 16 or 32 (default 16) */
    int32_t batch;         /* Gaussians staged per LDS batch: 32, 64 or 128, at most tile*tile */
    int32_t flags;         /* BGT_FLAG_* bits (default 0) */
    float z_near;          /* cull distance along the optical axis (0.2) */
    float g_min;           /* Gaussian support: G >= g_min (2^-15) */
    float t_min;           /* stop once transmittance < t_min (2^-15) */
    float alpha_max;       /* alpha clamp (0.99) */
    float dilation;        /* 2-D low-pass added to projected covariances (0.3) */
    float r_ref;           /* r_b = r_ref / sharpness (1e-2) */
    float bg[3];           /* background colour (0, 0, 0) */
    float pair_factor;     /* Gaussian-tile pair capacity per Gaussian record (4) */
    float bpair_factor;    /* boundary-tile pair capacity per pixel (2) */
    int32_t lattice;       /* 0: one Gaussian per foreground pixel (Sec. 3.2; default); m in
                              2..16: the lattice variant, m Gaussians per flat sub-triangle edge */
} bgt_config;

/* The lattice variant.  Sec. 3.2 places one Gaussian at every foreground
 * pixel, at I_uv(q).  With lattice = m the rendered Gaussians are instead
 * the nodes (a, b), a + b <= M, M = L (m - 1), of each patch's (u, v)
 * domain at (u, v) = (a/M, b/M): m per edge of every flat sub-triangle,
 * nodes on edges shared by two sub-triangles counted once, so a patch
 * carries NL = (M+1)(M+2)/2 Gaussians in every view, evaluated with Eq. 3-5
 * and the EWA projection like a pixel's.  The boundary points, and so the
 * blending coefficients of Eq. 6-7, stay those of the foreground pixels.
 * Records: the state's record array holds the N pixel records (boundary
 * points only, in this variant) followed by the lattice records, view v,
 * patch p, node k (a outer, b inner) at N + (v P + p) NL + k.  Each view
 * needs W H + P NL < 2^24 and all views N + V P NL < 2^31. */

void bgt_default_config(bgt_config *cfg);

/* Host-only argument checks (no device work, no context needed). */
bgt_status bgt_validate_config(const bgt_config *cfg);
bgt_status bgt_validate_prims(const bgt_prims *prims, const bgt_config *cfg);
bgt_status bgt_validate_views(const bgt_views *views);

/* Create a context on HIP device `device`; device -1 gives a host-only
 * context that can size and validate but not enqueue work.  A device context
 * allocates its 8-byte overflow word of pinned host memory here (the only
 * allocation the library makes; it is freed by bgt_destroy).  *out is NULL
 * on failure. */
bgt_status bgt_create(const bgt_config *cfg, int device, bgt_ctx **out);
void bgt_destroy(bgt_ctx *ctx);
/* Text of the last error on this context (never NULL). */
const char *bgt_last_error(const bgt_ctx *ctx);

/* Tessellation lattice (Sec. 3.1 Eq. 1 evaluated at the nodes of Sec. 3.2's
 * tessellation): verts[3][VL][P], VL = (L+1)(L+2)/2, node m enumerating
 * (a, b) with a = 0..L outer, b = 0..L-a inner at (u, v, w) = (a/L, b/L,
 * 1-(a+b)/L).  Evaluated in FP64, stored as float32. */
bgt_status bgt_tessellate(bgt_ctx *ctx, const bgt_prims *prims, float *verts, void *stream);

/* Bytes of the caller-owned state buffer for a (prims, views) shape.  The
 * state holds everything the backward pass reads plus the forward pass's
 * scratch; its pair lists are sized by pair_factor and bpair_factor. */
bgt_status bgt_state_size(bgt_ctx *ctx, const bgt_prims *prims, const bgt_views *views,
                          size_t *bytes);

/* Byte offsets (host out[BGT_STATE_FIELDS]) of the state's sections, for
 * inspection and tests.  Order: counters, zbuf(u64), I_tri(i32), I_uv(f32x2),
 * pflags(u8), rec(f32x16), gkey(u64), T_final(f32), last(i32), verts,
 * g_count, g_start, g_cursor, b_count, b_start, b_cursor, g_keys(u64),
 * g_list(u32), b_keys(u64), b_list(u32), gslot(f32x9 per record and tile
 * slot), gpos(i32 per record and tile slot), t_end(i32 per tile),
 * gwide(f32x9 per record), dbound(f32x3 per pixel), brec64(f64x3), big_tris,
 * scan, end. */
#define BGT_STATE_FIELDS 29
bgt_status bgt_state_layout(bgt_ctx *ctx, const bgt_prims *prims, const bgt_views *views,
                            int64_t *offsets);

/* Forward pass over all views: images [sum W H][3] (overwritten). */
bgt_status bgt_render_fwd(bgt_ctx *ctx, const bgt_prims *prims, const bgt_views *views,
                          float *images, void *state, size_t state_bytes, void *stream);

/* Backward pass (Supplementary Sec. C with I_id, I_uv and B frozen).
 * `images` are the forward outputs of the same call's state; grad_images is
 * dl/dC in the same layout.  All gradient arrays are overwritten. */
bgt_status bgt_render_bwd(bgt_ctx *ctx, const bgt_prims *prims, const bgt_views *views,
                          const float *images, const float *grad_images, void *state,
                          size_t state_bytes, const bgt_grads *grads, void *stream);

/* Synchronizes `stream` and reads the state's counters (host out[10]):
 * [0] overflow flags (bit0 Gaussian pairs, bit1 boundary pairs, bit2 big
 * triangle queue) of this state's last forward pass together with those of
 * every forward pass on the context not yet reported, [1] Gaussian pairs,
 * [2] boundary pairs, [3] foreground pixels, [4] boundary pixels, [5] big
 * triangles (a bounding box over 256 pixels, or corners 2^17 pixels or more
 * apart on an axis), [6] tiles needing the global sort, [7] tiles whose boundary
 * list exceeded LDS, [8] tiles with more boundary runs (primitives) than
 * the forward's gamma* maps hold (their other runs are searched per pixel),
 * [9] reserved (0).  Returns BGT_E_OVERFLOW when any overflow flag is set
 * (and clears the context's record of it). */
bgt_status bgt_query(bgt_ctx *ctx, const void *state, size_t state_bytes, int64_t *counters,
                     void *stream);

/* ---- One training step around the renderer (Sec. 3.3) ----------------- */

/* Photometric loss of Eq. 9, L = (1 - lambda) L2 + lambda D-SSIM (the paper
 * uses lambda = 0.2), over the packed images of all views.  L2 is the mean
 * squared error over every pixel and channel; D-SSIM = 1 - SSIM, SSIM being
 * the mean structural similarity (Wang et al. 2004: 11x11 Gaussian window of
 * standard deviation 1.5, C1 = 0.01^2, C2 = 0.03^2) per channel and view,
 * with the window zero outside each view.  images and targets are
 * [sum W H][3] device arrays; loss (device, float[3]) receives L, L2 and SSIM;
 * grad_images (device, same layout as images, may be NULL) receives dL/dC,
 * overwritten.  `workspace` is caller-owned device memory of at least
 * bgt_loss_workspace_size bytes (three per-pixel maps and the partial sums).
 * Only views->n_views and views->wh are read.  Deterministic: the sums are
 * taken in a fixed order. */
bgt_status bgt_loss_workspace_size(const bgt_views *views, size_t *bytes);
bgt_status bgt_loss(bgt_ctx *ctx, const bgt_views *views, const float *images, const float *targets,
                    float lambda, float *loss, float *grad_images, void *workspace, size_t workspace_bytes,
                    void *stream);

/* bgt_loss without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, serving loops, harnesses that
 * forbid hipMalloc).  The workspace is a fixed 64 MiB device array inside the
 * library, one per GPU, held until the process ends; its address is looked up
 * when a context is created on that GPU.  Views whose
 * bgt_loss_workspace_size exceeds 64 MiB (about 1.86 M pixels in all) give
 * BGT_E_NOMEM before any work is enqueued.  The call allocates nothing.
 * Every call on one GPU shares the array: calls that overlap on a GPU (other
 * streams, other host threads) race on it; calls in order on one stream do
 * not.  Results are bit-identical to bgt_loss's. */
bgt_status bgt_loss_noalloc(bgt_ctx *ctx, const bgt_views *views, const float *images, const float *targets,
                            float lambda, float *loss, float *grad_images, void *stream);

/* Cotangent of an L1 loss scale * sum |C - target| over n values (images
 * and targets device arrays of n floats): grad = scale * sign(C - target),
 * 0 where they are equal.  The L1 loss of the benchmark workload, mean over
 * the 3 sum W H values, takes scale = 1 / n. */
bgt_status bgt_l1_cotangent(bgt_ctx *ctx, int64_t n, const float *images, const float *targets, float scale,
                            float *grad_images, void *stream);

/* One Adam update (Kingma and Ba 2015, Algorithm 1, with bias correction)
 * of up to BGT_MAX_ADAM_GROUPS parameter arrays, each with its own learning
 * rate: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), in FP64 with
 * float storage.  The paper does not name its optimiser; Adam is the one of
 * the 3DGS framework it builds on.  `groups` is a host array; every pointer in
 * it is device memory of n floats (param, m and v updated in place, grad
 * read).  `step` (device int32) holds the number of updates already taken:
 * this call uses t = *step + 1 and then stores t, so a captured graph can
 * replay it. */
#define BGT_MAX_ADAM_GROUPS 8
typedef struct {
    float *param;
    const float *grad;
    float *m, *v;
    int64_t n;
    float lr;
    int32_t reserved;
} bgt_adam_group;
bgt_status bgt_adam_step(bgt_ctx *ctx, const bgt_adam_group *groups, int32_t n_groups, float beta1,
                         float beta2, float eps, int32_t *step, void *stream);

/* ---- Splitting and pruning (Sec. 3.3; implementation details) ---------- */

/* Per-patch statistics, device arrays of P entries (views_seen: one), all
 * accumulated across calls until the caller clears them (zero fill). */
typedef struct {
    int32_t *views_seen;   /* [1] views rendered since the last clear */
    int32_t *vis_views;    /* views in which the patch wins at least one pixel */
    uint64_t *tex;         /* visibility texture: bit s set once flat sub-triangle s was seen */
    uint64_t *view_bits;   /* scratch of one call (left zero) */
    float *grad_sum;       /* sum over visible calls of the mean |dL/dp| of the control points */
    int32_t *grad_cnt;     /* number of those calls */
    float *edge_sum;       /* sum of the edge prior over the patch's pixels */
    int32_t *edge_cnt;     /* number of those pixels */
} bgt_prim_stats;

/* Thresholds of the implementation details (defaults in brackets). */
typedef struct {
    float tau_g;   /* split: mean position gradient above (0.0018) */
    float tau_b;   /* split: mean edge prior above (13.0) */
    float tau_v;   /* prune: visibility count ratio below (0.08) */
    float tau_r;   /* prune: visibility texture ratio below (0.4) */
    float tau_a;   /* prune: area below (3e-4) */
    float tau_s;   /* prune: aspect ratio above (10) */
} bgt_densify_config;
void bgt_default_densify_config(bgt_densify_config *cfg);

/* Adds one rendered batch of views to the statistics: for each view, the
 * patches that win a pixel of I_id and the flat sub-triangles seen (from the
 * forward pass's state of the same prims and views); with `targets` (the
 * training images, [sum W H][3], or NULL) the edge prior, the Sobel gradient
 * magnitude of their grey level on a 0..255 scale (0 on view borders),
 * summed over each patch's pixels; with `grads` (the backward pass's
 * output, or NULL) the mean |dL/dp| of each visible patch's control points.
 * The tessellation level must be at most 8 (L^2 <= 64 texels). */
bgt_status bgt_stats_accumulate(bgt_ctx *ctx, const bgt_prims *prims, const bgt_views *views,
                                const void *state, size_t state_bytes, const float *targets,
                                const bgt_grads *grads, const bgt_prim_stats *stats, void *stream);

/* Decision per patch (device action[P]: 0 keep, 1 split, 2 prune).  A patch
 * is pruned when its visibility count ratio is below tau_v, its visibility
 * texture ratio below tau_r, its area (four planar triangles through the
 * corner and edge-midpoint surface points) below tau_a, or its aspect ratio
 * (longest corner edge over the corner triangle's height on it) above
 * tau_s; otherwise split when its mean position gradient exceeds tau_g or
 * its mean edge prior exceeds tau_b.  dst_index[P] (device) receives each
 * patch's first slot in the rebuilt arrays and count[0] (device) their
 * length. */
bgt_status bgt_densify_plan(bgt_ctx *ctx, const bgt_prims *prims, const bgt_prim_stats *stats,
                            const bgt_densify_config *cfg, int32_t *action, int32_t *dst_index,
                            int32_t *count, void *stream);

/* Rebuilt parameter arrays (layouts as in bgt_prims, with dst_prims
 * patches): kept patches are copied, a split patch is replaced by its four
 * children cut at the edge midpoints (corner u, corner v, corner w, middle),
 * whose control and colour nets are blossoms of the parent's, so each child
 * reproduces its part of the parent exactly; the other attributes are
 * copied.  dst_prims must equal the count from bgt_densify_plan (slots at or
 * beyond it are not written).  dst holds device arrays written in full. */
bgt_status bgt_densify_apply(bgt_ctx *ctx, const bgt_prims *prims, const int32_t *action,
                             const int32_t *dst_index, int32_t dst_prims, const bgt_grads *dst,
                             void *stream);

/* Optional stage timing.  While enabled, the context records a pair of HIP
 * events around each stage it enqueues; bgt_stage_times synchronizes on the
 * last recorded event and returns (host ms[BGT_NUM_STAGES]) the duration of
 * the most recent launch of each stage, -1 for stages not launched since
 * profiling was enabled.  Keep profiling off while a stream is captured.
 * Stages: 0 tessellation + projection + raster, 1 sub-primitive generation,
 * 2 tile binning (scan, scatter, sort), 3 blend forward, 4 blend backward,
 * 5 parameter backward.  The clears of the gradient buffers are not timed. */
#define BGT_NUM_STAGES 6
bgt_status bgt_profile(bgt_ctx *ctx, int enable);
bgt_status bgt_stage_times(bgt_ctx *ctx, float *ms);

#ifdef __cplusplus
}
#endif
#endif /* BGT_H */
