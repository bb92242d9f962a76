// Host side of the bgt C ABI: context, state layout and the launch sequence
// of the forward and backward passes.  Every entry point validates its
// arguments before enqueuing anything and never allocates device memory.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "bgt_internal.h"

struct bgt_ctx {
    bgt_config cfg;
    int device;
    std::string err;
    bool profiling = false;
    bool recorded[BGT_NUM_STAGES] = {};
    hipEvent_t ev0[BGT_NUM_STAGES] = {}, ev1[BGT_NUM_STAGES] = {};
    int last_stage = -1;
    // sticky overflow bits of the forward passes on this context, written by
    // the device into pinned host memory and cleared when reported
    unsigned long long *ovf_host = nullptr, *ovf_dev = nullptr;
};

namespace {

using namespace bgt;

enum Field {
    F_COUNTERS, F_ZBUF, F_ITRI, F_IUV, F_PFLAGS, F_REC, F_GKEY, F_TFINAL, F_LAST, F_VERTS, F_GCOUNT, F_GSTART,
    F_GCURSOR, F_BCOUNT, F_BSTART, F_BCURSOR, F_GKEYS, F_GLIST, F_BKEYS, F_BLIST, F_GSLOT, F_GPOS, F_TEND,
    F_GWIDE, F_DBOUND, F_BREC64, F_BIGTRI,
    F_SCAN, F_END
};
static_assert(F_END + 1 == BGT_STATE_FIELDS, "state field count");

struct Shape {
    ViewTable vt;
    Consts k;
    int64_t N, NT;
    int64_t NR;  // Gaussian records: the N pixel records, then the lattice Gaussians of every view
    int64_t off[BGT_STATE_FIELDS];
    int64_t wverts_off, patch_off;
};

bgt_status fail(bgt_ctx *ctx, bgt_status st, const char *msg) {
    if (ctx) ctx->err = msg;
    return st;
}

bgt_status hip_fail(bgt_ctx *ctx, hipError_t e, const char *where) {
    if (ctx) {
        ctx->err = std::string(where) + ": " + hipGetErrorString(e);
    }
    return BGT_E_HIP;
}

int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// Takes (and clears) the context's sticky overflow bits; no device wait: a
// pass that has not run yet is seen by a later call.
unsigned long long take_overflow(bgt_ctx *ctx) {
    if (!ctx->ovf_host || !__atomic_load_n(ctx->ovf_host, __ATOMIC_ACQUIRE)) return 0;
    return __atomic_exchange_n(ctx->ovf_host, 0ull, __ATOMIC_ACQ_REL);
}

bgt_status overflow_status(bgt_ctx *ctx, unsigned long long bits) {
    char msg[160];
    snprintf(msg, sizeof msg,
             "an earlier forward pass on this context exceeded a capacity (bits 0x%llx: 1 Gaussian pairs, "
             "2 boundary pairs, 4 big triangles); its outputs are incomplete: raise pair_factor/bpair_factor",
             bits);
    return fail(ctx, BGT_E_OVERFLOW, msg);
}

bgt_status make_shape(bgt_ctx *ctx, const bgt_prims *pr, const bgt_views *vw, Shape &sh) {
    bgt_status s;
    if ((s = bgt_validate_prims(pr, &ctx->cfg)) != BGT_OK) return fail(ctx, s, "invalid or unsupported prims");
    if ((s = bgt_validate_views(vw)) != BGT_OK) return fail(ctx, s, "invalid views");
    const bgt_config &c = ctx->cfg;
    memset(&sh, 0, sizeof(sh));
    Consts &k = sh.k;
    k.L = c.tess_level;
    k.L2 = k.L * k.L;
    k.VL = (k.L + 1) * (k.L + 2) / 2;
    k.tile = c.tile;
    k.degree = pr->degree;
    k.ncp = (pr->degree + 1) * (pr->degree + 2) / 2;
    k.P = pr->num_prims;
    k.T = pr->attr_res * (pr->attr_res + 1) / 2;
    k.K = (pr->sh_degree + 1) * (pr->sh_degree + 1) - 1;
    k.pdw = patch_dw(k.ncp, k.T, k.K);
    k.lat_level = c.lattice >= 2 ? k.L * (c.lattice - 1) : 0;
    k.NL = c.lattice >= 2 ? (k.lat_level + 1) * (k.lat_level + 2) / 2 : 0;
    k.batch = c.batch;
    k.flags = c.flags;
    k.z_near = c.z_near;
    k.g_min = c.g_min;
    k.t_min = c.t_min;
    k.alpha_max = c.alpha_max;
    k.dilation = c.dilation;
    k.r_ref = c.r_ref;
    for (int i = 0; i < 3; ++i) k.bg[i] = c.bg[i];
    const double k2 = 2.0 * log(1.0 / (double)c.g_min);
    k.kappa2 = (float)k2;
    k.kappa = sqrt(k2);
    ViewTable &vt = sh.vt;
    vt.n = vw->n_views;
    int64_t px = 0, tiles = 0, b8 = 0;
    for (int v = 0; v < vw->n_views; ++v) {
        ViewInfo &vi = vt.v[v];
        vi.W = vw->wh[2 * v];
        vi.H = vw->wh[2 * v + 1];
        vi.tiles_x = (vi.W + c.tile - 1) / c.tile;
        vi.tiles_y = (vi.H + c.tile - 1) / c.tile;
        vi.px_off = (int32_t)px;
        vi.tile_off = (int32_t)tiles;
        vi.b8_off = (int32_t)b8;
        vi.b8_x = (vi.W + 7) / 8;
        px += (int64_t)vi.W * vi.H;
        tiles += (int64_t)vi.tiles_x * vi.tiles_y;
        b8 += (int64_t)((vi.W + 7) / 8) * ((vi.H + 7) / 8);
    }
    vt.total_px = (int32_t)px;
    vt.total_tiles = (int32_t)tiles;
    vt.total_b8 = (int32_t)b8;
    sh.N = px;
    sh.NT = tiles;
    const int64_t lat_view = (int64_t)k.P * k.NL;
    for (int v = 0; v < vw->n_views; ++v)  // record ids within a view are the low 24 bits of the list keys
        if ((int64_t)vt.v[v].W * vt.v[v].H + lat_view >= ((int64_t)1 << 24))
            return fail(ctx, BGT_E_INVALID, "pixels plus lattice Gaussians of a view exceed 2^24");
    sh.NR = px + (int64_t)vw->n_views * lat_view;
    if (sh.NR >= ((int64_t)1 << 31)) return fail(ctx, BGT_E_INVALID, "Gaussian records exceed 2^31");
    const int64_t N = px, NT = tiles, NR = sh.NR;
    k.cap_g = (int64_t)ceil((double)c.pair_factor * (double)NR) + 1024;
    k.cap_b = (int64_t)ceil((double)c.bpair_factor * (double)N) + 1024;
    if (k.cap_g >= ((int64_t)1 << 31) || k.cap_b >= ((int64_t)1 << 31))
        return fail(ctx, BGT_E_INVALID, "pair capacity exceeds 2^31");
    k.cap_big = (int64_t)vt.n * k.L2 * k.P;
    const int64_t nb_scan = (NT + 1023) / 1024;
    int64_t o = 0;
    auto put = [&](int f, int64_t bytes) { sh.off[f] = o; o = align256(o + bytes); };
    put(F_COUNTERS, kCounterWords * 8);
    put(F_ZBUF, 8 * N);
    put(F_ITRI, 4 * N);
    put(F_IUV, 8 * N);
    put(F_PFLAGS, N);
    put(F_REC, 64 * NR);
    put(F_GKEY, 8 * NR);
    put(F_TFINAL, 4 * N);
    put(F_LAST, 4 * N);
    {
        const int64_t vbytes = (int64_t)sizeof(VertRec) * vt.n * k.VL * k.P;
        const int64_t wbytes = 24 * (int64_t)k.VL * k.P;
        sh.off[F_VERTS] = o;
        sh.wverts_off = align256(o + vbytes);
        sh.patch_off = align256(sh.wverts_off + wbytes);
        o = align256(sh.patch_off + 4 * (int64_t)k.pdw * k.P);
    }
    put(F_GCOUNT, 4 * NT);
    put(F_GSTART, 4 * NT);
    put(F_GCURSOR, 4 * NT);
    put(F_BCOUNT, 4 * NT);
    put(F_BSTART, 4 * NT);
    put(F_BCURSOR, 4 * NT);
    put(F_GKEYS, 8 * k.cap_g);
    put(F_GLIST, 4 * k.cap_g);
    put(F_BKEYS, 8 * k.cap_b);
    put(F_BLIST, 4 * k.cap_b);
    put(F_GSLOT, 4 * kSlotTiles * kSums * NR);
    put(F_GPOS, 4 * kSlotTiles * NR);
    put(F_TEND, 4 * NT);
    put(F_GWIDE, 4 * kSums * NR);
    put(F_DBOUND, 12 * N);
    put(F_BREC64, 24 * N);
    put(F_BIGTRI, 4 * k.cap_big);
    {
        sh.off[F_SCAN] = o;
        o = align256(o + 16 * nb_scan);
    }
    sh.off[F_END] = o;
    return BGT_OK;
}

StatePtrs state_ptrs(const Shape &sh, void *state) {
    char *b = (char *)state;
    StatePtrs p;
    p.counters = (int64_t *)(b + sh.off[F_COUNTERS]);
    p.zbuf = (unsigned long long *)(b + sh.off[F_ZBUF]);
    p.I_tri = (int32_t *)(b + sh.off[F_ITRI]);
    p.I_uv = (float2 *)(b + sh.off[F_IUV]);
    p.pflags = (uint8_t *)(b + sh.off[F_PFLAGS]);
    p.rec = (float4 *)(b + sh.off[F_REC]);
    p.gkey = (unsigned long long *)(b + sh.off[F_GKEY]);
    p.T_final = (float *)(b + sh.off[F_TFINAL]);
    p.last = (int32_t *)(b + sh.off[F_LAST]);
    p.verts = (VertRec *)(b + sh.off[F_VERTS]);
    p.wverts = (double *)(b + sh.wverts_off);
    p.patch = (float *)(b + sh.patch_off);
    p.g_count = (int32_t *)(b + sh.off[F_GCOUNT]);
    p.g_start = (int32_t *)(b + sh.off[F_GSTART]);
    p.g_cursor = (int32_t *)(b + sh.off[F_GCURSOR]);
    p.b_count = (int32_t *)(b + sh.off[F_BCOUNT]);
    p.b_start = (int32_t *)(b + sh.off[F_BSTART]);
    p.b_cursor = (int32_t *)(b + sh.off[F_BCURSOR]);
    p.g_keys = (unsigned long long *)(b + sh.off[F_GKEYS]);
    p.g_list = (uint32_t *)(b + sh.off[F_GLIST]);
    p.b_keys = (unsigned long long *)(b + sh.off[F_BKEYS]);
    p.b_list = (uint32_t *)(b + sh.off[F_BLIST]);
    p.n_rec = sh.NR;
    p.gslot = (float *)(b + sh.off[F_GSLOT]);
    p.gpos = (int32_t *)(b + sh.off[F_GPOS]);
    p.t_end = (int32_t *)(b + sh.off[F_TEND]);
    p.gwide = (float *)(b + sh.off[F_GWIDE]);
    p.dbound = (float *)(b + sh.off[F_DBOUND]);
    p.brec64 = (double *)(b + sh.off[F_BREC64]);
    p.big_tris = (int32_t *)(b + sh.off[F_BIGTRI]);
    p.scan_tmp = (int32_t *)(b + sh.off[F_SCAN]);
    return p;
}

PrimPtrs prim_ptrs(const bgt_prims *p) {
    PrimPtrs r;
    r.ctrl = p->ctrl;
    r.color = p->color_ctrl;
    r.log_scale = p->log_scale;
    r.quat = p->quat;
    r.opacity = p->opacity;
    r.sharp = p->sharpness;
    r.sh = p->sh_degree > 0 ? p->sh : nullptr;
    return r;
}

bgt_status use_device(bgt_ctx *ctx) {
    if (ctx->device < 0) return fail(ctx, BGT_E_INVALID, "host-only context cannot enqueue work");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipGetDevice");
    if (cur != ctx->device) {
        e = hipSetDevice(ctx->device);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
    }
    return BGT_OK;
}

// brackets one stage with the context's timing events when profiling is on
struct StageTimer {
    bgt_ctx *ctx;
    int stage;
    hipStream_t s;
    StageTimer(bgt_ctx *c, int st, hipStream_t str) : ctx(c), stage(st), s(str) {
        if (ctx->profiling) hipEventRecord(ctx->ev0[stage], s);
    }
    ~StageTimer() {
        if (ctx->profiling) {
            hipEventRecord(ctx->ev1[stage], s);
            ctx->recorded[stage] = true;
            ctx->last_stage = stage;
        }
    }
};

// the loss pass's tile table and workspace split (three float maps, then
// the per-workgroup partial sums)
bgt_status loss_table(const bgt_views *vw, float lambda, LossTable &lt, int64_t &maps_bytes, int64_t &ws_bytes) {
    if (!vw || vw->n_views < 1 || vw->n_views > BGT_MAX_VIEWS || !vw->wh) return BGT_E_INVALID;
    if (!(lambda >= 0.f && lambda <= 1.f)) return BGT_E_INVALID;
    memset(&lt, 0, sizeof(lt));
    lt.n = vw->n_views;
    int64_t px = 0, tiles = 0;
    for (int v = 0; v < vw->n_views; ++v) {
        const int W = vw->wh[2 * v], H = vw->wh[2 * v + 1];
        if (W < 1 || H < 1 || W > 16384 || H > 16384) return BGT_E_INVALID;
        int tx, nt;
        loss_tiles(W, H, &tx, &nt);
        lt.W[v] = W;
        lt.H[v] = H;
        lt.tiles_x[v] = tx;
        lt.tile_off[v] = (int32_t)tiles;
        lt.px_off[v] = (int32_t)px;
        px += (int64_t)W * H;
        tiles += nt;
        if (px >= ((int64_t)1 << 30)) return BGT_E_INVALID;
    }
    lt.tile_off[vw->n_views] = (int32_t)tiles;
    lt.total_tiles = (int32_t)tiles;
    lt.total_px = (int32_t)px;
    double sum = 0.0;
    for (int k = 0; k < 11; ++k) sum += (lt.taps[k] = exp(-(double)((k - 5) * (k - 5)) / (2.0 * 1.5 * 1.5)));
    for (int k = 0; k < 11; ++k) lt.taps[k] /= sum;
    lt.inv_n = 1.0 / (3.0 * (double)px);
    lt.lam = lambda;
    maps_bytes = align256(3 * 3 * px * (int64_t)sizeof(float));
    ws_bytes = maps_bytes + align256(2 * tiles * (int64_t)sizeof(double));
    return BGT_OK;
}

}  // namespace

namespace bgt {
int ctx_device(const bgt_ctx *ctx) { return ctx->device; }
bgt_status ctx_fail(bgt_ctx *ctx, bgt_status st, const char *msg) { return fail(ctx, st, msg); }
}  // namespace bgt

extern "C" {

bgt_status bgt_create(const bgt_config *cfg, int device, bgt_ctx **out) {
    if (!out) return BGT_E_INVALID;
    *out = nullptr;
    bgt_config c;
    if (cfg) c = *cfg; else bgt_default_config(&c);
    if (bgt_validate_config(&c) != BGT_OK) return BGT_E_INVALID;
    if (device != -1) {  // -1: host-only context (sizing and validation, no rendering)
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return BGT_E_INVALID;
    }
    bgt_ctx *ctx = new (std::nothrow) bgt_ctx;
    if (!ctx) return BGT_E_NOMEM;
    ctx->cfg = c;
    ctx->device = device;
    if (device >= 0) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || (cur != device && hipSetDevice(device) != hipSuccess) ||
            hipHostMalloc((void **)&ctx->ovf_host, sizeof(unsigned long long),
                          hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
            delete ctx;
            return BGT_E_HIP;
        }
        *ctx->ovf_host = 0;
        if (hipHostGetDevicePointer((void **)&ctx->ovf_dev, ctx->ovf_host, 0) != hipSuccess ||
            static_scratch_init(device) != hipSuccess) {  // the device address of bgt_loss_noalloc's workspace
            hipHostFree(ctx->ovf_host);
            delete ctx;
            return BGT_E_HIP;
        }
        if (cur >= 0 && cur != device) hipSetDevice(cur);
    }
    *out = ctx;
    return BGT_OK;
}

void bgt_destroy(bgt_ctx *ctx) {
    if (!ctx) return;
    for (int i = 0; i < BGT_NUM_STAGES; ++i) {
        if (ctx->ev0[i]) hipEventDestroy(ctx->ev0[i]);
        if (ctx->ev1[i]) hipEventDestroy(ctx->ev1[i]);
    }
    if (ctx->ovf_host) hipHostFree(ctx->ovf_host);
    delete ctx;
}

bgt_status bgt_profile(bgt_ctx *ctx, int enable) {
    if (!ctx) return BGT_E_INVALID;
    bgt_status s;
    if ((s = use_device(ctx)) != BGT_OK) return s;
    if (enable && !ctx->ev0[0]) {
        for (int i = 0; i < BGT_NUM_STAGES; ++i) {
            hipError_t e = hipEventCreate(&ctx->ev0[i]);
            if (e == hipSuccess) e = hipEventCreate(&ctx->ev1[i]);
            if (e != hipSuccess) return hip_fail(ctx, e, "hipEventCreate");
        }
    }
    ctx->profiling = enable != 0;
    for (int i = 0; i < BGT_NUM_STAGES; ++i) ctx->recorded[i] = false;
    ctx->last_stage = -1;
    return BGT_OK;
}

bgt_status bgt_stage_times(bgt_ctx *ctx, float *ms) {
    if (!ctx || !ms) return BGT_E_INVALID;
    bgt_status s;
    if ((s = use_device(ctx)) != BGT_OK) return s;
    if (ctx->last_stage >= 0) {
        hipError_t e = hipEventSynchronize(ctx->ev1[ctx->last_stage]);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventSynchronize");
    }
    for (int i = 0; i < BGT_NUM_STAGES; ++i) {
        ms[i] = -1.0f;
        if (ctx->recorded[i]) {
            hipError_t e = hipEventSynchronize(ctx->ev1[i]);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms[i], ctx->ev0[i], ctx->ev1[i]);
            if (e != hipSuccess) return hip_fail(ctx, e, "hipEventElapsedTime");
        }
    }
    return BGT_OK;
}

const char *bgt_last_error(const bgt_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

bgt_status bgt_tessellate(bgt_ctx *ctx, const bgt_prims *prims, float *verts, void *stream) {
    if (!ctx) return BGT_E_INVALID;
    bgt_status s = bgt_validate_prims(prims, &ctx->cfg);
    if (s != BGT_OK) return fail(ctx, s, "invalid or unsupported prims");
    if (!verts) return fail(ctx, BGT_E_INVALID, "verts is null");
    if ((s = use_device(ctx)) != BGT_OK) return s;
    Consts k;
    memset(&k, 0, sizeof(k));
    k.L = ctx->cfg.tess_level;
    k.L2 = k.L * k.L;
    k.VL = (k.L + 1) * (k.L + 2) / 2;
    k.degree = prims->degree;
    k.ncp = (prims->degree + 1) * (prims->degree + 2) / 2;
    k.P = prims->num_prims;
    hipError_t e = launch_tessellate(k, prim_ptrs(prims), nullptr, verts, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "tessellate");
    return BGT_OK;
}

bgt_status bgt_state_size(bgt_ctx *ctx, const bgt_prims *prims, const bgt_views *views, size_t *bytes) {
    if (!ctx || !bytes) return BGT_E_INVALID;
    Shape sh;
    bgt_status s = make_shape(ctx, prims, views, sh);
    if (s != BGT_OK) return s;
    *bytes = (size_t)sh.off[F_END];
    return BGT_OK;
}

bgt_status bgt_state_layout(bgt_ctx *ctx, const bgt_prims *prims, const bgt_views *views, int64_t *offsets) {
    if (!ctx || !offsets) return BGT_E_INVALID;
    Shape sh;
    bgt_status s = make_shape(ctx, prims, views, sh);
    if (s != BGT_OK) return s;
    for (int i = 0; i < BGT_STATE_FIELDS; ++i) offsets[i] = sh.off[i];
    return BGT_OK;
}

bgt_status bgt_render_fwd(bgt_ctx *ctx, const bgt_prims *prims, const bgt_views *views, float *images,
                          void *state, size_t state_bytes, void *stream) {
    if (!ctx) return BGT_E_INVALID;
    Shape sh;
    bgt_status s = make_shape(ctx, prims, views, sh);
    if (s != BGT_OK) return s;
    if (!images || !state) return fail(ctx, BGT_E_INVALID, "images or state is null");
    if (state_bytes < (size_t)sh.off[F_END]) return fail(ctx, BGT_E_NOMEM, "state buffer too small");
    if (const unsigned long long ov = take_overflow(ctx)) return overflow_status(ctx, ov);
    if ((s = use_device(ctx)) != BGT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const StatePtrs sp = state_ptrs(sh, state);
    const PrimPtrs pp = prim_ptrs(prims);
    hipError_t e;
    {  // counters, z-buffer and tile counts start at zero
        ZeroTable z;
        z.add(sp.counters, 2 * (int64_t)kCounterWords);
        z.add(sp.zbuf, 2 * (int64_t)sh.N);
        z.add(sp.g_count, sh.NT);
        z.add(sp.b_count, sh.NT);
        if ((e = launch_zero(z, st)) != hipSuccess) return hip_fail(ctx, e, "clear");
    }
    {
        StageTimer tm(ctx, 0, st);
        if ((e = launch_raster(sh.k, sh.vt, pp, views->cams, sp, st)) != hipSuccess) return hip_fail(ctx, e, "raster");
    }
    {
        StageTimer tm(ctx, 1, st);
        if ((e = launch_gen(sh.k, sh.vt, pp, views->cams, sp, st)) != hipSuccess) return hip_fail(ctx, e, "generation");
    }
    {
        StageTimer tm(ctx, 2, st);
        if ((e = launch_binning(sh.k, sh.vt, sp, st)) != hipSuccess) return hip_fail(ctx, e, "binning");
    }
    {
        StageTimer tm(ctx, 3, st);
        if ((e = launch_blend_fwd(sh.k, sh.vt, sp, images, st)) != hipSuccess) return hip_fail(ctx, e, "blend_fwd");
    }
    if (ctx->ovf_dev && (e = launch_note_overflow(sp, ctx->ovf_dev, st)) != hipSuccess)
        return hip_fail(ctx, e, "overflow note");
    return BGT_OK;
}

bgt_status bgt_render_bwd(bgt_ctx *ctx, const bgt_prims *prims, const bgt_views *views, const float *images,
                          const float *grad_images, void *state, size_t state_bytes, const bgt_grads *grads,
                          void *stream) {
    if (!ctx) return BGT_E_INVALID;
    Shape sh;
    bgt_status s = make_shape(ctx, prims, views, sh);
    if (s != BGT_OK) return s;
    if (!images || !grad_images || !state || !grads) return fail(ctx, BGT_E_INVALID, "null pointer argument");
    if (!grads->ctrl || !grads->color_ctrl || !grads->log_scale || !grads->quat || !grads->opacity ||
        !grads->sharpness)
        return fail(ctx, BGT_E_INVALID, "null gradient array");
    if (state_bytes < (size_t)sh.off[F_END]) return fail(ctx, BGT_E_NOMEM, "state buffer too small");
    if (const unsigned long long ov = take_overflow(ctx)) return overflow_status(ctx, ov);
    if ((s = use_device(ctx)) != BGT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const StatePtrs sp = state_ptrs(sh, state);
    const PrimPtrs pp = prim_ptrs(prims);
    GradPtrs gp;
    gp.ctrl = grads->ctrl;
    gp.color = grads->color_ctrl;
    gp.log_scale = grads->log_scale;
    gp.quat = grads->quat;
    gp.opacity = grads->opacity;
    gp.sharp = grads->sharpness;
    gp.sh = grads->sh;
    const Consts &k = sh.k;
    if (k.K > 0 && !gp.sh) return fail(ctx, BGT_E_INVALID, "null SH gradient array");
    hipError_t e = hipSuccess;
    const int64_t nc = 3LL * k.ncp * k.P;
    {  // the gradient arrays are sums: they start at zero
        ZeroTable z;
        if (k.K > 0) z.add(gp.sh, 3LL * k.K * k.P);
        z.add(gp.ctrl, nc);
        z.add(gp.color, nc);
        z.add(gp.log_scale, 3LL * k.T * k.P);
        z.add(gp.quat, 4LL * k.T * k.P);
        z.add(gp.opacity, k.P);
        z.add(gp.sharp, k.P);
        if ((e = launch_zero(z, st)) != hipSuccess) return hip_fail(ctx, e, "clear");
    }
    {
        StageTimer tm(ctx, 4, st);
        if ((e = launch_blend_bwd(k, sh.vt, sp, images, grad_images, st)) != hipSuccess) return hip_fail(ctx, e, "blend_bwd");
    }
    {
        StageTimer tm(ctx, 5, st);
        if ((e = launch_param_bwd(k, sh.vt, pp, views->cams, sp, gp, st)) != hipSuccess) return hip_fail(ctx, e, "param_bwd");
    }
    return BGT_OK;
}

bgt_status bgt_stats_accumulate(bgt_ctx *ctx, const bgt_prims *prims, const bgt_views *views,
                                const void *state, size_t state_bytes, const float *targets,
                                const bgt_grads *grads, const bgt_prim_stats *stats, void *stream) {
    if (!ctx) return BGT_E_INVALID;
    Shape sh;
    bgt_status s = make_shape(ctx, prims, views, sh);
    if (s != BGT_OK) return s;
    if (!state || !stats) return fail(ctx, BGT_E_INVALID, "null pointer argument");
    if (!stats->views_seen || !stats->vis_views || !stats->tex || !stats->view_bits || !stats->grad_sum ||
        !stats->grad_cnt || !stats->edge_sum || !stats->edge_cnt)
        return fail(ctx, BGT_E_INVALID, "null statistics array");
    if (grads && !grads->ctrl) return fail(ctx, BGT_E_INVALID, "null control-point gradient");
    if (sh.k.L2 > 64) return fail(ctx, BGT_E_UNSUPPORTED, "visibility texture needs L^2 <= 64");
    if (state_bytes < (size_t)sh.off[F_END]) return fail(ctx, BGT_E_NOMEM, "state buffer too small");
    if ((s = use_device(ctx)) != BGT_OK) return s;
    const StatePtrs stp = state_ptrs(sh, const_cast<void *>(state));
    StatsPtrs sp;
    sp.views_seen = stats->views_seen;
    sp.vis_views = stats->vis_views;
    sp.tex = (unsigned long long *)stats->tex;
    sp.view_bits = (unsigned long long *)stats->view_bits;
    sp.grad_sum = stats->grad_sum;
    sp.grad_cnt = stats->grad_cnt;
    sp.edge_sum = stats->edge_sum;
    sp.edge_cnt = stats->edge_cnt;
    hipError_t e = launch_stats(sh.k, sh.vt, stp.I_tri, targets, grads ? grads->ctrl : nullptr, sp,
                                (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "stats");
    return BGT_OK;
}

bgt_status bgt_densify_plan(bgt_ctx *ctx, const bgt_prims *prims, const bgt_prim_stats *stats,
                            const bgt_densify_config *cfg, int32_t *action, int32_t *dst_index,
                            int32_t *count, void *stream) {
    if (!ctx) return BGT_E_INVALID;
    bgt_status s = bgt_validate_prims(prims, &ctx->cfg);
    if (s != BGT_OK) return fail(ctx, s, "invalid or unsupported prims");
    if (!stats || !cfg || !action || !dst_index || !count) return fail(ctx, BGT_E_INVALID, "null pointer argument");
    if (!stats->views_seen || !stats->vis_views || !stats->tex || !stats->grad_sum || !stats->grad_cnt ||
        !stats->edge_sum || !stats->edge_cnt)
        return fail(ctx, BGT_E_INVALID, "null statistics array");
    const float t[6] = {cfg->tau_g, cfg->tau_b, cfg->tau_v, cfg->tau_r, cfg->tau_a, cfg->tau_s};
    for (float x : t)
        if (!isfinite(x)) return fail(ctx, BGT_E_INVALID, "thresholds must be finite");
    if (ctx->cfg.tess_level > 8) return fail(ctx, BGT_E_UNSUPPORTED, "visibility texture needs L^2 <= 64");
    if ((s = use_device(ctx)) != BGT_OK) return s;
    Consts k;
    memset(&k, 0, sizeof(k));
    k.L = ctx->cfg.tess_level;
    k.L2 = k.L * k.L;
    k.degree = prims->degree;
    k.ncp = (prims->degree + 1) * (prims->degree + 2) / 2;
    k.P = prims->num_prims;
    StatsPtrs sp;
    sp.views_seen = stats->views_seen;
    sp.vis_views = stats->vis_views;
    sp.tex = (unsigned long long *)stats->tex;
    sp.view_bits = (unsigned long long *)stats->view_bits;
    sp.grad_sum = stats->grad_sum;
    sp.grad_cnt = stats->grad_cnt;
    sp.edge_sum = stats->edge_sum;
    sp.edge_cnt = stats->edge_cnt;
    const DensifyRule rule = {cfg->tau_g, cfg->tau_b, cfg->tau_v, cfg->tau_r, cfg->tau_a, cfg->tau_s};
    hipError_t e = launch_plan(k, prims->ctrl, sp, rule, action, dst_index, count, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "densify plan");
    return BGT_OK;
}

bgt_status bgt_densify_apply(bgt_ctx *ctx, const bgt_prims *prims, const int32_t *action,
                             const int32_t *dst_index, int32_t dst_prims, const bgt_grads *dst,
                             void *stream) {
    if (!ctx) return BGT_E_INVALID;
    bgt_status s = bgt_validate_prims(prims, &ctx->cfg);
    if (s != BGT_OK) return fail(ctx, s, "invalid or unsupported prims");
    if (!action || !dst_index || !dst) return fail(ctx, BGT_E_INVALID, "null pointer argument");
    if (dst_prims < 0 || (int64_t)dst_prims > 4 * (int64_t)prims->num_prims)
        return fail(ctx, BGT_E_INVALID, "dst_prims outside [0, 4 P]");
    if (dst_prims > 0 && (!dst->ctrl || !dst->color_ctrl || !dst->log_scale || !dst->quat || !dst->opacity ||
                          !dst->sharpness))
        return fail(ctx, BGT_E_INVALID, "null output array");
    if ((s = use_device(ctx)) != BGT_OK) return s;
    if (dst_prims == 0) return BGT_OK;
    Consts k;
    memset(&k, 0, sizeof(k));
    k.degree = prims->degree;
    k.ncp = (prims->degree + 1) * (prims->degree + 2) / 2;
    k.P = prims->num_prims;
    k.T = prims->attr_res * (prims->attr_res + 1) / 2;
    k.K = (prims->sh_degree + 1) * (prims->sh_degree + 1) - 1;
    if (k.K > 0 && !dst->sh) return fail(ctx, BGT_E_INVALID, "null SH output array");
    GradPtrs gp;
    gp.ctrl = dst->ctrl;
    gp.color = dst->color_ctrl;
    gp.log_scale = dst->log_scale;
    gp.quat = dst->quat;
    gp.opacity = dst->opacity;
    gp.sharp = dst->sharpness;
    gp.sh = dst->sh;
    hipError_t e = launch_apply(k, prim_ptrs(prims), action, dst_index, dst_prims, gp, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "densify apply");
    return BGT_OK;
}

bgt_status bgt_loss_workspace_size(const bgt_views *views, size_t *bytes) {
    if (!bytes) return BGT_E_INVALID;
    LossTable lt;
    int64_t maps, ws;
    bgt_status s = loss_table(views, 0.f, lt, maps, ws);
    if (s != BGT_OK) return s;
    *bytes = (size_t)ws;
    return BGT_OK;
}

bgt_status bgt_loss(bgt_ctx *ctx, const bgt_views *views, const float *images, const float *targets,
                    float lambda, float *loss, float *grad_images, void *workspace, size_t workspace_bytes,
                    void *stream) {
    if (!ctx) return BGT_E_INVALID;
    LossTable lt;
    int64_t maps, ws;
    bgt_status s = loss_table(views, lambda, lt, maps, ws);
    if (s != BGT_OK) return fail(ctx, s, "invalid views or lambda outside [0, 1]");
    if (!images || !targets || !loss || !workspace) return fail(ctx, BGT_E_INVALID, "null buffer");
    if ((int64_t)workspace_bytes < ws) return fail(ctx, BGT_E_NOMEM, "loss workspace too small");
    if ((s = use_device(ctx)) != BGT_OK) return s;
    char *w = (char *)workspace;
    hipError_t e = launch_loss(lt, images, targets, loss, grad_images, (float *)w, (double *)(w + maps),
                               (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "loss");
    return BGT_OK;
}

bgt_status bgt_l1_cotangent(bgt_ctx *ctx, int64_t n, const float *images, const float *targets, float scale,
                            float *grad_images, void *stream) {
    if (!ctx) return BGT_E_INVALID;
    if (n < 0 || (n > 0 && (!images || !targets || !grad_images)) || !isfinite(scale))
        return fail(ctx, BGT_E_INVALID, "bad size, null buffer or non-finite scale");
    bgt_status s;
    if ((s = use_device(ctx)) != BGT_OK) return s;
    hipError_t e = launch_l1(n, images, targets, scale, grad_images, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "l1 cotangent");
    return BGT_OK;
}

bgt_status bgt_adam_step(bgt_ctx *ctx, const bgt_adam_group *groups, int32_t n_groups, float beta1,
                         float beta2, float eps, int32_t *step, void *stream) {
    if (!ctx) return BGT_E_INVALID;
    if (n_groups < 0 || n_groups > BGT_MAX_ADAM_GROUPS || (n_groups > 0 && !groups) || !step)
        return fail(ctx, BGT_E_INVALID, "bad group list or step counter");
    if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f) || isinf(eps))
        return fail(ctx, BGT_E_INVALID, "betas must lie in [0, 1) and eps be finite and >= 0");
    AdamTable at;
    memset(&at, 0, sizeof(at));
    at.n = n_groups;
    for (int g = 0; g < n_groups; ++g) {
        const bgt_adam_group &G = groups[g];
        if (G.n < 0 || !isfinite(G.lr)) return fail(ctx, BGT_E_INVALID, "bad group size or learning rate");
        if (G.n > 0 && (!G.param || !G.grad || !G.m || !G.v)) return fail(ctx, BGT_E_INVALID, "null group array");
        at.off[g + 1] = at.off[g] + G.n;
        at.param[g] = G.param;
        at.grad[g] = G.grad;
        at.m[g] = G.m;
        at.v[g] = G.v;
        at.lr[g] = G.lr;
    }
    bgt_status s;
    if ((s = use_device(ctx)) != BGT_OK) return s;
    hipError_t e = launch_adam(at, beta1, beta2, eps, step, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "adam");
    return BGT_OK;
}

bgt_status bgt_query(bgt_ctx *ctx, const void *state, size_t state_bytes, int64_t *counters, void *stream) {
    if (!ctx || !state || !counters || state_bytes < (size_t)(kCounterWords * 8)) return BGT_E_INVALID;
    bgt_status s;
    if ((s = use_device(ctx)) != BGT_OK) return s;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
    int64_t c[kCounterWords];
    e = hipMemcpy(c, state, sizeof(c), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpy");
    int64_t fg = 0, nb = 0;
    for (int i = 0; i < kStripes; ++i) {
        fg += c[C_NUM + i * kStripeStride];
        nb += c[C_NUM + i * kStripeStride + 1];
    }
    counters[0] = c[C_OVERFLOW];
    counters[1] = c[C_GPAIRS];
    counters[2] = c[C_BPAIRS];
    counters[3] = fg;
    counters[4] = nb;
    counters[5] = c[C_BIGTRI];
    counters[6] = c[C_BIGSORT];
    counters[7] = c[C_BIGBLIST];
    counters[8] = c[C_MANYRUNS];
    counters[9] = 0;
    // this state's last pass, and any pass on the context since the last report
    const unsigned long long ov = (unsigned long long)c[C_OVERFLOW] | take_overflow(ctx);
    counters[0] = (int64_t)ov;
    if (ov) return overflow_status(ctx, ov);
    return BGT_OK;
}

}  // extern "C"
