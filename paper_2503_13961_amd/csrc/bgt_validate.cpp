// Host-only argument validation of the bgt C ABI.  No HIP calls: these
// functions run (and are tested) on machines without a GPU.
#include <math.h>
#include <stdint.h>

#include "../../include/bgt.h"

extern "C" {

void bgt_default_config(bgt_config *c) {
    if (!c) return;
    c->tess_level = 4;
    c->tile = 16;
    c->batch = 64;
    c->flags = 0;
    c->z_near = 0.2f;
    c->g_min = 1.0f / 32768.0f;
    c->t_min = 1.0f / 32768.0f;
    c->alpha_max = 0.99f;
    c->dilation = 0.3f;
    c->r_ref = 1e-2f;
    c->bg[0] = c->bg[1] = c->bg[2] = 0.0f;
    c->pair_factor = 4.0f;
    c->bpair_factor = 2.0f;
    c->lattice = 0;
}

void bgt_default_densify_config(bgt_densify_config *c) {
    if (!c) return;
    c->tau_g = 0.0018f;
    c->tau_b = 13.0f;
    c->tau_v = 0.08f;
    c->tau_r = 0.4f;
    c->tau_a = 3e-4f;
    c->tau_s = 10.0f;
}

bgt_status bgt_validate_config(const bgt_config *c) {
    if (!c) return BGT_E_INVALID;
    if (c->tess_level < 1 || c->tess_level > 8) return BGT_E_INVALID;
    if (c->tile != 8 && c->tile != 16 && c->tile != 32) return BGT_E_INVALID;
    if (c->batch != 32 && c->batch != 64 && c->batch != 128) return BGT_E_INVALID;
    if (c->batch > c->tile * c->tile) return BGT_E_INVALID;  // one loader thread per batch slot
    if ((c->flags & ~BGT_FLAG_NO_BOUNDARY) != 0) return BGT_E_INVALID;
    if (!(c->z_near > 0.0f) || !isfinite(c->z_near)) return BGT_E_INVALID;
    if (!(c->g_min > 0.0f && c->g_min < 1.0f)) return BGT_E_INVALID;
    if (!(c->t_min >= 0.0f && c->t_min < 1.0f)) return BGT_E_INVALID;
    if (!(c->alpha_max > 0.0f && c->alpha_max < 1.0f)) return BGT_E_INVALID;
    if (!(c->dilation >= 0.0f) || !isfinite(c->dilation)) return BGT_E_INVALID;
    if (!(c->r_ref > 0.0f) || !isfinite(c->r_ref)) return BGT_E_INVALID;
    for (int i = 0; i < 3; ++i)
        if (!isfinite(c->bg[i])) return BGT_E_INVALID;
    if (!(c->pair_factor > 0.0f && c->pair_factor <= 1024.0f)) return BGT_E_INVALID;
    if (!(c->bpair_factor > 0.0f && c->bpair_factor <= 1024.0f)) return BGT_E_INVALID;
    if (c->lattice != 0 && (c->lattice < 2 || c->lattice > 16)) return BGT_E_INVALID;
    return BGT_OK;
}

bgt_status bgt_validate_prims(const bgt_prims *p, const bgt_config *c) {
    if (!p || !c) return BGT_E_INVALID;
    if (p->degree < 1 || p->degree > BGT_MAX_DEGREE) return BGT_E_INVALID;
    if (p->num_prims < 1) return BGT_E_INVALID;
    if (p->attr_res < 1) return BGT_E_INVALID;
    if (p->attr_res != 1 && p->attr_res != 3) return BGT_E_UNSUPPORTED;
    if (p->sh_degree < 0) return BGT_E_INVALID;
    if (p->sh_degree > 3) return BGT_E_UNSUPPORTED;
    if (p->sh_degree > 0 && !p->sh) return BGT_E_INVALID;
    // per-view sub-triangle ids live in 24 bits of the z-buffer word
    const int64_t L2 = (int64_t)c->tess_level * c->tess_level;
    if ((int64_t)p->num_prims * L2 >= (int64_t)1 << 24) return BGT_E_INVALID;
    if (!p->ctrl || !p->color_ctrl || !p->log_scale || !p->quat || !p->opacity || !p->sharpness)
        return BGT_E_INVALID;
    return BGT_OK;
}

bgt_status bgt_validate_views(const bgt_views *v) {
    if (!v) return BGT_E_INVALID;
    if (v->n_views < 1 || v->n_views > BGT_MAX_VIEWS) return BGT_E_INVALID;
    if (!v->wh || !v->cams) return BGT_E_INVALID;
    int64_t total = 0;
    for (int i = 0; i < v->n_views; ++i) {
        const int64_t W = v->wh[2 * i], H = v->wh[2 * i + 1];
        // pixel coordinates are packed in int16 and per-view pixel ids in 24 bits
        if (W < 1 || H < 1 || W > 16384 || H > 16384) return BGT_E_INVALID;
        if (W * H >= (int64_t)1 << 24) return BGT_E_INVALID;
        total += W * H;
    }
    if (total >= (int64_t)1 << 30) return BGT_E_INVALID;
    return BGT_OK;
}

}  // extern "C"
