/*
 * bgt_oracle.c -- plain, slow CPU reference of the BG-Triangle rendering path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP implementation.
 *
 * Precision: every continuous quantity is FP64.  The inputs are the float32
 * arrays of the scene (promoted to double on read).
 *
 * Paper: "BG-Triangle: Bezier Gaussian Triangle for 3D Vectorization and
 * Rendering" (CVPR 2025).  Each stage names the passage it follows:
 *   Sec. 3.1, Eq. 1-2   Bezier triangle / Bernstein basis
 *   Sec. 3.2 (Tessellation and Rasterization)  flat triangles, depth test,
 *                       I_uv / I_id maps, boundary set B
 *   Sec. 3.2 (Sub-Primitive Generation) Eq. 3-5  one Gaussian per foreground
 *                       pixel, colour from colour control points
 *   Sec. 3.2 (Discontinuity-Aware Alpha Blending) Eq. 6-8  boundary
 *                       Gaussians of scale r_b, radius sigma_i, w(q), alpha
 *   Sec. 3.2 (Rendering Acceleration)  tiles, per-tile boundary lists
 *                       sorted by primitive ID
 *   Supplementary Sec. C (Backward Derivative)  dl/dc, dl/dalpha, dl/dw,
 *                       dl/db, gamma', dl/dp_ijk
 *
 * Readings taken where the paper is silent (all listed in the design notes):
 *   - tessellation level L, lattice/sub-triangle numbering, pinhole camera
 *     with pixel centres at +0.5, near cull of sub-triangles, two-sided
 *     raster, vertices snapped to 1/256 px with round-half-even, top-left
 *     edge ownership, depth test on 1/z interpolated affinely in screen
 *     space (key truncated to its 40 high bits, tie -> lower triangle id),
 *     perspective-correct barycentrics from the unsnapped projection;
 *   - B uses the 4-neighbourhood, background counts as a different id,
 *     off-image neighbours are ignored;
 *   - w's search for b_i is restricted to boundary points of the Gaussian's
 *     own primitive g (case 1 of Eq. 6 read as "b_i must belong to g"); no
 *     such point within range gives gamma* = 1;
 *   - sigma_i = 3 sqrt(lambda_max) of the projected isotropic boundary
 *     Gaussian (scale r_b = r_ref / sharpness_g) plus the 0.3 px^2 low-pass;
 *   - 2-D covariance by the EWA projection with the 0.3 px^2 low-pass,
 *     support d^T Q d <= 2 ln(1/g_min), alpha = min(alpha_max, o w G),
 *     stop after compositing once T < T_min, background colour bg;
 *   - Gaussians sorted front to back by camera-space z of S_q (key truncated
 *     to its 40 high bits, tie -> raster order);
 *   - I_id, I_uv and B are frozen in the backward pass.
 */
#include <math.h>

/* boundary distances below this many pixels are the cone point of |q - b| */
#define D_KINK 1e-6
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOMEM 2

/* ------------------------------------------------------------------ types */

typedef struct {
    int degree, num_prims, attr_res;
    const float *ctrl, *color_ctrl, *log_scale, *quat, *opacity, *sharpness;
    int sh_degree;       /* bands 1..sh_degree of view-dependent colour (0: none) */
    const float *sh;     /* [3][K][P], K = (sh_degree+1)^2 - 1 */
} orc_scene;

typedef struct {
    int L, tile;
    double z_near, g_min, t_min, alpha_max, dilation, r_ref;
    double bg[3];
    int no_boundary;     /* the ablation variant without blending coefficients */
    int lattice;         /* 0: one Gaussian per foreground pixel (Sec. 3.2); m >= 2: instead a
                            lattice of m Gaussians per flat sub-triangle edge on every patch */
    int exact_keys;      /* 1: depth test and Gaussian order on the untruncated FP64 depths
                            (only to show what the 40-bit truncation changes) */
} orc_config;

/* per-pixel Gaussian record (doubles) */
enum {
    GR_MUX, GR_MUY, GR_QA, GR_QB, GR_QC, GR_CR, GR_CG, GR_CB, GR_DEPTH,
    GR_SIGMA, GR_SA, GR_SB, GR_SC, GR_PRIM, GR_RX, GR_RY,
    GR_SX, GR_SY, GR_SZ, GR_TX, GR_TY, GR_TZ, GR_N
};

typedef struct {
    orc_scene sc;
    orc_config cfg;
    double cam[16];
    int W, H, ncp, L2;
    int tiles_x, tiles_y, ntiles;
    double kappa2;
    int32_t *I_tri;      /* [H*W] sub-triangle id, -1 background */
    uint64_t *zkey;      /* [H*W] the winner's depth-key bits (truncated unless exact_keys) */
    double *I_uv;        /* [H*W][2] */
    uint8_t *is_b;       /* [H*W] boundary flag (and Gaussian valid) */
    uint8_t *valid;      /* [H*W + nlat] record is a rendered Gaussian */
    uint8_t *has_rec;    /* [H*W] the pixel's record exists (S_q in front of z_near) */
    int nlat, lat_level; /* lattice Gaussians per frame (P NL) and the lattice level */
    double *rec;         /* [H*W + nlat][GR_N]: pixel records, then lattice records */
    int32_t *g_start;    /* [ntiles+1] */
    int32_t *g_list;     /* pixel index of each Gaussian pair, sorted per tile */
    int32_t *b_start;    /* [ntiles+1] */
    int32_t *b_list;     /* pixel index of each boundary pair, sorted per tile */
} orc_frame;

static int ncp_of(int n) { return (n + 1) * (n + 2) / 2; }

/* ------------------------------------------------ Sec. 3.1, Eq. 1 and Eq. 2 */

static double factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

static double ipow(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

/* Bernstein polynomial B^n_ijk(u,v,w) = n!/(i!j!k!) u^i v^j w^k (Eq. 2),
 * listed in the order of Eq. 1's double sum: i = 0..n, j = 0..n-i. */
void orc_bernstein(int n, double u, double v, double w, double *B) {
    int idx = 0;
    for (int i = 0; i <= n; ++i)
        for (int j = 0; j <= n - i; ++j) {
            int k = n - i - j;
            B[idx++] = factorial(n) / (factorial(i) * factorial(j) * factorial(k)) *
                       ipow(u, i) * ipow(v, j) * ipow(w, k);
        }
}

/* S(u,v,w) = sum_ijk B^n_ijk p_ijk (Eq. 1); cp is [ncp][3]. */
void orc_surface(int n, const double *cp, double u, double v, double w, double *out) {
    double B[64];
    orc_bernstein(n, u, v, w, B);
    out[0] = out[1] = out[2] = 0.0;
    for (int c = 0; c < ncp_of(n); ++c)
        for (int d = 0; d < 3; ++d) out[d] += B[c] * cp[3 * c + d];
}

/* control points of primitive p, channel-interleaved: out[ncp][3] */
static void prim_points(const float *soa, int ncp, int P, int p, double *out) {
    for (int c = 0; c < ncp; ++c)
        for (int d = 0; d < 3; ++d) out[3 * c + d] = (double)soa[((size_t)d * ncp + c) * P + p];
}

/* ------------------------------------------------ Sec. 3.2 tessellation */

/* lattice node (a,b), a = 0..L outer, b = 0..L-a inner */
static int lattice_index(int L, int a, int b) { return a * (L + 1) - a * (a - 1) / 2 + b; }

/* the three lattice nodes of flat sub-triangle s: "up" triangles
 * (a,b),(a+1,b),(a,b+1) for a+b <= L-1 first, then "down" triangles
 * (a+1,b),(a+1,b+1),(a,b+1) for a+b <= L-2. */
static void subtri_nodes(int L, int s, int na[3], int nb[3]) {
    int up = L * (L + 1) / 2;
    int cnt = 0;
    if (s < up) {
        for (int a = 0; a < L; ++a)
            for (int b = 0; b < L - a; ++b, ++cnt)
                if (cnt == s) {
                    na[0] = a; nb[0] = b; na[1] = a + 1; nb[1] = b; na[2] = a; nb[2] = b + 1;
                    return;
                }
    }
    s -= up;
    cnt = 0;
    for (int a = 0; a < L - 1; ++a)
        for (int b = 0; b < L - 1 - a; ++b, ++cnt)
            if (cnt == s) {
                na[0] = a + 1; nb[0] = b; na[1] = a + 1; nb[1] = b + 1; na[2] = a; nb[2] = b + 1;
                return;
            }
}

/* world-space lattice vertices of every primitive, [3][VL][P] */
int orc_tessellate(const orc_scene *sc, int L, double *verts) {
    if (!sc || !verts || L < 1 || sc->degree < 1 || sc->degree > 5) return ORC_EINVAL;
    int n = sc->degree, ncp = ncp_of(n), P = sc->num_prims;
    int VL = (L + 1) * (L + 2) / 2;
    double cp[64 * 3];
    for (int p = 0; p < P; ++p) {
        prim_points(sc->ctrl, ncp, P, p, cp);
        for (int a = 0; a <= L; ++a)
            for (int b = 0; b <= L - a; ++b) {
                double S[3];
                orc_surface(n, cp, (double)a / L, (double)b / L, (double)(L - a - b) / L, S);
                int vi = lattice_index(L, a, b);
                for (int d = 0; d < 3; ++d) verts[((size_t)d * VL + vi) * P + p] = S[d];
            }
    }
    return ORC_OK;
}

/* ------------------------------------------------ pinhole camera */

static void cam_apply(const double *cam, const double *X, double *t) {
    const double *R = cam;
    for (int r = 0; r < 3; ++r) t[r] = R[3 * r] * X[0] + R[3 * r + 1] * X[1] + R[3 * r + 2] * X[2] + cam[9 + r];
}

/* ------------------------------------------------ Sec. 3.2 rasterization */

typedef struct {
    int ok;
    double x, y, iz;   /* unsnapped projection, 1/z */
    int64_t X, Y;      /* 1/256 px fixed point */
    double u, v;       /* lattice (Bezier-domain) coordinates */
} rvert;

static int64_t floor_div256(int64_t a) { return a >= 0 ? a / 256 : -((-a + 255) / 256); }
static int64_t ceil_div256(int64_t a) { return -floor_div256(-a); }

/* edge function of directed edge a->b at point p (positive on one side) */
static int64_t edge_i(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t px, int64_t py) {
    return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}

/* Top-left ownership of a directed edge: exactly one of a->b and b->a owns
 * the points lying on it, so a consistently wound mesh is watertight. */
static int edge_owned(int64_t dx, int64_t dy) { return dy > 0 || (dy == 0 && dx < 0); }

static void rasterize(orc_frame *f) {
    int L = f->cfg.L, P = f->sc.num_prims, n = f->sc.degree, ncp = f->ncp;
    int VL = (L + 1) * (L + 2) / 2;
    size_t npx = (size_t)f->W * f->H;
    uint64_t *zbuf = (uint64_t *)calloc(npx, sizeof(uint64_t));
    /* exact_keys: the full FP64 key and the winning id beside it */
    uint64_t *zfull = f->cfg.exact_keys ? (uint64_t *)calloc(npx, sizeof(uint64_t)) : NULL;
    uint32_t *ztri = f->cfg.exact_keys ? (uint32_t *)calloc(npx, sizeof(uint32_t)) : NULL;
    rvert *rv = (rvert *)malloc(sizeof(rvert) * VL);
    double cp[64 * 3];
    const double lim = 1048576.0; /* 2^20 px */
    for (int p = 0; p < P; ++p) {
        prim_points(f->sc.ctrl, ncp, P, p, cp);
        for (int a = 0; a <= L; ++a)
            for (int b = 0; b <= L - a; ++b) {
                rvert *r = &rv[lattice_index(L, a, b)];
                double S[3], t[3];
                orc_surface(n, cp, (double)a / L, (double)b / L, (double)(L - a - b) / L, S);
                cam_apply(f->cam, S, t);
                r->u = (double)a / L;
                r->v = (double)b / L;
                r->ok = t[2] > f->cfg.z_near;
                if (!r->ok) continue;
                r->x = f->cam[12] * t[0] / t[2] + f->cam[14];
                r->y = f->cam[13] * t[1] / t[2] + f->cam[15];
                r->iz = 1.0 / t[2];
                if (!(fabs(r->x) < lim && fabs(r->y) < lim)) { r->ok = 0; continue; }
                r->X = (int64_t)rint(r->x * 256.0);
                r->Y = (int64_t)rint(r->y * 256.0);
            }
        for (int s = 0; s < f->L2; ++s) {
            int na[3], nb[3];
            subtri_nodes(L, s, na, nb);
            const rvert *v[3];
            int okall = 1;
            for (int k = 0; k < 3; ++k) {
                v[k] = &rv[lattice_index(L, na[k], nb[k])];
                okall &= v[k]->ok;
            }
            if (!okall) continue; /* near-plane cull: any vertex at z <= z_near */
            int64_t A = edge_i(v[0]->X, v[0]->Y, v[1]->X, v[1]->Y, v[2]->X, v[2]->Y);
            if (A == 0) continue;
            if (A < 0) { const rvert *tmp = v[1]; v[1] = v[2]; v[2] = tmp; A = -A; }
            int64_t minX = v[0]->X, maxX = v[0]->X, minY = v[0]->Y, maxY = v[0]->Y;
            for (int k = 1; k < 3; ++k) {
                if (v[k]->X < minX) minX = v[k]->X;
                if (v[k]->X > maxX) maxX = v[k]->X;
                if (v[k]->Y < minY) minY = v[k]->Y;
                if (v[k]->Y > maxY) maxY = v[k]->Y;
            }
            int64_t i0 = ceil_div256(minX - 128), i1 = floor_div256(maxX - 128);
            int64_t j0 = ceil_div256(minY - 128), j1 = floor_div256(maxY - 128);
            if (i0 < 0) i0 = 0;
            if (j0 < 0) j0 = 0;
            if (i1 > f->W - 1) i1 = f->W - 1;
            if (j1 > f->H - 1) j1 = f->H - 1;
            int own0 = edge_owned(v[2]->X - v[1]->X, v[2]->Y - v[1]->Y);
            int own1 = edge_owned(v[0]->X - v[2]->X, v[0]->Y - v[2]->Y);
            int own2 = edge_owned(v[1]->X - v[0]->X, v[1]->Y - v[0]->Y);
            uint32_t tri = (uint32_t)(p * f->L2 + s);
            for (int64_t j = j0; j <= j1; ++j)
                for (int64_t i = i0; i <= i1; ++i) {
                    int64_t px = 256 * i + 128, py = 256 * j + 128;
                    int64_t E0 = edge_i(v[1]->X, v[1]->Y, v[2]->X, v[2]->Y, px, py);
                    int64_t E1 = edge_i(v[2]->X, v[2]->Y, v[0]->X, v[0]->Y, px, py);
                    int64_t E2 = edge_i(v[0]->X, v[0]->Y, v[1]->X, v[1]->Y, px, py);
                    int in0 = E0 > 0 || (E0 == 0 && own0);
                    int in1 = E1 > 0 || (E1 == 0 && own1);
                    int in2 = E2 > 0 || (E2 == 0 && own2);
                    if (!(in0 && in1 && in2)) continue;
                    /* 1/z is affine in screen space: barycentric blend of the
                     * vertices' 1/z with the exact integer edge weights */
                    double key = fma((double)E2, v[2]->iz, fma((double)E1, v[1]->iz, (double)E0 * v[0]->iz)) / (double)A;
                    uint64_t kb;
                    memcpy(&kb, &key, 8);
                    uint64_t cand = ((kb >> 24) << 24) | (uint64_t)(0xFFFFFFu - tri);
                    size_t pix = (size_t)j * f->W + (size_t)i;
                    if (zfull) {   /* largest key, lower id on an exactly equal key */
                        if (zbuf[pix] == 0 || kb > zfull[pix] || (kb == zfull[pix] && tri < ztri[pix])) {
                            zfull[pix] = kb;
                            ztri[pix] = tri;
                            zbuf[pix] = (uint64_t)(0xFFFFFFu - tri) | ((uint64_t)1 << 40);
                        }
                    } else if (cand > zbuf[pix]) zbuf[pix] = cand;
                }
        }
    }
    /* resolve: winning sub-triangle, perspective-correct Bezier-domain (u,v) */
    for (size_t pix = 0; pix < npx; ++pix) {
        if (zbuf[pix] == 0) { f->I_tri[pix] = -1; f->I_uv[2 * pix] = f->I_uv[2 * pix + 1] = 0.0; continue; }
        int tri = (int)(0xFFFFFFu - (uint32_t)(zbuf[pix] & 0xFFFFFFu));
        f->I_tri[pix] = tri;
        f->zkey[pix] = zfull ? zfull[pix] : (zbuf[pix] >> 24) << 24;
    }
    free(rv);
    free(zbuf);
    free(zfull);
    free(ztri);
}

/* Perspective-correct barycentrics of the pixel centre in the winning flat
 * triangle (unsnapped projection), mapped to the Bezier domain. */
static void compute_uv(orc_frame *f) {
    int L = f->cfg.L, P = f->sc.num_prims, n = f->sc.degree, ncp = f->ncp;
    size_t npx = (size_t)f->W * f->H;
    double cp[64 * 3];
    for (size_t pix = 0; pix < npx; ++pix) {
        int tri = f->I_tri[pix];
        if (tri < 0) continue;
        int p = tri / f->L2, s = tri % f->L2;
        if (p >= P) continue;
        int na[3], nb[3];
        subtri_nodes(L, s, na, nb);
        prim_points(f->sc.ctrl, ncp, P, p, cp);
        double x[3], y[3], iz[3], uu[3], vv[3];
        for (int k = 0; k < 3; ++k) {
            double S[3], t[3];
            uu[k] = (double)na[k] / L;
            vv[k] = (double)nb[k] / L;
            orc_surface(n, cp, uu[k], vv[k], 1.0 - uu[k] - vv[k], S);
            cam_apply(f->cam, S, t);
            x[k] = f->cam[12] * t[0] / t[2] + f->cam[14];
            y[k] = f->cam[13] * t[1] / t[2] + f->cam[15];
            iz[k] = 1.0 / t[2];
        }
        double qx = (double)(pix % f->W) + 0.5, qy = (double)(pix / f->W) + 0.5;
        double d = (x[1] - x[0]) * (y[2] - y[0]) - (y[1] - y[0]) * (x[2] - x[0]);
        double lam[3];
        if (d != 0.0) {
            lam[0] = ((x[2] - x[1]) * (qy - y[1]) - (y[2] - y[1]) * (qx - x[1])) / d;
            lam[1] = ((x[0] - x[2]) * (qy - y[2]) - (y[0] - y[2]) * (qx - x[2])) / d;
            lam[2] = ((x[1] - x[0]) * (qy - y[0]) - (y[1] - y[0]) * (qx - x[0])) / d;
        } else {
            lam[0] = lam[1] = lam[2] = 1.0 / 3.0;
        }
        double wsum = 0.0, beta[3];
        for (int k = 0; k < 3; ++k) { beta[k] = lam[k] * iz[k]; wsum += beta[k]; }
        double u = 0.0, v = 0.0;
        for (int k = 0; k < 3; ++k) { u += beta[k] / wsum * uu[k]; v += beta[k] / wsum * vv[k]; }
        f->I_uv[2 * pix] = u;
        f->I_uv[2 * pix + 1] = v;
    }
}

/* ------------------------------------------------ boundary set B (Sec. 3.2) */

static int prim_at(const orc_frame *f, int x, int y) {
    int t = f->I_tri[(size_t)y * f->W + x];
    return t < 0 ? -1 : t / f->L2;
}

static void find_boundary(orc_frame *f) {
    if (f->cfg.no_boundary) {  /* no boundary points without blending coefficients */
        memset(f->is_b, 0, (size_t)f->W * f->H);
        return;
    }
    for (int y = 0; y < f->H; ++y)
        for (int x = 0; x < f->W; ++x) {
            int h = prim_at(f, x, y), b = 0;
            if (h >= 0) {
                if (x > 0 && prim_at(f, x - 1, y) != h) b = 1;
                if (x + 1 < f->W && prim_at(f, x + 1, y) != h) b = 1;
                if (y > 0 && prim_at(f, x, y - 1) != h) b = 1;
                if (y + 1 < f->H && prim_at(f, x, y + 1) != h) b = 1;
            }
            f->is_b[(size_t)y * f->W + x] = (uint8_t)b;
        }
}

/* ------------------------------------------------ Eq. 3-5, EWA splatting */

static void quat_to_rot(const double *q, double *R) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* Theta of Eq. 5: a resolution-R attribute map holds one texel per node
 * (a, b), a + b <= R - 1, of the barycentric lattice of level R - 1 (texel
 * index in the lattice order, a outer); (u, v) takes the linear
 * interpolation of the three texels of the lattice triangle that contains
 * it.  R = 1 is the single texel.  Returns the number of texels used. */
static int theta_weights(int R, double u, double v, int *ti, double *tw) {
    if (R == 1) { ti[0] = 0; tw[0] = 1.0; return 1; }
    int m = R - 1;
    double U = m * u, V = m * v;
    int ia = (int)floor(U), ib = (int)floor(V);
    if (ia < 0) ia = 0;
    if (ib < 0) ib = 0;
    if (ia > m - 1) ia = m - 1;
    if (ib > m - 1) ib = m - 1;
    if (ia + ib > m - 1) ib = m - 1 - ia;   /* on the hypotenuse */
    double fu = U - ia, fv = V - ib;
    if (fu + fv <= 1.0) {                   /* "up" lattice triangle */
        ti[0] = lattice_index(m, ia, ib);     tw[0] = 1.0 - fu - fv;
        ti[1] = lattice_index(m, ia + 1, ib); tw[1] = fu;
        ti[2] = lattice_index(m, ia, ib + 1); tw[2] = fv;
    } else {                                /* "down" lattice triangle */
        ti[0] = lattice_index(m, ia + 1, ib);     tw[0] = 1.0 - fv;
        ti[1] = lattice_index(m, ia, ib + 1);     tw[1] = 1.0 - fu;
        ti[2] = lattice_index(m, ia + 1, ib + 1); tw[2] = fu + fv - 1.0;
    }
    return 3;
}

int orc_theta(int R, double u, double v, int32_t *ti, double *tw) {
    int t[3];
    int n = theta_weights(R, u, v, t, tw);
    for (int e = 0; e < n; ++e) ti[e] = t[e];
    return n;
}

/* rotation and scale of the Gaussian at (u, v) of patch p: the attribute
 * maps interpolated by Theta (log-scales and the raw quaternion, which is
 * then normalised) */
static void pixel_attr(const orc_frame *f, int p, double u, double v, double *log_s, double *qn, double *qnorm,
                       int *ti, double *tw, int *nt) {
    int P = f->sc.num_prims;
    int T = f->sc.attr_res * (f->sc.attr_res + 1) / 2;
    *nt = theta_weights(f->sc.attr_res, u, v, ti, tw);
    double q[4] = {0, 0, 0, 0}, nn = 0.0;
    for (int d = 0; d < 3; ++d) log_s[d] = 0.0;
    for (int e = 0; e < *nt; ++e) {
        for (int d = 0; d < 3; ++d) log_s[d] += tw[e] * f->sc.log_scale[((size_t)d * T + ti[e]) * P + p];
        for (int d = 0; d < 4; ++d) q[d] += tw[e] * f->sc.quat[((size_t)d * T + ti[e]) * P + p];
    }
    for (int d = 0; d < 4; ++d) nn += q[d] * q[d];
    nn = sqrt(nn);
    for (int d = 0; d < 4; ++d) qn[d] = q[d] / nn;
    *qnorm = nn;
}

/* Real spherical harmonics of bands 1..D (Condon-Shortley phase, m = -l..l
 * within a band) at the unit vector d, and their Cartesian gradients
 * dY[k][0..2] of the same polynomials.  The colour of a Gaussian adds
 * sum_k Y_k(d) sh_k to Eq. 4's diffuse colour, d pointing from the camera
 * centre to S_q. */
static int sh_count(int D) { return (D + 1) * (D + 1) - 1; }

static void sh_basis(int D, const double *d, double *Y, double (*dY)[3]) {
    const double pi = 3.14159265358979323846;
    double x = d[0], y = d[1], z = d[2];
    int k = 0;
    if (D >= 1) {
        double c = sqrt(3.0 / (4.0 * pi));
        Y[k] = -c * y; if (dY) { dY[k][0] = 0; dY[k][1] = -c; dY[k][2] = 0; } ++k;
        Y[k] = c * z;  if (dY) { dY[k][0] = 0; dY[k][1] = 0; dY[k][2] = c; } ++k;
        Y[k] = -c * x; if (dY) { dY[k][0] = -c; dY[k][1] = 0; dY[k][2] = 0; } ++k;
    }
    if (D >= 2) {
        double a = 0.5 * sqrt(15.0 / pi), b = 0.25 * sqrt(5.0 / pi), c = 0.25 * sqrt(15.0 / pi);
        Y[k] = a * x * y;  if (dY) { dY[k][0] = a * y; dY[k][1] = a * x; dY[k][2] = 0; } ++k;
        Y[k] = -a * y * z; if (dY) { dY[k][0] = 0; dY[k][1] = -a * z; dY[k][2] = -a * y; } ++k;
        Y[k] = b * (2 * z * z - x * x - y * y);
        if (dY) { dY[k][0] = -2 * b * x; dY[k][1] = -2 * b * y; dY[k][2] = 4 * b * z; } ++k;
        Y[k] = -a * x * z; if (dY) { dY[k][0] = -a * z; dY[k][1] = 0; dY[k][2] = -a * x; } ++k;
        Y[k] = c * (x * x - y * y); if (dY) { dY[k][0] = 2 * c * x; dY[k][1] = -2 * c * y; dY[k][2] = 0; } ++k;
    }
    if (D >= 3) {
        double a = 0.25 * sqrt(35.0 / (2 * pi)), b = 0.5 * sqrt(105.0 / pi), c = 0.25 * sqrt(21.0 / (2 * pi));
        double e = 0.25 * sqrt(7.0 / pi), g = 0.25 * sqrt(105.0 / pi);
        Y[k] = -a * y * (3 * x * x - y * y);
        if (dY) { dY[k][0] = -6 * a * x * y; dY[k][1] = -a * (3 * x * x - 3 * y * y); dY[k][2] = 0; } ++k;
        Y[k] = b * x * y * z;
        if (dY) { dY[k][0] = b * y * z; dY[k][1] = b * x * z; dY[k][2] = b * x * y; } ++k;
        Y[k] = -c * y * (4 * z * z - x * x - y * y);
        if (dY) { dY[k][0] = 2 * c * x * y; dY[k][1] = -c * (4 * z * z - x * x - 3 * y * y); dY[k][2] = -8 * c * y * z; } ++k;
        Y[k] = e * z * (2 * z * z - 3 * x * x - 3 * y * y);
        if (dY) { dY[k][0] = -6 * e * x * z; dY[k][1] = -6 * e * y * z; dY[k][2] = e * (6 * z * z - 3 * x * x - 3 * y * y); } ++k;
        Y[k] = -c * x * (4 * z * z - x * x - y * y);
        if (dY) { dY[k][0] = -c * (4 * z * z - 3 * x * x - y * y); dY[k][1] = 2 * c * x * y; dY[k][2] = -8 * c * x * z; } ++k;
        Y[k] = g * z * (x * x - y * y);
        if (dY) { dY[k][0] = 2 * g * x * z; dY[k][1] = -2 * g * y * z; dY[k][2] = g * (x * x - y * y); } ++k;
        Y[k] = -a * x * (x * x - 3 * y * y);
        if (dY) { dY[k][0] = -a * (3 * x * x - 3 * y * y); dY[k][1] = 6 * a * x * y; dY[k][2] = 0; } ++k;
    }
}

void orc_sh_basis(int D, double x, double y, double z, double *Y, double *dY) {
    double d[3] = {x, y, z};
    sh_basis(D, d, Y, (double (*)[3])dY);
}

/* camera centre in world coordinates, -R^T t */
static void cam_centre(const double *cam, double *C) {
    for (int c = 0; c < 3; ++c) C[c] = -(cam[c] * cam[9] + cam[3 + c] * cam[10] + cam[6 + c] * cam[11]);
}

/* The Gaussian of patch p at (u, v) into record r: Eq. 3 (position), Eq. 4
 * plus the SH colour, Eq. 5 (rotation and scale from the attribute maps) and
 * the EWA projection; with `boundary` also the radius of the boundary
 * Gaussian there.  Returns 0 when S lies behind z_near. */
static int make_record(const orc_frame *f, int p, double u, double v, int boundary, double *r) {
    int P = f->sc.num_prims, n = f->sc.degree, ncp = f->ncp;
    const double *Wc = f->cam;
    double fx = f->cam[12], fy = f->cam[13], cx = f->cam[14], cy = f->cam[15];
    double w = 1.0 - u - v;
    double cp[64 * 3], cc[64 * 3], S[3], col[3], t[3];
    prim_points(f->sc.ctrl, ncp, P, p, cp);
    prim_points(f->sc.color_ctrl, ncp, P, p, cc);
    orc_surface(n, cp, u, v, w, S);   /* Eq. 3 */
    orc_surface(n, cc, u, v, w, col); /* Eq. 4 */
    if (f->sc.sh_degree > 0) {        /* view-dependent colour of the patch's SH coefficients */
        int K = sh_count(f->sc.sh_degree);
        double C[3], dv[3], Y[15];
        cam_centre(f->cam, C);
        for (int c = 0; c < 3; ++c) dv[c] = S[c] - C[c];
        double len = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        for (int c = 0; c < 3; ++c) dv[c] /= len;
        sh_basis(f->sc.sh_degree, dv, Y, NULL);
        for (int ch = 0; ch < 3; ++ch)
            for (int k = 0; k < K; ++k) col[ch] += Y[k] * f->sc.sh[((size_t)ch * K + k) * P + p];
    }
    cam_apply(f->cam, S, t);
    if (!(t[2] > f->cfg.z_near)) return 0;
    double tz = t[2];
    double J[6] = {fx / tz, 0.0, -fx * t[0] / (tz * tz), 0.0, fy / tz, -fy * t[1] / (tz * tz)};
    double Tm[6];
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 3; ++c)
            Tm[3 * a + c] = J[3 * a] * Wc[c] + J[3 * a + 1] * Wc[3 + c] + J[3 * a + 2] * Wc[6 + c];
    /* Eq. 5: rotation and scale from the attribute maps at (u, v) */
    double ls[3], qn[4], qnorm, Rq[9], M[9], S3[9], tw[3];
    int ti[3], nt;
    pixel_attr(f, p, u, v, ls, qn, &qnorm, ti, tw, &nt);
    quat_to_rot(qn, Rq);
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) M[3 * a + c] = Rq[3 * a + c] * exp(ls[c]);
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c)
            S3[3 * a + c] = M[3 * a] * M[3 * c] + M[3 * a + 1] * M[3 * c + 1] + M[3 * a + 2] * M[3 * c + 2];
    double TS[6];
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 3; ++c)
            TS[3 * a + c] = Tm[3 * a] * S3[c] + Tm[3 * a + 1] * S3[3 + c] + Tm[3 * a + 2] * S3[6 + c];
    double SA = TS[0] * Tm[0] + TS[1] * Tm[1] + TS[2] * Tm[2] + f->cfg.dilation;
    double SB = TS[0] * Tm[3] + TS[1] * Tm[4] + TS[2] * Tm[5];
    double SC = TS[3] * Tm[3] + TS[4] * Tm[4] + TS[5] * Tm[5] + f->cfg.dilation;
    double det = SA * SC - SB * SB;
    r[GR_MUX] = fx * t[0] / tz + cx;
    r[GR_MUY] = fy * t[1] / tz + cy;
    r[GR_QA] = SC / det;
    r[GR_QB] = -SB / det;
    r[GR_QC] = SA / det;
    r[GR_CR] = col[0]; r[GR_CG] = col[1]; r[GR_CB] = col[2];
    r[GR_DEPTH] = tz;
    r[GR_SA] = SA; r[GR_SB] = SB; r[GR_SC] = SC;
    r[GR_PRIM] = p;
    double kappa = sqrt(f->kappa2);
    r[GR_RX] = kappa * sqrt(SA);
    r[GR_RY] = kappa * sqrt(SC);
    for (int d = 0; d < 3; ++d) { r[GR_SX + d] = S[d]; r[GR_TX + d] = t[d]; }
    r[GR_SIGMA] = 0.0;
    if (boundary) {
        /* isotropic boundary Gaussian of scale r_b projected to the image:
         * r_b^2 J J^T + low-pass; its radius is 3 sqrt(lambda_max) */
        double rb = f->cfg.r_ref / (double)f->sc.sharpness[p];
        double ma = rb * rb * (J[0] * J[0] + J[2] * J[2]) + f->cfg.dilation;
        double mb = rb * rb * (J[2] * J[5]);
        double mc = rb * rb * (J[4] * J[4] + J[5] * J[5]) + f->cfg.dilation;
        double lam = 0.5 * (ma + mc) + sqrt(0.25 * (ma - mc) * (ma - mc) + mb * mb);
        r[GR_SIGMA] = 3.0 * sqrt(lam);
    }
    return 1;
}

/* (u, v) of lattice Gaussian `node` (nodes (a, b), a + b <= level, in the
 * lattice order, a outer) */
static void lattice_uv(int level, int node, double *u, double *v) {
    int a = 0;
    while (node > level - a) { node -= level - a + 1; ++a; }
    *u = (double)a / level;
    *v = (double)node / level;
}

/* Gaussian records: one per foreground pixel at I_uv (Sec. 3.2, Sub-Primitive
 * Generation).  In the lattice variant the pixel records only serve the
 * boundary points, and the rendered Gaussians sit on a lattice of each
 * patch's (u, v) domain, view by view. */
static void gen_gaussians(orc_frame *f) {
    size_t npx = (size_t)f->W * f->H;
    #pragma omp parallel for schedule(static)
    for (long long pi = 0; pi < (long long)npx; ++pi) {
        size_t pix = (size_t)pi;
        double *r = &f->rec[pix * GR_N];
        f->valid[pix] = 0;
        f->has_rec[pix] = 0;
        int tri = f->I_tri[pix];
        if (tri < 0) { f->is_b[pix] = 0; continue; }
        int p = tri / f->L2;
        if (!make_record(f, p, f->I_uv[2 * pix], f->I_uv[2 * pix + 1], f->is_b[pix], r)) {
            f->is_b[pix] = 0;
            continue;
        }
        f->has_rec[pix] = 1;
        f->valid[pix] = f->nlat == 0;
    }
    if (f->nlat) {
        int NL = f->nlat / f->sc.num_prims;
        #pragma omp parallel for schedule(static)
        for (long long i = 0; i < (long long)f->nlat; ++i) {
            double u, v;
            lattice_uv(f->lat_level, (int)(i % NL), &u, &v);
            f->valid[npx + i] = (uint8_t)make_record(f, (int)(i / NL), u, v, 0, &f->rec[(npx + i) * GR_N]);
        }
    }
}

/* ------------------------------------------------ tile lists (Sec. 3.2,
 * Rendering Acceleration): Gaussians sorted front to back, boundary points
 * sorted by primitive ID. */

typedef struct { uint64_t key; int32_t pix; int32_t tile; } pair_t;

static int cmp_pair(const void *a, const void *b) {
    const pair_t *x = (const pair_t *)a, *y = (const pair_t *)b;
    if (x->tile != y->tile) return x->tile < y->tile ? -1 : 1;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->pix != y->pix) return x->pix < y->pix ? -1 : 1;
    return 0;
}

/* pixel-centre index range [lo, hi] of the closed interval [c - r, c + r] */
static void center_range(double c, double r, int n, int *lo, int *hi) {
    double a = ceil(c - r - 0.5), b = floor(c + r - 0.5);
    if (a < 0) a = 0;
    if (b > n - 1) b = n - 1;
    if (!(a <= b)) { *lo = 1; *hi = 0; return; }
    *lo = (int)a; *hi = (int)b;
}

static int build_lists(orc_frame *f, int which) {
    size_t npx = (size_t)f->W * f->H;
    int TS = f->cfg.tile;
    size_t cap = 0, cnt = 0;
    pair_t *pairs = NULL;
    size_t nrec = which == 0 ? npx + (size_t)f->nlat : npx;
    for (size_t pix = 0; pix < nrec; ++pix) {
        if (which == 0 && !f->valid[pix]) continue;                        /* rendered Gaussians */
        if (which == 1 && !(f->has_rec[pix] && f->is_b[pix])) continue;   /* boundary points */
        const double *r = &f->rec[pix * GR_N];
        int i0, i1, j0, j1;
        if (which == 0) {
            center_range(r[GR_MUX], r[GR_RX], f->W, &i0, &i1);
            center_range(r[GR_MUY], r[GR_RY], f->H, &j0, &j1);
        } else {
            center_range(r[GR_MUX], r[GR_SIGMA], f->W, &i0, &i1);
            center_range(r[GR_MUY], r[GR_SIGMA], f->H, &j0, &j1);
        }
        if (i0 > i1 || j0 > j1) continue;
        uint64_t key;
        if (which == 0) {
            double z = r[GR_DEPTH];
            uint64_t zb;
            memcpy(&zb, &z, 8);
            key = f->cfg.exact_keys ? zb : zb >> 24;   /* z > 0: bit order is numeric order */
        } else {
            key = (uint64_t)(int64_t)r[GR_PRIM];
        }
        for (int ty = j0 / TS; ty <= j1 / TS; ++ty)
            for (int tx = i0 / TS; tx <= i1 / TS; ++tx) {
                if (cnt == cap) {
                    cap = cap ? 2 * cap : 4096;
                    pair_t *np = (pair_t *)realloc(pairs, cap * sizeof(pair_t));
                    if (!np) { free(pairs); return ORC_ENOMEM; }
                    pairs = np;
                }
                pairs[cnt].key = key;
                pairs[cnt].pix = (int32_t)pix;
                pairs[cnt].tile = ty * f->tiles_x + tx;
                ++cnt;
            }
    }
    if (cnt) qsort(pairs, cnt, sizeof(pair_t), cmp_pair);
    int32_t *start = (int32_t *)calloc((size_t)f->ntiles + 1, sizeof(int32_t));
    int32_t *list = (int32_t *)malloc((cnt ? cnt : 1) * sizeof(int32_t));
    if (!start || !list) { free(pairs); free(start); free(list); return ORC_ENOMEM; }
    for (size_t e = 0; e < cnt; ++e) { start[pairs[e].tile + 1]++; list[e] = pairs[e].pix; }
    for (int t = 0; t < f->ntiles; ++t) start[t + 1] += start[t];
    free(pairs);
    if (which == 0) { f->g_start = start; f->g_list = list; }
    else { f->b_start = start; f->b_list = list; }
    return ORC_OK;
}

/* ------------------------------------------------ frame set-up */

void orc_frame_free(orc_frame *f) {
    if (!f) return;
    free(f->I_tri); free(f->zkey); free(f->I_uv); free(f->is_b); free(f->valid); free(f->has_rec); free(f->rec);
    free(f->g_start); free(f->g_list); free(f->b_start); free(f->b_list);
    free(f);
}

orc_frame *orc_frame_create(const orc_scene *sc, const float *cam, int W, int H,
                            const orc_config *cfg, const int32_t *I_tri_in, const double *I_uv_in) {
    if (!sc || !cam || !cfg || W <= 0 || H <= 0 || sc->degree < 1 || sc->degree > 5 ||
        sc->num_prims <= 0 || cfg->L < 1 || cfg->tile <= 0 || (sc->attr_res != 1 && sc->attr_res != 3) ||
        sc->sh_degree < 0 || sc->sh_degree > 3 || (sc->sh_degree > 0 && !sc->sh) ||
        cfg->lattice == 1 || cfg->lattice < 0 || cfg->lattice > 64)
        return NULL;
    orc_frame *f = (orc_frame *)calloc(1, sizeof(orc_frame));
    if (!f) return NULL;
    f->sc = *sc;
    f->cfg = *cfg;
    for (int i = 0; i < 16; ++i) f->cam[i] = (double)cam[i];
    f->W = W; f->H = H;
    f->ncp = ncp_of(sc->degree);
    f->L2 = cfg->L * cfg->L;
    f->tiles_x = (W + cfg->tile - 1) / cfg->tile;
    f->tiles_y = (H + cfg->tile - 1) / cfg->tile;
    f->ntiles = f->tiles_x * f->tiles_y;
    f->kappa2 = 2.0 * log(1.0 / cfg->g_min);
    size_t npx = (size_t)W * H;
    if (cfg->lattice >= 2) {
        /* m nodes per flat sub-triangle edge: the patch's lattice of level
         * L (m - 1), nodes on shared sub-triangle edges counted once */
        f->lat_level = cfg->L * (cfg->lattice - 1);
        f->nlat = sc->num_prims * ((f->lat_level + 1) * (f->lat_level + 2) / 2);
    }
    size_t nrec = npx + (size_t)f->nlat;
    f->I_tri = (int32_t *)malloc(npx * sizeof(int32_t));
    f->zkey = (uint64_t *)calloc(npx, sizeof(uint64_t));
    f->I_uv = (double *)calloc(2 * npx, sizeof(double));
    f->is_b = (uint8_t *)calloc(npx, 1);
    f->valid = (uint8_t *)calloc(nrec, 1);
    f->has_rec = (uint8_t *)calloc(npx, 1);
    f->rec = (double *)calloc(nrec * GR_N, sizeof(double));
    if (!f->I_tri || !f->zkey || !f->I_uv || !f->is_b || !f->valid || !f->has_rec || !f->rec) { orc_frame_free(f); return NULL; }
    if (I_tri_in) {
        memcpy(f->I_tri, I_tri_in, npx * sizeof(int32_t));
        if (I_uv_in) memcpy(f->I_uv, I_uv_in, 2 * npx * sizeof(double));
        else compute_uv(f);
    } else {
        rasterize(f);
        compute_uv(f);
    }
    find_boundary(f);
    gen_gaussians(f);
    if (build_lists(f, 0) != ORC_OK || build_lists(f, 1) != ORC_OK) { orc_frame_free(f); return NULL; }
    return f;
}

/* ------------------------------------------------ accessors */

void orc_frame_dims(const orc_frame *f, int32_t *out) {
    out[0] = f->W; out[1] = f->H; out[2] = f->tiles_x; out[3] = f->tiles_y;
    out[4] = f->g_start[f->ntiles]; out[5] = f->b_start[f->ntiles]; out[6] = GR_N; out[7] = f->nlat;
}

void orc_frame_raster(const orc_frame *f, int32_t *I_tri, double *I_uv, uint8_t *is_b, uint8_t *valid) {
    size_t npx = (size_t)f->W * f->H;
    if (I_tri) memcpy(I_tri, f->I_tri, npx * sizeof(int32_t));
    if (I_uv) memcpy(I_uv, f->I_uv, 2 * npx * sizeof(double));
    if (is_b) memcpy(is_b, f->is_b, npx);
    if (valid) memcpy(valid, f->has_rec, npx);   /* the pixel's Gaussian record exists */
}

/* depth-key bits of each pixel's winning sub-triangle (0: background or a
 * frame made from a given index map) */
void orc_frame_zkeys(const orc_frame *f, uint64_t *out) {
    memcpy(out, f->zkey, (size_t)f->W * f->H * sizeof(uint64_t));
}

/* records [H*W + nlat][GR_N] and which of them are rendered Gaussians */
void orc_frame_records(const orc_frame *f, double *rec, uint8_t *rendered) {
    size_t nrec = (size_t)f->W * f->H + f->nlat;
    if (rec) memcpy(rec, f->rec, nrec * GR_N * sizeof(double));
    if (rendered) memcpy(rendered, f->valid, nrec);
}

void orc_frame_lists(const orc_frame *f, int which, int32_t *start, int32_t *list) {
    const int32_t *s = which == 0 ? f->g_start : f->b_start;
    const int32_t *l = which == 0 ? f->g_list : f->b_list;
    memcpy(start, s, ((size_t)f->ntiles + 1) * sizeof(int32_t));
    memcpy(list, l, (size_t)s[f->ntiles] * sizeof(int32_t));
}

/* ------------------------------------------------ Eq. 6-8, alpha blending */

/* gamma(d; sigma) = min(2^(d/sigma - 1), 1)  (Eq. 7) */
static double gamma_fn(double d, double sigma) {
    double g = exp2(d / sigma - 1.0);
    return g < 1.0 ? g : 1.0;
}

/* gamma* of primitive g at pixel centre (qx,qy): the smallest gamma over the
 * boundary points of g listed for this tile; returns 1 when none is within
 * range.  *arg receives the point the gradient of gamma* is routed to: the
 * minimiser of d/sigma among the points with d/sigma < 1 (gamma is
 * increasing in d/sigma, so it is the point that attains the minimum of
 * Eq. 7), the lowest raster index among exactly equal ratios, or -1 when no
 * point is within range.  The list holds g's points in raster order. */
static double gamma_star(const orc_frame *f, int tile, int g, double qx, double qy, int *arg) {
    double best = 1.0, rbest = 1.0;
    *arg = -1;
    for (int e = f->b_start[tile]; e < f->b_start[tile + 1]; ++e) {
        int bp = f->b_list[e];
        const double *r = &f->rec[(size_t)bp * GR_N];
        if ((int)r[GR_PRIM] != g) continue;
        double dx = qx - r[GR_MUX], dy = qy - r[GR_MUY];
        double d = sqrt(dx * dx + dy * dy), ratio = d / r[GR_SIGMA];
        double gm = gamma_fn(d, r[GR_SIGMA]);
        if (gm < best) best = gm;
        if (ratio < 1.0 && (*arg < 0 || ratio < rbest)) { rbest = ratio; *arg = bp; }
    }
    return best;
}

/* gamma* of primitive g at pixel `pix` and the boundary point its gradient
 * goes to (record index, -1 for none); for the routing checks */
int orc_gamma_star(const orc_frame *f, int pix, int g, double *gamma, int32_t *arg) {
    if (!f || pix < 0 || pix >= f->W * f->H || !gamma || !arg) return ORC_EINVAL;
    int x = pix % f->W, y = pix / f->W;
    int tile = (y / f->cfg.tile) * f->tiles_x + x / f->cfg.tile;
    int a;
    *gamma = gamma_star(f, tile, g, x + 0.5, y + 0.5, &a);
    *arg = a;
    return ORC_OK;
}

typedef struct {
    int gpix;            /* pixel index of the Gaussian */
    double alpha, T, w, G, gamma;
    int clamped, barg;   /* alpha clamped to alpha_max; minimising boundary point */
    double dx, dy;
} contrib_t;

/* Walk the tile list of pixel `pix` front to back (Eq. 8 and point-based
 * alpha blending).  Returns number of contributors; fills C, T_final, the
 * number of list entries visited and, when `out` is given, the contributors. */
static int blend_pixel(const orc_frame *f, size_t pix, double *C, double *Tfin, int *visited,
                       contrib_t *out, int cap) {
    int x = (int)(pix % f->W), y = (int)(pix / f->W);
    double qx = x + 0.5, qy = y + 0.5;
    int tile = (y / f->cfg.tile) * f->tiles_x + x / f->cfg.tile;
    int h = f->I_tri[pix] < 0 ? -1 : f->I_tri[pix] / f->L2;
    double T = 1.0;
    C[0] = C[1] = C[2] = 0.0;
    int nc = 0, vis = 0;
    for (int e = f->g_start[tile]; e < f->g_start[tile + 1]; ++e) {
        vis = e - f->g_start[tile] + 1;
        int gp = f->g_list[e];
        const double *r = &f->rec[(size_t)gp * GR_N];
        double dx = qx - r[GR_MUX], dy = qy - r[GR_MUY];
        double power = r[GR_QA] * dx * dx + 2.0 * r[GR_QB] * dx * dy + r[GR_QC] * dy * dy;
        if (power > f->kappa2) continue;
        int g = (int)r[GR_PRIM];
        int barg = -1;
        double gs = 1.0, w = 1.0;
        /* Eq. 6; w = 1 throughout in the variant without blending
         * coefficients (ablation study, "w/o B") */
        if (!f->cfg.no_boundary) {
            gs = gamma_star(f, tile, g, qx, qy, &barg);
            w = (g == h) ? gs : 1.0 - gs;
        }
        if (w <= 0.0) continue;
        double G = exp(-0.5 * power);
        double o = (double)f->sc.opacity[g];
        double a = o * w * G;                  /* Eq. 8 */
        int clamped = a > f->cfg.alpha_max;
        if (clamped) a = f->cfg.alpha_max;
        if (out && nc < cap) {
            contrib_t *c = &out[nc];
            c->gpix = gp; c->alpha = a; c->T = T; c->w = w; c->G = G; c->gamma = gs;
            c->clamped = clamped; c->barg = barg; c->dx = dx; c->dy = dy;
        }
        C[0] += T * a * r[GR_CR];
        C[1] += T * a * r[GR_CG];
        C[2] += T * a * r[GR_CB];
        T *= (1.0 - a);
        ++nc;
        if (T < f->cfg.t_min) break;
    }
    *Tfin = T;
    *visited = vis;
    return nc;
}

/* Render the listed pixels (all pixels when pixels == NULL). */
int orc_frame_render(const orc_frame *f, const int32_t *pixels, int npix, double *image,
                     double *T_final, int32_t *visited, int32_t *n_contrib) {
    if (!f || !image) return ORC_EINVAL;
    long long N = pixels ? npix : (long long)f->W * f->H;
    #pragma omp parallel for schedule(dynamic, 64)
    for (long long k = 0; k < N; ++k) {
        size_t pix = pixels ? (size_t)pixels[k] : (size_t)k;
        double C[3], T;
        int vis;
        int nc = blend_pixel(f, pix, C, &T, &vis, NULL, 0);
        for (int c = 0; c < 3; ++c) image[3 * k + c] = C[c] + T * f->cfg.bg[c];
        if (T_final) T_final[k] = T;
        if (visited) visited[k] = vis;
        if (n_contrib) n_contrib[k] = nc;
    }
    return ORC_OK;
}

/* Contributors of one pixel (for invariance checks). */
int orc_pixel_trace(const orc_frame *f, int pix, int cap, int32_t *gpix, double *alpha,
                    double *T, double *w) {
    contrib_t *buf = (contrib_t *)malloc(sizeof(contrib_t) * (cap > 0 ? cap : 1));
    double C[3], Tf;
    int vis;
    int nc = blend_pixel(f, (size_t)pix, C, &Tf, &vis, buf, cap);
    for (int i = 0; i < nc && i < cap; ++i) {
        gpix[i] = buf[i].gpix; alpha[i] = buf[i].alpha; T[i] = buf[i].T; w[i] = buf[i].w;
    }
    free(buf);
    return nc;
}

/* ------------------------------------------------ backward (Suppl. Sec. C) */

/* per-pixel Gaussian gradient slots */
enum { DG_MUX, DG_MUY, DG_QA, DG_QB, DG_QC, DG_CR, DG_CG, DG_CB, DG_O, DG_SIGMA, DG_N };

static void atomic_add(double *p, double v) {
    #pragma omp atomic
    *p += v;
}

/* gradient of the loss w.r.t. every parameter; grad_image is [H*W][3];
 * outputs (overwritten) use the scene layouts. */
int orc_frame_grad(const orc_frame *f, const double *grad_image, double *d_ctrl, double *d_color,
                   double *d_log_scale, double *d_quat, double *d_opacity, double *d_sharp, double *d_sh) {
    if (!f || !grad_image) return ORC_EINVAL;
    if (f->sc.sh_degree > 0 && !d_sh) return ORC_EINVAL;
    size_t npx = (size_t)f->W * f->H, nrec = npx + (size_t)f->nlat;
    int P = f->sc.num_prims, n = f->sc.degree, ncp = f->ncp;
    int T = f->sc.attr_res * (f->sc.attr_res + 1) / 2, D = f->sc.sh_degree, K = sh_count(D);
    double *dg = (double *)calloc(nrec * DG_N, sizeof(double));
    if (!dg) return ORC_ENOMEM;
    const double ln2 = log(2.0);

    #pragma omp parallel
    {
        contrib_t *buf = NULL;
        int cap = 0;
        #pragma omp for schedule(dynamic, 64)
        for (long long pk = 0; pk < (long long)npx; ++pk) {
            size_t pix = (size_t)pk;
            const double *gimg = &grad_image[3 * pix];
            if (gimg[0] == 0.0 && gimg[1] == 0.0 && gimg[2] == 0.0) continue;
            int x = (int)(pix % f->W), y = (int)(pix / f->W);
            int tile = (y / f->cfg.tile) * f->tiles_x + x / f->cfg.tile;
            int len = f->g_start[tile + 1] - f->g_start[tile];
            if (len > cap) { free(buf); cap = len; buf = (contrib_t *)malloc(sizeof(contrib_t) * cap); }
            double C[3], Tn;
            int vis;
            int nc = blend_pixel(f, pix, C, &Tn, &vis, buf, cap);
            int h = f->I_tri[pix] < 0 ? -1 : f->I_tri[pix] / f->L2;
            double qx = x + 0.5, qy = y + 0.5;
            /* S_i = sum_{j>i} T_j alpha_j c_j + T_n c_bg, accumulated back to front */
            double S[3] = {Tn * f->cfg.bg[0], Tn * f->cfg.bg[1], Tn * f->cfg.bg[2]};
            for (int i = nc - 1; i >= 0; --i) {
                const contrib_t *c = &buf[i];
                const double *r = &f->rec[(size_t)c->gpix * GR_N];
                double *g = &dg[(size_t)c->gpix * DG_N];
                double col[3] = {r[GR_CR], r[GR_CG], r[GR_CB]};
                double dalpha = 0.0;
                for (int ch = 0; ch < 3; ++ch) {
                    atomic_add(&g[DG_CR + ch], c->T * c->alpha * gimg[ch]);          /* dl/dc_i */
                    dalpha += gimg[ch] * (c->T * col[ch] - S[ch] / (1.0 - c->alpha)); /* dl/dalpha_i */
                }
                for (int ch = 0; ch < 3; ++ch) S[ch] += c->T * c->alpha * col[ch];
                if (c->clamped) continue;
                int gid = (int)r[GR_PRIM];
                double o = (double)f->sc.opacity[gid];
                atomic_add(&g[DG_O], dalpha * c->w * c->G);
                double dG = dalpha * o * c->w;
                double dw = dalpha * o * c->G;                                /* dl/dw = dl/dalpha * alpha / w */
                double Qa = r[GR_QA], Qb = r[GR_QB], Qc = r[GR_QC];
                /* G = exp(-1/2 d^T Q d), d = q - mu */
                atomic_add(&g[DG_MUX], dG * c->G * (Qa * c->dx + Qb * c->dy));
                atomic_add(&g[DG_MUY], dG * c->G * (Qb * c->dx + Qc * c->dy));
                atomic_add(&g[DG_QA], dG * (-0.5 * c->G * c->dx * c->dx));
                atomic_add(&g[DG_QB], dG * (-c->G * c->dx * c->dy));
                atomic_add(&g[DG_QC], dG * (-0.5 * c->G * c->dy * c->dy));
                if (c->barg >= 0 && c->gamma < 1.0) {
                    /* w = gamma* (own primitive) or 1 - gamma* (others), Eq. 6;
                     * gamma' = ln2/sigma * gamma (Suppl. C); d = |q - b| */
                    double dgam = (gid == h) ? dw : -dw;
                    const double *rb = &f->rec[(size_t)c->barg * GR_N];
                    double *gb = &dg[(size_t)c->barg * DG_N];
                    double bx = qx - rb[GR_MUX], by = qy - rb[GR_MUY];
                    double d = sqrt(bx * bx + by * by), sg = rb[GR_SIGMA];
                    double dd = dgam * ln2 / sg * c->gamma;
                    /* |q - b| has its cone point at d = 0, where the subgradient
                     * taken is 0; a boundary point that sits on its own pixel
                     * centre (every boundary pixel of a planar patch) lands
                     * there up to rounding, so d below D_KINK counts as 0 */
                    if (d > D_KINK) {
                        atomic_add(&gb[DG_MUX], -dd * bx / d);   /* dd/db = -(q-b)/d */
                        atomic_add(&gb[DG_MUY], -dd * by / d);
                    }
                    atomic_add(&gb[DG_SIGMA], -dgam * ln2 * d / (sg * sg) * c->gamma);
                }
            }
        }
        free(buf);
    }

    /* chain to the BG-Triangle parameters through Eq. 3-5 and the EWA
     * projection (3DGS), and through the boundary radius sigma_i */
    size_t nc3 = (size_t)3 * ncp * P;
    memset(d_ctrl, 0, nc3 * sizeof(double));
    memset(d_color, 0, nc3 * sizeof(double));
    memset(d_log_scale, 0, (size_t)3 * T * P * sizeof(double));
    memset(d_quat, 0, (size_t)4 * T * P * sizeof(double));
    if (D > 0) memset(d_sh, 0, (size_t)3 * K * P * sizeof(double));
    memset(d_opacity, 0, (size_t)P * sizeof(double));
    memset(d_sharp, 0, (size_t)P * sizeof(double));
    const double *Wc = f->cam;
    double fx = f->cam[12], fy = f->cam[13];
    int NL = f->nlat ? f->nlat / P : 0;
    for (size_t ri = 0; ri < nrec; ++ri) {
        /* rendered Gaussians, and pixel records that only serve as boundary points */
        if (!(f->valid[ri] || (ri < npx && f->has_rec[ri]))) continue;
        const double *r = &f->rec[ri * GR_N];
        const double *g = &dg[ri * DG_N];
        int p = (int)r[GR_PRIM];
        double u, v;
        if (ri < npx) { u = f->I_uv[2 * ri]; v = f->I_uv[2 * ri + 1]; }
        else lattice_uv(f->lat_level, (int)((ri - npx) % NL), &u, &v);
        double B[64];
        orc_bernstein(n, u, v, 1.0 - u - v, B);
        /* colour, Eq. 4 */
        for (int c = 0; c < ncp; ++c)
            for (int ch = 0; ch < 3; ++ch)
                d_color[((size_t)ch * ncp + c) * P + p] += B[c] * g[DG_CR + ch];
        d_opacity[p] += g[DG_O];
        /* view-dependent colour: dl/dsh_k = Y_k dl/dc; the direction
         * d = (S - C) / |S - C| also moves with S */
        double dS_sh[3] = {0.0, 0.0, 0.0};
        if (D > 0) {
            double C[3], dv[3], Y[15], dY[15][3], gd[3] = {0.0, 0.0, 0.0};
            cam_centre(f->cam, C);
            for (int c = 0; c < 3; ++c) dv[c] = r[GR_SX + c] - C[c];
            double len = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
            for (int c = 0; c < 3; ++c) dv[c] /= len;
            sh_basis(D, dv, Y, dY);
            for (int ch = 0; ch < 3; ++ch)
                for (int k = 0; k < K; ++k) {
                    double coef = f->sc.sh[((size_t)ch * K + k) * P + p];
                    d_sh[((size_t)ch * K + k) * P + p] += Y[k] * g[DG_CR + ch];
                    for (int c = 0; c < 3; ++c) gd[c] += g[DG_CR + ch] * coef * dY[k][c];
                }
            double dot = dv[0] * gd[0] + dv[1] * gd[1] + dv[2] * gd[2];
            for (int c = 0; c < 3; ++c) dS_sh[c] = (gd[c] - dv[c] * dot) / len;
        }
        double tx = r[GR_TX], ty = r[GR_TY], tz = r[GR_TZ];
        double J[6] = {fx / tz, 0.0, -fx * tx / (tz * tz), 0.0, fy / tz, -fy * ty / (tz * tz)};
        double Tm[6];
        for (int a = 0; a < 2; ++a)
            for (int c = 0; c < 3; ++c)
                Tm[3 * a + c] = J[3 * a] * Wc[c] + J[3 * a + 1] * Wc[3 + c] + J[3 * a + 2] * Wc[6 + c];
        /* conic Q = Sigma2D^-1 with Sigma2D = [[A,B],[B,C]] */
        double A = r[GR_SA], Bs = r[GR_SB], Cc = r[GR_SC];
        double det = A * Cc - Bs * Bs, det2 = det * det;
        double dQa = g[DG_QA], dQb = g[DG_QB], dQc = g[DG_QC];
        double dA = dQa * (-Cc * Cc / det2) + dQb * (Bs * Cc / det2) + dQc * (-Bs * Bs / det2);
        double dB = dQa * (2.0 * Bs * Cc / det2) + dQb * (-(A * Cc + Bs * Bs) / det2) + dQc * (2.0 * A * Bs / det2);
        double dC = dQa * (-Bs * Bs / det2) + dQb * (A * Bs / det2) + dQc * (-A * A / det2);
        /* Sigma2D = Tm Sigma3D Tm^T + low-pass, Tm = J W */
        double ls[3], qn[4], qnorm, Rq[9], M[9], S3[9], s[3], tw[3];
        int ti[3], nt;
        pixel_attr(f, p, u, v, ls, qn, &qnorm, ti, tw, &nt);
        quat_to_rot(qn, Rq);
        for (int c = 0; c < 3; ++c) s[c] = exp(ls[c]);
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) M[3 * a + c] = Rq[3 * a + c] * s[c];
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c)
                S3[3 * a + c] = M[3 * a] * M[3 * c] + M[3 * a + 1] * M[3 * c + 1] + M[3 * a + 2] * M[3 * c + 2];
        double S3T0[3], S3T1[3];
        for (int a = 0; a < 3; ++a) {
            S3T0[a] = S3[3 * a] * Tm[0] + S3[3 * a + 1] * Tm[1] + S3[3 * a + 2] * Tm[2];
            S3T1[a] = S3[3 * a] * Tm[3] + S3[3 * a + 1] * Tm[4] + S3[3 * a + 2] * Tm[5];
        }
        double dTm[6];
        for (int c = 0; c < 3; ++c) {
            dTm[c] = 2.0 * dA * S3T0[c] + dB * S3T1[c];
            dTm[3 + c] = dB * S3T0[c] + 2.0 * dC * S3T1[c];
        }
        double G3[9];
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c)
                G3[3 * a + c] = dA * Tm[a] * Tm[c] + dB * Tm[a] * Tm[3 + c] + dC * Tm[3 + a] * Tm[3 + c];
        double dM[9];
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += (G3[3 * a + k] + G3[3 * k + a]) * M[3 * k + c];
                dM[3 * a + c] = acc;
            }
        double dRq[9];
        for (int c = 0; c < 3; ++c) {
            double ds = 0.0;
            for (int a = 0; a < 3; ++a) { ds += dM[3 * a + c] * Rq[3 * a + c]; dRq[3 * a + c] = dM[3 * a + c] * s[c]; }
            for (int e = 0; e < nt; ++e) d_log_scale[((size_t)c * T + ti[e]) * P + p] += tw[e] * ds * s[c];
        }
        {
            double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
            double dq[4];
            dq[0] = 2 * (-z * dRq[1] + y * dRq[2] + z * dRq[3] - x * dRq[5] - y * dRq[6] + x * dRq[7]);
            dq[1] = 2 * (y * dRq[1] + z * dRq[2] + y * dRq[3] - 2 * x * dRq[4] - w * dRq[5] + z * dRq[6] + w * dRq[7] - 2 * x * dRq[8]);
            dq[2] = 2 * (-2 * y * dRq[0] + x * dRq[1] + w * dRq[2] + x * dRq[3] + z * dRq[5] - w * dRq[6] + z * dRq[7] - 2 * y * dRq[8]);
            dq[3] = 2 * (-2 * z * dRq[0] - w * dRq[1] + x * dRq[2] + w * dRq[3] - 2 * z * dRq[4] + y * dRq[5] + x * dRq[6] + y * dRq[7]);
            double dot = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
            for (int c = 0; c < 4; ++c)
                for (int e = 0; e < nt; ++e)
                    d_quat[((size_t)c * T + ti[e]) * P + p] += tw[e] * (dq[c] - qn[c] * dot) / qnorm;
        }
        double dJ[6];
        for (int a = 0; a < 2; ++a)
            for (int c = 0; c < 3; ++c)
                dJ[3 * a + c] = dTm[3 * a] * Wc[3 * c] + dTm[3 * a + 1] * Wc[3 * c + 1] + dTm[3 * a + 2] * Wc[3 * c + 2];
        /* boundary radius sigma = 3 sqrt(lambda_max(r_b^2 J J^T + low-pass)) */
        if (ri < npx && f->is_b[ri] && g[DG_SIGMA] != 0.0) {
            double rb = f->cfg.r_ref / (double)f->sc.sharpness[p], r2 = rb * rb;
            double ma = r2 * (J[0] * J[0] + J[2] * J[2]) + f->cfg.dilation;
            double mb = r2 * (J[2] * J[5]);
            double mc = r2 * (J[4] * J[4] + J[5] * J[5]) + f->cfg.dilation;
            double sq = sqrt(0.25 * (ma - mc) * (ma - mc) + mb * mb);
            double lam = 0.5 * (ma + mc) + sq;
            double dlam = g[DG_SIGMA] * 1.5 / sqrt(lam);
            double dma, dmb, dmc;
            if (sq > 0.0) {
                dma = dlam * (0.5 + 0.25 * (ma - mc) / sq);
                dmc = dlam * (0.5 - 0.25 * (ma - mc) / sq);
                dmb = dlam * mb / sq;
            } else {
                dma = dmc = 0.5 * dlam;
                dmb = 0.0;
            }
            dJ[0] += dma * 2.0 * r2 * J[0];
            dJ[2] += dma * 2.0 * r2 * J[2] + dmb * r2 * J[5];
            dJ[5] += dmb * r2 * J[2] + dmc * 2.0 * r2 * J[5];
            dJ[4] += dmc * 2.0 * r2 * J[4];
            double dr2 = dma * (J[0] * J[0] + J[2] * J[2]) + dmb * J[2] * J[5] + dmc * (J[4] * J[4] + J[5] * J[5]);
            double sh = (double)f->sc.sharpness[p];
            d_sharp[p] += dr2 * 2.0 * rb * (-f->cfg.r_ref / (sh * sh));
        }
        /* mean (and boundary point, which is the same projected point) */
        double dmux = g[DG_MUX], dmuy = g[DG_MUY];
        double dt[3];
        dt[0] = dmux * fx / tz + dJ[2] * (-fx / (tz * tz));
        dt[1] = dmuy * fy / tz + dJ[5] * (-fy / (tz * tz));
        dt[2] = dmux * (-fx * tx / (tz * tz)) + dmuy * (-fy * ty / (tz * tz)) +
                dJ[0] * (-fx / (tz * tz)) + dJ[2] * (2.0 * fx * tx / (tz * tz * tz)) +
                dJ[4] * (-fy / (tz * tz)) + dJ[5] * (2.0 * fy * ty / (tz * tz * tz));
        double dS[3];
        for (int c = 0; c < 3; ++c) dS[c] = Wc[c] * dt[0] + Wc[3 + c] * dt[1] + Wc[6 + c] * dt[2] + dS_sh[c];
        /* dl/dp_ijk = dl/dS_q B^n_ijk(I_uv(q))  (Suppl. C) */
        for (int c = 0; c < ncp; ++c)
            for (int d = 0; d < 3; ++d) d_ctrl[((size_t)d * ncp + c) * P + p] += B[c] * dS[d];
    }
    free(dg);
    return ORC_OK;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
