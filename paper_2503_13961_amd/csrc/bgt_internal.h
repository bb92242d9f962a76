// Internal declarations shared by the HIP translation units of libbgt.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bgt.h"

namespace bgt {

// ---------------------------------------------------------------- sizes

constexpr int kMaxL = 8;
constexpr int kMaxNcp = (BGT_MAX_DEGREE + 1) * (BGT_MAX_DEGREE + 2) / 2;  // 21
constexpr int kSortLds = 2048;        // per-tile list length sorted in LDS
constexpr int kBigTriPixels = 256;    // bbox size above which a triangle is rasterized by a block

// state counter slots (int64)
enum Counter {
    C_OVERFLOW = 0,   // bit0 gauss pairs, bit1 boundary pairs, bit2 big-triangle queue
    C_GPAIRS = 1,
    C_BPAIRS = 2,
    C_FG = 3,        // (foreground and boundary pixels are tallied in the
    C_BOUNDARY = 4,  //  striped slots below and summed by bgt_query)
    C_BIGTRI = 5,
    C_BIGSORT = 6,
    C_BIGBLIST = 7,
    C_UNUSED8 = 8,
    C_UNUSED9 = 9,
    C_MANYRUNS = 10,  // tiles with more boundary runs than the forward's gamma* maps
    C_NUM = 16
};
// The per-wave foreground and boundary tallies go to kStripes slots 64 bytes
// apart (slot = 8x8 block index mod kStripes) after the C_NUM counters:
// 160,000 waves adding to one address serialize on it.
constexpr int kStripes = 64;
constexpr int kStripeStride = 8;  // int64 words per slot
constexpr int kCounterWords = C_NUM + kStripes * kStripeStride;

// per-pixel flags
constexpr uint8_t PF_VALID = 1;     // the pixel has a Gaussian
constexpr uint8_t PF_BOUNDARY = 2;  // the pixel is a boundary point

// ---------------------------------------------------------------- views

struct ViewInfo {
    int32_t W, H, tiles_x, tiles_y, px_off, tile_off;
    int32_t b8_off, b8_x;  // first 8x8 pixel block of the view, blocks per row
};

struct ViewTable {
    int32_t n, total_px, total_tiles, total_b8;  // total_b8: 8x8 pixel blocks over all views
    ViewInfo v[BGT_MAX_VIEWS];
};

__device__ __forceinline__ int view_of_pixel(const ViewTable &vt, int pix) {
    int lo = 0, hi = vt.n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (vt.v[mid].px_off <= pix) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int view_of_tile(const ViewTable &vt, int tile) {
    int lo = 0, hi = vt.n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (vt.v[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Pixel of lane `lane` in global 8x8 block `blk` (waves walk 8x8 blocks so
// that neighbouring pixels share a wave).  Returns false outside the image.
__device__ __forceinline__ bool block8_pixel(const ViewTable &vt, int blk, int lane, int &v, int &x, int &y) {
    int lo = 0, hi = vt.n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (vt.v[mid].b8_off <= blk) lo = mid; else hi = mid - 1;
    }
    v = lo;
    const ViewInfo &vi = vt.v[lo];
    const int lb = blk - vi.b8_off;
    x = (lb % vi.b8_x) * 8 + (lane & 7);
    y = (lb / vi.b8_x) * 8 + (lane >> 3);
    return blk < vt.total_b8 && x < vi.W && y < vi.H;
}

// Visit the tiles [tx0, tx1] x [ty0, ty1] of every lane's rectangle (row-major,
// empty when tx0 > tx1); lanes at the same tile are handled together:
// f(tile, group_mask, in_group, leader) is called by the whole wave once per
// group.  Saves one atomic per lane on per-tile counters.
template <typename F>
__device__ __forceinline__ void for_tiles_grouped(int tx0, int tx1, int ty0, int ty1, int tiles_x, int tile_off,
                                                  F &&f) {
    int cx = tx0, cy = ty0;
    bool alive = tx0 <= tx1 && ty0 <= ty1;
    while (true) {
        const unsigned long long am = __ballot(alive);
        if (!am) break;
        const int mine = alive ? tile_off + cy * tiles_x + cx : -1;
        const int leader = __ffsll((long long)am) - 1;
        const int t0 = __shfl(mine, leader, 64);
        const bool in = alive && mine == t0;
        const unsigned long long gm = __ballot(in);
        f(t0, gm, in, leader);
        if (in) {
            if (++cx > tx1) { cx = tx0; if (++cy > ty1) alive = false; }
        }
    }
}

// Workgroups go to the chip's 8 XCDs in turn (workgroup i to XCD i mod 8),
// each XCD with an L2 of its own.  This maps launch index i to a work item
// so that each XCD takes runs of C consecutive items (neighbouring tiles read
// many of the same records); indices past the last whole round of 8 C map to
// themselves.  A bijection of [0, n).
template <int C>
__device__ __forceinline__ int xcd_runs(int i, int n) {
    const int full = n / (8 * C) * (8 * C);
    if (i >= full) return i;
    const int x = i & 7, k = i >> 3;
    return ((k / C) * 8 + x) * C + k % C;
}

// ---------------------------------------------------------------- constants

struct Consts {
    int32_t L, L2, VL, tile;
    int32_t degree, ncp, P, T;
    int32_t batch, flags;  // flags: BGT_FLAG_* of the configuration
    int32_t K, pdw;        // SH coefficients per channel; dwords per patch record
    int32_t lat_level, NL; // lattice variant: level L (m - 1) and Gaussians per patch; NL = 0 otherwise
    float z_near, g_min, t_min, alpha_max, dilation, r_ref;
    float bg[3];
    float kappa2;          // 2 ln(1/g_min), float
    double kappa;          // sqrt(2 ln(1/g_min)), double
    int64_t cap_g, cap_b, cap_big;
};

struct PrimPtrs {
    const float *ctrl, *color, *log_scale, *quat, *opacity, *sharp, *sh;
};

struct GradPtrs {
    float *ctrl, *color, *log_scale, *quat, *opacity, *sharp, *sh;
};

// Packed per-patch record in dwords, written by k_prim_setup so that the
// generation pass reads a patch with a few scalar loads:
//   [0, 3 NCP)      control points, [c][d]
//   [3 NCP, 6 NCP)  colour control points, [c][d]
//   6 NCP           opacity, then one pad dword
//   6 NCP + 2 ...   ten doubles: R(q) diag(e^s) row-major of texel 0, then r_b^2
//   6 NCP + 22 ...  raw quaternion (4), log-scale (3) of texel 0, sharpness (1)
//   6 NCP + 30 ...  with resolution-3 maps or SH: every texel's raw quaternion
//                   and log-scale ([t][7]), then the SH coefficients ([k][c])
// rounded up to 16 dwords.
__host__ __device__ constexpr int patch_dw(int ncp, int T = 1, int K = 0) {
    return (6 * ncp + 30 + (T > 1 || K > 0 ? 7 * T + 3 * K : 0) + 15) / 16 * 16;
}
__host__ __device__ constexpr int patch_m_off(int ncp) { return 6 * ncp + 2; }
__host__ __device__ constexpr int patch_q_off(int ncp) { return 6 * ncp + 22; }
__host__ __device__ constexpr int patch_x_off(int ncp) { return 6 * ncp + 30; }
__host__ __device__ constexpr int patch_sh_off(int ncp, int T) { return 6 * ncp + 30 + 7 * T; }

// per-view projected lattice vertex

struct VertRec {
    double x, y, iz;       // unsnapped projection and 1/z
    int32_t X, Y;          // 1/256-px fixed point; X == INT32_MIN marks a culled vertex
};

// Gaussian record, 4 x float4 per pixel (and per lattice Gaussian):
//  r0 = (mu_x - x - 1/2, mu_y - y - 1/2, Q_a, Q_b): the mean relative to the
//       centre of the record's pixel (x, y) keeps FP32 offsets small;
//       conic Q = [[a, b], [b, c]]
//  r1 = (Q_c, c_r, c_g, c_b)
//  r2 = (opacity, prim (int bits), sigma_b, (x, y) as an int16 pair x | y << 16)
//  r3 = (g x-range, g y-range, b x-range, b y-range) as int16 pairs (lo | hi << 16)
// A pixel's record is at its own pixel; a lattice Gaussian's at the pixel
// (floor(mu_x), floor(mu_y)), clamped to +-30000.  The depth is kept in
// the sort key array (gkey) only.
// The backward's 9 sums of a Gaussian record in one tile of its range go to
// slot (ty mod 3) 3 + tx mod 3 of the record, and the sort writes the
// record's position in that tile's list to the same slot: within a range of
// at most 3 x 3 tiles ("narrow") no two tiles share a slot.  Slot-major
// arrays ([slot][record]), so that consecutive records are consecutive in
// memory for the parameter pass, which reads them in pixel order.  A record
// reaching more tiles ("wide") adds its sums into kSums floats of its own
// instead (float atomics).
constexpr int kSums = 9;
constexpr int kSlotTiles = 9;

struct StatePtrs {
    int64_t *counters;
    unsigned long long *zbuf;
    int32_t *I_tri;
    float2 *I_uv;
    uint8_t *pflags;
    float4 *rec;
    unsigned long long *gkey;
    float *T_final;
    int32_t *last;
    VertRec *verts;        // [V][VL][P]
    double *wverts;        // [VL][P][3] world lattice
    float *patch;          // [P][patch_dw(ncp)] packed per-patch record (see patch_dw)
    int32_t *g_count, *g_start, *g_cursor;
    int32_t *b_count, *b_start, *b_cursor;
    unsigned long long *g_keys, *b_keys;
    uint32_t *g_list, *b_list;
    int64_t n_rec;         // Gaussian records
    float *gslot;          // [kSlotTiles][records][kSums] the backward's sums of narrow records per tile slot,
                           // written for the tile's replayed prefix (zeros for entries no pixel reached)
    int32_t *gpos;         // [kSlotTiles][records] the record's position in the tile's sorted list (the sort)
    int32_t *t_end;        // [tiles] list position past the tile's replayed prefix, whose sums the backward wrote
    float *gwide;          // [records][kSums] the sums of wide records (zeroed by the generation, added by
                           // the backward, read and zeroed by the parameter pass)
    float *dbound;         // [pixels][3] dl/dsigma_b, dl/dmu (x, y) of each boundary point (zeroed by the
                           // generation, accumulated by the backward, read and zeroed by the parameter pass)
    double *brec64;        // [pixels][3] boundary points in FP64: mu - pixel centre (x, y), sigma
    int32_t *big_tris;     // [cap_big] queue of raster items
    int32_t *scan_tmp;     // block sums
};

__device__ __forceinline__ int pack16(int lo, int hi) { return (lo & 0xFFFF) | (hi << 16); }

// Record index of a tile-list key's low digits `lr`, the record's index
// within its view v: the view's pixels first, then its lattice Gaussians
// (lat_per_view = P NL of them, stored after all views' pixels).
__device__ __forceinline__ int record_of(const ViewTable &vt, int v, int lr, int lat_per_view) {
    const ViewInfo &vi = vt.v[v];
    const int npx = vi.W * vi.H;
    return lr < npx ? vi.px_off + lr : vt.total_px + v * lat_per_view + (lr - npx);
}
__device__ __forceinline__ int lo16(int v) { return (int)(int16_t)(v & 0xFFFF); }
__device__ __forceinline__ int hi16(int v) { return v >> 16; }

__device__ __forceinline__ int tile_slot(int tx, int ty) { return ty % 3 * 3 + tx % 3; }
// does the tile range of the packed pixel ranges gx, gy (lo | hi << 16, not
// empty) hold at most 3 x 3 tiles of side 1 << tsh?
__device__ __forceinline__ bool narrow_range(int gx, int gy, int tsh) {
    return (hi16(gx) >> tsh) - (lo16(gx) >> tsh) < 3 && (hi16(gy) >> tsh) - (lo16(gy) >> tsh) < 3;
}
__device__ __forceinline__ void zero_sums(float *g) {
#pragma unroll
    for (int f = 0; f < kSums; ++f) g[f] = 0.f;
}

// ---------------------------------------------------------------- training step

constexpr double kSsimC1 = 0.01 * 0.01, kSsimC2 = 0.03 * 0.03;

// views of the loss pass: 32x16 output tiles, view-major
struct LossTable {
    int32_t n, total_tiles, total_px, pad;
    int32_t W[BGT_MAX_VIEWS], H[BGT_MAX_VIEWS], tiles_x[BGT_MAX_VIEWS];
    int32_t tile_off[BGT_MAX_VIEWS + 1], px_off[BGT_MAX_VIEWS];
    double taps[11];   // normalised Gaussian window, sigma 1.5
    double inv_n;      // 1 / (3 * total pixels)
    double lam;        // weight of the D-SSIM term
};

struct AdamTable {
    int32_t n, pad;
    int64_t off[BGT_MAX_ADAM_GROUPS + 1];  // element offsets of the groups
    float *param[BGT_MAX_ADAM_GROUPS];
    const float *grad[BGT_MAX_ADAM_GROUPS];
    float *m[BGT_MAX_ADAM_GROUPS];
    float *v[BGT_MAX_ADAM_GROUPS];
    double lr[BGT_MAX_ADAM_GROUPS];
};

// ---------------------------------------------------------------- splitting and pruning

struct StatsPtrs {
    int32_t *views_seen;
    int32_t *vis_views;
    unsigned long long *tex, *view_bits;
    float *grad_sum;
    int32_t *grad_cnt;
    float *edge_sum;
    int32_t *edge_cnt;
};

struct DensifyRule {
    double tau_g, tau_b, tau_v, tau_r, tau_a, tau_s;
};

// ---------------------------------------------------------------- launchers

hipError_t launch_tessellate(const Consts &k, const PrimPtrs &pr, double *wverts, float *verts_out,
                             hipStream_t s);
hipError_t launch_raster(const Consts &k, const ViewTable &vt, const PrimPtrs &pr, const float *cams,
                         const StatePtrs &st, hipStream_t s);
hipError_t launch_gen(const Consts &k, const ViewTable &vt, const PrimPtrs &pr, const float *cams,
                      const StatePtrs &st, hipStream_t s);
hipError_t launch_binning(const Consts &k, const ViewTable &vt, const StatePtrs &st, hipStream_t s);
hipError_t launch_note_overflow(const StatePtrs &st, unsigned long long *flag, hipStream_t s);

// context internals for the entry points outside bgt_api.cpp
int ctx_device(const bgt_ctx *ctx);
bgt_status ctx_fail(bgt_ctx *ctx, bgt_status st, const char *msg);
// the static loss workspace of bgt_loss_noalloc (bgt_static.hip): its device
// address is fetched once per device, with that device current
hipError_t static_scratch_init(int device);
size_t static_scratch_bytes();
void *static_scratch(int device);
hipError_t launch_blend_fwd(const Consts &k, const ViewTable &vt, const StatePtrs &st, float *image,
                            hipStream_t s);
hipError_t launch_blend_bwd(const Consts &k, const ViewTable &vt, const StatePtrs &st,
                            const float *image, const float *grad_image, hipStream_t s);
hipError_t launch_param_bwd(const Consts &k, const ViewTable &vt, const PrimPtrs &pr, const float *cams,
                            const StatePtrs &st, const GradPtrs &gr, hipStream_t s);
// Arrays cleared by one launch, as 4-byte words (a segment with no words is
// left out): the pass's counters, z-buffer and tile counts, or a backward
// pass's gradient arrays
constexpr int kZeroSegs = 8;
struct ZeroTable {
    uint32_t *p[kZeroSegs];
    int64_t words[kZeroSegs];
    int n = 0;
    void add(void *ptr, int64_t w) {
        if (w > 0 && n < kZeroSegs) { p[n] = (uint32_t *)ptr; words[n] = w; ++n; }
    }
};
hipError_t launch_zero(const ZeroTable &t, hipStream_t s);
void loss_tiles(int W, int H, int *tiles_x, int *tiles);
hipError_t launch_loss(const LossTable &lt, const float *x, const float *y, float *loss, float *grad, float *maps,
                       double *partial, hipStream_t s);
hipError_t launch_stats(const Consts &k, const ViewTable &vt, const int32_t *I_tri, const float *targets,
                        const float *d_ctrl, const StatsPtrs &sp, hipStream_t s);
hipError_t launch_plan(const Consts &k, const float *ctrl, const StatsPtrs &sp, const DensifyRule &rule,
                       int32_t *action, int32_t *dst_index, int32_t *count, hipStream_t s);
hipError_t launch_apply(const Consts &k, const PrimPtrs &src, const int32_t *action, const int32_t *dst_index,
                        int Pd, const GradPtrs &dst, hipStream_t s);
hipError_t launch_l1(int64_t n, const float *x, const float *y, float scale, float *g, hipStream_t s);
hipError_t launch_adam(const AdamTable &at, double b1, double b2, double eps, int32_t *step, hipStream_t s);

}  // namespace bgt
