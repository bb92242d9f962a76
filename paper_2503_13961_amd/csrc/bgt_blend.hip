// Discontinuity-aware alpha blending (Sec. 3.2, Eq. 6-8) and its backward
// pass (Supplementary Sec. C) on gfx950.
//
// One workgroup renders one TSxTS tile; each wave owns an 8x8 pixel block
// and each 16-lane row of a wave a 4x4 sub-block.  The tile's boundary
// points (sorted by primitive id) are staged in LDS and split into runs of
// equal id.  For every run r the block builds
//     gamma*_r(q) = min over the run's points b of min(2^(|q-b|/sigma_b - 1), 1)
// for all pixels q of the tile by a scatter-min from each point over the
// pixels of its disc (LDS atomics), so the blend loop reads w from LDS
// instead of searching boundary points per (pixel, Gaussian) pair; a
// Gaussian of primitive g finds its run by binary search over the run ids.
// Gaussians are then composited front to back in LDS-staged batches.  A
// ballot per sub-block marks the batch entries whose pixel range touches it,
// and each row walks its own mask, so the four rows of a wave composite four
// (possibly different) Gaussians per step; a Gaussian that misses a
// sub-block costs that sub-block nothing.
#include <type_traits>

#include "bgt_internal.h"
#include "bgt_wave.h"

namespace bgt {

// Runs with an LDS gamma* map per tile (forward, backward) and boundary
// points staged in LDS.  The budget keeps 6 workgroups per CU at 16 px; on
// the 2000-patch sphere at 16 px a tile has at most 13 runs (mean 4.4) and
// 157 points (the 20,000-patch box: 24 and 251).  Runs and tiles beyond it
// take the slower paths, never a wrong one.  A 32 px tile meets about four
// times the runs; its workgroup of 16 waves is one per CU whatever its LDS
// (registers bound it), so it maps 24.  An 8 px workgroup is a single wave
// whose LDS sets how many waves share a SIMD: with 32-entry batches it stages
// 88 points and maps 8 runs (about 6 KB, six waves per SIMD), with 64-entry
// batches 128 points and 12 runs (four), for scenes with more runs per tile.
// The backward keeps a dl/dgamma* sum per (run, pixel) in registers for the
// first kDgrRuns runs only; a mapped run beyond those sends its boundary
// terms to the arg-min point at once.
template <int TS, int K>
struct RunMapsFwd {
    static constexpr int value = TS >= 32 ? 24 : (TS >= 16 || K > 32 ? 12 : 8);
};
template <int TS, int K>
struct RunMapsBwd {
    static constexpr int value = RunMapsFwd<TS, K>::value;
};
constexpr int kDgrRuns = 12;
template <int TS, int K>
struct BoundaryCap {
    static constexpr int value = TS >= 32 ? 512 : (TS >= 16 ? 256 : (K > 32 ? 128 : 88));
};

// Thread layout: wave w owns the 8x8 block (w % SPR, w / SPR); lane l of it
// the pixel (4 (q & 1) + (i & 3), 4 (q >> 1) + (i >> 2)) of that block, with
// q = l / 16 its row (4x4 sub-block) and i = l % 16.
template <int TS>
struct TileGeom {
    static constexpr int NT = TS * TS;
    static constexpr int SPR = TS / 8;  // 8x8 blocks per tile row
    __device__ static __forceinline__ void local_xy(int tid, int &lx, int &ly) {
        const int wave = tid >> 6, q = (tid >> 4) & 3, i = tid & 15;
        lx = (wave % SPR) * 8 + (q & 1) * 4 + (i & 3);
        ly = (wave / SPR) * 8 + (q >> 1) * 4 + (i >> 2);
    }
    __device__ static __forceinline__ int tid_of(int lx, int ly) {
        const int bx = lx & 7, by = ly & 7;
        return ((ly >> 3) * SPR + (lx >> 3)) * 64 + ((by >> 2) * 2 + (bx >> 2)) * 16 + (by & 3) * 4 + (bx & 3);
    }
};

// boundary staging shared by forward and backward
// Boundary point e sits at pixel (bix, biy) (tile-relative) plus the offset
// (bdx, bdy) of its projected position from that pixel's centre; distances
// to pixel (x, y) are (x - bix) - bdx etc., an exact integer minus one float,
// so every value depends only on the point and the pixel, never on the tile.
template <int TS, int K, int RM>
struct BoundaryLds {
    static constexpr int CAP = BoundaryCap<TS, K>::value;
    static constexpr int NMAP = RM;
    float bdx[CAP], bdy[CAP], bs[CAP];
    int bxy[CAP];  // tile-relative pixel x | y << 16 (int16 each)
    uint8_t brun[CAP];  // each point's run, 255 for runs from 255 on (only runs below NMAP are mapped)
    int run_prim[CAP];
    uint16_t run_start[CAP + 1];  // first point of each run (CAP fits 16 bits)
    int n_runs, nbl, max_rows;
    union {
        struct {
            int bp[CAP];            // each point's primitive, while the runs are found
            int wsum[33];           // and the scans' wave sums
        };
        unsigned map[RM][TS * TS];  // then gamma* bits per (run, pixel in thread order)
    };
    static_assert(RM * TS * TS >= CAP + 33, "the maps hold the staging ids");
    static_assert(RM < 255, "run indices of mapped runs fit brun");
    static_assert(CAP < 65536, "point indices fit run_start");
};

// A staged Gaussian's mean is kept per wave as (g - w0) + delta, where g is
// the Gaussian's own pixel, w0 the origin of the wave's 8x8 block and delta
// the mean's offset from g's centre: one rounding that does not depend on
// the tile size.
// BOUND: the forward's layout, whose colour carries the sub-block bound
template <int TS, int K, bool BOUND>
struct BatchLds {
    // per-wave mean offsets and (primitive id, run index); in the forward at
    // 8 px (one wave) side by side in 16-byte records like e and c, so that
    // one address serves every per-entry read (the backward, whose entry is
    // wave-uniform, keeps them apart: packed, its compiler moved the means to
    // scalar registers at two more instructions per entry)
    static constexpr bool PACK = TS == 8 && BOUND;
    struct MP {
        float2 m;
        int2 pr;
    };
    struct Packed {
        MP mp[K];
    };
    struct Apart {
        float2 m[TS * TS / 64][K];
        int2 pr[K];
    };
    typename std::conditional<PACK, Packed, Apart>::type mpr;
    float4 e[K];                // conic in exponent form kE (a, 2b, c), opacity
    float4 c[K];                // colour; w (forward): exponent below which no pixel of a 4x4 sub-block is in the support
    int xr[K], yr[K];
    __device__ __forceinline__ float2 &m(int w, int kk) {
        if constexpr (PACK) return mpr.mp[kk].m;
        else return mpr.m[w][kk];
    }
    __device__ __forceinline__ int2 &pr(int kk) {
        if constexpr (PACK) return mpr.mp[kk].pr;
        else return mpr.pr[kk];
    }
    __device__ __forceinline__ const float2 &m(int w, int kk) const {
        if constexpr (PACK) return mpr.mp[kk].m;
        else return mpr.m[w][kk];
    }
    __device__ __forceinline__ const int2 &pr(int kk) const {
        if constexpr (PACK) return mpr.mp[kk].pr;
        else return mpr.pr[kk];
    }
};

// |q - b| has its cone point at d = 0, where the subgradient taken is 0; a
// boundary point on its own pixel centre (every boundary pixel of a planar
// patch) lands there up to rounding, so distances below kDKink pixels count
// as 0 for the position gradient
constexpr float kDKink = 1e-6f;
// Bound on |d/sigma in FP32 - d/sigma in FP64| for the staged boundary
// points (offsets of at most a few pixels from their pixel centres, radii
// >= 3 sqrt(0.3)): FP32 rounds the stored offsets and radius and the
// distance and ratio.  Points whose FP32 ratios are within twice this of the
// smallest are re-decided from the FP64 records.
constexpr float kRatioBand = 4e-6f;

// -log2(e)/2: G = exp(-d^T Q d / 2) = 2^(kE d^T Q d)
constexpr float kE = -0.5f * 1.44269504088896341f;

// 2^e for the support exponent e in [log2(g_min), 0]: the hardware exp2
// (no denormal range reduction is needed there).  Forward and backward use
// this one function, so the backward's replay reproduces the forward's
// transmittance bit for bit.
__device__ __forceinline__ float support_exp2(float e) { return __builtin_amdgcn_exp2f(e); }

// block-wide exclusive scan of int flags (blockDim multiple of 64)
__device__ __forceinline__ int block_scan_excl(int x, int &total, int *ws) {
    const int lane = __lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) ws[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        int w = lane < nw ? ws[lane] : 0, wi = w;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int y = __shfl_up(wi, o, 64);
            if (lane >= o) wi += y;
        }
        if (lane < nw) ws[lane] = wi - w;
        if (lane == nw - 1) ws[32] = wi;
    }
    __syncthreads();
    const int res = inc - x + ws[wave];
    total = ws[32];
    __syncthreads();
    return res;
}

// Stage the tile's boundary points and find the runs of equal primitive id.
template <typename BL>
__device__ __forceinline__ void stage_boundary(BL &B, const StatePtrs &st, int bs0, int bc,
                                               int ox, int oy, const ViewInfo &vi) {
    const int nbl = bc < B.CAP ? bc : B.CAP;
    for (int e = threadIdx.x; e < nbl; e += blockDim.x) {
        const int bpix = (int)st.b_list[bs0 + e];
        const float4 r0 = st.rec[(int64_t)bpix * 4];
        const float4 r2 = st.rec[(int64_t)bpix * 4 + 2];
        const int a = __float_as_int(r2.w);                  // the record's pixel
        B.bxy[e] = pack16(lo16(a) - ox, hi16(a) - oy);       // relative to the tile origin
        B.bdx[e] = r0.x;
        B.bdy[e] = r0.y;
        B.bs[e] = r2.z;
        B.bp[e] = __float_as_int(r2.y);
    }
    if (threadIdx.x == 0) B.n_runs = 0;
    __syncthreads();
    for (int base = 0; base < nbl; base += blockDim.x) {
        const int e = base + threadIdx.x;
        const int f = (e < nbl && (e == 0 || B.bp[e] != B.bp[e - 1])) ? 1 : 0;
        int tot;
        const int nr0 = B.n_runs;
        const int ex = block_scan_excl(f, tot, B.wsum);
        if (e < nbl) {
            if (f) { B.run_prim[nr0 + ex] = B.bp[e]; B.run_start[nr0 + ex] = (uint16_t)e; }
            B.brun[e] = (uint8_t)min(nr0 + ex + f - 1, 255);
        }
        __syncthreads();
        if (threadIdx.x == 0) B.n_runs = nr0 + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) { B.run_start[B.n_runs] = (uint16_t)nbl; B.nbl = nbl; }
    __syncthreads();
}

// run index of primitive g among the tile's runs, -1 when absent
__device__ __forceinline__ int find_run(const int *run_prim, int n_runs, int g) {
    int lo = 0, hi = n_runs - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int pm = run_prim[mid];
        if (pm == g) return mid;
        if (pm < g) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

// |(dx, dy)| with an explicit rounding sequence, so every code path that
// evaluates a boundary distance produces the same bits
__device__ __forceinline__ float bdist(float dx, float dy) { return sqrtf(__fmaf_rn(dx, dx, __fmul_rn(dy, dy))); }

// gamma(d; sigma) = min(2^(d/sigma - 1), 1)  (Eq. 7)
__device__ __forceinline__ float gamma_fn(float d, float sigma) {
    const float g = exp2f(__fsub_rn(__fdiv_rn(d, sigma), 1.0f));
    return g < 1.0f ? g : 1.0f;
}

// The boundary point the gradient of gamma* goes to (Suppl. Sec. C, dl/db):
// the minimiser of d/sigma among the points with d/sigma < 1, the lowest list
// (raster) index among exactly equal ratios.  The FP32 pass finds the
// smallest ratio and the first point attaining it; when another point lies
// within 2 kRatioBand of it, the order is decided again on the FP64 records
// of the points in that band, which the generation pass keeps for every
// boundary point, so the choice is the one exact arithmetic makes.
struct ArgScan {
    float best = 1.0f;   // gamma* (FP32, the value the forward used)
    float q1 = 2.0f;     // smallest ratio below 1, and the runner-up
    float q2 = 2.0f;
    int e1 = -1;
    __device__ __forceinline__ void add(float g, float q, int e) {
        if (g < best) best = g;
        if (!(q < 1.0f)) return;
        if (q < q1) { q2 = q1; q1 = q; e1 = e; }
        else if (q < q2) q2 = q;
    }
    __device__ __forceinline__ bool ambiguous() const { return e1 >= 0 && q2 - q1 <= 2.0f * kRatioBand; }
};

// d/sigma in FP64 from pixel (x, y) to the boundary point of record bpix,
// whose pixel is (bx, by) (same frame as x, y)
__device__ __forceinline__ double ratio64(const StatePtrs &st, int bpix, int x, int y, int bx, int by) {
    const double *b = st.brec64 + (int64_t)bpix * 3;
    const double dx = (double)(x - bx) - b[0], dy = (double)(y - by) - b[1];
    return sqrt(dx * dx + dy * dy) / b[2];
}

// gamma* of run r at tile pixel (lx, ly) from the LDS points (the exact
// minimum, bit-identical to the map)
template <typename BL>
__device__ __forceinline__ float gamma_lds_value(const BL &B, int r, int lx, int ly) {
    float best = 1.0f;
    for (int e = B.run_start[r]; e < B.run_start[r + 1]; ++e) {
        const float dx = (float)(lx - lo16(B.bxy[e])) - B.bdx[e], dy = (float)(ly - hi16(B.bxy[e])) - B.bdy[e];
        const float g = gamma_fn(bdist(dx, dy), B.bs[e]);
        if (g < best) best = g;
    }
    return best;
}

// FP64 decision among the LDS entries of [e0, e1) whose FP32 ratio at tile
// pixel (lx, ly) is below 1 and within 2 kRatioBand of the smallest, q1
// (only near-ties come here)
template <typename BL>
__device__ __forceinline__ int redecide_lds(const BL *B, const StatePtrs &st, int bs0, int e0, int e1, float q1, int lx,
                                         int ly) {
    double rb = 2.0;
    int arg = -1;
    for (int e = e0; e < e1; ++e) {
        const float dx = (float)(lx - lo16(B->bxy[e])) - B->bdx[e], dy = (float)(ly - hi16(B->bxy[e])) - B->bdy[e];
        const float q32 = __fdiv_rn(bdist(dx, dy), B->bs[e]);
        if (!(q32 < 1.0f && q32 <= q1 + 2.0f * kRatioBand)) continue;
        const double q = ratio64(st, (int)st.b_list[bs0 + e], lx, ly, lo16(B->bxy[e]), hi16(B->bxy[e]));
        if (q < rb) { rb = q; arg = e; }
    }
    return arg;
}

// ... and in *arg the LDS entry the gradient goes to (-1: none in range)
template <typename BL>
__device__ __forceinline__ float gamma_lds(const BL &B, const StatePtrs &st, int bs0, int r, int lx, int ly,
                                           int *arg) {
    ArgScan a;
    const int e0 = B.run_start[r], e1 = B.run_start[r + 1];
    for (int e = e0; e < e1; ++e) {
        const float dx = (float)(lx - lo16(B.bxy[e])) - B.bdx[e], dy = (float)(ly - hi16(B.bxy[e])) - B.bdy[e];
        const float d = bdist(dx, dy);
        a.add(gamma_fn(d, B.bs[e]), __fdiv_rn(d, B.bs[e]), e);
    }
    *arg = a.ambiguous() ? redecide_lds(&B, st, bs0, e0, e1, a.q1, lx, ly) : a.e1;
    return a.best;
}

// gamma* straight from global memory (tiles with more boundary points than
// the LDS stage holds); with `arg`, also the entry of the tile's list the
// gradient goes to
__device__ __forceinline__ int first_of_prim(const StatePtrs &st, int bs0, int bc, int g) {
    int lo = 0, hi = bc;  // first entry with prim >= g
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int pm = __float_as_int(st.rec[(int64_t)st.b_list[bs0 + mid] * 4 + 2].y);
        if (pm < g) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ float gamma_global(const StatePtrs &st, int bs0, int bc, int g, int px, int py, int *arg) {
    ArgScan a;
    const int e0 = first_of_prim(st, bs0, bc, g);
    int e1 = e0;
    for (; e1 < bc; ++e1) {
        const int bpix = (int)st.b_list[bs0 + e1];
        const float4 r2 = st.rec[(int64_t)bpix * 4 + 2];
        if (__float_as_int(r2.y) != g) break;
        const float4 r0 = st.rec[(int64_t)bpix * 4];
        const int c = __float_as_int(r2.w);
        const float dx = (float)(px - lo16(c)) - r0.x, dy = (float)(py - hi16(c)) - r0.y;
        const float d = bdist(dx, dy);
        a.add(gamma_fn(d, r2.z), __fdiv_rn(d, r2.z), e1);
    }
    if (arg) {
        *arg = a.e1;
        if (a.ambiguous()) {
            double rb = 2.0;
            for (int e = e0; e < e1; ++e) {
                const int bpix = (int)st.b_list[bs0 + e];
                const float4 r0 = st.rec[(int64_t)bpix * 4];
                const float4 r2 = st.rec[(int64_t)bpix * 4 + 2];
                const int c = __float_as_int(r2.w);
                const float dx = (float)(px - lo16(c)) - r0.x, dy = (float)(py - hi16(c)) - r0.y;
                const float q32 = __fdiv_rn(bdist(dx, dy), r2.z);
                if (!(q32 < 1.0f && q32 <= a.q1 + 2.0f * kRatioBand)) continue;
                const double q = ratio64(st, bpix, px, py, lo16(c), hi16(c));
                if (q < rb) { rb = q; *arg = e; }
            }
        }
    }
    return a.best;
}

// Pixel rows [y0, y1] of the tile that a point's disc can reach, one row
// of margin each side (the per-pixel test decides); the whole tile for a
// radius that is not finite or exceeds two tiles.
template <int TS>
__device__ __forceinline__ void disc_rows(float yb, float sg, int &y0, int &y1) {
    if (!(sg < (float)(2 * TS))) {
        y0 = 0;
        y1 = TS - 1;
        return;
    }
    y0 = (int)fmaxf(floorf(yb - sg) - 1.0f, 0.0f);
    y1 = (int)fminf(ceilf(yb + sg) + 1.0f, (float)(TS - 1));
}

// Scatter-min of every staged point over the pixels of its disc, into the
// maps of the first B.NMAP runs (gamma bits compare as unsigned integers).
// The (point, row) items of all mapped points are spread over the threads,
// and a row visits the pixels its chord of the disc can reach: the points'
// discs differ in size and a thread per point waited for the largest.
template <int TS, typename BL>
__device__ __forceinline__ void build_gamma_maps(BL &B) {
    using G = TileGeom<TS>;
    const int nmap = B.n_runs < B.NMAP ? B.n_runs : B.NMAP;
    for (int i = threadIdx.x; i < nmap * G::NT; i += blockDim.x) B.map[i / G::NT][i % G::NT] = 0x3F800000u;
    if (threadIdx.x == 0) B.max_rows = 0;
    __syncthreads();
    for (int e = threadIdx.x; e < B.nbl; e += blockDim.x) {
        if (B.brun[e] >= B.NMAP) continue;
        int y0, y1;
        disc_rows<TS>((float)hi16(B.bxy[e]) + B.bdy[e], B.bs[e], y0, y1);
        if (y1 >= y0) atomicMax(&B.max_rows, y1 - y0 + 1);
    }
    __syncthreads();
    const int R = B.max_rows;
    for (int it = threadIdx.x; it < B.nbl * R; it += blockDim.x) {
        const int e = it / R, row = it - e * R;
        const int r = B.brun[e];
        if (r >= B.NMAP) continue;
        const int bix = lo16(B.bxy[e]), biy = hi16(B.bxy[e]);
        const float bdx = B.bdx[e], bdy = B.bdy[e], sg = B.bs[e];
        int y0, y1;
        disc_rows<TS>((float)biy + bdy, sg, y0, y1);
        const int y = y0 + row;
        if (y > y1) continue;
        const float dy = (float)(y - biy) - bdy;
        int x0 = 0, x1 = TS - 1;
        if (sg < (float)(2 * TS)) {
            const float xb = (float)bix + bdx, h = sqrtf(fmaxf(sg * sg - dy * dy, 0.0f));
            x0 = (int)fmaxf(floorf(xb - h) - 1.0f, 0.0f);
            x1 = (int)fminf(ceilf(xb + h) + 1.0f, (float)(TS - 1));
        }
        for (int x = x0; x <= x1; ++x) {
            const float dx = (float)(x - bix) - bdx;
            const float d = bdist(dx, dy);
            if (d < sg) {
                const float g = gamma_fn(d, sg);
                if (g < 1.0f) atomicMin(&B.map[r][G::tid_of(x, y)], __float_as_uint(g));
            }
        }
    }
    __syncthreads();
}

// Records of one batch slot, fetched from global memory one batch ahead of
// their use by the loader threads (tid < K); the list entry is fetched one
// batch earlier still, so neither load stalls the wave that issues it.
struct SlotPrefetch {
    float4 r0, r1, r2, r3;
    int gp = -1;       // pixel (record index) of the records in flight
    int gp_next = -1;  // list entry for the batch after them
    __device__ __forceinline__ void issue(const StatePtrs &st, int gs0, int n, int base_next, int tid, int K) {
        gp = gp_next;
        if (gp >= 0) {
            const float4 *rp = st.rec + (int64_t)gp * 4;
            r0 = rp[0]; r1 = rp[1]; r2 = rp[2]; r3 = rp[3];
        }
        const int i2 = base_next + K + tid;
        gp_next = (tid < K && i2 < n) ? (int)st.g_list[gs0 + i2] : -1;
    }
};

// For pixels q within rho of a point p, the triangle inequality in the conic's
// norm gives |q - mu|_Q >= |p - mu|_Q - sqrt(lambda_max(Q)) rho.  So no pixel
// of a 4x4 sub-block (its centres within rho = 1.5 sqrt 2 of the block's
// centre) has d^T Q d <= kappa^2 when the centre's exponent is below
// kE (kappa + sqrt(lambda_max) rho)^2; the bound is widened by 1e-3 (relative
// and absolute) so that FP32 rounding of either side never drops a live pixel.
__device__ __forceinline__ float sub_block_bound(float qa, float qb, float qc, float kappa) {
    const float h = 0.5f * (qa - qc);
    const float lmax = 0.5f * (qa + qc) + sqrtf(h * h + qb * qb);
    const float rad = (kappa + sqrtf(fmaxf(lmax, 0.0f)) * 2.1214f) * 1.001f + 1e-3f;
    return kE * rad * rad;
}

// BOUND: also store the sub-block bound (the forward's row masks use it)
template <int TS, int K, bool BOUND>
__device__ __forceinline__ void stage_slot(BatchLds<TS, K, BOUND> &S, const SlotPrefetch &P, int kk, int ox, int oy,
                                           const int *run_prim, int n_runs, bool slow_b, float kappa) {
    using G = TileGeom<TS>;
    // tile-relative pixel the Gaussian's mean is stored against
    const int a = __float_as_int(P.r2.w);
    const int x = lo16(a) - ox, y = hi16(a) - oy;
#pragma unroll
    for (int w = 0; w < G::NT / 64; ++w)
        S.m(w, kk) = make_float2((float)(x - (w % G::SPR) * 8) + P.r0.x, (float)(y - (w / G::SPR) * 8) + P.r0.y);
    S.e[kk] = make_float4(kE * P.r0.z, 2.0f * kE * P.r0.w, kE * P.r1.x, P.r2.x);
    S.c[kk] = make_float4(P.r1.y, P.r1.z, P.r1.w, BOUND ? sub_block_bound(P.r0.z, P.r0.w, P.r1.x, kappa) : 0.f);
    const int g = __float_as_int(P.r2.y);
    // a tile whose boundary list overflowed the LDS stage has its last staged
    // run cut short (n_runs counts complete runs only): a primitive not among
    // them is searched in global memory
    int r = find_run(run_prim, n_runs, g);
    if (r < 0 && slow_b) r = -2;
    S.pr(kk) = make_int2(g, r);
    S.xr[kk] = __float_as_int(P.r3.x);
    S.yr[kk] = __float_as_int(P.r3.y);
}

// the backward's staging of slot kk from record gp's words P; returns
// whether the record is wide (more than 3 x 3 tiles)
template <int TS, int K>
__device__ __forceinline__ bool stage_rec(BatchLds<TS, K, false> &S, const SlotPrefetch &P, int kk, int ox, int oy,
                                          const int *run_prim, int n_runs, bool slow_b) {
    stage_slot<TS, K, false>(S, P, kk, ox, oy, run_prim, n_runs, slow_b, 0.f);
    return !narrow_range(__float_as_int(P.r3.x), __float_as_int(P.r3.y), TS == 8 ? 3 : (TS == 16 ? 4 : 5));
}
__device__ __forceinline__ void load_rec(const StatePtrs &st, int gp, SlotPrefetch &P) {
    const float4 *rp = st.rec + (int64_t)gp * 4;
    P.r0 = rp[0]; P.r1 = rp[1]; P.r2 = rp[2]; P.r3 = rp[3];
}
// ... read at once
template <int TS, int K>
__device__ __forceinline__ bool load_stage(BatchLds<TS, K, false> &S, const StatePtrs &st, int gp, int kk, int ox, int oy,
                                           const int *run_prim, int n_runs, bool slow_b) {
    SlotPrefetch P;
    load_rec(st, gp, P);
    return stage_rec<TS, K>(S, P, kk, ox, oy, run_prim, n_runs, slow_b);
}

// does the pixel range (packed int16 pairs) touch the 4x4 sub-block at (x0, y0)?
__device__ __forceinline__ bool touches4(int xr, int yr, int x0, int y0) {
    return !(hi16(xr) < x0 || lo16(xr) > x0 + 3 || hi16(yr) < y0 || lo16(yr) > y0 + 3);
}

// Which of the batch entries [c0, c0 + 64) (below n) can reach each 4x4
// sub-block of the wave's 8x8 block at (wx0, wy0): one ballot per sub-block.
// An entry counts when its support box touches the sub-block and the
// sub-block's centre is within the conic bound of sub_block_bound (an entry
// left out has no live pixel there, so the result does not change).
template <int TS, int K>
__device__ __forceinline__ void sub_block_masks(const BatchLds<TS, K, true> &S, int wave, int c0, int n, int lane,
                                                int wx0, int wy0, unsigned long long (&mb)[4]) {
    const int j = c0 + lane, jj = j < K ? j : K - 1;
    const bool in = j < n;
    const int a = S.xr[jj], b = S.yr[jj];
    const float2 m = S.m(wave, jj);
    const float4 ex = S.e[jj];
    const float thr = S.c[jj].w;
    // exponents at the sub-block centres (1.5 | 5.5, 1.5 | 5.5) of the wave's block
    const float dx0 = 1.5f - m.x, dx1 = 5.5f - m.x, dy0 = 1.5f - m.y, dy1 = 5.5f - m.y;
    const float by0 = ex.y * dy0, by1 = ex.y * dy1, cy0 = ex.z * dy0 * dy0, cy1 = ex.z * dy1 * dy1;
    const bool n0 = fmaf(dx0, fmaf(ex.x, dx0, by0), cy0) < thr, n1 = fmaf(dx1, fmaf(ex.x, dx1, by0), cy0) < thr;
    const bool n2 = fmaf(dx0, fmaf(ex.x, dx0, by1), cy1) < thr, n3 = fmaf(dx1, fmaf(ex.x, dx1, by1), cy1) < thr;
    mb[0] = __ballot(in && !n0 && touches4(a, b, wx0, wy0));
    mb[1] = __ballot(in && !n1 && touches4(a, b, wx0 + 4, wy0));
    mb[2] = __ballot(in && !n2 && touches4(a, b, wx0, wy0 + 4));
    mb[3] = __ballot(in && !n3 && touches4(a, b, wx0 + 4, wy0 + 4));
}

// ... this lane's row's mask (the forward's rows walk their own sub-block)
template <int TS, int K>
__device__ __forceinline__ unsigned long long row_mask(const BatchLds<TS, K, true> &S, int wave, int c0, int n, int lane,
                                                       int wx0, int wy0) {
    unsigned long long mb[4];
    sub_block_masks<TS, K>(S, wave, c0, n, lane, wx0, wy0, mb);
    const int q = lane >> 4;
    return q == 0 ? mb[0] : (q == 1 ? mb[1] : (q == 2 ? mb[2] : mb[3]));
}

// index of the lowest set bit of m; 0 when m is 0, so that a row with
// nothing left reads the first entry of the half batch (always a staged,
// finite record, which its lanes then ignore)
__device__ __forceinline__ int low_bit(unsigned m) { return m ? __builtin_ctz(m) : 0; }

// do all 16 lanes of this lane's row have the flag set?
__device__ __forceinline__ bool row_all(bool f, int lane) {
    return ((__ballot(f) >> (lane & 48)) & 0xFFFFull) == 0xFFFFull;
}



// Row reduce-scatter of nine per-lane values: butterflies over lane bits 0
// (quad_perm [1,0,3,2]), 1 (quad_perm [2,3,0,1]) and 3 (row_ror:8) each halve
// the set of values a lane carries (v[0..7]; v[8] is summed in every lane),
// then row_shr:4 folds bit 2.  Afterwards, in every 16-lane row, the lane
// with bit 2 set and bits (b3, b1, b0) holds the row total of
// v[4 b3 + 2 b1 + b0] in v[0], and every lane with bit 2 set the row total
// of v[8] in v[8]: 26 VALU operations instead of 36 for nine plain row sums.
__device__ __forceinline__ void row_reduce_scatter9(float *v, int lane) {
    const bool b0 = (lane & 1) != 0, b1 = (lane & 2) != 0, b3 = (lane & 8) != 0;
    float u[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float keep = b0 ? v[2 * k + 1] : v[2 * k], send = b0 ? v[2 * k] : v[2 * k + 1];
        u[k] = keep + dpp_f<0xB1, 0xF>(send);
    }
    float s8 = v[8] + dpp_f<0xB1, 0xF>(v[8]);
    float w[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const float keep = b1 ? u[2 * m + 1] : u[2 * m], send = b1 ? u[2 * m] : u[2 * m + 1];
        w[m] = keep + dpp_f<0x4E, 0xF>(send);
    }
    s8 += dpp_f<0x4E, 0xF>(s8);
    const float keep = b3 ? w[1] : w[0], send = b3 ? w[0] : w[1];
    float x = keep + dpp_f<0x128, 0xF>(send);
    s8 += dpp_f<0x128, 0xF>(s8);
    x += dpp_f<0x114, 0xF>(x);  // row_shr:4
    s8 += dpp_f<0x114, 0xF>(s8);
    v[0] = x;
    v[8] = s8;
}

// Sum over the four 16-lane rows, in every row: exchanges with lane xor 32
// and xor 16 through the LDS crossbar (ds_bpermute), off the vector ALU.
__device__ __forceinline__ float cross_row_sum_bp(float x, int lane) {
    x += __int_as_float(__builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, __float_as_int(x)));
    return x + __int_as_float(__builtin_amdgcn_ds_bpermute((lane ^ 16) << 2, __float_as_int(x)));
}

// ------------------------------------------------------------ forward

template <int TS, int K>
__global__ void __launch_bounds__(TS *TS) k_blend_fwd(Consts k, ViewTable vt, StatePtrs st, float *image) {
    using G = TileGeom<TS>;
    using BL = BoundaryLds<TS, K, RunMapsFwd<TS, K>::value>;
    constexpr int RM = BL::NMAP;
    __shared__ BL B;
    __shared__ BatchLds<TS, K, true> S;
    const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int v = view_of_tile(vt, t);
    const ViewInfo vi = vt.v[v];
    const int tl = t - vi.tile_off, tx = tl % vi.tiles_x, ty = tl / vi.tiles_x;
    int lx, ly;
    G::local_xy(tid, lx, ly);
    const int px = tx * TS + lx, py = ty * TS + ly;
    const bool inside = px < vi.W && py < vi.H;
    const int pix = vi.px_off + py * vi.W + px;
    int h = -1;
    if (inside) {
        const int tri = st.I_tri[pix];
        h = tri < 0 ? -1 : tri / k.L2;
    }
    const int ox = tx * TS, oy = ty * TS;
    const float qx = (float)(lx & 7), qy = (float)(ly & 7);  // position in the wave's 8x8 block
    const int wx0 = tx * TS + (wave % G::SPR) * 8, wy0 = ty * TS + (wave / G::SPR) * 8;

    const int bs0 = st.b_start[t], bc = st.b_count[t];
    const bool slow_b = bc > BoundaryCap<TS, K>::value;
    if (slow_b && tid == 0) atomicAdd((unsigned long long *)&st.counters[C_BIGBLIST], 1ull);
    if (st.g_count[t] == 0) {
        // no Gaussian reaches the tile (most of the background): T = 1
        if (inside) {
            image[3 * (int64_t)pix + 0] = k.bg[0];
            image[3 * (int64_t)pix + 1] = k.bg[1];
            image[3 * (int64_t)pix + 2] = k.bg[2];
            st.T_final[pix] = 1.0f;
            st.last[pix] = 0;
        }
        return;
    }
    // the first batch's records are read before the boundary points are
    // staged, so that the two waits overlap
    const int gs0 = st.g_start[t], gc = st.g_count[t];
    SlotPrefetch pf;
    pf.gp_next = (tid < K && tid < gc) ? (int)st.g_list[gs0 + tid] : -1;
    pf.issue(st, gs0, gc, 0, tid, K);
    stage_boundary(B, st, bs0, bc, ox, oy, vi);
    const int n_full = slow_b ? B.n_runs - 1 : B.n_runs;  // runs staged in full
    if (B.n_runs > RM && tid == 0) atomicAdd((unsigned long long *)&st.counters[C_MANYRUNS], 1ull);
    build_gamma_maps<TS>(B);

    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    bool done = !inside;
    int last = gc;
    const float amax = k.alpha_max, tmin = k.t_min;
    const bool nob = (k.flags & BGT_FLAG_NO_BOUNDARY) != 0;
    // can an entry's run lack a gamma* map (more runs than maps, or a list
    // beyond the stage)?  Only then do the loops below look for such entries
    const bool rare = slow_b || B.n_runs > RM;
    // support test d^T Q d <= 2 ln(1/g_min) as a base-2 exponent: G = 2^e, e >= log2(g_min)
    const float e_min = kE * k.kappa2;
    const float kappa = sqrtf(k.kappa2);
    if (pf.gp >= 0) stage_slot<TS, K, true>(S, pf, tid, ox, oy, B.run_prim, n_full, slow_b, kappa);
    for (int base = 0; base < gc; base += K) {
        if (__syncthreads_and(done ? 1 : 0)) break;  // also publishes the staged batch
        int stop_kk = -1;  // batch index of the entry at which this pixel stops in this batch
        pf.issue(st, gs0, gc, base + K, tid, K);     // next batch's records, in flight during compositing
        const int nk = min(K, gc - base);
        if (!__all(done)) {
            for (int c0 = 0; c0 < nk; c0 += 64) {
                unsigned long long mine = row_mask<TS, K>(S, wave, c0, nk, lane, wx0, wy0);
                if (row_all(done, lane)) mine = 0;  // this row has stopped
#pragma unroll
                for (int hb = 0; hb < 64; hb += 32) {
                    unsigned mm = (unsigned)(mine >> hb);
                    if (__any(mm != 0u)) do {
                        // each row composites its own next entry: branch-free per
                        // lane, a lane that does not composite it takes alpha = 0,
                        // which leaves T and C bit-identical
                        const bool act = mm != 0u;
                        const int kk = c0 + hb + low_bit(mm);
                        mm &= mm - 1u;
                        const int2 pr = S.pr(kk);
                        const float2 m = S.m(wave, kk);
                        const float4 ex = S.e[kk];
                        const float4 c = S.c[kk];
                        const int g = pr.x, r = pr.y;  // uniform within the row
                        const bool own = g == h || nob;  // w = 1 for all without coefficients
                        const float dx = qx - m.x, dy = qy - m.y;
                        const float e = fmaf(dx, fmaf(ex.x, dx, ex.y * dy), ex.z * dy * dy);
                        // w = 0 without a boundary point of g near this tile, or outside the support
                        bool live = act && !done && (own || r != -1) && e >= e_min;
                        // (at 16 and 32 px a step in which no lane's support
                        // is reached leaves before the gamma* lookups, as in
                        // the backward; T and C would not change)
                        if (TS >= 16 && !__any(live)) continue;
                        const bool mapped = r >= 0 && r < RM;
                        float gam = __uint_as_float(B.map[min(max(r, 0), RM - 1)][tid]);
                        gam = mapped ? gam : 1.0f;
                        if (rare && __any(live && r != -1 && !mapped)) {  // runs without a map, big lists
                            if (live && r >= RM) gam = gamma_lds_value(B, r, lx, ly);
                            else if (live && r == -2) gam = gamma_global(st, bs0, bc, g, px, py, nullptr);
                        }
                        // w = 0 (gamma* = 1 for another patch's Gaussian) gives
                        // a = 0 with no test: T and C stay as they are
                        const float w = own ? gam : 1.0f - gam;
                        // min(raw, alpha_max) as integers: the same as fminf for
                        // every non-NaN raw, alpha_max being positive (one
                        // instruction; fminf also canonicalizes alpha_max)
                        float a = __int_as_float(min(__float_as_int(ex.w * w * support_exp2(e)), __float_as_int(amax)));
                        a = live ? a : 0.0f;
                        const float ta = T * a;
                        C0 += ta * c.x;
                        C1 += ta * c.y;
                        C2 += ta * c.z;
                        T = T * (1.0f - a);
                        // (the stopping entry's batch index; the list index is
                        // formed once per batch below)
                        const bool stop = live && T < tmin;
                        done = done || stop;
                        stop_kk = stop ? kk : stop_kk;
                    } while (__any(mm != 0u));
                }
            }
        }
        if (stop_kk >= 0) last = base + stop_kk + 1;
        __syncthreads();  // everyone is done with this batch
        if (pf.gp >= 0) stage_slot<TS, K, true>(S, pf, tid, ox, oy, B.run_prim, n_full, slow_b, kappa);
    }
    if (inside) {
        image[3 * (int64_t)pix + 0] = C0 + T * k.bg[0];
        image[3 * (int64_t)pix + 1] = C1 + T * k.bg[1];
        image[3 * (int64_t)pix + 2] = C2 + T * k.bg[2];
        st.T_final[pix] = T;
        st.last[pix] = last;
    }
}

// ------------------------------------------------------------ backward

// Front-to-back replay of the forward per pixel: T_i is recomputed exactly as
// the forward did, the suffix S_i = sum_{j>i} T_j a_j c_j + T_n bg is the
// forward colour minus the running prefix (carried as its dot product with
// dl/dC), and
//   dl/dc_i = T_i a_i dl/dC,  dl/da_i = dl/dC . (T_i c_i - S_i / (1 - a_i)),
//   dl/dw = dl/da a / w (Supplementary Sec. C), G = exp(-d^T Q d / 2).
// Per Gaussian the 9 gradient values are summed over each row with DPP and
// over rows and waves in LDS (an 8x8 tile is one wave: no LDS), then stored
// once per tile in the record's slot for the tile (plain stores: the
// parameter pass sums a record's slots over its tiles in a fixed order, so
// the result does not depend on scheduling; a record reaching more than
// 3 x 3 tiles adds into sums of its own by float atomics instead).
// The boundary terms accumulate per (run, pixel) and go to the minimising
// boundary point at the end of the tile.
// Waves per SIMD the backward's registers must allow: at 16 px the LDS of
// up to 64-entry batches lets six workgroups share a CU, which 80 registers
// per lane keep (the compiler otherwise takes 82 and five); elsewhere no bound.
template <int TS, int K>
struct BwdWaves {
    static constexpr int value = TS == 16 && K <= 64 ? 6 : 1;
};

template <int TS, int K>
__global__ void __launch_bounds__(TS *TS) __attribute__((amdgpu_waves_per_eu(BwdWaves<TS, K>::value)))
k_blend_bwd(Consts k, ViewTable vt, StatePtrs st, const float *image,
                                                     const float *grad_image) {
    using G = TileGeom<TS>;
    using BL = BoundaryLds<TS, K, RunMapsBwd<TS, K>::value>;
    constexpr int RM = BL::NMAP;
    __shared__ BL B;
    // the batch stage and its gradient sums are dead once the list is done;
    // the per-point boundary sums reuse their space
    // a 8x8 tile is one wave, whose totals are the tile's: they go straight
    // to global memory, and the workgroup needs no LDS sums (its smaller
    // footprint lets more workgroups share a CU)
    constexpr bool ONE = TS == 8;
    struct LoopLds {
        BatchLds<TS, K, false> S;
        float acc[ONE ? 1 : K * 9];  // gradient sums of the staged entries
    };
    union TailLds {
        LoopLds loop;
        float bacc[BoundaryCap<TS, K>::value][3];
    };
    __shared__ TailLds U;
    // (kept at kDgrRuns even where fewer runs are mapped: below about ten
    // entries the compiler indexes the array by select chains, not registers)
    constexpr int RD = kDgrRuns;
    float dgr[RD];  // sums of dl/dgamma* per tracked run at this pixel (uniform index: indexed registers)
#pragma unroll
    for (int i = 0; i < RD; ++i) dgr[i] = 0.f;
    __shared__ int max_last;
    BatchLds<TS, K, false> &S = U.loop.S;
    float *acc = U.loop.acc;
    // runs of 64 neighbouring tiles per XCD: the sums of a record's tiles
    // then mostly meet in one L2
    const int t = xcd_runs<64>(blockIdx.x, gridDim.x), tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int gc = st.g_count[t];
    if (gc == 0) {  // no Gaussian reaches the tile: nothing to differentiate
        if (tid == 0) st.t_end[t] = 0;
        return;
    }
    const int v = view_of_tile(vt, t);
    const ViewInfo vi = vt.v[v];
    const int tl = t - vi.tile_off, tx = tl % vi.tiles_x, ty = tl / vi.tiles_x;
    int lx, ly;
    G::local_xy(tid, lx, ly);
    const int px = tx * TS + lx, py = ty * TS + ly;
    const bool inside = px < vi.W && py < vi.H;
    const int pix = vi.px_off + py * vi.W + px;
    int h = -1, mylast = 0;
    float g0 = 0.f, g1 = 0.f, g2 = 0.f, im0 = 0.f, im1 = 0.f, im2 = 0.f;
    if (inside) {
        const int tri = st.I_tri[pix];
        h = tri < 0 ? -1 : tri / k.L2;
        mylast = min(max(st.last[pix], 0), gc);
        g0 = grad_image[3 * (int64_t)pix]; g1 = grad_image[3 * (int64_t)pix + 1]; g2 = grad_image[3 * (int64_t)pix + 2];
        im0 = image[3 * (int64_t)pix]; im1 = image[3 * (int64_t)pix + 1]; im2 = image[3 * (int64_t)pix + 2];
        if (g0 == 0.f && g1 == 0.f && g2 == 0.f) mylast = 0;
    }
    const int ox = tx * TS, oy = ty * TS;
    const float qx = (float)(lx & 7), qy = (float)(ly & 7);
    const int wx0 = tx * TS + (wave % G::SPR) * 8, wy0 = ty * TS + (wave / G::SPR) * 8;
    // this tile's slot of the narrow records' sums
    float *const gs_tile = st.gslot + (int64_t)tile_slot(tx, ty) * st.n_rec * kSums;

    if (tid == 0) max_last = 0;
    if (!ONE)
        for (int i = tid; i < K * 9; i += blockDim.x) acc[i] = 0.f;
    __syncthreads();
    atomicMax(&max_last, mylast);
    int wave_last = mylast;  // last list entry any lane of this wave replays
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) wave_last = max(wave_last, __shfl_xor(wave_last, o, 64));

    // the first batch's records are read before the boundary points are
    // staged, so that the two waits overlap (entries past the replayed
    // prefix, known once the stop indices are combined, are dropped then)
    const int gs0 = st.g_start[t];
    const int gp0 = (tid < K && tid < gc) ? (int)st.g_list[gs0 + tid] : -1;
    SlotPrefetch P0;
    if (gp0 >= 0) load_rec(st, gp0, P0);
    const int bs0 = st.b_start[t], bc = st.b_count[t];
    stage_boundary(B, st, bs0, bc, ox, oy, vi);  // (syncs)
    const bool slow_b = bc > BoundaryCap<TS, K>::value;
    const int n_full = slow_b ? B.n_runs - 1 : B.n_runs;  // runs staged in full
    build_gamma_maps<TS>(B);

    const int nlast = max_last;
    if (tid == 0) st.t_end[t] = gs0 + nlast;  // the prefix of the list whose sums are written below
    // dl/dC . S: the suffix colour S = C - prefix enters dl/dalpha only through
    // its dot product with dl/dC, so that product is carried instead of S
    float T = 1.0f, GS = g0 * im0 + g1 * im1 + g2 * im2;
    const float amax = k.alpha_max;
    const bool nob = (k.flags & BGT_FLAG_NO_BOUNDARY) != 0;
    const float e_min = kE * k.kappa2;
    const float LN2 = 0.69314718055994531f;
    // the loaders read their records at the end of the previous batch, not
    // ahead of it: registers held across the replay would cost a wave per SIMD
    int cur_gp = tid < nlast ? gp0 : -1;
    bool wide = false;
    if (cur_gp >= 0) wide = stage_rec<TS, K>(S, P0, tid, ox, oy, B.run_prim, n_full, slow_b);
    unsigned long long wide_b = __ballot(wide);  // the wave's loaders of wide records
    for (int base = 0; base < nlast; base += K) {
        __syncthreads();  // publishes the staged batch
        unsigned long long stored = 0ull;  // (one wave) entries whose sums went to memory
        const int nkw = min(min(K, nlast - base), wave_last - base);  // entries this wave replays
        for (int c0 = 0; c0 < nkw; c0 += 64) {
            const int j = c0 + lane, jj = j < K ? j : K - 1;
            unsigned long long mask = __ballot(j < nkw && !(hi16(S.xr[jj]) < wx0 || lo16(S.xr[jj]) > wx0 + 7 ||
                                                             hi16(S.yr[jj]) < wy0 || lo16(S.yr[jj]) > wy0 + 7));
            while (mask) {
                const int kk = c0 + __ffsll((long long)mask) - 1;  // wave-uniform
                mask &= mask - 1;
                const int2 prk = S.pr(kk);
                const int g = prk.x;
                const int r = __builtin_amdgcn_readfirstlane(prk.y);
                const float2 m = S.m(wave, kk);
                const float4 ex = S.e[kk];
                const float4 c = S.c[kk];
                const bool own = g == h || nob;  // w = 1 for all without coefficients
                const float dx = qx - m.x, dy = qy - m.y;
                const float e = fmaf(dx, fmaf(ex.x, dx, ex.y * dy), ex.z * dy * dy);  // as in the forward
                bool live = base + kk < mylast && (own || r != -1) && e >= e_min;
                // at 16 and 32 px an entry that no lane's support reaches
                // leaves before the gamma* lookups (common where the
                // Gaussians are small against the 8x8 blocks; at 8 px the
                // branch costs more than it saves)
                if (TS >= 16 && !__any(live)) continue;
                const bool mapped = r >= 0 && r < RM;
                const bool tracked = r >= 0 && r < RD;  // (uniform) dgr holds its dl/dgamma*
                float gam = 1.0f;
                int arg = -1;
                if (mapped) {
                    gam = __uint_as_float(B.map[r][tid]);
                } else if (r >= 0) {
                    if (live) gam = gamma_lds(B, st, bs0, r, lx, ly, &arg);
                } else if (r == -2) {
                    if (live) gam = gamma_global(st, bs0, bc, g, px, py, &arg);
                }
                const float w = own ? gam : 1.0f - gam;
                live = live && w > 0.0f;
                if (!__any(live)) continue;
                const float o = ex.w;
                const float Gv = support_exp2(e);
                const float raw = o * w * Gv;
                const bool clamped = raw > amax;
                // min(raw, alpha_max) as integers, as in the forward (the same
                // as the clamp for every non-NaN raw, alpha_max being positive)
                float a = __int_as_float(min(__float_as_int(raw), __float_as_int(amax)));
                a = live ? a : 0.0f;
                const float ta = T * a;
                const float d_c0 = ta * g0, d_c1 = ta * g1, d_c2 = ta * g2;
                const float gc = g0 * c.x + g1 * c.y + g2 * c.z;  // dl/dC . c_i
                GS -= ta * gc;
                const float inv = __builtin_amdgcn_rcpf(1.0f - a);
                const float dalpha = T * gc - GS * inv;
                T = T * (1.0f - a);
                const bool smooth = live && !clamped;
                const float d_o = smooth ? dalpha * w * Gv : 0.0f;
                const float dG = d_o * o;  // dl/dG * G
                // dl/dmu = Q sum dG d and dl/dQ = -1/2 sum dG d d^T over the
                // pixels (d = q - mu): the sums are taken of the moments, and
                // the Gaussian's conic is applied once per Gaussian after them
                const float gx = dG * dx, gy = dG * dy;
                if (r != -1) {
                    const float dgm = (smooth && gam < 1.0f) ? (own ? 1.0f : -1.0f) * dalpha * o * Gv : 0.0f;
                    if (mapped && !tracked && __any(dgm != 0.0f)) {  // the arg-min where it is needed
                        if (dgm != 0.0f) gamma_lds(B, st, bs0, r, lx, ly, &arg);
                    }
                    if (tracked) {
                        if (__any(dgm != 0.0f)) dgr[r] += dgm;  // only near the run's boundary points
                    } else if (dgm != 0.0f && arg >= 0) {
                        float ddx, ddy, sg;
                        const int bpix = (int)st.b_list[bs0 + arg];
                        if (r >= 0) {
                            ddx = (float)(lx - lo16(B.bxy[arg])) - B.bdx[arg];
                            ddy = (float)(ly - hi16(B.bxy[arg])) - B.bdy[arg];
                            sg = B.bs[arg];
                        } else {
                            const float4 r0 = st.rec[(int64_t)bpix * 4];
                            const float4 r2 = st.rec[(int64_t)bpix * 4 + 2];
                            const int a = __float_as_int(r2.w);
                            ddx = (float)(px - lo16(a)) - r0.x;
                            ddy = (float)(py - hi16(a)) - r0.y;
                            sg = r2.z;
                        }
                        const float d = bdist(ddx, ddy);
                        const float gb = gamma_fn(d, sg);  // gamma of the routed point
                        const float dd = dgm * LN2 / sg * gb;
                        float *dst = st.dbound + (int64_t)bpix * 3;
                        if (d > kDKink) {
                            unsafeAtomicAdd(&dst[1], -dd * ddx / d);
                            unsafeAtomicAdd(&dst[2], -dd * ddy / d);
                        }
                        unsafeAtomicAdd(&dst[0], -dgm * LN2 * d / (sg * sg) * gb);
                    }
                }
                // wave totals, scattered over the lanes of row 0 with bit 2 set,
                // go to the entry's LDS sums: nine single-lane adds in two
                // instructions
                float vals[9] = {gx, gy, gx * dx, gx * dy, gy * dy, d_c0, d_c1, d_c2, d_o};
                row_reduce_scatter9(vals, lane);
                vals[0] = cross_row_sum_bp(vals[0], lane);
                vals[8] = cross_row_sum_bp(vals[8], lane);
                if constexpr (ONE) {
                    const int rec = __builtin_amdgcn_readlane(cur_gp, kk);  // the entry's loader holds it
                    if (lane < 16 && (lane & 4)) {
                        const int f = ((lane >> 1) & 4) | (lane & 2) | (lane & 1);
                        if ((wide_b >> kk) & 1ull) {
                            float *dst = st.gwide + (int64_t)rec * kSums;
                            unsafeAtomicAdd(&dst[f], vals[0]);
                            if (lane == 4) unsafeAtomicAdd(&dst[8], vals[8]);
                        } else {
                            float *dst = gs_tile + (int64_t)rec * kSums;
                            dst[f] = vals[0];
                            if (lane == 4) dst[8] = vals[8];
                        }
                    }
                    stored |= 1ull << kk;
                } else if (lane < 16 && (lane & 4)) {
                    float *dst = acc + kk * 9;
                    atomicAdd(&dst[((lane >> 1) & 4) | (lane & 2) | (lane & 1)], vals[0]);
                    if (lane == 4) atomicAdd(&dst[8], vals[8]);
                }
            }
        }
        __syncthreads();
        // the next batch is staged before this batch's sums are stored: a
        // load issued after the stores would wait for them too (acc is not
        // part of the stage)
        const int next_gp = (tid < K && base + K + tid < nlast) ? (int)st.g_list[gs0 + base + K + tid] : -1;
        bool next_wide = false;
        if (next_gp >= 0) next_wide = load_stage<TS, K>(S, st, next_gp, tid, ox, oy, B.run_prim, n_full, slow_b);
        if (tid < K && cur_gp >= 0) {  // each loader stores its own entry's sums
            const bool wide_me = (wide_b >> lane) & 1ull;
            if constexpr (ONE) {
                // zero sums for the entries the wave skipped
                if (!wide_me && !((stored >> tid) & 1ull)) zero_sums(gs_tile + (int64_t)cur_gp * kSums);
            } else {
                float *a = acc + tid * 9;
                if (wide_me) {
                    float *dst = st.gwide + (int64_t)cur_gp * kSums;
#pragma unroll
                    for (int f = 0; f < 9; ++f)
                        if (a[f] != 0.f) unsafeAtomicAdd(&dst[f], a[f]);
                } else {
                    float *dst = gs_tile + (int64_t)cur_gp * kSums;
#pragma unroll
                    for (int f = 0; f < 9; ++f) dst[f] = a[f];
                }
#pragma unroll
                for (int f = 0; f < 9; ++f) a[f] = 0.f;
            }
        }
        cur_gp = next_gp;
        wide_b = __ballot(next_wide);
    }
    // boundary points at the arg-min of each (run, pixel): d gamma / d b, d sigma.
    // The arg-min is searched again over the run (gamma_lds: the smallest
    // d/sigma, near-ties decided in FP64, the lowest raster index among
    // exactly equal ratios).
    __syncthreads();  // the loaders' last flush reads acc, which bacc overlays
    constexpr int BCAP = BoundaryCap<TS, K>::value;
    float(&bacc)[BCAP][3] = U.bacc;
    for (int i = tid; i < BCAP * 3; i += blockDim.x) (&bacc[0][0])[i] = 0.f;
    __syncthreads();
    const int nmap = B.n_runs < RD ? B.n_runs : RD;
    for (int r = 0; r < nmap; ++r) {  // not unrolled: one copy of the arg-min search
        float dg = 0.f;               // dgr[r] by selects (r is uniform; dgr stays in registers)
#pragma unroll
        for (int i = 0; i < RD; ++i) dg = i == r ? dgr[i] : dg;
        if (dg == 0.f) continue;
        int e = -1;
        const float gst = gamma_lds(B, st, bs0, r, lx, ly, &e);
        if (e < 0 || !(gst < 1.0f)) continue;
        const float ddx = (float)(lx - lo16(B.bxy[e])) - B.bdx[e], ddy = (float)(ly - hi16(B.bxy[e])) - B.bdy[e];
        const float sg = B.bs[e];
        const float d = bdist(ddx, ddy);
        const float gam = gamma_fn(d, sg);  // gamma of the routed point (gamma* up to FP32 rounding)
        const float dd = dg * LN2 / sg * gam;
        if (d > kDKink) {
            atomicAdd(&bacc[e][0], -dd * ddx / d);
            atomicAdd(&bacc[e][1], -dd * ddy / d);
        }
        atomicAdd(&bacc[e][2], -dg * LN2 * d / (sg * sg) * gam);
    }
    __syncthreads();
    for (int e = tid; e < B.nbl; e += blockDim.x) {
        const float a0 = bacc[e][0], a1 = bacc[e][1], a2 = bacc[e][2];
        if (a0 == 0.f && a1 == 0.f && a2 == 0.f) continue;
        float *dst = st.dbound + (int64_t)st.b_list[bs0 + e] * 3;
        if (a0 != 0.f) unsafeAtomicAdd(&dst[1], a0);
        if (a1 != 0.f) unsafeAtomicAdd(&dst[2], a1);
        if (a2 != 0.f) unsafeAtomicAdd(&dst[0], a2);
    }
}

template <int TS, int K>
static hipError_t launch_fwd_t(const Consts &k, const ViewTable &vt, const StatePtrs &st, float *image, hipStream_t s) {
    hipLaunchKernelGGL((k_blend_fwd<TS, K>), dim3(vt.total_tiles), dim3(TS * TS), 0, s, k, vt, st, image);
    return hipGetLastError();
}

template <int TS, int K>
static hipError_t launch_bwd_t(const Consts &k, const ViewTable &vt, const StatePtrs &st, const float *image,
                               const float *grad, hipStream_t s) {
    hipLaunchKernelGGL((k_blend_bwd<TS, K>), dim3(vt.total_tiles), dim3(TS * TS), 0, s, k, vt, st, image, grad);
    return hipGetLastError();
}

// (tile, batch) pairs with a kernel; a batch is loaded by one thread per
// slot, so it cannot exceed the tile's pixel count
#define BGT_BLEND_CONFIGS(X) X(8, 32) X(8, 64) X(16, 32) X(16, 64) X(16, 128) X(32, 32) X(32, 64) X(32, 128)

hipError_t launch_blend_fwd(const Consts &k, const ViewTable &vt, const StatePtrs &st, float *image, hipStream_t s) {
#define BGT_CASE(TS, K) \
    if (k.tile == TS && k.batch == K) return launch_fwd_t<TS, K>(k, vt, st, image, s);
    BGT_BLEND_CONFIGS(BGT_CASE)
#undef BGT_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_blend_bwd(const Consts &k, const ViewTable &vt, const StatePtrs &st, const float *image,
                            const float *grad_image, hipStream_t s) {
#define BGT_CASE(TS, K) \
    if (k.tile == TS && k.batch == K) return launch_bwd_t<TS, K>(k, vt, st, image, grad_image, s);
    BGT_BLEND_CONFIGS(BGT_CASE)
#undef BGT_CASE
    return hipErrorInvalidValue;
}

}  // namespace bgt
