// Discontinuity-aware alpha blending (Sec. 3.2, Eq. 6-8) and its backward
// pass (Supplementary Sec. C) on gfx950.
//
// One workgroup renders one TSxTS tile; each wave owns an 8x8 pixel block.
// The tile's boundary points (sorted by primitive id) are staged in LDS and
// split into runs of equal id.  For every run r the block builds
//     gamma*_r(q) = min over the run's points b of min(2^(|q-b|/sigma_b - 1), 1)
// for all pixels q of the tile by a scatter-min from each point over the
// pixels of its disc (LDS atomics), so the blend loop reads w from LDS
// instead of searching boundary points per (pixel, Gaussian) pair; a
// Gaussian of primitive g finds its run by binary search over the run ids.
// Gaussians are then composited front to back in LDS-staged batches; a wave
// skips any Gaussian whose pixel range misses its 8x8 block.
#include "bgt_internal.h"

namespace bgt {

// Per tile size: runs with an LDS gamma* map and boundary points staged in
// LDS.  The budget keeps 5-6 workgroups per CU; on the 2000-patch sphere at
// 16 px a tile has at most 13 runs and 157 points (the 20,000-patch box: 24
// and 251).  Tiles beyond it take the slower paths, never a wrong one.
template <int TS>
struct RunMaps {
    static constexpr int value = TS >= 32 ? 4 : 12;
};
template <int TS>
struct BoundaryCap {
    static constexpr int value = TS >= 32 ? 512 : (TS >= 16 ? 256 : 128);
};

template <int TS>
struct TileGeom {
    static constexpr int NT = TS * TS;
    static constexpr int SPR = TS / 8;  // 8x8 sub-blocks per row
    __device__ static __forceinline__ void local_xy(int tid, int &lx, int &ly) {
        const int wave = tid >> 6, lane = tid & 63;
        lx = (wave % SPR) * 8 + (lane & 7);
        ly = (wave / SPR) * 8 + (lane >> 3);
    }
    __device__ static __forceinline__ int tid_of(int lx, int ly) {
        return ((ly >> 3) * SPR + (lx >> 3)) * 64 + (ly & 7) * 8 + (lx & 7);
    }
};

// boundary staging shared by forward and backward
// Boundary point e sits at pixel (bix, biy) (tile-relative) plus the offset
// (bdx, bdy) of its projected position from that pixel's centre; distances
// to pixel (x, y) are (x - bix) - bdx etc., an exact integer minus one float,
// so every value depends only on the point and the pixel, never on the tile.
template <int TS, typename MapT>
struct BoundaryLds {
    static constexpr int CAP = BoundaryCap<TS>::value;
    float bdx[CAP], bdy[CAP], bs[CAP];
    int bxy[CAP];  // tile-relative pixel x | y << 16 (int16 each)
    int bp[CAP], brun[CAP];
    int run_prim[CAP], run_start[CAP + 1];
    int wsum[33];
    int n_runs, nbl;
    MapT map[RunMaps<TS>::value][TS * TS];
};

// A staged Gaussian's mean is kept per wave as (g - w0) + delta, where g is
// the Gaussian's own pixel, w0 the origin of the wave's 8x8 block and delta
// the mean's offset from g's centre: one rounding that does not depend on
// the tile size.
// A staged Gaussian's mean is kept per wave as (g - w0) + delta, where g is
// the Gaussian's own pixel, w0 the origin of the wave's 8x8 block and delta
// the mean's offset from g's centre: one rounding that does not depend on
// the tile size.
template <int TS, int K>
struct BatchLds {
    float2 m[TS * TS / 64][K];  // per-wave mean offsets
    float4 e[K];                // conic in exponent form kE (a, 2b, c), opacity
    float4 c[K];                // colour, unused
    int2 pr[K];                 // primitive id, run index
    int xr[K], yr[K];
};

// -log2(e)/2: G = exp(-d^T Q d / 2) = 2^(kE d^T Q d)
constexpr float kE = -0.5f * 1.44269504088896341f;

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
template <int TS, typename MapT>
__device__ __forceinline__ void stage_boundary(BoundaryLds<TS, MapT> &B, const StatePtrs &st, int bs0, int bc,
                                               int ox, int oy, const ViewInfo &vi) {
    const int nbl = bc < B.CAP ? bc : B.CAP;
    for (int e = threadIdx.x; e < nbl; e += blockDim.x) {
        const int bpix = (int)st.b_list[bs0 + e];
        const float4 r0 = st.rec[(int64_t)bpix * 4];
        const float4 r2 = st.rec[(int64_t)bpix * 4 + 2];
        const int lp = bpix - vi.px_off;
        B.bxy[e] = pack16(lp % vi.W - ox, lp / vi.W - oy);  // relative to the tile origin
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
            if (f) { B.run_prim[nr0 + ex] = B.bp[e]; B.run_start[nr0 + ex] = e; }
            B.brun[e] = nr0 + ex + f - 1;
        }
        __syncthreads();
        if (threadIdx.x == 0) B.n_runs = nr0 + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) { B.run_start[B.n_runs] = nbl; B.nbl = nbl; }
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

// gamma* from the LDS points of run r (runs without a map); *arg = entry
template <int TS, typename MapT>
__device__ __forceinline__ float gamma_lds(const BoundaryLds<TS, MapT> &B, int r, int lx, int ly, int *arg) {
    float best = 1.0f;
    *arg = -1;
    for (int e = B.run_start[r]; e < B.run_start[r + 1]; ++e) {
        const float dx = (float)(lx - lo16(B.bxy[e])) - B.bdx[e], dy = (float)(ly - hi16(B.bxy[e])) - B.bdy[e];
        const float g = gamma_fn(bdist(dx, dy), B.bs[e]);
        if (g < best) { best = g; *arg = e; }
    }
    return best;
}

// gamma* straight from global memory (tiles with more boundary points than
// the LDS stage holds); *arg = entry index in the tile's list
__device__ __forceinline__ float gamma_global(const StatePtrs &st, const ViewInfo &vi, int bs0, int bc, int g,
                                              int px, int py, int *arg) {
    int lo = 0, hi = bc;  // first entry with prim >= g
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int pm = __float_as_int(st.rec[(int64_t)st.b_list[bs0 + mid] * 4 + 2].y);
        if (pm < g) lo = mid + 1; else hi = mid;
    }
    float best = 1.0f;
    *arg = -1;
    for (int e = lo; e < bc; ++e) {
        const int bpix = (int)st.b_list[bs0 + e];
        const float4 r2 = st.rec[(int64_t)bpix * 4 + 2];
        if (__float_as_int(r2.y) != g) break;
        const float4 r0 = st.rec[(int64_t)bpix * 4];
        const int lp = bpix - vi.px_off;
        const float dx = (float)(px - lp % vi.W) - r0.x, dy = (float)(py - lp / vi.W) - r0.y;
        const float gm = gamma_fn(bdist(dx, dy), r2.z);
        if (gm < best) { best = gm; *arg = e; }
    }
    return best;
}

// Scatter-min of every staged point over the pixels of its disc.
// MapT = unsigned (gamma bits) or unsigned long long (gamma bits << 32 | entry).
template <int TS, typename MapT>
__device__ __forceinline__ void build_gamma_maps(BoundaryLds<TS, MapT> &B) {
    using G = TileGeom<TS>;
    const int nmap = B.n_runs < RunMaps<TS>::value ? B.n_runs : RunMaps<TS>::value;
    for (int i = threadIdx.x; i < nmap * G::NT; i += blockDim.x) {
        if (sizeof(MapT) == 4) B.map[i / G::NT][i % G::NT] = (MapT)0x3F800000u;
        else B.map[i / G::NT][i % G::NT] = (MapT)(0x3F800000ull << 32) | (MapT)0xFFFFFFFFull;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < B.nbl; e += blockDim.x) {
        const int r = B.brun[e];
        if (r >= RunMaps<TS>::value) continue;
        const int bix = lo16(B.bxy[e]), biy = hi16(B.bxy[e]);
        const float bdx = B.bdx[e], bdy = B.bdy[e], sg = B.bs[e];
        const float rf = sg + fabsf(bdx) + fabsf(bdy);
        const int rad = rf < (float)(2 * TS) ? (int)ceilf(rf) + 1 : 2 * TS;  // NaN/inf -> whole tile
        const int x0 = max(bix - rad, 0), x1 = min(bix + rad, TS - 1);
        const int y0 = max(biy - rad, 0), y1 = min(biy + rad, TS - 1);
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) {
                const float dx = (float)(x - bix) - bdx, dy = (float)(y - biy) - bdy;
                const float d = bdist(dx, dy);
                if (d < sg) {
                    const float g = gamma_fn(d, sg);
                    if (g < 1.0f) {
                        if (sizeof(MapT) == 4)
                            atomicMin((unsigned *)&B.map[r][G::tid_of(x, y)], __float_as_uint(g));
                        else
                            atomicMin((unsigned long long *)&B.map[r][G::tid_of(x, y)],
                                      ((unsigned long long)__float_as_uint(g) << 32) | (unsigned long long)e);
                    }
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

template <int TS, int K>
__device__ __forceinline__ void stage_slot(BatchLds<TS, K> &S, const SlotPrefetch &P, const ViewInfo &vi, int kk,
                                           int ox, int oy, const int *run_prim, int n_runs, bool slow_b) {
    using G = TileGeom<TS>;
    const int gp = P.gp;
    const int lp = gp - vi.px_off;
    const int x = lp % vi.W - ox, y = lp / vi.W - oy;  // tile-relative pixel of the Gaussian
#pragma unroll
    for (int w = 0; w < G::NT / 64; ++w)
        S.m[w][kk] = make_float2((float)(x - (w % G::SPR) * 8) + P.r0.x, (float)(y - (w / G::SPR) * 8) + P.r0.y);
    S.e[kk] = make_float4(kE * P.r0.z, 2.0f * kE * P.r0.w, kE * P.r1.x, P.r2.x);
    S.c[kk] = make_float4(P.r1.y, P.r1.z, P.r1.w, 0.f);
    const int g = __float_as_int(P.r2.y);
    S.pr[kk] = make_int2(g, slow_b ? -2 : find_run(run_prim, n_runs, g));
    S.xr[kk] = __float_as_int(P.r3.x);
    S.yr[kk] = __float_as_int(P.r3.y);
}

// does the pixel range (packed int16 pairs) touch the 8x8 block at (x0, y0)?
__device__ __forceinline__ bool touches_block(int xr, int yr, int x0, int y0) {
    return !(hi16(xr) < x0 || lo16(xr) > x0 + 7 || hi16(yr) < y0 || lo16(yr) > y0 + 7);
}

// Nine sums over the wave at once, step-major, so that consecutive DPP adds
// are independent (no hazard stalls between the steps of one sum).
__device__ __forceinline__ void wave_sum9_to_63(float *v);

template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f(float v) {
    // bound_ctrl: lanes whose source is outside the row/wave read 0
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true));
}

// Sum over the 64 lanes with DPP: row shifts leave each 16-lane row's sum in
// its lane 15, then two row broadcasts add rows 0-2 into lane 63.  Only lane
// 63's result is meaningful (the other lanes hold partial sums).
__device__ __forceinline__ float wave_sum_to_63(float v) {
    v += dpp_f<0x111, 0xF>(v);  // row_shr:1
    v += dpp_f<0x112, 0xF>(v);  // row_shr:2
    v += dpp_f<0x114, 0xF>(v);  // row_shr:4
    v += dpp_f<0x118, 0xF>(v);  // row_shr:8
    v += dpp_f<0x142, 0xF>(v);  // row_bcast:15: lane 63 += lane 47 (row 2)
    v += dpp_f<0x143, 0xF>(v);  // row_bcast:31: lane 63 += lane 31 (rows 0 + 1)
    return v;
}

template <int CTRL>
__device__ __forceinline__ void dpp_step9(float *v) {
#pragma unroll
    for (int i = 0; i < 9; ++i) v[i] += dpp_f<CTRL, 0xF>(v[i]);
}

__device__ __forceinline__ void wave_sum9_to_63(float *v) {
    dpp_step9<0x111>(v);  // row_shr:1
    dpp_step9<0x112>(v);  // row_shr:2
    dpp_step9<0x114>(v);  // row_shr:4
    dpp_step9<0x118>(v);  // row_shr:8
    dpp_step9<0x142>(v);  // row_bcast:15
    dpp_step9<0x143>(v);  // row_bcast:31
}

// ------------------------------------------------------------ forward

template <int TS, int K>
__global__ void __launch_bounds__(TS *TS) k_blend_fwd(Consts k, ViewTable vt, StatePtrs st, float *image) {
    using G = TileGeom<TS>;
    __shared__ BoundaryLds<TS, unsigned> B;
    __shared__ BatchLds<TS, K> S;
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
    stage_boundary<TS>(B, st, bs0, bc, ox, oy, vi);
    const bool slow_b = bc > BoundaryCap<TS>::value;
    if (slow_b && tid == 0) atomicAdd((unsigned long long *)&st.counters[C_BIGBLIST], 1ull);
    build_gamma_maps<TS>(B);

    const int gs0 = st.g_start[t], gc = st.g_count[t];
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    bool done = !inside;
    int last = gc;
    const float amax = k.alpha_max, tmin = k.t_min;
    // support test d^T Q d <= 2 ln(1/g_min) as a base-2 exponent: G = 2^e, e >= log2(g_min)
    const float e_min = kE * k.kappa2;
    SlotPrefetch pf;
    pf.gp_next = (tid < K && tid < gc) ? (int)st.g_list[gs0 + tid] : -1;
    pf.issue(st, gs0, gc, 0, tid, K);
    if (pf.gp >= 0) stage_slot<TS, K>(S, pf, vi, tid, ox, oy, B.run_prim, B.n_runs, slow_b);
    for (int base = 0; base < gc; base += K) {
        if (__syncthreads_and(done ? 1 : 0)) break;  // also publishes the staged batch
        pf.issue(st, gs0, gc, base + K, tid, K);     // next batch's records, in flight during compositing
        const int nk = min(K, gc - base);
        if (!__all(done)) {
        for (int c0 = 0; c0 < K; c0 += 64) {
            const int j = c0 + lane, jj = j < K ? j : K - 1;
            unsigned long long mask = __ballot(j < nk && touches_block(S.xr[jj], S.yr[jj], wx0, wy0));
            if (!mask) continue;
            // software pipeline: the next Gaussian's LDS record is read while
            // the current one is composited
            int kk = c0 + __ffsll((long long)mask) - 1;
            mask &= mask - 1;
            int2 pr = S.pr[kk];
            float2 m = S.m[wave][kk];
            float4 ex = S.e[kk];
            float4 c = S.c[kk];
            while (true) {
                const int kn = mask ? c0 + __ffsll((long long)mask) - 1 : -1;
                int2 pr_n = pr;
                float2 m_n = m;
                float4 ex_n = ex, c_n = c;
                if (kn >= 0) {
                    mask &= mask - 1;
                    pr_n = S.pr[kn];
                    m_n = S.m[wave][kn];
                    ex_n = S.e[kn];
                    c_n = S.c[kn];
                }
                const int g = pr.x, r = pr.y;
                if (!done && (g == h || r != -1)) {  // else w = 0: no boundary point of g near this tile
                    const float dx = qx - m.x, dy = qy - m.y;
                    const float e = fmaf(dx, fmaf(ex.x, dx, ex.y * dy), ex.z * dy * dy);
                    if (e >= e_min) {
                        float gam = 1.0f;
                        if (r >= 0) {
                            int arg;
                            gam = r < RunMaps<TS>::value ? __uint_as_float(B.map[r][tid])
                                                         : gamma_lds<TS>(B, r, lx, ly, &arg);
                        } else if (r == -2) {
                            int arg;
                            gam = gamma_global(st, vi, bs0, bc, g, px, py, &arg);
                        }
                        const float w = g == h ? gam : 1.0f - gam;
                        if (w > 0.0f) {
                            float a = ex.w * w * exp2f(e);
                            a = a > amax ? amax : a;
                            const float ta = T * a;
                            C0 += ta * c.x;
                            C1 += ta * c.y;
                            C2 += ta * c.z;
                            T = T * (1.0f - a);
                            if (T < tmin) { done = true; last = base + kk + 1; }
                        }
                    }
                }
                if (kn < 0) break;
                kk = kn; pr = pr_n; m = m_n; ex = ex_n; c = c_n;
            }
        }
        }
        __syncthreads();  // everyone is done with this batch
        if (pf.gp >= 0) stage_slot<TS, K>(S, pf, vi, tid, ox, oy, B.run_prim, B.n_runs, slow_b);
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
// forward colour minus the running prefix, and
//   dl/dc_i = T_i a_i dl/dC,  dl/da_i = dl/dC . (T_i c_i - S_i / (1 - a_i)),
//   dl/dw = dl/da a / w (Supplementary Sec. C), G = exp(-d^T Q d / 2).
// Per Gaussian the 9 gradient values are summed over the wave with DPP and
// over the waves in LDS, then added to global memory once per tile.  The
// boundary terms accumulate per (run, pixel) and go to the minimising
// boundary point at the end of the tile.
template <int TS, int K>
__global__ void __launch_bounds__(TS *TS) k_blend_bwd(Consts k, ViewTable vt, StatePtrs st, const float *image,
                                                     const float *grad_image) {
    using G = TileGeom<TS>;
    constexpr int RM = RunMaps<TS>::value;
    __shared__ BoundaryLds<TS, unsigned> B;
    // the batch stage and its gradient sums are dead once the list is done;
    // the per-point boundary sums reuse their space
    struct LoopLds {
        BatchLds<TS, K> S;
        float acc[K][9];
    };
    union TailLds {
        LoopLds loop;
        float bacc[BoundaryCap<TS>::value][3];
    };
    __shared__ TailLds U;
    __shared__ int max_last;
    BatchLds<TS, K> &S = U.loop.S;
    float(&acc)[K][9] = U.loop.acc;
    float dgam[RM];  // per-run sums of dl/dgamma* at this pixel (registers, uniform index)
#pragma unroll
    for (int i = 0; i < RM; ++i) dgam[i] = 0.f;
    const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int v = view_of_tile(vt, t);
    const ViewInfo vi = vt.v[v];
    const int tl = t - vi.tile_off, tx = tl % vi.tiles_x, ty = tl / vi.tiles_x;
    int lx, ly;
    G::local_xy(tid, lx, ly);
    const int px = tx * TS + lx, py = ty * TS + ly;
    const bool inside = px < vi.W && py < vi.H;
    const int pix = vi.px_off + py * vi.W + px;
    const int gc = st.g_count[t];
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

    if (tid == 0) max_last = 0;
    for (int i = tid; i < K * 9; i += blockDim.x) (&acc[0][0])[i] = 0.f;
    __syncthreads();
    atomicMax(&max_last, mylast);
    int wave_last = mylast;  // last list entry any lane of this wave replays
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) wave_last = max(wave_last, __shfl_xor(wave_last, o, 64));

    const int bs0 = st.b_start[t], bc = st.b_count[t];
    stage_boundary<TS>(B, st, bs0, bc, ox, oy, vi);  // (syncs)
    const bool slow_b = bc > BoundaryCap<TS>::value;
    build_gamma_maps<TS>(B);

    const int gs0 = st.g_start[t];
    const int nlast = max_last;
    float T = 1.0f, P0 = 0.f, P1 = 0.f, P2 = 0.f;
    const float amax = k.alpha_max;
    const float e_min = kE * k.kappa2;
    const float LN2 = 0.69314718055994531f;
    SlotPrefetch pf;
    pf.gp_next = (tid < K && tid < nlast) ? (int)st.g_list[gs0 + tid] : -1;
    pf.issue(st, gs0, nlast, 0, tid, K);
    if (pf.gp >= 0) stage_slot<TS, K>(S, pf, vi, tid, ox, oy, B.run_prim, B.n_runs, slow_b);
    for (int base = 0; base < nlast; base += K) {
        __syncthreads();  // publishes the staged batch
        const int cur_gp = pf.gp;
        pf.issue(st, gs0, nlast, base + K, tid, K);  // next batch's records, in flight during the replay
        const int nk = min(K, nlast - base);
        for (int c0 = 0; c0 < K && base + c0 < wave_last; c0 += 64) {
            const int j = c0 + lane, jj = j < K ? j : K - 1;
            unsigned long long mask =
                __ballot(j < nk && base + j < wave_last && touches_block(S.xr[jj], S.yr[jj], wx0, wy0));
            while (mask) {
                const int kk = c0 + __ffsll((long long)mask) - 1;
                mask &= mask - 1;
                float d_mx = 0.f, d_my = 0.f, d_qa = 0.f, d_qb = 0.f, d_qc = 0.f, d_c0 = 0.f, d_c1 = 0.f, d_c2 = 0.f,
                      d_o = 0.f;
                bool contrib = false;
                const int2 prk = S.pr[kk];
                const int g = prk.x;
                const int r = __builtin_amdgcn_readfirstlane(prk.y);  // wave-uniform
                if (base + kk < mylast && (g == h || r != -1)) {
                    const float2 m = S.m[wave][kk];
                    const float4 ex = S.e[kk];
                    const float dx = qx - m.x, dy = qy - m.y;
                    const float e = fmaf(dx, fmaf(ex.x, dx, ex.y * dy), ex.z * dy * dy);  // as in the forward
                    if (e >= e_min) {
                        float gam = 1.0f;
                        int arg = -1;
                        if (r >= 0) {
                            gam = r < RM ? __uint_as_float(B.map[r][tid]) : gamma_lds<TS>(B, r, lx, ly, &arg);
                        } else if (r == -2) {
                            gam = gamma_global(st, vi, bs0, bc, g, px, py, &arg);
                        }
                        const float w = g == h ? gam : 1.0f - gam;
                        if (w > 0.0f) {
                            contrib = true;
                            // conic back from its exponent form
                            const float4 q = make_float4(ex.x * (1.0f / kE), ex.y * (0.5f / kE), ex.z * (1.0f / kE), ex.w);
                            const float Gv = exp2f(e);
                            const float o = q.w;
                            const float raw = o * w * Gv;
                            const bool clamped = raw > amax;
                            const float a = clamped ? amax : raw;
                            const float ta = T * a;
                            const float4 c = S.c[kk];
                            d_c0 = ta * g0; d_c1 = ta * g1; d_c2 = ta * g2;
                            P0 += ta * c.x; P1 += ta * c.y; P2 += ta * c.z;
                            const float inv = __builtin_amdgcn_rcpf(1.0f - a);
                            const float dalpha = g0 * (T * c.x - (im0 - P0) * inv) + g1 * (T * c.y - (im1 - P1) * inv) +
                                                 g2 * (T * c.z - (im2 - P2) * inv);
                            T = T * (1.0f - a);
                            if (!clamped) {
                                d_o = dalpha * w * Gv;
                                const float dG = d_o * o;  // dl/dG * G
                                d_mx = dG * (q.x * dx + q.y * dy);
                                d_my = dG * (q.y * dx + q.z * dy);
                                d_qa = -0.5f * dG * dx * dx;
                                d_qb = -dG * dx * dy;
                                d_qc = -0.5f * dG * dy * dy;
                                if (r != -1 && gam < 1.0f) {
                                    const float dgm = (g == h ? 1.0f : -1.0f) * dalpha * o * Gv;
                                    if (r >= 0 && r < RM) {
                                        dgam[r] += dgm;  // r is wave-uniform: indexed register access
                                    } else if (arg >= 0) {
                                        // no map for this run: push the boundary-point gradient now
                                        float ddx, ddy, sg;
                                        const int bpix = (int)st.b_list[bs0 + arg];
                                        if (r >= 0) {
                                            ddx = (float)(lx - lo16(B.bxy[arg])) - B.bdx[arg];
                                            ddy = (float)(ly - hi16(B.bxy[arg])) - B.bdy[arg];
                                            sg = B.bs[arg];
                                        } else {
                                            const float4 r0 = st.rec[(int64_t)bpix * 4];
                                            const int lp = bpix - vi.px_off;
                                            ddx = (float)(px - lp % vi.W) - r0.x;
                                            ddy = (float)(py - lp / vi.W) - r0.y;
                                            sg = st.rec[(int64_t)bpix * 4 + 2].z;
                                        }
                                        const float d = sqrtf(ddx * ddx + ddy * ddy);
                                        const float dd = dgm * LN2 / sg * gam;
                                        float *dst = st.dgauss + (int64_t)bpix * 12;
                                        if (d > 0.f) {
                                            unsafeAtomicAdd(&dst[0], -dd * ddx / d);
                                            unsafeAtomicAdd(&dst[1], -dd * ddy / d);
                                        }
                                        unsafeAtomicAdd(&dst[9], -dgm * LN2 * d / (sg * sg) * gam);
                                    }
                                }
                            }
                        }
                    }
                }
                if (__any(contrib)) {
                    float vals[9] = {d_mx, d_my, d_qa, d_qb, d_qc, d_c0, d_c1, d_c2, d_o};
                    wave_sum9_to_63(vals);
                    if (lane == 63) {
#pragma unroll
                        for (int f = 0; f < 9; ++f) atomicAdd(&acc[kk][f], vals[f]);
                    }
                }
            }
        }
        __syncthreads();
        if (tid < K && cur_gp >= 0) {  // each loader flushes its own slot, then stages the next batch
#pragma unroll
            for (int f = 0; f < 9; ++f) {
                const float val = acc[tid][f];
                if (val != 0.f) {
                    unsafeAtomicAdd(&st.dgauss[(int64_t)cur_gp * 12 + f], val);
                    acc[tid][f] = 0.f;
                }
            }
        }
        if (pf.gp >= 0) stage_slot<TS, K>(S, pf, vi, tid, ox, oy, B.run_prim, B.n_runs, slow_b);
    }
    // boundary points at the arg-min of each (run, pixel): d gamma / d b, d sigma.
    // The arg-min is searched again over the run (first, i.e. lowest raster
    // index, among equal minima).
    __syncthreads();  // the loaders' last flush reads acc, which bacc overlays
    float(&bacc)[BoundaryCap<TS>::value][3] = U.bacc;
    for (int i = tid; i < BoundaryCap<TS>::value * 3; i += blockDim.x) (&bacc[0][0])[i] = 0.f;
    __syncthreads();
    const int nmap = B.n_runs < RM ? B.n_runs : RM;
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        const float dg = dgam[r];
        if (r >= nmap || dg == 0.f) continue;
        int e = -1;
        const float gam = gamma_lds<TS>(B, r, lx, ly, &e);
        if (e < 0 || !(gam < 1.0f)) continue;
        const float ddx = (float)(lx - lo16(B.bxy[e])) - B.bdx[e], ddy = (float)(ly - hi16(B.bxy[e])) - B.bdy[e];
        const float sg = B.bs[e];
        const float d = sqrtf(ddx * ddx + ddy * ddy);
        const float dd = dg * LN2 / sg * gam;
        if (d > 0.f) {
            atomicAdd(&bacc[e][0], -dd * ddx / d);
            atomicAdd(&bacc[e][1], -dd * ddy / d);
        }
        atomicAdd(&bacc[e][2], -dg * LN2 * d / (sg * sg) * gam);
    }
    __syncthreads();
    for (int e = tid; e < B.nbl; e += blockDim.x) {
        const float a0 = bacc[e][0], a1 = bacc[e][1], a2 = bacc[e][2];
        if (a0 == 0.f && a1 == 0.f && a2 == 0.f) continue;
        float *dst = st.dgauss + (int64_t)st.b_list[bs0 + e] * 12;
        if (a0 != 0.f) unsafeAtomicAdd(&dst[0], a0);
        if (a1 != 0.f) unsafeAtomicAdd(&dst[1], a1);
        if (a2 != 0.f) unsafeAtomicAdd(&dst[9], a2);
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
