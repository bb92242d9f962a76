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

// runs with an LDS gamma* map (fewer for 32x32 tiles to fit the LDS budget)
template <int TS>
struct RunMaps {
    static constexpr int value = TS >= 32 ? 4 : 16;
};
constexpr int kBoundaryLds = 512; // boundary points staged in LDS per tile

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
    float bdx[kBoundaryLds], bdy[kBoundaryLds], bs[kBoundaryLds];
    int bix[kBoundaryLds], biy[kBoundaryLds];
    int bp[kBoundaryLds], brun[kBoundaryLds];
    int run_prim[kBoundaryLds], run_start[kBoundaryLds + 1];
    int wsum[33];
    int n_runs, nbl;
    MapT map[RunMaps<TS>::value][TS * TS];
};

// A staged Gaussian's mean is kept per wave as (g - w0) + delta, where g is
// the Gaussian's own pixel, w0 the origin of the wave's 8x8 block and delta
// the mean's offset from g's centre: one rounding that does not depend on
// the tile size.
template <int TS, int K>
struct BatchLds {
    float mx[TS * TS / 64][K], my[TS * TS / 64][K];
    float qa[K], qb[K], qc[K], cr[K], cg[K], cb[K], op[K];
    int prim[K], run[K], xr[K], yr[K], gp[K];
};

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
    const int nbl = bc < kBoundaryLds ? bc : kBoundaryLds;
    for (int e = threadIdx.x; e < nbl; e += blockDim.x) {
        const int bpix = (int)st.b_list[bs0 + e];
        const float4 r0 = st.rec[(int64_t)bpix * 4];
        const float4 r2 = st.rec[(int64_t)bpix * 4 + 2];
        const int lp = bpix - vi.px_off;
        B.bix[e] = lp % vi.W - ox;  // relative to the tile origin
        B.biy[e] = lp / vi.W - oy;
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

__device__ __forceinline__ float gamma_fn(float d, float sigma) {
    const float g = exp2f(d / sigma - 1.0f);
    return g < 1.0f ? g : 1.0f;
}

// gamma* from the LDS points of run r (runs without a map); *arg = entry
template <int TS, typename MapT>
__device__ __forceinline__ float gamma_lds(const BoundaryLds<TS, MapT> &B, int r, int lx, int ly, int *arg) {
    float best = 1.0f;
    *arg = -1;
    for (int e = B.run_start[r]; e < B.run_start[r + 1]; ++e) {
        const float dx = (float)(lx - B.bix[e]) - B.bdx[e], dy = (float)(ly - B.biy[e]) - B.bdy[e];
        const float g = gamma_fn(sqrtf(dx * dx + dy * dy), B.bs[e]);
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
        const float gm = gamma_fn(sqrtf(dx * dx + dy * dy), r2.z);
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
        const int bix = B.bix[e], biy = B.biy[e];
        const float bdx = B.bdx[e], bdy = B.bdy[e], sg = B.bs[e];
        const float rf = sg + fabsf(bdx) + fabsf(bdy);
        const int rad = rf < (float)(2 * TS) ? (int)ceilf(rf) + 1 : 2 * TS;  // NaN/inf -> whole tile
        const int x0 = max(bix - rad, 0), x1 = min(bix + rad, TS - 1);
        const int y0 = max(biy - rad, 0), y1 = min(biy + rad, TS - 1);
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) {
                const float dx = (float)(x - bix) - bdx, dy = (float)(y - biy) - bdy;
                const float d = sqrtf(dx * dx + dy * dy);
                if (d < sg) {
                    const float g = exp2f(d / sg - 1.0f);
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

template <int TS, int K>
__device__ __forceinline__ void load_batch(BatchLds<TS, K> &S, const StatePtrs &st, const ViewInfo &vi, int gs0,
                                           int i, int kk, int ox, int oy, const int *run_prim, int n_runs,
                                           bool slow_b) {
    using G = TileGeom<TS>;
    const int gp = (int)st.g_list[gs0 + i];
    const float4 *rp = st.rec + (int64_t)gp * 4;
    const float4 r0 = rp[0], r1 = rp[1], r2 = rp[2], r3 = rp[3];
    const int lp = gp - vi.px_off;
    const int x = lp % vi.W - ox, y = lp / vi.W - oy;  // tile-relative pixel of the Gaussian
#pragma unroll
    for (int w = 0; w < G::NT / 64; ++w) {
        S.mx[w][kk] = (float)(x - (w % G::SPR) * 8) + r0.x;
        S.my[w][kk] = (float)(y - (w / G::SPR) * 8) + r0.y;
    }
    S.qa[kk] = r0.z; S.qb[kk] = r0.w; S.qc[kk] = r1.x;
    S.cr[kk] = r1.y; S.cg[kk] = r1.z; S.cb[kk] = r1.w;
    S.op[kk] = r2.x;
    const int g = __float_as_int(r2.y);
    S.prim[kk] = g;
    S.run[kk] = slow_b ? -2 : find_run(run_prim, n_runs, g);
    S.xr[kk] = __float_as_int(r3.x);
    S.yr[kk] = __float_as_int(r3.y);
    S.gp[kk] = gp;
}

// ------------------------------------------------------------ forward

template <int TS, int K>
__global__ void __launch_bounds__(TS *TS) k_blend_fwd(Consts k, ViewTable vt, StatePtrs st, float *image) {
    using G = TileGeom<TS>;
    __shared__ BoundaryLds<TS, unsigned> B;
    __shared__ BatchLds<TS, K> S;
    const int t = blockIdx.x, tid = threadIdx.x;
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
    const int wave = tid >> 6;
    const int wx0 = tx * TS + (wave % G::SPR) * 8, wy0 = ty * TS + (wave / G::SPR) * 8;

    const int bs0 = st.b_start[t], bc = st.b_count[t];
    stage_boundary<TS>(B, st, bs0, bc, ox, oy, vi);
    const bool slow_b = bc > kBoundaryLds;
    if (slow_b && tid == 0) atomicAdd((unsigned long long *)&st.counters[C_BIGBLIST], 1ull);
    build_gamma_maps<TS>(B);

    const int gs0 = st.g_start[t], gc = st.g_count[t];
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    bool done = !inside;
    int last = gc;
    const float kappa2 = k.kappa2, amax = k.alpha_max, tmin = k.t_min;
    for (int base = 0; base < gc; base += K) {
        if (__syncthreads_and(done ? 1 : 0)) break;
        if (tid < K && base + tid < gc) load_batch<TS, K>(S, st, vi, gs0, base + tid, tid, ox, oy, B.run_prim, B.n_runs, slow_b);
        __syncthreads();
        const int nk = min(K, gc - base);
        if (!done) {
            for (int kk = 0; kk < nk; ++kk) {
                const int xr = S.xr[kk], yr = S.yr[kk];
                if (hi16(xr) < wx0 || lo16(xr) > wx0 + 7 || hi16(yr) < wy0 || lo16(yr) > wy0 + 7) continue;
                const int g = S.prim[kk], r = S.run[kk];
                if (g != h && r == -1) continue;  // w = 0: no boundary of g near this tile
                const float dx = qx - S.mx[wave][kk], dy = qy - S.my[wave][kk];
                const float power = S.qa[kk] * dx * dx + 2.0f * S.qb[kk] * dx * dy + S.qc[kk] * dy * dy;
                if (power > kappa2) continue;
                float gam = 1.0f;
                if (r >= 0) {
                    int arg;
                    gam = r < RunMaps<TS>::value ? __uint_as_float(B.map[r][tid]) : gamma_lds<TS>(B, r, lx, ly, &arg);
                } else if (r == -2) {
                    int arg;
                    gam = gamma_global(st, vi, bs0, bc, g, px, py, &arg);
                }
                const float w = g == h ? gam : 1.0f - gam;
                if (w <= 0.0f) continue;
                const float Gv = __expf(-0.5f * power);
                float a = S.op[kk] * w * Gv;
                a = a > amax ? amax : a;
                const float ta = T * a;
                C0 += ta * S.cr[kk];
                C1 += ta * S.cg[kk];
                C2 += ta * S.cb[kk];
                T = T * (1.0f - a);
                if (T < tmin) { done = true; last = base + kk + 1; break; }
            }
        }
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

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

template <int TS, int K>
__global__ void __launch_bounds__(TS *TS) k_blend_bwd(Consts k, ViewTable vt, StatePtrs st, const float *image,
                                                     const float *grad_image) {
    using G = TileGeom<TS>;
    __shared__ BoundaryLds<TS, unsigned long long> B;
    __shared__ BatchLds<TS, K> S;
    __shared__ float acc[K][9];
    __shared__ float dgam[RunMaps<TS>::value][TS * TS];
    __shared__ float bacc[kBoundaryLds][3];
    __shared__ int max_last;
    const int t = blockIdx.x, tid = threadIdx.x;
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
        mylast = min(max(st.last[pix], 0), st.g_count[t]);
        g0 = grad_image[3 * (int64_t)pix]; g1 = grad_image[3 * (int64_t)pix + 1]; g2 = grad_image[3 * (int64_t)pix + 2];
        im0 = image[3 * (int64_t)pix]; im1 = image[3 * (int64_t)pix + 1]; im2 = image[3 * (int64_t)pix + 2];
        if (g0 == 0.f && g1 == 0.f && g2 == 0.f) mylast = 0;
    }
    const int ox = tx * TS, oy = ty * TS;
    const float qx = (float)(lx & 7), qy = (float)(ly & 7);  // position in the wave's 8x8 block
    const int wave = tid >> 6, lane = tid & 63;
    const int wx0 = tx * TS + (wave % G::SPR) * 8, wy0 = ty * TS + (wave / G::SPR) * 8;

    if (tid == 0) max_last = 0;
    for (int i = tid; i < K * 9; i += blockDim.x) (&acc[0][0])[i] = 0.f;
    for (int i = tid; i < RunMaps<TS>::value * TS * TS; i += blockDim.x) (&dgam[0][0])[i] = 0.f;
    for (int i = tid; i < kBoundaryLds * 3; i += blockDim.x) (&bacc[0][0])[i] = 0.f;
    __syncthreads();
    atomicMax(&max_last, mylast);

    const int bs0 = st.b_start[t], bc = st.b_count[t];
    stage_boundary<TS>(B, st, bs0, bc, ox, oy, vi);  // (syncs)
    const bool slow_b = bc > kBoundaryLds;
    build_gamma_maps<TS>(B);

    const int gs0 = st.g_start[t];
    const int nlast = max_last;
    float T = 1.0f, P0 = 0.f, P1 = 0.f, P2 = 0.f;
    const float kappa2 = k.kappa2, amax = k.alpha_max;
    const float bg0 = k.bg[0], bg1 = k.bg[1], bg2 = k.bg[2];
    (void)bg0; (void)bg1; (void)bg2;
    const float LN2 = 0.69314718055994531f;
    for (int base = 0; base < nlast; base += K) {
        if (tid < K && base + tid < nlast) load_batch<TS, K>(S, st, vi, gs0, base + tid, tid, ox, oy, B.run_prim, B.n_runs, slow_b);
        __syncthreads();
        const int nk = min(K, nlast - base);
        for (int kk = 0; kk < nk; ++kk) {
            const int xr = S.xr[kk], yr = S.yr[kk];
            if (hi16(xr) < wx0 || lo16(xr) > wx0 + 7 || hi16(yr) < wy0 || lo16(yr) > wy0 + 7) continue;  // wave-uniform
            float d_mx = 0.f, d_my = 0.f, d_qa = 0.f, d_qb = 0.f, d_qc = 0.f, d_c0 = 0.f, d_c1 = 0.f, d_c2 = 0.f, d_o = 0.f;
            bool contrib = false;
            if (base + kk < mylast) {
                const int g = S.prim[kk], r = S.run[kk];
                if (!(g != h && r == -1)) {
                    const float dx = qx - S.mx[wave][kk], dy = qy - S.my[wave][kk];
                    const float qa = S.qa[kk], qb = S.qb[kk], qc = S.qc[kk];
                    const float power = qa * dx * dx + 2.0f * qb * dx * dy + qc * dy * dy;
                    if (power <= kappa2) {
                        float gam = 1.0f;
                        int arg = -1;
                        if (r >= 0) {
                            if (r < RunMaps<TS>::value) {
                                const unsigned long long mv = B.map[r][tid];
                                gam = __uint_as_float((unsigned)(mv >> 32));
                                arg = (int)(mv & 0xFFFFFFFFull);
                            } else {
                                gam = gamma_lds<TS>(B, r, lx, ly, &arg);
                            }
                        } else if (r == -2) {
                            gam = gamma_global(st, vi, bs0, bc, g, px, py, &arg);
                        }
                        const float w = g == h ? gam : 1.0f - gam;
                        if (w > 0.0f) {
                            contrib = true;
                            const float Gv = __expf(-0.5f * power);
                            const float o = S.op[kk];
                            const float raw = o * w * Gv;
                            const bool clamped = raw > amax;
                            const float a = clamped ? amax : raw;
                            const float ta = T * a;
                            const float c0 = S.cr[kk], c1 = S.cg[kk], c2 = S.cb[kk];
                            d_c0 = ta * g0; d_c1 = ta * g1; d_c2 = ta * g2;
                            P0 += ta * c0; P1 += ta * c1; P2 += ta * c2;
                            // S_i = sum_{j>i} T_j a_j c_j + T_n bg = C - prefix_{<=i}
                            const float inv = 1.0f / (1.0f - a);
                            const float dalpha = g0 * (T * c0 - (im0 - P0) * inv) + g1 * (T * c1 - (im1 - P1) * inv) +
                                                 g2 * (T * c2 - (im2 - P2) * inv);
                            T = T * (1.0f - a);
                            if (!clamped) {
                                d_o = dalpha * w * Gv;
                                const float dG = dalpha * o * w * Gv;  // dl/dG * G
                                d_mx = dG * (qa * dx + qb * dy);
                                d_my = dG * (qb * dx + qc * dy);
                                d_qa = -0.5f * dG * dx * dx;
                                d_qb = -dG * dx * dy;
                                d_qc = -0.5f * dG * dy * dy;
                                if (arg >= 0 && gam < 1.0f) {
                                    const float dgm = (g == h ? 1.0f : -1.0f) * dalpha * o * Gv;
                                    if (r >= 0 && r < RunMaps<TS>::value) {
                                        dgam[r][tid] += dgm;
                                    } else {
                                        // no map: push the boundary-point gradient now
                                        float ddx, ddy, sg;
                                        const int bpix = (int)st.b_list[bs0 + arg];
                                        if (r >= 0) {
                                            ddx = (float)(lx - B.bix[arg]) - B.bdx[arg];
                                            ddy = (float)(ly - B.biy[arg]) - B.bdy[arg];
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
            }
            if (__any(contrib)) {
                d_mx = wave_sum(d_mx); d_my = wave_sum(d_my);
                d_qa = wave_sum(d_qa); d_qb = wave_sum(d_qb); d_qc = wave_sum(d_qc);
                d_c0 = wave_sum(d_c0); d_c1 = wave_sum(d_c1); d_c2 = wave_sum(d_c2);
                d_o = wave_sum(d_o);
                if (lane == 0) {
                    atomicAdd(&acc[kk][0], d_mx); atomicAdd(&acc[kk][1], d_my);
                    atomicAdd(&acc[kk][2], d_qa); atomicAdd(&acc[kk][3], d_qb); atomicAdd(&acc[kk][4], d_qc);
                    atomicAdd(&acc[kk][5], d_c0); atomicAdd(&acc[kk][6], d_c1); atomicAdd(&acc[kk][7], d_c2);
                    atomicAdd(&acc[kk][8], d_o);
                }
            }
        }
        __syncthreads();
        for (int i = tid; i < nk * 9; i += blockDim.x) {
            const float val = (&acc[0][0])[i];
            if (val != 0.f) {
                const int kk = i / 9, f = i % 9;
                unsafeAtomicAdd(&st.dgauss[(int64_t)S.gp[kk] * 12 + f], val);
            }
            (&acc[0][0])[i] = 0.f;
        }
        __syncthreads();
    }
    // boundary points at the arg-min of each (run, pixel): d gamma / d b, d sigma
    const int nmap = B.n_runs < RunMaps<TS>::value ? B.n_runs : RunMaps<TS>::value;
    for (int r = 0; r < nmap; ++r) {
        const float dg = dgam[r][tid];
        if (dg == 0.f) continue;
        const unsigned long long mv = B.map[r][tid];
        const float gam = __uint_as_float((unsigned)(mv >> 32));
        const int e = (int)(mv & 0xFFFFFFFFull);
        if (!(gam < 1.0f) || e < 0 || e >= B.nbl) continue;
        const float ddx = (float)(lx - B.bix[e]) - B.bdx[e], ddy = (float)(ly - B.biy[e]) - B.bdy[e];
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

hipError_t launch_blend_fwd(const Consts &k, const ViewTable &vt, const StatePtrs &st, float *image, hipStream_t s) {
    switch (k.tile) {
        case 8: return launch_fwd_t<8, 64>(k, vt, st, image, s);
        case 16: return launch_fwd_t<16, 64>(k, vt, st, image, s);
        case 32: return launch_fwd_t<32, 64>(k, vt, st, image, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_blend_bwd(const Consts &k, const ViewTable &vt, const StatePtrs &st, const float *image,
                            const float *grad_image, hipStream_t s) {
    switch (k.tile) {
        case 8: return launch_bwd_t<8, 64>(k, vt, st, image, grad_image, s);
        case 16: return launch_bwd_t<16, 64>(k, vt, st, image, grad_image, s);
        case 32: return launch_bwd_t<32, 64>(k, vt, st, image, grad_image, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bgt
