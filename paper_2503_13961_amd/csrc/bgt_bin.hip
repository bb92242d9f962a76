// Tile binning for the rendering acceleration of Sec. 3.2: Gaussians go to
// every tile their support reaches, sorted front to back within the tile;
// boundary points go to every tile their radius reaches, sorted by primitive
// id.  The sort is a two-level radix split: a counting pass on the tile id
// (the high key digit) places each pair in its tile's segment, then each
// segment is sorted on the low digits (depth, record index) or (primitive,
// record index): by one wave in registers (a bitonic network over up to 512
// keys), longer segments by a workgroup (runs of 64 keys sorted in registers,
// merged pairwise by rank in LDS; segments beyond the LDS buffer: a bitonic
// network in global memory).  The low digits make every key unique, so the
// result does not depend on the order of the atomics that filled the segment.
#include "bgt_internal.h"

namespace bgt {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanBlock = kScanThreads * kScanItems;  // 1024

// inclusive scan over a wave (64 lanes)
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

// exclusive block scan of one value per thread; returns the block total
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T x, T &total, T *lds_waves) {
    const int lane = __lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    T inc = wave_inclusive_scan(x);
    if (lane == 63) lds_waves[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        T w = lane < nw ? lds_waves[lane] : T(0);
        T wi = wave_inclusive_scan(w);
        if (lane < nw) lds_waves[lane] = wi - w;
        if (lane == nw - 1) lds_waves[32] = wi;
    }
    __syncthreads();
    T res = inc - x + lds_waves[wave];
    total = lds_waves[32];
    __syncthreads();
    return res;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const int32_t *gc, const int32_t *bc, int n,
                                                              int64_t *sums, int nb) {
    __shared__ int64_t ws[33];
    const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
    int64_t sg = 0, sb = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) { sg += gc[base + i]; sb += bc[base + i]; }
    int64_t tg, tb;
    block_exclusive_scan<int64_t>(sg, tg, ws);
    block_exclusive_scan<int64_t>(sb, tb, ws);
    if (threadIdx.x == 0) { sums[blockIdx.x] = tg; sums[nb + blockIdx.x] = tb; }
}

// exclusive scan of the block sums (one block), totals into the counters
__global__ void __launch_bounds__(1024) k_scan_top(int64_t *sums, int nb, int64_t *counters) {
    __shared__ int64_t ws[33];
    for (int which = 0; which < 2; ++which) {
        int64_t carry = 0;
        int64_t *s = sums + (int64_t)which * nb;
        for (int base = 0; base < nb; base += blockDim.x) {
            const int i = base + threadIdx.x;
            int64_t x = i < nb ? s[i] : 0, tot;
            int64_t ex = block_exclusive_scan<int64_t>(x, tot, ws);
            if (i < nb) s[i] = ex + carry;
            carry += tot;
        }
        if (threadIdx.x == 0) counters[which == 0 ? C_GPAIRS : C_BPAIRS] = carry;
    }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_down(int32_t *gc, int32_t *gs, int32_t *gcur, int32_t *bc,
                                                            int32_t *bs, int32_t *bcur, const int64_t *sums,
                                                            int n, int nb, int64_t cap_g, int64_t cap_b,
                                                            int64_t *counters) {
    __shared__ int64_t ws[33];
    const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
    for (int which = 0; which < 2; ++which) {
        int32_t *cnt = which == 0 ? gc : bc;
        int32_t *st = which == 0 ? gs : bs;
        int32_t *cur = which == 0 ? gcur : bcur;
        const int64_t cap = which == 0 ? cap_g : cap_b;
        int64_t v[kScanItems], s = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            v[i] = base + i < n ? cnt[base + i] : 0;
            s += v[i];
        }
        int64_t tot;
        int64_t off = block_exclusive_scan<int64_t>(s, tot, ws) + sums[(int64_t)which * nb + blockIdx.x];
        bool ovf = false;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if (base + i < n) {
                int64_t c = v[i];
                if (off + c > cap) { c = off < cap ? cap - off : 0; ovf = true; }
                const int64_t sclamp = off < cap ? off : cap;
                st[base + i] = (int32_t)sclamp;
                cur[base + i] = (int32_t)sclamp;
                cnt[base + i] = (int32_t)c;
            }
            off += v[i];
        }
        if (ovf) atomicOr((unsigned long long *)&counters[C_OVERFLOW], which == 0 ? 1ull : 2ull);
    }
}

// ------------------------------------------------------------ scatter

// A lane's tile rectangle [x0, x1] x [y0, y1] (empty: x0 > x1).
struct TileRect {
    int x0 = 1, x1 = 0, y0 = 1, y1 = 0;
    __device__ bool has(int tx, int ty) const { return tx >= x0 && tx <= x1 && ty >= y0 && ty <= y1; }
};

// The pairs of the lanes whose rectangles lie within the 3x3 tiles around
// (cx, cy), the tile of the wave's 8x8 block, for both lists: one cursor
// atomic per (list, neighbouring tile) for the whole wave, all issued by one
// instruction (lane j takes the Gaussian list of tile j, lane 9 + j its
// boundary list) together with the loads of the segments' ends, so the wave
// waits for one round trip; a lane's slot in a tile is the tile's base plus
// its rank among the lanes there (slots past the segment's end, after a
// capacity overflow, are dropped).  Every base and end goes to scalar
// registers before the first key is stored: reading them between the stores
// would make each store wait for the previous one.  Lanes whose rectangle
// reaches further (gin, bin false) are left to the caller.
template <typename EG, typename EB>
__device__ __forceinline__ void near_tiles(bool gin, const TileRect &g, bool bin, const TileRect &b, int cx, int cy,
                                           const ViewInfo &vi, const StatePtrs &st, int lane, EG &&emit_g,
                                           EB &&emit_b) {
    const unsigned long long below = (1ull << lane) - 1ull;
    int cnt = 0;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        const int tx = cx + j % 3 - 1, ty = cy + j / 3 - 1;
        const unsigned long long mg = __ballot(gin && g.has(tx, ty));
        const unsigned long long mb = __ballot(bin && b.has(tx, ty));
        if (lane == j) cnt = __popcll(mg);
        if (lane == 9 + j) cnt = __popcll(mb);
    }
    int base = 0, s0 = 0, c0 = 0;
    if (cnt > 0) {
        const bool isg = lane < 9;
        const int j = isg ? lane : lane - 9;
        const int tl = vi.tile_off + (cy + j / 3 - 1) * vi.tiles_x + cx + j % 3 - 1;
        s0 = (isg ? st.g_start : st.b_start)[tl];
        c0 = (isg ? st.g_count : st.b_count)[tl];
        base = atomicAdd((isg ? st.g_cursor : st.b_cursor) + tl, cnt);
    }
    const int end = s0 + c0;
    int bs[18], es[18];
#pragma unroll
    for (int j = 0; j < 18; ++j) {
        bs[j] = __builtin_amdgcn_readlane(base, j);
        es[j] = __builtin_amdgcn_readlane(end, j);
    }
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        const int tx = cx + j % 3 - 1, ty = cy + j / 3 - 1;
        const bool ig = gin && g.has(tx, ty), ib = bin && b.has(tx, ty);
        const unsigned long long mg = __ballot(ig), mb = __ballot(ib);
        const int sg = bs[j] + __popcll(mg & below), sb = bs[9 + j] + __popcll(mb & below);
        if (ig && sg < es[j]) emit_g(sg);
        if (ib && sb < es[9 + j]) emit_b(sb);
    }
}

__global__ void __launch_bounds__(256) k_scatter(Consts k, ViewTable vt, StatePtrs st) {
    const int lane = threadIdx.x & 63;
    int v, x, y;
    const int blk = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    const bool act = block8_pixel(vt, blk, lane, v, x, y);
    const ViewInfo vi = vt.v[v];
    const int TSH = __builtin_ctz(k.tile);  // tile side 8, 16 or 32: pixel ranges (>= 0) shift to tiles
    // the tile of the wave's block (x - (lane & 7) is its left edge)
    const int cx = __builtin_amdgcn_readfirstlane((x - (lane & 7)) >> TSH);
    const int cy = __builtin_amdgcn_readfirstlane((y - (lane >> 3)) >> TSH);
    TileRect g, b;
    unsigned long long gkey = 0ull, bkey = 0ull;
    if (act) {
        const int lp = y * vi.W + x, pix = vi.px_off + lp;
        const uint8_t fl = st.pflags[pix];
        if (fl & PF_VALID) {
            // (the three loads in one round trip: the primitive is read for
            // every record, used for boundary points)
            const float4 r3 = st.rec[(int64_t)pix * 4 + 3];
            const unsigned long long depth = st.gkey[pix];
            const int prim = __float_as_int(st.rec[(int64_t)pix * 4 + 2].y);
            const int gx = __float_as_int(r3.x), gy = __float_as_int(r3.y);
            // (in the lattice variant a pixel record is a boundary point only)
            if (k.NL == 0 && lo16(gx) <= hi16(gx) && lo16(gy) <= hi16(gy)) {
                g.x0 = lo16(gx) >> TSH; g.x1 = hi16(gx) >> TSH; g.y0 = lo16(gy) >> TSH; g.y1 = hi16(gy) >> TSH;
            }
            gkey = (depth << 24) | (unsigned long long)lp;
            if (fl & PF_BOUNDARY) {
                const int bx = __float_as_int(r3.z), by = __float_as_int(r3.w);
                if (lo16(bx) <= hi16(bx) && lo16(by) <= hi16(by)) {
                    b.x0 = lo16(bx) >> TSH; b.x1 = hi16(bx) >> TSH; b.y0 = lo16(by) >> TSH; b.y1 = hi16(by) >> TSH;
                }
                bkey = ((unsigned long long)prim << 24) | (unsigned long long)lp;
            }
        }
    }
    // rectangles within the 3x3 tiles around the block's tile (nearly all):
    // one round of cursor atomics for both lists; the rest one cursor atomic
    // per group of lanes at the same tile, each lane taking the slot of its rank
    const bool gnear = g.x0 <= g.x1 && g.y0 <= g.y1 && g.x0 >= cx - 1 && g.x1 <= cx + 1 && g.y0 >= cy - 1 &&
                       g.y1 <= cy + 1;
    const bool bnear = b.x0 <= b.x1 && b.y0 <= b.y1 && b.x0 >= cx - 1 && b.x1 <= cx + 1 && b.y0 >= cy - 1 &&
                       b.y1 <= cy + 1;
    near_tiles(gnear, g, bnear, b, cx, cy, vi, st, lane, [&](int slot) { st.g_keys[slot] = gkey; },
               [&](int slot) { st.b_keys[slot] = bkey; });
    const unsigned long long below = (1ull << lane) - 1ull;
    if (gnear) g = TileRect();
    if (bnear) b = TileRect();
    for_tiles_grouped(g.x0, g.x1, g.y0, g.y1, vi.tiles_x, vi.tile_off,
                      [&](int t, unsigned long long gm, bool in, int leader) {
        int base = 0;
        if (lane == leader) base = atomicAdd(&st.g_cursor[t], __popcll(gm));
        base = __shfl(base, leader, 64);
        if (in) {
            const int slot = base + __popcll(gm & below);
            if (slot < st.g_start[t] + st.g_count[t]) st.g_keys[slot] = gkey;
        }
    });
    for_tiles_grouped(b.x0, b.x1, b.y0, b.y1, vi.tiles_x, vi.tile_off,
                      [&](int t, unsigned long long gm, bool in, int leader) {
        int base = 0;
        if (lane == leader) base = atomicAdd(&st.b_cursor[t], __popcll(gm));
        base = __shfl(base, leader, 64);
        if (in) {
            const int slot = base + __popcll(gm & below);
            if (slot < st.b_start[t] + st.b_count[t]) st.b_keys[slot] = bkey;
        }
    });
}

// Lattice variant: the pairs of the lattice Gaussians, one lane per record;
// a record's key digit is its index within its view, after the view's pixels.
__global__ void __launch_bounds__(256) k_scatter_lattice(Consts k, ViewTable vt, StatePtrs st) {
    const int lane = threadIdx.x & 63;
    const int64_t per_view = (int64_t)k.P * k.NL;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool act = i < (int64_t)vt.n * per_view;
    const int v = act ? (int)(i / per_view) : 0;
    const ViewInfo vi = vt.v[v];
    const int TSH = __builtin_ctz(k.tile);  // tile side 8, 16 or 32: pixel ranges (>= 0) shift to tiles
    int gt0 = 1, gt1 = 0, gu0 = 1, gu1 = 0;
    unsigned long long gkey = 0ull;
    if (act) {
        const int64_t rid = vt.total_px + i;
        const float4 r3 = st.rec[rid * 4 + 3];
        const int gx = __float_as_int(r3.x), gy = __float_as_int(r3.y);
        if (lo16(gx) <= hi16(gx) && lo16(gy) <= hi16(gy)) {
            gt0 = lo16(gx) >> TSH; gt1 = hi16(gx) >> TSH; gu0 = lo16(gy) >> TSH; gu1 = hi16(gy) >> TSH;
        }
        const int lr = vi.W * vi.H + (int)(i - v * per_view);
        gkey = (st.gkey[rid] << 24) | (unsigned long long)lr;
    }
    // rectangles within the 3x3 tiles around the middle of the wave's first
    // rectangle (the wave's records are neighbouring nodes of one or two
    // patches), in that rectangle's view: one round of cursor atomics; the
    // rest one cursor atomic per group of lanes at the same tile
    TileRect g;
    g.x0 = gt0; g.x1 = gt1; g.y0 = gu0; g.y1 = gu1;
    const unsigned long long has = __ballot(gt0 <= gt1);
    if (has) {
        const int f = __ffsll((long long)has) - 1;
        const int cx = __builtin_amdgcn_readlane((gt0 + gt1) >> 1, f);
        const int cy = __builtin_amdgcn_readlane((gu0 + gu1) >> 1, f);
        const int vw = __builtin_amdgcn_readlane(v, f);
        const bool near = gt0 <= gt1 && v == vw && gt0 >= cx - 1 && gt1 <= cx + 1 && gu0 >= cy - 1 && gu1 <= cy + 1;
        near_tiles(near, g, false, TileRect(), cx, cy, vt.v[vw], st, lane, [&](int slot) { st.g_keys[slot] = gkey; },
                   [&](int) {});
        if (near) g = TileRect();
    }
    const unsigned long long below = (1ull << lane) - 1ull;
    for_tiles_grouped(g.x0, g.x1, g.y0, g.y1, vi.tiles_x, vi.tile_off,
                      [&](int t, unsigned long long gm, bool in, int leader) {
        int base = 0;
        if (lane == leader) base = atomicAdd(&st.g_cursor[t], __popcll(gm));
        base = __shfl(base, leader, 64);
        if (in) {
            const int slot = base + __popcll(gm & below);
            if (slot < st.g_start[t] + st.g_count[t]) st.g_keys[slot] = gkey;
        }
    });
}

// ------------------------------------------------------------ segment sort

// Ascending bitonic network whose first step of every merge compares mirrored
// positions; positions >= n behave as +inf and never move, so a segment is
// padded virtually to the next power of two.
template <typename Get, typename CmpX>
__device__ __forceinline__ void bitonic_steps(int n2, CmpX cmpx) {
    for (int kk = 2; kk <= n2; kk <<= 1) {
        const int half = kk >> 1;
        for (int q = threadIdx.x; q < (n2 >> 1); q += blockDim.x) {
            const int blk = q / half, pos = q % half;
            cmpx(blk * kk + pos, blk * kk + kk - 1 - pos);
        }
        __syncthreads();
        for (int j = kk >> 2; j >= 1; j >>= 1) {
            for (int q = threadIdx.x; q < (n2 >> 1); q += blockDim.x) {
                const int blk = q / j, pos = q % j;
                const int a = blk * 2 * j + pos;
                cmpx(a, a + j);
            }
            __syncthreads();
        }
    }
}

struct NoGet {};

// Ascending bitonic sort of one key per lane across the wave (64 keys),
// through lane exchanges only (no LDS, no barriers).
__device__ __forceinline__ unsigned long long wave_sort64(unsigned long long x, int lane) {
    for (int kk = 2; kk <= 64; kk <<= 1)
        for (int j = kk >> 1; j >= 1; j >>= 1) {
            const unsigned long long y = __shfl_xor(x, j, 64);
            // the lower lane of a pair keeps the smaller key in ascending runs
            const bool keep_min = ((lane & j) == 0) == ((lane & kk) == 0);
            x = keep_min ? (y < x ? y : x) : (y < x ? x : y);
        }
    return x;
}

// Keys of the sorted a[0, n) below x (UPPER: not above x).
template <bool UPPER>
__device__ __forceinline__ int rank_in(const unsigned long long *a, int n, unsigned long long x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (UPPER ? a[mid] <= x : a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// The list positions of tile t (of view v) under its slot: gpos[rec] is
// the position of record rec in the tile's list.
__device__ __forceinline__ int32_t *list_positions(const ViewTable &vt, const StatePtrs &st, int v, int t) {
    const int tl = t - vt.v[v].tile_off, tx = tl % vt.v[v].tiles_x, ty = tl / vt.v[v].tiles_x;
    return st.gpos + (int64_t)tile_slot(tx, ty) * st.n_rec;
}

// The key of lane l ^ m (m a power of two below 64): DPP within quads
// (plain VALU moves), an LDS swizzle within 32-lane halves, a permute across
// them.
__device__ __forceinline__ int xor_lane(int v, int m) {
    if (m == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // quad_perm [1, 0, 3, 2]
    if (m == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // quad_perm [2, 3, 0, 1]
    if (m == 4) return __builtin_amdgcn_ds_swizzle(v, 0x101F);               // bit mode: and 31, xor 4
    if (m == 8) return __builtin_amdgcn_ds_swizzle(v, 0x201F);
    if (m == 16) return __builtin_amdgcn_ds_swizzle(v, 0x401F);
    return __shfl_xor(v, m, 64);
}
__device__ __forceinline__ unsigned long long xor_lane(unsigned long long v, int m) {
    const int lo = xor_lane((int)(unsigned)v, m), hi = xor_lane((int)(unsigned)(v >> 32), m);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

// Ascending bitonic sort of the 64 R keys x[r] of lane l (key l R + r)
// across the wave: partners fewer than R apart are in the same lane, the
// others (fewer steps) are exchanged between lanes.  Padding keys (~0) sort
// last.
template <int R>
__device__ __forceinline__ void wave_sort_regs(unsigned long long (&x)[R], int lane) {
#pragma unroll
    for (int k = 2; k <= 64 * R; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j >= 1; j >>= 1) {
            if (j < R) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int r2 = r ^ j;
                    if (r2 < r) continue;
                    // ascending where bit k of the key index l R + r is clear
                    const bool up = (((lane * R) | r) & k) == 0;
                    const unsigned long long a = x[r], b = x[r2];
                    const bool sw = (b < a) == up;  // (equal keys: either)
                    x[r] = sw ? b : a;
                    x[r2] = sw ? a : b;
                }
            } else {
                const int m = j / R;  // partner lane l ^ m
                // the lower lane of a pair keeps the smaller key in ascending
                // runs: it takes the partner's key when that is smaller, the
                // upper lane when it is larger (equal keys: either)
                const bool keep_min = ((lane & m) == 0) == (((lane * R) & k) == 0);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const unsigned long long y = xor_lane(x[r], m);
                    x[r] = (y < x[r]) == keep_min ? y : x[r];
                }
            }
        }
    }
}

// Lists up to this length are sorted by one wave in registers; longer ones
// are queued for a workgroup each.
constexpr int kWaveSort = 512;

// LDS slot of key i of a wave's staging buffer: 8 bytes of padding after
// every 8 keys, so that lanes reading 8 consecutive keys each hit distinct
// banks
__device__ __forceinline__ int stage_slot(int i) { return i + (i >> 3); }
constexpr int kStageKeys = kWaveSort + kWaveSort / 8;

// Sorts one list of cnt <= 64 R keys.  Multi-key lanes load and store
// through the wave's LDS buffer sb, so that global memory is read and written
// in 64-lane runs while each lane sorts consecutive keys.
template <int R, typename Emit>
__device__ __forceinline__ void wave_sort_list(const unsigned long long *src, int cnt, int lane, unsigned long long *sb,
                                               Emit &&emit) {
    unsigned long long x[R];
    if constexpr (R == 1) {
        x[0] = lane < cnt ? src[lane] : ~0ull;
        wave_sort_regs<1>(x, lane);
        if (lane < cnt) emit(lane, x[0]);
        return;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = r * 64 + lane;
        sb[stage_slot(i)] = i < cnt ? src[i] : ~0ull;
    }
    // (one wave's LDS accesses complete in order: the fence keeps the
    // compiler from moving them across each other)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = sb[stage_slot(lane * R + r)];
    wave_sort_regs<R>(x, lane);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < R; ++r) sb[stage_slot(lane * R + r)] = x[r];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = r * 64 + lane;
        if (i < cnt) emit(i, sb[stage_slot(i)]);
    }
}

// Sorts one list of 256 < cnt <= 256 + 64 RB keys without sorting padding up
// to 512: the first 256 keys (4 per lane) and the rest (RB per lane) are
// sorted in registers as two runs, then merged along the merge path, each
// lane writing per = ceil(cnt / 64) consecutive outputs: a binary search
// finds how many of them come from the first run, then one comparison per
// output walks both runs (keys of the first run go before equal keys of the
// second).
template <int RB, typename Emit>
__device__ __forceinline__ void wave_sort_split(const unsigned long long *src, int cnt, int lane,
                                                unsigned long long *sb, Emit &&emit) {
    constexpr int RA = 4, NA = 64 * RA;
    unsigned long long x[RA], y[RB];
#pragma unroll
    for (int r = 0; r < RA + RB; ++r) {
        const int i = r * 64 + lane;
        sb[stage_slot(i)] = i < cnt ? src[i] : ~0ull;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < RA; ++r) x[r] = sb[stage_slot(lane * RA + r)];
#pragma unroll
    for (int r = 0; r < RB; ++r) y[r] = sb[stage_slot(NA + lane * RB + r)];
    wave_sort_regs<RA>(x, lane);
    wave_sort_regs<RB>(y, lane);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < RA; ++r) sb[stage_slot(lane * RA + r)] = x[r];
#pragma unroll
    for (int r = 0; r < RB; ++r) sb[stage_slot(NA + lane * RB + r)] = y[r];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int lb = cnt - NA, per = (cnt + 63) >> 6, d = lane * per;
    if (d >= cnt) return;
    int lo = max(0, d - lb), hi = min(d, NA);
    while (lo < hi) {
        const int c = (lo + hi) >> 1;
        if (sb[stage_slot(c)] <= sb[stage_slot(NA + d - 1 - c)]) lo = c + 1;
        else hi = c;
    }
    int i = lo, j = d - lo;
    // (a read one past the first run is the second run's first key, one past
    // the second a padding slot; neither is taken)
    unsigned long long ka = sb[stage_slot(i)], kb = sb[stage_slot(NA + j)];
    const int m = min(per, cnt - d);
#pragma unroll
    for (int k = 0; k < RA + RB; ++k)
        if (k < m) {
            const bool take_a = i < NA && (j >= lb || ka <= kb);
            emit(d + k, take_a ? ka : kb);
            i += take_a;
            j += !take_a;
            const unsigned long long nx = sb[stage_slot(take_a ? i : NA + j)];
            ka = take_a ? nx : ka;
            kb = take_a ? kb : nx;
        }
}

// One wave per list: list L < n_tiles is the Gaussian list of tile L, the
// others the boundary lists.  Empty lists cost a wave a few instructions.
__global__ void __launch_bounds__(256) k_sort_lists(ViewTable vt, StatePtrs st, int lat_per_view) {
    __shared__ unsigned long long stage[4][kStageKeys];
    const int lane = threadIdx.x & 63;
    const int L = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (L >= 2 * vt.total_tiles) return;
    const int which = L < vt.total_tiles ? 0 : 1, t = which == 0 ? L : L - vt.total_tiles;
    const int cnt = which == 0 ? st.g_count[t] : st.b_count[t];
    if (cnt == 0 || cnt > kWaveSort) return;  // (longer lists: k_sort_long)
    const int start = which == 0 ? st.g_start[t] : st.b_start[t];
    const unsigned long long *src = (which == 0 ? st.g_keys : st.b_keys) + start;
    const int v = view_of_tile(vt, t);
    uint32_t *dst = (which == 0 ? st.g_list : st.b_list) + start;
    // a Gaussian list also records each entry's position under its record's
    // tile slot, for the parameter pass
    int32_t *gpos = which == 0 ? list_positions(vt, st, v, t) : nullptr;
    auto emit = [&](int i, unsigned long long key) {
        const int rec = record_of(vt, v, (int)(key & 0xFFFFFFull), lat_per_view);
        dst[i] = (uint32_t)rec;
        if (gpos) gpos[rec] = start + i;
    };
    unsigned long long *sb = stage[threadIdx.x >> 6];
    if (cnt <= 64) wave_sort_list<1>(src, cnt, lane, sb, emit);
    else if (cnt <= 128) wave_sort_list<2>(src, cnt, lane, sb, emit);
    else if (cnt <= 256) wave_sort_list<4>(src, cnt, lane, sb, emit);
    else if (cnt <= 320) wave_sort_split<1>(src, cnt, lane, sb, emit);
    else if (cnt <= 384) wave_sort_split<2>(src, cnt, lane, sb, emit);
    else wave_sort_list<8>(src, cnt, lane, sb, emit);
}

// Lists longer than a wave sorts, one workgroup per list: workgroup b takes
// the long lists among kLongChunk tiles, whose counts its threads read at
// once (no queue, no global atomic).  Tile i of the launch is tile
// i (2^31 - 1) mod n, a permutation (2^31 - 1 is a prime above n) that
// spreads the long lists, which cluster in neighbouring tiles and at the
// same place in similar views, over the workgroups.  Up to kSortLds keys:
// runs of kWaveSort keys sorted in registers, one wave per run (padded with
// ~0, above every key), then merged pairwise, level by level.  A thread
// writes `per` consecutive outputs of a level (a power of two, at most
// kSortLds / 256): a binary search along the merge path finds how many of
// them come from the pair's first run, then one comparison per output walks
// both runs (keys of the first run go before equal keys of the second).  In
// place: every thread merges its outputs into registers first and all write
// after a barrier, so the block needs one buffer (18 KB); the last level's
// outputs go to the list at once.  Longer lists (rare; a correctness path):
// the bitonic network on global memory.
constexpr int kLongChunk = 16;
static_assert(kSortLds == 4 * kWaveSort, "the four waves of a workgroup sort one run each");

__global__ void __launch_bounds__(256) k_sort_long(ViewTable vt, StatePtrs st, int lat_per_view) {
    __shared__ unsigned long long keys[kSortLds + kSortLds / 8 + 1];
    __shared__ int long_tiles[kLongChunk], n_long;
    const int which = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) n_long = 0;
    __syncthreads();
    if (threadIdx.x < kLongChunk) {
        const int i = blockIdx.x * kLongChunk + threadIdx.x;
        if (i < vt.total_tiles) {
            const int t = (int)((int64_t)i * 2147483647ll % vt.total_tiles);
            if ((which == 0 ? st.g_count[t] : st.b_count[t]) > kWaveSort) long_tiles[atomicAdd(&n_long, 1)] = t;
        }
    }
    __syncthreads();
    for (int li = 0; li < n_long; ++li) {
        const int t = long_tiles[li];
        const int cnt = which == 0 ? st.g_count[t] : st.b_count[t];
        const int start = which == 0 ? st.g_start[t] : st.b_start[t];
        unsigned long long *src = (which == 0 ? st.g_keys : st.b_keys) + start;
        const int v = view_of_tile(vt, t);
        uint32_t *dst = (which == 0 ? st.g_list : st.b_list) + start;
        int32_t *gpos = which == 0 ? list_positions(vt, st, v, t) : nullptr;
        auto emit = [&](int i, unsigned long long key) {
            const int rec = record_of(vt, v, (int)(key & 0xFFFFFFull), lat_per_view);
            dst[i] = (uint32_t)rec;
            if (gpos) gpos[rec] = start + i;
        };
        if (cnt > kSortLds) {
            if (threadIdx.x == 0) atomicAdd((unsigned long long *)&st.counters[C_BIGSORT], 1ull);
            int n2 = 1;
            while (n2 < cnt) n2 <<= 1;
            bitonic_steps<NoGet>(n2, [&](int a, int b) {
                if (b >= cnt) return;
                const unsigned long long x = src[a], y = src[b];
                if (y < x) { src[a] = y; src[b] = x; }
            });
            for (int i = threadIdx.x; i < cnt; i += blockDim.x) emit(i, src[i]);
            __syncthreads();
            continue;
        }
        // runs of 512 keys, one wave each: loaded into the buffer in 64-lane
        // runs, read by each lane as 8 consecutive keys, sorted in registers
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) keys[stage_slot(i)] = src[i];
        __syncthreads();
        if (wave * kWaveSort < cnt) {
            unsigned long long x[8];
            const int b0 = wave * kWaveSort + lane * 8;
#pragma unroll
            for (int r = 0; r < 8; ++r) x[r] = b0 + r < cnt ? keys[stage_slot(b0 + r)] : ~0ull;
            wave_sort_regs<8>(x, lane);
#pragma unroll
            for (int r = 0; r < 8; ++r)
                if (b0 + r < cnt) keys[stage_slot(b0 + r)] = x[r];
        }
        __syncthreads();
        // outputs per thread: a power of two, so that no thread's outputs
        // straddle two pairs of runs
        int per = 1;
        while (per * 256 < cnt) per <<= 1;
        for (int L = kWaveSort; L < cnt; L <<= 1) {
            unsigned long long x[kSortLds / 256];
            const int d0 = threadIdx.x * per;
            int m = 0;
            if (d0 < cnt) {
                const int p0 = d0 & ~(2 * L - 1);
                const int mid = min(p0 + L, cnt), end = min(p0 + 2 * L, cnt);
                const int la = mid - p0, lb = end - mid, d = d0 - p0;
                // how many of the pair's first d outputs come from the first
                // run (the first run's keys go before equal keys of the second)
                int lo = max(0, d - lb), hi = min(d, la);
                while (lo < hi) {
                    const int c = (lo + hi) >> 1;
                    if (keys[stage_slot(p0 + c)] <= keys[stage_slot(mid + d - 1 - c)]) lo = c + 1;
                    else hi = c;
                }
                int i = lo, j = d - lo;
                // (reads one past a run's end stay in the buffer, which has a
                // slot past the last key; their values are never taken)
                unsigned long long ka = keys[stage_slot(p0 + i)], kb = keys[stage_slot(mid + j)];
                m = min(per, end - d0);
#pragma unroll
                for (int k = 0; k < kSortLds / 256; ++k)
                    if (k < m) {
                        const bool take_a = i < la && (j >= lb || ka <= kb);
                        x[k] = take_a ? ka : kb;
                        i += take_a;
                        j += !take_a;
                        const unsigned long long nx = keys[stage_slot(take_a ? p0 + i : mid + j)];
                        ka = take_a ? nx : ka;
                        kb = take_a ? kb : nx;
                    }
            }
            if (2 * L >= cnt) {  // the last level: its outputs are the list
#pragma unroll
                for (int k = 0; k < kSortLds / 256; ++k)
                    if (k < m) emit(d0 + k, x[k]);
            } else {  // in place: all read, then all write
                __syncthreads();
#pragma unroll
                for (int k = 0; k < kSortLds / 256; ++k)
                    if (k < m) keys[stage_slot(d0 + k)] = x[k];
                __syncthreads();
            }
        }
        __syncthreads();  // the next list reuses the buffer
    }
}

// Copies the pass's overflow bits, when there are any, into the context's
// word of pinned host memory: a later call on the context (and bgt_query)
// reads it without waiting for the device.  A plain system-scope store, not
// an atomic, so nothing depends on the host bridge's atomics.
__global__ void k_note_overflow(const int64_t *counters, unsigned long long *flag) {
    if (threadIdx.x != 0) return;
    const unsigned long long f = (unsigned long long)counters[C_OVERFLOW];
    if (f) __hip_atomic_store(flag, f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_note_overflow(const StatePtrs &st, unsigned long long *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_note_overflow, dim3(1), dim3(64), 0, s, (const int64_t *)st.counters, flag);
    return hipGetLastError();
}

hipError_t launch_binning(const Consts &k, const ViewTable &vt, const StatePtrs &st, hipStream_t s) {
    const int n = vt.total_tiles;
    const int nb = (n + kScanBlock - 1) / kScanBlock;
    int64_t *sums = (int64_t *)st.scan_tmp;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, (const int32_t *)st.g_count,
                       (const int32_t *)st.b_count, n, sums, nb);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, sums, nb, st.counters);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kScanThreads), 0, s, st.g_count, st.g_start, st.g_cursor,
                       st.b_count, st.b_start, st.b_cursor, (const int64_t *)sums, n, nb, k.cap_g, k.cap_b,
                       st.counters);
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)((vt.total_b8 + 3) / 4)), dim3(256), 0, s, k, vt, st);
    const int lat_per_view = k.P * k.NL;
    if (lat_per_view > 0) {
        const int64_t nl = (int64_t)vt.n * lat_per_view;
        hipLaunchKernelGGL(k_scatter_lattice, dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, s, k, vt, st);
    }
    hipLaunchKernelGGL(k_sort_lists, dim3((unsigned)((2 * (int64_t)n + 3) / 4)), dim3(256), 0, s, vt, st,
                       lat_per_view);
    hipLaunchKernelGGL(k_sort_long, dim3((unsigned)((n + kLongChunk - 1) / kLongChunk), 2), dim3(256), 0, s, vt, st,
                       lat_per_view);
    return hipGetLastError();
}

}  // namespace bgt
