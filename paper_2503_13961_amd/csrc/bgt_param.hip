// Parameter backward pass: per-Gaussian gradients (mean, conic, colour,
// opacity) and per-boundary-point gradients (position, radius) flow through
// the EWA projection and the boundary radius to the BG-Triangle parameters:
//   dl/dp_ijk   = sum_q B^n_ijk(I_uv(q)) dl/dS_q     (Supplementary Sec. C)
//   dl/dp^c_ijk = sum_q B^n_ijk(I_uv(q)) dl/dc_q     (Eq. 4)
// plus log-scale, rotation, opacity and sharpness.  A workgroup covers a
// 32x32 pixel region, its waves one 8x8 block at a time; pixels of the same
// primitive are summed across the wave (segmented by primitive id) and the
// wave sums across the region in an LDS table keyed by primitive, which
// issues one global atomic per (region, primitive, parameter): the
// primitives' gradient words are the hottest addresses of the pass, and
// same-address atomics from many workgroups serialize.  In the lattice
// variant a second launch walks the lattice Gaussians, 1024 consecutive
// records (about a dozen patches) per workgroup, at their nodes' (u, v).
#include "bgt_internal.h"
#include "bgt_sh.h"
#include "bgt_wave.h"

namespace bgt {

// the hardware reciprocal (within 1 ulp): the gradient terms below need far
// less than correctly rounded division, which takes ten instructions
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

template <int DEG>
__device__ __forceinline__ void bern_f(float u, float v, float w, float *B) {
    constexpr float fact[6] = {1.f, 1.f, 2.f, 6.f, 24.f, 120.f};
    float pu[DEG + 1], pv[DEG + 1], pw[DEG + 1];
    pu[0] = pv[0] = pw[0] = 1.f;
#pragma unroll
    for (int e = 1; e <= DEG; ++e) { pu[e] = pu[e - 1] * u; pv[e] = pv[e - 1] * v; pw[e] = pw[e - 1] * w; }
    int idx = 0;
#pragma unroll
    for (int i = 0; i <= DEG; ++i)
#pragma unroll
        for (int j = 0; j <= DEG - i; ++j) {
            const int kk = DEG - i - j;
            B[idx++] = fact[DEG] / (fact[i] * fact[j] * fact[kk]) * pu[i] * pv[j] * pw[kk];
        }
}

// One chunk of up to 64 of a wave's NV per-lane values (from `value`, taken
// on the lanes where `mine`): reduce-scattered over the wave, then each lane
// holding a total adds it to row `slot` of the workgroup's LDS table, or,
// without a row (the table is full), to its global target.
template <int BASE, int NV, typename V, typename T>
__device__ __forceinline__ void reduce_chunk(V &value, T &target, bool mine, int gl, int lane, float *table,
                                             int slot) {
    constexpr int N = NV - BASE < 64 ? NV - BASE : 64;
    float v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = mine ? value(BASE + i) : 0.f;
    wave_reduce_scatter<N>(v, lane);
    const int j = BASE + scatter_index(lane);
    if (j < BASE + N && v[0] != 0.f) {
        if (slot >= 0) {
            atomicAdd(&table[slot * NV + j], v[0]);
        } else {
            float *t = target(j, gl);
            if (t) unsafeAtomicAdd(t, v[0]);
        }
    }
}

// Row of primitive p (wave-uniform) in the workgroup's table: open
// addressing over the rows' primitive ids, claimed by compare-and-swap;
// -1 when every row holds another primitive.
template <int SLOTS>
__device__ __forceinline__ int table_slot(int *slot_prim, int p, int lane) {
    int s = -1;
    if (lane == 0) {
        const int h = (int)(((unsigned)p * 2654435761u) >> 16) & (SLOTS - 1);
        for (int n = 0; n < SLOTS; ++n) {
            const int q = (h + n) & (SLOTS - 1);
            const int old = atomicCAS(&slot_prim[q], -1, p);
            if (old == -1 || old == p) {
                s = q;
                break;
            }
        }
    }
    return __builtin_amdgcn_readfirstlane(s);
}

constexpr int kRegion = 32;      // pixels per side of a workgroup's region
constexpr int kRegionPasses = 4; // 8x8 blocks per wave: (32/8)^2 blocks over 4 waves
constexpr int kLatPerGroup = 256 * kRegionPasses;

// view, region origin of workgroup `reg` (regions of kRegion px, row-major per view)
__device__ __forceinline__ int region_view(const ViewTable &vt, int reg, int &rx0, int &ry0) {
    int acc = 0;
    for (int v = 0; v < vt.n; ++v) {
        const int nx = (vt.v[v].W + kRegion - 1) / kRegion, ny = (vt.v[v].H + kRegion - 1) / kRegion;
        if (reg < acc + nx * ny) {
            const int l = reg - acc;
            rx0 = (l % nx) * kRegion;
            ry0 = (l / nx) * kRegion;
            return v;
        }
        acc += nx * ny;
    }
    rx0 = ry0 = 0;
    return -1;
}

// The blend pass's sums g[0..8] of record `rid` of view vi: one per tile its
// Gaussian was binned to (the tile range of the binning pass), added in
// raster order, so the result does not depend on scheduling.  A narrow
// record (at most 3 x 3 tiles) has them at its slot of each tile, valid where
// its position in the tile's list (which the sort wrote to the same slot)
// lies before the end of the tile's replayed prefix: the backward writes
// every entry of that prefix and no other.  The tiles are taken three at a
// time with every load issued before any is used (a slot past the prefix is
// loaded and not added), so a record of up to three tiles waits for one
// round trip.  A wide record's sums were added into its own floats, which are
// read and cleared for the next backward pass.  `ovf`: lists overflowed their
// capacity and lack entries, whose slots hold no position of this pass; no
// sums are taken then.
__device__ __forceinline__ void gauss_sums(const Consts &k, const ViewInfo &vi, const StatePtrs &st, int rid,
                                           bool ovf, float *g) {
    const int4 r3 = *(const int4 *)(st.rec + (int64_t)rid * 4 + 3);
    const int gx = r3.x, gy = r3.y;
    if (!((lo16(gx) <= hi16(gx)) & (lo16(gy) <= hi16(gy)))) return;
    const int TSH = __builtin_ctz(k.tile);
    if (!narrow_range(gx, gy, TSH)) {
        float *w = st.gwide + (int64_t)rid * kSums;
#pragma unroll
        for (int f = 0; f < kSums; ++f) { g[f] = w[f]; w[f] = 0.f; }
        return;
    }
    if (ovf) return;
    const int gt0 = lo16(gx) >> TSH, gu0 = lo16(gy) >> TSH;
    const int nx = (hi16(gx) >> TSH) - gt0 + 1, nt = nx * ((hi16(gy) >> TSH) - gu0 + 1);
    for (int j0 = 0; j0 < nt; j0 += 3) {
        int p[3], e[3];
        float q[3][kSums];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int j = min(j0 + c, nt - 1);  // (past the range: the last tile again, not added)
            const int tx = gt0 + j % nx, ty = gu0 + j / nx;
            const int64_t si = (int64_t)tile_slot(tx, ty) * st.n_rec + rid;
            p[c] = st.gpos[si];
            e[c] = st.t_end[vi.tile_off + ty * vi.tiles_x + tx];
#pragma unroll
            for (int f = 0; f < kSums; ++f) q[c][f] = st.gslot[si * kSums + f];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const bool ok = j0 + c < nt && p[c] < e[c];
#pragma unroll
            for (int f = 0; f < kSums; ++f) g[f] += ok ? q[c][f] : 0.f;
        }
    }
}

template <int DEG, bool EXT, bool LAT>
__global__ void __launch_bounds__(256) k_param_bwd(Consts k, ViewTable vt, PrimPtrs pr, const float *cams,
                                                  StatePtrs st, GradPtrs gr, const float *__restrict__ patch) {
    constexpr int NCP = (DEG + 1) * (DEG + 2) / 2;
    constexpr int QO = patch_q_off(NCP);
    const int PD = k.pdw;
    // values per pixel: control points, colour control points, log-scales and
    // quaternions of the map's texels (at most 6), opacity, sharpness, SH
    // coefficients (at most 15 per channel)
    constexpr int TM = EXT ? 6 : 1, KM = EXT ? 15 : 0;
    constexpr int NV = 6 * NCP + 7 * TM + 2 + 3 * KM;
    constexpr int SLOTS = NV > 100 ? 32 : 64;
    __shared__ int slot_prim[SLOTS];
    __shared__ float table[SLOTS * NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool ovf = (st.counters[C_OVERFLOW] & 1) != 0;  // the Gaussian lists overflowed
    for (int i = threadIdx.x; i < SLOTS; i += blockDim.x) slot_prim[i] = -1;
    for (int i = threadIdx.x; i < SLOTS * NV; i += blockDim.x) table[i] = 0.f;
    int rx0 = 0, ry0 = 0, rv = 0;
    if constexpr (!LAT) rv = region_view(vt, blockIdx.x, rx0, ry0);
    __syncthreads();
    auto target = [&](int j, int gl) -> float * {
        if (j < 3 * NCP) return gr.ctrl + (int64_t)j * k.P + gl;  // [d][c] with j = d NCP + c
        if (j < 6 * NCP) return gr.color + (int64_t)(j - 3 * NCP) * k.P + gl;
        const int r = j - 6 * NCP;
        if (r < 3 * TM) {
            const int d = r / TM, t = r % TM;
            return t < k.T ? gr.log_scale + ((int64_t)d * k.T + t) * k.P + gl : nullptr;
        }
        if (r < 7 * TM) {
            const int d = (r - 3 * TM) / TM, t = (r - 3 * TM) % TM;
            return t < k.T ? gr.quat + ((int64_t)d * k.T + t) * k.P + gl : nullptr;
        }
        if (r == 7 * TM) return gr.opacity + gl;
        if (r == 7 * TM + 1) return gr.sharp + gl;
        const int h = r - 7 * TM - 2, c = h / (KM > 0 ? KM : 1), jj = h % (KM > 0 ? KM : 1);
        return jj < k.K ? gr.sh + ((int64_t)c * k.K + jj) * k.P + gl : nullptr;
    };
#pragma unroll 1
    for (int pass = 0; pass < kRegionPasses; ++pass) {
    // locate the view and pixel (or lattice record) of this lane
    int pix = -1, prim = -1;
    float dS[3] = {0.f, 0.f, 0.f}, dcol[3] = {0.f, 0.f, 0.f}, dls[3] = {0.f, 0.f, 0.f}, dq[4] = {0.f, 0.f, 0.f, 0.f};
    float dop = 0.f, dsh = 0.f;
    float tw6[TM];  // this pixel's weight of each texel (Eq. 5)
    float Yv[KM > 0 ? KM : 1];  // SH basis at its view direction
#pragma unroll
    for (int t = 0; t < TM; ++t) tw6[t] = 0.f;
#pragma unroll
    for (int j = 0; j < (KM > 0 ? KM : 1); ++j) Yv[j] = 0.f;
    float B[NCP];
#pragma unroll
    for (int c = 0; c < NCP; ++c) B[c] = 0.f;
    bool act = false;
    float g[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) g[i] = 0.f;
    int v0 = 0;  // view of the lane's record
    float2 uv = make_float2(0.f, 0.f);
    if constexpr (LAT) {
        // record total_px + i: view i / (P NL), patch, node (a, b) at (a, b) / M
        const int64_t per_view = (int64_t)k.P * k.NL;
        const int64_t i = (int64_t)blockIdx.x * kLatPerGroup + pass * 256 + threadIdx.x;
        if (i < (int64_t)vt.n * per_view) {
            v0 = (int)(i / per_view);
            const int64_t r = i - v0 * per_view;
            const int p = (int)(r / k.NL);
            int node = (int)(r - (int64_t)p * k.NL), a = 0;
            while (node > k.lat_level - a) { node -= k.lat_level - a + 1; ++a; }
            uv = make_float2((float)a / (float)k.lat_level, (float)node / (float)k.lat_level);
            pix = vt.total_px + (int)i;
            prim = p;
        }
    } else if (rv >= 0) {
        // block wave + 4 pass of the region's 4x4 blocks of 8x8 pixels
        const int b = wave + 4 * pass;
        const int x0 = rx0 + (b & 3) * 8 + (lane & 7), y0 = ry0 + (b >> 2) * 8 + (lane >> 3);
        v0 = rv;
        const int lr = y0 * vt.v[rv].W + x0;
        if (x0 < vt.v[rv].W && y0 < vt.v[rv].H) pix = vt.v[rv].px_off + lr;
    }
    {
        const uint8_t fl = (!LAT && pix >= 0) ? st.pflags[pix] : (uint8_t)0;
        if (pix >= 0 && (LAT || (fl & PF_VALID))) {
            // the blend sums: moments m0..m4 = sum dG (dx, dy, dx dx, dx dy, dy dy)
            // of dl/dG G, colour, opacity (the record's Gaussian; a pixel
            // record of the lattice variant has none), boundary radius and
            // position (a boundary point's)
            // (the pixel's triangle and uv are read before the cleared words
            // are written: a load issued after a store waits for it too)
            int tri = 0;
            float2 uvp = make_float2(0.f, 0.f);
            if constexpr (!LAT) {
                tri = st.I_tri[pix];
                uvp = st.I_uv[pix];
            }
            if (LAT || k.NL == 0) gauss_sums(k, vt.v[v0], st, pix, ovf, g);
            if (!LAT && (fl & PF_BOUNDARY)) {  // read and cleared for the next backward pass
                float *bp = st.dbound + (int64_t)pix * 3;
                g[9] = bp[0]; g[10] = bp[1]; g[11] = bp[2];
                bp[0] = 0.f; bp[1] = 0.f; bp[2] = 0.f;
            }
            bool nz = false;
#pragma unroll
            for (int i = 0; i < 12; ++i) nz = nz || g[i] != 0.f;
            if (nz) {
                act = true;
                if constexpr (!LAT) {
                    prim = tri / k.L2;
                    uv = uvp;
                }
            }
        }
    }
    // the patches of this wave through the scalar unit: the wave walks its
    // distinct ids and each lane keeps its own patch's points and attributes
    float cp[3 * NCP], raw[8];
#pragma unroll
    for (int i = 0; i < 3 * NCP; ++i) cp[i] = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) raw[i] = 0.f;
    for (unsigned long long todo = __ballot(act); todo;) {
        const int pu = __builtin_amdgcn_readlane(prim, __ffsll((long long)todo) - 1);
        const bool mine = act && prim == pu;
        todo &= ~__ballot(mine);
        const float *src = patch + (int64_t)pu * PD;
        if (mine) {
#pragma unroll
            for (int i = 0; i < 3 * NCP; ++i) cp[i] = src[i];
#pragma unroll
            for (int i = 0; i < 8; ++i) raw[i] = src[QO + i];
        }
    }
    {
        if (act) {
            const float m0 = g[0], m1 = g[1];
            const float dqa = -0.5f * g[2], dqb = -g[3], dqc = -0.5f * g[4];
            dcol[0] = g[5]; dcol[1] = g[6]; dcol[2] = g[7];
            dop = g[8];
            const float dsig = g[9], dbx = g[10], dby = g[11];
            {
                const int p = prim;
                bern_f<DEG>(uv.x, uv.y, 1.f - uv.x - uv.y, B);
                float S[3] = {0.f, 0.f, 0.f};
#pragma unroll
                for (int c = 0; c < NCP; ++c)
#pragma unroll
                    for (int d = 0; d < 3; ++d) S[d] += B[c] * cp[3 * c + d];
                const float *cm = cams + 16 * v0;
                float W[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) W[i] = cm[i];
                const float fx = cm[12], fy = cm[13];
                float t[3];
#pragma unroll
                for (int r = 0; r < 3; ++r) t[r] = W[3 * r] * S[0] + W[3 * r + 1] * S[1] + W[3 * r + 2] * S[2] + cm[9 + r];
                const float iz = rcp(t[2]);
                const float J00 = fx * iz, J02 = -fx * t[0] * iz * iz, J11 = fy * iz, J12 = -fy * t[1] * iz * iz;
                float Tm[6];
#pragma unroll
                for (int c = 0; c < 3; ++c) { Tm[c] = J00 * W[c] + J02 * W[6 + c]; Tm[3 + c] = J11 * W[3 + c] + J12 * W[6 + c]; }
                // rotation and scale: the patch's (resolution 1) or the
                // interpolation of its maps at I_uv (Eq. 5)
                const float *rec = patch + (int64_t)p * PD;
                float q[4], qn = 0.f, lsv[3];
#pragma unroll
                for (int d = 0; d < 4; ++d) q[d] = raw[d];
#pragma unroll
                for (int d = 0; d < 3; ++d) lsv[d] = raw[4 + d];
                if constexpr (EXT) {
                    int ti[3];
                    float tw[3];
                    theta_weights<float>(k.T > 1 ? 3 : 1, uv.x, uv.y, ti, tw);
#pragma unroll
                    for (int d = 0; d < 4; ++d) q[d] = 0.f;
#pragma unroll
                    for (int d = 0; d < 3; ++d) lsv[d] = 0.f;
#pragma unroll
                    for (int e = 0; e < 3; ++e) {
                        const float *tt = rec + patch_x_off(NCP) + 7 * ti[e];
#pragma unroll
                        for (int d = 0; d < 4; ++d) q[d] += tw[e] * tt[d];
#pragma unroll
                        for (int d = 0; d < 3; ++d) lsv[d] += tw[e] * tt[4 + d];
#pragma unroll
                        for (int t = 0; t < TM; ++t) tw6[t] += ti[e] == t ? tw[e] : 0.f;
                    }
                }
#pragma unroll
                for (int d = 0; d < 4; ++d) qn += q[d] * q[d];
                const float iqn = __builtin_amdgcn_rsqf(qn);  // 1 / |q|
                const float qw = q[0] * iqn, qx = q[1] * iqn, qy = q[2] * iqn, qz = q[3] * iqn;
                const float R[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                                    2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                                    2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
                float s[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) s[d] = __expf(lsv[d]);
                float M[9];  // R diag(s)
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int c = 0; c < 3; ++c) M[3 * r + c] = R[3 * r + c] * s[c];
                float V[6];  // Tm M, Sigma2D = V V^T + low-pass
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int c = 0; c < 3; ++c) V[3 * a + c] = Tm[3 * a] * M[c] + Tm[3 * a + 1] * M[3 + c] + Tm[3 * a + 2] * M[6 + c];
                const float SA = V[0] * V[0] + V[1] * V[1] + V[2] * V[2] + k.dilation;
                const float SB = V[0] * V[3] + V[1] * V[4] + V[2] * V[5];
                const float SC = V[3] * V[3] + V[4] * V[4] + V[5] * V[5] + k.dilation;
                // conic = inverse: a = C/det, b = -B/det, c = A/det
                const float det = SA * SC - SB * SB, idet = rcp(det), id2 = idet * idet;
                // dl/dmu = Q (m0, m1) plus the boundary point's own position gradient
                const float dmux = (SC * m0 - SB * m1) * idet + dbx;
                const float dmuy = (SA * m1 - SB * m0) * idet + dby;
                const float dA = (-SC * SC * dqa + SB * SC * dqb - SB * SB * dqc) * id2;
                const float dB = (2.f * SB * SC * dqa - (SA * SC + SB * SB) * dqb + 2.f * SA * SB * dqc) * id2;
                const float dC = (-SB * SB * dqa + SA * SB * dqb - SA * SA * dqc) * id2;
                // d/dV = 2 Gs V with Gs = [[dA, dB/2], [dB/2, dC]]
                float dV[6];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    dV[c] = 2.f * dA * V[c] + dB * V[3 + c];
                    dV[3 + c] = dB * V[c] + 2.f * dC * V[3 + c];
                }
                float dTm[6], dM[9];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int r = 0; r < 3; ++r)
                        dTm[3 * a + r] = dV[3 * a] * M[3 * r] + dV[3 * a + 1] * M[3 * r + 1] + dV[3 * a + 2] * M[3 * r + 2];
#pragma unroll
                for (int r = 0; r < 3; ++r)
#pragma unroll
                    for (int c = 0; c < 3; ++c) dM[3 * r + c] = Tm[r] * dV[c] + Tm[3 + r] * dV[3 + c];
                float dR[9];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float ds = 0.f;
#pragma unroll
                    for (int r = 0; r < 3; ++r) { ds += dM[3 * r + c] * R[3 * r + c]; dR[3 * r + c] = dM[3 * r + c] * s[c]; }
                    dls[c] = ds * s[c];
                }
                {   // rotation matrix -> unit quaternion -> raw quaternion
                    float gw = 2.f * (-qz * dR[1] + qy * dR[2] + qz * dR[3] - qx * dR[5] - qy * dR[6] + qx * dR[7]);
                    float gx = 2.f * (qy * dR[1] + qz * dR[2] + qy * dR[3] - 2.f * qx * dR[4] - qw * dR[5] + qz * dR[6] + qw * dR[7] - 2.f * qx * dR[8]);
                    float gy = 2.f * (-2.f * qy * dR[0] + qx * dR[1] + qw * dR[2] + qx * dR[3] + qz * dR[5] - qw * dR[6] + qz * dR[7] - 2.f * qy * dR[8]);
                    float gz = 2.f * (-2.f * qz * dR[0] - qw * dR[1] + qx * dR[2] + qw * dR[3] - 2.f * qz * dR[4] + qy * dR[5] + qx * dR[6] + qy * dR[7]);
                    const float dot = qw * gw + qx * gx + qy * gy + qz * gz;
                    dq[0] = (gw - qw * dot) * iqn; dq[1] = (gx - qx * dot) * iqn;
                    dq[2] = (gy - qy * dot) * iqn; dq[3] = (gz - qz * dot) * iqn;
                }
                // dJ = dTm W^T (J has four non-zero entries)
                float dJ00 = dTm[0] * W[0] + dTm[1] * W[1] + dTm[2] * W[2];
                float dJ02 = dTm[0] * W[6] + dTm[1] * W[7] + dTm[2] * W[8];
                float dJ11 = dTm[3] * W[3] + dTm[4] * W[4] + dTm[5] * W[5];
                float dJ12 = dTm[3] * W[6] + dTm[4] * W[7] + dTm[5] * W[8];
                if (dsig != 0.f) {
                    // sigma = 3 sqrt(lambda_max(r_b^2 J J^T + low-pass)), r_b = r_ref / sharpness
                    const float sh = raw[7];
                    const float ish = rcp(sh), rb = k.r_ref * ish, r2 = rb * rb;
                    const float ma = r2 * (J00 * J00 + J02 * J02) + k.dilation;
                    const float mb = r2 * J02 * J12;
                    const float mc = r2 * (J11 * J11 + J12 * J12) + k.dilation;
                    const float hd = 0.5f * (ma - mc);
                    const float sq = sqrtf(hd * hd + mb * mb);
                    const float lam = 0.5f * (ma + mc) + sq;
                    const float dlam = dsig * 1.5f * __builtin_amdgcn_rsqf(lam);
                    float dma, dmb, dmc;
                    if (sq > 0.f) {
                        const float isq = rcp(sq);
                        dma = dlam * (0.5f + 0.5f * hd * isq);
                        dmc = dlam * (0.5f - 0.5f * hd * isq);
                        dmb = dlam * mb * isq;
                    } else {
                        dma = dmc = 0.5f * dlam;
                        dmb = 0.f;
                    }
                    dJ00 += 2.f * r2 * J00 * dma;
                    dJ02 += 2.f * r2 * J02 * dma + r2 * J12 * dmb;
                    dJ12 += r2 * J02 * dmb + 2.f * r2 * J12 * dmc;
                    dJ11 += 2.f * r2 * J11 * dmc;
                    const float dr2 = dma * (J00 * J00 + J02 * J02) + dmb * J02 * J12 + dmc * (J11 * J11 + J12 * J12);
                    dsh = dr2 * 2.f * rb * (-rb * ish);
                }
                // mu = (fx t_x/t_z + cx, fy t_y/t_z + cy) and J(t)
                const float iz2 = iz * iz, iz3 = iz2 * iz;
                float dt[3];
                dt[0] = dmux * fx * iz - dJ02 * fx * iz2;
                dt[1] = dmuy * fy * iz - dJ12 * fy * iz2;
                dt[2] = -dmux * fx * t[0] * iz2 - dmuy * fy * t[1] * iz2 - dJ00 * fx * iz2 + dJ02 * 2.f * fx * t[0] * iz3 -
                        dJ11 * fy * iz2 + dJ12 * 2.f * fy * t[1] * iz3;
#pragma unroll
                for (int c = 0; c < 3; ++c) dS[c] = W[c] * dt[0] + W[3 + c] * dt[1] + W[6 + c] * dt[2];
                if constexpr (EXT) {
                    if (k.K > 0) {
                        // SH colour: dl/dsh_j = Y_j dl/dc; the view direction
                        // d = (S - C) / |S - C| moves with S: dl/dS += (I - d d^T) g / |S - C|
                        float C[3], dv[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c) C[c] = -(W[c] * cm[9] + W[3 + c] * cm[10] + W[6 + c] * cm[11]);
#pragma unroll
                        for (int c = 0; c < 3; ++c) dv[c] = S[c] - C[c];
                        const float len = sqrtf(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]), il = rcp(len);
#pragma unroll
                        for (int c = 0; c < 3; ++c) dv[c] *= il;
                        // g = sum_j (dl/dc . sh_j) grad Y_j, taken as the basis is built
                        const float *shc = rec + patch_sh_off(NCP, k.T);
                        float gd[3] = {0.f, 0.f, 0.f};
                        sh_basis_cb<float>(sh_degree_of(k.K), dv[0], dv[1], dv[2],
                                           [&](int j, float Yj, float gx, float gy, float gz) {
                            Yv[j] = Yj;
                            const float w = dcol[0] * shc[3 * j] + dcol[1] * shc[3 * j + 1] + dcol[2] * shc[3 * j + 2];
                            gd[0] += w * gx;
                            gd[1] += w * gy;
                            gd[2] += w * gz;
                        });
                        const float dot = dv[0] * gd[0] + dv[1] * gd[1] + dv[2] * gd[2];
#pragma unroll
                        for (int c = 0; c < 3; ++c) dS[c] += (gd[c] - dv[c] * dot) * il;
                    }
                }
            }
        }
    }
    // per primitive present in the wave: a reduce-scatter of its NV sums over
    // the wave, then one multi-lane atomic add per 64 values
    // value order: ctrl [d][c], colour [d][c], log-scale [d][t], quaternion
    // [d][t], opacity, sharpness, SH [c][j]
    auto value = [&](int j) -> float {  // j is a compile-time constant after unrolling
        if (j < 3 * NCP) return B[j % NCP] * dS[j / NCP];
        if (j < 6 * NCP) return B[(j - 3 * NCP) % NCP] * dcol[(j - 3 * NCP) / NCP];
        const int r = j - 6 * NCP;
        if (r < 3 * TM) return EXT ? dls[r / TM] * tw6[r % TM] : dls[r];
        if (r < 7 * TM) return EXT ? dq[(r - 3 * TM) / TM] * tw6[(r - 3 * TM) % TM] : dq[r - 3];
        if (r == 7 * TM) return dop;
        if (r == 7 * TM + 1) return dsh;
        const int h = r - 7 * TM - 2;
        return KM > 0 ? Yv[h % (KM > 0 ? KM : 1)] * dcol[h / (KM > 0 ? KM : 1)] : 0.f;
    };
    for (unsigned long long pending = __ballot(act); pending;) {
        const int gl = __builtin_amdgcn_readlane(prim, __ffsll((long long)pending) - 1);
        const bool mine = act && prim == gl;
        pending &= ~__ballot(mine);
        const int slot = table_slot<SLOTS>(slot_prim, gl, lane);
        reduce_chunk<0, NV>(value, target, mine, gl, lane, table, slot);
        if constexpr (NV > 64) reduce_chunk<64, NV>(value, target, mine, gl, lane, table, slot);
        if constexpr (NV > 128) reduce_chunk<128, NV>(value, target, mine, gl, lane, table, slot);
        if constexpr (NV > 192) reduce_chunk<192, NV>(value, target, mine, gl, lane, table, slot);
    }
    }  // passes
    // the region's sums: one global atomic per (primitive, parameter)
    __syncthreads();
    for (int i = threadIdx.x; i < SLOTS * NV; i += blockDim.x) {
        const int s = i / NV, j = i - s * NV;
        const int p = slot_prim[s];
        const float val = table[i];
        if (p >= 0 && val != 0.f) {
            float *t = target(j, p);
            if (t) unsafeAtomicAdd(t, val);
        }
    }
}

hipError_t launch_param_bwd(const Consts &k, const ViewTable &vt, const PrimPtrs &pr, const float *cams,
                            const StatePtrs &st, const GradPtrs &gr, hipStream_t s) {
    const bool ext = k.T > 1 || k.K > 0;  // resolution-3 maps or SH colour
    // pixel records (in the lattice variant: boundary points only), then the lattice Gaussians
    int64_t regions = 0;
    for (int v = 0; v < vt.n; ++v)
        regions += (int64_t)((vt.v[v].W + kRegion - 1) / kRegion) * ((vt.v[v].H + kRegion - 1) / kRegion);
    for (int lat = 0; lat < (k.NL > 0 ? 2 : 1); ++lat) {
        const int64_t groups = lat ? ((int64_t)vt.n * k.P * k.NL + kLatPerGroup - 1) / kLatPerGroup : regions;
        dim3 grid((unsigned)groups), block(256);
#define BGT_PB(D, E, LT) hipLaunchKernelGGL((k_param_bwd<D, E, LT>), grid, block, 0, s, k, vt, pr, cams, st, gr, st.patch)
#define BGT_PB_CASE(D)                                  \
    case D:                                             \
        if (lat) {                                      \
            if (ext) BGT_PB(D, true, true);             \
            else BGT_PB(D, false, true);                \
        } else {                                        \
            if (ext) BGT_PB(D, true, false);            \
            else BGT_PB(D, false, false);               \
        }                                               \
        break;
        switch (k.degree) {
            BGT_PB_CASE(1) BGT_PB_CASE(2) BGT_PB_CASE(3) BGT_PB_CASE(4) BGT_PB_CASE(5)
            default: return hipErrorInvalidValue;
        }
#undef BGT_PB_CASE
#undef BGT_PB
    }
    return hipGetLastError();
}

}  // namespace bgt
