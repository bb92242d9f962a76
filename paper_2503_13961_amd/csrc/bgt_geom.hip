// Geometry stages of the BG-Triangle rasterizer on gfx950:
//   tessellation lattice (Sec. 3.1 Eq. 1-2 at the nodes of Sec. 3.2),
//   projection + fixed-point snapping, depth-tested raster into a 64-bit
//   z-buffer, and per-pixel resolve + sub-primitive generation (Sec. 3.2,
//   Eq. 3-5, EWA splatting) with the boundary set B and boundary radii.
//
// Every quantity that decides an integer (snapped coordinates, coverage,
// depth order, tile ranges) is computed in FP64.  The blending stages read
// FP32 copies.
#include "bgt_internal.h"
#include "bgt_sh.h"

namespace bgt {

// ------------------------------------------------------------ clearing

// Clears the table's segments laid end to end in 16-byte chunks, each
// segment's chunks starting at its own base: one store per chunk, or word by
// word for a segment's last chunk and for a base that is not 16-byte aligned.
__global__ void k_zero(ZeroTable t, int64_t total_chunks) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < total_chunks;
         c += (int64_t)gridDim.x * blockDim.x) {
        int s = 0;
        int64_t first = 0;  // first chunk of segment s
        while (s + 1 < t.n && c >= first + ((t.words[s] + 3) >> 2)) {
            first += (t.words[s] + 3) >> 2;
            ++s;
        }
        const int64_t w = (c - first) * 4, n = t.words[s];
        uint32_t *q = t.p[s] + w;
        if (w + 4 <= n && ((uintptr_t)t.p[s] & 15) == 0) {
            *(uint4 *)q = make_uint4(0u, 0u, 0u, 0u);
        } else {
            for (int i = 0; i < 4 && w + i < n; ++i) q[i] = 0u;
        }
    }
}

hipError_t launch_zero(const ZeroTable &t, hipStream_t s) {
    int64_t chunks = 0;
    for (int i = 0; i < t.n; ++i) chunks += (t.words[i] + 3) >> 2;
    if (chunks == 0) return hipSuccess;
    int64_t b = (chunks + 255) / 256;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)b), dim3(256), 0, s, t, chunks);
    return hipGetLastError();
}

// ------------------------------------------------------------ Bernstein basis

// n!/(i! j! k!) u^i v^j w^k in the order of Eq. 1's double sum.
template <int DEG, typename T>
__device__ __forceinline__ void bernstein(T u, T v, T w, T *B) {
    constexpr double fact[6] = {1.0, 1.0, 2.0, 6.0, 24.0, 120.0};
    T pu[DEG + 1], pv[DEG + 1], pw[DEG + 1];
    pu[0] = pv[0] = pw[0] = T(1);
#pragma unroll
    for (int e = 1; e <= DEG; ++e) {
        pu[e] = pu[e - 1] * u;
        pv[e] = pv[e - 1] * v;
        pw[e] = pw[e - 1] * w;
    }
    int idx = 0;
#pragma unroll
    for (int i = 0; i <= DEG; ++i)
#pragma unroll
        for (int j = 0; j <= DEG - i; ++j) {
            const int kk = DEG - i - j;
            B[idx++] = T(fact[DEG] / (fact[i] * fact[j] * fact[kk])) * pu[i] * pv[j] * pw[kk];
        }
}

// ------------------------------------------------------------ tessellation

// (a, b) of lattice node m: a = 0..L outer, b = 0..L-a inner
__device__ __forceinline__ void lattice_node(int L, int m, int &a, int &b) {
    a = 0;
    while (m > L - a) { m -= L - a + 1; ++a; }
    b = m;
}

__device__ __forceinline__ int lattice_index(int L, int a, int b) { return a * (L + 1) - a * (a - 1) / 2 + b; }

// lattice indices of the three corners of flat sub-triangle s (up triangles
// (a,b),(a+1,b),(a,b+1) first, then down triangles (a+1,b),(a+1,b+1),(a,b+1))
__device__ __forceinline__ void subtri_corners(int L, int s, int *m) {
    const int up = L * (L + 1) / 2;
    int a = 0;
    if (s < up) {
        while (s >= L - a) { s -= L - a; ++a; }
        m[0] = lattice_index(L, a, s);
        m[1] = lattice_index(L, a + 1, s);
        m[2] = lattice_index(L, a, s + 1);
    } else {
        s -= up;
        while (s >= L - 1 - a) { s -= L - 1 - a; ++a; }
        m[0] = lattice_index(L, a + 1, s);
        m[1] = lattice_index(L, a + 1, s + 1);
        m[2] = lattice_index(L, a, s + 1);
    }
}

// the same corners with their lattice coordinates (a, b)
__device__ __forceinline__ void subtri_corners_ab(int L, int s, int *m, int *ca, int *cb) {
    const int up = L * (L + 1) / 2;
    int a = 0;
    if (s < up) {
        while (s >= L - a) { s -= L - a; ++a; }
        ca[0] = a; cb[0] = s; ca[1] = a + 1; cb[1] = s; ca[2] = a; cb[2] = s + 1;
    } else {
        s -= up;
        while (s >= L - 1 - a) { s -= L - 1 - a; ++a; }
        ca[0] = a + 1; cb[0] = s; ca[1] = a + 1; cb[1] = s + 1; ca[2] = a; cb[2] = s + 1;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) m[c] = lattice_index(L, ca[c], cb[c]);
}

template <int DEG>
__global__ void k_tessellate(Consts k, PrimPtrs pr, double *wverts, float *verts_out) {
    constexpr int NCP = (DEG + 1) * (DEG + 2) / 2;
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)k.VL * k.P) return;
    const int p = (int)(idx % k.P), m = (int)(idx / k.P);
    int a, b;
    lattice_node(k.L, m, a, b);
    const double u = (double)a / k.L, v = (double)b / k.L, w = (double)(k.L - a - b) / k.L;
    double B[NCP];
    bernstein<DEG>(u, v, w, B);
    double S[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < NCP; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) S[d] += B[c] * (double)pr.ctrl[((int64_t)d * NCP + c) * k.P + p];
    if (wverts)
        for (int d = 0; d < 3; ++d) wverts[((int64_t)m * k.P + p) * 3 + d] = S[d];
    if (verts_out)
        for (int d = 0; d < 3; ++d) verts_out[((int64_t)d * k.VL + m) * k.P + p] = (float)S[d];
}

hipError_t launch_tessellate(const Consts &k, const PrimPtrs &pr, double *wverts, float *verts_out,
                             hipStream_t s) {
    int64_t n = (int64_t)k.VL * k.P;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    switch (k.degree) {
        case 1: hipLaunchKernelGGL(k_tessellate<1>, grid, block, 0, s, k, pr, wverts, verts_out); break;
        case 2: hipLaunchKernelGGL(k_tessellate<2>, grid, block, 0, s, k, pr, wverts, verts_out); break;
        case 3: hipLaunchKernelGGL(k_tessellate<3>, grid, block, 0, s, k, pr, wverts, verts_out); break;
        case 4: hipLaunchKernelGGL(k_tessellate<4>, grid, block, 0, s, k, pr, wverts, verts_out); break;
        case 5: hipLaunchKernelGGL(k_tessellate<5>, grid, block, 0, s, k, pr, wverts, verts_out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ per-patch setup

// Per-patch record (layout at patch_dw): the control and colour points and
// the opacity copied as they are, and Eq. 5 with a resolution-1 attribute
// map, one rotation and scale per patch: R(q/|q|) diag(exp(log_scale)) and
// r_b^2 = (r_ref / sharpness)^2 in FP64.
__global__ void k_prim_setup(Consts k, PrimPtrs pr, float *patch) {
    // one thread per word of a patch record, the patch index fastest (the
    // parameter arrays are read in runs of consecutive patches); the thread
    // of M's first word computes the rotation-scale setup and writes all 20
    // of its words
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= (int64_t)k.P * k.pdw) return;
    const int p = (int)(idx % k.P), i = (int)(idx / k.P);
    const int ncp = k.ncp, mo = patch_m_off(ncp), qo = patch_q_off(ncp);
    const int xo = patch_x_off(ncp), so = patch_sh_off(ncp, k.T);
    const bool ext = k.T > 1 || k.K > 0;  // the texels and SH coefficients are stored
    float *o = patch + (int64_t)p * k.pdw;
    if (i < 6 * ncp) {
        const float *src = i < 3 * ncp ? pr.ctrl : pr.color;
        const int j = i < 3 * ncp ? i : i - 3 * ncp, c = j / 3, d = j % 3;
        o[i] = src[((int64_t)d * ncp + c) * k.P + p];
    } else if (i == 6 * ncp) {
        o[i] = pr.opacity[p];
    } else if (i == 6 * ncp + 1) {
        o[i] = 0.f;
    } else if (i == mo) {
        double q[4], qn = 0.0;
#pragma unroll
        for (int d = 0; d < 4; ++d) { q[d] = pr.quat[(int64_t)d * k.T * k.P + p]; qn += q[d] * q[d]; }
        qn = sqrt(qn);
#pragma unroll
        for (int d = 0; d < 4; ++d) q[d] /= qn;
        const double w = q[0], x = q[1], y = q[2], z = q[3];
        const double Rq[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                              2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                              2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
        double sc[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) sc[d] = exp((double)pr.log_scale[(int64_t)d * k.T * k.P + p]);
        double *m = (double *)(o + mo);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) m[3 * r + c] = Rq[3 * r + c] * sc[c];
        const double rb = (double)k.r_ref / (double)pr.sharp[p];
        m[9] = rb * rb;
    } else if (i < qo) {
        // (M's other words)
    } else if (i < qo + 4) {  // the raw quaternion, log-scales and sharpness
        o[i] = pr.quat[(int64_t)(i - qo) * k.T * k.P + p];
    } else if (i < qo + 7) {
        o[i] = pr.log_scale[(int64_t)(i - qo - 4) * k.T * k.P + p];
    } else if (i == qo + 7) {
        o[i] = pr.sharp[p];
    } else if (ext && i < xo + 7 * k.T) {  // every texel of the rotation and scale maps
        const int t = (i - xo) / 7, e = (i - xo) % 7;
        o[i] = e < 4 ? pr.quat[((int64_t)e * k.T + t) * k.P + p] : pr.log_scale[((int64_t)(e - 4) * k.T + t) * k.P + p];
    } else if (ext && i < so + 3 * k.K) {  // then the SH coefficients
        const int j = (i - so) / 3, c = (i - so) % 3;
        o[i] = pr.sh[((int64_t)c * k.K + j) * k.P + p];
    } else {
        o[i] = 0.f;
    }
}

// ------------------------------------------------------------ projection

struct Cam {
    double R[9], t[3], fx, fy, cx, cy;
};

__device__ __forceinline__ Cam load_cam(const float *cams, int v) {
    Cam c;
    const float *q = cams + 16 * v;
#pragma unroll
    for (int i = 0; i < 9; ++i) c.R[i] = (double)q[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) c.t[i] = (double)q[9 + i];
    c.fx = q[12]; c.fy = q[13]; c.cx = q[14]; c.cy = q[15];
    return c;
}

__device__ __forceinline__ void cam_apply(const Cam &c, const double *X, double *t) {
#pragma unroll
    for (int r = 0; r < 3; ++r) t[r] = c.R[3 * r] * X[0] + c.R[3 * r + 1] * X[1] + c.R[3 * r + 2] * X[2] + c.t[r];
}

__global__ void k_project(Consts k, ViewTable vt, const float *cams, const double *wverts, VertRec *verts) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t per_view = (int64_t)k.VL * k.P;
    if (idx >= per_view * vt.n) return;
    const int v = (int)(idx / per_view);
    const int64_t mp = idx % per_view;
    const Cam c = load_cam(cams, v);
    double X[3] = {wverts[mp * 3], wverts[mp * 3 + 1], wverts[mp * 3 + 2]}, t[3];
    cam_apply(c, X, t);
    VertRec r;
    r.x = r.y = r.iz = 0.0;
    r.X = INT32_MIN;
    r.Y = 0;
    if (t[2] > (double)k.z_near) {
        const double x = c.fx * t[0] / t[2] + c.cx;
        const double y = c.fy * t[1] / t[2] + c.cy;
        const double lim = 1048576.0;  // 2^20 px keeps edge functions inside int64
        if (fabs(x) < lim && fabs(y) < lim) {
            r.x = x;
            r.y = y;
            r.iz = 1.0 / t[2];
            r.X = (int32_t)rint(x * 256.0);
            r.Y = (int32_t)rint(y * 256.0);
        }
    }
    verts[idx] = r;
}

// ------------------------------------------------------------ raster

struct TriSetup {
    int64_t X[3], Y[3];
    double iz[3];
    int64_t A;
    bool own[3];
    int i0, i1, j0, j1;
};

__device__ __forceinline__ int64_t floor_div256(int64_t a) { return a >> 8; }
__device__ __forceinline__ int64_t ceil_div256(int64_t a) { return -((-a) >> 8); }

// Top-left ownership of a directed edge (exactly one of a->b, b->a owns it).
__device__ __forceinline__ bool owned(int64_t dx, int64_t dy) { return dy > 0 || (dy == 0 && dx < 0); }

__device__ __forceinline__ int64_t edge_fn(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t px, int64_t py) {
    return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}

// Returns false when the triangle is culled or misses the image.
__device__ __forceinline__ bool tri_setup(const Consts &k, const ViewInfo &vi, const VertRec *vv, int s, int p,
                                          TriSetup &ts) {
    int m[3];
    subtri_corners(k.L, s, m);
    // (the three corners are loaded before any is tested, so the lane waits
    // for one round trip)
    int32_t X[3], Y[3];
    double iz[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {  // (iz, X, Y: the record's last 16 bytes, one load)
        const int4 w = *(const int4 *)((const char *)(vv + (int64_t)m[c] * k.P + p) + offsetof(VertRec, iz));
        iz[c] = __hiloint2double(w.y, w.x);
        X[c] = w.z;
        Y[c] = w.w;
    }
    const bool culled = (X[0] == INT32_MIN) | (X[1] == INT32_MIN) | (X[2] == INT32_MIN);  // near-plane cull
    VertRec r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) { r[c].X = X[c]; r[c].Y = Y[c]; r[c].iz = iz[c]; }
    int64_t A = edge_fn(r[0].X, r[0].Y, r[1].X, r[1].Y, r[2].X, r[2].Y);
    if (culled | (A == 0)) return false;
    int o1 = 1, o2 = 2;
    if (A < 0) { o1 = 2; o2 = 1; A = -A; }
    const int ord[3] = {0, o1, o2};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        ts.X[c] = r[ord[c]].X;
        ts.Y[c] = r[ord[c]].Y;
        ts.iz[c] = r[ord[c]].iz;
    }
    ts.A = A;
    ts.own[0] = owned(ts.X[2] - ts.X[1], ts.Y[2] - ts.Y[1]);
    ts.own[1] = owned(ts.X[0] - ts.X[2], ts.Y[0] - ts.Y[2]);
    ts.own[2] = owned(ts.X[1] - ts.X[0], ts.Y[1] - ts.Y[0]);
    int64_t minX = min(ts.X[0], min(ts.X[1], ts.X[2])), maxX = max(ts.X[0], max(ts.X[1], ts.X[2]));
    int64_t minY = min(ts.Y[0], min(ts.Y[1], ts.Y[2])), maxY = max(ts.Y[0], max(ts.Y[1], ts.Y[2]));
    int64_t i0 = ceil_div256(minX - 128), i1 = floor_div256(maxX - 128);
    int64_t j0 = ceil_div256(minY - 128), j1 = floor_div256(maxY - 128);
    if (i0 < 0) i0 = 0;
    if (j0 < 0) j0 = 0;
    if (i1 > vi.W - 1) i1 = vi.W - 1;
    if (j1 > vi.H - 1) j1 = vi.H - 1;
    if (i0 > i1 || j0 > j1) return false;
    ts.i0 = (int)i0; ts.i1 = (int)i1; ts.j0 = (int)j0; ts.j1 = (int)j1;
    return true;
}

// Coverage of pixel centre (i, j) and, when covered, the z-buffer candidate:
// the 1/z plane (affine in screen space) at the centre, high 40 bits of its
// FP64 pattern, then the inverted triangle id (lower id wins ties).
__device__ __forceinline__ unsigned long long raster_pixel(const TriSetup &ts, int i, int j, uint32_t tri) {
    const int64_t px = 256 * (int64_t)i + 128, py = 256 * (int64_t)j + 128;
    const int64_t E0 = edge_fn(ts.X[1], ts.Y[1], ts.X[2], ts.Y[2], px, py);
    const int64_t E1 = edge_fn(ts.X[2], ts.Y[2], ts.X[0], ts.Y[0], px, py);
    const int64_t E2 = edge_fn(ts.X[0], ts.Y[0], ts.X[1], ts.Y[1], px, py);
    const bool in = (E0 > 0 || (E0 == 0 && ts.own[0])) && (E1 > 0 || (E1 == 0 && ts.own[1])) &&
                    (E2 > 0 || (E2 == 0 && ts.own[2]));
    if (!in) return 0ull;
    const double key = fma((double)E2, ts.iz[2], fma((double)E1, ts.iz[1], (double)E0 * ts.iz[0])) / (double)ts.A;
    const unsigned long long kb = (unsigned long long)__double_as_longlong(key);
    return ((kb >> 24) << 24) | (unsigned long long)(0xFFFFFFu - tri);
}

// Triangles whose corners lie within this many 1/256 px of each other on
// both axes have edge functions that FP64 holds exactly at every pixel centre
// of their bounding box: each product is an integer below 2^50 and their
// difference one below 2^51.  Wider ones (rare: a small box clipped from a
// huge triangle) go to the int64 path of k_raster_big.
constexpr int64_t kExactExtent = 1ll << 25;

// Edge function of the directed edge a -> b at p, as raster_pixel's int64
// edge_fn, in FP64: exact for coordinates within kExactExtent of each other
// (the int32 differences cannot overflow: coordinates are below 2^28).
__device__ __forceinline__ double edge_f64(int ax, int ay, int bx, int by, int px, int py) {
    return fma((double)(bx - ax), (double)(py - ay), -((double)(by - ay) * (double)(px - ax)));
}

// Inclusive max-scan of x over the wave's lanes (lane l gets the largest x of
// lanes 0..l): shifts by 1, 2, 4 and 8 within each row of 16 lanes, then row
// 15's and row 31's last lanes carried into the rows after them.  A lane
// reads only lanes below it.
__device__ __forceinline__ int wave_max_scan(int x) {
    x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x111, 0xF, 0xF, false));  // row_shr:1
    x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x112, 0xF, 0xF, false));  // row_shr:2
    x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x114, 0xF, 0xF, false));  // row_shr:4
    x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x118, 0xF, 0xF, false));  // row_shr:8
    x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x142, 0xA, 0xF, false));  // row_bcast:15
    x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return x;
}

// Set-ups of a wave's 64 triangles, for the lanes that rasterize their pixels.
// (5 KB: eight waves' worth fit a CU's LDS four workgroups at a time)
struct RasterWaveLds {
    int32_t start[64];      // first pixel of the triangle in the wave's pixel sequence
    int32_t X[3][64], Y[3][64];
    double iz[3][64];
    double A[64];           // twice the area, in 1/256^2 px^2 (an integer below 2^51)
    int32_t ij0[64];        // box corner: i0 | j0 << 16
    int32_t bwo[64];        // box width | top-left ownership bits of the edges << 9 | image width << 12
    int32_t px_off[64];
    int32_t mark[64];       // per chunk of 64 pixels: the last triangle starting at each pixel
    uint32_t tri[64];
};
static_assert(sizeof(RasterWaveLds) == 5120, "four waves' set-ups in 20 KB");

// One lane per (view, sub-triangle) sets the triangle up; then the wave
// rasterizes the bounding boxes of its 64 triangles together, one pixel per
// lane over the concatenated boxes, so that lanes are not held by the
// largest box of the wave.  Coverage and the z-buffer word are those of
// raster_pixel (exact edge functions, here in FP64; FP64 1/z plane).
__global__ void __launch_bounds__(256) k_raster(Consts k, ViewTable vt, const VertRec *verts,
                                                unsigned long long *zbuf, int32_t *big, int64_t *counters) {
    __shared__ RasterWaveLds R[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    RasterWaveLds &Rw = R[wave];
    const int64_t per_view = (int64_t)k.L2 * k.P, n_tri = per_view * vt.n;
    // lane l of the launch takes triangle group (l / 8) (2^31 - 1) mod
    // n_groups, member l mod 8 (a permutation: 2^31 - 1 is a prime above the
    // group count): a wave's eight groups come from all over the views, so
    // that the waves' pixel counts vary less than those of 64 neighbouring
    // patches, while each group's corner loads stay contiguous
    const int64_t gi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, ng = (n_tri + 7) >> 3;
    const int64_t idx = (gi >> 3) < ng ? ((gi >> 3) * 2147483647ll % ng) * 8 + (gi & 7) : n_tri;
    int area = 0;
    if (idx < n_tri) {
        const int v = (int)(idx / per_view);
        const int64_t sp = idx % per_view;
        const int s = (int)(sp / k.P), p = (int)(sp % k.P);
        const ViewInfo vi = vt.v[v];
        TriSetup ts;
        if (tri_setup(k, vi, verts + (int64_t)v * k.VL * k.P, s, p, ts)) {
            const int64_t a = (int64_t)(ts.i1 - ts.i0 + 1) * (ts.j1 - ts.j0 + 1);
            const int64_t ext = max(max(ts.X[0], max(ts.X[1], ts.X[2])) - min(ts.X[0], min(ts.X[1], ts.X[2])),
                                    max(ts.Y[0], max(ts.Y[1], ts.Y[2])) - min(ts.Y[0], min(ts.Y[1], ts.Y[2])));
            if (a > kBigTriPixels || ext >= kExactExtent) {
                const long long slot = atomicAdd((unsigned long long *)&counters[C_BIGTRI], 1ull);
                if (slot < k.cap_big) big[slot] = (int32_t)idx;
                else atomicOr((unsigned long long *)&counters[C_OVERFLOW], 4ull);
            } else {
                area = (int)a;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    Rw.X[c][lane] = (int32_t)ts.X[c];
                    Rw.Y[c][lane] = (int32_t)ts.Y[c];
                    Rw.iz[c][lane] = ts.iz[c];
                }
                Rw.A[lane] = (double)ts.A;
                Rw.ij0[lane] = ts.i0 | ts.j0 << 16;  // (images are at most 16384 px a side)
                // (box width at most 256, image width at most 16384)
                Rw.bwo[lane] = (ts.i1 - ts.i0 + 1) | ((ts.own[0] ? 1 : 0) | (ts.own[1] ? 2 : 0) | (ts.own[2] ? 4 : 0)) << 9 |
                               vi.W << 12;
                Rw.px_off[lane] = vi.px_off;
                Rw.tri[lane] = (uint32_t)(p * k.L2 + s);
            }
        }
    }
    int incl = area;  // inclusive scan of the box areas over the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    const int my_start = incl - area;
    Rw.start[lane] = my_start;
    const int total = __shfl(incl, 63, 64);
    __syncthreads();
    for (int base = 0; base < total; base += 64) {
        // the triangle holding pixel e = base + lane: the last one starting
        // at or before it (a triangle with an empty box starts where the next
        // one does).  Each triangle marks its start within the chunk (those
        // before it mark pixel 0) with its index, the largest index winning;
        // a max-scan of the marks over the lanes then gives every pixel's.
        // (LDS operations of one wave complete in order: the fences keep the
        // compiler from moving them across each other)
        Rw.mark[lane] = -1;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (my_start - base < 64) atomicMax(&Rw.mark[max(my_start - base, 0)], lane);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int q = wave_max_scan(Rw.mark[lane]);  // (pixel 0's mark is set: triangle 0 starts at 0)
        const int e = base + lane;
        if (e >= total) continue;  // (the last chunk's tail; the scan above needed every lane)
        const int r = e - Rw.start[q], bwo = Rw.bwo[q], bw = bwo & 0x1FF, ij0 = Rw.ij0[q];
        // row of pixel r of the box: (r + 1/2) / bw lies at least 1/512 from
        // an integer (r < 256), far beyond the reciprocal's error
        const int dy = (int)(((float)r + 0.5f) * __builtin_amdgcn_rcpf((float)bw));
        const int i = (ij0 & 0xFFFF) + (r - dy * bw), j = (ij0 >> 16) + dy;
        // raster_pixel's coverage and z-buffer word, with the edge functions
        // in FP64 (exact here: the triangle is narrower than kExactExtent)
        const int px = 256 * i + 128, py = 256 * j + 128;
        const int X0 = Rw.X[0][q], X1 = Rw.X[1][q], X2 = Rw.X[2][q];
        const int Y0 = Rw.Y[0][q], Y1 = Rw.Y[1][q], Y2 = Rw.Y[2][q];
        const double E0 = edge_f64(X1, Y1, X2, Y2, px, py);
        const double E1 = edge_f64(X2, Y2, X0, Y0, px, py);
        const double E2 = edge_f64(X0, Y0, X1, Y1, px, py);
        const int own = (bwo >> 9) & 7;
        const bool in = (E0 > 0.0 || (E0 == 0.0 && (own & 1))) && (E1 > 0.0 || (E1 == 0.0 && (own & 2))) &&
                        (E2 > 0.0 || (E2 == 0.0 && (own & 4)));
        if (in) {
            const double key = fma(E2, Rw.iz[2][q], fma(E1, Rw.iz[1][q], E0 * Rw.iz[0][q])) / Rw.A[q];
            const unsigned long long kb = (unsigned long long)__double_as_longlong(key);
            const unsigned long long c = ((kb >> 24) << 24) | (unsigned long long)(0xFFFFFFu - Rw.tri[q]);
            // the z-buffer only grows: a word already at or above c (however
            // stale the read) means the atomic would change nothing
            unsigned long long *z = &zbuf[Rw.px_off[q] + (int64_t)j * (bwo >> 12) + i];
            if (__hip_atomic_load(z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < c) atomicMax(z, c);
        }
    }
}

// Triangles with a large bounding box: one block each, pixels over threads.
__global__ void k_raster_big(Consts k, ViewTable vt, const VertRec *verts, unsigned long long *zbuf,
                             const int32_t *big, const int64_t *counters) {
    int64_t n = counters[C_BIGTRI];
    if (n > k.cap_big) n = k.cap_big;
    const int64_t per_view = (int64_t)k.L2 * k.P;
    for (int64_t q = blockIdx.x; q < n; q += gridDim.x) {
        const int64_t idx = big[q];
        const int v = (int)(idx / per_view);
        const int64_t sp = idx % per_view;
        const int s = (int)(sp / k.P), p = (int)(sp % k.P);
        const ViewInfo vi = vt.v[v];
        TriSetup ts;
        if (!tri_setup(k, vi, verts + (int64_t)v * k.VL * k.P, s, p, ts)) continue;
        const uint32_t tri = (uint32_t)(p * k.L2 + s);
        const int bw = ts.i1 - ts.i0 + 1;
        const int64_t area = (int64_t)bw * (ts.j1 - ts.j0 + 1);
        unsigned long long *zb = zbuf + vi.px_off;
        for (int64_t e = threadIdx.x; e < area; e += blockDim.x) {
            const int i = ts.i0 + (int)(e % bw), j = ts.j0 + (int)(e / bw);
            const unsigned long long c = raster_pixel(ts, i, j, tri);
            if (c) atomicMax(&zb[(int64_t)j * vi.W + i], c);
        }
    }
}

// ------------------------------------------------------------ resolve + generation

__device__ __forceinline__ int zb_prim(unsigned long long z, int L2) {
    return z == 0ull ? -1 : (int)((0xFFFFFFu - (uint32_t)(z & 0xFFFFFFull)) / (uint32_t)L2);
}

// pixel-centre index range [lo, hi] covered by the closed interval [c - r, c + r]
__device__ __forceinline__ void centre_range(double c, double r, int n, int &lo, int &hi) {
    double a = ceil(c - r - 0.5), b = floor(c + r - 0.5);
    if (a < 0.0) a = 0.0;
    if (b > (double)(n - 1)) b = (double)(n - 1);
    if (!(a <= b)) { lo = 1; hi = 0; return; }
    lo = (int)a;
    hi = (int)b;
}

// EWA projection of a Gaussian at camera-space point t with M = R diag(s)
// (Eq. 5): mean, J, and Sigma2D = (J W M)(J W M)^T + low-pass.  False when
// t lies behind z_near.
struct Ewa {
    double tz, J00, J02, J11, J12, SA, SB, SC, mux, muy;
};

__device__ __forceinline__ bool ewa_project(const Consts &k, const Cam &c, const double *t, const double *Mv, Ewa &e) {
    if (!(t[2] > (double)k.z_near)) return false;
    const double tz = t[2], iz = 1.0 / tz;
    e.tz = tz;
    e.J00 = c.fx * iz;
    e.J02 = -c.fx * t[0] * iz * iz;
    e.J11 = c.fy * iz;
    e.J12 = -c.fy * t[1] * iz * iz;
    double Tm[6];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
        Tm[cc] = e.J00 * c.R[cc] + e.J02 * c.R[6 + cc];
        Tm[3 + cc] = e.J11 * c.R[3 + cc] + e.J12 * c.R[6 + cc];
    }
    double V0[3], V1[3];  // V = Tm M, Sigma2D = V V^T + low-pass
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
        V0[cc] = Tm[0] * Mv[cc] + Tm[1] * Mv[3 + cc] + Tm[2] * Mv[6 + cc];
        V1[cc] = Tm[3] * Mv[cc] + Tm[4] * Mv[3 + cc] + Tm[5] * Mv[6 + cc];
    }
    e.SA = V0[0] * V0[0] + V0[1] * V0[1] + V0[2] * V0[2] + k.dilation;
    e.SB = V0[0] * V1[0] + V0[1] * V1[1] + V0[2] * V1[2];
    e.SC = V1[0] * V1[0] + V1[1] * V1[1] + V1[2] * V1[2] + k.dilation;
    e.mux = c.fx * t[0] * iz + c.cx;
    e.muy = c.fy * t[1] * iz + c.cy;
    return true;
}

// rotation-scale M = R(q / |q|) diag(e^s) of Eq. 5 from a raw quaternion and log-scales
__device__ __forceinline__ void rot_scale(const double *qi, const double *lsi, double *Mv) {
    const double qn = 1.0 / sqrt(qi[0] * qi[0] + qi[1] * qi[1] + qi[2] * qi[2] + qi[3] * qi[3]);
    const double w = qi[0] * qn, x = qi[1] * qn, y = qi[2] * qn, z = qi[3] * qn;
    const double Rq[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                          2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                          2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    const double sc[3] = {exp(lsi[0]), exp(lsi[1]), exp(lsi[2])};
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) Mv[3 * r + cc] = Rq[3 * r + cc] * sc[cc];
}

template <int DEG, bool EXT>
__global__ void __launch_bounds__(256) k_gen(Consts k, ViewTable vt, PrimPtrs pr, const float *cams, StatePtrs st,
                                             const float *__restrict__ patch) {
    constexpr int NCP = (DEG + 1) * (DEG + 2) / 2;
    constexpr int MO = patch_m_off(NCP);
    const int PD = k.pdw;
    const int lane = threadIdx.x & 63;
    // the 8x8 block is wave-uniform, so its view is found with scalar loads
    const int blk = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    int v, x, y;
    const bool act = block8_pixel(vt, blk, lane, v, x, y);
    bool fg = false, isb = false;
    int gt0 = 1, gt1 = 0, gu0 = 1, gu1 = 0, bt0 = 1, bt1 = 0, bu0 = 1, bu1 = 0;  // tile rectangles
    const ViewInfo vi = vt.v[v];
    const int lp = y * vi.W + x, pix = vi.px_off + lp;
    // the pixel's z-buffer word and its in-image 4-neighbours' (an edge pixel
    // reads itself in place of a missing neighbour), loaded together
    int tri = -1, p = -1;
    bool bnd = false;
    if (act) {
        const unsigned long long *zr = st.zbuf + vi.px_off;
        const int nl = x > 0 ? lp - 1 : lp, nr = x + 1 < vi.W ? lp + 1 : lp;
        const int nu = y > 0 ? lp - vi.W : lp, nd = y + 1 < vi.H ? lp + vi.W : lp;
        const unsigned long long z = zr[lp], z0 = zr[nl], z1 = zr[nr], z2 = zr[nu], z3 = zr[nd];
        tri = z == 0ull ? -1 : (int)(0xFFFFFFu - (uint32_t)(z & 0xFFFFFFull));
        // B: a neighbour shows another primitive (or the background)
        p = zb_prim(z, k.L2);
        // (none in the variant without blending coefficients)
        bnd = !(k.flags & BGT_FLAG_NO_BOUNDARY) &&
              (zb_prim(z0, k.L2) != p || zb_prim(z1, k.L2) != p || zb_prim(z2, k.L2) != p || zb_prim(z3, k.L2) != p);
    }
    // perspective-correct barycentrics in the winning flat triangle and the
    // Bernstein weights there (foreground lanes)
    double B[NCP];
    float2 uvo = make_float2(0.f, 0.f);
    int ti[3] = {0, 0, 0};      // Eq. 5: texels of the pixel's lattice triangle and their weights
    double tw[3] = {0.0, 0.0, 0.0};
    if (tri >= 0) {
        const int s = tri % k.L2;
        int m[3], ca[3], cb[3];
        subtri_corners_ab(k.L, s, m, ca, cb);
        const VertRec *vv = st.verts + (int64_t)v * k.VL * k.P;
        double vx[3], vy[3], viz[3], lu[3], lv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const VertRec r = vv[(int64_t)m[c] * k.P + p];
            vx[c] = r.x; vy[c] = r.y; viz[c] = r.iz;
            lu[c] = (double)ca[c] / k.L;
            lv[c] = (double)cb[c] / k.L;
        }
        const double qx = x + 0.5, qy = y + 0.5;
        const double d = (vx[1] - vx[0]) * (vy[2] - vy[0]) - (vy[1] - vy[0]) * (vx[2] - vx[0]);
        // screen-space barycentrics (edge functions / area), then weights lambda_k / z_k
        double beta[3];
        if (d != 0.0) {
            beta[0] = ((vx[2] - vx[1]) * (qy - vy[1]) - (vy[2] - vy[1]) * (qx - vx[1])) * viz[0];
            beta[1] = ((vx[0] - vx[2]) * (qy - vy[2]) - (vy[0] - vy[2]) * (qx - vx[2])) * viz[1];
            beta[2] = ((vx[1] - vx[0]) * (qy - vy[0]) - (vy[1] - vy[0]) * (qx - vx[0])) * viz[2];
        } else {
            beta[0] = viz[0]; beta[1] = viz[1]; beta[2] = viz[2];
        }
        // the common factor 1/area cancels in the normalisation
        const double iws = 1.0 / (beta[0] + beta[1] + beta[2]);
        double u = 0.0, vb = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) { u += beta[c] * iws * lu[c]; vb += beta[c] * iws * lv[c]; }
        uvo = make_float2((float)u, (float)vb);
        bernstein<DEG>(u, vb, 1.0 - u - vb, B);
        if constexpr (EXT) theta_weights<double>(k.T > 1 ? 3 : 1, u, vb, ti, tw);
    }
    // camera centre -R^T t (for the SH view direction)
    double Cc[3] = {0.0, 0.0, 0.0};
    if constexpr (EXT) {
        if (k.K > 0) {
            const float *cm = cams + 16 * v;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                Cc[c] = -((double)cm[c] * cm[9] + (double)cm[3 + c] * cm[10] + (double)cm[6 + c] * cm[11]);
        }
    }
    double qi[4] = {0.0, 0.0, 0.0, 0.0}, lsi[3] = {0.0, 0.0, 0.0};  // interpolated raw quaternion, log-scales
    // Eq. 3 (position) and Eq. 4 (diffuse colour) with the patch records read
    // through the scalar unit: an 8x8 block sees a few patches, the wave walks
    // its distinct ids (wave-uniform), the lanes of each id sum their points
    // against its record and keep its rotation-scale setup and opacity
    double S[3] = {0.0, 0.0, 0.0}, col[3] = {0.0, 0.0, 0.0};
    float Rm[21];
#pragma unroll
    for (int i = 0; i < 21; ++i) Rm[i] = 0.f;
    for (unsigned long long todo = __ballot(p >= 0); todo;) {
        const int pu = __builtin_amdgcn_readlane(p, __ffsll((long long)todo) - 1);
        const bool mine = p == pu;
        todo &= ~__ballot(mine);
        const float *src = patch + (int64_t)pu * PD;
        if (mine) {
#pragma unroll
            for (int c = 0; c < NCP; ++c)
#pragma unroll
                for (int dd = 0; dd < 3; ++dd) {
                    S[dd] += B[c] * (double)src[3 * c + dd];
                    col[dd] += B[c] * (double)src[3 * NCP + 3 * c + dd];
                }
#pragma unroll
            for (int i = 0; i < 20; ++i) Rm[i] = src[MO + i];
            Rm[20] = src[6 * NCP];
            if constexpr (EXT) {
                // this pixel's texels of the rotation and scale maps
                const float *tx = src + patch_x_off(NCP);
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    const float *tt = tx + 7 * ti[e];
#pragma unroll
                    for (int dd = 0; dd < 4; ++dd) qi[dd] += tw[e] * (double)tt[dd];
#pragma unroll
                    for (int dd = 0; dd < 3; ++dd) lsi[dd] += tw[e] * (double)tt[4 + dd];
                }
                if (k.K > 0) {
                    // view-dependent colour: sum_j Y_j(d) sh_j, d from the camera centre to S_q
                    double dv[3] = {S[0] - Cc[0], S[1] - Cc[1], S[2] - Cc[2]};
                    const double il = 1.0 / sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
                    const float *shc = src + patch_sh_off(NCP, k.T);
                    sh_basis_cb<double>(sh_degree_of(k.K), dv[0] * il, dv[1] * il, dv[2] * il,
                                        [&](int j, double Yj, double, double, double) {
#pragma unroll
                        for (int dd = 0; dd < 3; ++dd) col[dd] += Yj * (double)shc[3 * j + dd];
                    });
                }
            }
        }
    }
    if (act) {
        st.I_tri[pix] = tri;
        uint8_t flags = 0;
        if (tri >= 0) {
            double Mv[10];
#pragma unroll
            for (int i = 0; i < 10; ++i) Mv[i] = __hiloint2double(__float_as_int(Rm[2 * i + 1]), __float_as_int(Rm[2 * i]));
            // Eq. 5 from the interpolated maps (M per pixel), else the patch's M
            if constexpr (EXT) rot_scale(qi, lsi, Mv);
            const float opa = Rm[20];
            const Cam c = load_cam(cams, v);
            double t[3];
            cam_apply(c, S, t);
            Ewa e;
            if (ewa_project(k, c, t, Mv, e)) {
                const double tz = e.tz, J00 = e.J00, J02 = e.J02, J11 = e.J11, J12 = e.J12;
                const double SA = e.SA, SB = e.SB, SC = e.SC, mux = e.mux, muy = e.muy;
                const double idet = 1.0 / (SA * SC - SB * SB);
                int gi0, gi1, gj0, gj1;
                centre_range(mux, k.kappa * sqrt(SA), vi.W, gi0, gi1);
                centre_range(muy, k.kappa * sqrt(SC), vi.H, gj0, gj1);
                float sigma = 0.f;
                int bi0 = 1, bi1 = 0, bj0 = 1, bj1 = 0;
                if (bnd) {
                    // isotropic boundary Gaussian of scale r_b: r_b^2 J J^T + low-pass
                    const double r2 = Mv[9];
                    const double ma = r2 * (J00 * J00 + J02 * J02) + k.dilation;
                    const double mb = r2 * (J02 * J12);
                    const double mc = r2 * (J11 * J11 + J12 * J12) + k.dilation;
                    const double lam_max = 0.5 * (ma + mc) + sqrt(0.25 * (ma - mc) * (ma - mc) + mb * mb);
                    const double sg = 3.0 * sqrt(lam_max);
                    sigma = (float)sg;
                    // the FP64 point, for the exact arg-min of the backward
                    double *b64 = st.brec64 + (int64_t)pix * 3;
                    b64[0] = mux - (x + 0.5);
                    b64[1] = muy - (y + 0.5);
                    b64[2] = sg;
                    // the point's gradient accumulator starts at zero (the
                    // parameter pass clears it again after reading it)
                    float *db = st.dbound + (int64_t)pix * 3;
                    db[0] = 0.f; db[1] = 0.f; db[2] = 0.f;
                    centre_range(mux, sg, vi.W, bi0, bi1);
                    centre_range(muy, sg, vi.H, bj0, bj1);
                    flags |= PF_BOUNDARY;
                }
                flags |= PF_VALID;
                float4 *rec = st.rec + (int64_t)pix * 4;
                rec[0] = make_float4((float)(mux - (x + 0.5)), (float)(muy - (y + 0.5)), (float)(SC * idet),
                                     (float)(-SB * idet));
                rec[1] = make_float4((float)(SA * idet), (float)col[0], (float)col[1], (float)col[2]);
                rec[2] = make_float4(opa, __int_as_float(p), sigma, __int_as_float(pack16(x, y)));
                rec[3] = make_float4(__int_as_float(pack16(gi0, gi1)), __int_as_float(pack16(gj0, gj1)),
                                     __int_as_float(pack16(bi0, bi1)), __int_as_float(pack16(bj0, bj1)));
                st.gkey[pix] = ((unsigned long long)__double_as_longlong(tz)) >> 24;
                // tiles reached by the Gaussian's support and by the boundary disc
                const int TSH = __builtin_ctz(k.tile);  // tile side 8, 16 or 32: pixel ranges (>= 0) shift to tiles
                // (in the lattice variant the pixel records are boundary points only)
                if (gi0 <= gi1 && gj0 <= gj1 && k.NL == 0) {
                    gt0 = gi0 >> TSH; gt1 = gi1 >> TSH; gu0 = gj0 >> TSH; gu1 = gj1 >> TSH;
                    // a wide record's sums start at zero (the parameter pass
                    // clears them again after reading them)
                    if (!narrow_range(pack16(gi0, gi1), pack16(gj0, gj1), TSH)) zero_sums(st.gwide + (int64_t)pix * kSums);
                }
                if (bi0 <= bi1 && bj0 <= bj1) { bt0 = bi0 >> TSH; bt1 = bi1 >> TSH; bu0 = bj0 >> TSH; bu1 = bj1 >> TSH; }
            }
            fg = true;
            isb = (flags & PF_BOUNDARY) != 0;
        }
        st.I_uv[pix] = uvo;
        st.pflags[pix] = flags;
    }
    // pair counts per tile, one atomic per group of lanes at the same tile
    for_tiles_grouped(gt0, gt1, gu0, gu1, vi.tiles_x, vi.tile_off, [&](int t, unsigned long long gm, bool, int leader) {
        if (lane == leader) atomicAdd(&st.g_count[t], __popcll(gm));
    });
    for_tiles_grouped(bt0, bt1, bu0, bu1, vi.tiles_x, vi.tile_off, [&](int t, unsigned long long gm, bool, int leader) {
        if (lane == leader) atomicAdd(&st.b_count[t], __popcll(gm));
    });
    const unsigned long long mf = __ballot(fg), mb = __ballot(isb);
    if (lane == 0) {
        unsigned long long *slot = (unsigned long long *)&st.counters[C_NUM + (blk % kStripes) * kStripeStride];
        if (mf) atomicAdd(&slot[0], (unsigned long long)__popcll(mf));
        if (mb) atomicAdd(&slot[1], (unsigned long long)__popcll(mb));
    }
}

// Lattice variant: the Gaussian of view v, patch p at node (a, b) of the
// level-M lattice of the patch's domain, (u, v) = (a, b) / M, M = L (m - 1);
// one lane per record, consecutive lanes walk one patch's nodes.  Eq. 3-5,
// the SH colour and the EWA projection as for a pixel's Gaussian; the mean
// is stored relative to the pixel (floor(mu_x), floor(mu_y)), kept in r2.w.
template <int DEG, bool EXT>
__global__ void __launch_bounds__(256) k_gen_lattice(Consts k, ViewTable vt, const float *cams, StatePtrs st,
                                                     const float *__restrict__ patch) {
    constexpr int NCP = (DEG + 1) * (DEG + 2) / 2;
    constexpr int MO = patch_m_off(NCP);
    const int lane = threadIdx.x & 63;
    const int64_t per_view = (int64_t)k.P * k.NL;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool act = i < (int64_t)vt.n * per_view;
    int v = 0, p = 0, node = 0;
    if (act) {
        v = (int)(i / per_view);
        const int64_t r = i - v * per_view;
        p = (int)(r / k.NL);
        node = (int)(r - (int64_t)p * k.NL);
    }
    const ViewInfo vi = vt.v[v];
    int gt0 = 1, gt1 = 0, gu0 = 1, gu1 = 0;
    if (act) {
        int a, b;
        lattice_node(k.lat_level, node, a, b);
        const double u = (double)a / k.lat_level, vb = (double)b / k.lat_level;
        double B[NCP];
        bernstein<DEG>(u, vb, 1.0 - u - vb, B);
        const float *src = patch + (int64_t)p * k.pdw;
        const Cam c = load_cam(cams, v);
        // S (Eq. 1 summed in control-point order) and its camera coordinates
        // with each product rounded before its sum (no FMA contraction).  The
        // depth key decides the list order; a node that two patches share
        // (on their common edge) has equal depths in exact arithmetic, and
        // with an axis-aligned camera such depths often fall exactly on a key
        // boundary, where a one-ulp difference in rounding swaps the two
        // copies.  Evaluated as plain IEEE sums and products in this order,
        // the depth is reproducible by any evaluation in the same order.
        double S[3] = {0.0, 0.0, 0.0}, col[3] = {0.0, 0.0, 0.0}, t[3];
        {
#pragma clang fp contract(off)
#pragma unroll
            for (int cc = 0; cc < NCP; ++cc)
#pragma unroll
                for (int d = 0; d < 3; ++d) S[d] += B[cc] * (double)src[3 * cc + d];
#pragma unroll
            for (int r = 0; r < 3; ++r) t[r] = c.R[3 * r] * S[0] + c.R[3 * r + 1] * S[1] + c.R[3 * r + 2] * S[2] + c.t[r];
        }
#pragma unroll
        for (int cc = 0; cc < NCP; ++cc)
#pragma unroll
            for (int d = 0; d < 3; ++d) col[d] += B[cc] * (double)src[3 * NCP + 3 * cc + d];
        double Mv[10];
        const double *md = (const double *)(src + MO);  // 8-byte aligned: pdw is a multiple of 16
#pragma unroll
        for (int j = 0; j < 9; ++j) Mv[j] = md[j];
        if constexpr (EXT) {
            int ti[3];
            double tw[3], qi[4] = {0.0, 0.0, 0.0, 0.0}, lsi[3] = {0.0, 0.0, 0.0};
            theta_weights<double>(k.T > 1 ? 3 : 1, u, vb, ti, tw);
            const float *tx = src + patch_x_off(NCP);
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                const float *tt = tx + 7 * ti[e];
#pragma unroll
                for (int d = 0; d < 4; ++d) qi[d] += tw[e] * (double)tt[d];
#pragma unroll
                for (int d = 0; d < 3; ++d) lsi[d] += tw[e] * (double)tt[4 + d];
            }
            rot_scale(qi, lsi, Mv);
            if (k.K > 0) {
                const float *cm = cams + 16 * v;
                double dv[3];
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    dv[c] = S[c] + ((double)cm[c] * cm[9] + (double)cm[3 + c] * cm[10] + (double)cm[6 + c] * cm[11]);
                const double il = 1.0 / sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
                const float *shc = src + patch_sh_off(NCP, k.T);
                sh_basis_cb<double>(sh_degree_of(k.K), dv[0] * il, dv[1] * il, dv[2] * il,
                                    [&](int j, double Yj, double, double, double) {
#pragma unroll
                    for (int d = 0; d < 3; ++d) col[d] += Yj * (double)shc[3 * j + d];
                });
            }
        }
        Ewa e;
        float4 *rec = st.rec + ((int64_t)vt.total_px + i) * 4;
        if (ewa_project(k, c, t, Mv, e)) {
            const double idet = 1.0 / (e.SA * e.SC - e.SB * e.SB);
            int gi0, gi1, gj0, gj1;
            centre_range(e.mux, k.kappa * sqrt(e.SA), vi.W, gi0, gi1);
            centre_range(e.muy, k.kappa * sqrt(e.SC), vi.H, gj0, gj1);
            const double fx = floor(e.mux), fy = floor(e.muy);
            const int ax = (int)fmin(fmax(fx, -30000.0), 30000.0), ay = (int)fmin(fmax(fy, -30000.0), 30000.0);
            rec[0] = make_float4((float)(e.mux - (ax + 0.5)), (float)(e.muy - (ay + 0.5)), (float)(e.SC * idet),
                                 (float)(-e.SB * idet));
            rec[1] = make_float4((float)(e.SA * idet), (float)col[0], (float)col[1], (float)col[2]);
            rec[2] = make_float4(src[6 * NCP], __int_as_float(p), 0.f, __int_as_float(pack16(ax, ay)));
            rec[3] = make_float4(__int_as_float(pack16(gi0, gi1)), __int_as_float(pack16(gj0, gj1)),
                                 __int_as_float(pack16(1, 0)), __int_as_float(pack16(1, 0)));
            st.gkey[vt.total_px + i] = ((unsigned long long)__double_as_longlong(e.tz)) >> 24;
            const int TSH = __builtin_ctz(k.tile);  // tile side 8, 16 or 32: pixel ranges (>= 0) shift to tiles
            if (gi0 <= gi1 && gj0 <= gj1) {
                gt0 = gi0 >> TSH; gt1 = gi1 >> TSH; gu0 = gj0 >> TSH; gu1 = gj1 >> TSH;
                if (!narrow_range(pack16(gi0, gi1), pack16(gj0, gj1), TSH))
                    zero_sums(st.gwide + ((int64_t)vt.total_px + i) * kSums);
            }
        } else {
            // behind z_near: empty ranges, never listed
            rec[0] = make_float4(0.f, 0.f, 0.f, 0.f);
            rec[1] = make_float4(0.f, 0.f, 0.f, 0.f);
            rec[2] = make_float4(0.f, __int_as_float(p), 0.f, 0.f);
            rec[3] = make_float4(__int_as_float(pack16(1, 0)), __int_as_float(pack16(1, 0)), __int_as_float(pack16(1, 0)),
                                 __int_as_float(pack16(1, 0)));
            st.gkey[vt.total_px + i] = 0ull;
        }
    }
    for_tiles_grouped(gt0, gt1, gu0, gu1, vi.tiles_x, vi.tile_off, [&](int t, unsigned long long gm, bool, int leader) {
        if (lane == leader) atomicAdd(&st.g_count[t], __popcll(gm));
    });
}

hipError_t launch_raster(const Consts &k, const ViewTable &vt, const PrimPtrs &pr, const float *cams,
                         const StatePtrs &st, hipStream_t s) {
    hipError_t e;
    if ((e = launch_tessellate(k, pr, st.wverts, nullptr, s)) != hipSuccess) return e;
    {
        const int64_t n = (int64_t)vt.n * k.VL * k.P;
        hipLaunchKernelGGL(k_project, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, k, vt, cams,
                           (const double *)st.wverts, st.verts);
    }
    {
        const int64_t n = (int64_t)vt.n * k.L2 * k.P;
        hipLaunchKernelGGL(k_raster, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, k, vt,
                           (const VertRec *)st.verts, st.zbuf, st.big_tris, st.counters);
        hipLaunchKernelGGL(k_raster_big, dim3(1024), dim3(256), 0, s, k, vt, (const VertRec *)st.verts, st.zbuf,
                           (const int32_t *)st.big_tris, (const int64_t *)st.counters);
    }
    return hipGetLastError();
}

hipError_t launch_gen(const Consts &k, const ViewTable &vt, const PrimPtrs &pr, const float *cams,
                      const StatePtrs &st, hipStream_t s) {
    hipLaunchKernelGGL(k_prim_setup, dim3((unsigned)(((int64_t)k.P * k.pdw + 255) / 256)), dim3(256), 0, s, k, pr,
                       st.patch);
    const bool ext = k.T > 1 || k.K > 0;  // resolution-3 maps or SH colour
    {
        dim3 grid((unsigned)((vt.total_b8 + 3) / 4)), block(256);  // one wave per 8x8 block
        switch (k.degree) {
            case 1:
                if (ext) hipLaunchKernelGGL((k_gen<1, true>), grid, block, 0, s, k, vt, pr, cams, st, st.patch);
                else hipLaunchKernelGGL((k_gen<1, false>), grid, block, 0, s, k, vt, pr, cams, st, st.patch);
                break;
            case 2:
                if (ext) hipLaunchKernelGGL((k_gen<2, true>), grid, block, 0, s, k, vt, pr, cams, st, st.patch);
                else hipLaunchKernelGGL((k_gen<2, false>), grid, block, 0, s, k, vt, pr, cams, st, st.patch);
                break;
            case 3:
                if (ext) hipLaunchKernelGGL((k_gen<3, true>), grid, block, 0, s, k, vt, pr, cams, st, st.patch);
                else hipLaunchKernelGGL((k_gen<3, false>), grid, block, 0, s, k, vt, pr, cams, st, st.patch);
                break;
            case 4:
                if (ext) hipLaunchKernelGGL((k_gen<4, true>), grid, block, 0, s, k, vt, pr, cams, st, st.patch);
                else hipLaunchKernelGGL((k_gen<4, false>), grid, block, 0, s, k, vt, pr, cams, st, st.patch);
                break;
            case 5:
                if (ext) hipLaunchKernelGGL((k_gen<5, true>), grid, block, 0, s, k, vt, pr, cams, st, st.patch);
                else hipLaunchKernelGGL((k_gen<5, false>), grid, block, 0, s, k, vt, pr, cams, st, st.patch);
                break;
            default: return hipErrorInvalidValue;
        }
    }
    if (k.NL > 0) {
        const int64_t n = (int64_t)vt.n * k.P * k.NL;
        dim3 grid((unsigned)((n + 255) / 256)), block(256);
        switch (k.degree) {
#define BGT_LAT(D)                                                                                               \
    case D:                                                                                                      \
        if (ext) hipLaunchKernelGGL((k_gen_lattice<D, true>), grid, block, 0, s, k, vt, cams, st, st.patch);    \
        else hipLaunchKernelGGL((k_gen_lattice<D, false>), grid, block, 0, s, k, vt, cams, st, st.patch);       \
        break;
            BGT_LAT(1) BGT_LAT(2) BGT_LAT(3) BGT_LAT(4) BGT_LAT(5)
#undef BGT_LAT
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

}  // namespace bgt
