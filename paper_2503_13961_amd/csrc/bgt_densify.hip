// Splitting and pruning (Sec. 3.3 and the implementation details): per-patch
// statistics gathered from the index map of rendered views, the per-patch
// decision, and the rebuilt parameter arrays in which a split patch is
// replaced by its four midpoint children.
//
// Pixel statistics run one thread per pixel; a wave groups its lanes by
// (patch, view) and adds each group's totals with one atomic per array, so a
// patch covering a few hundred pixels costs a few atomics per wave rather
// than one per pixel.  The children's control nets are blossoms of the
// parent's net at the corners of their sub-domains, taken by de Casteljau
// steps in FP64.
#include "bgt_internal.h"

namespace bgt {

namespace {

constexpr int kThreads = 256;

// linear index of p_ijk in Eq. 1's summation order (i outer, j inner)
__host__ __device__ constexpr int cidx(int n, int i, int j) { return i * (n + 1) - i * (i - 1) / 2 + j; }

__device__ __forceinline__ float grey255(const float *img, int64_t pix) {
    return (img[3 * pix] + img[3 * pix + 1] + img[3 * pix + 2]) * (255.0f / 3.0f);
}

}  // namespace

// Visibility (views, sub-triangle texels) and the edge prior, per pixel.
__global__ void __launch_bounds__(kThreads) k_stats_pixels(ViewTable vt, int L2, const int32_t *I_tri,
                                                           const float *targets, StatsPtrs sp) {
    const int64_t pix = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int key = -1, g = 0, s = 0, v = 0;
    float e = 0.f;
    if (pix < vt.total_px) {
        const int tri = I_tri[pix];
        if (tri >= 0) {
            v = view_of_pixel(vt, (int)pix);
            g = tri / L2;
            s = tri - g * L2;
            key = g * BGT_MAX_VIEWS + v;
            if (targets) {
                // Sobel magnitude of the grey level; 0 on the view's border
                const ViewInfo &vi = vt.v[v];
                const int lp = (int)(pix - vi.px_off), x = lp % vi.W, y = lp / vi.W;
                if (x > 0 && y > 0 && x + 1 < vi.W && y + 1 < vi.H) {
                    const int64_t c = pix;
                    const int64_t W = vi.W;
                    const float a = grey255(targets, c - W - 1), b = grey255(targets, c - W),
                                cc = grey255(targets, c - W + 1), d = grey255(targets, c - 1),
                                f = grey255(targets, c + 1), gg = grey255(targets, c + W - 1),
                                h = grey255(targets, c + W), i = grey255(targets, c + W + 1);
                    const float gx = (cc + 2.f * f + i) - (a + 2.f * d + gg);
                    const float gy = (gg + 2.f * h + i) - (a + 2.f * b + cc);
                    e = sqrtf(gx * gx + gy * gy);
                }
            }
        }
    }
    // one group of lanes per distinct (patch, view)
    bool pending = key >= 0;
    while (__any(pending)) {
        const int first = __ffsll((long long)__ballot(pending)) - 1;
        const int k0 = __shfl(key, first, 64);
        const bool mine = pending && key == k0;
        unsigned long long bits = mine ? (1ull << s) : 0ull;
        float es = mine ? e : 0.f;
        int cnt = mine ? 1 : 0;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            bits |= __shfl_xor(bits, o, 64);
            es += __shfl_xor(es, o, 64);
            cnt += __shfl_xor(cnt, o, 64);
        }
        if (lane == first) {
            atomicOr(&sp.tex[g], bits);
            atomicOr(&sp.view_bits[g], 1ull << v);
            if (targets) {
                atomicAdd(&sp.edge_sum[g], es);
                atomicAdd(&sp.edge_cnt[g], cnt);
            }
        }
        pending = pending && !mine;
    }
}

// Per patch: fold this call's view bits into the visibility count, and the
// mean |dL/dp| over the control points into the gradient accumulator for
// the patches that were visible.
__global__ void __launch_bounds__(kThreads) k_stats_prims(int P, int ncp, int n_views, const float *d_ctrl,
                                                          StatsPtrs sp) {
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p == 0) sp.views_seen[0] += n_views;
    if (p >= P) return;
    const unsigned long long vb = sp.view_bits[p];
    sp.view_bits[p] = 0ull;
    const int nv = __popcll(vb);
    sp.vis_views[p] += nv;
    if (d_ctrl && nv > 0) {
        double acc = 0.0;
        for (int m = 0; m < ncp; ++m) {
            const double x = d_ctrl[(0 * (int64_t)ncp + m) * P + p], y = d_ctrl[(1 * (int64_t)ncp + m) * P + p],
                         z = d_ctrl[(2 * (int64_t)ncp + m) * P + p];
            acc += sqrt(x * x + y * y + z * z);
        }
        sp.grad_sum[p] += (float)(acc / ncp);
        sp.grad_cnt[p] += 1;
    }
}

template <int DEG>
__device__ void surface_at(const float *ctrl, int P, int p, double u, double v, double w, double *out) {
    constexpr int NCP = (DEG + 1) * (DEG + 2) / 2;
    // de Casteljau down to one point (no factorials)
    double net[NCP][3];
    for (int m = 0; m < NCP; ++m)
        for (int d = 0; d < 3; ++d) net[m][d] = ctrl[((int64_t)d * NCP + m) * P + p];
    for (int deg = DEG; deg > 0; --deg)
        for (int i = 0; i < deg; ++i)
            for (int j = 0; j < deg - i; ++j)
                for (int d = 0; d < 3; ++d)
                    net[cidx(deg - 1, i, j)][d] = u * net[cidx(deg, i + 1, j)][d] + v * net[cidx(deg, i, j + 1)][d] +
                                                  w * net[cidx(deg, i, j)][d];
    for (int d = 0; d < 3; ++d) out[d] = net[0][d];
}

__device__ double tri_area(const double *a, const double *b, const double *c) {
    const double e0[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e1[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    const double x = e0[1] * e1[2] - e0[2] * e1[1], y = e0[2] * e1[0] - e0[0] * e1[2], z = e0[0] * e1[1] - e0[1] * e1[0];
    return 0.5 * sqrt(x * x + y * y + z * z);
}

// Decision per patch; dst_index receives the number of output slots (1 keep,
// 4 split, 0 prune), turned into offsets by k_scan_slots.
template <int DEG>
__global__ void __launch_bounds__(kThreads) k_plan(int P, int L2, const float *ctrl, StatsPtrs sp, DensifyRule rule,
                                                   int32_t *action, int32_t *dst_index) {
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= P) return;
    double S[6][3];
    surface_at<DEG>(ctrl, P, p, 1, 0, 0, S[0]);
    surface_at<DEG>(ctrl, P, p, 0, 1, 0, S[1]);
    surface_at<DEG>(ctrl, P, p, 0, 0, 1, S[2]);
    surface_at<DEG>(ctrl, P, p, 0.5, 0.5, 0, S[3]);
    surface_at<DEG>(ctrl, P, p, 0, 0.5, 0.5, S[4]);
    surface_at<DEG>(ctrl, P, p, 0.5, 0, 0.5, S[5]);
    const double area = tri_area(S[0], S[3], S[5]) + tri_area(S[3], S[1], S[4]) + tri_area(S[5], S[4], S[2]) +
                        tri_area(S[4], S[5], S[3]);
    // aspect of the corner triangle: longest edge over its height on it
    double len2 = 0.0;
    for (int e = 0; e < 3; ++e) {
        const double *a = S[e], *b = S[(e + 1) % 3];
        const double d2 = (b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) + (b[2] - a[2]) * (b[2] - a[2]);
        len2 = d2 > len2 ? d2 : len2;
    }
    const double twice = 2.0 * tri_area(S[0], S[1], S[2]);
    const bool thin = twice == 0.0 || len2 / twice > rule.tau_s;
    const int seen = sp.views_seen[0];
    const double vis_ratio = seen > 0 ? (double)sp.vis_views[p] / seen : 0.0;
    const double tex_ratio = (double)__popcll(sp.tex[p]) / L2;
    int act = 0, slots = 1;
    if (vis_ratio < rule.tau_v || tex_ratio < rule.tau_r || area < rule.tau_a || thin) {
        act = 2;
        slots = 0;
    } else {
        const double g = sp.grad_cnt[p] ? (double)sp.grad_sum[p] / sp.grad_cnt[p] : 0.0;
        const double eb = sp.edge_cnt[p] ? (double)sp.edge_sum[p] / sp.edge_cnt[p] : 0.0;
        if (g > rule.tau_g || eb > rule.tau_b) {
            act = 1;
            slots = 4;
        }
    }
    action[p] = act;
    dst_index[p] = slots;
}

// Exclusive scan of the slot counts in one workgroup (chunks of 1024 with a
// running carry); count[0] receives the total.
__global__ void __launch_bounds__(1024) k_scan_slots(int P, int32_t *slots, int32_t *count) {
    __shared__ int32_t wsum[16];
    __shared__ int32_t carry;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < P; base += 1024) {
        const int i = base + tid;
        const int x = i < P ? slots[i] : 0;
        int incl = x;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        int before = carry;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (i < P) slots[i] = before + incl - x;
        __syncthreads();
        if (tid == 1023) carry = before + incl;
        __syncthreads();
    }
    if (tid == 0) count[0] = carry;
}

// The rebuilt arrays: thread (p, c) writes the kept patch (c = 0) or child c
// of a split patch at dst_index[p] + c.
template <int DEG>
__global__ void __launch_bounds__(kThreads) k_apply(int P, int T, int K, PrimPtrs src, const int32_t *action,
                                                    const int32_t *dst_index, int Pd, GradPtrs dst) {
    constexpr int NCP = (DEG + 1) * (DEG + 2) / 2;
    const int64_t t = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (t >= 4 * (int64_t)P) return;
    const int p = (int)(t >> 2), c = (int)(t & 3);
    const int act = action[p];
    if (act == 2 || (act == 0 && c > 0)) return;
    const int slot = dst_index[p] + (act == 1 ? c : 0);
    if (slot < 0 || slot >= Pd) return;  // outputs sized below the planned count
    // attributes are the parent's
    for (int d = 0; d < 3; ++d)
        for (int k = 0; k < T; ++k)
            dst.log_scale[((int64_t)d * T + k) * Pd + slot] = src.log_scale[((int64_t)d * T + k) * P + p];
    for (int d = 0; d < 4; ++d)
        for (int k = 0; k < T; ++k) dst.quat[((int64_t)d * T + k) * Pd + slot] = src.quat[((int64_t)d * T + k) * P + p];
    dst.opacity[slot] = src.opacity[p];
    dst.sharp[slot] = src.sharp[p];
    for (int j = 0; j < 3 * K; ++j) dst.sh[(int64_t)j * Pd + slot] = src.sh[(int64_t)j * P + p];
    // domain corners of the child: corner u, corner v, corner w, middle (half turn)
    const double corners[4][3][3] = {{{1, 0, 0}, {0.5, 0.5, 0}, {0.5, 0, 0.5}},
                                     {{0.5, 0.5, 0}, {0, 1, 0}, {0, 0.5, 0.5}},
                                     {{0.5, 0, 0.5}, {0, 0.5, 0.5}, {0, 0, 1}},
                                     {{0, 0.5, 0.5}, {0.5, 0, 0.5}, {0.5, 0.5, 0}}};
    for (int which = 0; which < 2; ++which) {
        const float *in = which == 0 ? src.ctrl : src.color;
        float *out = which == 0 ? dst.ctrl : dst.color;
        double net0[NCP][3];
        for (int m = 0; m < NCP; ++m)
            for (int d = 0; d < 3; ++d) net0[m][d] = in[((int64_t)d * NCP + m) * P + p];
        for (int i = 0; i <= DEG; ++i)
            for (int j = 0; j <= DEG - i; ++j) {
                double q[3];
                if (act == 0) {
                    for (int d = 0; d < 3; ++d) q[d] = net0[cidx(DEG, i, j)][d];
                } else {
                    // blossom at (A^i, B^j, C^k): one de Casteljau step per argument
                    double net[NCP][3];
                    for (int m = 0; m < NCP; ++m)
                        for (int d = 0; d < 3; ++d) net[m][d] = net0[m][d];
                    int step = 0;
                    for (int deg = DEG; deg > 0; --deg, ++step) {
                        const int arg = step < i ? 0 : (step < i + j ? 1 : 2);
                        const double a = corners[c][arg][0], b = corners[c][arg][1], w = corners[c][arg][2];
                        for (int ii = 0; ii < deg; ++ii)
                            for (int jj = 0; jj < deg - ii; ++jj)
                                for (int d = 0; d < 3; ++d)
                                    net[cidx(deg - 1, ii, jj)][d] = a * net[cidx(deg, ii + 1, jj)][d] +
                                                                    b * net[cidx(deg, ii, jj + 1)][d] +
                                                                    w * net[cidx(deg, ii, jj)][d];
                    }
                    for (int d = 0; d < 3; ++d) q[d] = net[0][d];
                }
                for (int d = 0; d < 3; ++d) out[((int64_t)d * NCP + cidx(DEG, i, j)) * Pd + slot] = (float)q[d];
            }
    }
}

hipError_t launch_stats(const Consts &k, const ViewTable &vt, const int32_t *I_tri, const float *targets,
                        const float *d_ctrl, const StatsPtrs &sp, hipStream_t s) {
    const int64_t blocks = ((int64_t)vt.total_px + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_stats_pixels, dim3((unsigned)blocks), dim3(kThreads), 0, s, vt, k.L2, I_tri, targets, sp);
    hipLaunchKernelGGL(k_stats_prims, dim3((k.P + kThreads - 1) / kThreads), dim3(kThreads), 0, s, k.P, k.ncp, vt.n,
                       d_ctrl, sp);
    return hipGetLastError();
}

template <int DEG>
static void plan_deg(const Consts &k, const float *ctrl, const StatsPtrs &sp, const DensifyRule &rule,
                     int32_t *action, int32_t *dst_index, hipStream_t s) {
    hipLaunchKernelGGL(k_plan<DEG>, dim3((k.P + kThreads - 1) / kThreads), dim3(kThreads), 0, s, k.P, k.L2, ctrl, sp,
                       rule, action, dst_index);
}

hipError_t launch_plan(const Consts &k, const float *ctrl, const StatsPtrs &sp, const DensifyRule &rule,
                       int32_t *action, int32_t *dst_index, int32_t *count, hipStream_t s) {
    switch (k.degree) {
        case 1: plan_deg<1>(k, ctrl, sp, rule, action, dst_index, s); break;
        case 2: plan_deg<2>(k, ctrl, sp, rule, action, dst_index, s); break;
        case 3: plan_deg<3>(k, ctrl, sp, rule, action, dst_index, s); break;
        case 4: plan_deg<4>(k, ctrl, sp, rule, action, dst_index, s); break;
        default: plan_deg<5>(k, ctrl, sp, rule, action, dst_index, s); break;
    }
    hipLaunchKernelGGL(k_scan_slots, dim3(1), dim3(1024), 0, s, k.P, dst_index, count);
    return hipGetLastError();
}

template <int DEG>
static void apply_deg(const Consts &k, const PrimPtrs &src, const int32_t *action, const int32_t *dst_index, int Pd,
                      const GradPtrs &dst, hipStream_t s) {
    const int64_t n = 4 * (int64_t)k.P;
    hipLaunchKernelGGL(k_apply<DEG>, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, k.P, k.T,
                       k.K, src, action, dst_index, Pd, dst);
}

hipError_t launch_apply(const Consts &k, const PrimPtrs &src, const int32_t *action, const int32_t *dst_index,
                        int Pd, const GradPtrs &dst, hipStream_t s) {
    switch (k.degree) {
        case 1: apply_deg<1>(k, src, action, dst_index, Pd, dst, s); break;
        case 2: apply_deg<2>(k, src, action, dst_index, Pd, dst, s); break;
        case 3: apply_deg<3>(k, src, action, dst_index, Pd, dst, s); break;
        case 4: apply_deg<4>(k, src, action, dst_index, Pd, dst, s); break;
        default: apply_deg<5>(k, src, action, dst_index, Pd, dst, s); break;
    }
    return hipGetLastError();
}

}  // namespace bgt
