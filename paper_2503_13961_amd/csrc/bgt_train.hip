// One training step around the renderer (Sec. 3.3): the photometric loss of
// Eq. 9, L = (1 - lambda) L2 + lambda (1 - SSIM), with its image gradient,
// and the Adam update of the parameters.
//
// SSIM takes five window moments per pixel and channel (mu_x, mu_y, E[x^2],
// E[y^2], E[xy]) under an 11x11 Gaussian window, zero outside the view.  A
// workgroup owns a 32x16 output tile of one view: it stages the tile plus a
// 5-pixel apron in LDS, sums the window rows (horizontal pass) into LDS and
// then the columns (vertical pass), in FP64 -- E[x^2] - mu_x^2 cancels, and
// FP64 vector arithmetic runs at the FP32 rate on this GPU.  The per-pixel
// SSIM and its derivatives with respect to the three moments that depend on
// the image go to three maps; the gradient pass runs the same window over
// the maps (the window is symmetric, so its transpose is itself).  Loss
// partial sums are per workgroup and reduced in a fixed order.
#include "bgt_internal.h"

namespace bgt {

namespace {

constexpr int kWin = 11, kApron = 5;
constexpr int kTW = 32, kTH = 16;                                   // output tile
constexpr int kIW = kTW + 2 * kApron, kIH = kTH + 2 * kApron;       // staged region 42 x 26
constexpr int kThreads = 256;

}  // namespace

__device__ __forceinline__ int loss_view_of_tile(const LossTable &lt, int t) {
    int lo = 0, hi = lt.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (lt.tile_off[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// sum of a double over the workgroup in a fixed order (result in thread 0)
__device__ double block_sum(double v, double *red) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    return s;
}

// Window moments, SSIM and its derivative maps; per-workgroup sums of the
// SSIM map and of the squared error.
__global__ void __launch_bounds__(kThreads) k_ssim_fwd(LossTable lt, const float *x, const float *y, float *map_a,
                                                       float *map_b, float *map_c, double *partial) {
    __shared__ float sx[kIH][kIW], sy[kIH][kIW];
    __shared__ double hs[5][kIH][kTW];
    __shared__ double red[kThreads / 64];
    const int t = blockIdx.x, tid = threadIdx.x;
    const int v = loss_view_of_tile(lt, t);
    const int W = lt.W[v], H = lt.H[v];
    const int tl = t - lt.tile_off[v], tx = tl % lt.tiles_x[v], ty = tl / lt.tiles_x[v];
    const int gx0 = tx * kTW - kApron, gy0 = ty * kTH - kApron;
    const int64_t base = lt.px_off[v];
    double s_ssim = 0.0, s_sq = 0.0;
    for (int c = 0; c < 3; ++c) {
        __syncthreads();  // the previous channel is done with the stage
        for (int i = tid; i < kIH * kIW; i += kThreads) {
            const int ry = i / kIW, rx = i % kIW, gx = gx0 + rx, gy = gy0 + ry;
            float a = 0.f, b = 0.f;
            if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
                const int64_t o = (base + (int64_t)gy * W + gx) * 3 + c;
                a = x[o];
                b = y[o];
            }
            sx[ry][rx] = a;
            sy[ry][rx] = b;
        }
        __syncthreads();
        for (int i = tid; i < kIH * kTW; i += kThreads) {
            const int ry = i / kTW, j = i % kTW;
            double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0;
#pragma unroll
            for (int k = 0; k < kWin; ++k) {
                const double a = sx[ry][j + k], b = sy[ry][j + k];
                const double wa = lt.taps[k] * a, wb = lt.taps[k] * b;
                m0 += wa;
                m1 += wb;
                m2 = fma(wa, a, m2);
                m3 = fma(wb, b, m3);
                m4 = fma(wa, b, m4);
            }
            hs[0][ry][j] = m0;
            hs[1][ry][j] = m1;
            hs[2][ry][j] = m2;
            hs[3][ry][j] = m3;
            hs[4][ry][j] = m4;
        }
        __syncthreads();
        for (int i = tid; i < kTH * kTW; i += kThreads) {
            const int oy = i / kTW, j = i % kTW;
            const int gx = tx * kTW + j, gy = ty * kTH + oy;
            if (gx >= W || gy >= H) continue;
            double mx = 0.0, my = 0.0, exx = 0.0, eyy = 0.0, exy = 0.0;
#pragma unroll
            for (int k = 0; k < kWin; ++k) {
                const double w = lt.taps[k];
                mx = fma(w, hs[0][oy + k][j], mx);
                my = fma(w, hs[1][oy + k][j], my);
                exx = fma(w, hs[2][oy + k][j], exx);
                eyy = fma(w, hs[3][oy + k][j], eyy);
                exy = fma(w, hs[4][oy + k][j], exy);
            }
            const double sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
            const double A1 = 2.0 * mx * my + kSsimC1, A2 = 2.0 * sxy + kSsimC2;
            const double B1 = mx * mx + my * my + kSsimC1, B2 = sxx + syy + kSsimC2;
            const double iA1 = 1.0 / A1, iA2 = 1.0 / A2, iB1 = 1.0 / B1, iB2 = 1.0 / B2;
            const double S = A1 * A2 * iB1 * iB2;
            // dS/dmu_x, dS/dE[x^2], dS/dE[xy] with sigma_x^2 = E[x^2] - mu_x^2, sigma_xy = E[xy] - mu_x mu_y
            const double da = 2.0 * S * (my * (iA1 - iA2) + mx * (iB2 - iB1));
            const int64_t o = (base + (int64_t)gy * W + gx) * 3 + c;
            map_a[o] = (float)da;
            map_b[o] = (float)(-S * iB2);
            map_c[o] = (float)(2.0 * S * iA2);
            const double d = (double)sx[oy + kApron][j + kApron] - (double)sy[oy + kApron][j + kApron];
            s_ssim += S;
            s_sq = fma(d, d, s_sq);
        }
    }
    const double a = block_sum(s_ssim, red);
    const double b = block_sum(s_sq, red);
    if (tid == 0) {
        partial[2 * (int64_t)t] = a;
        partial[2 * (int64_t)t + 1] = b;
    }
}

// dL/dC = (1 - lambda) 2 (x - y) / n - lambda / n * (W*a + 2 x W*b + y W*c)
__global__ void __launch_bounds__(kThreads) k_ssim_grad(LossTable lt, const float *x, const float *y,
                                                        const float *map_a, const float *map_b,
                                                        const float *map_c, float *grad) {
    __shared__ float sa[kIH][kIW], sb[kIH][kIW], sc[kIH][kIW];
    __shared__ double hs[3][kIH][kTW];
    const int t = blockIdx.x, tid = threadIdx.x;
    const int v = loss_view_of_tile(lt, t);
    const int W = lt.W[v], H = lt.H[v];
    const int tl = t - lt.tile_off[v], tx = tl % lt.tiles_x[v], ty = tl / lt.tiles_x[v];
    const int gx0 = tx * kTW - kApron, gy0 = ty * kTH - kApron;
    const int64_t base = lt.px_off[v];
    for (int c = 0; c < 3; ++c) {
        __syncthreads();
        for (int i = tid; i < kIH * kIW; i += kThreads) {
            const int ry = i / kIW, rx = i % kIW, gx = gx0 + rx, gy = gy0 + ry;
            float a = 0.f, b = 0.f, cc = 0.f;
            if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
                const int64_t o = (base + (int64_t)gy * W + gx) * 3 + c;
                a = map_a[o];
                b = map_b[o];
                cc = map_c[o];
            }
            sa[ry][rx] = a;
            sb[ry][rx] = b;
            sc[ry][rx] = cc;
        }
        __syncthreads();
        for (int i = tid; i < kIH * kTW; i += kThreads) {
            const int ry = i / kTW, j = i % kTW;
            double m0 = 0.0, m1 = 0.0, m2 = 0.0;
#pragma unroll
            for (int k = 0; k < kWin; ++k) {
                m0 = fma(lt.taps[k], (double)sa[ry][j + k], m0);
                m1 = fma(lt.taps[k], (double)sb[ry][j + k], m1);
                m2 = fma(lt.taps[k], (double)sc[ry][j + k], m2);
            }
            hs[0][ry][j] = m0;
            hs[1][ry][j] = m1;
            hs[2][ry][j] = m2;
        }
        __syncthreads();
        for (int i = tid; i < kTH * kTW; i += kThreads) {
            const int oy = i / kTW, j = i % kTW;
            const int gx = tx * kTW + j, gy = ty * kTH + oy;
            if (gx >= W || gy >= H) continue;
            double A = 0.0, B = 0.0, C = 0.0;
#pragma unroll
            for (int k = 0; k < kWin; ++k) {
                const double w = lt.taps[k];
                A = fma(w, hs[0][oy + k][j], A);
                B = fma(w, hs[1][oy + k][j], B);
                C = fma(w, hs[2][oy + k][j], C);
            }
            const int64_t o = (base + (int64_t)gy * W + gx) * 3 + c;
            const double xv = x[o], yv = y[o];
            grad[o] = (float)((1.0 - lt.lam) * 2.0 * (xv - yv) * lt.inv_n - lt.lam * lt.inv_n * (A + 2.0 * xv * B + yv * C));
        }
    }
}

// loss[0] = L, loss[1] = L2, loss[2] = SSIM, from the per-workgroup sums
__global__ void __launch_bounds__(kThreads) k_loss_final(const double *partial, int nblocks, double inv_n, double lam,
                                                         float *loss) {
    __shared__ double red[kThreads / 64];
    double s = 0.0, q = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += kThreads) {
        s += partial[2 * (int64_t)i];
        q += partial[2 * (int64_t)i + 1];
    }
    const double S = block_sum(s, red);
    const double Q = block_sum(q, red);
    if (threadIdx.x == 0) {
        const double l2 = Q * inv_n, ssim = S * inv_n;
        loss[0] = (float)((1.0 - lam) * l2 + lam * (1.0 - ssim));
        loss[1] = (float)l2;
        loss[2] = (float)ssim;
    }
}

hipError_t launch_loss(const LossTable &lt, const float *x, const float *y, float *loss, float *grad, float *maps,
                       double *partial, hipStream_t s) {
    const int64_t n = 3 * (int64_t)lt.total_px;
    float *ma = maps, *mb = maps + n, *mc = maps + 2 * n;
    hipLaunchKernelGGL(k_ssim_fwd, dim3(lt.total_tiles), dim3(kThreads), 0, s, lt, x, y, ma, mb, mc, partial);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(kThreads), 0, s, (const double *)partial, lt.total_tiles,
                       lt.inv_n, lt.lam, loss);
    if (grad)
        hipLaunchKernelGGL(k_ssim_grad, dim3(lt.total_tiles), dim3(kThreads), 0, s, lt, x, y, (const float *)ma,
                           (const float *)mb, (const float *)mc, grad);
    return hipGetLastError();
}

void loss_tiles(int W, int H, int *tiles_x, int *tiles) {
    *tiles_x = (W + kTW - 1) / kTW;
    *tiles = *tiles_x * ((H + kTH - 1) / kTH);
}

// ------------------------------------------------------------------- L1

__global__ void __launch_bounds__(kThreads) k_l1_cotangent(int64_t n, const float *x, const float *y, float scale,
                                                           float *g) {
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const float d = x[i] - y[i];
        g[i] = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
    }
}

hipError_t launch_l1(int64_t n, const float *x, const float *y, float scale, float *g, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + kThreads - 1) / kThreads;
    blocks = blocks > 8192 ? 8192 : blocks;
    hipLaunchKernelGGL(k_l1_cotangent, dim3((unsigned)blocks), dim3(kThreads), 0, s, n, x, y, scale, g);
    return hipGetLastError();
}

// ------------------------------------------------------------------- Adam

// One Adam update (Kingma and Ba, Algorithm 1) over every group, at step
// *step + 1; FP64 arithmetic, moments stored as float.
__global__ void __launch_bounds__(kThreads) k_adam(AdamTable at, double b1, double b2, double eps,
                                                   const int32_t *step) {
    const int64_t total = at.off[at.n];
    const int t1 = step[0] + 1;
    const double bc1 = 1.0 - pow(b1, (double)t1), bc2 = 1.0 - pow(b2, (double)t1);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int g = 0;
        while (i >= at.off[g + 1]) ++g;
        const int64_t j = i - at.off[g];
        const double gr = at.grad[g][j];
        const double m = b1 * (double)at.m[g][j] + (1.0 - b1) * gr;
        const double v = b2 * (double)at.v[g][j] + (1.0 - b2) * gr * gr;
        at.m[g][j] = (float)m;
        at.v[g][j] = (float)v;
        at.param[g][j] = (float)((double)at.param[g][j] - at.lr[g] * (m / bc1) / (sqrt(v / bc2) + eps));
    }
}

__global__ void k_step_advance(int32_t *step) {
    if (threadIdx.x == 0) step[0] += 1;
}

hipError_t launch_adam(const AdamTable &at, double b1, double b2, double eps, int32_t *step, hipStream_t s) {
    const int64_t total = at.off[at.n];
    if (total > 0) {
        int64_t blocks = (total + kThreads - 1) / kThreads;
        if (blocks > 2048) blocks = 2048;
        hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(kThreads), 0, s, at, b1, b2, eps,
                           (const int32_t *)step);
    }
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, s, step);
    return hipGetLastError();
}

}  // namespace bgt
