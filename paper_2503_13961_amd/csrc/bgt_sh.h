// Attribute maps of resolution 1 or 3 (Eq. 5's interpolation) and the real
// spherical harmonics of the view-dependent colour, for the generation and
// parameter passes.
#pragma once
#include <hip/hip_runtime.h>

namespace bgt {

// Texels of a resolution-R map sit on the nodes (a, b), a + b <= R - 1, of
// the barycentric lattice of level R - 1 (index in the lattice order, a
// outer).  (u, v) takes the linear interpolation of the three nodes of the
// lattice triangle holding it; R = 1 is the single texel (weights 1, 0, 0).
template <typename T>
__device__ __forceinline__ void theta_weights(int R, T u, T v, int *ti, T *tw) {
    // every output is a select, not a store under a branch, so that the
    // caller's arrays stay in registers
    const int m = R > 1 ? R - 1 : 1;
    const T U = m * u, V = m * v;
    int ia = (int)floor(U), ib = (int)floor(V);
    ia = ia < 0 ? 0 : (ia > m - 1 ? m - 1 : ia);
    ib = ib < 0 ? 0 : (ib > m - 1 ? m - 1 : ib);
    if (ia + ib > m - 1) ib = m - 1 - ia;  // on the hypotenuse
    const T fu = U - ia, fv = V - ib;
    auto node = [m](int a, int b) { return a * (m + 1) - a * (a - 1) / 2 + b; };
    const bool one = R == 1, lower = fu + fv <= T(1);
    ti[0] = one ? 0 : (lower ? node(ia, ib) : node(ia + 1, ib));
    ti[1] = one ? 0 : (lower ? node(ia + 1, ib) : node(ia, ib + 1));
    ti[2] = one ? 0 : (lower ? node(ia, ib + 1) : node(ia + 1, ib + 1));
    tw[0] = one ? T(1) : (lower ? T(1) - fu - fv : T(1) - fv);
    tw[1] = one ? T(0) : (lower ? fu : T(1) - fu);
    tw[2] = one ? T(0) : (lower ? fv : fu + fv - T(1));
}

// Real SH of bands 1..D (Condon-Shortley phase, m = -l..l in a band) at the
// unit vector (x, y, z): f(k, Y_k, dY_k/dx, dY_k/dy, dY_k/dz) is called for
// k = 0 .. (D+1)^2 - 2 in order.  The normalisations are
// sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) (times sqrt 2 for m != 0) written
// out per function.  Every k is a constant at its call, so whatever f
// indexes or accumulates stays in registers (a loop over a stored basis
// with a run-time bound would put it in scratch memory).
template <typename T, typename F>
__device__ __forceinline__ void sh_basis_cb(int D, T x, T y, T z, F &&put) {
    const T pi = T(3.14159265358979323846);
    if (D >= 1) {
        const T c = sqrt(T(3) / (T(4) * pi));
        put(0, -c * y, T(0), -c, T(0));
        put(1, c * z, T(0), T(0), c);
        put(2, -c * x, -c, T(0), T(0));
    }
    if (D >= 2) {
        const T a = T(0.5) * sqrt(T(15) / pi), b = T(0.25) * sqrt(T(5) / pi), c = T(0.25) * sqrt(T(15) / pi);
        put(3, a * x * y, a * y, a * x, T(0));
        put(4, -a * y * z, T(0), -a * z, -a * y);
        put(5, b * (T(2) * z * z - x * x - y * y), -T(2) * b * x, -T(2) * b * y, T(4) * b * z);
        put(6, -a * x * z, -a * z, T(0), -a * x);
        put(7, c * (x * x - y * y), T(2) * c * x, -T(2) * c * y, T(0));
    }
    if (D >= 3) {
        const T a = T(0.25) * sqrt(T(35) / (T(2) * pi)), b = T(0.5) * sqrt(T(105) / pi);
        const T c = T(0.25) * sqrt(T(21) / (T(2) * pi)), e = T(0.25) * sqrt(T(7) / pi), g = T(0.25) * sqrt(T(105) / pi);
        const T xx = x * x, yy = y * y, zz = z * z;
        put(8, -a * y * (T(3) * xx - yy), -T(6) * a * x * y, -a * (T(3) * xx - T(3) * yy), T(0));
        put(9, b * x * y * z, b * y * z, b * x * z, b * x * y);
        put(10, -c * y * (T(4) * zz - xx - yy), T(2) * c * x * y, -c * (T(4) * zz - xx - T(3) * yy), -T(8) * c * y * z);
        put(11, e * z * (T(2) * zz - T(3) * xx - T(3) * yy), -T(6) * e * x * z, -T(6) * e * y * z,
            e * (T(6) * zz - T(3) * xx - T(3) * yy));
        put(12, -c * x * (T(4) * zz - xx - yy), -c * (T(4) * zz - T(3) * xx - yy), T(2) * c * x * y, -T(8) * c * x * z);
        put(13, g * z * (xx - yy), T(2) * g * x * z, -T(2) * g * y * z, g * (xx - yy));
        put(14, -a * x * (xx - T(3) * yy), -a * (T(3) * xx - T(3) * yy), T(6) * a * x * y, T(0));
    }
}

// SH degree from the coefficient count per channel, K = (D+1)^2 - 1
__host__ __device__ constexpr int sh_degree_of(int K) { return K >= 15 ? 3 : (K >= 8 ? 2 : (K >= 3 ? 1 : 0)); }

}  // namespace bgt
