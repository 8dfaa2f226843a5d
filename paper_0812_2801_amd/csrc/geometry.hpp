// Minimum-image geometry of the Gaussian projector.  Used by the table
// builder, the stencil's nonlocal scatter and the force gather, so all three
// take the same membership decision and the same projector value.
#pragma once
#include "common.hpp"

namespace me {

#pragma clang fp contract(off)

__device__ __forceinline__ double min_image(double d, double L) {
    return d - L * rint(d * (1.0 / L));
}

// squared minimum-image distance between grid point (ix,iy,iz) and r
__device__ __forceinline__ double kb_d2(const KbGeom& g, int ix, int iy, int iz,
                                        double rx, double ry, double rz,
                                        double& dx, double& dy, double& dz) {
    dx = min_image(g.h * (double)ix - rx, g.L[0]);
    dy = min_image(g.h * (double)iy - ry, g.L[1]);
    dz = min_image(g.h * (double)iz - rz, g.L[2]);
    return dx * dx + dy * dy + dz * dz;
}

// projector value for a point inside the cutoff: (pi s^2)^(-3/4) exp(-d^2/(2 s^2))
__device__ __forceinline__ double kb_value(const KbGeom& g, double d2) {
    return g.pnorm * exp(-d2 * g.inv2s2);
}

// The nonlocal term at one point, in the order and rounding that the fix-up
// kernels share: s += p c over the covering projectors in ascending ion
// order, then v += (gr + i gi) s.
template <typename T>
__device__ __forceinline__ void nl_acc(T p, cx_t<T> c, T& sr, T& si) {
    sr = sr + p * c.x;
    si = si + p * c.y;
}
template <typename T>
__device__ __forceinline__ cx_t<T> nl_add(cx_t<T> v, T sr, T si, T gr, T gi) {
    v.x = v.x + (gr * sr - gi * si);
    v.y = v.y + (gr * si + gi * sr);
    return v;
}

#pragma clang fp contract(on)

// blocks are dispatched round-robin over the 8 XCDs; give every XCD a
// contiguous range of logical block ids so neighbouring tiles share its L2
__device__ __forceinline__ int xcd_remap(int b, int n) {
    const int X = 8;
    const int q = n / X, r = n % X;
    const int x = b % X, k = b / X;
    return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ int wrap1(int i, int n) {
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

}  // namespace me
