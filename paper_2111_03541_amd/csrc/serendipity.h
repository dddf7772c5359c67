// The quadratic elements of Sec. 4: shape functions and reference gradients of the
// 20-node serendipity hexahedron on [-1, 1]^3, the 8-node serendipity quadrilateral on
// [-1, 1]^2 and the 10-node tetrahedron on the reference tetrahedron.  Local node order: corners a = ax + 2 ay + 4 az, then
// the midpoints of the x-, y- and z-directed edges, four each, ordered by the bits of the
// two other axes (ascending axis order).
//   corner   N = (1/8)(1 + s_x x)(1 + s_y y)(1 + s_z z)(s_x x + s_y y + s_z z - 2)
//   edge     N = (1/4)(1 - x_e^2)(1 + s_0 x_0)(1 + s_1 x_1)
#pragma once

#include <hip/hip_runtime.h>

namespace mf {

__device__ __forceinline__ double bit_sign(int b) { return b ? 1.0 : -1.0; }

// Shape functions and reference gradients of node a at xi.
__device__ __forceinline__ void shape20(int a, const double (&x)[3], double& N, double (&dN)[3])
{
    if (a < 8) {
        const double s[3] = {bit_sign(a & 1), bit_sign((a >> 1) & 1), bit_sign(a >> 2)};
        const double f[3] = {1.0 + s[0] * x[0], 1.0 + s[1] * x[1], 1.0 + s[2] * x[2]};
        const double t = s[0] * x[0] + s[1] * x[1] + s[2] * x[2] - 2.0;
        N = 0.125 * f[0] * f[1] * f[2] * t;
        dN[0] = 0.125 * s[0] * f[1] * f[2] * (t + f[0]);
        dN[1] = 0.125 * s[1] * f[0] * f[2] * (t + f[1]);
        dN[2] = 0.125 * s[2] * f[0] * f[1] * (t + f[2]);
        return;
    }
    const int m = a - 8, ax = m >> 2, k = m & 3;
    // the two other axes in ascending order carry the signs of bits 0 and 1 of k
    const int o0 = ax == 0 ? 1 : 0, o1 = ax == 2 ? 1 : 2;
    const double s0 = bit_sign(k & 1), s1 = bit_sign(k >> 1);
    const double g = 1.0 - x[ax] * x[ax], h0 = 1.0 + s0 * x[o0], h1 = 1.0 + s1 * x[o1];
    N = 0.25 * g * h0 * h1;
    dN[ax] = -0.5 * x[ax] * h0 * h1;
    dN[o0] = 0.25 * g * s0 * h1;
    dN[o1] = 0.25 * g * h0 * s1;
}

// The 8-node serendipity quadrilateral: corners a = ax + 2 ay, then the x-edge midpoints
// at y = -1, +1 and the y-edge midpoints at x = -1, +1.
//   corner  N = (1/4)(1 + s_x x)(1 + s_y y)(s_x x + s_y y - 1)
//   x-edge  N = (1/2)(1 - x^2)(1 + s_y y),   y-edge  N = (1/2)(1 - y^2)(1 + s_x x)
__device__ __forceinline__ void shape8(int a, const double (&x)[2], double& N, double (&dN)[2])
{
    if (a < 4) {
        const double sx = bit_sign(a & 1), sy = bit_sign(a >> 1);
        const double fx = 1.0 + sx * x[0], fy = 1.0 + sy * x[1], t = sx * x[0] + sy * x[1] - 1.0;
        N = 0.25 * fx * fy * t;
        dN[0] = 0.25 * sx * fy * (t + fx);
        dN[1] = 0.25 * sy * fx * (t + fy);
        return;
    }
    const int ax = (a - 4) >> 1;  // 0: edge along x, 1: edge along y
    const double s = bit_sign((a - 4) & 1);
    const double g = 1.0 - x[ax] * x[ax], h = 1.0 + s * x[1 - ax];
    N = 0.5 * g * h;
    dN[ax] = -x[ax] * h;
    dN[1 - ax] = 0.5 * g * s;
}

// The 10-node quadratic tetrahedron on the reference tetrahedron xi >= 0, sum xi <= 1:
// barycentric l_0 = 1 - xi_1 - xi_2 - xi_3, l_k = xi_k; vertices N_i = l_i (2 l_i - 1),
// edge midpoints N_ij = 4 l_i l_j for the edges (0,1), (1,2), (2,0), (0,3), (1,3), (2,3).
__device__ __forceinline__ void shape10(int a, const double (&x)[3], double& N, double (&dN)[3])
{
    auto lam = [&](int i) { return i == 0 ? 1.0 - x[0] - x[1] - x[2] : x[i - 1]; };
    auto dlam = [&](int i, int m) { return i == 0 ? -1.0 : (m == i - 1 ? 1.0 : 0.0); };
    if (a < 4) {
        const double l = lam(a);
        N = l * (2.0 * l - 1.0);
#pragma unroll
        for (int m = 0; m < 3; ++m) dN[m] = (4.0 * l - 1.0) * dlam(a, m);
        return;
    }
    constexpr int EI[6] = {0, 1, 2, 0, 1, 2}, EJ[6] = {1, 2, 0, 3, 3, 3};
    const int i = EI[a - 4], j = EJ[a - 4];
    const double li = lam(i), lj = lam(j);
    N = 4.0 * li * lj;
#pragma unroll
    for (int m = 0; m < 3; ++m) dN[m] = 4.0 * (li * dlam(j, m) + lj * dlam(i, m));
}

// Whether local node a lies on the face xi_axis = (side ? +1 : -1).
__device__ __forceinline__ bool on_face20(int a, int axis, int side)
{
    if (a < 8) return ((a >> axis) & 1) == side;
    const int m = a - 8, ax = m >> 2, k = m & 3;
    if (ax == axis) return false;
    const int o0 = ax == 0 ? 1 : 0;
    return (axis == o0 ? (k & 1) : (k >> 1)) == side;
}

}  // namespace mf
