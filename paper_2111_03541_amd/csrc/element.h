// Device-side Q1 element machinery shared by the assembly kernels of libmf.so:
// Gauss points, reference basis, FP64 geometry, and the per-integration-point
// contributions of each weak form to one row of the element matrix.
//
// Numerical integration of a bilinear form (Sec. 2.1): each integration point gamma
// contributes w_gamma * integrand, with the basis and its derivatives evaluated there.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mf.h"

namespace mf {

// 2-point Gauss-Legendre abscissa 1/sqrt(3); both weights are 1.
constexpr double kGaussPt = 0.57735026918962576450914878050196;

// Reference element [-1,1]^DIM, local node a = ax + 2 ay + 4 az, corner sign
// s_{a,d} = +1 if bit d of a is set, else -1.  Integration point q uses the same bit
// layout: xi_d = +1/sqrt(3) if bit d of q is set, else -1/sqrt(3).
template <int DIM>
__host__ __device__ __forceinline__ constexpr double ref_N(int a, int q)
{
    double v = 1.0;
    for (int d = 0; d < DIM; ++d) {
        double s = ((a >> d) & 1) ? 1.0 : -1.0;
        double xi = ((q >> d) & 1) ? kGaussPt : -kGaussPt;
        v *= 0.5 * (1.0 + s * xi);
    }
    return v;
}

template <int DIM>
__host__ __device__ __forceinline__ constexpr double ref_dN(int a, int q, int d)
{
    double v = ((a >> d) & 1) ? 0.5 : -0.5;
    for (int k = 0; k < DIM; ++k) {
        if (k == d) continue;
        double s = ((a >> k) & 1) ? 1.0 : -1.0;
        double xi = ((q >> k) & 1) ? kGaussPt : -kGaussPt;
        v *= 0.5 * (1.0 + s * xi);
    }
    return v;
}

// Reference basis at the 8 Gauss points of the hexahedron, for loops over q that are
// not unrolled (q is uniform across a wavefront, so the reads are scalar loads).
struct RefTablesHex {
    double N[8][8];      // [q][a]
    double dN[8][8][3];  // [q][a][d]
    constexpr RefTablesHex() : N{}, dN{}
    {
        for (int q = 0; q < 8; ++q)
            for (int a = 0; a < 8; ++a) {
                N[q][a] = ref_N<3>(a, q);
                for (int d = 0; d < 3; ++d) dN[q][a][d] = ref_dN<3>(a, q, d);
            }
    }
};
__constant__ constexpr RefTablesHex kRefHex{};

// Hexahedron geometry at a runtime integration point q (tables above); same arithmetic
// as geometry_at<3>.
__device__ __forceinline__ double geometry_hex_rt(const double (&x)[8][3], int q, double (&g)[8][3])
{
    double J[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < 8; ++a) s = fma(x[a][i], kRefHex.dN[q][a][j], s);
            J[i][j] = s;
        }
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double r = 1.0 / det;
    double Ji[3][3];
    Ji[0][0] = c00 * r;
    Ji[1][0] = c01 * r;
    Ji[2][0] = c02 * r;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) s = fma(kRefHex.dN[q][a][j], Ji[j][m], s);
            g[a][m] = s;
        }
    return det;
}

// Geometry at integration point q (FP64): J_ij = sum_a x_{a,i} dN_a/dxi_j, inverse by
// cofactors, g[a][m] = dN_a/dx_m = sum_j dN_a/dxi_j (J^-1)_{jm}.  Returns det J.
template <int DIM>
__device__ __forceinline__ double geometry_at(const double (&x)[1 << DIM][DIM], int q,
                                              double (&g)[1 << DIM][DIM])
{
    constexpr int NEN = 1 << DIM;
    double J[DIM][DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < NEN; ++a) s = fma(x[a][i], ref_dN<DIM>(a, q, j), s);
            J[i][j] = s;
        }
    double Ji[DIM][DIM];
    double det;
    if constexpr (DIM == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        double r = 1.0 / det;
        Ji[0][0] = J[1][1] * r;
        Ji[0][1] = -J[0][1] * r;
        Ji[1][0] = -J[1][0] * r;
        Ji[1][1] = J[0][0] * r;
    } else {
        double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        double r = 1.0 / det;
        Ji[0][0] = c00 * r;
        Ji[1][0] = c01 * r;
        Ji[2][0] = c02 * r;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
    }
#pragma unroll
    for (int a = 0; a < NEN; ++a)
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < DIM; ++j) s = fma(ref_dN<DIM>(a, q, j), Ji[j][m], s);
            g[a][m] = s;
        }
    return det;
}

template <int FORM, int DIM>
struct FormTraits;
template <int DIM>
struct FormTraits<MF_FORM_MASS, DIM> { static constexpr int NF = 1, NSRC = 1; };
template <int DIM>
struct FormTraits<MF_FORM_POISSON, DIM> { static constexpr int NF = 1, NSRC = 1; };
template <int DIM>
struct FormTraits<MF_FORM_ELASTICITY, DIM> { static constexpr int NF = DIM, NSRC = DIM; };
template <int DIM>
struct FormTraits<MF_FORM_NS_SUPG, DIM> { static constexpr int NF = DIM + 1, NSRC = DIM + 1; };

// Scalar coefficients of a form in the working precision T.
template <typename T>
struct Coef {
    T c;      // MASS density / POISSON conductivity (times elem_param)
    T lam;    // ELASTICITY Lame first parameter (Sec. 4.2)
    T mu;     // ELASTICITY shear modulus, or NS dynamic viscosity
    T rho, tau_m, tau_c;
};

template <typename T>
__device__ __forceinline__ Coef<T> make_coef(int form, const mf_form& f, double ep)
{
    Coef<T> c{};
    if (form == MF_FORM_ELASTICITY) {
        double E = f.coef * ep, nu = f.nu;
        c.lam = (T)(E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)));
        c.mu = (T)(E / (2.0 * (1.0 + nu)));
    } else if (form == MF_FORM_NS_SUPG) {
        c.rho = (T)f.rho;
        c.mu = (T)f.mu;
        c.tau_m = (T)f.tau_m;
        c.tau_c = (T)f.tau_c;
    } else {
        c.c = (T)(f.coef * ep);
    }
    return c;
}

// Contribution of one integration point to row (a, i) of the element tangent and
// element residual.  N[b], g[b][m] and W = w_q det J are in precision T; U[b][f] are
// the nodal values of the state (NS) or sources (others).
//   krow[b*NF + j] += W * dR_(a,i)/dU_(b,j)
//   rrow           += W * R_(a,i)
template <int FORM, int DIM, typename T>
__device__ __forceinline__ void row_update(int a, int i, const Coef<T>& C, const T (&N)[1 << DIM],
                                           const T (&g)[1 << DIM][DIM], T W,
                                           const T (&U)[1 << DIM][FormTraits<FORM, DIM>::NSRC],
                                           T (&krow)[(1 << DIM) * FormTraits<FORM, DIM>::NF], T& rrow)
{
    constexpr int NEN = 1 << DIM;
    constexpr int NF = FormTraits<FORM, DIM>::NF;
    if constexpr (FORM == MF_FORM_MASS || FORM == MF_FORM_POISSON) {
        T f = 0;
#pragma unroll
        for (int b = 0; b < NEN; ++b) f += N[b] * U[b][0];
        if constexpr (FORM == MF_FORM_MASS) {
            T wa = W * C.c * N[a];
#pragma unroll
            for (int b = 0; b < NEN; ++b) krow[b] += wa * N[b];
            rrow -= wa * f;                       // R = int c N_a (u - f) at u = 0
        } else {
            T ga[DIM];
#pragma unroll
            for (int m = 0; m < DIM; ++m) ga[m] = W * C.c * g[a][m];
#pragma unroll
            for (int b = 0; b < NEN; ++b) {
                T s = 0;
#pragma unroll
                for (int m = 0; m < DIM; ++m) s += ga[m] * g[b][m];
                krow[b] += s;
            }
            rrow -= W * N[a] * f;                 // R = int k grad N_a . grad u - N_a f at u = 0
        }
    } else if constexpr (FORM == MF_FORM_ELASTICITY) {
        // K_(a,i),(b,j) = lam g_ai g_bj + mu g_aj g_bi + mu delta_ij g_a . g_b
        T li = W * C.lam * g[a][i];
        T mg[DIM];
#pragma unroll
        for (int m = 0; m < DIM; ++m) mg[m] = W * C.mu * g[a][m];
#pragma unroll
        for (int b = 0; b < NEN; ++b) {
            T dot = 0;
#pragma unroll
            for (int m = 0; m < DIM; ++m) dot += mg[m] * g[b][m];
#pragma unroll
            for (int j = 0; j < DIM; ++j) {
                T v = li * g[b][j] + mg[j] * g[b][i];
                if (j == i) v += dot;
                krow[b * NF + j] += v;
            }
        }
        T bi = 0;
#pragma unroll
        for (int b = 0; b < NEN; ++b) bi += N[b] * U[b][i];
        rrow -= W * N[a] * bi;                    // R = int eps(N_a e_i) : sigma(u) - N_a b_i at u = 0
    } else {  // MF_FORM_NS_SUPG, Sec. 4.3 (NS_BASE + NS_SUPG)
        const T rho = C.rho, mu = C.mu, tm = C.tau_m, tc = C.tau_c;
        T u[DIM], p = 0, gu[DIM][DIM], gp[DIM];
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
            u[m] = 0;
            gp[m] = 0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) gu[m][k] = 0;
        }
#pragma unroll
        for (int b = 0; b < NEN; ++b) {
#pragma unroll
            for (int m = 0; m < DIM; ++m) {
                u[m] += N[b] * U[b][m];
#pragma unroll
                for (int k = 0; k < DIM; ++k) gu[m][k] += g[b][k] * U[b][m];  // du_m/dx_k
            }
            p += N[b] * U[b][DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) gp[k] += g[b][k] * U[b][DIM];
        }
        T div = 0;
#pragma unroll
        for (int m = 0; m < DIM; ++m) div += gu[m][m];
        T Rm[DIM];
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
            T c = 0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) c += u[k] * gu[m][k];
            Rm[m] = rho * c + gp[m];
        }
        T adv[NEN];
#pragma unroll
        for (int b = 0; b < NEN; ++b) {
            T s = 0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) s += u[k] * g[b][k];
            adv[b] = s;
        }
        if (i < DIM) {
            // momentum row (a, i)
            T visc = 0;
#pragma unroll
            for (int j = 0; j < DIM; ++j) visc += g[a][j] * gu[i][j];
            rrow += W * (-rho * adv[a] * u[i] - g[a][i] * p + mu * visc + tm * rho * adv[a] * Rm[i] +
                         tc * g[a][i] * div);
            const T w_adv_a = W * adv[a];
#pragma unroll
            for (int b = 0; b < NEN; ++b) {
                T gg = 0;
#pragma unroll
                for (int m = 0; m < DIM; ++m) gg += g[a][m] * g[b][m];
                // diagonal-in-(i,l) part
                T diag = -rho * adv[a] * N[b] + mu * gg + tm * rho * rho * adv[a] * adv[b];
#pragma unroll
                for (int l = 0; l < DIM; ++l) {
                    T v = (-rho * u[i] + tm * rho * Rm[i]) * g[a][l] * N[b] +
                          tm * rho * rho * adv[a] * N[b] * gu[i][l] + tc * g[a][i] * g[b][l];
                    if (l == i) v += diag;
                    krow[b * NF + l] += W * v;
                }
                krow[b * NF + DIM] += W * (-g[a][i] * N[b]) + tm * rho * w_adv_a * g[b][i];
            }
        } else {
            // continuity row (a, p)
            T gRm = 0;
#pragma unroll
            for (int m = 0; m < DIM; ++m) gRm += g[a][m] * Rm[m];
            rrow += W * (N[a] * div + tm * gRm);
            T sgu[DIM];  // sum_i g_ai du_i/dx_l
#pragma unroll
            for (int l = 0; l < DIM; ++l) {
                T s = 0;
#pragma unroll
                for (int m = 0; m < DIM; ++m) s += g[a][m] * gu[m][l];
                sgu[l] = s;
            }
#pragma unroll
            for (int b = 0; b < NEN; ++b) {
                T gg = 0;
#pragma unroll
                for (int m = 0; m < DIM; ++m) gg += g[a][m] * g[b][m];
#pragma unroll
                for (int l = 0; l < DIM; ++l)
                    krow[b * NF + l] += W * (N[a] * g[b][l] + tm * rho * (N[b] * sgu[l] + g[a][l] * adv[b]));
                krow[b * NF + DIM] += W * tm * gg;
            }
        }
    }
}

}  // namespace mf
