// Assembly on quadratic elements (used by every experiment of Sec. 4; element order is
// an input of the problem statement, Sec. 1): 20-node serendipity hexahedra, 8-node
// serendipity quadrilaterals (3-point Gauss rule per axis) and 10-node tetrahedra
// (collapsed 64-point rule), with the mass, conduction and elasticity forms of the linear
// kernel (Sec. 4.1, 4.2; K = dR/dU, d = -R at the zero state; plane strain in 2D) and the
// steady flow form with its stabilisation terms at a given state (Sec. 4.3; K the full
// Newton tangent, d = -R).
//
// One workgroup per element:
//   1. lanes load the element's node coordinates and sources (the state, for the flow
//      form) into LDS;
//   2. one lane per Gauss point builds J = sum_b x_b (x) grad_xi N_b in FP64, its
//      determinant and inverse, and stores g_b = J^-T grad_xi N_b for every node, the
//      weight W = w det J and the interpolated source in LDS (for the flow form: the
//      velocity, its gradient, the pressure, the momentum residual Rm and div u);
//   3. lane (row (a, i), part) sums the entries of row (a, i) for the column nodes b of
//      its part (a fixed share of the element's nodes) over the Gauss points and adds them
//      into K through the element-to-nonzero rank map (part 0 also adds d_(a,i)).
// Elements go colour by colour (no two elements of one colour share a node), one launch
// per colour, so the adds are plain read-modify-writes: every entry of K and d has one
// writer per launch, and the stream orders the launches.
// Local node orders: serendipity.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "mf_internal.h"
#include "serendipity.h"

namespace mf {
namespace {

enum ElemKind { kHex20 = 0, kQuad8 = 1, kTet10 = 2, kHex8 = 3 };

// Per element type: dimension, nodes and Gauss points.
template <int ET>
struct Elem;
template <>
struct Elem<kHex20> {
    static constexpr int DIM = 3, NEN = 20, NQ = 27;
};
template <>
struct Elem<kQuad8> {
    static constexpr int DIM = 2, NEN = 8, NQ = 9;
};
template <>
struct Elem<kTet10> {
    static constexpr int DIM = 3, NEN = 10, NQ = 64;
};
template <>
struct Elem<kHex8> {  // the flow form on 8-node bricks (2 Gauss points per axis)
    static constexpr int DIM = 3, NEN = 8, NQ = 8;
};

// Per element type and form: fields per node, the number of parts the column nodes of a
// row are split into (one lane per row and part), threads per workgroup, and the values
// per Gauss point that the flow form keeps in LDS (u, grad u, p, Rm, div u).
template <int ET, int FORM>
struct Cfg {
    static constexpr int DIM = Elem<ET>::DIM, NEN = Elem<ET>::NEN, NQ = Elem<ET>::NQ;
    static constexpr bool NS = FORM == MF_FORM_NS_SUPG;
    static constexpr int NF = FORM == MF_FORM_ELASTICITY ? DIM : NS ? DIM + 1 : 1;
    // 8-node bricks: one column node per lane, so the 96 momentum-row lanes and the 64
    // continuity-row lanes fill whole waves
    static constexpr int NPART = ET == kHex8 ? 8 : (NS || ET == kTet10) ? 2 : 4;
    static constexpr int ROWS = NEN * NF * NPART;
    // flow form: the momentum row lanes first, then the continuity row lanes from the next
    // wave on, so that no wave holds both kinds of row (their entries differ)
    static constexpr int MOM_LANES = NEN * DIM * NPART;
    static constexpr int CONT0 = (MOM_LANES + 63) / 64 * 64;
    static constexpr int ROW_LANES = NS ? CONT0 + NEN * NPART : ROWS;
    static constexpr int NEED = ROW_LANES > NQ ? ROW_LANES : NQ;
    static constexpr int THREADS = (NEED + 63) / 64 * 64;
    static constexpr int NSQ = NS ? 2 * DIM + DIM * DIM + 2 : 1;
    static constexpr int Q_U = 0, Q_GU = DIM, Q_P = DIM + DIM * DIM, Q_RM = Q_P + 1, Q_DIV = Q_RM + DIM;
    static_assert(NEN * DIM <= THREADS && NEN * NF <= THREADS && NEN % NPART == 0,
                  "one lane per row part, Gauss point and coordinate");
};

template <int ET>
__device__ __forceinline__ void shape(int a, const double (&x)[Elem<ET>::DIM], double& N,
                                      double (&dN)[Elem<ET>::DIM])
{
    if constexpr (ET == kHex20)
        shape20(a, x, N, dN);
    else if constexpr (ET == kQuad8)
        shape8(a, x, N, dN);
    else if constexpr (ET == kHex8) {
        // trilinear: N_a = prod_d (1 + s_d x_d) / 2, s_d = +1 where bit d of a is set
        double f[3], s[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            s[d] = ((a >> d) & 1) ? 1.0 : -1.0;
            f[d] = 0.5 * (1.0 + s[d] * x[d]);
        }
        N = f[0] * f[1] * f[2];
        dN[0] = 0.5 * s[0] * f[1] * f[2];
        dN[1] = 0.5 * s[1] * f[0] * f[2];
        dN[2] = 0.5 * s[2] * f[0] * f[1];
    } else
        shape10(a, x, N, dN);
}

// Gauss point q and its weight.  20-node bricks: 3 points per axis, first axis fastest;
// 8-node bricks: 2 points per axis, bit d of q the side along axis d.
// Tetrahedra: the 4-point Gauss-Legendre rule on each axis of the unit cube (u, v, w),
// collapsed by xi = (u, v (1 - u), w (1 - u)(1 - v)) with Jacobian (1 - u)^2 (1 - v).
template <int ET>
__device__ __forceinline__ void gauss_point(int q, double (&x)[Elem<ET>::DIM], double& w)
{
    if constexpr (ET == kTet10) {
        const double pts[4] = {0.5 * (1.0 - 0.8611363115940526), 0.5 * (1.0 - 0.3399810435848563),
                               0.5 * (1.0 + 0.3399810435848563), 0.5 * (1.0 + 0.8611363115940526)};
        const double wts[4] = {0.5 * 0.3478548451374538, 0.5 * 0.6521451548625461, 0.5 * 0.6521451548625461,
                               0.5 * 0.3478548451374538};
        const int i = q & 3, j = (q >> 2) & 3, k = q >> 4;
        const double u = pts[i], v = pts[j], t = pts[k];
        x[0] = u;
        x[1] = v * (1.0 - u);
        x[2] = t * (1.0 - u) * (1.0 - v);
        w = wts[i] * wts[j] * wts[k] * (1.0 - u) * (1.0 - u) * (1.0 - v);
    } else if constexpr (ET == kHex8) {
        const double g = 0.57735026918962576;  // 1/sqrt(3), weight 1; bit d of q picks the sign
#pragma unroll
        for (int d = 0; d < 3; ++d) x[d] = ((q >> d) & 1) ? g : -g;
        w = 1.0;
    } else {
        constexpr int DIM = Elem<ET>::DIM;
        const double p = 0.7745966692414834;  // sqrt(3/5)
        const double pts[3] = {-p, 0.0, p};
        const double wts[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
        w = 1.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const int k = q % 3;
            q /= 3;
            x[d] = pts[k];
            w *= wts[k];
        }
    }
}

// det J and (J^-1)[n][m] = dxi_n / dx_m (zero when det J <= 0)
template <int DIM>
__device__ __forceinline__ double invert(const double (&J)[DIM][DIM], double (&Ji)[DIM][DIM])
{
    if constexpr (DIM == 3) {
        const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        const double r = det > 0.0 ? 1.0 / det : 0.0;
        Ji[0][0] = c00 * r;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
        Ji[1][0] = c01 * r;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
        Ji[2][0] = c02 * r;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
        return det;
    } else {
        const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        const double r = det > 0.0 ? 1.0 / det : 0.0;
        Ji[0][0] = J[1][1] * r;
        Ji[0][1] = -J[0][1] * r;
        Ji[1][0] = -J[1][0] * r;
        Ji[1][1] = J[0][0] * r;
        return det;
    }
}

struct Q2Params {
    mf_form form;
    int64_t n_el, n_nodes;
    const int32_t* elems;  // the elements of one colour
    int64_t n_list;
    const int32_t* conn;
    const double* coords;
    const int32_t* row_ptr;
    const int32_t* nbr_ptr;
    const uint8_t* rank;
    const void* elem_param;
    const void* src;
    int field_major;
    void* K;
    void* d;
    unsigned long long* status;
};

// Geometry and the state at the points are formed in FP64; what the row phase reads (g, N,
// W, f, fs) is stored in the precision R of the assembly (FP64, or FP32 for MF_F32).
template <int ET, int FORM, typename R>
struct Q2Shared {
    using C = Cfg<ET, FORM>;
    double x[C::NEN][C::DIM];
    double src[C::NEN][C::NF];
    R g[C::NQ][C::NEN][C::DIM];
    R N[C::NQ][C::NEN];
    R W[C::NQ];
    R f[C::NQ][C::NF];
    R fs[C::NQ][C::NSQ];  // flow form: the state at the Gauss point
    int bad;
};

// Flow form, entries of row (a, i) against the columns (b, 0..dim) at one Gauss point
// (the tangent of the Q1 kernel, Sec. 4.3): a momentum row i < dim (CONT false), or the
// continuity row i = dim (CONT true).  F holds u, grad u (gu[i][k] = du_i/dx_k), p, Rm and
// div u at the point.
template <int DIM, bool CONT, typename R>
__device__ __forceinline__ void ns_entries(const mf_form& fm, int i, R Na, const R* ga, R Nb, const R* gb, const R* F,
                                           R (&v)[DIM + 1])
{
    const R rho = (R)fm.rho, mu = (R)fm.mu, tm = (R)fm.tau_m, tc = (R)fm.tau_c;
    const R* u = F;
    const R* gu = F + DIM;
    const R* Rm = F + DIM + DIM * DIM + 1;  // after p
    R adva = 0, advb = 0, gg = 0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        adva = fma(u[k], ga[k], adva);
        advb = fma(u[k], gb[k], advb);
        gg = fma(ga[k], gb[k], gg);
    }
    if constexpr (!CONT) {
        const R gai = ga[i];
        const R c_nb = (tm * rho * Rm[i] - rho * u[i]) * Nb;  // times g_al
        const R c_diag = -rho * adva * Nb + mu * gg + tm * rho * rho * adva * advb;
        const R c_gu = tm * rho * rho * adva * Nb;  // times gu[i][l]
#pragma unroll
        for (int l = 0; l < DIM; ++l)
            v[l] = c_nb * ga[l] + c_gu * gu[i * DIM + l] + tc * gai * gb[l] + (l == i ? c_diag : R(0));
        v[DIM] = -gai * Nb + tm * rho * adva * gb[i];
    } else {
#pragma unroll
        for (int l = 0; l < DIM; ++l) {
            R sl = 0;
#pragma unroll
            for (int m = 0; m < DIM; ++m) sl = fma(ga[m], gu[m * DIM + l], sl);
            v[l] = Na * gb[l] + tm * rho * (Nb * sl + ga[l] * advb);
        }
        v[DIM] = tm * gg;
    }
}

// Flow form, the residual entry R_(a,i) at one Gauss point.
template <int DIM, typename R>
__device__ __forceinline__ R ns_residual(const mf_form& fm, int i, R Na, const R* ga, const R* F)
{
    const R rho = (R)fm.rho, mu = (R)fm.mu, tm = (R)fm.tau_m, tc = (R)fm.tau_c;
    const R* u = F;
    const R* gu = F + DIM;
    const R p = F[DIM + DIM * DIM];
    const R* Rm = F + DIM + DIM * DIM + 1;
    const R div = F[2 * DIM + DIM * DIM + 1];
    if (i < DIM) {
        R adva = 0, visc = 0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            adva = fma(u[k], ga[k], adva);
            visc = fma(ga[k], gu[i * DIM + k], visc);
        }
        return -rho * adva * u[i] - ga[i] * p + mu * visc + tm * rho * adva * Rm[i] + tc * ga[i] * div;
    }
    R gRm = 0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) gRm = fma(ga[k], Rm[k], gRm);
    return Na * div + tm * gRm;
}

template <typename T>
__global__ void k_fill(T* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = T(0);
}

// The FP32 flow form on 20-node bricks is built for three workgroups per CU (168 VGPRs,
// 52 spilled: 1.23 ms against 1.28 ms on 24^3 bricks); the FP64 one spills 127 VGPRs at
// that budget and takes 2.78 ms against 1.67 ms, so it keeps the compiler's choice.
template <int ET, int FORM, typename T>
constexpr int q2_min_blocks()
{
    return (ET == kHex20 && FORM == MF_FORM_NS_SUPG && sizeof(T) == 4) ? 3 : 1;
}

template <int ET, int FORM, typename T>
__global__ void __launch_bounds__((Cfg<ET, FORM>::THREADS), (q2_min_blocks<ET, FORM, T>()))
    k_assemble_quadratic(Q2Params p)
{
    using C = Cfg<ET, FORM>;
    constexpr int DIM = C::DIM, NEN = C::NEN, NQ = C::NQ, NPART = C::NPART, NF = C::NF;
    constexpr int NBQ = NEN / NPART;
    using R = T;  // precision of the row phase
    __shared__ Q2Shared<ET, FORM, R> S;
    const int lane = threadIdx.x;
    const int64_t li = blockIdx.x;
    const bool live = li < p.n_list;  // uniform across the workgroup
    const int64_t e = live ? p.elems[li] : 0;
    if (live) {
        if (lane < NEN * DIM) {
            const int b = lane / DIM, m = lane % DIM;
            const int32_t v = p.conn[(int64_t)b * p.n_el + e];
            S.x[b][m] = p.coords[(int64_t)m * p.n_nodes + v];
        }
        if (lane < NEN * NF) {
            const int b = lane / NF, j = lane % NF;
            const int32_t v = p.conn[(int64_t)b * p.n_el + e];
            S.src[b][j] = p.src ? (double)((const T*)p.src)[(int64_t)j * p.n_nodes + v] : 0.0;
        }
        if (lane == 0) S.bad = 0;
    }
    __syncthreads();
    if (live && lane < NQ) {
        double xi[DIM], w;
        gauss_point<ET>(lane, xi, w);
        double J[DIM][DIM];
#pragma unroll
        for (int m = 0; m < DIM; ++m)
#pragma unroll
            for (int n = 0; n < DIM; ++n) J[m][n] = 0.0;
        for (int b = 0; b < NEN; ++b) {
            double Nb, dN[DIM];
            shape<ET>(b, xi, Nb, dN);
#pragma unroll
            for (int m = 0; m < DIM; ++m)
#pragma unroll
                for (int n = 0; n < DIM; ++n) J[m][n] = fma(S.x[b][m], dN[n], J[m][n]);
        }
        double Ji[DIM][DIM];
        const double det = invert<DIM>(J, Ji);
        if (!(det > 0.0)) {
            atomicMin(p.status, (unsigned long long)e);
            S.bad = 1;
        }
        double f[NF];
#pragma unroll
        for (int j = 0; j < NF; ++j) f[j] = 0.0;
        // flow form: the state's gradients at the point, from the FP64 basis gradients
        double gu[DIM][DIM], gp[DIM];
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
            gp[m] = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) gu[m][k] = 0.0;
        }
        for (int b = 0; b < NEN; ++b) {
            double Nb, dN[DIM], gb[DIM];
            shape<ET>(b, xi, Nb, dN);
#pragma unroll
            for (int m = 0; m < DIM; ++m) {
                double gm = 0.0;
#pragma unroll
                for (int n = 0; n < DIM; ++n) gm = fma(Ji[n][m], dN[n], gm);
                gb[m] = gm;
                S.g[lane][b][m] = (R)gm;
            }
            S.N[lane][b] = (R)Nb;
#pragma unroll
            for (int j = 0; j < NF; ++j) f[j] = fma(Nb, S.src[b][j], f[j]);
            if constexpr (C::NS) {
#pragma unroll
                for (int k = 0; k < DIM; ++k) {
#pragma unroll
                    for (int m = 0; m < DIM; ++m) gu[m][k] = fma(gb[k], S.src[b][m], gu[m][k]);
                    gp[k] = fma(gb[k], S.src[b][DIM], gp[k]);
                }
            }
        }
        S.W[lane] = (R)(w * det);
#pragma unroll
        for (int j = 0; j < NF; ++j) S.f[lane][j] = (R)f[j];
        if constexpr (C::NS) {
            // the state at the point: f holds (u, p) interpolated
            R* F = S.fs[lane];
            double div = 0.0;
#pragma unroll
            for (int m = 0; m < DIM; ++m) {
                F[C::Q_U + m] = (R)f[m];
                div += gu[m][m];
                double c = 0.0;
#pragma unroll
                for (int k = 0; k < DIM; ++k) {
                    F[C::Q_GU + m * DIM + k] = (R)gu[m][k];
                    c = fma(f[k], gu[m][k], c);
                }
                F[C::Q_RM + m] = (R)(p.form.rho * c + gp[m]);
            }
            F[C::Q_P] = (R)f[DIM];
            F[C::Q_DIV] = (R)div;
        }
    }
    __syncthreads();
    // lane -> (row node a, field i, part of the column nodes)
    int a = 0, i = 0, quarter = 0;
    bool active;
    if constexpr (C::NS) {
        if (lane < C::MOM_LANES) {
            quarter = lane / (NEN * DIM);
            a = lane % (NEN * DIM) / DIM;
            i = lane % DIM;
            active = true;
        } else {
            const int r = lane - C::CONT0;
            active = r >= 0 && r < NEN * NPART;
            quarter = r / NEN;
            a = r % NEN;
            i = DIM;
        }
    } else {
        const int rowl = lane % (NEN * NF);
        quarter = lane / (NEN * NF);
        a = rowl / NF;
        i = rowl % NF;
        active = lane < C::ROWS;
    }
    if (!live || S.bad || !active) return;
    const double ep = p.elem_param ? (double)((const T*)p.elem_param)[e] : 1.0;
    const double coef = p.form.coef * ep;
    double lam = 0.0, mu = 0.0;
    if constexpr (FORM == MF_FORM_ELASTICITY) {
        const double nu = p.form.nu;
        lam = coef * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
        mu = coef / (2.0 * (1.0 + nu));
    }
    const int32_t va = p.conn[(int64_t)a * p.n_el + e];
    const int64_t row = p.field_major ? (int64_t)i * p.n_nodes + va : (int64_t)NF * va + i;
    const int64_t rs = p.row_ptr[row];
    const int64_t deg = p.nbr_ptr[va + 1] - p.nbr_ptr[va];
    T* K = (T*)p.K;
    const int b0 = NBQ * quarter;
    // the part's column nodes all at once, Gauss point by Gauss point (the sum over the
    // points of each entry keeps its order)
    R acc[NBQ][NF];
#pragma unroll
    for (int bb = 0; bb < NBQ; ++bb)
#pragma unroll
        for (int j = 0; j < NF; ++j) acc[bb][j] = 0;
    const R coefr = (R)coef, lamr = (R)lam, mur = (R)mu;
    if constexpr (C::NS) {
        // i is the same on every lane of the wave: each branch holds its whole loop
        auto flow_rows = [&](auto cont) {
            constexpr bool CONT = decltype(cont)::value;
            for (int q = 0; q < NQ; ++q) {
                const R W = S.W[q];
#pragma unroll
                for (int bb = 0; bb < NBQ; ++bb) {
                    const int b = b0 + bb;
                    R v[NF];
                    ns_entries<DIM, CONT, R>(p.form, i, S.N[q][a], S.g[q][a], S.N[q][b], S.g[q][b], S.fs[q], v);
#pragma unroll
                    for (int j = 0; j < NF; ++j) acc[bb][j] = fma(W, v[j], acc[bb][j]);
                }
            }
        };
        if (i < DIM) flow_rows(std::false_type{});
        else flow_rows(std::true_type{});
    }
    for (int q = 0; q < (C::NS ? 0 : NQ); ++q) {
        const R W = S.W[q];
#pragma unroll
        for (int bb = 0; bb < NBQ; ++bb) {
            const int b = b0 + bb;
            if constexpr (C::NS) {
            } else if constexpr (FORM == MF_FORM_MASS) {
                acc[bb][0] = fma(W * coefr * S.N[q][a], S.N[q][b], acc[bb][0]);
            } else {
                R ga[DIM], gb[DIM], gg = 0;
#pragma unroll
                for (int m = 0; m < DIM; ++m) {
                    ga[m] = S.g[q][a][m];
                    gb[m] = S.g[q][b][m];
                    gg = fma(ga[m], gb[m], gg);
                }
                if constexpr (FORM == MF_FORM_POISSON) {
                    acc[bb][0] = fma(W * coefr, gg, acc[bb][0]);
                } else {
#pragma unroll
                    for (int j = 0; j < NF; ++j)
                        acc[bb][j] += W * (lamr * ga[i] * gb[j] + mur * ga[j] * gb[i] + (i == j ? mur * gg : R(0)));
                }
            }
        }
    }
    // every old value of the part is loaded before the first store, so the lane's
    // read-modify-writes overlap instead of running one after another
    int rk[NBQ];
#pragma unroll
    for (int bb = 0; bb < NBQ; ++bb) rk[bb] = p.rank[(int64_t)(a * NEN + b0 + bb) * p.n_el + e];
    auto pos_of = [&](int bb, int j) -> int64_t {
        return p.field_major ? rs + j * deg + rk[bb] : rs + (int64_t)rk[bb] * NF + j;
    };
    T old[NBQ][NF];
#pragma unroll
    for (int bb = 0; bb < NBQ; ++bb)
#pragma unroll
        for (int j = 0; j < NF; ++j) old[bb][j] = K[pos_of(bb, j)];
#pragma unroll
    for (int bb = 0; bb < NBQ; ++bb)
#pragma unroll
        for (int j = 0; j < NF; ++j) K[pos_of(bb, j)] = old[bb][j] + (T)acc[bb][j];
    if (quarter != 0) return;
    R dv = 0;
    if constexpr (C::NS) {
        for (int q = 0; q < NQ; ++q) dv -= S.W[q] * ns_residual<DIM, R>(p.form, i, S.N[q][a], S.g[q][a], S.fs[q]);
    } else {
        const R cd = FORM == MF_FORM_MASS ? coefr : R(1);
        for (int q = 0; q < NQ; ++q) dv = fma(S.W[q] * cd * S.N[q][a], S.f[q][i], dv);
    }
    ((T*)p.d)[row] += (T)dv;
    // a non-finite element parameter, source, state or form constant shows in the
    // coefficients or in dv
    double chk = (double)dv + coef + lam + mu;
    if constexpr (C::NS) chk += p.form.rho + p.form.mu + p.form.tau_m + p.form.tau_c;
    if (!isfinite(chk)) atomicMin(p.status + 2, (unsigned long long)e);
}

constexpr int kFillThreads = 256;
int blocks_for(int64_t n) { return (int)((n + kFillThreads - 1) / kFillThreads); }

template <int ET, int FORM, typename T>
mf_status launch(const AssembleArgs& A)
{
    const mf_pattern_s* P = A.P;
    Q2Params p{};
    p.form = *A.form;
    p.n_el = P->n_elems;
    p.n_nodes = P->n_nodes;
    p.conn = P->conn;
    p.coords = A.coords;
    p.row_ptr = P->row_ptr;
    p.nbr_ptr = P->nbr_ptr;
    p.rank = P->rank;
    p.elem_param = A.elem_param;
    p.src = FORM == MF_FORM_NS_SUPG ? A.lin_state : A.nodal_src;
    p.field_major = P->numbering == MF_FIELD_MAJOR;
    p.K = A.K;
    p.d = A.d;
    p.status = P->status;
    if (P->nnz > 0) k_fill<T><<<blocks_for(P->nnz), kFillThreads, 0, A.stream>>>((T*)A.K, P->nnz);
    if (P->n_rows > 0) k_fill<T><<<blocks_for(P->n_rows), kFillThreads, 0, A.stream>>>((T*)A.d, P->n_rows);
    MF_HIP(hipGetLastError());
    if (P->n_elems == 0) return MF_OK;
    mf_status st = ensure_coloring(P, A.stream);
    if (st != MF_OK) return st;
    for (size_t c = 0; c + 1 < P->color_ptr.size(); ++c) {
        p.elems = P->color_elems + P->color_ptr[c];
        p.n_list = P->color_ptr[c + 1] - P->color_ptr[c];
        if (p.n_list > 0)
            k_assemble_quadratic<ET, FORM, T><<<(unsigned)p.n_list, Cfg<ET, FORM>::THREADS, 0, A.stream>>>(p);
    }
    MF_HIP(hipGetLastError());
    return MF_OK;
}

template <int ET, typename T>
mf_status dispatch(const AssembleArgs& A)
{
    switch (A.form->kind) {
        case MF_FORM_MASS: return launch<ET, MF_FORM_MASS, T>(A);
        case MF_FORM_POISSON: return launch<ET, MF_FORM_POISSON, T>(A);
        case MF_FORM_ELASTICITY: return launch<ET, MF_FORM_ELASTICITY, T>(A);
        case MF_FORM_NS_SUPG: return launch<ET, MF_FORM_NS_SUPG, T>(A);
        default: return set_error(MF_ERR_UNSUPPORTED, "form %d on serendipity elements", (int)A.form->kind);
    }
}

}  // namespace

mf_status assemble_quadratic(const AssembleArgs& A)
{
    if (A.P->nen == 8 && A.P->dim == 3) {
        if (A.form->kind != MF_FORM_NS_SUPG) return MF_ERR_UNSUPPORTED;  // nothing launched or recorded
        return A.prec == MF_F64 ? launch<kHex8, MF_FORM_NS_SUPG, double>(A) : launch<kHex8, MF_FORM_NS_SUPG, float>(A);
    }
    if (A.P->nen == 20) return A.prec == MF_F64 ? dispatch<kHex20, double>(A) : dispatch<kHex20, float>(A);
    if (A.P->nen == 10) return A.prec == MF_F64 ? dispatch<kTet10, double>(A) : dispatch<kTet10, float>(A);
    return A.prec == MF_F64 ? dispatch<kQuad8, double>(A) : dispatch<kQuad8, float>(A);
}

}  // namespace mf
