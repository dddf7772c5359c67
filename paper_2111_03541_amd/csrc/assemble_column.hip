// Owner-computes assembly on structured grids, streamed through columns of nodes
// (numerical integration and scatter of Sec. 2.2 D-2 and D-3, with no atomic increments
// into global memory).
//
// A workgroup owns the nodes of a 4x2 column cross-section over a range of node layers
// [z0, z1) and walks up the column one node layer kz at a time:
//   phase A  computes the element layer kz (the 5x3 elements around the column) into an
//            LDS ring: at each Gauss point q of element e, h_a(q) = sqrt(det J) grad N_a
//            for the eight element nodes (FP64 geometry, stored in the working
//            precision), W_q f(x_q) for the load vector, and the element coefficients;
//            it also writes out the rows of node layer kz-1, finished in the previous
//            step;
//   phase B  forms the rows of node layer kz from the element layers kz-1 and kz: lane
//            (a, e, half) contracts the four Gauss points of its half for the eight
//            node pairs (a, b), b in e; the two halves are added across adjacent lanes
//            and the blocks of the eight elements around a are summed into a per-node
//            LDS row buffer (FP64 in both precisions).  The flow form has its own
//            phase B on the matrix cores, described further down.
// Each value of K is written exactly once, in CSR row order, with the Dirichlet
// elimination applied on the way out.  The geometry of an element is computed once per
// column that sees it (15 elements per 8 owned nodes per layer); the small cross-section
// keeps the LDS of the FP64 elasticity case under half a CU, so two workgroups share
// each CU and overlap their phases.
//
// For a symmetric form the block of pair (a, b) is sum_q h_a h_b^T scaled by the element
// coefficients: mass c W N_a N_b, Poisson c h_a . h_b, elasticity
// lam M + mu M^T + mu tr(M) I with M = sum_q h_a h_b^T (Sec. 4.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "element.h"
#include "mf_internal.h"

namespace mf {
namespace {

constexpr int CX = 4, CY = 2;              // owned nodes per layer of a column
constexpr int kColNodes = CX * CY;
constexpr int EXH = CX + 1, EYH = CY + 1;  // elements per layer around the column
constexpr int kLayerElems = EXH * EYH;
constexpr int TX = CX + 2, TY = CY + 2;    // node tile per layer
constexpr int kTileNodes = TX * TY;
// Column cross-sections of the symmetric forms: XW owned nodes along x by kColNodes / XW
// along y, 4x2 or 2x4.  Both have the same node, element and tile counts, so one LDS
// layout and one lane layout serve both; only the index arithmetic differs.
template <int XW>
struct Cs {
    static constexpr int CX = XW, CY = kColNodes / XW;
    static constexpr int EXH = CX + 1, EYH = CY + 1, TX = CX + 2, TY = CY + 2;
    static_assert(CX * CY == kColNodes && EXH * EYH == kLayerElems && TX * TY == kTileNodes,
                  "the counts of the 4x2 cross-section");
};
constexpr int kThreads = kColNodes * 8 * 4;  // phase B: one lane per (node, element, quarter)
constexpr int kGeomThreads = 128;            // phase A: geometry on these, write-out on the rest
// workgroups per CU that the LDS of each case allows (FP64 and the flow form: 2; FP32
// symmetric forms: 3)
template <int FORM, typename T>
struct MinBlocks {
    static constexpr int value = (sizeof(T) == 4 && FORM != MF_FORM_NS_SUPG) ? 3 : 2;
};
// the batched kernel: its LDS is the union of the symmetric forms' (FP32: 49.5 KB)
template <typename T>
struct BatchMinBlocks {
    static constexpr int value = sizeof(T) == 4 ? 3 : 2;
};
constexpr int kGeomItems = kLayerElems * 8;  // (element, Gauss point)
constexpr int kPfElemT0 = 64, kPfInfoT0 = 96;  // phase B prefetch roles: [0, tile), [64, ..), [96, ..)
static_assert(kGeomItems <= kGeomThreads && kGeomThreads < kThreads, "one lane per (element, Gauss point)");
static_assert(kGeomThreads % 64 == 0 && kThreads % 64 == 0, "the write-out works in whole waves");
static_assert(kTileNodes <= kPfElemT0 && kPfElemT0 + kLayerElems <= kPfInfoT0 && kPfInfoT0 + kColNodes <= kThreads,
              "prefetch roles");

// LDS layout of the per-Gauss-point records (in units of T).  Symmetric forms store h
// (24 values); the flow form stores (sqrt(W) N_a, sqrt(W) grad N_a) for the eight nodes
// and the state terms u, grad u, Rm, sqrt(W), p and div u (50 values, NsRec below).  The strides spread the
// phase-B reads of one wave (eight nodes x two elements x four quarters) over the LDS
// banks: with an odd FP64 element stride the ten elements a wave reads start on distinct
// banks, which cuts the conflict degree of the h_b reads from 5 to 3 (32 banks).
template <int FORM, typename T>
struct HLayout {
    static constexpr bool NS = FORM == MF_FORM_NS_SUPG;
    static constexpr int SQ = NS ? 52 : (sizeof(T) == 8 ? 26 : 28);           // per Gauss point
    static constexpr int SE = 8 * SQ + (sizeof(T) == 8 ? 1 : 4);              // per element
    static constexpr int SL = kLayerElems * SE;                               // per element layer
};

constexpr int kNsTile = 68;  // floats per coefficient tile in LDS (64 used)

// Offsets inside one flow-form record: for each element node a, the four values
// (sqrt(W) N_a, sqrt(W) grad N_a) at R_PHI + 4 a, then the state at the point.
enum NsRec { R_PHI = 0, R_U = 32, R_GU = 35, R_RM = 44, R_S = 47, R_P = 48, R_DIV = 49 };

struct ColParams {
    mf_form form;
    int nx, ny, nz;  // elements per axis
    int lz;          // node layers per workgroup
    int n_nodes;
    const double* coords;
    const int32_t* nbr_ptr;
    const void* elem_param;
    const void* src;
    const uint8_t* dirichlet;
    int field_major;
    int n_pairs;
    void* K;
    void* d;
    unsigned long long* status;
    double lam_f, mu_f;  // elasticity: lambda = E lam_f, mu = E mu_f (from nu, on the host)
    int xw;              // cross-section of the batched launch's columns: 4 (4x2) or 2 (2x4)
};

// Row-buffer accumulators: FP64 for the symmetric forms in both precisions (FP32 rows,
// added with ds_add_f32, made the FP32 64^3 elasticity assembly 3.5x slower: 1,026 vs
// 291 us), FP32 for the flow form, whose rows are updated without atomics.
template <int FORM, typename T>
using AccT = typename std::conditional<FORM == MF_FORM_NS_SUPG, float, double>::type;

// value of the lane (lane ^ 1) or (lane ^ 2) of the same quad: DPP quad_perm [1,0,3,2]
// (0xB1) and [2,3,0,1] (0x4E)
template <int CTRL>
__device__ __forceinline__ double quad_swap(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float quad_swap(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
// sum over the four lanes of a quad, in every lane of it
template <typename T>
__device__ __forceinline__ T quad_sum(T v)
{
    v += quad_swap<0xB1>(v);
    return v + quad_swap<0x4E>(v);
}

// 1D linear basis factors at the Gauss point of bit qb: F[0] = (1 - xi)/2, F[1] = (1 + xi)/2
__device__ __forceinline__ void gauss_factors(int qb, double (&F)[2])
{
    const double xi = qb ? kGaussPt : -kGaussPt;
    F[0] = 0.5 * (1.0 - xi);
    F[1] = 0.5 * (1.0 + xi);
}

template <int FORM, typename T>
struct ColShared {
    static constexpr int NF = FormTraits<FORM, 3>::NF;
    static constexpr int NSRC = FormTraits<FORM, 3>::NSRC;
    static constexpr int NB = NF * NF;
    static constexpr bool NS = FORM == MF_FORM_NS_SUPG;
    // the flow form keeps one element layer of records and two row buffers (node layers kz
    // and kz + 1, which element layer kz feeds); the symmetric forms two element layers
    // and one row buffer
    static constexpr int RING = NS ? 1 : 2;
    static constexpr int NRB = NS ? 2 : 1;
    alignas(16) T h[RING * HLayout<FORM, T>::SL];
    T wf[2][kLayerElems][NS ? 1 : 8][NF];
    T cf[2][kLayerElems][2];
    double x[3][kTileNodes][3];
    T u[3][kTileNodes][NSRC];
    double ep[2][kLayerElems];
    alignas(16) AccT<FORM, T> rowK[NRB][kColNodes][27 * NB];
    AccT<FORM, T> rowD[NRB][kColNodes][NF];
    // flow form: per wave, the coefficient tiles of two (node, element) pairs, [pair][q]
    // tiles of [16][4] values, each padded to kNsTile floats (spreads the LDS banks)
    alignas(16) float dt[NS ? kThreads / 64 : 1][NS ? 2 * 8 * kNsTile : 1];
    int ni[kColNodes][4];  // node id, first pair offset, degree, boundary bits
    // Dirichlet flags of the tile's DOFs for node layers L = kz-2 .. kz+1 (slot L & 3): the
    // write-out of layer kz-1 reads its rows' and its neighbours' flags here, so no global
    // load follows its stores (a load would wait for every store in flight)
    uint8_t msk[4][kTileNodes][NF];
};

__device__ __forceinline__ int ring3(int L) { return (L + 3) % 3; }

// Global loads of one node of the tile of node layer L (registers), and their LDS store.
template <int NSRC, int NF, bool MASK, typename T>
struct NodeLoad {
    double x[3];
    T u[NSRC];
    int m;  // Dirichlet flag of field k in bit k
    bool ok;
    template <int XW = CX>
    __device__ __forceinline__ void load(const ColParams& p, int L, int tn, int i0, int j0)
    {
        const int NX = p.nx + 1, NY = p.ny + 1;
        const int gi = i0 - 1 + tn % Cs<XW>::TX, gj = j0 - 1 + tn / Cs<XW>::TX;
        ok = L >= 0 && L <= p.nz && gi >= 0 && gi < NX && gj >= 0 && gj < NY;
        if (!ok) return;
        const int node = gi + NX * (gj + NY * L);
#pragma unroll
        for (int c = 0; c < 3; ++c) x[c] = p.coords[(int64_t)c * p.n_nodes + node];
        const T* s = (const T*)p.src;
#pragma unroll
        for (int k = 0; k < NSRC; ++k) u[k] = s ? s[(int64_t)k * p.n_nodes + node] : T(0);
        m = 0;
        if (MASK && p.dirichlet) {
#pragma unroll
            for (int k = 0; k < NF; ++k)
                m |= (p.dirichlet[p.field_major ? (int64_t)k * p.n_nodes + node : (int64_t)NF * node + k] != 0) << k;
        }
    }
    template <int FORM>
    __device__ __forceinline__ void store(ColShared<FORM, T>& S, int L, int tn) const
    {
        if (!ok) return;
        const int r = ring3(L);
#pragma unroll
        for (int c = 0; c < 3; ++c) S.x[r][tn][c] = x[c];
#pragma unroll
        for (int k = 0; k < NSRC; ++k) S.u[r][tn][k] = u[k];
        if constexpr (MASK) {
#pragma unroll
            for (int k = 0; k < NF; ++k) S.msk[L & 3][tn][k] = (uint8_t)((m >> k) & 1);
        }
    }
};

template <int XW = CX>
__device__ __forceinline__ bool elem_param_of(const ColParams& p, int L, int el, int i0, int j0, bool f32,
                                              double& v)
{
    const int ex = i0 - 1 + el % Cs<XW>::EXH, ey = j0 - 1 + el / Cs<XW>::EXH;
    if (L < 0 || L >= p.nz || ex < 0 || ex >= p.nx || ey < 0 || ey >= p.ny) return false;
    const int e = ex + p.nx * (ey + p.ny * L);
    v = p.elem_param ? (f32 ? (double)((const float*)p.elem_param)[e] : ((const double*)p.elem_param)[e]) : 1.0;
    return true;
}

// Phase A: geometry of element `el` of element layer L at Gauss point q.
template <int FORM, typename T, int XW = CX>
__device__ __forceinline__ void geometry_item(const ColParams& p, ColShared<FORM, T>& S, int L, int el, int q,
                                              int i0, int j0)
{
    constexpr int NF = FormTraits<FORM, 3>::NF;
    const int hx = el % Cs<XW>::EXH, hy = el / Cs<XW>::EXH;
    const int ex = i0 - 1 + hx, ey = j0 - 1 + hy;
    if (L < 0 || L >= p.nz || ex < 0 || ex >= p.nx || ey < 0 || ey >= p.ny) return;
    // nodes are streamed from the LDS tile and the basis at the point is rebuilt from the
    // 1D factors where it is used, to keep few values live
    double F[3][2];
    gauss_factors(q & 1, F[0]);
    gauss_factors((q >> 1) & 1, F[1]);
    gauss_factors((q >> 2) & 1, F[2]);
    auto node_slot = [&](int a, int& r, int& tn) {
        r = ring3(L + (a >> 2));
        tn = (hx + (a & 1)) + Cs<XW>::TX * (hy + ((a >> 1) & 1));
    };
    auto N_of = [&](int a) { return F[0][a & 1] * F[1][(a >> 1) & 1] * F[2][a >> 2]; };
    auto dN_of = [&](int a, double (&d)[3]) {
        const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
        d[0] = (ax ? 0.5 : -0.5) * F[1][ay] * F[2][az];
        d[1] = (ay ? 0.5 : -0.5) * F[0][ax] * F[2][az];
        d[2] = (az ? 0.5 : -0.5) * F[0][ax] * F[1][ay];
    };
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    if constexpr (sizeof(T) == 8) {
        // FP64 kernels are bounded by LDS, not registers: load the eight nodes first
        double x[8][3];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            int r, tn;
            node_slot(a, r, tn);
#pragma unroll
            for (int i = 0; i < 3; ++i) x[a][i] = S.x[r][tn][i];
        }
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            double d[3];
            dN_of(a, d);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) J[i][j] = fma(x[a][i], d[j], J[i][j]);
        }
    } else {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            int r, tn;
            node_slot(a, r, tn);
            double d[3];
            dN_of(a, d);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double xa = S.x[r][tn][i];
#pragma unroll
                for (int j = 0; j < 3; ++j) J[i][j] = fma(xa, d[j], J[i][j]);
            }
        }
    }
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const int slot = L & 1;
    if (!(det > 0.0)) atomicMin(p.status, (unsigned long long)(ex + p.nx * (ey + p.ny * L)));
    const double ep = FORM == MF_FORM_NS_SUPG ? 1.0 : S.ep[slot][el];
    double coefA = 0.0, coefB = 0.0;
    if constexpr (FORM == MF_FORM_ELASTICITY) {
        const double E = p.form.coef * ep;
        coefA = E * p.lam_f;
        coefB = E * p.mu_f;
    } else {
        coefA = p.form.coef * ep;
    }
    T* hq = S.h + (ColShared<FORM, T>::RING == 1 ? 0 : slot) * HLayout<FORM, T>::SL + el * HLayout<FORM, T>::SE +
            q * HLayout<FORM, T>::SQ;
    if constexpr (FORM == MF_FORM_NS_SUPG) {
        // g = J^-T grad_xi N (FP64); state at the point: u, grad u, p, grad p, Rm, div u.
        // 1/det and sqrt(det) both from one reciprocal square root
        const double rs = rsqrt(det), r = rs * rs;
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
        auto g_of = [&](int a, double (&g)[3]) {
            double d[3];
            dN_of(a, d);
#pragma unroll
            for (int m = 0; m < 3; ++m) g[m] = fma(d[0], Ji[0][m], fma(d[1], Ji[1][m], d[2] * Ji[2][m]));
        };
        double u[3] = {0, 0, 0}, gu[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, pr = 0.0, gp[3] = {0, 0, 0};
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            int r, tn;
            node_slot(b, r, tn);
            double g[3];
            g_of(b, g);
            const double Nb = N_of(b);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const double Ub = (double)S.u[r][tn][m];
                u[m] = fma(Nb, Ub, u[m]);
#pragma unroll
                for (int k = 0; k < 3; ++k) gu[m][k] = fma(g[k], Ub, gu[m][k]);  // du_m/dx_k
            }
            const double Pb = (double)S.u[r][tn][3];
            pr = fma(Nb, Pb, pr);
#pragma unroll
            for (int k = 0; k < 3; ++k) gp[k] = fma(g[k], Pb, gp[k]);
        }
        const double rho = p.form.rho;
        const double sw = det * rs;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            double g[3];
            g_of(a, g);
            hq[R_PHI + 4 * a] = (T)(sw * N_of(a));
#pragma unroll
            for (int m = 0; m < 3; ++m) hq[R_PHI + 4 * a + 1 + m] = (T)(sw * g[m]);
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            hq[R_U + m] = (T)u[m];
            double c = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                hq[R_GU + 3 * m + k] = (T)gu[m][k];
                c = fma(u[k], gu[m][k], c);
            }
            hq[R_RM + m] = (T)(rho * c + gp[m]);
        }
        hq[R_S] = (T)sw;
        hq[R_P] = (T)pr;
        hq[R_DIV] = (T)(gu[0][0] + gu[1][1] + gu[2][2]);
        // a non-finite state value shows in the sum of the interpolated state and gradients
        double chk = pr + gp[0] + gp[1] + gp[2];
#pragma unroll
        for (int m = 0; m < 3; ++m) chk += u[m] + gu[m][0] + gu[m][1] + gu[m][2];
        if (!isfinite(chk)) atomicMin(p.status + 2, (unsigned long long)(ex + p.nx * (ey + p.ny * L)));
        return;
    } else if constexpr (FORM == MF_FORM_MASS) {
        hq[0] = (T)det;
    } else {
        double A[3][3];  // sqrt(det) * J^-1 = cofactor^T / sqrt(det): one reciprocal square root
        const double s = rsqrt(det);
        A[0][0] = c00 * s;
        A[1][0] = c01 * s;
        A[2][0] = c02 * s;
        A[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * s;
        A[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * s;
        A[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * s;
        A[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * s;
        A[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * s;
        A[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * s;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            double d[3];
            dN_of(a, d);
#pragma unroll
            for (int m = 0; m < 3; ++m) hq[3 * a + m] = (T)fma(d[0], A[0][m], fma(d[1], A[1][m], d[2] * A[2][m]));
        }
    }
    if constexpr (FORM != MF_FORM_NS_SUPG) {
        // load vector integrand W f(x_q) (times c for the mass form)
        const double wscale = det * (FORM == MF_FORM_MASS ? coefA : 1.0);
        double f[NF];
#pragma unroll
        for (int i = 0; i < NF; ++i) f[i] = 0.0;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            int r, tn;
            node_slot(a, r, tn);
            const double Na = N_of(a);
#pragma unroll
            for (int i = 0; i < NF; ++i) f[i] = fma(Na, (double)S.u[r][tn][i], f[i]);
        }
        double chk = coefA + coefB;
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            S.wf[slot][el][q][i] = (T)(wscale * f[i]);
            chk += f[i];
        }
        // a non-finite element parameter or source value (the coordinates are checked by
        // det J > 0 above)
        if (!isfinite(chk)) atomicMin(p.status + 2, (unsigned long long)(ex + p.nx * (ey + p.ny * L)));
        if (q == 0) {
            S.cf[slot][el][0] = (T)coefA;
            S.cf[slot][el][1] = (T)coefB;
        }
    }
}

// Phase B: lane (node al, element eps around it, quarter bq) of node layer kz: the pair
// blocks (a, b) for the two element nodes b = 2 bq, 2 bq + 1, over all eight Gauss
// points.  The element's load-vector share of a is split by Gauss-point pairs between
// the four lanes of (al, eps) and added across them.
template <int FORM, typename T, int XW>
__device__ __forceinline__ void pair_item(const ColParams& p, ColShared<FORM, T>& S, int kz, int i0, int j0)
{
    constexpr int NF = FormTraits<FORM, 3>::NF;
    using Acc = AccT<FORM, T>;
    static_assert(FORM != MF_FORM_NS_SUPG, "the flow form has its own phase B");
    constexpr int NV = FORM == MF_FORM_ELASTICITY ? 9 : 1;
    const int tid = threadIdx.x;
    const int bq = tid & 3, pe = tid >> 2;
    const int al = pe & (kColNodes - 1), eps = pe / kColNodes;
    const int alx = al % Cs<XW>::CX, aly = al / Cs<XW>::CX;
    const int gi = i0 + alx, gj = j0 + aly;
    const int dx = eps & 1, dy = (eps >> 1) & 1, dz = eps >> 2;
    const int ex = gi - 1 + dx, ey = gj - 1 + dy, ez = kz - 1 + dz;
    const bool valid = gi <= p.nx && gj <= p.ny && ex >= 0 && ex < p.nx && ey >= 0 && ey < p.ny && ez >= 0 &&
                       ez < p.nz;
    const int alpha = 7 - eps;  // the node's local index in the element
    const int slot = ez & 1, el = (alx + dx) + Cs<XW>::EXH * (aly + dy);
    const T* he = S.h + slot * HLayout<FORM, T>::SL + el * HLayout<FORM, T>::SE;

    T M[2][NV];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < NV; ++v) M[b][v] = T(0);
    T dp[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) dp[i] = T(0);

    if (valid) {
        const int fb = 2 * bq;  // first element node of this lane's pair
        // FP64: unrolled over the eight points; FP32 (three workgroups per CU) keeps two
        // per trip, which holds it within its register budget
        constexpr int kUnrollQ = sizeof(T) == 8 ? 8 : 2;
#pragma unroll kUnrollQ
        for (int q = 0; q < 8; ++q) {
            const T* hq = he + q * HLayout<FORM, T>::SQ;
            if constexpr (FORM == MF_FORM_MASS) {
                double Fx[2], Fy[2], Fz[2];
                gauss_factors(q & 1, Fx);
                gauss_factors((q >> 1) & 1, Fy);
                gauss_factors(q >> 2, Fz);
                const double Na = Fx[alpha & 1] * Fy[(alpha >> 1) & 1] * Fz[alpha >> 2];
                const T wa = hq[0] * (T)Na;
#pragma unroll
                for (int b = 0; b < 2; ++b) M[b][0] += wa * (T)(Fx[b] * Fy[bq & 1] * Fz[bq >> 1]);
            } else {
                T hb[2][3];
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int m = 0; m < 3; ++m) hb[b][m] = hq[3 * (fb + b) + m];
                T ha[3];
#pragma unroll
                for (int m = 0; m < 3; ++m) ha[m] = hq[3 * alpha + m];
                if constexpr (FORM == MF_FORM_ELASTICITY) {
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int i = 0; i < 3; ++i)
#pragma unroll
                            for (int j = 0; j < 3; ++j) M[b][3 * i + j] += ha[i] * hb[b][j];
                } else {
#pragma unroll
                    for (int b = 0; b < 2; ++b) M[b][0] += ha[0] * hb[b][0] + ha[1] * hb[b][1] + ha[2] * hb[b][2];
                }
            }
        }
        // load vector over this lane's two points
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int q = 2 * bq + k;
            double Fx[2], Fy[2], Fz[2];
            gauss_factors(k, Fx);
            gauss_factors(bq & 1, Fy);
            gauss_factors(bq >> 1, Fz);
            const double Na = Fx[alpha & 1] * Fy[(alpha >> 1) & 1] * Fz[alpha >> 2];
#pragma unroll
            for (int i = 0; i < NF; ++i) dp[i] += (T)Na * S.wf[slot][el][q][i];
        }
    }
#pragma unroll
    for (int i = 0; i < NF; ++i) dp[i] = quad_sum(dp[i]);
    if (!valid) return;

    const T cA = S.cf[slot][el][0];
    const T cB = S.cf[slot][el][1];
    const int ax = alpha & 1, ay = (alpha >> 1) & 1, az = alpha >> 2;
    Acc* row = &S.rowK[0][al][0];  // K order: [(i * 27 + slot) * NF + j]
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int nslot = ((bq >> 1) - az + 1) * 9 + ((bq & 1) - ay + 1) * 3 + (b - ax + 1);
        if constexpr (FORM == MF_FORM_ELASTICITY) {
            const T tr = M[b][0] + M[b][4] + M[b][8];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const T v = cA * M[b][3 * i + j] + cB * M[b][3 * j + i] + (i == j ? cB * tr : T(0));
                    unsafeAtomicAdd(row + (i * 27 + nslot) * 3 + j, (Acc)v);
                }
        } else {
            unsafeAtomicAdd(row + nslot, (Acc)(cA * M[b][0]));
        }
    }
    if (bq == 0) {
#pragma unroll
        for (int i = 0; i < NF; ++i) unsafeAtomicAdd(&S.rowD[0][al][i], (Acc)dp[i]);
    }
}

// Rows of node layer kz from the row buffers (cleared on the way for the next layer),
// by the workers wid in [0, nw) (whole waves).  Each wave takes whole nodes: their
// values are loaded from LDS in 64-lane chunks before any store, and the buffer is in
// the order of a node-major CSR row block, so an interior node's rows are one contiguous
// copy; boundary nodes, field-major numbering and Dirichlet masks take the general
// mapping.  K is written once and is far larger than the caches: non-temporal stores.
template <int FORM, bool MASK, typename T, int XW = CX>
__device__ __forceinline__ void write_layer(const ColParams& p, ColShared<FORM, T>& S, int L, int wid, int nw,
                                            int rb = 0)
{
    constexpr int WX = Cs<XW>::CX, WTX = Cs<XW>::TX;
    constexpr int NF = FormTraits<FORM, 3>::NF;
    constexpr int NB = NF * NF;
    constexpr int kNodeVals = 27 * NB;
    constexpr int NCH = (kNodeVals + 63) / 64;
    using Acc = AccT<FORM, T>;
    T* K = (T*)p.K;
    T* d = (T*)p.d;
    const int nn = p.n_nodes;
    const bool masked = MASK && p.dirichlet;
    const bool plain = !p.field_major && !masked;
    int lane = wid & 63;
    // flow form: the per-chunk index arithmetic below depends only on the lane; keep the
    // compiler from hoisting it out of the layer loop, where it would hold registers
    // throughout (the kernel spilled)
    if constexpr (FORM == MF_FORM_NS_SUPG) asm volatile("" : "+v"(lane));
    const int wv = wid >> 6, nwv = nw >> 6;
    for (int il = wv; il < kColNodes; il += nwv) {
        Acc vals[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int o = lane + 64 * c;
            vals[c] = o < kNodeVals ? S.rowK[rb][il][o] : Acc(0);
        }
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int o = lane + 64 * c;
            if (o < kNodeVals) S.rowK[rb][il][o] = Acc(0);
        }
        const int node = S.ni[il][0];
        if (node < 0) continue;
        const int bits = S.ni[il][3];
        const int P = S.ni[il][1];
        bool contiguous = plain && bits == 63;
        if constexpr (MASK) {
            // an interior node with no flag on itself or its 26 neighbours keeps the
            // contiguous copy (one lane per neighbour; the node is wave-uniform)
            if (masked && !p.field_major && bits == 63) {
                bool hit = false;
                if (lane < 27) {
                    const int tn = il % WX + 1 + WTX * (il / WX + 1) + (lane % 3 - 1) + WTX * ((lane / 3) % 3 - 1);
#pragma unroll
                    for (int k = 0; k < NF; ++k) hit |= S.msk[(L + lane / 9 - 1) & 3][tn][k] != 0;
                }
                contiguous = !__any(hit);
            }
        }
        if (contiguous) {
            T* dst = K + (int64_t)P * NB;
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int o = lane + 64 * c;
                if (o < kNodeVals) __builtin_nontemporal_store((T)vals[c], &dst[o]);
            }
            continue;
        }
        const int deg = S.ni[il][2];
        const int lo_x = bits & 1, lo_y = (bits >> 2) & 1, lo_z = (bits >> 4) & 1;
        const int mx = 1 + lo_x + ((bits >> 1) & 1), my = 1 + lo_y + ((bits >> 3) & 1);
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int o = lane + 64 * c;  // (i * 27 + slot) * NF + j
            if (o >= kNodeVals) continue;
            const int i = o / (27 * NF);
            const int rem = o - i * (27 * NF);
            const int slot = rem / NF, j = rem - slot * NF;
            const int ddx = slot % 3 - 1, ddy = (slot / 3) % 3 - 1, ddz = slot / 9 - 1;
            const int need = (ddx < 0 ? 1 : 0) | (ddx > 0 ? 2 : 0) | (ddy < 0 ? 4 : 0) | (ddy > 0 ? 8 : 0) |
                             (ddz < 0 ? 16 : 0) | (ddz > 0 ? 32 : 0);
            if ((bits & need) != need) continue;
            const int rank = ((ddz + lo_z) * my + (ddy + lo_y)) * mx + (ddx + lo_x);
            const int kpos = p.field_major ? i * NF * p.n_pairs + NF * P + j * deg + rank
                                           : P * NB + i * NF * deg + rank * NF + j;
            T v = (T)vals[c];
            if (masked) {
                const int tn = il % WX + 1 + WTX * (il / WX + 1);  // the node in the tile
                if (S.msk[L & 3][tn][i]) v = (slot == 13 && j == i) ? T(1) : T(0);
                else if (S.msk[(L + ddz) & 3][tn + ddx + WTX * ddy][j]) v = T(0);
            }
            __builtin_nontemporal_store(v, &K[kpos]);
        }
    }
    if (wid < kColNodes * NF) {
        const int il = wid / NF, i = wid - il * NF;
        const Acc acc = S.rowD[rb][il][i];
        S.rowD[rb][il][i] = Acc(0);
        const int node = S.ni[il][0];
        if (node >= 0) {
            const int row = p.field_major ? i * nn + node : NF * node + i;
            d[row] = (masked && S.msk[L & 3][il % WX + 1 + WTX * (il / WX + 1)][i]) ? T(0) : (T)acc;
        }
    }
}

// One column chunk b of one problem (b = column + columns * chunk); called by the
// single-problem kernel and by the persistent batched kernel.
template <int FORM, bool MASK, typename T, int XW = CX>
__device__ __forceinline__ void column_body(const ColParams& p, int b, ColShared<FORM, T>& S)
{
    constexpr int NF = FormTraits<FORM, 3>::NF;
    constexpr int NSRC = FormTraits<FORM, 3>::NSRC;
    constexpr int NB = NF * NF;
    const int tid = threadIdx.x;
    const int NX = p.nx + 1, NY = p.ny + 1, NZ = p.nz + 1;
    constexpr int BX = Cs<XW>::CX, BY = Cs<XW>::CY;
    const int ncx = (NX + BX - 1) / BX, ncy = (NY + BY - 1) / BY;
    const int cx = b % ncx, cy = (b / ncx) % ncy, ch = b / (ncx * ncy);
    const int i0 = cx * BX, j0 = cy * BY;
    const int z0 = ch * p.lz, z1 = min(z0 + p.lz, NZ);
    const bool f32 = sizeof(T) == 4;

    for (int k = tid; k < kColNodes * 27 * NB; k += kThreads) (&S.rowK[0][0][0])[k] = 0.0;
    for (int k = tid; k < kColNodes * NF; k += kThreads) (&S.rowD[0][0][0])[k] = 0.0;
    // prologue: node layers z0-1 .. z0+1, element parameters of layers z0-1 and z0
    for (int it = tid; it < 3 * kTileNodes; it += kThreads) {
        NodeLoad<NSRC, NF, MASK, T> ld;
        const int L = z0 - 1 + it / kTileNodes, tn = it % kTileNodes;
        ld.template load<XW>(p, L, tn, i0, j0);
        ld.template store<FORM>(S, L, tn);
    }
    for (int it = tid; it < 2 * kLayerElems; it += kThreads) {
        const int L = z0 - 1 + it / kLayerElems, el = it % kLayerElems;
        double v;
        if (elem_param_of<XW>(p, L, el, i0, j0, f32, v)) S.ep[L & 1][el] = v;
    }
    __syncthreads();

    for (int kz = z0; kz < z1; ++kz) {
        // ---- phase A: geometry of element layer kz (and kz-1 on the first step); rows of kz-1
        const int first = kz == z0 ? kz - 1 : kz;
        if (tid < kGeomThreads) {
            for (int it = tid; it < (kz - first + 1) * kGeomItems; it += kGeomThreads) {
                const int L = first + it / kGeomItems, r = it % kGeomItems;
                geometry_item<FORM, T, XW>(p, S, L, r >> 3, r & 7, i0, j0);
            }
        } else if (kz > z0) {
            write_layer<FORM, MASK, T, XW>(p, S, kz - 1, tid - kGeomThreads, kThreads - kGeomThreads);
        }
        __syncthreads();

        // ---- phase B: rows of node layer kz; prefetch for the next step
        NodeLoad<NSRC, NF, MASK, T> ld;
        ld.ok = false;
        double epv = 0.0;
        bool ep_ok = false;
        int info[4] = {-1, 0, 0, 0};
        if (tid < kTileNodes) {
            ld.template load<XW>(p, kz + 2, tid, i0, j0);
        } else if (tid >= kPfElemT0 && tid < kPfElemT0 + kLayerElems) {
            ep_ok = elem_param_of<XW>(p, kz + 1, tid - kPfElemT0, i0, j0, f32, epv);
        } else if (tid >= kPfInfoT0 && tid < kPfInfoT0 + kColNodes) {
            const int il = tid - kPfInfoT0;
            const int gi = i0 + il % BX, gj = j0 + il / BX;
            if (gi < NX && gj < NY) {
                const int node = gi + NX * (gj + NY * kz);
                const int mx = 1 + (gi > 0) + (gi < p.nx), my = 1 + (gj > 0) + (gj < p.ny),
                          mz = 1 + (kz > 0) + (kz < p.nz);
                info[0] = node;
                info[1] = p.nbr_ptr[node];
                info[2] = mx * my * mz;
                info[3] = (gi > 0) | ((gi < p.nx) << 1) | ((gj > 0) << 2) | ((gj < p.ny) << 3) | ((kz > 0) << 4) |
                          ((kz < p.nz) << 5);
            }
        }
        pair_item<FORM, T, XW>(p, S, kz, i0, j0);
        if (tid < kTileNodes) ld.template store<FORM>(S, kz + 2, tid);
        if (ep_ok) S.ep[(kz + 1) & 1][tid - kPfElemT0] = epv;
        if (tid >= kPfInfoT0 && tid < kPfInfoT0 + kColNodes) {
#pragma unroll
            for (int k = 0; k < 4; ++k) S.ni[tid - kPfInfoT0][k] = info[k];
        }
        __syncthreads();
    }
    if (z0 < z1) write_layer<FORM, MASK, T, XW>(p, S, z1 - 1, tid, kThreads);
}

// ------------------------------------------------------------------------------------
// Flow form (FP32): the pair contraction on the matrix cores.
//
// For one owned node a and one element e around it, the 4x4 blocks of row a against the
// eight element nodes b factor through the b-side values phi_t(b) at each Gauss point q
// (t = 0: sqrt(W) N_b, t = 1..3: sqrt(W) dN_b/dx_t, so every product carries W):
//     K[(a,i),(b,l)] += sum_{q,t} C[a,q][i][l][t] phi_t(b, q),
// where C collects the a-side factors of each term of the Jacobian (Sec. 4.3 form,
// differentiated as the oracle does).  That is a product of a [16 x 32] coefficient tile
// (rows (i, l), columns (q, t)) and the [32 x 8] table phi (rows (q, t), columns b).
// v_mfma_f32_4x4x1_16b runs sixteen independent 4x4 outer products: block (pair, i, b
// half) takes row i's four l values against four b, one (q, t) per instruction, so a wave
// forms two (node, element) pairs in 32 instructions with every lane busy.  The
// coefficient tiles are computed once per (node, element, q) by 16 lanes and passed
// through LDS; each wave owns two nodes, so its row-buffer updates are plain
// read-modify-writes with no atomics.
//
// Element layer kz feeds node layer kz (through the elements above it) and node layer
// kz + 1 (below it); the body keeps one element layer of records and two row buffers.
// ------------------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));

// orders the LDS accesses of the lanes of one wave
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// owned node al, element eps around it (bits dx, dy, dz), node layer Ln: whether the pair
// contributes, the element's position in the layer's record ring and the node's local
// index in the element
struct NsPair {
    bool ok;
    int el;
    int alpha;
};
__device__ __forceinline__ NsPair ns_pair(const ColParams& p, int al, int eps, int Ln, int zend, int i0, int j0)
{
    const int alx = al % CX, aly = al / CX;
    const int gi = i0 + alx, gj = j0 + aly;
    const int dx = eps & 1, dy = (eps >> 1) & 1, dz = eps >> 2;
    const int ex = gi - 1 + dx, ey = gj - 1 + dy, ez = Ln - 1 + dz;
    NsPair r;
    r.ok = gi <= p.nx && gj <= p.ny && Ln < zend && ex >= 0 && ex < p.nx && ey >= 0 && ey < p.ny && ez >= 0 &&
           ez < p.nz;
    r.el = (alx + dx) + EXH * (aly + dy);
    r.alpha = 7 - eps;
    return r;
}

// Row i of the coefficient tile C[a,q] of one pair at one Gauss point (four column
// fields l of four values t), written to dst [4][4]; the pair's share of (d = -R)_i at
// the point is added to dpi.  i is the lane's row field (3 = pressure).
__device__ __forceinline__ void ns_coef_row(const ColParams& p, const float* __restrict__ hq, int a, int i,
                                            float* __restrict__ dst, float& dpi)
{
    const float rho = (float)p.form.rho, mu = (float)p.form.mu, tm = (float)p.form.tau_m, tc = (float)p.form.tau_c;
    const f32x4 pa4 = *(const f32x4*)(hq + R_PHI + 4 * a);
    const float Nta = pa4.x, ha[3] = {pa4.y, pa4.z, pa4.w};
    // state at the point: u (3), grad u (9, du_m/dx_k at 3 m + k), Rm (3), sqrt(W), p, div u
    const f32x4 s0 = *(const f32x4*)(hq + R_U), s1 = *(const f32x4*)(hq + R_U + 4),
                s2 = *(const f32x4*)(hq + R_U + 8), s3 = *(const f32x4*)(hq + R_U + 12),
                s4 = *(const f32x4*)(hq + R_U + 16);
    const float u[3] = {s0.x, s0.y, s0.z};
    const float gu[3][3] = {{s0.w, s1.x, s1.y}, {s1.z, s1.w, s2.x}, {s2.y, s2.z, s2.w}};
    const float Rm[3] = {s3.x, s3.y, s3.z};
    const float sw = s3.w, pr = s4.x, div = s4.y;
    const float aa = u[0] * ha[0] + u[1] * ha[1] + u[2] * ha[2];  // sqrt(W) u . grad N_a
    const float d3 = tm * rho * rho * aa;
    // the lane's row values (i < 3; i = 3 reads row 2, unused)
    const bool r0 = i == 0, r1 = i == 1;
    const float ui = r0 ? u[0] : (r1 ? u[1] : u[2]);
    const float Rmi = r0 ? Rm[0] : (r1 ? Rm[1] : Rm[2]);
    const float hai = r0 ? ha[0] : (r1 ? ha[1] : ha[2]);
    float gui[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) gui[k] = r0 ? gu[0][k] : (r1 ? gu[1][k] : gu[2][k]);
    f32x4 v[4];
    if (i < 3) {
        const float ci = tm * rho * Rmi - rho * ui;
        const float cH = tc * hai;
        const float dd = -rho * aa;                                   // (i == l) part of the N column
        const float dk[3] = {mu * ha[0] + d3 * u[0], mu * ha[1] + d3 * u[1], mu * ha[2] + d3 * u[2]};
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const bool il = i == l;
            v[l].x = ci * ha[l] + d3 * gui[l] + (il ? dd : 0.0f);
            v[l].y = (il ? dk[0] : 0.0f) + (l == 0 ? cH : 0.0f);
            v[l].z = (il ? dk[1] : 0.0f) + (l == 1 ? cH : 0.0f);
            v[l].w = (il ? dk[2] : 0.0f) + (l == 2 ? cH : 0.0f);
        }
        const float pa = tm * rho * aa;
        v[3].x = -hai;
        v[3].y = r0 ? pa : 0.0f;
        v[3].z = r1 ? pa : 0.0f;
        v[3].w = i == 2 ? pa : 0.0f;
        const float visc = ha[0] * gui[0] + ha[1] * gui[1] + ha[2] * gui[2];
        dpi -= sw * (-rho * aa * ui - hai * pr + mu * visc + tm * rho * aa * Rmi + tc * hai * div);
    } else {
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const float sgu = ha[0] * gu[0][l] + ha[1] * gu[1][l] + ha[2] * gu[2][l];
            v[l].x = tm * rho * sgu;
            v[l].y = (l == 0 ? Nta : 0.0f) + tm * rho * ha[l] * u[0];
            v[l].z = (l == 1 ? Nta : 0.0f) + tm * rho * ha[l] * u[1];
            v[l].w = (l == 2 ? Nta : 0.0f) + tm * rho * ha[l] * u[2];
        }
        v[3].x = 0.0f;
        v[3].y = tm * ha[0];
        v[3].z = tm * ha[1];
        v[3].w = tm * ha[2];
        dpi -= sw * (Nta * div + tm * (ha[0] * Rm[0] + ha[1] * Rm[1] + ha[2] * Rm[2]));
    }
#pragma unroll
    for (int l = 0; l < 4; ++l) *(f32x4*)(dst + 4 * l) = v[l];
}

// Contributions of element layer Le (its records in the ring) to the rows of node layer
// Le (when hi) and node layer Le + 1 (when lo; rows in buffer (Le + 1) & 1), for the
// two nodes of this wave.  Software-pipelined over the eight pair groups: the operands
// of group g are read into registers, then the coefficient rows of group g + 1 are
// formed (vector units) while the products of group g run (matrix cores).
template <typename T>
__device__ __forceinline__ void ns_phase_b(const ColParams& p, ColShared<MF_FORM_NS_SUPG, T>& S, int Le, int zend,
                                           int i0, int j0, bool hi, bool lo)
{
    static_assert(sizeof(T) == 4, "the flow-form gather is FP32");
    constexpr int SE = HLayout<MF_FORM_NS_SUPG, T>::SE, SQ = HLayout<MF_FORM_NS_SUPG, T>::SQ;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    float* dt = S.dt[w];
    // coefficient lanes: (pair n, Gauss point q, row field i)
    const int cn = lane >> 5, cq = (lane >> 2) & 7, ci = lane & 3;
    float dph = 0.0f, dpl = 0.0f;
    // product lanes: block (pair n, row field i, b half), lane r in the block
    const int n = lane >> 5, ri = (lane >> 3) & 3, bh = (lane >> 2) & 1, r = lane & 3;
    const int b = 4 * bh + r;
    // groups: g < 4 -> node layer Le through the elements above it (eps = 4 + g),
    // g >= 4 -> node layer Le + 1 through the elements below it (eps = g - 4)
    const int g0 = hi ? 0 : 4, g1 = lo ? 8 : 4;
    auto coef = [&](int g) {
        const bool to_hi = g < 4;
        const int eps = to_hi ? 4 + g : g - 4;
        const NsPair pr = ns_pair(p, 2 * w + cn, eps, to_hi ? Le : Le + 1, zend, i0, j0);
        float* dst = dt + (cn * 8 + cq) * kNsTile + 16 * ci;
        if (pr.ok) {
            ns_coef_row(p, S.h + pr.el * SE + cq * SQ, pr.alpha, ci, dst, to_hi ? dph : dpl);
        } else {
#pragma unroll
            for (int l = 0; l < 4; ++l) *(f32x4*)(dst + 4 * l) = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    };
    if (g0 < g1) coef(g0);
#pragma unroll 1
    for (int g = g0; g < g1; ++g) {
        const bool to_hi = g < 4;
        const int eps = to_hi ? 4 + g : g - 4;
        const int Ln = to_hi ? Le : Le + 1;
        wave_lds_sync();  // the tiles of group g are written
        const NsPair pr = ns_pair(p, 2 * w + n, eps, Ln, zend, i0, j0);
        const float* At = dt + n * 8 * kNsTile + (4 * ri + r) * 4;
        const float* Bt = S.h + pr.el * SE + R_PHI + 4 * b;
        f32x4 A[8], B[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            A[q] = *(const f32x4*)(At + q * kNsTile);
            B[q] = *(const f32x4*)(Bt + q * SQ);
        }
        wave_lds_sync();  // every lane has its operands: the tiles may be rewritten
        if (g + 1 < g1) coef(g + 1);
        f32x4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            acc0 = __builtin_amdgcn_mfma_f32_4x4x1f32(A[q].x, B[q].x, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_4x4x1f32(A[q].y, B[q].y, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_4x4x1f32(A[q].z, B[q].z, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_4x4x1f32(A[q].w, B[q].w, acc1, 0, 0, 0);
        }
        if (pr.ok) {
            // lane holds K[(a, i), (b, l)] for l = 0..3: one 16-byte row-buffer update
            const int ax = pr.alpha & 1, ay = (pr.alpha >> 1) & 1, az = pr.alpha >> 2;
            const int nslot = ((b >> 2) - az + 1) * 9 + (((b >> 1) & 1) - ay + 1) * 3 + ((b & 1) - ax + 1);
            f32x4* dstk = (f32x4*)&S.rowK[Ln & 1][2 * w + n][(ri * 27 + nslot) * 4];
            *dstk = *dstk + acc0 + acc1;
        }
    }
    // d: sum the Gauss-point lanes of each (node, row field): lanes cn * 32 + 4 cq + ci
#pragma unroll
    for (int off = 4; off < 32; off <<= 1) {
        dph += __shfl_xor(dph, off, 64);
        dpl += __shfl_xor(dpl, off, 64);
    }
    if (cq == 0) {
        const int al = 2 * w + cn;
        if (hi) S.rowD[Le & 1][al][ci] += dph;
        if (lo) S.rowD[(Le + 1) & 1][al][ci] += dpl;
    }
}

// One column chunk of the flow form: element layer by element layer, each feeding the
// node layer below it and the one above it.
template <bool MASK, typename T>
__device__ __forceinline__ void column_body_ns(const ColParams& p, int b, ColShared<MF_FORM_NS_SUPG, T>& S)
{
    constexpr int FORM = MF_FORM_NS_SUPG;
    constexpr int NF = 4, NSRC = 4, NB = 16;
    using Sh = ColShared<FORM, T>;
    const int tid = threadIdx.x;
    const int NX = p.nx + 1, NY = p.ny + 1, NZ = p.nz + 1;
    const int ncx = (NX + CX - 1) / CX, ncy = (NY + CY - 1) / CY;
    const int cx = b % ncx, cy = (b / ncx) % ncy, ch = b / (ncx * ncy);
    const int i0 = cx * CX, j0 = cy * CY;
    const int z0 = ch * p.lz, z1 = min(z0 + p.lz, NZ);

    for (int k = tid; k < Sh::NRB * kColNodes * 27 * NB; k += kThreads) (&S.rowK[0][0][0])[k] = 0.0f;
    for (int k = tid; k < Sh::NRB * kColNodes * NF; k += kThreads) (&S.rowD[0][0][0])[k] = 0.0f;
    for (int it = tid; it < 3 * kTileNodes; it += kThreads) {
        NodeLoad<NSRC, NF, MASK, T> ld;
        const int L = z0 - 1 + it / kTileNodes, tn = it % kTileNodes;
        ld.load(p, L, tn, i0, j0);
        ld.template store<FORM>(S, L, tn);
    }
    __syncthreads();
    // element layer z0 - 1 feeds the first node layer of the chunk
    if (tid < kGeomThreads) {
        for (int it = tid; it < kGeomItems; it += kGeomThreads)
            geometry_item<FORM, T>(p, S, z0 - 1, it >> 3, it & 7, i0, j0);
    }
    __syncthreads();
    ns_phase_b<T>(p, S, z0 - 1, z1, i0, j0, false, true);
    __syncthreads();

    for (int kz = z0; kz < z1; ++kz) {
        // ---- phase A: records of element layer kz; rows of node layer kz - 1
        if (tid < kGeomThreads) {
            for (int it = tid; it < kGeomItems; it += kGeomThreads)
                geometry_item<FORM, T>(p, S, kz, it >> 3, it & 7, i0, j0);
        } else if (kz > z0) {
            write_layer<FORM, MASK, T>(p, S, kz - 1, tid - kGeomThreads, kThreads - kGeomThreads, (kz - 1) & 1);
        }
        __syncthreads();

        // ---- phase B: element layer kz into node layers kz and kz + 1; prefetch
        NodeLoad<NSRC, NF, MASK, T> ld;
        ld.ok = false;
        int info[4] = {-1, 0, 0, 0};
        if (tid < kTileNodes) {
            ld.load(p, kz + 2, tid, i0, j0);
        } else if (tid >= kPfInfoT0 && tid < kPfInfoT0 + kColNodes) {
            const int il = tid - kPfInfoT0;
            const int gi = i0 + il % CX, gj = j0 + il / CX;
            if (gi < NX && gj < NY) {
                const int node = gi + NX * (gj + NY * kz);
                const int mx = 1 + (gi > 0) + (gi < p.nx), my = 1 + (gj > 0) + (gj < p.ny),
                          mz = 1 + (kz > 0) + (kz < p.nz);
                info[0] = node;
                info[1] = p.nbr_ptr[node];
                info[2] = mx * my * mz;
                info[3] = (gi > 0) | ((gi < p.nx) << 1) | ((gj > 0) << 2) | ((gj < p.ny) << 3) | ((kz > 0) << 4) |
                          ((kz < p.nz) << 5);
            }
        }
        ns_phase_b<T>(p, S, kz, z1, i0, j0, true, kz + 1 < z1);
        if (tid < kTileNodes) ld.template store<FORM>(S, kz + 2, tid);
        if (tid >= kPfInfoT0 && tid < kPfInfoT0 + kColNodes) {
#pragma unroll
            for (int k = 0; k < 4; ++k) S.ni[tid - kPfInfoT0][k] = info[k];
        }
        __syncthreads();
    }
    if (z0 < z1) write_layer<FORM, MASK, T>(p, S, z1 - 1, tid, kThreads, (z1 - 1) & 1);
}

// MASK: the problem has Dirichlet flags (the unmasked instantiation carries none of their
// loads or registers)
template <int FORM, bool MASK, typename T>
__global__ void __launch_bounds__(kThreads, (MinBlocks<FORM, T>::value)) k_assemble_column(ColParams p)
{
    __shared__ ColShared<FORM, T> S;
    if constexpr (FORM == MF_FORM_NS_SUPG) {
        column_body_ns<MASK, T>(p, blockIdx.x, S);
    } else if constexpr (sizeof(T) == 8) {
        // workgroups are dealt to the eight XCDs in turn; give each XCD a run of
        // consecutive columns, so that the halo nodes neighbouring columns share are read
        // into one L2 (a bijection of [0, gridDim.x); the FP32 forms measured slower with it)
        const int nb = (int)gridDim.x, full = nb / 8, rem = nb % 8;
        const int x = (int)blockIdx.x % 8, k = (int)blockIdx.x / 8;
        column_body<FORM, MASK, T>(p, x * full + min(x, rem) + k, S);
    } else {
        column_body<FORM, MASK, T>(p, blockIdx.x, S);
    }
}

// ------------------------------------------------------------------------------------
// Batched persistent launch: many structured problems in one kernel.  Work items are
// (problem, column) pairs in an order chosen on the host; each workgroup pops the next
// item from a device counter until the list is exhausted (every wave reaches the exit).
// ------------------------------------------------------------------------------------
struct BatchProblemDev {
    ColParams cp;
    int kind;
};

template <typename T, bool ELAST>
union BatchShared;
template <typename T>
union BatchShared<T, true> {
    ColShared<MF_FORM_ELASTICITY, T> elasticity;
};
template <typename T>
union BatchShared<T, false> {
    ColShared<MF_FORM_MASS, T> mass;
    ColShared<MF_FORM_POISSON, T> poisson;
};

__global__ void k_batch_reset(int* counter, unsigned long long* const* status, int n_status)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 2) counter[i] = 0;
    if (i < n_status) {
        status[i][0] = ~0ull;
        status[i][1] = ~0ull;
        status[i][2] = ~0ull;
    }
}

// MASK: some problem of the batch has Dirichlet flags; ELAST: the elasticity items (one
// kernel), else the mass and Poisson items (another), so that each kernel's registers are
// those of its own forms
template <typename T, bool MASK, bool ELAST>
__global__ void __launch_bounds__(kThreads, (BatchMinBlocks<T>::value))
    k_batch_persistent(const BatchProblemDev* __restrict__ probs, const int2* __restrict__ items, int n_items,
                       int* __restrict__ counter)
{
    __shared__ BatchShared<T, ELAST> S;
    __shared__ int sItem;
    while (true) {
        __syncthreads();  // the previous item's write-out is done with the LDS
        if (threadIdx.x == 0) sItem = atomicAdd(counter, 1);
        __syncthreads();
        const int it = sItem;
        if (it >= n_items) break;
        const int2 w = items[it];
        const ColParams cp = probs[w.x].cp;
        if constexpr (ELAST) {
            if (cp.xw == 2)
                column_body<MF_FORM_ELASTICITY, MASK, T, 2>(cp, w.y, S.elasticity);
            else
                column_body<MF_FORM_ELASTICITY, MASK, T, 4>(cp, w.y, S.elasticity);
        } else {
            const int kind = probs[w.x].kind;
            if (cp.xw == 2) {
                if (kind == MF_FORM_POISSON)
                    column_body<MF_FORM_POISSON, MASK, T, 2>(cp, w.y, S.poisson);
                else
                    column_body<MF_FORM_MASS, MASK, T, 2>(cp, w.y, S.mass);
            } else {
                if (kind == MF_FORM_POISSON)
                    column_body<MF_FORM_POISSON, MASK, T, 4>(cp, w.y, S.poisson);
                else
                    column_body<MF_FORM_MASS, MASK, T, 4>(cp, w.y, S.mass);
            }
        }
    }
}

int device_cus()
{
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cached[dev] = n;
    }
    return cached[dev];
}

// Node layers per workgroup: minimise (rounds of workgroups over the CUs) x (layers per
// workgroup + the one extra element layer each workgroup computes first).
int choose_lz(int64_t columns, int NZ, int cus)
{
    int best = NZ;
    double best_cost = 1e300;
    for (int n_ch = 1; n_ch <= NZ; ++n_ch) {
        const int lz = (NZ + n_ch - 1) / n_ch;
        const int64_t wgs = columns * ((NZ + lz - 1) / lz);
        const double rounds = (double)((wgs + cus - 1) / cus);
        const double cost = rounds * (lz + 1);
        if (cost < best_cost) {
            best_cost = cost;
            best = lz;
        }
    }
    return best;
}

ColParams make_params(const AssembleArgs& A)
{
    const mf_pattern_s* P = A.P;
    ColParams p{};
    p.form = *A.form;
    p.nx = (int)P->gx;
    p.ny = (int)P->gy;
    p.nz = (int)P->gz;
    p.n_nodes = (int)P->n_nodes;
    p.coords = A.coords;
    p.nbr_ptr = P->nbr_ptr;
    p.elem_param = A.elem_param;
    p.src = A.form->kind == MF_FORM_NS_SUPG ? A.lin_state : A.nodal_src;
    p.dirichlet = A.dirichlet;
    p.field_major = P->numbering == MF_FIELD_MAJOR;
    p.n_pairs = (int)P->n_pairs;
    p.K = A.K;
    p.d = A.d;
    p.status = P->status;
    p.lz = p.nz + 1;
    p.xw = CX;
    const double nu = A.form->nu;
    p.lam_f = nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    p.mu_f = 1.0 / (2.0 * (1.0 + nu));
    return p;
}

int64_t column_count(const mf_pattern_s* P, int xw = CX)
{
    const int cy = kColNodes / xw;
    return (int64_t)((P->gx + 1 + xw - 1) / xw) * ((P->gy + 1 + cy - 1) / cy);
}

template <int FORM, typename T>
mf_status launch_column(const AssembleArgs& A)
{
    ColParams p = make_params(A);
    const int NZ = p.nz + 1;
    const int64_t columns = column_count(A.P);
    p.lz = choose_lz(columns, NZ, device_cus() * MinBlocks<FORM, T>::value);
    const int64_t wgs = columns * ((NZ + p.lz - 1) / p.lz);
    if (wgs <= 0) return MF_OK;
    if (wgs > 0x7fffffff) return set_error(MF_ERR_OVERFLOW, "grid of %lld workgroups", (long long)wgs);
    if (p.dirichlet)
        k_assemble_column<FORM, true, T><<<(unsigned)wgs, kThreads, 0, A.stream>>>(p);
    else
        k_assemble_column<FORM, false, T><<<(unsigned)wgs, kThreads, 0, A.stream>>>(p);
    MF_HIP(hipGetLastError());
    return MF_OK;
}

template <typename T>
mf_status dispatch(const AssembleArgs& A)
{
    switch (A.form->kind) {
        case MF_FORM_MASS: return launch_column<MF_FORM_MASS, T>(A);
        case MF_FORM_POISSON: return launch_column<MF_FORM_POISSON, T>(A);
        case MF_FORM_ELASTICITY: return launch_column<MF_FORM_ELASTICITY, T>(A);
        case MF_FORM_NS_SUPG:
            if constexpr (sizeof(T) == 4) return launch_column<MF_FORM_NS_SUPG, T>(A);
            return MF_ERR_UNSUPPORTED;
        default: return MF_ERR_UNSUPPORTED;
    }
}

}  // namespace

// ---------------- batched launch: host side ----------------
// A work item is one tile of a problem: a node column of the cross-section, cut along z
// into a number of chunks (the tile height) that the autotuner chooses per (form, size)
// class of problems.

int64_t batch_units_of(const mf_pattern_s* P, int chunks, int xw)
{
    const int NZ = (int)P->gz + 1;
    const int c = std::max(1, std::min(chunks, NZ));
    const int lz = (NZ + c - 1) / c;
    return column_count(P, xw) * ((NZ + lz - 1) / lz);
}

mf_status batch_check(const AssembleArgs& A)
{
    const mf_pattern_s* P = A.P;
    if (!P->is_grid || P->dim != 3 || !P->full_coupling || P->n_elems == 0)
        return set_error(MF_ERR_UNSUPPORTED, "batched problems must be non-empty structured 3D grids with full coupling");
    if (A.form->kind == MF_FORM_NS_SUPG) return set_error(MF_ERR_UNSUPPORTED, "batched launch covers mass, Poisson and elasticity");
    if (P->n_nodes >= 0x7fffffff) return set_error(MF_ERR_OVERFLOW, "problem too large for the batched launch");
    return MF_OK;
}

mf_status batch_upload(const std::vector<AssembleArgs>& probs, const std::vector<int>& chunks,
                       const std::vector<int>& xw, void** dev_probs, void** dev_status)
{
    std::vector<BatchProblemDev> h(probs.size());
    std::vector<unsigned long long*> st(probs.size());
    for (size_t k = 0; k < probs.size(); ++k) {
        h[k].cp = make_params(probs[k]);
        // tile height: the column of NZ node layers in `chunks` work items
        const int NZ = h[k].cp.nz + 1;
        const int c = std::max(1, std::min(chunks[k], NZ));
        h[k].cp.lz = (NZ + c - 1) / c;
        h[k].cp.xw = xw[k] == 2 ? 2 : 4;
        h[k].kind = probs[k].form->kind;
        st[k] = probs[k].P->status;
    }
    if (!*dev_probs) MF_HIP(hipMalloc(dev_probs, sizeof(BatchProblemDev) * (h.size() > 0 ? h.size() : 1)));
    MF_HIP(hipMemcpy(*dev_probs, h.data(), sizeof(BatchProblemDev) * h.size(), hipMemcpyHostToDevice));
    if (!*dev_status) MF_HIP(hipMalloc(dev_status, sizeof(void*) * (st.size() > 0 ? st.size() : 1)));
    MF_HIP(hipMemcpy(*dev_status, st.data(), sizeof(void*) * st.size(), hipMemcpyHostToDevice));
    return MF_OK;
}

template <typename T, bool MASK>
void launch_batch_group(bool elast, const BatchProblemDev* pr, const int2* it, int n, int* ctr, int n_wg,
                        hipStream_t s)
{
    if (elast)
        k_batch_persistent<T, MASK, true><<<n_wg, kThreads, 0, s>>>(pr, it, n, ctr);
    else
        k_batch_persistent<T, MASK, false><<<n_wg, kThreads, 0, s>>>(pr, it, n, ctr);
}

mf_status batch_launch(const void* dev_probs, void* dev_status, int n_probs, const int2* items, int n_first,
                       int n_items, bool first_elastic, int* counter, int n_wg, mf_precision prec, bool masked,
                       hipStream_t s)
{
    k_batch_reset<<<(n_probs + 255) / 256 > 0 ? (n_probs + 255) / 256 : 1, 256, 0, s>>>(
        counter, (unsigned long long* const*)dev_status, n_probs);
    const BatchProblemDev* pr = (const BatchProblemDev*)dev_probs;
    // items [0, n_first) of one group (elasticity when first_elastic), then the other's
    for (int g = 0; g < 2; ++g) {
        const int2* it = items + (g == 0 ? 0 : n_first);
        const int n = g == 0 ? n_first : n_items - n_first;
        if (n <= 0) continue;
        const bool elast = (g == 0) == first_elastic;
        if (prec == MF_F64) {
            if (masked)
                launch_batch_group<double, true>(elast, pr, it, n, counter + g, n_wg, s);
            else
                launch_batch_group<double, false>(elast, pr, it, n, counter + g, n_wg, s);
        } else {
            if (masked)
                launch_batch_group<float, true>(elast, pr, it, n, counter + g, n_wg, s);
            else
                launch_batch_group<float, false>(elast, pr, it, n, counter + g, n_wg, s);
        }
    }
    MF_HIP(hipGetLastError());
    return MF_OK;
}

int batch_max_wg_per_cu(mf_precision prec) { return prec == MF_F64 ? BatchMinBlocks<double>::value : BatchMinBlocks<float>::value; }

// Returns MF_ERR_UNSUPPORTED (without launching) when the case is not covered:
// unstructured meshes, 2D, partial coupling, or the flow form in FP64.
mf_status assemble_column(const AssembleArgs& A)
{
    const mf_pattern_s* P = A.P;
    if (!P->is_grid || P->dim != 3 || !P->full_coupling) return MF_ERR_UNSUPPORTED;
    if (P->n_elems == 0) return MF_ERR_UNSUPPORTED;
    return A.prec == MF_F64 ? dispatch<double>(A) : dispatch<float>(A);
}

}  // namespace mf
