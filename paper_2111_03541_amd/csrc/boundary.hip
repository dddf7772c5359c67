// Boundary forms: the physics one dimension lower (Sec. 2.2 opening of the algorithm),
// integrated over element faces and added into an assembled K and d.  The forms are the
// ones of Sec. 4.1 (convection, radiation, penalty fix with its flux term), Sec. 4.2
// (load traction, penalty fix) and Sec. 4.3 (flow inflow, outflow and fix), with the sign
// reading of the domain forms: R = -d_paper for the thermal and elastic physics,
// R = +d_paper for the flow, K = dR/dU, exported d = -R(U).
//
// 8-node hexahedra (all forms): one thread per (element, element node a, field i), one
// launch per element colour.  The faces are first marked per element (a bit per listed
// local face and its count); a thread of an element with listed faces loops over them,
// integrates the 2x2 Gauss rule of each face (xi_axis = -1 or +1) with the element's
// trilinear map in FP64 (surface measure |t_u x t_v|, outward unit normal, and for the
// flux term the volume gradients J^-T grad_xi N_b), and accumulates row (a, i) of the
// face tangent and residual.  The row nodes of a face are its four nodes, or every node
// of the element for the flow forms, whose inflow and fix terms carry the test gradient.
// Elements of one colour share no node, so each row is added by a single thread of the
// launch with plain stores through the element-to-nonzero rank map, and the colours run
// in stream order: the sums are the same on every run, with no host synchronisation.
//
// 20-node hexahedra, 10-node tetrahedra and quadrilateral edges: one thread per (face,
// row node, field), atomics through the rank map, with the faces in buckets keyed by
// (colour of the face's element, local face), one launch per bucket in key order.
// Within a bucket every value of K and d receives contributions of one face only (or of
// identical copies of it, when a face is listed twice): again run-to-run identical sums;
// the call synchronises once to size the buckets.
//
// A face whose element id or local face is out of range is skipped and its index
// recorded in the pattern's second status word.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "element.h"
#include "mf_internal.h"
#include "serendipity.h"

namespace mf {
namespace {

constexpr int kThreads = 256;

struct BParams {
    mf_bform form;
    int64_t n_el, n_nodes, n_faces;
    const int32_t* conn;
    const double* coords;
    const int32_t* row_ptr;
    const int32_t* nbr_ptr;
    const uint8_t* rank;
    const int32_t* face_elem;
    const uint8_t* face_id;
    const void* state;   // [nf][n_nodes] or null (zero)
    const void* target;  // [nf][n_nodes] or null (the constant form->value)
    int field_major;
    void* K;
    void* d;
    unsigned long long* status;
    // faces of this launch: order[f_begin + k] for k < n_faces (one colour bucket)
    const int32_t* order;
    int64_t f_begin;
    // 8-node hexahedra: per element, the listed local faces (bit fid) and their counts
    const uint32_t* face_mask;  // [n_el]
    const uint32_t* face_cnt;   // [n_el][6]
};

__device__ __forceinline__ int64_t face_of(const BParams& p, int64_t k) { return p.order[p.f_begin + k]; }

__device__ __forceinline__ double lin1(int s, double xi) { return 0.5 * (1.0 + (s ? xi : -xi)); }

// (J^-1)[n][m] = dxi_n / dx_m by cofactors; false when det J <= 0
__device__ __forceinline__ bool inverse_jacobian(const double (&J)[3][3], double (&Ji)[3][3])
{
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    if (!(det > 0.0)) return false;
    const double r = 1.0 / det;
    Ji[0][0] = c00 * r;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
    Ji[1][0] = c01 * r;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
    Ji[2][0] = c02 * r;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
    return true;
}

// row nodes per face: the flow forms (four fields) take every node of the element
// Row (a, i) of element e over the listed faces of e (local faces in `fmask`, each
// counted cnt[6 e + fid] times), for 8-node hexahedra.  FI >= 0 fixes the field at compile
// time (the flow forms, so that every per-field array index is static); FI < 0 takes the
// runtime field fi, and then only field fi of the state and target and the (a, fi) x
// (b, fi) block are held.  The caller runs one element colour per launch: no other
// thread of the launch touches row a, so the row is added with plain stores.
template <int NF, int FI, typename T>
__device__ __forceinline__ void boundary_row(const BParams& p, int64_t e, uint32_t fmask, int a, int fi)
{
    const int i = FI >= 0 ? FI : fi;

    // fields of the state and target held: all four for the flow forms, else the
    // thread's own field i (slot li)
    constexpr int NL = NF == 4 ? 4 : 1;
    const int li = NL == 1 ? 0 : i;
    int32_t node[8];
    double x[8][3];
    double U[8][NL], G[8][NL];
    const T* st = (const T*)p.state;
    const T* tg = (const T*)p.target;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        node[b] = p.conn[(int64_t)b * p.n_el + e];
#pragma unroll
        for (int m = 0; m < 3; ++m) x[b][m] = p.coords[(int64_t)m * p.n_nodes + node[b]];
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const int j = NL == 1 ? i : l;
            U[b][l] = st ? (double)st[(int64_t)j * p.n_nodes + node[b]] : 0.0;
            G[b][l] = tg ? (double)tg[(int64_t)j * p.n_nodes + node[b]] : p.form.value[j];
        }
    }
    const mf_bform_kind kind = p.form.kind;
    const double c = p.form.coef;
    constexpr int KC = NL;  // columns held per node: all fields, or field i alone (slot li)
    double krow[8][KC];
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
        for (int j = 0; j < KC; ++j) krow[b][j] = 0.0;
    double rrow = 0.0;

    for (int fid = 0; fid < 6; ++fid) {
    if (!((fmask >> fid) & 1)) continue;
    const int axis = fid >> 1, side = fid & 1;
    // the row nodes of a face are its four nodes (every node of the element for the
    // flow forms, whose terms carry the test gradient)
    if (NF != 4 && ((a >> axis) & 1) != side) continue;
    const double mult = (double)p.face_cnt[6 * e + fid];
    const int u = (axis + 1) % 3, v = (axis + 2) % 3;
    for (int q = 0; q < 4; ++q) {
        double xi[3];
        xi[axis] = side ? 1.0 : -1.0;
        xi[u] = (q & 1) ? kGaussPt : -kGaussPt;
        xi[v] = (q >> 1) ? kGaussPt : -kGaussPt;
        double N[8], dN[8][3];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
            const double Fx = lin1(bx, xi[0]), Fy = lin1(by, xi[1]), Fz = lin1(bz, xi[2]);
            N[b] = Fx * Fy * Fz;
            dN[b][0] = (bx ? 0.5 : -0.5) * Fy * Fz;
            dN[b][1] = (by ? 0.5 : -0.5) * Fx * Fz;
            dN[b][2] = (bz ? 0.5 : -0.5) * Fx * Fy;
        }
        double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // J[m][n] = dx_m / dxi_n
#pragma unroll
        for (int b = 0; b < 8; ++b)
#pragma unroll
            for (int m = 0; m < 3; ++m)
#pragma unroll
                for (int n = 0; n < 3; ++n) J[m][n] = fma(x[b][m], dN[b][n], J[m][n]);
        const double tu[3] = {J[0][u], J[1][u], J[2][u]}, tv[3] = {J[0][v], J[1][v], J[2][v]};
        const double sg = side ? 1.0 : -1.0;
        double nr[3] = {sg * (tu[1] * tv[2] - tu[2] * tv[1]), sg * (tu[2] * tv[0] - tu[0] * tv[2]),
                        sg * (tu[0] * tv[1] - tu[1] * tv[0])};
        const double dS = sqrt(nr[0] * nr[0] + nr[1] * nr[1] + nr[2] * nr[2]);
        if (!(dS > 0.0)) {
            atomicMin(p.status, (unsigned long long)e);
            return;
        }
        const double nv[3] = {nr[0] / dS, nr[1] / dS, nr[2] / dS};
        const double w = mult * dS;  // unit Gauss weights on [-1, 1]^2, times the face's count
        const double Na = N[a];
        double uq[NL], gq[NL];
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            uq[j] = 0.0;
            gq[j] = 0.0;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                uq[j] = fma(N[b], U[b][j], uq[j]);
                gq[j] = fma(N[b], G[b][j], gq[j]);
            }
        }
        if constexpr (NF == 4) {
            // flow forms (value: u^w [0..3), rho [3], mu [4]; coef = tau^b)
            double Ji[3][3];
            if (!inverse_jacobian(J, Ji)) {
                atomicMin(p.status, (unsigned long long)e);
                return;
            }
            double gn[8];  // n . grad N_b
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                gn[b] = 0.0;
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    gn[b] += nv[m] * (Ji[0][m] * dN[b][0] + Ji[1][m] * dN[b][1] + Ji[2][m] * dN[b][2]);
            }
            const double rho = p.form.value[3], mu = p.form.value[4], tau = c;
            const bool wall = kind != MF_BFORM_NS_OUTFLOW;
            double uw[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) uw[m] = kind == MF_BFORM_NS_INFLOW ? gq[m] : 0.0;
            const double un = uq[0] * nv[0] + uq[1] * nv[1] + uq[2] * nv[2];
            if (i < 3) {
                // base: p n_i - mu u_i,j n_j
                double gu = 0.0;
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    gu = fma(gn[b], U[b][i], gu);
                    krow[b][3] += w * Na * nv[i] * N[b];
                    krow[b][i] -= w * mu * Na * gn[b];
                }
                rrow += w * Na * (uq[3] * nv[i] - mu * gu);
                if (wall) {
                    const double uwn = uw[0] * nv[0] + uw[1] * nv[1] + uw[2] * nv[2];
                    rrow += w * (rho * Na * uw[i] * uwn + mu * gn[a] * (uw[i] - uq[i]) +
                                 tau * rho * Na * (uq[i] - uw[i]));
#pragma unroll
                    for (int b = 0; b < 8; ++b) krow[b][i] += w * (tau * rho * Na - mu * gn[a]) * N[b];
                } else {
                    rrow += w * rho * Na * uq[i] * un;
#pragma unroll
                    for (int b = 0; b < 8; ++b)
#pragma unroll
                        for (int k = 0; k < 3; ++k)
                            krow[b][k] += w * rho * Na * N[b] * ((k == i ? un : 0.0) + uq[i] * nv[k]);
                }
            } else if (wall) {
                rrow += w * Na * ((uw[0] - uq[0]) * nv[0] + (uw[1] - uq[1]) * nv[1] + (uw[2] - uq[2]) * nv[2]);
#pragma unroll
                for (int b = 0; b < 8; ++b)
#pragma unroll
                    for (int k = 0; k < 3; ++k) krow[b][k] -= w * Na * N[b] * nv[k];
            }
        } else if (kind == MF_BFORM_PENALTY || kind == MF_BFORM_CONVECTION) {
            // R = int c N_a (u_i - g_i)
#pragma unroll
            for (int b = 0; b < 8; ++b) krow[b][li] += c * w * Na * N[b];
            rrow += c * w * Na * (uq[li] - gq[li]);
        } else if (kind == MF_BFORM_RADIATION) {
            // R = int c N_a (T^4 - T_env^4), c = e_m sigma
            const double T1 = uq[0], Te = gq[0];
#pragma unroll
            for (int b = 0; b < 8; ++b) krow[b][li] += c * w * Na * 4.0 * T1 * T1 * T1 * N[b];
            rrow += c * w * Na * (T1 * T1 * T1 * T1 - Te * Te * Te * Te);
        } else if (kind == MF_BFORM_TRACTION) {
            // R = -int N_a t_i, t = sigma^l n or the interpolated nodal traction
            const double* S = p.form.value;
            const double ti = tg ? gq[li] : S[3 * i] * nv[0] + S[3 * i + 1] * nv[1] + S[3 * i + 2] * nv[2];
            rrow -= w * Na * ti;
        } else {  // MF_BFORM_FLUX: R = -int c N_a n . grad T
            double Ji[3][3];
            if (!inverse_jacobian(J, Ji)) {
                atomicMin(p.status, (unsigned long long)e);
                return;
            }
            double ngT = 0.0;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                double ng = 0.0;  // n . grad N_b,  grad N_b = J^-T grad_xi N_b
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    ng += nv[m] * (Ji[0][m] * dN[b][0] + Ji[1][m] * dN[b][1] + Ji[2][m] * dN[b][2]);
                krow[b][li] -= c * w * Na * ng;
                ngT = fma(ng, U[b][li], ngT);
            }
            rrow -= c * w * Na * ngT;
        }
    }
    }

    const int64_t va = node[a];
    const int64_t row = p.field_major ? (int64_t)i * p.n_nodes + va : (int64_t)NF * va + i;
    const int64_t rs = p.row_ptr[row];
    const int64_t deg = p.nbr_ptr[va + 1] - p.nbr_ptr[va];
    T* K = (T*)p.K;
    T* d = (T*)p.d;
    // nonzero entries only; every old value is loaded before the first store, so the
    // thread's read-modify-writes overlap instead of running one after another
    int rk[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        bool any = false;
#pragma unroll
        for (int l = 0; l < KC; ++l) any = any || krow[b][l] != 0.0;
        rk[b] = any ? (int)p.rank[(int64_t)(a * 8 + b) * p.n_el + e] : 0;
    }
    auto pos_of = [&](int b, int l) -> int64_t {
        const int j = KC == 1 ? i : l;
        return p.field_major ? rs + j * deg + rk[b] : rs + (int64_t)rk[b] * NF + j;
    };
    T old[8][KC];
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
        for (int l = 0; l < KC; ++l) old[b][l] = krow[b][l] != 0.0 ? K[pos_of(b, l)] : T(0);
    const T dold = rrow != 0.0 ? d[row] : T(0);
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
        for (int l = 0; l < KC; ++l)
            if (krow[b][l] != 0.0) K[pos_of(b, l)] = old[b][l] + (T)krow[b][l];
    if (rrow != 0.0) d[row] = dold + (T)(-rrow);
}

// Items (element with listed faces of the colour, element node a, field i), strided over
// the grid; the colour's element list and its length come from k_face_mark.
template <int NF, typename T>
__global__ void __launch_bounds__(kThreads) k_boundary(BParams p, const int32_t* __restrict__ elems,
                                                       const uint32_t* __restrict__ n_el_c)
{
    const int64_t nc = *n_el_c;
    const int64_t n = nc * 8 * NF;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = elems[t % nc];
        const uint32_t fmask = p.face_mask[e];
        const int ki = (int)(t / nc);
        const int a = ki / NF, i = ki % NF;
        if constexpr (NF == 4) {
            switch (i) {
                case 0: boundary_row<NF, 0, T>(p, e, fmask, a, i); break;
                case 1: boundary_row<NF, 1, T>(p, e, fmask, a, i); break;
                case 2: boundary_row<NF, 2, T>(p, e, fmask, a, i); break;
                default: boundary_row<NF, 3, T>(p, e, fmask, a, i); break;
            }
        } else {
            boundary_row<NF, -1, T>(p, e, fmask, a, i);
        }
    }
}

// Faces of 20-node hexahedra: one thread per (face f, face node k, field i), with the
// eight nodes of the face (the other twelve basis functions vanish on it, with their
// tangential derivatives) and the 3x3 Gauss rule of the face; penalty, convection,
// radiation and traction as above.
template <int NF, typename T>
__global__ void __launch_bounds__(kThreads) k_boundary20(BParams p)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p.n_faces * 8 * NF) return;
    const int64_t f = face_of(p, t % p.n_faces);
    const int ki = (int)(t / p.n_faces);
    const int kf = ki / NF, i = ki % NF;
    const int64_t e = p.face_elem[f];
    const int fid = p.face_id[f];
    if (e < 0 || e >= p.n_el || fid > 5) {
        if (ki == 0) atomicMin(p.status + 1, (unsigned long long)f);
        return;
    }
    const int axis = fid >> 1, side = fid & 1;
    const int u = (axis + 1) % 3, v = (axis + 2) % 3;
    int loc[8];  // local ids of the face nodes, ascending
    for (int a = 0, k = 0; a < 20; ++a)
        if (on_face20(a, axis, side)) loc[k++] = a;
    double x[8][3], U[8], G[8];  // coordinates, and field i of the state and target
    int32_t node[8];
    const T* st = (const T*)p.state;
    const T* tg = (const T*)p.target;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        node[b] = p.conn[(int64_t)loc[b] * p.n_el + e];
#pragma unroll
        for (int m = 0; m < 3; ++m) x[b][m] = p.coords[(int64_t)m * p.n_nodes + node[b]];
        U[b] = st ? (double)st[(int64_t)i * p.n_nodes + node[b]] : 0.0;
        G[b] = tg ? (double)tg[(int64_t)i * p.n_nodes + node[b]] : p.form.value[i];
    }
    const mf_bform_kind kind = p.form.kind;
    const double c = p.form.coef;
    double krow[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) krow[b] = 0.0;
    double rrow = 0.0;
    const double gp = 0.7745966692414834;  // sqrt(3/5)
    for (int q = 0; q < 9; ++q) {
        const int qu = q % 3, qv = q / 3;
        double xi[3];
        xi[axis] = side ? 1.0 : -1.0;
        xi[u] = (qu - 1) * gp;
        xi[v] = (qv - 1) * gp;
        const double wq = (qu == 1 ? 8.0 : 5.0) * (qv == 1 ? 8.0 : 5.0) / 81.0;
        double N[8], tu[3] = {0, 0, 0}, tv[3] = {0, 0, 0};
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            double dN[3];
            shape20(loc[b], xi, N[b], dN);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                tu[m] = fma(x[b][m], dN[u], tu[m]);
                tv[m] = fma(x[b][m], dN[v], tv[m]);
            }
        }
        const double sg = side ? 1.0 : -1.0;
        const double nr[3] = {sg * (tu[1] * tv[2] - tu[2] * tv[1]), sg * (tu[2] * tv[0] - tu[0] * tv[2]),
                              sg * (tu[0] * tv[1] - tu[1] * tv[0])};
        const double dS = sqrt(nr[0] * nr[0] + nr[1] * nr[1] + nr[2] * nr[2]);
        if (!(dS > 0.0)) {
            atomicMin(p.status, (unsigned long long)e);
            return;
        }
        const double w = wq * dS;
        const double Na = N[kf];
        double uq = 0.0, gq = 0.0;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uq = fma(N[b], U[b], uq);
            gq = fma(N[b], G[b], gq);
        }
        if (kind == MF_BFORM_PENALTY || kind == MF_BFORM_CONVECTION) {
#pragma unroll
            for (int b = 0; b < 8; ++b) krow[b] += c * w * Na * N[b];
            rrow += c * w * Na * (uq - gq);
        } else if (kind == MF_BFORM_RADIATION) {
#pragma unroll
            for (int b = 0; b < 8; ++b) krow[b] += c * w * Na * 4.0 * uq * uq * uq * N[b];
            rrow += c * w * Na * (uq * uq * uq * uq - gq * gq * gq * gq);
        } else {  // MF_BFORM_TRACTION
            const double* S = p.form.value;
            const double ti = tg ? gq : (S[3 * i] * nr[0] + S[3 * i + 1] * nr[1] + S[3 * i + 2] * nr[2]) / dS;
            rrow -= w * Na * ti;
        }
    }
    const int a = loc[kf];
    const int64_t va = node[kf];
    const int64_t row = p.field_major ? (int64_t)i * p.n_nodes + va : (int64_t)NF * va + i;
    const int64_t rs = p.row_ptr[row];
    const int64_t deg = p.nbr_ptr[va + 1] - p.nbr_ptr[va];
    T* K = (T*)p.K;
    T* d = (T*)p.d;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        if (krow[b] == 0.0) continue;
        const int64_t rk = p.rank[(int64_t)(a * 20 + loc[b]) * p.n_el + e];
        const int64_t pos = p.field_major ? rs + i * deg + rk : rs + rk * NF + i;
        unsafeAtomicAdd(K + pos, (T)krow[b]);
    }
    if (rrow != 0.0) unsafeAtomicAdd(d + row, (T)(-rrow));
}

// Faces of 10-node tetrahedra: one thread per (face f, face node m, field i).  Face k is
// the face opposite vertex k: its three vertices and the three edge midpoints among them.
// The face is the reference triangle p0 + s (p1 - p0) + t (p2 - p0) over its vertices,
// integrated with the collapsed 4 x 4 Gauss rule of the triangle; the normal points away
// from vertex k.  Penalty, convection, radiation and traction as above.
template <int NF, typename T>
__global__ void __launch_bounds__(kThreads) k_boundary_tet10(BParams p)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p.n_faces * 6 * NF) return;
    const int64_t f = face_of(p, t % p.n_faces);
    const int ki = (int)(t / p.n_faces);
    const int mf = ki / NF, i = ki % NF;
    const int64_t e = p.face_elem[f];
    const int k = p.face_id[f];
    if (e < 0 || e >= p.n_el || k > 3) {
        if (ki == 0) atomicMin(p.status + 1, (unsigned long long)f);
        return;
    }
    // face nodes: the vertices other than k, then the edges among them (local ids 4..9 are
    // the edges (0,1), (1,2), (2,0), (0,3), (1,3), (2,3))
    constexpr int EI[6] = {0, 1, 2, 0, 1, 2}, EJ[6] = {1, 2, 0, 3, 3, 3};
    int loc[6];
    for (int v = 0, c = 0; v < 4; ++v)
        if (v != k) loc[c++] = v;
    for (int m = 0, c = 3; m < 6; ++m)
        if (EI[m] != k && EJ[m] != k) loc[c++] = 4 + m;
    double pv[3][3];  // reference coordinates of the face vertices
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int m = 0; m < 3; ++m) pv[c][m] = loc[c] == m + 1 ? 1.0 : 0.0;
    double x[6][3], U[6], G[6], xk[3];
    int32_t node[6];
    const T* st = (const T*)p.state;
    const T* tg = (const T*)p.target;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
        node[b] = p.conn[(int64_t)loc[b] * p.n_el + e];
#pragma unroll
        for (int m = 0; m < 3; ++m) x[b][m] = p.coords[(int64_t)m * p.n_nodes + node[b]];
        U[b] = st ? (double)st[(int64_t)i * p.n_nodes + node[b]] : 0.0;
        G[b] = tg ? (double)tg[(int64_t)i * p.n_nodes + node[b]] : p.form.value[i];
    }
    {
        const int32_t vk = p.conn[(int64_t)k * p.n_el + e];
#pragma unroll
        for (int m = 0; m < 3; ++m) xk[m] = p.coords[(int64_t)m * p.n_nodes + vk];
    }
    const mf_bform_kind kind = p.form.kind;
    const double c = p.form.coef;
    double krow[6];
#pragma unroll
    for (int b = 0; b < 6; ++b) krow[b] = 0.0;
    double rrow = 0.0;
    const double g4[4] = {0.5 * (1.0 - 0.8611363115940526), 0.5 * (1.0 - 0.3399810435848563),
                          0.5 * (1.0 + 0.3399810435848563), 0.5 * (1.0 + 0.8611363115940526)};
    const double w4[4] = {0.5 * 0.3478548451374538, 0.5 * 0.6521451548625461, 0.5 * 0.6521451548625461,
                          0.5 * 0.3478548451374538};
    for (int q = 0; q < 16; ++q) {
        const double s_ = g4[q & 3], t_ = g4[q >> 2] * (1.0 - s_);
        const double wq = w4[q & 3] * w4[q >> 2] * (1.0 - s_);
        double xi[3], e1[3], e2[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            e1[m] = pv[1][m] - pv[0][m];
            e2[m] = pv[2][m] - pv[0][m];
            xi[m] = pv[0][m] + s_ * e1[m] + t_ * e2[m];
        }
        double N[6], ts[3] = {0, 0, 0}, tt[3] = {0, 0, 0}, xq[3] = {0, 0, 0};
#pragma unroll
        for (int b = 0; b < 6; ++b) {
            double dN[3];
            shape10(loc[b], xi, N[b], dN);
            const double ds = dN[0] * e1[0] + dN[1] * e1[1] + dN[2] * e1[2];
            const double dt = dN[0] * e2[0] + dN[1] * e2[1] + dN[2] * e2[2];
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                ts[m] = fma(x[b][m], ds, ts[m]);
                tt[m] = fma(x[b][m], dt, tt[m]);
                xq[m] = fma(x[b][m], N[b], xq[m]);
            }
        }
        double nr[3] = {ts[1] * tt[2] - ts[2] * tt[1], ts[2] * tt[0] - ts[0] * tt[2], ts[0] * tt[1] - ts[1] * tt[0]};
        if (nr[0] * (xq[0] - xk[0]) + nr[1] * (xq[1] - xk[1]) + nr[2] * (xq[2] - xk[2]) < 0.0) {
#pragma unroll
            for (int m = 0; m < 3; ++m) nr[m] = -nr[m];
        }
        const double dS = sqrt(nr[0] * nr[0] + nr[1] * nr[1] + nr[2] * nr[2]);
        if (!(dS > 0.0)) {
            atomicMin(p.status, (unsigned long long)e);
            return;
        }
        const double w = wq * dS;
        const double Na = N[mf];
        double uq = 0.0, gq = 0.0;
#pragma unroll
        for (int b = 0; b < 6; ++b) {
            uq = fma(N[b], U[b], uq);
            gq = fma(N[b], G[b], gq);
        }
        if (kind == MF_BFORM_PENALTY || kind == MF_BFORM_CONVECTION) {
#pragma unroll
            for (int b = 0; b < 6; ++b) krow[b] += c * w * Na * N[b];
            rrow += c * w * Na * (uq - gq);
        } else if (kind == MF_BFORM_RADIATION) {
#pragma unroll
            for (int b = 0; b < 6; ++b) krow[b] += c * w * Na * 4.0 * uq * uq * uq * N[b];
            rrow += c * w * Na * (uq * uq * uq * uq - gq * gq * gq * gq);
        } else {  // MF_BFORM_TRACTION
            const double* S = p.form.value;
            const double ti = tg ? gq : (S[3 * i] * nr[0] + S[3 * i + 1] * nr[1] + S[3 * i + 2] * nr[2]) / dS;
            rrow -= w * Na * ti;
        }
    }
    const int a = loc[mf];
    const int64_t va = node[mf];
    const int64_t row = p.field_major ? (int64_t)i * p.n_nodes + va : (int64_t)NF * va + i;
    const int64_t rs = p.row_ptr[row];
    const int64_t deg = p.nbr_ptr[va + 1] - p.nbr_ptr[va];
    T* K = (T*)p.K;
    T* d = (T*)p.d;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
        if (krow[b] == 0.0) continue;
        const int64_t rk = p.rank[(int64_t)(a * 10 + loc[b]) * p.n_el + e];
        const int64_t pos = p.field_major ? rs + i * deg + rk : rs + rk * NF + i;
        unsafeAtomicAdd(K + pos, (T)krow[b]);
    }
    if (rrow != 0.0) unsafeAtomicAdd(d + row, (T)(-rrow));
}

// Edges of quadrilaterals (NEN = 4 or 8): one thread per (edge, edge node, field).  Edge
// eid = 2 * axis + side is xi_axis = -1 or +1, with its two corners and, for the 8-node
// element, its midpoint; Gauss rule with 2 or 3 points along the edge; ds = |dx/dt| and n
// the unit normal pointing away from the element's centre.  Penalty, convection,
// radiation and traction (sigma^l: the leading 2x2 block of value, or a nodal target).
template <int NEN, int NF, typename T>
__global__ void __launch_bounds__(kThreads) k_boundary_2d(BParams p)
{
    constexpr int NE = NEN == 8 ? 3 : 2;  // nodes per edge, and Gauss points
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p.n_faces * NE * NF) return;
    const int64_t f = face_of(p, t % p.n_faces);
    const int ki = (int)(t / p.n_faces);
    const int me = ki / NF, i = ki % NF;
    const int64_t e = p.face_elem[f];
    const int eid = p.face_id[f];
    if (e < 0 || e >= p.n_el || eid > 3) {
        if (ki == 0) atomicMin(p.status + 1, (unsigned long long)f);
        return;
    }
    const int axis = eid >> 1, side = eid & 1, other = 1 - axis;
    int loc[3];
    for (int a = 0, c = 0; a < 4; ++a)
        if (((a >> axis) & 1) == side) loc[c++] = a;
    if (NEN == 8) loc[2] = axis == 0 ? 6 + side : 4 + side;
    double x[NE][2], U[NE], G[NE], centre[2] = {0.0, 0.0};
    int32_t node[NE];
    const T* st = (const T*)p.state;
    const T* tg = (const T*)p.target;
#pragma unroll
    for (int b = 0; b < NE; ++b) {
        node[b] = p.conn[(int64_t)loc[b] * p.n_el + e];
#pragma unroll
        for (int m = 0; m < 2; ++m) x[b][m] = p.coords[(int64_t)m * p.n_nodes + node[b]];
        U[b] = st ? (double)st[(int64_t)i * p.n_nodes + node[b]] : 0.0;
        G[b] = tg ? (double)tg[(int64_t)i * p.n_nodes + node[b]] : p.form.value[i];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int32_t v = p.conn[(int64_t)a * p.n_el + e];
#pragma unroll
        for (int m = 0; m < 2; ++m) centre[m] += 0.25 * p.coords[(int64_t)m * p.n_nodes + v];
    }
    const mf_bform_kind kind = p.form.kind;
    const double c = p.form.coef;
    double krow[NE];
#pragma unroll
    for (int b = 0; b < NE; ++b) krow[b] = 0.0;
    double rrow = 0.0;
    const double g3 = 0.7745966692414834;  // sqrt(3/5)
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const double tq = NE == 3 ? (q - 1) * g3 : (q ? kGaussPt : -kGaussPt);
        const double wq = NE == 3 ? (q == 1 ? 8.0 / 9.0 : 5.0 / 9.0) : 1.0;
        double xi[2];
        xi[axis] = side ? 1.0 : -1.0;
        xi[other] = tq;
        double N[NE], tang[2] = {0.0, 0.0}, xq[2] = {0.0, 0.0};
#pragma unroll
        for (int b = 0; b < NE; ++b) {
            double dN[2];
            if constexpr (NEN == 8) {
                shape8(loc[b], xi, N[b], dN);
            } else {
                const int bx = loc[b] & 1, by = loc[b] >> 1;
                const double fx = 0.5 * (1.0 + (bx ? xi[0] : -xi[0])), fy = 0.5 * (1.0 + (by ? xi[1] : -xi[1]));
                N[b] = fx * fy;
                dN[0] = (bx ? 0.5 : -0.5) * fy;
                dN[1] = (by ? 0.5 : -0.5) * fx;
            }
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                tang[m] = fma(x[b][m], dN[other], tang[m]);
                xq[m] = fma(x[b][m], N[b], xq[m]);
            }
        }
        const double ds = sqrt(tang[0] * tang[0] + tang[1] * tang[1]);
        if (!(ds > 0.0)) {
            atomicMin(p.status, (unsigned long long)e);
            return;
        }
        double nv[2] = {tang[1] / ds, -tang[0] / ds};
        if (nv[0] * (xq[0] - centre[0]) + nv[1] * (xq[1] - centre[1]) < 0.0) {
            nv[0] = -nv[0];
            nv[1] = -nv[1];
        }
        const double w = wq * ds;
        const double Na = N[me];
        double uq = 0.0, gq = 0.0;
#pragma unroll
        for (int b = 0; b < NE; ++b) {
            uq = fma(N[b], U[b], uq);
            gq = fma(N[b], G[b], gq);
        }
        if (kind == MF_BFORM_PENALTY || kind == MF_BFORM_CONVECTION) {
#pragma unroll
            for (int b = 0; b < NE; ++b) krow[b] += c * w * Na * N[b];
            rrow += c * w * Na * (uq - gq);
        } else if (kind == MF_BFORM_RADIATION) {
#pragma unroll
            for (int b = 0; b < NE; ++b) krow[b] += c * w * Na * 4.0 * uq * uq * uq * N[b];
            rrow += c * w * Na * (uq * uq * uq * uq - gq * gq * gq * gq);
        } else {  // MF_BFORM_TRACTION
            const double* S = p.form.value;
            const double ti = tg ? gq : S[3 * i] * nv[0] + S[3 * i + 1] * nv[1];
            rrow -= w * Na * ti;
        }
    }
    const int a = loc[me];
    const int64_t va = node[me];
    const int64_t row = p.field_major ? (int64_t)i * p.n_nodes + va : (int64_t)NF * va + i;
    const int64_t rs = p.row_ptr[row];
    const int64_t deg = p.nbr_ptr[va + 1] - p.nbr_ptr[va];
    T* K = (T*)p.K;
    T* d = (T*)p.d;
#pragma unroll
    for (int b = 0; b < NE; ++b) {
        if (krow[b] == 0.0) continue;
        const int64_t rk = p.rank[(int64_t)(a * NEN + loc[b]) * p.n_el + e];
        const int64_t pos = p.field_major ? rs + i * deg + rk : rs + rk * NF + i;
        unsafeAtomicAdd(K + pos, (T)krow[b]);
    }
    if (rrow != 0.0) unsafeAtomicAdd(d + row, (T)(-rrow));
}

template <int NEN, int NF, typename T>
mf_status launch_boundary_2d(const BParams& p, hipStream_t s)
{
    constexpr int NE = NEN == 8 ? 3 : 2;
    const int64_t n = p.n_faces * NE * NF;
    if (n == 0) return MF_OK;
    if (n > 0xffffffffLL - kThreads) return set_error(MF_ERR_ARG, "too many edges for one launch");
    k_boundary_2d<NEN, NF, T><<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(p);
    MF_HIP(hipGetLastError());
    return MF_OK;
}

template <int NF, typename T>
mf_status launch_boundary_tet10(const BParams& p, hipStream_t s)
{
    const int64_t n = p.n_faces * 6 * NF;
    if (n == 0) return MF_OK;
    if (n > 0xffffffffLL - kThreads) return set_error(MF_ERR_ARG, "too many faces for one launch");
    k_boundary_tet10<NF, T><<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(p);
    MF_HIP(hipGetLastError());
    return MF_OK;
}

template <int NF, typename T>
mf_status launch_boundary20(const BParams& p, hipStream_t s)
{
    const int64_t n = p.n_faces * 8 * NF;
    if (n == 0) return MF_OK;
    if (n > 0xffffffffLL - kThreads) return set_error(MF_ERR_ARG, "too many faces for one launch");
    k_boundary20<NF, T><<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(p);
    MF_HIP(hipGetLastError());
    return MF_OK;
}

__global__ void k_face_zero(uint32_t* __restrict__ w, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w[i] = 0u;
}

// per element: bit fid of mask[e] for each listed local face, cnt[6 e + fid] its count;
// an element's first face appends it to the list of its colour (list of colour c at
// clist[cptr[c] ..], length ccount[c]; the order within a list does not matter, as
// elements of one colour write disjoint rows).  A face out of range is skipped and
// reported through the second status word.
__global__ void k_face_mark(const int32_t* __restrict__ fe, const uint8_t* __restrict__ fid, int64_t n,
                            int64_t n_el, const int32_t* __restrict__ ecol, const int64_t* __restrict__ cptr,
                            uint32_t* __restrict__ mask, uint32_t* __restrict__ cnt, int32_t* __restrict__ clist,
                            uint32_t* __restrict__ ccount, unsigned long long* __restrict__ status)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t e = -1;
    int c = -1;  // colour of an element this face touches first
    if (f < n) {
        e = fe[f];
        const int lf = fid[f];
        if (e < 0 || e >= n_el || lf > 5) {
            atomicMin(status + 1, (unsigned long long)f);
        } else {
            atomicAdd(cnt + 6 * e + lf, 1u);
            if (atomicOr(mask + e, 1u << lf) == 0u) c = ecol[e];
        }
    }
    // append to the colour lists with one counter update per (wave, colour): the lanes
    // of one colour take consecutive slots after the leader's atomic add
    const int lane = (int)(threadIdx.x & 63);
    unsigned long long pending = __ballot(c >= 0);
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int cc = __shfl(c, leader, 64);
        const unsigned long long group = __ballot(c == cc);
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(ccount + cc, (uint32_t)__popcll(group));
        base = (uint32_t)__shfl((int)base, leader, 64);
        if (c == cc) {
            const uint32_t below = (uint32_t)__popcll(group & ((1ull << lane) - 1ull));
            clist[cptr[cc] + base + below] = (int32_t)e;
        }
        pending &= ~group;
    }
}

// 8-node hexahedra: mark the listed faces per element, then one launch per element
// colour (elements of a colour share no node, so each row is added by one thread of the
// launch, and the colours follow each other in the stream: the sums do not depend on
// the run, and nothing waits on the host)
template <int NF, typename T>
mf_status launch_boundary(BParams p, const mf_pattern_s* Pc, hipStream_t s)
{
    mf_pattern_s* P = const_cast<mf_pattern_s*>(Pc);
    if (p.n_faces == 0 || P->n_elems == 0) return MF_OK;
    mf_status st = ensure_coloring(P, s);
    if (st != MF_OK) return st;
    const int n_col = (int)P->color_ptr.size() - 1;
    // workspace: mask [n_el], counts [6 n_el], colour lists [n_el], list lengths [n_col],
    // colour offsets (int64) [n_col + 1]
    const int64_t n_el = P->n_elems;
    const int64_t words = 8 * n_el + n_col + 2 * (n_col + 1) + 2;
    if (!P->face_elem_work) {
        MF_HIP(hipMalloc(&P->face_elem_work, sizeof(uint32_t) * (size_t)words));
        int64_t* cptr = (int64_t*)(P->face_elem_work + 8 * n_el + n_col + ((8 * n_el + n_col) & 1));
        MF_HIP(hipMemcpyAsync(cptr, P->color_ptr.data(), sizeof(int64_t) * (n_col + 1), hipMemcpyHostToDevice, s));
        MF_HIP(hipStreamSynchronize(s));
    }
    uint32_t* mask = P->face_elem_work;
    uint32_t* cnt = mask + n_el;
    int32_t* clist = (int32_t*)(cnt + 6 * n_el);
    uint32_t* ccount = (uint32_t*)(clist + n_el);
    const int64_t* cptr = (const int64_t*)(P->face_elem_work + 8 * n_el + n_col + ((8 * n_el + n_col) & 1));
    k_face_zero<<<(unsigned)((7 * n_el + kThreads - 1) / kThreads), kThreads, 0, s>>>(mask, 7 * n_el);
    k_face_zero<<<(unsigned)((n_col + kThreads - 1) / kThreads), kThreads, 0, s>>>(ccount, n_col);
    k_face_mark<<<(unsigned)((p.n_faces + kThreads - 1) / kThreads), kThreads, 0, s>>>(
        p.face_elem, p.face_id, p.n_faces, n_el, P->elem_color, cptr, mask, cnt, clist, ccount, P->status);
    p.face_mask = mask;
    p.face_cnt = cnt;
    for (int c = 0; c < n_col; ++c) {
        // at most min(colour size, faces) elements of the colour carry faces
        const int64_t bound = std::min<int64_t>(P->color_ptr[c + 1] - P->color_ptr[c], p.n_faces) * 8 * NF;
        if (bound == 0) continue;
        const unsigned blocks = (unsigned)std::min<int64_t>(2048, (bound + kThreads - 1) / kThreads);
        k_boundary<NF, T><<<blocks, kThreads, 0, s>>>(p, clist + P->color_ptr[c], ccount + c);
    }
    MF_HIP(hipGetLastError());
    return MF_OK;
}

__global__ void k_face_clear(int32_t* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// bucket of a face: colour of its element x local faces + local face; the last bucket
// holds the faces whose element or local face is out of range (the kernels report them)
__device__ __forceinline__ int face_key(const int32_t* fe, const uint8_t* fid, int64_t f, const int32_t* ecol,
                                        int64_t n_el, int n_local, int n_keys)
{
    const int64_t e = fe[f];
    const int lf = fid[f];
    return (e >= 0 && e < n_el && lf < n_local) ? ecol[e] * n_local + lf : n_keys - 1;
}

__global__ void k_face_hist(const int32_t* fe, const uint8_t* fid, int64_t n, const int32_t* ecol, int64_t n_el,
                            int n_local, int n_keys, int32_t* cnt)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f < n) atomicAdd(cnt + face_key(fe, fid, f, ecol, n_el, n_local, n_keys), 1);
}

// cursor := exclusive scan of cnt (a few hundred buckets at most: one lane)
__global__ void k_face_scan(const int32_t* cnt, int n_keys, int32_t* cursor)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int32_t acc = 0;
    for (int k = 0; k < n_keys; ++k) {
        cursor[k] = acc;
        acc += cnt[k];
    }
}

__global__ void k_face_place(const int32_t* fe, const uint8_t* fid, int64_t n, const int32_t* ecol, int64_t n_el,
                             int n_local, int n_keys, int32_t* cursor, int32_t* order)
{
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f < n) order[atomicAdd(cursor + face_key(fe, fid, f, ecol, n_el, n_local, n_keys), 1)] = (int32_t)f;
}

// Sorts the faces into colour buckets: order (device, in the pattern's workspace) lists
// the faces bucket by bucket, bucket k being order[off[k] .. off[k+1]).  Synchronises the
// stream once to read the bucket sizes.
mf_status bucket_faces(const mf_pattern_s* Pc, int n_local, const int32_t* fe, const uint8_t* fid, int64_t n,
                       hipStream_t s, std::vector<int64_t>& off, const int32_t*& order)
{
    mf_pattern_s* P = const_cast<mf_pattern_s*>(Pc);
    mf_status st = ensure_coloring(P, s);
    if (st != MF_OK) return st;
    const int n_colors = std::max(0, (int)P->color_ptr.size() - 1);
    const int n_keys = n_colors * n_local + 1;
    const int64_t need = 2 * (int64_t)n_keys + n;
    if (P->face_work_cap < need) {
        MF_HIP(hipStreamSynchronize(s));
        (void)hipFree(P->face_work);
        P->face_work = nullptr;
        P->face_work_cap = 0;
        MF_HIP(hipMalloc(&P->face_work, sizeof(int32_t) * (size_t)need));
        P->face_work_cap = need;
    }
    int32_t* cnt = P->face_work;
    int32_t* cursor = cnt + n_keys;
    int32_t* ord = cursor + n_keys;
    const unsigned blocks = (unsigned)((n + kThreads - 1) / kThreads);
    k_face_clear<<<(n_keys + kThreads - 1) / kThreads, kThreads, 0, s>>>(cnt, n_keys);
    k_face_hist<<<blocks, kThreads, 0, s>>>(fe, fid, n, P->elem_color, P->n_elems, n_local, n_keys, cnt);
    k_face_scan<<<1, 64, 0, s>>>(cnt, n_keys, cursor);
    k_face_place<<<blocks, kThreads, 0, s>>>(fe, fid, n, P->elem_color, P->n_elems, n_local, n_keys, cursor, ord);
    MF_HIP(hipGetLastError());
    std::vector<int32_t> h((size_t)n_keys);
    MF_HIP(hipMemcpyAsync(h.data(), cnt, sizeof(int32_t) * (size_t)n_keys, hipMemcpyDeviceToHost, s));
    MF_HIP(hipStreamSynchronize(s));
    off.assign((size_t)n_keys + 1, 0);
    for (int k = 0; k < n_keys; ++k) off[(size_t)k + 1] = off[(size_t)k] + h[(size_t)k];
    order = ord;
    return MF_OK;
}

}  // namespace
}  // namespace mf

using namespace mf;

extern "C" mf_status mf_assemble_boundary(const mf_pattern_t* P, const mf_bform* form, const double* coords,
                                          int64_t n_faces, const int32_t* face_elem, const uint8_t* face_id,
                                          const void* state, const void* target, mf_precision prec, void* K,
                                          void* d, void* stream)
{
    clear_error();
    if (!P || !form) return set_error(MF_ERR_ARG, "pattern or form is NULL");
    const bool two_d = P->dim == 2;
    if (two_d ? (P->nen != 4 && P->nen != 8) : (P->nen != 8 && P->nen != 20 && P->nen != 10))
        return set_error(MF_ERR_UNSUPPORTED, "boundary forms need quadrilaterals, hexahedra or tetrahedra");
    const bool quad = P->order == 2;
    const bool tet = P->nen == 10;
    if (prec != MF_F64 && prec != MF_F32) return set_error(MF_ERR_ARG, "unknown precision %d", (int)prec);
    if (n_faces < 0 || n_faces > ((int64_t)1 << 28)) return set_error(MF_ERR_ARG, "n_faces out of range");
    if (n_faces > 0 && (!face_elem || !face_id || !coords || !K || !d))
        return set_error(MF_ERR_ARG, "NULL faces, coords, K or d");
    if (!P->full_coupling) return set_error(MF_ERR_ARG, "boundary forms need a fully coupled pattern");
    const int nf = P->nf;
    switch (form->kind) {
        case MF_BFORM_PENALTY:
            if (nf != 1 && nf != P->dim)
                return set_error(MF_ERR_ARG, "penalty needs 1 or %d fields, pattern has %d", P->dim, nf);
            break;
        case MF_BFORM_CONVECTION:
        case MF_BFORM_RADIATION:
        case MF_BFORM_FLUX:
            if (nf != 1) return set_error(MF_ERR_ARG, "this boundary form is scalar; pattern has %d fields", nf);
            break;
        case MF_BFORM_TRACTION:
            if (nf != P->dim) return set_error(MF_ERR_ARG, "traction needs %d fields, pattern has %d", P->dim, nf);
            break;
        case MF_BFORM_NS_INFLOW:
        case MF_BFORM_NS_OUTFLOW:
        case MF_BFORM_NS_FIX:
            if (nf != 4) return set_error(MF_ERR_ARG, "flow boundary forms need 4 fields, pattern has %d", nf);
            break;
        default: return set_error(MF_ERR_ARG, "unknown boundary form %d", (int)form->kind);
    }
    if ((quad || two_d) && (form->kind == MF_BFORM_FLUX || nf == 4))
        return set_error(MF_ERR_UNSUPPORTED, "the flux and flow boundary forms need 8-node hexahedra");
    if (tet && n_faces > 0 && !face_id) return set_error(MF_ERR_ARG, "NULL face_id");
    hipStream_t s = (hipStream_t)stream;
    BParams p{};
    p.form = *form;
    p.n_el = P->n_elems;
    p.n_nodes = P->n_nodes;
    p.n_faces = n_faces;
    p.conn = P->conn;
    p.coords = coords;
    p.row_ptr = P->row_ptr;
    p.nbr_ptr = P->nbr_ptr;
    p.rank = P->rank;
    p.face_elem = face_elem;
    p.face_id = face_id;
    p.state = state;
    p.target = target;
    p.field_major = P->numbering == MF_FIELD_MAJOR;
    p.K = K;
    p.d = d;
    p.status = P->status;
    const_cast<mf_pattern_s*>(P)->last_stream = s;
    using Launch = mf_status (*)(const BParams&, hipStream_t);
    Launch launch = nullptr;
    const bool f64 = prec == MF_F64;
    int n_local = 6;  // local faces (edges in 2D) per element
    if (two_d) {
        if (nf != 1 && nf != 2) return set_error(MF_ERR_ARG, "edge forms need 1 or 2 fields, pattern has %d", nf);
        n_local = 4;
        if (P->nen == 8)
            launch = f64 ? (nf == 1 ? launch_boundary_2d<8, 1, double> : launch_boundary_2d<8, 2, double>)
                         : (nf == 1 ? launch_boundary_2d<8, 1, float> : launch_boundary_2d<8, 2, float>);
        else
            launch = f64 ? (nf == 1 ? launch_boundary_2d<4, 1, double> : launch_boundary_2d<4, 2, double>)
                         : (nf == 1 ? launch_boundary_2d<4, 1, float> : launch_boundary_2d<4, 2, float>);
    } else if (tet) {
        n_local = 4;
        launch = f64 ? (nf == 1 ? launch_boundary_tet10<1, double> : launch_boundary_tet10<3, double>)
                     : (nf == 1 ? launch_boundary_tet10<1, float> : launch_boundary_tet10<3, float>);
    } else if (quad) {
        launch = f64 ? (nf == 1 ? launch_boundary20<1, double> : launch_boundary20<3, double>)
                     : (nf == 1 ? launch_boundary20<1, float> : launch_boundary20<3, float>);
    } else {
        // 8-node hexahedra: element by element, colour by colour (no buckets)
        if (nf == 4) return f64 ? launch_boundary<4, double>(p, P, s) : launch_boundary<4, float>(p, P, s);
        if (nf == 1) return f64 ? launch_boundary<1, double>(p, P, s) : launch_boundary<1, float>(p, P, s);
        return f64 ? launch_boundary<3, double>(p, P, s) : launch_boundary<3, float>(p, P, s);
    }
    if (n_faces == 0) return MF_OK;
    std::vector<int64_t> off;
    const int32_t* order = nullptr;
    mf_status st = bucket_faces(P, n_local, face_elem, face_id, n_faces, s, off, order);
    if (st != MF_OK) return st;
    p.order = order;
    for (size_t k = 0; k + 1 < off.size(); ++k) {
        if (off[k + 1] == off[k]) continue;
        p.f_begin = off[k];
        p.n_faces = off[k + 1] - off[k];
        st = launch(p, s);
        if (st != MF_OK) return st;
    }
    return MF_OK;
}
