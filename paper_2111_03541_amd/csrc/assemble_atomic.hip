// Element-parallel assembly for meshes of any topology (Sec. 2.2 D-2 and D-3).
//
// One thread per (element e, local row (a, i)).  The thread computes the FP64 geometry
// at every Gauss point of e, accumulates row (a, i) of the element tangent and the
// element residual in precision T, and adds them into K and d, locating each entry
// through the element-to-nonzero rank map.  Two ways to add:
//   atomic    the paper's own scheme: all elements in one launch, hardware atomics;
//   coloured  the elements of one colour per launch (no two share a node), plain
//             read-modify-writes: each entry has one writer per launch and the stream
//             orders the colours, so the sums are the same on every run.
// K and d are cleared by fill kernels first, so the call overwrites them entirely.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "element.h"
#include "mf_internal.h"

namespace mf {
namespace {

constexpr int kThreads = 256;

struct AtomicParams {
    mf_form form;
    int64_t n_el, n_nodes;
    const int32_t* conn;
    const double* coords;
    const int32_t* row_ptr;
    const int32_t* nbr_ptr;
    const uint8_t* rank;
    const void* elem_param;
    const void* src;  // nodal sources (MASS/POISSON/ELASTICITY) or state (NS)
    const int32_t* elems;  // coloured: the elements of one colour
    int64_t n_list;        // coloured: their count
    int field_major;
    void* K;
    void* d;
    unsigned long long* status;
};

template <typename T>
__global__ void k_fill(T* p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = T(0);
}

// Item t = (local row (a, i), element of the list): the row's entries of K and d.
template <int FORM, int DIM, bool COLOURED, typename T>
__device__ __forceinline__ void atomic_item(const AtomicParams& p, int64_t t)
{
    constexpr int NEN = 1 << DIM;
    constexpr int NF = FormTraits<FORM, DIM>::NF;
    constexpr int NSRC = FormTraits<FORM, DIM>::NSRC;
    const int64_t n_el = p.n_el;
    const int64_t n_items = COLOURED ? p.n_list : n_el;
    if (t >= n_items * NEN * NF) return;
    const int64_t e = COLOURED ? (int64_t)p.elems[t % n_items] : t % n_el;
    const int ai = (int)(t / n_items);
    const int a = ai / NF, i = ai % NF;

    int32_t node[NEN];
    double x[NEN][DIM];
    T U[NEN][NSRC];
    const T* src = (const T*)p.src;
#pragma unroll
    for (int b = 0; b < NEN; ++b) {
        node[b] = p.conn[(int64_t)b * n_el + e];
#pragma unroll
        for (int m = 0; m < DIM; ++m) x[b][m] = p.coords[(int64_t)m * p.n_nodes + node[b]];
#pragma unroll
        for (int s = 0; s < NSRC; ++s) U[b][s] = src ? src[(int64_t)s * p.n_nodes + node[b]] : T(0);
    }
    const double ep = p.elem_param ? (double)((const T*)p.elem_param)[e] : 1.0;
    const Coef<T> C = make_coef<T>(FORM, p.form, ep);

    T krow[NEN * NF];
#pragma unroll
    for (int k = 0; k < NEN * NF; ++k) krow[k] = T(0);
    T rrow = T(0);
#pragma unroll
    for (int q = 0; q < NEN; ++q) {  // 2^DIM Gauss points, unit weights
        double gd[NEN][DIM];
        const double det = geometry_at<DIM>(x, q, gd);
        if (!(det > 0.0)) {
            atomicMin(p.status, (unsigned long long)e);
            return;
        }
        T N[NEN], g[NEN][DIM];
#pragma unroll
        for (int b = 0; b < NEN; ++b) {
            N[b] = (T)ref_N<DIM>(b, q);
#pragma unroll
            for (int m = 0; m < DIM; ++m) g[b][m] = (T)gd[b][m];
        }
        row_update<FORM, DIM, T>(a, i, C, N, g, (T)det, U, krow, rrow);
    }

    {
        // a non-finite input (element parameter, source or state) shows in the row sums
        T chk = rrow;
#pragma unroll
        for (int k = 0; k < NEN * NF; ++k) chk += krow[k];
        if (!isfinite(chk)) atomicMin(p.status + 2, (unsigned long long)e);
    }
    const int64_t va = node[a];
    const int64_t row = p.field_major ? (int64_t)i * p.n_nodes + va : (int64_t)NF * va + i;
    const int64_t rs = p.row_ptr[row];
    const int64_t deg = p.nbr_ptr[va + 1] - p.nbr_ptr[va];
    T* K = (T*)p.K;
    T* d = (T*)p.d;
    int rk[NEN];
#pragma unroll
    for (int b = 0; b < NEN; ++b) rk[b] = p.rank[(int64_t)(a * NEN + b) * n_el + e];
    auto pos_of = [&](int b, int j) -> int64_t {
        return p.field_major ? rs + j * deg + rk[b] : rs + (int64_t)rk[b] * NF + j;
    };
    if constexpr (COLOURED) {
        // every old value of the row is loaded before the first store, so the thread's
        // read-modify-writes overlap instead of running one after another
        T old[NEN * NF];
#pragma unroll
        for (int b = 0; b < NEN; ++b)
#pragma unroll
            for (int j = 0; j < NF; ++j) old[b * NF + j] = K[pos_of(b, j)];
        const T dold = d[row];
#pragma unroll
        for (int b = 0; b < NEN; ++b)
#pragma unroll
            for (int j = 0; j < NF; ++j) K[pos_of(b, j)] = old[b * NF + j] + krow[b * NF + j];
        d[row] = dold - rrow;
    } else {
#pragma unroll
        for (int b = 0; b < NEN; ++b)
#pragma unroll
            for (int j = 0; j < NF; ++j) unsafeAtomicAdd(K + pos_of(b, j), krow[b * NF + j]);
        unsafeAtomicAdd(d + row, -rrow);
    }
}

template <int FORM, int DIM, bool COLOURED, typename T>
__global__ void __launch_bounds__(kThreads) k_assemble_atomic(AtomicParams p)
{
    atomic_item<FORM, DIM, COLOURED, T>(p, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Homogeneous Dirichlet elimination of row r (structure kept): a constrained row becomes a
// unit row with d = 0, a constrained column is zeroed in the other rows.
template <typename T>
__device__ __forceinline__ void dirichlet_row(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
                                              const uint8_t* __restrict__ mask, int64_t r, T* __restrict__ K,
                                              T* __restrict__ d)
{
    const int64_t k0 = row_ptr[r], k1 = row_ptr[r + 1];
    if (mask[r]) {
        for (int64_t k = k0; k < k1; ++k) K[k] = (col_idx[k] == r) ? T(1) : T(0);
        d[r] = T(0);
    } else {
        for (int64_t k = k0; k < k1; ++k)
            if (mask[col_idx[k]]) K[k] = T(0);
    }
}

// Small 2D meshes in one launch of one workgroup: status reset, clear, the colours one after
// another behind workgroup barriers (the same plain read-modify-writes and order as the
// per-colour launches), then the Dirichlet elimination.  The whole call is then one launch
// instead of eight, which is what its time is made of at this size.
constexpr int kSmallThreads = 1024;
constexpr int kSmallMaxColors = 16;
constexpr int64_t kSmallMaxItems = 16 * kSmallThreads;  // per colour: at most 16 items a thread
struct SmallColors {
    int n;
    int64_t off[kSmallMaxColors + 1];
};

template <int FORM, typename T>
__global__ void __launch_bounds__(kSmallThreads) k_assemble_small(AtomicParams p, const int32_t* __restrict__ color_elems,
                                                                  SmallColors cl, const uint8_t* __restrict__ mask,
                                                                  int64_t nnz, int64_t n_rows,
                                                                  const int32_t* __restrict__ col_idx)
{
    constexpr int NEN = 4;
    constexpr int NF = FormTraits<FORM, 2>::NF;
    const int tid = threadIdx.x;
    if (tid < 3) p.status[tid] = ~0ull;
    T* K = (T*)p.K;
    T* d = (T*)p.d;
    for (int64_t k = tid; k < nnz; k += kSmallThreads) K[k] = T(0);
    for (int64_t k = tid; k < n_rows; k += kSmallThreads) d[k] = T(0);
    __syncthreads();
    for (int c = 0; c < cl.n; ++c) {
        AtomicParams pc = p;
        pc.elems = color_elems + cl.off[c];
        pc.n_list = cl.off[c + 1] - cl.off[c];
        const int64_t n = pc.n_list * NEN * NF;
        for (int64_t t = tid; t < n; t += kSmallThreads) atomic_item<FORM, 2, true, T>(pc, t);
        __syncthreads();
    }
    if (mask)
        for (int64_t r = tid; r < n_rows; r += kSmallThreads) dirichlet_row(p.row_ptr, col_idx, mask, r, K, d);
}

template <typename T>
__global__ void k_dirichlet(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
                            const uint8_t* __restrict__ mask, int64_t n_rows, T* __restrict__ K,
                            T* __restrict__ d)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    dirichlet_row(row_ptr, col_idx, mask, r, K, d);
}

// dirichlet_row with LANES lanes per row (consecutive lanes take consecutive entries, so
// the column loads of a row group are one contiguous access); every entry gets the same
// value as in dirichlet_row
template <typename T, int LANES>
__global__ void __launch_bounds__(kThreads) k_dirichlet_lanes(const int32_t* __restrict__ row_ptr,
                                                              const int32_t* __restrict__ col_idx,
                                                              const uint8_t* __restrict__ mask, int64_t n_rows,
                                                              T* __restrict__ K, T* __restrict__ d)
{
    const int lane = threadIdx.x % LANES;
    const int64_t rows_per_pass = (int64_t)gridDim.x * (kThreads / LANES);
    for (int64_t r = ((int64_t)blockIdx.x * kThreads + threadIdx.x) / LANES; r < n_rows; r += rows_per_pass) {
        const int64_t k0 = row_ptr[r], k1 = row_ptr[r + 1];
        if (mask[r]) {
            for (int64_t k = k0 + lane; k < k1; k += LANES) K[k] = (col_idx[k] == r) ? T(1) : T(0);
            if (lane == 0) d[r] = T(0);
        } else {
            for (int64_t k = k0 + lane; k < k1; k += LANES)
                if (mask[col_idx[k]]) K[k] = T(0);
        }
    }
}

template <typename T>
void launch_dirichlet(const mf_pattern_s* P, const uint8_t* mask, T* K, T* d, hipStream_t s)
{
    const int64_t n = P->n_rows;
    const int64_t avg = P->nnz / n;
    const int lanes = avg >= 48 ? 8 : avg >= 12 ? 4 : 1;
    if (lanes == 1) {
        k_dirichlet<T><<<blocks_for(n, kThreads), kThreads, 0, s>>>(P->row_ptr, P->col_idx, mask, n, K, d);
        return;
    }
    const unsigned g = (unsigned)std::min<int64_t>(8192, (n * lanes + kThreads - 1) / kThreads);
    if (lanes == 8) k_dirichlet_lanes<T, 8><<<g, kThreads, 0, s>>>(P->row_ptr, P->col_idx, mask, n, K, d);
    else k_dirichlet_lanes<T, 4><<<g, kThreads, 0, s>>>(P->row_ptr, P->col_idx, mask, n, K, d);
}

__global__ void k_reset_status(unsigned long long* s)
{
    s[0] = ~0ull;
    s[1] = ~0ull;
    s[2] = ~0ull;
}

template <int FORM, int DIM, typename T>
mf_status launch_atomic(const AssembleArgs& A, bool coloured)
{
    constexpr int NEN = 1 << DIM;
    constexpr int NF = FormTraits<FORM, DIM>::NF;
    const mf_pattern_s* P = A.P;
    AtomicParams p{};
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
    if (P->nnz > 0) k_fill<T><<<blocks_for(P->nnz, kThreads), kThreads, 0, A.stream>>>((T*)A.K, P->nnz);
    if (P->n_rows > 0) k_fill<T><<<blocks_for(P->n_rows, kThreads), kThreads, 0, A.stream>>>((T*)A.d, P->n_rows);
    MF_HIP(hipGetLastError());
    if (P->n_elems == 0) return MF_OK;
    if (!coloured) {
        const int64_t n = P->n_elems * NEN * NF;
        k_assemble_atomic<FORM, DIM, false, T><<<blocks_for(n, kThreads), kThreads, 0, A.stream>>>(p);
        MF_HIP(hipGetLastError());
        return MF_OK;
    }
    const mf_status st = ensure_coloring(P, A.stream);
    if (st != MF_OK) return st;
    for (size_t c = 0; c + 1 < P->color_ptr.size(); ++c) {
        p.elems = P->color_elems + P->color_ptr[c];
        p.n_list = P->color_ptr[c + 1] - P->color_ptr[c];
        const int64_t n = p.n_list * NEN * NF;
        if (n > 0) k_assemble_atomic<FORM, DIM, true, T><<<blocks_for(n, kThreads), kThreads, 0, A.stream>>>(p);
    }
    MF_HIP(hipGetLastError());
    return MF_OK;
}

template <int FORM, typename T>
mf_status launch_small(const AssembleArgs& A, const SmallColors& cl)
{
    const mf_pattern_s* P = A.P;
    AtomicParams p{};
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
    k_assemble_small<FORM, T><<<1, kSmallThreads, 0, A.stream>>>(p, P->color_elems, cl, A.dirichlet, P->nnz,
                                                                  P->n_rows, P->col_idx);
    MF_HIP(hipGetLastError());
    return MF_OK;
}

template <typename T>
mf_status dispatch_small(const AssembleArgs& A, const SmallColors& cl)
{
    switch (A.form->kind) {
        case MF_FORM_MASS: return launch_small<MF_FORM_MASS, T>(A, cl);
        case MF_FORM_POISSON: return launch_small<MF_FORM_POISSON, T>(A, cl);
        case MF_FORM_ELASTICITY: return launch_small<MF_FORM_ELASTICITY, T>(A, cl);
        case MF_FORM_NS_SUPG: return launch_small<MF_FORM_NS_SUPG, T>(A, cl);
    }
    return set_error(MF_ERR_ARG, "unknown form kind %d", (int)A.form->kind);
}

template <typename T>
mf_status dispatch_atomic(const AssembleArgs& A, bool c)
{
    const int dim = A.P->dim;
    switch (A.form->kind) {
        case MF_FORM_MASS:
            return dim == 2 ? launch_atomic<MF_FORM_MASS, 2, T>(A, c) : launch_atomic<MF_FORM_MASS, 3, T>(A, c);
        case MF_FORM_POISSON:
            return dim == 2 ? launch_atomic<MF_FORM_POISSON, 2, T>(A, c) : launch_atomic<MF_FORM_POISSON, 3, T>(A, c);
        case MF_FORM_ELASTICITY:
            return dim == 2 ? launch_atomic<MF_FORM_ELASTICITY, 2, T>(A, c)
                            : launch_atomic<MF_FORM_ELASTICITY, 3, T>(A, c);
        case MF_FORM_NS_SUPG:
            return dim == 2 ? launch_atomic<MF_FORM_NS_SUPG, 2, T>(A, c) : launch_atomic<MF_FORM_NS_SUPG, 3, T>(A, c);
    }
    return set_error(MF_ERR_ARG, "unknown form kind %d", (int)A.form->kind);
}

}  // namespace

mf_status assemble_atomic(const AssembleArgs& A, bool coloured)
{
    return A.prec == MF_F64 ? dispatch_atomic<double>(A, coloured) : dispatch_atomic<float>(A, coloured);
}

mf_status assemble_small(const AssembleArgs& A)
{
    const mf_pattern_s* P = A.P;
    if (P->dim != 2 || P->order != 1 || P->n_elems == 0) return MF_ERR_UNSUPPORTED;
    mf_status st = ensure_coloring(P, A.stream);
    if (st != MF_OK) return st;
    const int n_col = (int)P->color_ptr.size() - 1;
    if (n_col < 1 || n_col > kSmallMaxColors) return MF_ERR_UNSUPPORTED;
    SmallColors cl{};
    cl.n = n_col;
    const int64_t rows_per_elem = 4 * (int64_t)P->nf;
    for (int c = 0; c <= n_col; ++c) cl.off[c] = P->color_ptr[c];
    for (int c = 0; c < n_col; ++c)
        if ((cl.off[c + 1] - cl.off[c]) * rows_per_elem > kSmallMaxItems) return MF_ERR_UNSUPPORTED;
    return A.prec == MF_F64 ? dispatch_small<double>(A, cl) : dispatch_small<float>(A, cl);
}

mf_status apply_dirichlet(const AssembleArgs& A)
{
    const mf_pattern_s* P = A.P;
    if (!A.dirichlet || P->n_rows == 0) return MF_OK;
    if (A.prec == MF_F64) launch_dirichlet<double>(P, A.dirichlet, (double*)A.K, (double*)A.d, A.stream);
    else launch_dirichlet<float>(P, A.dirichlet, (float*)A.K, (float*)A.d, A.stream);
    MF_HIP(hipGetLastError());
    return MF_OK;
}

mf_status reset_status(const mf_pattern_s* P, hipStream_t s)
{
    k_reset_status<<<1, 1, 0, s>>>(P->status);
    MF_HIP(hipGetLastError());
    return MF_OK;
}

}  // namespace mf
