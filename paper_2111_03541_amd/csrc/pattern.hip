// Sparsity pattern of K on the GPU (Sec. 2.2 Block B).
//
//  B-1  element-to-node map -> node incidence (counting sort by node id)
//       node pairs: N(v) = sorted unique nodes sharing an element with v
//  B-3  DOF map: node-major dof = nf*v + i, field-major dof = i*n_nodes + v
//  B-4  sparse layout, as CSR instead of the paper's COO: row dof(v,i) holds dof(w,j)
//       for w in N(v) and coupling(i,j), ascending; plus the element-to-nonzero rank map
//       rank[(a*nen+b)][e] = position of conn[b][e] in N(conn[a][e]).
//
// All integer work, bit-exact by construction (sorted sets do not depend on the order
// in which atomics fill the incidence lists).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <vector>

#include "mf_internal.h"

namespace mf {
namespace {

constexpr int kThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kThreads * kScanItems;

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// error flags: bit 0 node id out of range, bit 1 valence overflow, bit 2 grid mismatch
__global__ void k_count_incidence(const int32_t* __restrict__ conn, int64_t n_entries,
                                  int64_t n_nodes, int32_t* __restrict__ cnt, int* flag)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_entries) return;
    int32_t v = conn[t];
    if (v < 0 || v >= n_nodes) {
        atomicOr(flag, 1);
        return;
    }
    atomicAdd(&cnt[v], 1);
}

__global__ void k_fill_incidence(const int32_t* __restrict__ conn, int64_t n_el, int nen,
                                 const int64_t* __restrict__ inc_ptr, int32_t* __restrict__ cursor,
                                 int32_t* __restrict__ inc)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_el * nen) return;
    int64_t e = t % n_el;
    int32_t v = conn[t];
    int32_t pos = atomicAdd(&cursor[v], 1);
    inc[inc_ptr[v] + pos] = (int32_t)e;
}

// Distinct neighbours of v in ascending order, by repeated selection of the smallest
// candidate above the last one taken.  write == nullptr: count only.
__global__ void k_node_neighbours(const int32_t* __restrict__ conn, int64_t n_el, int nen,
                                  int64_t n_nodes, const int64_t* __restrict__ inc_ptr,
                                  const int32_t* __restrict__ inc, int32_t* __restrict__ deg,
                                  const int64_t* __restrict__ out_ptr, int32_t* __restrict__ out,
                                  int* flag)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_nodes) return;
    int64_t k0 = inc_ptr[v], k1 = inc_ptr[v + 1];
    int32_t last = -1;
    int cnt = 0;
    while (true) {
        int32_t next = INT_MAX;
        for (int64_t k = k0; k < k1; ++k) {
            int32_t e = inc[k];
            for (int b = 0; b < nen; ++b) {
                int32_t c = conn[(int64_t)b * n_el + e];
                if (c > last && c < next) next = c;
            }
        }
        if (next == INT_MAX) break;
        if (out) out[out_ptr[v] + cnt] = next;
        ++cnt;
        last = next;
        if (cnt > 255) {  // rank must fit uint8
            atomicOr(flag, 2);
            break;
        }
    }
    if (!out) deg[v] = cnt;
}

struct FieldTable {
    int nf;
    int C;            // sum_i c_i (columns per neighbour summed over rows of a node)
    int c[4];         // c_i = number of fields coupled to row field i
    int cpre[4];      // prefix of c_i
    int jidx[4][4];   // position of field j among the fields coupled to i (-1 if none)
};

// row_ptr from the node-graph offsets (no further scan needed):
//   node-major : start(v,i) = P_v * C + deg_v * cpre_i
//   field-major: start(v,i) = cpre_i * n_pairs + c_i * P_v
__global__ void k_row_ptr(const int64_t* __restrict__ nbr_ptr, int64_t n_nodes, int64_t n_pairs,
                          FieldTable ft, int field_major, int32_t* __restrict__ row_ptr)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_nodes) return;
    int64_t Pv = nbr_ptr[v];
    int64_t deg = nbr_ptr[v + 1] - Pv;
    for (int i = 0; i < ft.nf; ++i) {
        int64_t start, row;
        if (field_major) {
            start = (int64_t)ft.cpre[i] * n_pairs + (int64_t)ft.c[i] * Pv;
            row = (int64_t)i * n_nodes + v;
        } else {
            start = Pv * ft.C + deg * ft.cpre[i];
            row = (int64_t)ft.nf * v + i;
        }
        row_ptr[row] = (int32_t)start;
    }
    if (v == n_nodes - 1) row_ptr[(int64_t)ft.nf * n_nodes] = (int32_t)(n_pairs * ft.C);
}

__global__ void k_col_idx(const int64_t* __restrict__ nbr_ptr, const int32_t* __restrict__ nbr,
                          int64_t n_nodes, FieldTable ft, int field_major,
                          const int32_t* __restrict__ row_ptr, int32_t* __restrict__ col_idx)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_nodes) return;
    int64_t Pv = nbr_ptr[v];
    int64_t deg = nbr_ptr[v + 1] - Pv;
    for (int i = 0; i < ft.nf; ++i) {
        int64_t row = field_major ? (int64_t)i * n_nodes + v : (int64_t)ft.nf * v + i;
        int64_t base = row_ptr[row];
        for (int64_t r = 0; r < deg; ++r) {
            int64_t w = nbr[Pv + r];
            for (int j = 0; j < ft.nf; ++j) {
                int jj = ft.jidx[i][j];
                if (jj < 0) continue;
                int64_t col = field_major ? (int64_t)j * n_nodes + w : (int64_t)ft.nf * w + j;
                int64_t pos = field_major ? base + jj * deg + r : base + r * ft.c[i] + jj;
                col_idx[pos] = (int32_t)col;
            }
        }
    }
}

__global__ void k_rank(const int32_t* __restrict__ conn, int64_t n_el, int nen,
                       const int64_t* __restrict__ nbr_ptr, const int32_t* __restrict__ nbr,
                       uint8_t* __restrict__ rank)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_el * nen * nen) return;
    int64_t e = t % n_el;
    int ab = (int)(t / n_el);
    int a = ab / nen, b = ab % nen;
    int32_t va = conn[(int64_t)a * n_el + e], vb = conn[(int64_t)b * n_el + e];
    int64_t lo = nbr_ptr[va], hi = nbr_ptr[va + 1] - 1;
    int64_t r = 255;
    while (lo <= hi) {
        int64_t mid = (lo + hi) >> 1;
        int32_t x = nbr[mid];
        if (x == vb) { r = mid - nbr_ptr[va]; break; }
        if (x < vb) lo = mid + 1; else hi = mid - 1;
    }
    rank[t] = (uint8_t)r;
}

// Does conn equal the lexicographic grid numbering for (nx, ny, nz)?
__global__ void k_check_grid(const int32_t* __restrict__ conn, int64_t n_el, int nen, int dim,
                             int64_t nx, int64_t ny, int* flag)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_el * nen) return;
    int64_t e = t % n_el;
    int a = (int)(t / n_el);
    int64_t ex = e % nx, r = e / nx, ey = r % ny, ez = r / ny;
    int64_t i = ex + (a & 1), j = ey + ((a >> 1) & 1), k = dim == 3 ? ez + ((a >> 2) & 1) : 0;
    int64_t node = i + (nx + 1) * (j + (ny + 1) * k);
    if (conn[t] != node) atomicOr(flag, 4);
}

// --- exclusive scan of int32 counts into int64 offsets (out has n+1 entries) ---------

__device__ int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t* total)
{
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
        int64_t add = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int64_t incl = sh[t];
    *total = sh[kThreads - 1];
    __syncthreads();
    return incl - v;
}

template <typename TIn>
__global__ void k_scan_tiles(const TIn* __restrict__ in, int64_t n, int64_t* __restrict__ out,
                             int64_t* __restrict__ tile_sums)
{
    __shared__ int64_t sh[kThreads];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t vals[kScanItems];
    int64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t idx = base + k;
        vals[k] = idx < n ? (int64_t)in[idx] : 0;
        s += vals[k];
    }
    int64_t total;
    int64_t run = block_exclusive_scan(s, sh, &total);
    for (int k = 0; k < kScanItems; ++k) {
        int64_t idx = base + k;
        if (idx < n) out[idx] = run;
        run += vals[k];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void k_scan_add(int64_t* __restrict__ out, int64_t n, const int64_t* __restrict__ tile_off)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += tile_off[i / kScanTile];
}

// out[0..n] = exclusive prefix sums of in[0..n-1], out[n] = total.
template <typename TIn>
mf_status exclusive_scan(const TIn* in, int64_t n, int64_t* out, hipStream_t s)
{
    int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles == 0) tiles = 1;
    int64_t* sums = nullptr;
    int64_t* offs = nullptr;
    MF_HIP(hipMalloc(&sums, sizeof(int64_t) * tiles));
    MF_HIP(hipMalloc(&offs, sizeof(int64_t) * (tiles + 1)));
    if (n == 0) {
        MF_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), s));
        MF_HIP(hipStreamSynchronize(s));
        MF_HIP(hipFree(sums));
        MF_HIP(hipFree(offs));
        return MF_OK;
    }
    k_scan_tiles<TIn><<<(unsigned)tiles, kThreads, 0, s>>>(in, n, out, sums);
    MF_HIP(hipGetLastError());
    mf_status st = MF_OK;
    if (tiles > 1) {
        st = exclusive_scan<int64_t>(sums, tiles, offs, s);
    } else {
        MF_HIP(hipMemsetAsync(offs, 0, sizeof(int64_t), s));
        MF_HIP(hipMemcpyAsync(offs + 1, sums, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    }
    if (st == MF_OK) {
        k_scan_add<<<blocks_for(n, kThreads), kThreads, 0, s>>>(out, n, offs);
        MF_HIP(hipGetLastError());
        MF_HIP(hipMemcpyAsync(out + n, offs + tiles, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    }
    MF_HIP(hipStreamSynchronize(s));
    MF_HIP(hipFree(sums));
    MF_HIP(hipFree(offs));
    return st;
}

__global__ void k_i64_to_i32(const int64_t* __restrict__ in, int64_t n, int32_t* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int32_t)in[i];
}

struct Scratch {
    std::vector<void*> ptrs;
    ~Scratch() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    mf_status alloc(T** p, int64_t n) {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, (size_t)(n > 0 ? n : 1) * sizeof(T));
        if (e != hipSuccess) return set_error(MF_ERR_OOM, "device allocation of %lld bytes failed",
                                              (long long)(n * (int64_t)sizeof(T)));
        ptrs.push_back(q);
        *p = (T*)q;
        return MF_OK;
    }
};

#define MF_TRY(x)                          \
    do {                                   \
        mf_status st_ = (x);               \
        if (st_ != MF_OK) return st_;      \
    } while (0)

}  // namespace

mf_status build_pattern(mf_pattern_s* P, const int32_t* conn_in, hipStream_t s)
{
    const int nen = P->nen;
    const int64_t n_el = P->n_elems, n_nodes = P->n_nodes;
    const int64_t n_ent = n_el * nen;
    Scratch tmp;
    int* flag = nullptr;
    int32_t *cnt = nullptr, *cursor = nullptr, *inc = nullptr, *deg = nullptr;
    int64_t *inc_ptr = nullptr, *nbr_ptr64 = nullptr;
    MF_TRY(tmp.alloc(&flag, 1));
    MF_TRY(tmp.alloc(&cnt, n_nodes));
    MF_TRY(tmp.alloc(&cursor, n_nodes));
    MF_TRY(tmp.alloc(&inc, n_ent));
    MF_TRY(tmp.alloc(&deg, n_nodes));
    MF_TRY(tmp.alloc(&inc_ptr, n_nodes + 1));
    MF_TRY(tmp.alloc(&nbr_ptr64, n_nodes + 1));

    // library-owned copy of the connectivity
    MF_HIP(hipMalloc(&P->conn, sizeof(int32_t) * (size_t)(n_ent > 0 ? n_ent : 1)));
    if (n_ent > 0)
        MF_HIP(hipMemcpyAsync(P->conn, conn_in, sizeof(int32_t) * (size_t)n_ent, hipMemcpyDeviceToDevice, s));
    const int32_t* conn = P->conn;

    k_fill_i32<<<1, 1, 0, s>>>((int32_t*)flag, 1, 0);
    if (n_nodes > 0) {
        k_fill_i32<<<blocks_for(n_nodes, kThreads), kThreads, 0, s>>>(cnt, n_nodes, 0);
        k_fill_i32<<<blocks_for(n_nodes, kThreads), kThreads, 0, s>>>(cursor, n_nodes, 0);
    }
    if (n_ent > 0)
        k_count_incidence<<<blocks_for(n_ent, kThreads), kThreads, 0, s>>>(conn, n_ent, n_nodes, cnt, flag);
    MF_HIP(hipGetLastError());
    int hflag = 0;
    MF_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    MF_HIP(hipStreamSynchronize(s));
    if (hflag & 1) return set_error(MF_ERR_BAD_MESH, "conn holds a node id outside [0, %lld)",
                                    (long long)n_nodes);
    MF_TRY(exclusive_scan<int32_t>(cnt, n_nodes, inc_ptr, s));
    if (n_ent > 0)
        k_fill_incidence<<<blocks_for(n_ent, kThreads), kThreads, 0, s>>>(conn, n_el, nen, inc_ptr, cursor, inc);
    if (n_nodes > 0)
        k_node_neighbours<<<blocks_for(n_nodes, kThreads), kThreads, 0, s>>>(
            conn, n_el, nen, n_nodes, inc_ptr, inc, deg, nullptr, nullptr, flag);
    MF_HIP(hipGetLastError());
    MF_TRY(exclusive_scan<int32_t>(deg, n_nodes, nbr_ptr64, s));
    MF_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    int64_t n_pairs = 0;
    MF_HIP(hipMemcpyAsync(&n_pairs, nbr_ptr64 + n_nodes, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MF_HIP(hipStreamSynchronize(s));
    if (hflag & 2) return set_error(MF_ERR_OVERFLOW, "a node has more than 255 neighbours");

    // field table
    FieldTable ft{};
    ft.nf = P->nf;
    int C = 0;
    for (int i = 0; i < P->nf; ++i) {
        int ci = 0;
        for (int j = 0; j < P->nf; ++j) {
            ft.jidx[i][j] = P->coupling[i * P->nf + j] ? ci++ : -1;
        }
        ft.c[i] = ci;
        ft.cpre[i] = C;
        C += ci;
    }
    ft.C = C;
    const int64_t nnz = n_pairs * C;
    if (n_pairs >= INT_MAX || nnz >= INT_MAX)
        return set_error(MF_ERR_OVERFLOW, "nnz = %lld does not fit int32 CSR offsets", (long long)nnz);
    P->n_pairs = n_pairs;
    P->nnz = nnz;

    MF_HIP(hipMalloc(&P->nbr_ptr, sizeof(int32_t) * (size_t)(n_nodes + 1)));
    MF_HIP(hipMalloc(&P->nbr, sizeof(int32_t) * (size_t)(n_pairs > 0 ? n_pairs : 1)));
    MF_HIP(hipMalloc(&P->row_ptr, sizeof(int32_t) * (size_t)(P->n_rows + 1)));
    MF_HIP(hipMalloc(&P->col_idx, sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1)));
    MF_HIP(hipMalloc(&P->rank, (size_t)(nen * nen * (n_el > 0 ? n_el : 1))));
    MF_HIP(hipMalloc(&P->status, 3 * sizeof(unsigned long long)));  // bad element, bad face, non-finite element

    k_i64_to_i32<<<blocks_for(n_nodes + 1, kThreads), kThreads, 0, s>>>(nbr_ptr64, n_nodes + 1, P->nbr_ptr);
    if (n_nodes > 0)
        k_node_neighbours<<<blocks_for(n_nodes, kThreads), kThreads, 0, s>>>(
            conn, n_el, nen, n_nodes, inc_ptr, inc, deg, nbr_ptr64, P->nbr, flag);
    int fm = P->numbering == MF_FIELD_MAJOR ? 1 : 0;
    if (n_nodes > 0) {
        k_row_ptr<<<blocks_for(n_nodes, kThreads), kThreads, 0, s>>>(nbr_ptr64, n_nodes, n_pairs, ft, fm,
                                                                    P->row_ptr);
        k_col_idx<<<blocks_for(n_nodes, kThreads), kThreads, 0, s>>>(nbr_ptr64, P->nbr, n_nodes, ft, fm,
                                                                    P->row_ptr, P->col_idx);
    } else {
        k_fill_i32<<<1, 1, 0, s>>>(P->row_ptr, 1, 0);
    }
    if (n_el > 0)
        k_rank<<<blocks_for(n_el * nen * nen, kThreads), kThreads, 0, s>>>(conn, n_el, nen, nbr_ptr64,
                                                                           P->nbr, P->rank);
    MF_HIP(hipGetLastError());

    // structured-grid detection from the first element's nodes
    P->is_grid = 0;
    if (n_el > 0 && nen == (1 << P->dim)) {  // lexicographic Q1 grids only
        std::vector<int32_t> first(nen);
        for (int a = 0; a < nen; ++a)
            MF_HIP(hipMemcpyAsync(&first[a], conn + (int64_t)a * n_el, sizeof(int32_t),
                                  hipMemcpyDeviceToHost, s));
        MF_HIP(hipStreamSynchronize(s));
        int64_t nx = (int64_t)first[2] - 1;  // node (0,1[,0]) = nx + 1
        int64_t ny = 0, nz = 1;
        bool ok = first[0] == 0 && first[1] == 1 && nx >= 1;
        if (ok && P->dim == 3) {
            ny = (int64_t)first[4] / (nx + 1) - 1;  // node (0,0,1) = (nx+1)(ny+1)
            ok = ny >= 1 && (int64_t)first[4] % (nx + 1) == 0 && n_el % (nx * ny) == 0;
            if (ok) nz = n_el / (nx * ny);
            ok = ok && (nx + 1) * (ny + 1) * (nz + 1) == n_nodes;
        } else if (ok) {
            ok = n_el % nx == 0;
            if (ok) ny = n_el / nx;
            ok = ok && (nx + 1) * (ny + 1) == n_nodes;
        }
        if (ok) {
            k_fill_i32<<<1, 1, 0, s>>>((int32_t*)flag, 1, 0);
            k_check_grid<<<blocks_for(n_ent, kThreads), kThreads, 0, s>>>(conn, n_el, nen, P->dim, nx, ny, flag);
            MF_HIP(hipGetLastError());
            MF_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
            MF_HIP(hipStreamSynchronize(s));
            if (!(hflag & 4)) {
                P->is_grid = 1;
                P->gx = nx;
                P->gy = ny;
                P->gz = P->dim == 3 ? nz : 1;
            }
        }
    }
    MF_HIP(hipStreamSynchronize(s));
    return MF_OK;
}

// Greedy colouring of the elements in id order: each element takes the smallest colour
// not used by an element that shares one of its nodes.  Host work over the node-element
// incidence, once per pattern; elements are then listed colour by colour on the device.
mf_status ensure_coloring(const mf_pattern_s* Pc, hipStream_t s)
{
    mf_pattern_s* P = const_cast<mf_pattern_s*>(Pc);
    if (P->color_elems || P->n_elems == 0) return MF_OK;
    const int64_t n_el = P->n_elems, nn = P->n_nodes;
    const int nen = P->nen;
    std::vector<int32_t> conn((size_t)(n_el * nen));
    MF_HIP(hipMemcpyAsync(conn.data(), P->conn, sizeof(int32_t) * conn.size(), hipMemcpyDeviceToHost, s));
    MF_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> inc_ptr((size_t)nn + 1, 0);
    for (int64_t k = 0; k < n_el * nen; ++k) ++inc_ptr[(size_t)conn[(size_t)k] + 1];
    for (int64_t v = 0; v < nn; ++v) inc_ptr[(size_t)v + 1] += inc_ptr[(size_t)v];
    std::vector<int32_t> inc((size_t)(n_el * nen));
    std::vector<int64_t> cur(inc_ptr.begin(), inc_ptr.end() - 1);
    for (int64_t e = 0; e < n_el; ++e)
        for (int a = 0; a < nen; ++a) inc[(size_t)cur[(size_t)conn[(size_t)(a * n_el + e)]]++] = (int32_t)e;
    std::vector<int32_t> color((size_t)n_el, -1);
    std::vector<int64_t> seen_at(64, -1);  // colour -> last element that saw it taken
    int n_colors = 0;
    for (int64_t e = 0; e < n_el; ++e) {
        for (int a = 0; a < nen; ++a) {
            const int32_t v = conn[(size_t)(a * n_el + e)];
            for (int64_t k = inc_ptr[(size_t)v]; k < inc_ptr[(size_t)v + 1]; ++k) {
                const int32_t c = color[(size_t)inc[(size_t)k]];
                if (c >= 0) {
                    if ((size_t)c >= seen_at.size()) seen_at.resize((size_t)c + 1, -1);
                    seen_at[(size_t)c] = e;
                }
            }
        }
        int c = 0;
        while ((size_t)c < seen_at.size() && seen_at[(size_t)c] == e) ++c;
        color[(size_t)e] = c;
        n_colors = std::max(n_colors, c + 1);
    }
    P->color_ptr.assign((size_t)n_colors + 1, 0);
    for (int64_t e = 0; e < n_el; ++e) ++P->color_ptr[(size_t)color[(size_t)e] + 1];
    for (int c = 0; c < n_colors; ++c) P->color_ptr[(size_t)c + 1] += P->color_ptr[(size_t)c];
    std::vector<int32_t> order((size_t)n_el);
    std::vector<int64_t> at(P->color_ptr.begin(), P->color_ptr.end() - 1);
    for (int64_t e = 0; e < n_el; ++e) order[(size_t)at[(size_t)color[(size_t)e]]++] = (int32_t)e;
    int32_t* dev = nullptr;
    int32_t* ecol = nullptr;
    MF_HIP(hipMalloc(&dev, sizeof(int32_t) * (size_t)n_el));
    hipError_t err = hipMalloc(&ecol, sizeof(int32_t) * (size_t)n_el);
    if (err == hipSuccess)
        err = hipMemcpyAsync(dev, order.data(), sizeof(int32_t) * (size_t)n_el, hipMemcpyHostToDevice, s);
    if (err == hipSuccess)
        err = hipMemcpyAsync(ecol, color.data(), sizeof(int32_t) * (size_t)n_el, hipMemcpyHostToDevice, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    if (err != hipSuccess) {
        (void)hipFree(dev);
        (void)hipFree(ecol);
        P->color_ptr.clear();
        return hip_error(err, "colour upload");
    }
    P->color_elems = dev;
    P->elem_color = ecol;
    return MF_OK;
}

}  // namespace mf
