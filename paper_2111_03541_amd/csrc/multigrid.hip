// Geometric multigrid V-cycle on structured grids of 8-node hexahedra, the preconditioner
// of the Newton step's Krylov solve (Sec. 2.1) where Jacobi is too weak; the paper leaves
// the solver of Sec. 2.2 D-4 open.  Textbook multigrid:
//   levels     level l+1 halves the elements per axis of level l; its node (i,j,k) is the
//              level-l node (2i,2j,2k)
//   operators  rediscretisation: the same form assembled (FP64) on each coarse grid from the
//              coordinates, linearisation state and Dirichlet flags of the coincident fine
//              nodes (injection), an element coefficient field averaged over the eight
//              children, and boundary face sets coarsened with the grid
//   transfers  P = trilinear interpolation field by field, R = P^T (full weighting)
//   smoother   damped Jacobi x <- x + omega D^-1 (b - A x)
//   cycle      V(l, b): pre sweeps from x = 0, r = b - A x, b_c = R r (0 on coarse Dirichlet
//              rows), x += P V(l+1, b_c), post sweeps; coarsest level: sweeps from x = 0.
//
// Kernels (one grid-stride pass each, all on the caller's stream, nothing allocated or
// cleared with memset, so a cycle can be captured in a HIP graph):
//   k_mg_sweep     one Jacobi sweep, out of place, with the SpMV fused (8 lanes per row for
//                  the 4-field flow rows of up to 108 entries, 4 otherwise); the same kernel
//                  forms the first sweep from x = 0 (no SpMV) and the residual b - A x;
//                  scalar patterns run it on a slot-major ELL copy, one row per thread
//                  (k_mg_sweep_ell), node-major flow rows with the columns taken from
//                  the node graph (k_mg_sweep_nodes)
//   k_mg_restrict  one thread per coarse node and field gathers its 27 fine neighbours
//   k_mg_prolong   one thread per fine node interpolates from its 1, 2, 4 or 8 parents
//   k_mg_coarse    the coarsest level in one workgroup, the iterate in LDS, all sweeps in
//                  one launch, rows cached in registers when there are at most 256 (levels
//                  of more than kCoarseMax rows use k_mg_sweep)
// Sweeps alternate between two buffers per level; the first one is chosen so that the last
// sweep writes the level's output and no copy is needed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "mf_internal.h"
#include "pcg.h"

struct mf_mg_s {
    struct Level {
        int64_t nx = 0, ny = 0, nz = 0, n_nodes = 0, n_rows = 0;
        mf_pattern_s* P = nullptr;         // owned for l >= 1
        const mf_pattern_s* Pv = nullptr;  // this level's pattern
        double* K = nullptr;               // owned for l >= 1
        const double* Kv = nullptr;        // this level's operator (level 0: the caller's)
        double* d = nullptr;               // l >= 1: right side written by the assembly
        double* coords = nullptr;          // l >= 1: [3][n_nodes]
        double* state = nullptr;           // l >= 1: [4][n_nodes] linearisation state
        uint8_t* mask = nullptr;           // l >= 1: [n_rows]
        double* elem = nullptr;            // l >= 1: [n_elems] element coefficient field
        double* dinv = nullptr;            // [n_rows]
        double* x = nullptr;               // l >= 1: the cycle's output on this level
        double* b = nullptr;               // l >= 1: the restricted right side
        double* t = nullptr;               // second sweep buffer and residual
        // scalar patterns: the operator in slot-major ELL form (slot k of row i at
        // k * n_rows + i; padding has value 0 and column i), refreshed at every update
        int width = 0;
        int32_t* ecol = nullptr;
        double* eval = nullptr;
        // node-major rows of four fields: sweeps take the columns from the node graph
        bool node_cols = false;
    };
    int n_levels = 0;
    int nf = 0;
    int fm = 0;  // field-major numbering
    mf_mg_opts opts{};
    bool has_mask = false;
    bool updated = false;
    Level L[MF_MG_MAX_LEVELS];
    std::vector<void*> owned;
};

namespace mf {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 8192;
constexpr int kCoarseMax = 4096;      // rows of a coarsest level solved in one workgroup
constexpr int kCoarseThreads = 1024;
constexpr int kCoarseLanes = 4;       // lanes per row in the coarsest-level kernel
// field counts whose levels sweep on an ELL copy (index: fields per node): scalar rows
// (27 entries; 96^3 conduction 10.8 -> 9.7 ms per PCG solve).  The flow's 108-entry rows
// stay on the 8-lane CSR sweep: with ELL, one thread per row, the 48^3 Newton solve took
// 155-157 ms against 144 ms.
constexpr bool kEllFields[5] = {false, true, false, false, false};

__device__ __forceinline__ int64_t dof_of(int64_t node, int f, int64_t n_nodes, int nf, int fm)
{
    return fm ? (int64_t)f * n_nodes + node : node * nf + f;
}

// Connectivity of the lexicographic grid: corner a of element (ex,ey,ez) is node
// (ex + (a&1), ey + ((a>>1)&1), ez + ((a>>2)&1)).
__global__ void __launch_bounds__(kThreads) k_mg_conn(int64_t nx, int64_t ny, int64_t n_el, int32_t* __restrict__ conn)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < 8 * n_el;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int a = (int)(t / n_el);
        const int64_t e = t % n_el;
        const int64_t ex = e % nx, r = e / nx, ey = r % ny, ez = r / ny;
        const int64_t i = ex + (a & 1), j = ey + ((a >> 1) & 1), k = ez + ((a >> 2) & 1);
        conn[t] = (int32_t)(i + (nx + 1) * (j + (ny + 1) * k));
    }
}

// Coarse node v = (i,j,k) takes the values of fine node (2i,2j,2k): coordinates, the
// 4-field state (when given) and the Dirichlet flags of every field (when given).
__global__ void __launch_bounds__(kThreads) k_mg_inject(int64_t cx, int64_t cy, int64_t cn, int64_t fx, int64_t fy,
                                                        int64_t fn, int nf, int fm,
                                                        const double* __restrict__ fcoords,
                                                        double* __restrict__ ccoords,
                                                        const double* __restrict__ fstate,
                                                        double* __restrict__ cstate,
                                                        const uint8_t* __restrict__ fmask,
                                                        uint8_t* __restrict__ cmask)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < cn; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = v % (cx + 1), r = v / (cx + 1), j = r % (cy + 1), k = r / (cy + 1);
        const int64_t w = 2 * i + (fx + 1) * (2 * j + (fy + 1) * (2 * k));
#pragma unroll
        for (int c = 0; c < 3; ++c) ccoords[c * cn + v] = fcoords[c * fn + w];
        if (fstate) {
#pragma unroll
            for (int c = 0; c < 4; ++c) cstate[c * cn + v] = fstate[c * fn + w];
        }
        if (fmask) {
            for (int f = 0; f < nf; ++f) cmask[dof_of(v, f, cn, nf, fm)] = fmask[dof_of(w, f, fn, nf, fm)];
        }
    }
}

// rows x n_nodes nodal values (a boundary form's target) injected like the state
__global__ void __launch_bounds__(kThreads) k_mg_inject_nodal(int64_t cx, int64_t cy, int64_t cn, int64_t fx,
                                                              int64_t fy, int64_t fn, int rows,
                                                              const double* __restrict__ f, double* __restrict__ c)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < cn; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = v % (cx + 1), r = v / (cx + 1), j = r % (cy + 1), k = r / (cy + 1);
        const int64_t w = 2 * i + (fx + 1) * (2 * j + (fy + 1) * (2 * k));
        for (int q = 0; q < rows; ++q) c[q * cn + v] = f[q * fn + w];
    }
}

// Boundary faces of the next level: the fine face (element (ex,ey,ez), local face
// 2 axis + side) stands for the coarse face of element (ex/2, ey/2, ez/2) with the same
// local face when its two in-plane indices are even and its index along the axis is even
// for side 0, odd for side 1 (so each coarse face keeps exactly one of its four fine
// faces); other faces, and faces out of range (reported by the fine level's assembly),
// drop out.  The kept faces are appended through *count, in no fixed order: the face
// scatter adds an element's faces in a fixed order whatever the list order.
__global__ void __launch_bounds__(kThreads) k_mg_faces(int64_t n, const int32_t* __restrict__ fe,
                                                       const uint8_t* __restrict__ fi, int64_t nx, int64_t ny,
                                                       int64_t nz, int* __restrict__ count, int32_t* __restrict__ ce,
                                                       uint8_t* __restrict__ cf)
{
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < n; f += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = fe[f];
        const int lf = fi[f];
        if (e < 0 || e >= nx * ny * nz || lf > 5) continue;
        const int64_t idx[3] = {e % nx, (e / nx) % ny, e / (nx * ny)};
        const int axis = lf >> 1, side = lf & 1;
        bool keep = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) keep = keep && (idx[a] & 1) == (a == axis ? side : 0);
        if (keep) {
            const int slot = atomicAdd(count, 1);
            ce[slot] = (int32_t)(idx[0] / 2 + (nx / 2) * (idx[1] / 2 + (ny / 2) * (idx[2] / 2)));
            cf[slot] = (uint8_t)lf;
        }
    }
}

// Coarse element (ex,ey,ez): the mean of the fine elements (2ex+a, 2ey+b, 2ez+c), summed
// with the first axis fastest.
__global__ void __launch_bounds__(kThreads) k_mg_coarsen_elem(int64_t cx, int64_t cy, int64_t cz, int64_t fx,
                                                              int64_t fy, const double* __restrict__ f,
                                                              double* __restrict__ c)
{
    const int64_t n = cx * cy * cz;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ex = e % cx, r = e / cx, ey = r % cy, ez = r / cy;
        double sum = 0.0;
        for (int k = 0; k < 2; ++k)
            for (int j = 0; j < 2; ++j)
                for (int i = 0; i < 2; ++i) sum += f[(2 * ex + i) + fx * ((2 * ey + j) + fy * (2 * ez + k))];
        c[e] = sum / 8.0;
    }
}

// A = a K + b M on one pattern, Dirichlet rows unit rows and their columns zero
__global__ void __launch_bounds__(kThreads) k_mg_combine(int64_t n, const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ ci, const double* __restrict__ K,
                                                         const double* __restrict__ M, double a, double b,
                                                         const uint8_t* __restrict__ mask, double* __restrict__ A)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const bool fixed = mask && mask[r];
        for (int k = rp[r]; k < rp[r + 1]; ++k) {
            const int c = ci[k];
            double v = a * K[k] + b * M[k];
            if (fixed || (mask && mask[c])) v = c == r ? 1.0 : 0.0;
            A[k] = v;
        }
    }
}

__global__ void k_mg_zero_int(int* p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// dinv[i] = 1 / A_ii, 0 where the diagonal is 0; kDiagLanes lanes scan a row, and the
// one that meets column i writes (a row holds its diagonal once)
constexpr int kDiagLanes = 8;
__global__ void __launch_bounds__(kThreads) k_mg_dinv(int64_t n, const int32_t* __restrict__ rp,
                                                      const int32_t* __restrict__ ci, const double* __restrict__ A,
                                                      double* __restrict__ dinv)
{
    const int lane = threadIdx.x % kDiagLanes;
    const int64_t rows_per_pass = (int64_t)gridDim.x * (kThreads / kDiagLanes);
    for (int64_t i = (blockIdx.x * (int64_t)kThreads + threadIdx.x) / kDiagLanes; i < n; i += rows_per_pass) {
        const int k1 = rp[i + 1];
        bool found = false;
        double di = 0.0;
        for (int k = rp[i] + lane; k < k1; k += kDiagLanes)
            if (ci[k] == i) {
                di = A[k];
                found = true;
            }
        const unsigned long long hit = __ballot(found);
        const int base = (threadIdx.x % 64) / kDiagLanes * kDiagLanes;
        const unsigned long long mine = (hit >> base) & ((1ull << kDiagLanes) - 1);
        if (found) dinv[i] = di != 0.0 ? 1.0 / di : 0.0;
        else if (mine == 0 && lane == 0) dinv[i] = 0.0;
    }
}

enum SweepMode { kSweep = 0, kFirst = 1, kResidual = 2 };

// ELL columns of a CSR pattern (fixed with the pattern)
__global__ void __launch_bounds__(kThreads) k_mg_ell_cols(int64_t n, int width, const int32_t* __restrict__ rp,
                                                          const int32_t* __restrict__ ci, int32_t* __restrict__ ecol)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int k0 = rp[i], len = rp[i + 1] - k0;
        for (int k = 0; k < width; ++k) ecol[k * n + i] = k < len ? ci[k0 + k] : (int32_t)i;
    }
}

// ELL values of the level's operator
__global__ void __launch_bounds__(kThreads) k_mg_ell_vals(int64_t n, int width, const int32_t* __restrict__ rp,
                                                          const double* __restrict__ A, double* __restrict__ eval)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int k0 = rp[i], len = rp[i + 1] - k0;
        for (int k = 0; k < width; ++k) eval[k * n + i] = k < len ? A[k0 + k] : 0.0;
    }
}

// The sweep of k_mg_sweep on the ELL copy, one row per thread: consecutive rows read
// consecutive addresses of every slot.
template <int MODE>
__global__ void __launch_bounds__(kThreads) k_mg_sweep_ell(int64_t n, int width, const int32_t* __restrict__ ecol,
                                                           const double* __restrict__ eval,
                                                           const double* __restrict__ dinv,
                                                           const double* __restrict__ b,
                                                           const double* __restrict__ in, double* __restrict__ out,
                                                           double omega)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
#pragma unroll 9
        for (int k = 0; k < width; ++k) s = fma(eval[k * n + i], in[ecol[k * n + i]], s);
        if (MODE == kSweep) out[i] = in[i] + omega * dinv[i] * (b[i] - s);
        else out[i] = b[i] - s;
    }
}

// kSweep:    out = in + omega dinv (b - A in)
// kFirst:    out = omega dinv b            (the sweep from x = 0; A and in unused)
// kResidual: out = b - A in
// LANES consecutive threads share a row; every lane of a row group runs the same trip
// count, so the group's shuffles see only active lanes.
template <int LANES, int MODE>
__global__ void __launch_bounds__(kThreads) k_mg_sweep(int64_t n, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci,
                                                       const double* __restrict__ A,
                                                       const double* __restrict__ dinv,
                                                       const double* __restrict__ b,
                                                       const double* __restrict__ in, double* __restrict__ out,
                                                       double omega)
{
    const int lane = threadIdx.x % LANES;
    const int64_t rows_per_pass = (int64_t)gridDim.x * (kThreads / LANES);
    for (int64_t row = (blockIdx.x * (int64_t)kThreads + threadIdx.x) / LANES; row < n; row += rows_per_pass) {
        double s = 0.0;
        if (MODE != kFirst) {
            const int k0 = rp[row], k1 = rp[row + 1];
#pragma unroll 4
            for (int k = k0 + lane; k < k1; k += LANES) s = fma(A[k], in[ci[k]], s);
#pragma unroll
            for (int off = LANES / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, LANES);
        }
        if (lane == 0) {
            if (MODE == kFirst) out[row] = omega * dinv[row] * b[row];
            else if (MODE == kSweep) out[row] = in[row] + omega * dinv[row] * (b[row] - s);
            else out[row] = b[row] - s;
        }
    }
}

// k_mg_sweep (kSweep, kResidual) for node-major rows of four fully coupled fields. Row
// (v, f) starts at 16 P_v + 4 deg_v f (P_v, deg_v: node v's offset and degree in the node
// graph) and its entry o has column 4 w + o % 4, w the (o / 4)-th neighbour of v, so the
// columns come from the node graph (27 indices shared by 432 entries) instead of col_idx:
// 8 bytes per entry read instead of 12.  Lanes take the same entries in the same order as
// k_mg_sweep<8, MODE>, so the sums are identical.
template <int MODE>
__global__ void __launch_bounds__(kThreads) k_mg_sweep_nodes(int64_t n, const int32_t* __restrict__ np,
                                                             const int32_t* __restrict__ nb,
                                                             const double* __restrict__ A,
                                                             const double* __restrict__ dinv,
                                                             const double* __restrict__ b,
                                                             const double* __restrict__ in,
                                                             double* __restrict__ out, double omega)
{
    constexpr int LANES = 8;
    const int lane = threadIdx.x % LANES;
    const int g = lane % 4;
    const int64_t rows_per_pass = (int64_t)gridDim.x * (kThreads / LANES);
    for (int64_t row = (blockIdx.x * (int64_t)kThreads + threadIdx.x) / LANES; row < n; row += rows_per_pass) {
        const int64_t v = row / 4;
        const int p0 = np[v], deg = np[v + 1] - p0;
        const int len = 4 * deg;
        const double* a = A + 16 * (int64_t)p0 + (int64_t)len * (row % 4);
        const int32_t* w = nb + p0;
        double s = 0.0;
#pragma unroll 4
        for (int o = lane; o < len; o += LANES) s = fma(a[o], in[4 * (int64_t)w[o / 4] + g], s);
#pragma unroll
        for (int off = LANES / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, LANES);
        if (lane == 0) {
            if (MODE == kSweep) out[row] = in[row] + omega * dinv[row] * (b[row] - s);
            else out[row] = b[row] - s;
        }
    }
}

// bc = R rf on every coarse DOF (0 on coarse Dirichlet rows): coarse node (i,j,k) gathers
// the fine nodes (2i+di, 2j+dj, 2k+dk), di,dj,dk in {-1,0,1}, with weight 1/2 per nonzero
// offset.
__global__ void __launch_bounds__(kThreads) k_mg_restrict(int64_t cx, int64_t cy, int64_t cn, int64_t fx, int64_t fy,
                                                          int64_t fz, int64_t fn, int nf, int fm,
                                                          const double* __restrict__ rf,
                                                          const uint8_t* __restrict__ cmask,
                                                          double* __restrict__ bc)
{
    // one thread per (coarse node, field): the fields of a node are adjacent threads
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < cn * nf; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = t / nf;
        const int f = (int)(t % nf);
        const int64_t i = v % (cx + 1), r = v / (cx + 1), j = r % (cy + 1), k = r / (cy + 1);
        double acc = 0.0;
        for (int dk = -1; dk <= 1; ++dk) {
            const int64_t c = 2 * k + dk;
            if (c < 0 || c > fz) continue;
            const double wz = dk ? 0.5 : 1.0;
            for (int dj = -1; dj <= 1; ++dj) {
                const int64_t bb = 2 * j + dj;
                if (bb < 0 || bb > fy) continue;
                const double wy = dj ? wz * 0.5 : wz;
                for (int di = -1; di <= 1; ++di) {
                    const int64_t a = 2 * i + di;
                    if (a < 0 || a > fx) continue;
                    const double w = di ? wy * 0.5 : wy;
                    const int64_t node = a + (fx + 1) * (bb + (fy + 1) * c);
                    acc = fma(w, rf[dof_of(node, f, fn, nf, fm)], acc);
                }
            }
        }
        const int64_t d = dof_of(v, f, cn, nf, fm);
        bc[d] = (cmask && cmask[d]) ? 0.0 : acc;
    }
}

// x = (ADD ? x : 0) + P xc: fine node (a,b,c) interpolates from the coarse nodes
// (floor(a/2) or a/2 +- 1/2 per axis), weight 1/2 per odd index.
template <bool ADD>
__global__ void __launch_bounds__(kThreads) k_mg_prolong(int64_t fx, int64_t fy, int64_t fn, int64_t cx, int64_t cy,
                                                         int64_t cn, int nf, int fm, const double* __restrict__ xc,
                                                         double* __restrict__ x)
{
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < fn; w += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = w % (fx + 1), r = w / (fx + 1), bb = r % (fy + 1), c = r / (fy + 1);
        const int na = (a & 1) ? 2 : 1, nb = (bb & 1) ? 2 : 1, nc = (c & 1) ? 2 : 1;
        const double wt = ((a & 1) ? 0.5 : 1.0) * ((bb & 1) ? 0.5 : 1.0) * ((c & 1) ? 0.5 : 1.0);
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int sc = 0; sc < nc; ++sc) {
            const int64_t kc = (c >> 1) + sc;
            for (int sb = 0; sb < nb; ++sb) {
                const int64_t jc = (bb >> 1) + sb;
                for (int sa = 0; sa < na; ++sa) {
                    const int64_t ic = (a >> 1) + sa;
                    const int64_t node = ic + (cx + 1) * (jc + (cy + 1) * kc);
                    for (int f = 0; f < nf; ++f) acc[f] = fma(wt, xc[dof_of(node, f, cn, nf, fm)], acc[f]);
                }
            }
        }
        for (int f = 0; f < nf; ++f) {
            const int64_t d = dof_of(w, f, fn, nf, fm);
            x[d] = ADD ? x[d] + acc[f] : acc[f];
        }
    }
}

// The coarsest level: `sweeps` damped Jacobi sweeps from x = 0 in one workgroup, the
// iterate alternating between two LDS arrays (n <= kCoarseMax), kCoarseLanes lanes per row.
// CACHED (n <= kCoarseGroups, rows of at most kCoarseLanes * kCoarseCache entries): each
// row group keeps its row's entries and columns in registers for all sweeps, so a sweep
// reads only LDS; otherwise the entries are read from memory (L2) every sweep.
constexpr int kCoarseGroups = kCoarseThreads / kCoarseLanes;
constexpr int kCoarseCache = 32;
template <bool CACHED>
__global__ void __launch_bounds__(kCoarseThreads) k_mg_coarse(int n, const int32_t* __restrict__ rp,
                                                              const int32_t* __restrict__ ci,
                                                              const double* __restrict__ A,
                                                              const double* __restrict__ dinv,
                                                              const double* __restrict__ b, double* __restrict__ x,
                                                              double omega, int sweeps)
{
    __shared__ double xs[2][kCoarseMax];
    const int lane = threadIdx.x % kCoarseLanes;
    const int group = threadIdx.x / kCoarseLanes;
    if (sweeps <= 0) {
        for (int i = threadIdx.x; i < n; i += kCoarseThreads) x[i] = 0.0;
        return;
    }
    for (int i = threadIdx.x; i < n; i += kCoarseThreads) xs[0][i] = omega * dinv[i] * b[i];
    int cur = 0;
    if (CACHED) {
        const int row = group;  // n <= kCoarseGroups: one row per group
        const bool live = row < n;
        double a[kCoarseCache];
        int c[kCoarseCache];
        const int k0 = live ? rp[row] : 0, k1 = live ? rp[row + 1] : 0;
#pragma unroll
        for (int t = 0; t < kCoarseCache; ++t) {
            const int k = k0 + lane + t * kCoarseLanes;
            const bool in = k < k1;
            a[t] = in ? A[k] : 0.0;
            c[t] = in ? ci[k] : 0;  // a padded slot reads x[0] with weight 0
        }
        const double di = live ? omega * dinv[row] : 0.0, bi = live ? b[row] : 0.0;
        __syncthreads();
        for (int s = 1; s < sweeps; ++s) {
            const double* xi = xs[cur];
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < kCoarseCache; ++t) acc = fma(a[t], xi[c[t]], acc);
#pragma unroll
            for (int off = kCoarseLanes / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kCoarseLanes);
            if (live && lane == 0) xs[cur ^ 1][row] = xi[row] + di * (bi - acc);
            __syncthreads();
            cur ^= 1;
        }
    } else {
        __syncthreads();
        for (int s = 1; s < sweeps; ++s) {
            const double* xi = xs[cur];
            double* xo = xs[cur ^ 1];
            for (int row = group; row < n; row += kCoarseGroups) {
                double acc = 0.0;
                for (int k = rp[row] + lane; k < rp[row + 1]; k += kCoarseLanes) acc = fma(A[k], xi[ci[k]], acc);
#pragma unroll
                for (int off = kCoarseLanes / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kCoarseLanes);
                if (lane == 0) xo[row] = xi[row] + omega * dinv[row] * (b[row] - acc);
            }
            __syncthreads();
            cur ^= 1;
        }
    }
    for (int i = threadIdx.x; i < n; i += kCoarseThreads) x[i] = xs[cur][i];
}

unsigned grid_for(int64_t work, int per_block)
{
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(kMaxBlocks, (work + per_block - 1) / per_block));
}

void launch_sweep(int mode, const mf_mg_s::Level& Lv, int nf, const double* b, const double* in, double* out,
                  double omega, hipStream_t s)
{
    const int64_t n = Lv.n_rows;
    const int32_t* rp = Lv.Pv->row_ptr;
    const int32_t* ci = Lv.Pv->col_idx;
    if (Lv.eval && mode != kFirst) {
        const unsigned g = grid_for(n, kThreads);
        if (mode == kSweep)
            k_mg_sweep_ell<kSweep><<<g, kThreads, 0, s>>>(n, Lv.width, Lv.ecol, Lv.eval, Lv.dinv, b, in, out, omega);
        else
            k_mg_sweep_ell<kResidual><<<g, kThreads, 0, s>>>(n, Lv.width, Lv.ecol, Lv.eval, Lv.dinv, b, in, out, omega);
        return;
    }
    if (nf >= 4) {
        const unsigned g = grid_for(n * 8, kThreads);
        if (Lv.node_cols && mode != kFirst) {
            const int32_t* np = Lv.Pv->nbr_ptr;
            const int32_t* nb = Lv.Pv->nbr;
            if (mode == kSweep)
                k_mg_sweep_nodes<kSweep><<<g, kThreads, 0, s>>>(n, np, nb, Lv.Kv, Lv.dinv, b, in, out, omega);
            else
                k_mg_sweep_nodes<kResidual><<<g, kThreads, 0, s>>>(n, np, nb, Lv.Kv, Lv.dinv, b, in, out, omega);
            return;
        }
        if (mode == kFirst) k_mg_sweep<8, kFirst><<<g, kThreads, 0, s>>>(n, rp, ci, Lv.Kv, Lv.dinv, b, in, out, omega);
        else if (mode == kSweep) k_mg_sweep<8, kSweep><<<g, kThreads, 0, s>>>(n, rp, ci, Lv.Kv, Lv.dinv, b, in, out, omega);
        else k_mg_sweep<8, kResidual><<<g, kThreads, 0, s>>>(n, rp, ci, Lv.Kv, Lv.dinv, b, in, out, omega);
    } else {
        const unsigned g = grid_for(n * 4, kThreads);
        if (mode == kFirst) k_mg_sweep<4, kFirst><<<g, kThreads, 0, s>>>(n, rp, ci, Lv.Kv, Lv.dinv, b, in, out, omega);
        else if (mode == kSweep) k_mg_sweep<4, kSweep><<<g, kThreads, 0, s>>>(n, rp, ci, Lv.Kv, Lv.dinv, b, in, out, omega);
        else k_mg_sweep<4, kResidual><<<g, kThreads, 0, s>>>(n, rp, ci, Lv.Kv, Lv.dinv, b, in, out, omega);
    }
}

// count sweeps; the first from x = 0 when *cur is null.  Buffers alternate: each sweep
// writes the buffer *cur does not hold.
void sweeps(const mf_mg_s::Level& Lv, int nf, const double* b, double** cur, double* first_dst, double* other,
            int count, double omega, hipStream_t s)
{
    for (int k = 0; k < count; ++k) {
        double* dst = *cur == nullptr ? first_dst : (*cur == first_dst ? other : first_dst);
        launch_sweep(*cur == nullptr ? kFirst : kSweep, Lv, nf, b, *cur, dst, omega, s);
        *cur = dst;
    }
}

// out = V(l, b); out and the level's t are the two sweep buffers.
void vcycle(const mf_mg_s* mg, int l, const double* b, double* out, hipStream_t s)
{
    const mf_mg_s::Level& Lv = mg->L[l];
    const int nf = mg->nf, fm = mg->fm;
    const double omega = mg->opts.omega;
    if (l == mg->n_levels - 1) {
        const int cs = mg->opts.coarse_sweeps;
        // a hexahedral grid row holds at most 27 nodes x 4 fields = 108 <= 128 entries
        static_assert(27 * 4 <= kCoarseLanes * kCoarseCache, "row cache too small");
        if (Lv.n_rows <= kCoarseGroups) {
            k_mg_coarse<true><<<1, kCoarseThreads, 0, s>>>((int)Lv.n_rows, Lv.Pv->row_ptr, Lv.Pv->col_idx, Lv.Kv,
                                                           Lv.dinv, b, out, omega, cs);
        } else if (Lv.n_rows <= kCoarseMax) {
            k_mg_coarse<false><<<1, kCoarseThreads, 0, s>>>((int)Lv.n_rows, Lv.Pv->row_ptr, Lv.Pv->col_idx, Lv.Kv,
                                                            Lv.dinv, b, out, omega, cs);
        } else {
            double* cur = nullptr;
            double* first = (cs % 2 == 1) ? out : Lv.t;  // the last of cs sweeps writes out
            sweeps(Lv, nf, b, &cur, first, first == out ? Lv.t : out, cs, omega, s);
            if (cs == 0) launch_sweep(kFirst, Lv, nf, b, nullptr, out, 0.0, s);  // x = 0
        }
        return;
    }
    const mf_mg_s::Level& Lc = mg->L[l + 1];
    const int pre = mg->opts.pre_sweeps, post = mg->opts.post_sweeps;
    double* cur = nullptr;
    // pick the first buffer so that the last write of the cycle on this level lands in out
    double* first;
    if (pre > 0) first = ((pre + post) % 2 == 1) ? out : Lv.t;
    else first = (post % 2 == 0) ? out : Lv.t;
    double* other = first == out ? Lv.t : out;
    sweeps(Lv, nf, b, &cur, first, other, pre, omega, s);
    const double* res = b;  // the residual of x = 0
    if (cur) {
        double* rbuf = cur == first ? other : first;
        launch_sweep(kResidual, Lv, nf, b, cur, rbuf, omega, s);
        res = rbuf;
    }
    k_mg_restrict<<<grid_for(Lc.n_nodes * nf, kThreads), kThreads, 0, s>>>(Lc.nx, Lc.ny, Lc.n_nodes, Lv.nx, Lv.ny, Lv.nz,
                                                                      Lv.n_nodes, nf, fm, res,
                                                                      mg->has_mask ? Lc.mask : nullptr, Lc.b);
    vcycle(mg, l + 1, Lc.b, Lc.x, s);
    if (cur) {
        k_mg_prolong<true><<<grid_for(Lv.n_nodes, kThreads), kThreads, 0, s>>>(Lv.nx, Lv.ny, Lv.n_nodes, Lc.nx, Lc.ny,
                                                                              Lc.n_nodes, nf, fm, Lc.x, cur);
    } else {
        cur = first;
        k_mg_prolong<false><<<grid_for(Lv.n_nodes, kThreads), kThreads, 0, s>>>(Lv.nx, Lv.ny, Lv.n_nodes, Lc.nx,
                                                                               Lc.ny, Lc.n_nodes, nf, fm, Lc.x, cur);
    }
    for (int k = 0; k < post; ++k) {
        double* dst = cur == first ? other : first;
        launch_sweep(kSweep, Lv, nf, b, cur, dst, omega, s);
        cur = dst;
    }
}

mf_status mg_apply_cb(void* ctx, const double* r, double* z, hipStream_t s)
{
    vcycle((const mf_mg_s*)ctx, 0, r, z, s);
    MF_HIP(hipGetLastError());
    return MF_OK;
}

}  // namespace

// The cycle for A = wa Ka + wb Kb (two scalar forms, fa with the element field elem_param,
// fb without), with the Dirichlet elimination, on every level; A0 is level 0's operator.
mf_status mg_update_combined(mf_mg_t* mg, const mf_form* fa, const double* elem_param, double wa,
                             const mf_form* fb, double wb, const double* coords, const uint8_t* dirichlet,
                             const mf_quadrature* quad, const double* A0, hipStream_t s)
{
    mg->updated = false;
    mg->has_mask = dirichlet != nullptr;
    mg->L[0].Kv = A0;
    for (int l = 1; l < mg->n_levels; ++l) {
        mf_mg_s::Level& Lf = mg->L[l - 1];
        mf_mg_s::Level& Lc = mg->L[l];
        k_mg_inject<<<grid_for(Lc.n_nodes, kThreads), kThreads, 0, s>>>(
            Lc.nx, Lc.ny, Lc.n_nodes, Lf.nx, Lf.ny, Lf.n_nodes, mg->nf, mg->fm, l == 1 ? coords : Lf.coords,
            Lc.coords, nullptr, Lc.state, dirichlet ? (l == 1 ? dirichlet : Lf.mask) : nullptr, Lc.mask);
        if (elem_param)
            k_mg_coarsen_elem<<<grid_for(Lc.nx * Lc.ny * Lc.nz, kThreads), kThreads, 0, s>>>(
                Lc.nx, Lc.ny, Lc.nz, Lf.nx, Lf.ny, l == 1 ? elem_param : Lf.elem, Lc.elem);
        MF_HIP(hipGetLastError());
        // Kb into the level's sweep buffers would not fit (nnz > rows): assemble it into K,
        // Ka into a scratch of nnz, then combine into K
        double* Ka = nullptr;
        if (hipMalloc(&Ka, sizeof(double) * std::max<int64_t>(Lc.P->nnz, 1)) != hipSuccess)
            return set_error(MF_ERR_OOM, "multigrid workspace allocation failed");
        struct FreeKa {
            double* p;
            hipStream_t s;
            ~FreeKa() {
                (void)hipStreamSynchronize(s);
                (void)hipFree(p);
            }
        } fka{Ka, s};
        mf_fields Fa{};
        Fa.elem_param = elem_param ? Lc.elem : nullptr;
        mf_status st = mf_assemble(Lc.P, fa, Lc.coords, &Fa, quad, MF_F64, Ka, Lc.d, s);
        if (st != MF_OK) return st;
        mf_fields Fb{};
        st = mf_assemble(Lc.P, fb, Lc.coords, &Fb, quad, MF_F64, Lc.K, Lc.d, s);
        if (st != MF_OK) return st;
        k_mg_combine<<<grid_for(Lc.n_rows, kThreads), kThreads, 0, s>>>(Lc.n_rows, Lc.P->row_ptr, Lc.P->col_idx, Ka,
                                                                       Lc.K, wa, wb, dirichlet ? Lc.mask : nullptr,
                                                                       Lc.K);
        MF_HIP(hipGetLastError());
        int64_t bad = -1;
        st = mf_status_poll(Lc.P, &bad);
        if (st != MF_OK) return st;
    }
    for (int l = 0; l < mg->n_levels; ++l) {
        const mf_mg_s::Level& Lv = mg->L[l];
        k_mg_dinv<<<grid_for(Lv.n_rows, kThreads), kThreads, 0, s>>>(Lv.n_rows, Lv.Pv->row_ptr, Lv.Pv->col_idx, Lv.Kv,
                                                                     Lv.dinv);
        if (Lv.eval)
            k_mg_ell_vals<<<grid_for(Lv.n_rows, kThreads), kThreads, 0, s>>>(Lv.n_rows, Lv.width, Lv.Pv->row_ptr,
                                                                             Lv.Kv, Lv.eval);
    }
    MF_HIP(hipGetLastError());
    MF_HIP(hipStreamSynchronize(s));
    mg->updated = true;
    return MF_OK;
}

mf_status mg_bind_pcg(const mf_mg_t* mg, int64_t n_rows, const double* values, PcgArgs* a)
{
    if (!mg->updated) return set_error(MF_ERR_ARG, "call mf_mg_update before the solve");
    if (n_rows != mg->L[0].n_rows)
        return set_error(MF_ERR_ARG, "multigrid level 0 has %lld rows, system %lld", (long long)mg->L[0].n_rows,
                         (long long)n_rows);
    if (values != mg->L[0].Kv) return set_error(MF_ERR_ARG, "the multigrid cycle was updated for a different matrix");
    a->precond = MF_PRECOND_EXTERNAL;
    a->apply = mg_apply_cb;
    a->apply_ctx = (void*)mg;
    a->apply_graph_safe = 1;
    return MF_OK;
}

}  // namespace mf

using namespace mf;

static void free_mg(mf_mg_s* mg)
{
    if (!mg) return;
    for (int l = 1; l < mg->n_levels; ++l)
        if (mg->L[l].P) mf_pattern_destroy(mg->L[l].P);
    for (void* p : mg->owned) (void)hipFree(p);
    delete mg;
}

extern "C" mf_status mf_mg_create(const mf_pattern_t* P, const mf_mg_opts* opts, void* stream, mf_mg_t** out)
{
    if (!out) return set_error(MF_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!P || !opts) return set_error(MF_ERR_ARG, "pattern or opts is NULL");
    if (P->dim != 3 || P->nen != 8 || !P->is_grid)
        return set_error(MF_ERR_UNSUPPORTED, "multigrid needs a structured grid of 8-node hexahedra");
    if (!P->full_coupling) return set_error(MF_ERR_UNSUPPORTED, "multigrid needs full field coupling");
    const int max_levels = opts->max_levels == 0 ? MF_MG_MAX_LEVELS : opts->max_levels;
    if (max_levels < 1 || max_levels > MF_MG_MAX_LEVELS)
        return set_error(MF_ERR_ARG, "max_levels must be 0..%d", MF_MG_MAX_LEVELS);
    if (opts->coarse_rows < 0 || opts->pre_sweeps < 0 || opts->post_sweeps < 0 || opts->coarse_sweeps < 0)
        return set_error(MF_ERR_ARG, "coarse_rows and sweep counts must be >= 0");
    if (!(opts->omega > 0.0 && opts->omega <= 1.0)) return set_error(MF_ERR_ARG, "omega must be in (0, 1]");
    for (int l = 0; l < MF_MG_MAX_LEVELS; ++l)
        if (!(opts->tau_m[l] >= 0.0) || !(opts->tau_c[l] >= 0.0))
            return set_error(MF_ERR_ARG, "tau_m and tau_c must be >= 0");
    const int64_t coarse_rows = opts->coarse_rows == 0 ? 512 : opts->coarse_rows;
    hipStream_t s = (hipStream_t)stream;

    mf_mg_s* mg = new (std::nothrow) mf_mg_s();
    if (!mg) return set_error(MF_ERR_OOM, "host allocation failed");
    mg->opts = *opts;
    mg->nf = P->nf;
    mg->fm = P->numbering == MF_FIELD_MAJOR ? 1 : 0;
    auto dalloc = [&](size_t bytes) -> void* {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(bytes, 8)) != hipSuccess) return nullptr;
        mg->owned.push_back(p);
        return p;
    };
    // level grids
    int64_t nx = P->gx, ny = P->gy, nz = P->gz;
    int n = 0;
    for (;;) {
        mf_mg_s::Level& Lv = mg->L[n];
        Lv.nx = nx;
        Lv.ny = ny;
        Lv.nz = nz;
        Lv.n_nodes = (nx + 1) * (ny + 1) * (nz + 1);
        Lv.n_rows = Lv.n_nodes * P->nf;
        ++n;
        const bool even = nx % 2 == 0 && ny % 2 == 0 && nz % 2 == 0;
        if (n >= max_levels || Lv.n_rows <= coarse_rows || !even) break;
        nx /= 2;
        ny /= 2;
        nz /= 2;
    }
    mg->n_levels = n;
    mg->L[0].Pv = P;
    mf_status st = MF_OK;
    for (int l = 0; l < n && st == MF_OK; ++l) {
        mf_mg_s::Level& Lv = mg->L[l];
        const size_t rows = (size_t)Lv.n_rows, nodes = (size_t)Lv.n_nodes;
        Lv.dinv = (double*)dalloc(sizeof(double) * rows);
        Lv.t = (double*)dalloc(sizeof(double) * rows);
        if (!Lv.dinv || !Lv.t) {
            st = set_error(MF_ERR_OOM, "multigrid workspace allocation failed");
            break;
        }
        if (l == 0) continue;
        Lv.x = (double*)dalloc(sizeof(double) * rows);
        Lv.b = (double*)dalloc(sizeof(double) * rows);
        Lv.d = (double*)dalloc(sizeof(double) * rows);
        Lv.coords = (double*)dalloc(sizeof(double) * 3 * nodes);
        Lv.state = (double*)dalloc(sizeof(double) * 4 * nodes);
        Lv.mask = (uint8_t*)dalloc(rows);
        const int64_t n_el = Lv.nx * Lv.ny * Lv.nz;
        Lv.elem = (double*)dalloc(sizeof(double) * (size_t)n_el);
        int32_t* conn = nullptr;
        if (hipMalloc(&conn, sizeof(int32_t) * 8 * (size_t)n_el) != hipSuccess) conn = nullptr;
        if (!Lv.x || !Lv.b || !Lv.d || !Lv.coords || !Lv.state || !Lv.mask || !Lv.elem || !conn) {
            if (conn) (void)hipFree(conn);
            st = set_error(MF_ERR_OOM, "multigrid workspace allocation failed");
            break;
        }
        k_mg_conn<<<grid_for(8 * n_el, kThreads), kThreads, 0, s>>>(Lv.nx, Lv.ny, n_el, conn);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            (void)hipFree(conn);
            st = hip_error(e, "k_mg_conn");
            break;
        }
        mf_mesh mesh{3, Lv.n_nodes, n_el, conn};
        mf_dofs dofs{P->nf, nullptr, P->numbering};
        st = mf_pattern(&mesh, MF_HEX8, 1, &dofs, stream, &Lv.P);  // synchronises the stream
        (void)hipFree(conn);
        if (st != MF_OK) break;
        if (!Lv.P->is_grid) {
            st = set_error(MF_ERR_HIP, "multigrid level %d is not recognised as a grid", l);
            break;
        }
        Lv.Pv = Lv.P;
        Lv.K = (double*)dalloc(sizeof(double) * (size_t)Lv.P->nnz);
        Lv.Kv = Lv.K;
        if (!Lv.K) st = set_error(MF_ERR_OOM, "multigrid workspace allocation failed");
    }
    // node-major 4-field levels (full coupling: 16 entries per node pair) take the sweep
    // that reads the node graph instead of the column indices
    for (int l = 0; l < n && st == MF_OK; ++l) {
        mf_mg_s::Level& Lv = mg->L[l];
        Lv.node_cols = P->nf == 4 && !mg->fm && Lv.Pv->nnz == 16 * Lv.Pv->n_pairs;
    }
    // ELL copies of every level but the one-workgroup coarsest (rows of a hexahedral grid
    // hold at most 27 nodes x nf entries)
    const int ell_width = 27 * P->nf;
    for (int l = 0; l < n && st == MF_OK && kEllFields[P->nf]; ++l) {
        mf_mg_s::Level& Lv = mg->L[l];
        if (l == n - 1 && Lv.n_rows <= kCoarseMax) break;
        Lv.width = ell_width;
        Lv.ecol = (int32_t*)dalloc(sizeof(int32_t) * ell_width * (size_t)Lv.n_rows);
        Lv.eval = (double*)dalloc(sizeof(double) * ell_width * (size_t)Lv.n_rows);
        if (!Lv.ecol || !Lv.eval) {
            st = set_error(MF_ERR_OOM, "multigrid workspace allocation failed");
            break;
        }
        k_mg_ell_cols<<<grid_for(Lv.n_rows, kThreads), kThreads, 0, s>>>(Lv.n_rows, ell_width, Lv.Pv->row_ptr,
                                                                         Lv.Pv->col_idx, Lv.ecol);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) st = hip_error(e, "k_mg_ell_cols");
    }
    if (st == MF_OK) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_error(e, "hipStreamSynchronize");
    }
    if (st != MF_OK) {
        (void)hipStreamSynchronize(s);
        free_mg(mg);
        return st;
    }
    *out = mg;
    return MF_OK;
}

extern "C" mf_status mf_mg_levels(const mf_mg_t* mg, int32_t* n_levels, int64_t* dims)
{
    if (!mg) return set_error(MF_ERR_ARG, "mg is NULL");
    if (n_levels) *n_levels = mg->n_levels;
    if (dims)
        for (int l = 0; l < mg->n_levels; ++l) {
            dims[3 * l] = mg->L[l].nx;
            dims[3 * l + 1] = mg->L[l].ny;
            dims[3 * l + 2] = mg->L[l].nz;
        }
    return MF_OK;
}

extern "C" mf_status mf_mg_update_ex(mf_mg_t* mg, const mf_form* form, const double* coords,
                                     const mf_fields* fields, const mf_bset* bsets, int32_t n_bsets,
                                     const mf_quadrature* quad, const double* K, void* stream)
{
    if (!mg || !form || !quad) return set_error(MF_ERR_ARG, "mg, form or quad is NULL");
    if (!coords || !K) return set_error(MF_ERR_ARG, "coords or K is NULL");
    if (fields && fields->nodal_src)
        return set_error(MF_ERR_UNSUPPORTED, "multigrid coarse levels take no nodal_src (the cycle needs no right side)");
    if (n_bsets < 0 || (n_bsets > 0 && !bsets)) return set_error(MF_ERR_ARG, "n_bsets < 0 or bsets NULL");
    for (int b = 0; b < n_bsets; ++b)
        if (bsets[b].n_faces < 0 || (bsets[b].n_faces > 0 && (!bsets[b].face_elem || !bsets[b].face_id)))
            return set_error(MF_ERR_ARG, "face set %d: n_faces < 0 or NULL face arrays", b);
    hipStream_t s = (hipStream_t)stream;
    const double* lin_state = fields ? (const double*)fields->lin_state : nullptr;
    const uint8_t* dirichlet = fields ? fields->dirichlet : nullptr;
    const double* elem_param = fields ? (const double*)fields->elem_param : nullptr;
    mg->updated = false;
    mg->has_mask = dirichlet != nullptr;
    mg->L[0].Kv = K;

    // the coarse face lists and targets live only for this call
    std::vector<void*> tmp;
    struct Free {
        std::vector<void*>* v;
        hipStream_t s;
        ~Free() {
            (void)hipStreamSynchronize(s);
            for (void* p : *v) (void)hipFree(p);
        }
    } fr{&tmp, s};
    auto talloc = [&](size_t bytes) -> void* {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(bytes, 8)) != hipSuccess) return nullptr;
        tmp.push_back(p);
        return p;
    };
    std::vector<const int32_t*> fe(n_bsets);
    std::vector<const uint8_t*> fi(n_bsets);
    std::vector<int64_t> nfc(n_bsets);
    std::vector<const double*> tg(n_bsets);
    for (int b = 0; b < n_bsets; ++b) {
        fe[b] = bsets[b].face_elem;
        fi[b] = bsets[b].face_id;
        nfc[b] = bsets[b].n_faces;
        tg[b] = bsets[b].target;
    }
    int* counter = n_bsets > 0 ? (int*)talloc(sizeof(int) * n_bsets) : nullptr;
    if (n_bsets > 0 && !counter) return set_error(MF_ERR_OOM, "multigrid face workspace allocation failed");

    for (int l = 1; l < mg->n_levels; ++l) {
        mf_mg_s::Level& Lf = mg->L[l - 1];
        mf_mg_s::Level& Lc = mg->L[l];
        const double* fc = l == 1 ? coords : Lf.coords;
        const double* fs = lin_state ? (l == 1 ? lin_state : Lf.state) : nullptr;
        const uint8_t* fmk = dirichlet ? (l == 1 ? dirichlet : Lf.mask) : nullptr;
        k_mg_inject<<<grid_for(Lc.n_nodes, kThreads), kThreads, 0, s>>>(Lc.nx, Lc.ny, Lc.n_nodes, Lf.nx, Lf.ny,
                                                                        Lf.n_nodes, mg->nf, mg->fm, fc, Lc.coords, fs,
                                                                        Lc.state, fmk, Lc.mask);
        if (elem_param) {
            k_mg_coarsen_elem<<<grid_for(Lc.nx * Lc.ny * Lc.nz, kThreads), kThreads, 0, s>>>(
                Lc.nx, Lc.ny, Lc.nz, Lf.nx, Lf.ny, l == 1 ? elem_param : Lf.elem, Lc.elem);
        }
        MF_HIP(hipGetLastError());
        if (n_bsets > 0) {
            k_mg_zero_int<<<1, 64, 0, s>>>(counter, n_bsets);
            std::vector<int32_t*> ce(n_bsets, nullptr);
            std::vector<uint8_t*> cf(n_bsets, nullptr);
            for (int b = 0; b < n_bsets; ++b) {
                if (tg[b]) {
                    double* t = (double*)talloc(sizeof(double) * mg->nf * (size_t)Lc.n_nodes);
                    if (!t) return set_error(MF_ERR_OOM, "multigrid face workspace allocation failed");
                    k_mg_inject_nodal<<<grid_for(Lc.n_nodes, kThreads), kThreads, 0, s>>>(
                        Lc.nx, Lc.ny, Lc.n_nodes, Lf.nx, Lf.ny, Lf.n_nodes, mg->nf, tg[b], t);
                    tg[b] = t;
                }
                if (nfc[b] == 0) continue;
                ce[b] = (int32_t*)talloc(sizeof(int32_t) * (size_t)nfc[b]);
                cf[b] = (uint8_t*)talloc((size_t)nfc[b]);
                if (!ce[b] || !cf[b]) return set_error(MF_ERR_OOM, "multigrid face workspace allocation failed");
                k_mg_faces<<<grid_for(nfc[b], kThreads), kThreads, 0, s>>>(nfc[b], fe[b], fi[b], Lf.nx, Lf.ny,
                                                                           Lf.nz, counter + b, ce[b], cf[b]);
            }
            MF_HIP(hipGetLastError());
            std::vector<int> cnt(n_bsets, 0);
            MF_HIP(hipMemcpyAsync(cnt.data(), counter, sizeof(int) * n_bsets, hipMemcpyDeviceToHost, s));
            MF_HIP(hipStreamSynchronize(s));
            for (int b = 0; b < n_bsets; ++b) {
                nfc[b] = cnt[b];
                fe[b] = ce[b];
                fi[b] = cf[b];
            }
        }
        mf_form fl = *form;
        if (form->kind == MF_FORM_NS_SUPG) {
            if (mg->opts.tau_m[l] > 0.0) fl.tau_m = mg->opts.tau_m[l];
            if (mg->opts.tau_c[l] > 0.0) fl.tau_c = mg->opts.tau_c[l];
        }
        mf_fields F{};
        F.lin_state = lin_state ? Lc.state : nullptr;
        F.elem_param = elem_param ? Lc.elem : nullptr;
        // with face sets the elimination comes after the faces are added
        F.dirichlet = (dirichlet && n_bsets == 0) ? Lc.mask : nullptr;
        mf_status st = mf_assemble(Lc.P, &fl, Lc.coords, &F, quad, MF_F64, Lc.K, Lc.d, stream);
        if (st != MF_OK) return st;
        for (int b = 0; b < n_bsets; ++b) {
            st = mf_assemble_boundary(Lc.P, &bsets[b].form, Lc.coords, nfc[b], fe[b], fi[b],
                                      lin_state ? Lc.state : nullptr, tg[b], MF_F64, Lc.K, Lc.d, stream);
            if (st != MF_OK) return st;
        }
        if (n_bsets > 0 && dirichlet) {
            AssembleArgs elim{};
            elim.P = Lc.P;
            elim.dirichlet = Lc.mask;
            elim.prec = MF_F64;
            elim.K = Lc.K;
            elim.d = Lc.d;
            elim.stream = s;
            st = apply_dirichlet(elim);
            if (st != MF_OK) return st;
        }
        int64_t bad = -1;
        st = mf_status_poll(Lc.P, &bad);
        if (st != MF_OK) return st;
    }
    for (int l = 0; l < mg->n_levels; ++l) {
        const mf_mg_s::Level& Lv = mg->L[l];
        k_mg_dinv<<<grid_for(Lv.n_rows, kThreads), kThreads, 0, s>>>(Lv.n_rows, Lv.Pv->row_ptr, Lv.Pv->col_idx, Lv.Kv,
                                                                     Lv.dinv);
        if (Lv.eval)
            k_mg_ell_vals<<<grid_for(Lv.n_rows, kThreads), kThreads, 0, s>>>(Lv.n_rows, Lv.width, Lv.Pv->row_ptr,
                                                                             Lv.Kv, Lv.eval);
    }
    MF_HIP(hipGetLastError());
    MF_HIP(hipStreamSynchronize(s));
    mg->updated = true;
    return MF_OK;
}

extern "C" mf_status mf_mg_update(mf_mg_t* mg, const mf_form* form, const double* coords, const mf_fields* fields,
                                  const mf_quadrature* quad, const double* K, void* stream)
{
    return mf_mg_update_ex(mg, form, coords, fields, nullptr, 0, quad, K, stream);
}

extern "C" mf_status mf_mg_apply(const mf_mg_t* mg, const double* r, double* z, void* stream)
{
    if (!mg) return set_error(MF_ERR_ARG, "mg is NULL");
    if (!mg->updated) return set_error(MF_ERR_ARG, "call mf_mg_update before mf_mg_apply");
    if (mg->L[0].n_rows > 0 && (!r || !z || r == z)) return set_error(MF_ERR_ARG, "r and z must be distinct vectors");
    return mg_apply_cb((void*)mg, r, z, (hipStream_t)stream);
}

extern "C" void mf_mg_destroy(mf_mg_t* mg) { free_mg(mg); }
