// Owner-computes gather assembly on structured grids (Sec. 2.2 D-2 and D-3 without the
// atomic increments into global memory).
//
// Each workgroup owns a 4x4x4 brick of nodes and produces their complete rows of K and
// entries of d: it computes every element that touches the brick (a 5x5x5 halo of
// elements, clipped to the mesh), accumulates the element blocks that land in owned
// rows in LDS, then writes each owned row once, coalesced, with Dirichlet elimination
// applied on the way out.  No global atomics, no clearing pass; each value of K is
// written exactly once.
//
// Element teams: two lanes per element.  The element matrix of a symmetric form is
// made of 36 node-pair blocks (a <= b).  Lane 0 works in the element's own labelling,
// lane 1 in the labelling rotated by 180 degrees about the z axis (local node a ->
// a ^ 3, which keeps det J > 0).  Both lanes run the same code over the same list of
// 20 pair blocks: under the rotation the list and its image cover all 36 blocks; the
// four pairs {a, a^3} that the rotation maps to themselves appear in both lanes and
// carry weight 1/2.  Geometry is FP64 in both precisions (rounded to T afterwards).
#include <hip/hip_runtime.h>

#include <vector>

#include "element.h"
#include "mf_internal.h"

namespace mf {
namespace {

constexpr int BX = 4, BY = 4, BZ = 4;  // owned nodes per brick
constexpr int HX = BX + 1, HY = BY + 1, HZ = BZ + 1;  // halo elements per axis
constexpr int kOwned = BX * BY * BZ;
constexpr int kHalo = HX * HY * HZ;
constexpr int kThreads = 256;
static_assert(2 * kHalo <= kThreads, "two lanes per halo element");

// Pair blocks computed by every lane, in the lane's own frame.
constexpr int kNumPairs = 20;
__device__ constexpr int kPairA[kNumPairs] = {0, 1, 4, 5,                          // diagonal
                                               0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 4, 4,  // orbit reps
                                               0, 1, 4, 5};                         // self-mapped
__device__ constexpr int kPairB[kNumPairs] = {0, 1, 4, 5,
                                               1, 2, 4, 5, 6, 7, 4, 5, 6, 7, 5, 6,
                                               3, 2, 7, 6};
constexpr int kFirstHalf = 16;  // pairs >= kFirstHalf carry weight 1/2
constexpr int kFrameMask = 3;   // lane 1 frame: a -> a ^ 3

struct GatherParams {
    mf_form form;
    int64_t nx, ny, nz;  // elements per axis
    int64_t n_nodes;
    const double* coords;
    const int32_t* nbr_ptr;
    const void* elem_param;
    const void* src;
    const uint8_t* dirichlet;
    int field_major;
    int64_t n_pairs;
    void* K;
    void* d;
    unsigned long long* status;
};

__device__ __forceinline__ int slot_of(int dx, int dy, int dz) { return (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1); }

// Passes over the pair list: accumulators of one pass stay in registers (the
// geometry is recomputed per pass).  FP64 elasticity needs three, FP32 two.
template <int FORM, typename T>
struct GatherShape {
    static constexpr int kPasses = FORM != MF_FORM_ELASTICITY ? 1 : (sizeof(T) == 8 ? 3 : 2);
    static constexpr int kPerPass = (kNumPairs + kPasses - 1) / kPasses;
    static constexpr int kMinBlocks = sizeof(T) == 8 && FORM == MF_FORM_ELASTICITY ? 1 : 2;
};

// One brick of one problem; called by the single-problem kernel and by the persistent
// batched kernel.  accK/accD/nodeInfo are the workgroup's LDS arrays.
template <int FORM, typename T>
__device__ __forceinline__ void gather_brick_body(const GatherParams& p, int b, T* __restrict__ accK,
                                                  T* __restrict__ accD, int (*nodeInfo)[4])
{
    constexpr int NF = FormTraits<FORM, 3>::NF;
    constexpr int NSRC = FormTraits<FORM, 3>::NSRC;
    constexpr int NB = NF * NF;                 // values per node-pair block
    constexpr int ROWVALS = 27 * NB;            // values of one owned node's rows
    constexpr int NV = FORM == MF_FORM_ELASTICITY ? 9 : 1;
    constexpr int PASSES = GatherShape<FORM, T>::kPasses, PER = GatherShape<FORM, T>::kPerPass;

    const int tid = threadIdx.x;
    const int nx = (int)p.nx, ny = (int)p.ny, nz = (int)p.nz;
    const int NX = nx + 1, NY = ny + 1, NZ = nz + 1;  // nodes per axis
    const int nbx = (NX + BX - 1) / BX, nby = (NY + BY - 1) / BY;
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int i0 = bx * BX, j0 = by * BY, k0 = bz * BZ;

    for (int k = tid; k < kOwned * ROWVALS; k += kThreads) accK[k] = T(0);
    for (int k = tid; k < kOwned * NF; k += kThreads) accD[k] = T(0);
    if (tid < kOwned) {
        const int lx = tid % BX, ly = (tid / BX) % BY, lz = tid / (BX * BY);
        const int gi = i0 + lx, gj = j0 + ly, gk = k0 + lz;
        if (gi < NX && gj < NY && gk < NZ) {
            const int node = gi + NX * (gj + NY * gk);
            const int mx = 1 + (gi > 0) + (gi < nx), my = 1 + (gj > 0) + (gj < ny), mz = 1 + (gk > 0) + (gk < nz);
            nodeInfo[tid][0] = node;
            nodeInfo[tid][1] = p.nbr_ptr[node];
            nodeInfo[tid][2] = mx * my * mz;
            nodeInfo[tid][3] = (gi > 0) | ((gi < nx) << 1) | ((gj > 0) << 2) | ((gj < ny) << 3) |
                               ((gk > 0) << 4) | ((gk < nz) << 5);
        } else {
            nodeInfo[tid][0] = -1;
        }
    }
    __syncthreads();

    // ---------------- element phase ----------------
    const int team = tid >> 1, h = tid & 1;
    const int fm = h ? kFrameMask : 0;
    const int tx = team % HX, ty = (team / HX) % HY, tz = team / (HX * HY);
    const int ex = i0 - 1 + tx, ey = j0 - 1 + ty, ez = k0 - 1 + tz;
    const bool active = team < kHalo && ex >= 0 && ex < nx && ey >= 0 && ey < ny && ez >= 0 && ez < nz;
    if (active) {
        const int e = ex + nx * (ey + ny * ez);
        // nodes in the lane frame: local a' is element node a' ^ fm
        double x[8][3];
        T U[8][NSRC];
        const T* src = (const T*)p.src;
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int A = a ^ fm;
            const int node = (ex + (A & 1)) + NX * ((ey + ((A >> 1) & 1)) + NY * (ez + ((A >> 2) & 1)));
#pragma unroll
            for (int m = 0; m < 3; ++m) x[a][m] = p.coords[(int64_t)m * p.n_nodes + node];
#pragma unroll
            for (int s2 = 0; s2 < NSRC; ++s2) U[a][s2] = src ? src[(int64_t)s2 * p.n_nodes + node] : T(0);
        }
        const double ep = p.elem_param ? (double)((const T*)p.elem_param)[e] : 1.0;
        const Coef<T> C = make_coef<T>(FORM, p.form, ep);
        bool bad = false;

#pragma unroll
        for (int pass = 0; pass < PASSES; ++pass) {
            constexpr int dummy = 0;
            (void)dummy;
            const int kbeg = pass * PER;
            T acc[PER][NV];
#pragma unroll
            for (int k = 0; k < PER; ++k)
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[k][v] = T(0);
            T dv[4][NF];  // residual of the lane's diagonal rows (first pass only)
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int i = 0; i < NF; ++i) dv[r][i] = T(0);

#pragma unroll 1
            for (int q = 0; q < 8; ++q) {
                double gd[8][3];
                const double det = geometry_hex_rt(x, q, gd);
                if (!(det > 0.0)) { bad = true; break; }
                const T W = (T)det;
                T g[8][3];
#pragma unroll
                for (int a = 0; a < 8; ++a)
#pragma unroll
                    for (int m = 0; m < 3; ++m) g[a][m] = (T)gd[a][m];
#pragma unroll
                for (int kk = 0; kk < PER; ++kk) {
                    const int k = kbeg + kk;
                    if (k >= kNumPairs) break;
                    const int A = kPairA[k], B = kPairB[k];
                    if constexpr (FORM == MF_FORM_ELASTICITY) {
#pragma unroll
                        for (int i = 0; i < 3; ++i) {
                            const T wgi = W * g[A][i];
#pragma unroll
                            for (int j = 0; j < 3; ++j) acc[kk][i * 3 + j] += wgi * g[B][j];
                        }
                    } else if constexpr (FORM == MF_FORM_POISSON) {
                        acc[kk][0] += W * (g[A][0] * g[B][0] + g[A][1] * g[B][1] + g[A][2] * g[B][2]);
                    } else {
                        acc[kk][0] += W * ((T)kRefHex.N[q][A] * (T)kRefHex.N[q][B]);
                    }
                }
                if (pass == 0) {
                    // element residual of the lane's diagonal rows: d = int N_a f (times c for MASS)
#pragma unroll
                    for (int i = 0; i < NF; ++i) {
                        T fq = T(0);
#pragma unroll
                        for (int a = 0; a < 8; ++a) fq += (T)kRefHex.N[q][a] * U[a][i];
                        const T wf = (FORM == MF_FORM_MASS ? C.c : T(1)) * W * fq;
#pragma unroll
                        for (int r = 0; r < 4; ++r) dv[r][i] += wf * (T)kRefHex.N[q][kPairA[r]];
                    }
                }
            }
            if (bad) break;
            // epilogue and scatter of this pass's blocks into the owned rows
#pragma unroll
            for (int kk = 0; kk < PER; ++kk) {
                const int k = kbeg + kk;
                if (k >= kNumPairs) break;
                const int A = kPairA[k] ^ fm, B = kPairB[k] ^ fm;  // element-local labels
                const T w = k >= kFirstHalf ? T(0.5) : T(1);
                T Kb[NB];
                if constexpr (FORM == MF_FORM_ELASTICITY) {
                    const T tr = acc[kk][0] + acc[kk][4] + acc[kk][8];
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j)
                            Kb[i * 3 + j] = w * (C.lam * acc[kk][i * 3 + j] + C.mu * acc[kk][j * 3 + i] +
                                                 (i == j ? C.mu * tr : T(0)));
                } else {
                    Kb[0] = w * C.c * acc[kk][0];
                }
                const int ax = A & 1, ay = (A >> 1) & 1, az = (A >> 2) & 1;
                const int bxx = B & 1, byy = (B >> 1) & 1, bzz = (B >> 2) & 1;
                const int lax = ex + ax - i0, lay = ey + ay - j0, laz = ez + az - k0;
                const int lbx = ex + bxx - i0, lby = ey + byy - j0, lbz = ez + bzz - k0;
                const bool ownA = (unsigned)lax < BX && (unsigned)lay < BY && (unsigned)laz < BZ;
                const bool ownB = (unsigned)lbx < BX && (unsigned)lby < BY && (unsigned)lbz < BZ;
                if (ownA) {
                    T* dst = accK + ((laz * BY + lay) * BX + lax) * ROWVALS +
                             slot_of(bxx - ax, byy - ay, bzz - az) * NB;
#pragma unroll
                    for (int v = 0; v < NB; ++v) unsafeAtomicAdd(dst + v, Kb[v]);
                }
                if (A != B && ownB) {
                    T* dst = accK + ((lbz * BY + lby) * BX + lbx) * ROWVALS +
                             slot_of(ax - bxx, ay - byy, az - bzz) * NB;
#pragma unroll
                    for (int i = 0; i < NF; ++i)
#pragma unroll
                        for (int j = 0; j < NF; ++j) unsafeAtomicAdd(dst + j * NF + i, Kb[i * NF + j]);
                }
            }
            if (pass == 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int A = kPairA[r] ^ fm;
                    const int lax = ex + (A & 1) - i0, lay = ey + ((A >> 1) & 1) - j0, laz = ez + ((A >> 2) & 1) - k0;
                    if ((unsigned)lax < BX && (unsigned)lay < BY && (unsigned)laz < BZ) {
#pragma unroll
                        for (int i = 0; i < NF; ++i)
                            unsafeAtomicAdd(accD + ((laz * BY + lay) * BX + lax) * NF + i, dv[r][i]);
                    }
                }
            }
        }
        if (bad) atomicMin(p.status, (unsigned long long)e);
    }
    __syncthreads();

    // ---------------- write-out: each owned row once ----------------
    // Work item = (owned node, row field i, neighbour slot, column field j); all divisors
    // are compile-time constants and per-node data comes from the LDS table.
    T* K = (T*)p.K;
    T* d = (T*)p.d;
    const int nn = (int)p.n_nodes;
    const int fmaj = p.field_major;
    constexpr int kRowSlots = 27 * NF;
    for (int flat = tid; flat < kOwned * NF * kRowSlots; flat += kThreads) {
        const int rloc = flat / kRowSlots;
        const int sj = flat - rloc * kRowSlots;
        const int slot = sj / NF, j = sj - slot * NF;
        const int il = rloc / NF, i = rloc - il * NF;
        const int node = nodeInfo[il][0];
        if (node < 0) continue;
        const int bits = nodeInfo[il][3];
        const int dx = slot % 3 - 1, dy = (slot / 3) % 3 - 1, dz = slot / 9 - 1;
        // neighbour exists: bit 2*axis for -1, 2*axis+1 for +1
        const int need = (dx < 0 ? 1 : 0) | (dx > 0 ? 2 : 0) | (dy < 0 ? 4 : 0) | (dy > 0 ? 8 : 0) |
                         (dz < 0 ? 16 : 0) | (dz > 0 ? 32 : 0);
        if ((bits & need) != need) continue;
        const int lo_x = bits & 1, lo_y = (bits >> 2) & 1, lo_z = (bits >> 4) & 1;
        const int mx = 1 + lo_x + ((bits >> 1) & 1), my = 1 + lo_y + ((bits >> 3) & 1);
        const int rank = ((dz + lo_z) * my + (dy + lo_y)) * mx + (dx + lo_x);
        const int deg = nodeInfo[il][2];
        const int P = nodeInfo[il][1];
        int row, kpos;
        if (fmaj) {
            row = i * nn + node;
            kpos = i * NF * (int)p.n_pairs + NF * P + j * deg + rank;
        } else {
            row = NF * node + i;
            kpos = P * NB + i * NF * deg + rank * NF + j;
        }
        T v = accK[(il * 27 + slot) * NB + i * NF + j];
        if (p.dirichlet) {
            const int nb = node + dx + NX * (dy + NY * dz);
            const int col = fmaj ? j * nn + nb : NF * nb + j;
            if (p.dirichlet[row]) v = (col == row) ? T(1) : T(0);
            else if (p.dirichlet[col]) v = T(0);
        }
        K[kpos] = v;
        if (slot == 13 && j == 0) {
            T dvv = accD[il * NF + i];
            if (p.dirichlet && p.dirichlet[row]) dvv = T(0);
            d[row] = dvv;
        }
    }
}

template <int FORM, typename T>
__global__ void __launch_bounds__(kThreads, (GatherShape<FORM, T>::kMinBlocks)) k_gather_brick(GatherParams p)
{
    constexpr int NF = FormTraits<FORM, 3>::NF;
    __shared__ T accK[kOwned * 27 * NF * NF];
    __shared__ T accD[kOwned * NF];
    __shared__ int nodeInfo[kOwned][4];  // node id, first pair offset, degree, boundary bits
    gather_brick_body<FORM, T>(p, blockIdx.x, accK, accD, nodeInfo);
}


// ------------------------------------------------------------------------------------
// Batched persistent launch: many structured problems in one kernel.  Work items are
// (problem, brick) pairs in an order chosen on the host; each workgroup pops the next
// item from a device counter until the list is exhausted (every wave reaches the exit).
// ------------------------------------------------------------------------------------
struct BatchProblemDev {
    GatherParams gp;
    int kind;
};

__global__ void k_batch_reset(int* counter, unsigned long long* const* status, int n_status)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *counter = 0;
    if (i < n_status) *status[i] = ~0ull;
}

template <typename T>
__global__ void __launch_bounds__(kThreads, (sizeof(T) == 8 ? 1 : 2))
    k_batch_persistent(const BatchProblemDev* __restrict__ probs, const int2* __restrict__ items, int n_items,
                       int* __restrict__ counter)
{
    __shared__ T accK[kOwned * 27 * 9];
    __shared__ T accD[kOwned * 3];
    __shared__ int nodeInfo[kOwned][4];
    __shared__ int sItem;
    while (true) {
        __syncthreads();  // the previous item's write-out is done with the LDS
        if (threadIdx.x == 0) sItem = atomicAdd(counter, 1);
        __syncthreads();
        const int it = sItem;
        if (it >= n_items) break;
        const int2 w = items[it];
        const GatherParams gp = probs[w.x].gp;
        const int kind = probs[w.x].kind;
        if (kind == MF_FORM_ELASTICITY)
            gather_brick_body<MF_FORM_ELASTICITY, T>(gp, w.y, accK, accD, nodeInfo);
        else if (kind == MF_FORM_POISSON)
            gather_brick_body<MF_FORM_POISSON, T>(gp, w.y, accK, accD, nodeInfo);
        else
            gather_brick_body<MF_FORM_MASS, T>(gp, w.y, accK, accD, nodeInfo);
    }
}

GatherParams make_params(const AssembleArgs& A)
{
    const mf_pattern_s* P = A.P;
    GatherParams p{};
    p.form = *A.form;
    p.nx = P->gx;
    p.ny = P->gy;
    p.nz = P->gz;
    p.n_nodes = P->n_nodes;
    p.coords = A.coords;
    p.nbr_ptr = P->nbr_ptr;
    p.elem_param = A.elem_param;
    p.src = A.nodal_src;
    p.dirichlet = A.dirichlet;
    p.field_major = P->numbering == MF_FIELD_MAJOR;
    p.n_pairs = P->n_pairs;
    p.K = A.K;
    p.d = A.d;
    p.status = P->status;
    return p;
}

int64_t brick_count(const mf_pattern_s* P)
{
    return ((P->gx + 1 + BX - 1) / BX) * ((P->gy + 1 + BY - 1) / BY) * ((P->gz + 1 + BZ - 1) / BZ);
}

template <int FORM, typename T>
mf_status launch_gather(const AssembleArgs& A)
{
    const GatherParams p = make_params(A);
    const int64_t nb = brick_count(A.P);
    k_gather_brick<FORM, T><<<(unsigned)nb, kThreads, 0, A.stream>>>(p);
    MF_HIP(hipGetLastError());
    return MF_OK;
}

template <typename T>
mf_status dispatch(const AssembleArgs& A)
{
    switch (A.form->kind) {
        case MF_FORM_MASS: return launch_gather<MF_FORM_MASS, T>(A);
        case MF_FORM_POISSON: return launch_gather<MF_FORM_POISSON, T>(A);
        case MF_FORM_ELASTICITY: return launch_gather<MF_FORM_ELASTICITY, T>(A);
        default: return MF_ERR_UNSUPPORTED;
    }
}

}  // namespace


// ---------------- batched launch: host side ----------------

int64_t brick_count_of(const mf_pattern_s* P) { return brick_count(P); }

mf_status batch_check(const AssembleArgs& A)
{
    const mf_pattern_s* P = A.P;
    if (!P->is_grid || P->dim != 3 || !P->full_coupling || P->n_elems == 0)
        return set_error(MF_ERR_UNSUPPORTED, "batched problems must be non-empty structured 3D grids with full coupling");
    if (A.form->kind == MF_FORM_NS_SUPG) return set_error(MF_ERR_UNSUPPORTED, "batched launch covers mass, Poisson and elasticity");
    return MF_OK;
}

mf_status batch_upload(const std::vector<AssembleArgs>& probs, void** dev_probs, void** dev_status)
{
    std::vector<BatchProblemDev> h(probs.size());
    std::vector<unsigned long long*> st(probs.size());
    for (size_t k = 0; k < probs.size(); ++k) {
        h[k].gp = make_params(probs[k]);
        h[k].kind = probs[k].form->kind;
        st[k] = probs[k].P->status;
    }
    MF_HIP(hipMalloc(dev_probs, sizeof(BatchProblemDev) * (h.size() > 0 ? h.size() : 1)));
    MF_HIP(hipMemcpy(*dev_probs, h.data(), sizeof(BatchProblemDev) * h.size(), hipMemcpyHostToDevice));
    MF_HIP(hipMalloc(dev_status, sizeof(void*) * (st.size() > 0 ? st.size() : 1)));
    MF_HIP(hipMemcpy(*dev_status, st.data(), sizeof(void*) * st.size(), hipMemcpyHostToDevice));
    return MF_OK;
}

mf_status batch_launch(const void* dev_probs, void* dev_status, int n_probs, const int2* items, int n_items,
                       int* counter, int n_wg, mf_precision prec, hipStream_t s)
{
    k_batch_reset<<<(n_probs + 255) / 256 > 0 ? (n_probs + 255) / 256 : 1, 256, 0, s>>>(
        counter, (unsigned long long* const*)dev_status, n_probs);
    if (prec == MF_F64)
        k_batch_persistent<double><<<n_wg, kThreads, 0, s>>>((const BatchProblemDev*)dev_probs, items, n_items, counter);
    else
        k_batch_persistent<float><<<n_wg, kThreads, 0, s>>>((const BatchProblemDev*)dev_probs, items, n_items, counter);
    MF_HIP(hipGetLastError());
    return MF_OK;
}

// Returns MF_ERR_UNSUPPORTED (without launching) when the gather path does not cover
// the case: unstructured meshes, 2D, partial coupling, or the flow form.
mf_status assemble_gather(const AssembleArgs& A)
{
    const mf_pattern_s* P = A.P;
    if (!P->is_grid || P->dim != 3 || !P->full_coupling) return MF_ERR_UNSUPPORTED;
    if (A.form->kind == MF_FORM_NS_SUPG) return MF_ERR_UNSUPPORTED;
    if (P->n_elems == 0) return MF_ERR_UNSUPPORTED;
    return A.prec == MF_F64 ? dispatch<double>(A) : dispatch<float>(A);
}

}  // namespace mf
