// Preconditioned conjugate gradients on an assembled K (the linear solve of Sec. 2.2 D-4,
// which the paper leaves open).  FP64 throughout.
//
// One iteration, all scalars kept on the device:
//   k_spmv_dir_dot  p = z + beta p (double-buffered) and q = K p in one pass, partial
//                sums of p.q; the last block to finish sums the partials (fixed order)
//                into alpha = (r.z) / (p.q)
//   k_update_dots  x += alpha p, r -= alpha q, z = M r, partial sums of r.z, r.r; its
//                last block forms beta = (r.z)_new / (r.z).  For an external apply the
//                update (k_update), the apply and the dots (k_dots: r.z, r.r, z.r_old,
//                flexible beta = (z.(r - r_old)) / (r.z)_old) are separate steps.
// Partial sums use fixed block order, so a run is bit-reproducible.  Chunks of
// iterations are captured once into a HIP graph and replayed; between chunks the host
// reads the recurrence residual, and a candidate solution is accepted only when the
// true residual |b - K x| / |b| meets the tolerance.
//
// Preconditioners: Jacobi (z = r / diag K), none, or an external apply (the learned
// network) that writes z from r; for the external one the flexible beta is used and
// any iteration with z.r <= 0 or a non-finite z falls back to the Jacobi z.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "mf_internal.h"
#include "pcg.h"

namespace mf {
namespace {

constexpr int kThreads = 256;
constexpr int kRowsPerWave = 4;  // 16 lanes per row
constexpr int kLanesPerRow = 64 / kRowsPerWave;
constexpr int kMaxBlocks = 2048;  // partial-sum slots per reduction

__device__ __forceinline__ double warp_sum_lanes16(double v)
{
#pragma unroll
    for (int off = kLanesPerRow / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kLanesPerRow);
    return v;
}

__device__ __forceinline__ double block_sum(double v, double* sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x / 64); ++k) s += sh[k];
    __syncthreads();
    return s;  // valid in thread 0
}

// True in every thread of the block that finishes last among the grid's blocks.  Each
// block's thread 0 has written its partial sums before the call; the release fence and
// the counter make them visible to the last block, which re-arms the counter.
__device__ __forceinline__ bool last_block(unsigned int* cnt)
{
    __shared__ int is_last;
    if (threadIdx.x == 0) {
        __threadfence();
        is_last = atomicAdd(cnt, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last;
}

// Scalars (device): s[0] = rz, s[1] = pq, s[2] = alpha, s[3] = beta, s[4] = rr, s[5] = rz_new,
// s[6] = zdr (flexible numerator), s[7] = fallback count, s[8] = breakdown flag
enum { S_RZ = 0, S_PQ, S_ALPHA, S_BETA, S_RR, S_RZNEW, S_ZDR, S_FALLBACK, S_BREAK, S_COUNT };

// alpha = (r.z) / (p.q) from nb block partials of p.q, summed in a fixed order by one
// block (all its threads call this); cnt (if any) is re-armed.
__device__ __forceinline__ void finish_alpha(const double* partial, int nb, double* s, double* sh,
                                             unsigned int* cnt)
{
    double v = 0.0;
    for (int k = threadIdx.x; k < nb; k += blockDim.x) v += partial[k];
    const double pq = block_sum(v, sh);
    if (threadIdx.x == 0) {
        s[S_PQ] = pq;
        const bool ok = pq > 0.0 && isfinite(pq);
        if (!ok) s[S_BREAK] = 1.0;
        s[S_ALPHA] = ok ? s[S_RZ] / pq : 0.0;
        if (cnt) *cnt = 0u;
    }
}

// beta from the partials [0..nb) r.z, [nb..2nb) r.r, [2nb..3nb) z.r_old;
// flexible: beta = (z.r - z.r_old) / rz_old
__device__ __forceinline__ void finish_beta(const double* partial, int nb, double* s, int flexible, double* sh,
                                            unsigned int* cnt)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
        a += partial[k];
        b += partial[nb + k];
        c += partial[2 * nb + k];
    }
    const double rz = block_sum(a, sh);
    const double rr = block_sum(b, sh);
    const double zro = block_sum(c, sh);
    if (threadIdx.x == 0) {
        const double rz_old = s[S_RZ];
        const double num = flexible ? rz - zro : rz;
        s[S_BETA] = rz_old != 0.0 ? num / rz_old : 0.0;
        s[S_RZNEW] = rz;
        s[S_RZ] = rz;
        s[S_RR] = rr;
        if (!(rz > 0.0) || !isfinite(rz)) s[S_BREAK] = 1.0;
        if (cnt) *cnt = 0u;
    }
}

// y = A x (CSR), partial[block] = sum over the block's rows of w[row] * y[row] (w may be null)
__global__ void __launch_bounds__(kThreads) k_spmv_dot(int n, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci,
                                                       const double* __restrict__ v,
                                                       const double* __restrict__ x, double* __restrict__ y,
                                                       const double* __restrict__ w, double* partial,
                                                       unsigned int* cnt, double* s)
{
    __shared__ double sh[kThreads / 64];
    const int lane = threadIdx.x % kLanesPerRow;
    const int sub = threadIdx.x / kLanesPerRow;  // row slot within the block
    constexpr int kSlots = kThreads / kLanesPerRow;
    double acc_dot = 0.0;
    for (int base = blockIdx.x * kSlots; base < n; base += gridDim.x * kSlots) {
        const int row = base + sub;
        double s = 0.0;
        if (row < n) {
            const int k1 = rp[row + 1];
            for (int k = rp[row] + lane; k < k1; k += kLanesPerRow) s = fma(v[k], x[ci[k]], s);
        }
        s = warp_sum_lanes16(s);
        if (row < n && lane == 0) {
            y[row] = s;
            if (w) acc_dot = fma(w[row], s, acc_dot);
        }
    }
    const double t = block_sum(acc_dot, sh);
    if (threadIdx.x == 0 && partial) partial[blockIdx.x] = t;
    if (cnt && last_block(cnt)) finish_alpha(partial, gridDim.x, s, sh, cnt);
}


// p_new = z + beta p_old and q = K p_new in one pass (the direction update of the previous
// iteration folded into the SpMV: each column value is formed on the fly, bit-identical
// to the stored p_new); partial sums of p_new.q, finished into alpha by the last block.
__global__ void __launch_bounds__(kThreads) k_spmv_dir_dot(int n, const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const double* __restrict__ v,
                                                           const double* __restrict__ z,
                                                           const double* __restrict__ p_old,
                                                           double* __restrict__ p_new, double* __restrict__ q,
                                                           double* s, double* partial, unsigned int* cnt)
{
    __shared__ double sh[kThreads / 64];
    const double beta = s[S_BETA];
    const int lane = threadIdx.x % kLanesPerRow;
    const int sub = threadIdx.x / kLanesPerRow;
    constexpr int kSlots = kThreads / kLanesPerRow;
    double acc_dot = 0.0;
    for (int base = blockIdx.x * kSlots; base < n; base += gridDim.x * kSlots) {
        const int row = base + sub;
        double sum = 0.0;
        if (row < n) {
            const int k1 = rp[row + 1];
            for (int k = rp[row] + lane; k < k1; k += kLanesPerRow) {
                const int c = ci[k];
                sum = fma(v[k], fma(beta, p_old[c], z[c]), sum);
            }
        }
        sum = warp_sum_lanes16(sum);
        if (row < n && lane == 0) {
            const double pn = fma(beta, p_old[row], z[row]);
            p_new[row] = pn;
            q[row] = sum;
            acc_dot = fma(pn, sum, acc_dot);
        }
    }
    const double t = block_sum(acc_dot, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
    if (last_block(cnt)) finish_alpha(partial, gridDim.x, s, sh, cnt);
}

// x += alpha p; r -= alpha q; z = precond(r) (Jacobi here; external apply overwrites z
// afterwards); partials: [0..nb) r.z, [nb..2nb) r.r, [2nb..3nb) z.r_old
__global__ void __launch_bounds__(kThreads) k_update(int n, const double* __restrict__ s,
                                                     double* __restrict__ x, double* __restrict__ r,
                                                     double* __restrict__ r_old, const double* __restrict__ p,
                                                     const double* __restrict__ q, const double* __restrict__ dinv,
                                                     double* __restrict__ z, int jacobi, int keep_old)
{
    const double alpha = s[S_ALPHA];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        x[i] = fma(alpha, p[i], x[i]);
        const double ri = fma(-alpha, q[i], r[i]);
        if (keep_old) r_old[i] = r[i];
        r[i] = ri;
        if (jacobi >= 0) z[i] = jacobi ? dinv[i] * ri : ri;
    }
}

// Jacobi iteration body in one pass: x += alpha p; r -= alpha q; z = D^-1 r (or z = r);
// partial sums of r.z and r.r (the z.r_old slot is zero)
__global__ void __launch_bounds__(kThreads) k_update_dots(int n, double* s, double* __restrict__ x,
                                                          double* __restrict__ r, const double* __restrict__ p,
                                                          const double* __restrict__ q,
                                                          const double* __restrict__ dinv, double* __restrict__ z,
                                                          int jacobi, double* partial, int nb, unsigned int* cnt)
{
    __shared__ double sh[kThreads / 64];
    const double alpha = s[S_ALPHA];
    double rz = 0.0, rr = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        x[i] = fma(alpha, p[i], x[i]);
        const double ri = fma(-alpha, q[i], r[i]);
        r[i] = ri;
        const double zi = jacobi ? dinv[i] * ri : ri;
        z[i] = zi;
        rz = fma(ri, zi, rz);
        rr = fma(ri, ri, rr);
    }
    const double a = block_sum(rz, sh);
    const double b = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = a;
        partial[nb + blockIdx.x] = b;
        partial[2 * nb + blockIdx.x] = 0.0;
    }
    if (last_block(cnt)) finish_beta(partial, nb, s, 0, sh, cnt);
}

// partial dots after z is known: r.z, r.r, z.r_old
__global__ void __launch_bounds__(kThreads) k_dots(int n, const double* __restrict__ r, const double* __restrict__ z,
                                                   const double* __restrict__ r_old, double* partial, int nb,
                                                   unsigned int* cnt, double* s, int flexible)
{
    __shared__ double sh[kThreads / 64];
    double rz = 0.0, rr = 0.0, zro = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double ri = r[i], zi = z[i];
        rz = fma(ri, zi, rz);
        rr = fma(ri, ri, rr);
        if (r_old) zro = fma(zi, r_old[i], zro);
    }
    const double a = block_sum(rz, sh);
    const double b = block_sum(rr, sh);
    const double c = block_sum(zro, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = a;
        partial[nb + blockIdx.x] = b;
        partial[2 * nb + blockIdx.x] = c;
    }
    if (cnt && last_block(cnt)) finish_beta(partial, nb, s, flexible, sh, cnt);
}

__global__ void k_reduce_beta(const double* partial, int nb, double* s, int flexible)
{
    __shared__ double sh[kThreads / 64];
    finish_beta(partial, nb, s, flexible, sh, nullptr);
}

// diag inverse, x = 0, r = b, z = M b, p = z
__global__ void __launch_bounds__(kThreads) k_init(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                   const double* __restrict__ v, const double* __restrict__ b,
                                                   double* __restrict__ dinv, double* __restrict__ x,
                                                   double* __restrict__ r, double* __restrict__ z,
                                                   double* __restrict__ p, int jacobi)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double di = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] == i) di = v[k];
        dinv[i] = di != 0.0 ? 1.0 / di : 1.0;
        x[i] = 0.0;
        r[i] = b[i];
        if (jacobi >= 0) {
            z[i] = jacobi ? dinv[i] * b[i] : b[i];
            p[i] = z[i];
        }
    }
}

// true residual partial sums: |b - A x|^2 and |b|^2
__global__ void __launch_bounds__(kThreads) k_true_res(int n, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                       const double* __restrict__ x, const double* __restrict__ b,
                                                       double* __restrict__ partial, int nb)
{
    __shared__ double sh[kThreads / 64];
    const int lane = threadIdx.x % kLanesPerRow;
    const int sub = threadIdx.x / kLanesPerRow;
    constexpr int kSlots = kThreads / kLanesPerRow;
    double e2 = 0.0, b2 = 0.0;
    for (int base = blockIdx.x * kSlots; base < n; base += gridDim.x * kSlots) {
        const int row = base + sub;
        double sacc = 0.0;
        if (row < n)
            for (int k = rp[row] + lane; k < rp[row + 1]; k += kLanesPerRow) sacc = fma(v[k], x[ci[k]], sacc);
        sacc = warp_sum_lanes16(sacc);
        if (row < n && lane == 0) {
            const double e = b[row] - sacc;
            e2 = fma(e, e, e2);
            b2 = fma(b[row], b[row], b2);
        }
    }
    const double a = block_sum(e2, sh);
    const double c = block_sum(b2, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = a;
        partial[nb + blockIdx.x] = c;
    }
}

__global__ void k_reduce2(const double* __restrict__ partial, int nb, double* __restrict__ out)
{
    __shared__ double sh[kThreads / 64];
    double a = 0.0, c = 0.0;
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
        a += partial[k];
        c += partial[nb + k];
    }
    const double A = block_sum(a, sh);
    const double Cc = block_sum(c, sh);
    if (threadIdx.x == 0) {
        out[0] = A;
        out[1] = Cc;
    }
}

// z := Jacobi z where the external preconditioner failed (z.r <= 0 or non-finite z)
__global__ void k_check_external(const double* __restrict__ partial_rz, int nb, double* __restrict__ s, int* flag)
{
    __shared__ double sh[kThreads / 64];
    double a = 0.0;
    for (int k = threadIdx.x; k < nb; k += blockDim.x) a += partial_rz[k];
    const double rz = block_sum(a, sh);
    if (threadIdx.x == 0) {
        const int bad = !(rz > 0.0) || !isfinite(rz);
        *flag = bad;
        if (bad) s[S_FALLBACK] += 1.0;
    }
}

__global__ void __launch_bounds__(kThreads) k_jacobi_if(int n, const int* __restrict__ flag,
                                                        const double* __restrict__ dinv,
                                                        const double* __restrict__ r, double* __restrict__ z)
{
    if (!*flag) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) z[i] = dinv[i] * r[i];
}

__global__ void k_set(double* p, int n, double v)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

mf_status run_spmv(const mf_csr* A, const double* x, double* y, hipStream_t s)
{
    const int n = (int)A->n_rows;
    if (n == 0) return MF_OK;
    const int blocks = (int)std::min<int64_t>(kMaxBlocks, (n + (kThreads / kLanesPerRow) - 1) / (kThreads / kLanesPerRow));
    k_spmv_dot<<<blocks, kThreads, 0, s>>>(n, A->row_ptr, A->col_idx, A->values, x, y, nullptr, nullptr, nullptr,
                                           nullptr);
    MF_HIP(hipGetLastError());
    return MF_OK;
}

mf_status run_pcg(const PcgArgs& a, mf_pcg_result* res)
{
    const int n = (int)a.n;
    hipStream_t s = a.stream;
    res->iterations = 0;
    res->true_relres = 0.0;
    res->fallbacks = 0;
    res->converged = 0;
    if (n == 0) {
        res->converged = 1;
        return MF_OK;
    }
    const int vec_blocks = (int)std::min<int64_t>(kMaxBlocks, (n + kThreads - 1) / kThreads);
    const int spmv_blocks = (int)std::min<int64_t>(kMaxBlocks, (n + (kThreads / kLanesPerRow) - 1) / (kThreads / kLanesPerRow));
    const int nb = std::max(vec_blocks, spmv_blocks);

    // workspace: dinv r r_old z p q | partial[3 nb] | scalars | flag
    std::vector<void*> owned;
    auto dalloc = [&](size_t bytes) -> void* {
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        owned.push_back(p);
        return p;
    };
    struct Free {
        std::vector<void*>* v;
        ~Free() { for (void* p : *v) (void)hipFree(p); }
    } fr{&owned};
    double* dinv = (double*)dalloc(sizeof(double) * n);
    double* r = (double*)dalloc(sizeof(double) * n);
    double* r_old = (double*)dalloc(sizeof(double) * n);
    double* z = (double*)dalloc(sizeof(double) * n);
    double* p = (double*)dalloc(sizeof(double) * n);
    double* p2 = (double*)dalloc(sizeof(double) * n);
    double* q = (double*)dalloc(sizeof(double) * n);
    double* partial = (double*)dalloc(sizeof(double) * 3 * nb);
    double* sc = (double*)dalloc(sizeof(double) * (S_COUNT + 2));
    int* flag = (int*)dalloc(sizeof(int));
    unsigned int* cnt = (unsigned int*)dalloc(sizeof(unsigned int) * 2);
    if (!dinv || !r || !r_old || !z || !p || !p2 || !q || !partial || !sc || !flag || !cnt)
        return set_error(MF_ERR_OOM, "PCG workspace allocation failed");

    const bool external = a.precond == MF_PRECOND_EXTERNAL;
    const int jac = a.precond == MF_PRECOND_JACOBI ? 1 : (a.precond == MF_PRECOND_NONE ? 0 : -1);
    const int flexible = external ? 1 : 0;

    k_set<<<1, 64, 0, s>>>(sc, S_COUNT + 2, 0.0);
    MF_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned int) * 2, s));
    k_init<<<vec_blocks, kThreads, 0, s>>>(n, a.row_ptr, a.col_idx, a.values, a.b, dinv, a.x, r, z, p, external ? 1 : jac);
    if (external) {
        mf_status st = a.apply(a.apply_ctx, r, z, s);
        if (st != MF_OK) return st;
        k_dots<<<vec_blocks, kThreads, 0, s>>>(n, r, z, nullptr, partial, vec_blocks, nullptr, nullptr, 0);
        k_check_external<<<1, kThreads, 0, s>>>(partial, vec_blocks, sc, flag);
        k_jacobi_if<<<vec_blocks, kThreads, 0, s>>>(n, flag, dinv, r, z);
        MF_HIP(hipMemcpyAsync(p, z, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
    k_dots<<<vec_blocks, kThreads, 0, s>>>(n, r, z, nullptr, partial, vec_blocks, nullptr, nullptr, 0);
    k_reduce_beta<<<1, kThreads, 0, s>>>(partial, vec_blocks, sc, 0);
    MF_HIP(hipGetLastError());

    // |b|
    double hb2[2] = {0, 0};
    k_true_res<<<spmv_blocks, kThreads, 0, s>>>(n, a.row_ptr, a.col_idx, a.values, a.x, a.b, partial, spmv_blocks);
    k_reduce2<<<1, kThreads, 0, s>>>(partial, spmv_blocks, sc + S_COUNT);
    MF_HIP(hipMemcpyAsync(hb2, sc + S_COUNT, sizeof(hb2), hipMemcpyDeviceToHost, s));
    MF_HIP(hipStreamSynchronize(s));
    const double bnorm = std::sqrt(hb2[1]);
    if (bnorm == 0.0) {
        res->converged = 1;
        return MF_OK;
    }

    // the direction alternates between two buffers: iteration k reads p_old = pb[k & 1]
    // and writes p_new = pb[(k + 1) & 1]
    double* pb[2] = {p, p2};
    auto iteration = [&](int k) -> mf_status {
        double* p_old = pb[k & 1];
        double* p_new = pb[(k + 1) & 1];
        k_spmv_dir_dot<<<spmv_blocks, kThreads, 0, s>>>(n, a.row_ptr, a.col_idx, a.values, z, p_old, p_new, q, sc,
                                                        partial, cnt);
        if (!external) {
            k_update_dots<<<vec_blocks, kThreads, 0, s>>>(n, sc, a.x, r, p_new, q, dinv, z, jac, partial, vec_blocks,
                                                          cnt + 1);
            return MF_OK;
        }
        k_update<<<vec_blocks, kThreads, 0, s>>>(n, sc, a.x, r, r_old, p_new, q, dinv, z, -1, flexible);
        {
            mf_status st = a.apply(a.apply_ctx, r, z, s);
            if (st != MF_OK) return st;
            k_dots<<<vec_blocks, kThreads, 0, s>>>(n, r, z, nullptr, partial, vec_blocks, nullptr, nullptr, 0);
            k_check_external<<<1, kThreads, 0, s>>>(partial, vec_blocks, sc, flag);
            k_jacobi_if<<<vec_blocks, kThreads, 0, s>>>(n, flag, dinv, r, z);
        }
        k_dots<<<vec_blocks, kThreads, 0, s>>>(n, r, z, flexible ? r_old : nullptr, partial, vec_blocks, cnt + 1, sc,
                                               flexible);
        return MF_OK;
    };

    int chunk = a.check_every > 0 ? a.check_every : 8;
    // capture one chunk of iterations as a graph when the preconditioner allows it; a
    // graphed chunk is even so that the direction buffers are in step across replays
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    bool use_graph = a.use_graph && (!external || a.apply_graph_safe);
    if (use_graph) chunk += chunk & 1;
    if (use_graph) {
        hipStreamCaptureMode mode = hipStreamCaptureModeThreadLocal;
        if (hipStreamBeginCapture(s, mode) == hipSuccess) {
            mf_status st = MF_OK;
            for (int k = 0; k < chunk && st == MF_OK; ++k) st = iteration(k);
            hipError_t e = hipStreamEndCapture(s, &graph);
            if (st != MF_OK) return st;
            if (e != hipSuccess || hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                use_graph = false;
                (void)hipGetLastError();
            }
        } else {
            use_graph = false;
            (void)hipGetLastError();
        }
    }
    struct GraphFree {
        hipGraphExec_t* e;
        hipGraph_t* g;
        ~GraphFree() {
            if (*e) (void)hipGraphExecDestroy(*e);
            if (*g) (void)hipGraphDestroy(*g);
        }
    } gf{&exec, &graph};

    double h[S_COUNT];
    int it = 0;
    const double tol = a.tol;
    while (it < a.maxit) {
        const int todo = std::min(chunk, a.maxit - it);
        if (use_graph && todo == chunk) {
            MF_HIP(hipGraphLaunch(exec, s));
        } else {
            for (int k = 0; k < todo; ++k) {
                mf_status st = iteration(it + k);
                if (st != MF_OK) return st;
            }
        }
        MF_HIP(hipGetLastError());
        it += todo;
        MF_HIP(hipMemcpyAsync(h, sc, sizeof(h), hipMemcpyDeviceToHost, s));
        MF_HIP(hipStreamSynchronize(s));
        res->fallbacks = (int)h[S_FALLBACK];
        if (h[S_BREAK] != 0.0 || !std::isfinite(h[S_RR])) {
            res->iterations = it;
            return set_error(MF_ERR_NONFINITE, "PCG breakdown (p.Kp <= 0 or r.z <= 0) near iteration %d", it);
        }
        if (std::sqrt(h[S_RR]) / bnorm <= tol) {
            // true residual as judge
            k_true_res<<<spmv_blocks, kThreads, 0, s>>>(n, a.row_ptr, a.col_idx, a.values, a.x, a.b, partial,
                                                        spmv_blocks);
            k_reduce2<<<1, kThreads, 0, s>>>(partial, spmv_blocks, sc + S_COUNT);
            MF_HIP(hipMemcpyAsync(hb2, sc + S_COUNT, sizeof(hb2), hipMemcpyDeviceToHost, s));
            MF_HIP(hipStreamSynchronize(s));
            res->true_relres = std::sqrt(hb2[0]) / bnorm;
            if (res->true_relres <= tol) {
                res->iterations = it;
                res->converged = 1;
                return MF_OK;
            }
        }
    }
    k_true_res<<<spmv_blocks, kThreads, 0, s>>>(n, a.row_ptr, a.col_idx, a.values, a.x, a.b, partial, spmv_blocks);
    k_reduce2<<<1, kThreads, 0, s>>>(partial, spmv_blocks, sc + S_COUNT);
    MF_HIP(hipMemcpyAsync(hb2, sc + S_COUNT, sizeof(hb2), hipMemcpyDeviceToHost, s));
    MF_HIP(hipStreamSynchronize(s));
    res->true_relres = std::sqrt(hb2[0]) / bnorm;
    res->iterations = it;
    return set_error(MF_ERR_NOT_CONVERGED, "PCG reached maxit = %d (true relative residual %.3e)", a.maxit,
                     res->true_relres);
}

}  // namespace mf
