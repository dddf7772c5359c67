// Preconditioned conjugate gradients on an assembled K (the linear solve of Sec. 2.2 D-4,
// which the paper leaves open).  FP64 throughout.
//
// One Jacobi iteration, all scalars kept on the device:
//   k_spmv_ell_dot q = K p and block partial sums of p.q on an ELL copy of K made once
//                  per solve (slot-major, one row per lane, so every load of a wave is
//                  one contiguous access); CSR with four lanes per row when the padding
//                  would be large.  Rows are split into one contiguous range per block,
//                  laid out so that each XCD (workgroups go to the 8 XCDs round robin)
//                  streams one contiguous eighth of K and gathers from one eighth of p.
//                  BiCGStab on node-major 4-field rows (the Newton tangent) uses
//                  k_spmv_nodes_dot instead: K in place, columns from the node graph.
//   k_reduce_alpha one block: alpha = (r.z) / (p.q) from the partials in a fixed order
//   k_update_dots  x += alpha p, r -= alpha q, z = D^-1 r, block partials of r.z and r.r
//   k_reduce_beta  one block: beta = (r.z)_new / (r.z)
//   k_dir          p = z + beta p
// Partial sums use a fixed order, so a run is bit-reproducible.  Chunks of iterations
// are captured once into a HIP graph and replayed; between chunks the host reads the
// recurrence residual, and a candidate solution is accepted only when the true residual
// |b - K x| / |b| meets the tolerance.
//
// Preconditioners: Jacobi (z = r / diag K), none, or an external apply (the learned
// network) that writes z from r; for the external one the flexible beta
// (z.(r - r_old)) / (r.z)_old is used, and any iteration with z.r <= 0 or a non-finite z
// falls back to the Jacobi z.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "mf_internal.h"
#include "pcg.h"

namespace mf {
namespace {

constexpr int kThreads = 256;
constexpr int kLanesPerRow = 4;
constexpr int kSlots = kThreads / kLanesPerRow;  // rows per block per step
constexpr int kUnroll = 8;                       // row loads issued together (32 entries)
constexpr int kSpmvBlocks = 2048;                // a multiple of the 8 XCDs
constexpr int kVecBlocks = 2048;
constexpr int kXcds = 8;

// Scalars (device): RZ = r.z, PQ, ALPHA, BETA, RR, FALLBACK, BREAK
enum { S_RZ = 0, S_PQ, S_ALPHA, S_BETA, S_RR, S_FALLBACK, S_BREAK, S_COUNT };

__device__ __forceinline__ double row_lanes_sum(double v)
{
#pragma unroll
    for (int off = kLanesPerRow / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kLanesPerRow);
    return v;
}

// sum over k in [k0, k1) of v[k] x[ci[k]] for this lane's share (stride kLanesPerRow);
// the first kUnroll loads of the lane are issued before any is used
__device__ __forceinline__ double row_dot(int k0, int k1, int lane, const int32_t* __restrict__ ci,
                                          const double* __restrict__ v, const double* __restrict__ x)
{
    double vals[kUnroll];
    int cols[kUnroll];
#pragma unroll
    for (int t = 0; t < kUnroll; ++t) {
        const int k = k0 + lane + t * kLanesPerRow;
        const bool in = k < k1;
        vals[t] = in ? v[k] : 0.0;
        cols[t] = in ? ci[k] : -1;
    }
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < kUnroll; ++t)
        if (cols[t] >= 0) s = fma(vals[t], x[cols[t]], s);
    for (int k = k0 + lane + kUnroll * kLanesPerRow; k < k1; k += kLanesPerRow) s = fma(v[k], x[ci[k]], s);
    return s;
}

// Sum over the block, returned in every thread.
__device__ __forceinline__ double block_sum_all(double v, double* sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    __syncthreads();  // sh may still be read by a previous call
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < (int)(blockDim.x / 64); ++k) s += sh[k];
    return s;
}

// Sum of nb partials in a fixed order (the same in every block), in every thread.
__device__ __forceinline__ double sum_partials(const double* __restrict__ partial, int nb, double* sh)
{
    double v = 0.0;
    for (int k = threadIdx.x; k < nb; k += blockDim.x) v += partial[k];
    return block_sum_all(v, sh);
}

// Contiguous row range of block b (XCD-aware order).
__device__ __forceinline__ void row_range(int n, int& r0, int& r1)
{
    const int nb = gridDim.x;
    const int per_xcd = nb / kXcds;
    const int logical = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
    const int rows = ((n + nb - 1) / nb + kSlots - 1) / kSlots * kSlots;
    r0 = min(n, logical * rows);
    r1 = min(n, r0 + rows);
}

// y = A x (CSR, 16 lanes per row); partial[block] = sum of w[row] y[row] (w may be null)
__global__ void __launch_bounds__(kThreads) k_spmv_dot(int n, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci,
                                                       const double* __restrict__ v,
                                                       const double* __restrict__ x, double* __restrict__ y,
                                                       const double* __restrict__ w, double* __restrict__ partial)
{
    __shared__ double sh[kThreads / 64];
    const int lane = threadIdx.x % kLanesPerRow;
    const int sub = threadIdx.x / kLanesPerRow;
    int r0, r1;
    row_range(n, r0, r1);
    double acc_dot = 0.0;
    for (int base = r0; base < r1; base += kSlots) {
        const int row = base + sub;
        double s = 0.0;
        if (row < r1) s = row_dot(rp[row], rp[row + 1], lane, ci, v, x);
        s = row_lanes_sum(s);
        if (row < r1 && lane == 0) {
            y[row] = s;
            if (w) acc_dot = fma(w[row], s, acc_dot);
        }
    }
    if (partial) {
        const double t = block_sum_all(acc_dot, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = t;
    }
}

// Longest row (for the ELL width).
__global__ void k_max_row(int n, const int32_t* __restrict__ rp, int* __restrict__ out)
{
    int m = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        m = max(m, rp[i + 1] - rp[i]);
    atomicMax(out, m);
}

// CSR -> ELL, slot-major: entry t of row i at t * n + i, padded with (i, 0.0)
__global__ void __launch_bounds__(kThreads) k_to_ell(int n, int width, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                     int32_t* __restrict__ ecol, double* __restrict__ eval)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int k0 = rp[i], len = rp[i + 1] - k0;
        for (int t = 0; t < width; ++t) {
            const int64_t o = (int64_t)t * n + i;
            const bool in = t < len;
            ecol[o] = in ? ci[k0 + t] : i;
            eval[o] = in ? v[k0 + t] : 0.0;
        }
    }
}

// y = A x in ELL (one row per lane, every load of a wave is one contiguous 512-byte
// access); partial[block] = sum of w[row] y[row].  XCD-aware contiguous row ranges.
__global__ void __launch_bounds__(kThreads) k_spmv_ell_dot(int n, int width, const int32_t* __restrict__ ecol,
                                                           const double* __restrict__ eval,
                                                           const double* __restrict__ x, double* __restrict__ y,
                                                           const double* __restrict__ w, double* __restrict__ partial)
{
    __shared__ double sh[kThreads / 64];
    const int nb = gridDim.x;
    const int per_xcd = nb / kXcds;
    const int logical = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
    const int rows = ((n + nb - 1) / nb + kThreads - 1) / kThreads * kThreads;
    const int r0 = min(n, logical * rows), r1 = min(n, r0 + rows);
    double acc_dot = 0.0;
    for (int row = r0 + threadIdx.x; row < r1; row += kThreads) {
        double s = 0.0;
#pragma unroll 9
        for (int t = 0; t < width; ++t) {
            const int64_t o = (int64_t)t * n + row;
            s = fma(eval[o], x[ecol[o]], s);
        }
        y[row] = s;
        if (w) acc_dot = fma(w[row], s, acc_dot);
    }
    if (partial) {
        const double t = block_sum_all(acc_dot, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = t;
    }
}

// y = A x for node-major rows of four fully coupled fields, with the columns taken from
// the node graph: row (v, f) starts at 16 P_v + 4 deg_v f (P_v, deg_v: node v's offset
// and degree) and its entry o has column 4 w + o % 4, w the (o / 4)-th neighbour of v.
// 8 lanes per row read 8 bytes per entry (12 for CSR or ELL) and K needs no copy.
// partial[block] = sum of w[row] y[row], in a fixed order.
__global__ void __launch_bounds__(kThreads) k_spmv_nodes_dot(int n, const int32_t* __restrict__ np,
                                                             const int32_t* __restrict__ nb,
                                                             const double* __restrict__ A,
                                                             const double* __restrict__ x, double* __restrict__ y,
                                                             const double* __restrict__ w, double* __restrict__ partial)
{
    __shared__ double sh[kThreads / 64];
    constexpr int kLanes = 8;
    const int lane = threadIdx.x % kLanes, g = lane % 4;
    const int rows_per_pass = gridDim.x * (kThreads / kLanes);
    double acc_dot = 0.0;
    for (int row = (blockIdx.x * kThreads + threadIdx.x) / kLanes; row < n; row += rows_per_pass) {
        const int p0 = np[row / 4], len = 4 * (np[row / 4 + 1] - p0);
        const double* a = A + 16 * (int64_t)p0 + (int64_t)len * (row % 4);
        const int32_t* nbr = nb + p0;
        double s = 0.0;
#pragma unroll 4
        for (int o = lane; o < len; o += kLanes) s = fma(a[o], x[4 * nbr[o / 4] + g], s);
#pragma unroll
        for (int off = kLanes / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kLanes);
        if (lane == 0) {
            y[row] = s;
            if (w) acc_dot = fma(w[row], s, acc_dot);
        }
    }
    if (partial) {
        const double t = block_sum_all(acc_dot, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = t;
    }
}

// one block: alpha = (r.z) / (p.q) from the SpMV partials
__global__ void k_reduce_alpha(const double* __restrict__ pq_part, int nb, double* s)
{
    __shared__ double sh[kThreads / 64];
    const double pq = sum_partials(pq_part, nb, sh);
    if (threadIdx.x == 0) {
        const bool ok = pq > 0.0 && isfinite(pq);
        s[S_PQ] = pq;
        s[S_ALPHA] = ok ? s[S_RZ] / pq : 0.0;
        if (!ok) s[S_BREAK] = 1.0;
    }
}

// Jacobi (or no) preconditioner, one pass: x += alpha p; r -= alpha q; z = D^-1 r (or r);
// partials [0..nb) r.z, [nb..2nb) r.r, [2nb..3nb) 0
__global__ void __launch_bounds__(kThreads) k_update_dots(int n, const double* __restrict__ s,
                                                          double* __restrict__ x, double* __restrict__ r,
                                                          const double* __restrict__ p, const double* __restrict__ q,
                                                          const double* __restrict__ dinv, double* __restrict__ z,
                                                          int jacobi, double* __restrict__ partial)
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
    const double a = block_sum_all(rz, sh);
    const double b = block_sum_all(rr, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = a;
        partial[gridDim.x + blockIdx.x] = b;
        partial[2 * gridDim.x + blockIdx.x] = 0.0;
    }
}

// External preconditioner: x += alpha p; r_old = r; r -= alpha q (z comes from the apply)
__global__ void __launch_bounds__(kThreads) k_update_ext(int n, const double* __restrict__ s,
                                                         double* __restrict__ x, double* __restrict__ r,
                                                         double* __restrict__ r_old, const double* __restrict__ p,
                                                         const double* __restrict__ q)
{
    const double alpha = s[S_ALPHA];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        x[i] = fma(alpha, p[i], x[i]);
        const double ro = r[i];
        r_old[i] = ro;
        r[i] = fma(-alpha, q[i], ro);
    }
}

// partials [0..nb) r.z, [nb..2nb) r.r, [2nb..3nb) z.r_old (r_old may be null)
__global__ void __launch_bounds__(kThreads) k_dots(int n, const double* __restrict__ r, const double* __restrict__ z,
                                                   const double* __restrict__ r_old, double* __restrict__ partial)
{
    __shared__ double sh[kThreads / 64];
    double rz = 0.0, rr = 0.0, zro = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double ri = r[i], zi = z[i];
        rz = fma(ri, zi, rz);
        rr = fma(ri, ri, rr);
        if (r_old) zro = fma(zi, r_old[i], zro);
    }
    const double a = block_sum_all(rz, sh);
    const double b = block_sum_all(rr, sh);
    const double c = block_sum_all(zro, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = a;
        partial[gridDim.x + blockIdx.x] = b;
        partial[2 * gridDim.x + blockIdx.x] = c;
    }
}

// one block: beta from the dot partials (flexible: (z.r - z.r_old) / rz_old); first
// call (init != 0) only records r.z and r.r
__global__ void k_reduce_beta(const double* __restrict__ partial, int nb, double* s, int flexible, int init)
{
    __shared__ double sh[kThreads / 64];
    const double rz = sum_partials(partial, nb, sh);
    const double rr = sum_partials(partial + nb, nb, sh);
    const double zro = sum_partials(partial + 2 * nb, nb, sh);
    if (threadIdx.x == 0) {
        const double rz_old = s[S_RZ];
        const double num = flexible ? rz - zro : rz;
        s[S_BETA] = (!init && rz_old != 0.0) ? num / rz_old : 0.0;
        s[S_RZ] = rz;
        s[S_RR] = rr;
        if (!(rz > 0.0) || !isfinite(rz)) s[S_BREAK] = 1.0;
    }
}

__global__ void __launch_bounds__(kThreads) k_dir(int n, const double* __restrict__ s, const double* __restrict__ z,
                                                  double* __restrict__ p)
{
    const double beta = s[S_BETA];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = fma(beta, p[i], z[i]);
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
        z[i] = jacobi ? dinv[i] * b[i] : b[i];
        p[i] = z[i];
    }
}

// true residual partial sums: |b - A x|^2 and |b|^2
__global__ void __launch_bounds__(kThreads) k_true_res(int n, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                       const double* __restrict__ x, const double* __restrict__ b,
                                                       double* __restrict__ partial)
{
    __shared__ double sh[kThreads / 64];
    const int lane = threadIdx.x % kLanesPerRow;
    const int sub = threadIdx.x / kLanesPerRow;
    int r0, r1;
    row_range(n, r0, r1);
    double e2 = 0.0, b2 = 0.0;
    for (int base = r0; base < r1; base += kSlots) {
        const int row = base + sub;
        double sacc = 0.0;
        if (row < r1) sacc = row_dot(rp[row], rp[row + 1], lane, ci, v, x);
        sacc = row_lanes_sum(sacc);
        if (row < r1 && lane == 0) {
            const double e = b[row] - sacc;
            e2 = fma(e, e, e2);
            b2 = fma(b[row], b[row], b2);
        }
    }
    const double a = block_sum_all(e2, sh);
    const double c = block_sum_all(b2, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = a;
        partial[gridDim.x + blockIdx.x] = c;
    }
}

// restart from the current x: r = b - A x, z = D^-1 r (or r), p = z
__global__ void __launch_bounds__(kThreads) k_restart(int n, const int32_t* __restrict__ rp,
                                                      const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                      const double* __restrict__ x, const double* __restrict__ b,
                                                      const double* __restrict__ dinv, int jacobi,
                                                      double* __restrict__ r, double* __restrict__ z,
                                                      double* __restrict__ p)
{
    const int lane = threadIdx.x % kLanesPerRow;
    const int sub = threadIdx.x / kLanesPerRow;
    int r0, r1;
    row_range(n, r0, r1);
    for (int base = r0; base < r1; base += kSlots) {
        const int row = base + sub;
        double sacc = 0.0;
        if (row < r1) sacc = row_dot(rp[row], rp[row + 1], lane, ci, v, x);
        sacc = row_lanes_sum(sacc);
        if (row < r1 && lane == 0) {
            const double ri = b[row] - sacc;
            const double zi = jacobi ? dinv[row] * ri : ri;
            r[row] = ri;
            z[row] = zi;
            p[row] = zi;
        }
    }
}

__global__ void k_reduce2(const double* __restrict__ partial, int nb, double* __restrict__ out)
{
    __shared__ double sh[kThreads / 64];
    const double A = sum_partials(partial, nb, sh);
    const double C = sum_partials(partial + nb, nb, sh);
    if (threadIdx.x == 0) {
        out[0] = A;
        out[1] = C;
    }
}

// z := Jacobi z where the external preconditioner failed (z.r <= 0 or non-finite z)
__global__ void k_check_external(const double* __restrict__ partial_rz, int nb, double* __restrict__ s, int* flag)
{
    __shared__ double sh[kThreads / 64];
    const double rz = sum_partials(partial_rz, nb, sh);
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

// ------------------------------------------------------------------------------------
// BiCGStab for non-symmetric K (the Newton tangent of the flow form), right-preconditioned
// by Jacobi (M = diag K) or by an external apply (a multigrid cycle, which then overwrites
// ph and sh), from x0 = 0 with the shadow residual rh = b, all scalars on the device.
// One iteration:
//   k_bcg_dir              p = r + beta (p - omega v),  ph = M^-1 p
//   SpMV                   v = K ph, partials rh.v
//   k_bcg_alpha (1 block)  alpha = rho / rh.v
//   k_bcg_s                s = r - alpha v (in r),  sh = M^-1 s
//   SpMV                   t = K sh
//   k_bcg_dots2            partials t.s and t.t
//   k_bcg_omega (1 block)  omega = t.s / t.t
//   k_bcg_update           x += alpha ph + omega sh,  r = s - omega t, partials rh.r, r.r
//   k_bcg_beta  (1 block)  rho = rh.r, r.r; beta = (rho / rho_old)(alpha / omega)
// A zero or non-finite rh.v, t.t, t.s or rho sets the breakdown flag (alpha or omega is
// then 0, so x stays finite) and the host judges the true residual.
// ------------------------------------------------------------------------------------
enum { B_RHO = 0, B_ALPHA, B_OMEGA, B_BETA, B_RR, B_BREAK, B_COUNT };

__global__ void k_bcg_beta(const double* __restrict__ partial, int nb, double* s, int init)
{
    __shared__ double sh[kThreads / 64];
    const double rho = sum_partials(partial, nb, sh);
    const double rr = sum_partials(partial + nb, nb, sh);
    if (threadIdx.x == 0) {
        const double rho_old = s[B_RHO], alpha = s[B_ALPHA], omega = s[B_OMEGA];
        double beta = 0.0;
        if (init) s[B_BREAK] = 0.0;  // a (re)start clears the breakdown flag
        if (!init) {
            if (rho_old != 0.0 && omega != 0.0) beta = (rho / rho_old) * (alpha / omega);
            else s[B_BREAK] = 1.0;
        }
        if (!isfinite(rho) || rho == 0.0) s[B_BREAK] = 1.0;
        s[B_BETA] = beta;
        s[B_RHO] = rho;
        s[B_RR] = rr;
    }
}

__global__ void __launch_bounds__(kThreads) k_bcg_dir(int n, const double* __restrict__ s,
                                                      const double* __restrict__ r, const double* __restrict__ v,
                                                      const double* __restrict__ dinv, double* __restrict__ p,
                                                      double* __restrict__ ph)
{
    const double beta = s[B_BETA], omega = s[B_OMEGA];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double pi = fma(beta, fma(-omega, v[i], p[i]), r[i]);
        p[i] = pi;
        ph[i] = dinv[i] * pi;
    }
}

__global__ void k_bcg_alpha(const double* __restrict__ part, int nb, double* s)
{
    __shared__ double sh[kThreads / 64];
    const double rv = sum_partials(part, nb, sh);
    if (threadIdx.x == 0) {
        const bool ok = rv != 0.0 && isfinite(rv);
        s[B_ALPHA] = ok ? s[B_RHO] / rv : 0.0;
        if (!ok) s[B_BREAK] = 1.0;
    }
}

__global__ void __launch_bounds__(kThreads) k_bcg_s(int n, const double* __restrict__ s, double* __restrict__ r,
                                                    const double* __restrict__ v, const double* __restrict__ dinv,
                                                    double* __restrict__ shat)
{
    const double alpha = s[B_ALPHA];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double si = fma(-alpha, v[i], r[i]);
        r[i] = si;
        shat[i] = dinv[i] * si;
    }
}

// partials [0..nb) t.s, [nb..2nb) t.t
__global__ void __launch_bounds__(kThreads) k_bcg_dots2(int n, const double* __restrict__ t,
                                                        const double* __restrict__ sv, double* __restrict__ partial)
{
    __shared__ double sh[kThreads / 64];
    double ts = 0.0, tt = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double ti = t[i];
        ts = fma(ti, sv[i], ts);
        tt = fma(ti, ti, tt);
    }
    const double a = block_sum_all(ts, sh);
    const double b = block_sum_all(tt, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = a;
        partial[gridDim.x + blockIdx.x] = b;
    }
}

__global__ void k_bcg_omega(const double* __restrict__ partial, int nb, double* s)
{
    __shared__ double sh[kThreads / 64];
    const double ts = sum_partials(partial, nb, sh);
    const double tt = sum_partials(partial + nb, nb, sh);
    if (threadIdx.x == 0) {
        const bool ok = tt > 0.0 && isfinite(tt) && isfinite(ts);
        s[B_OMEGA] = ok ? ts / tt : 0.0;
        if (!ok || ts == 0.0) s[B_BREAK] = 1.0;
    }
}

// x += alpha ph + omega sh; r = s - omega t (s is in r); partials [0..nb) rh.r, [nb..2nb) r.r
__global__ void __launch_bounds__(kThreads) k_bcg_update(int n, const double* __restrict__ s, double* __restrict__ x,
                                                         double* __restrict__ r, const double* __restrict__ t,
                                                         const double* __restrict__ ph,
                                                         const double* __restrict__ shat,
                                                         const double* __restrict__ rh, double* __restrict__ partial)
{
    __shared__ double sh[kThreads / 64];
    const double alpha = s[B_ALPHA], omega = s[B_OMEGA];
    double a = 0.0, b = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        x[i] = fma(omega, shat[i], fma(alpha, ph[i], x[i]));
        const double ri = fma(-omega, t[i], r[i]);
        r[i] = ri;
        a = fma(rh[i], ri, a);
        b = fma(ri, ri, b);
    }
    const double A = block_sum_all(a, sh);
    const double B = block_sum_all(b, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = A;
        partial[gridDim.x + blockIdx.x] = B;
    }
}

// restart from the current x: r = rh = b - Ax (Ax given), p = v = 0; partials rh.r, r.r
__global__ void __launch_bounds__(kThreads) k_bcg_restart(int n, const double* __restrict__ b,
                                                          const double* __restrict__ ax, double* __restrict__ r,
                                                          double* __restrict__ rh, double* __restrict__ p,
                                                          double* __restrict__ vv, double* __restrict__ partial)
{
    __shared__ double sh[kThreads / 64];
    double a = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double ri = b[i] - ax[i];
        r[i] = ri;
        rh[i] = ri;
        p[i] = 0.0;
        vv[i] = 0.0;
        a = fma(ri, ri, a);
    }
    const double A = block_sum_all(a, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = A;
        partial[gridDim.x + blockIdx.x] = A;
    }
}

// diag inverse (Jacobi or identity), x = 0, r = rh = b, p = v = 0; partials rh.r, r.r
__global__ void __launch_bounds__(kThreads) k_bcg_init(int n, const int32_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci, const double* __restrict__ v,
                                                       const double* __restrict__ b, double* __restrict__ dinv,
                                                       double* __restrict__ x, double* __restrict__ r,
                                                       double* __restrict__ rh, double* __restrict__ p,
                                                       double* __restrict__ vv, int jacobi, double* __restrict__ partial)
{
    __shared__ double sh[kThreads / 64];
    double a = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double di = 0.0;
        if (jacobi)
            for (int k = rp[i]; k < rp[i + 1]; ++k)
                if (ci[k] == i) di = v[k];
        dinv[i] = (jacobi && di != 0.0) ? 1.0 / di : 1.0;
        x[i] = 0.0;
        const double bi = b[i];
        r[i] = bi;
        rh[i] = bi;
        p[i] = 0.0;
        vv[i] = 0.0;
        a = fma(bi, bi, a);
    }
    const double A = block_sum_all(a, sh);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = A;
        partial[gridDim.x + blockIdx.x] = A;
    }
}

int spmv_blocks_for(int n)
{
    const int want = (n + kSlots - 1) / kSlots;
    return std::max(kXcds, std::min(kSpmvBlocks, (want + kXcds - 1) / kXcds * kXcds));
}

}  // namespace

mf_status run_spmv(const mf_csr* A, const double* x, double* y, hipStream_t s)
{
    const int n = (int)A->n_rows;
    if (n == 0) return MF_OK;
    k_spmv_dot<<<spmv_blocks_for(n), kThreads, 0, s>>>(n, A->row_ptr, A->col_idx, A->values, x, y, nullptr, nullptr);
    MF_HIP(hipGetLastError());
    return MF_OK;
}

namespace {
// dinv r r_old z p q | pq partials | dot partials [3 nb] | scalars | flag, each slot
// rounded up to 256 bytes
constexpr int64_t slot256(int64_t v) { return (v + 31) / 32 * 32; }
constexpr int64_t scratch_doubles_for(int64_t n)
{
    return 6 * slot256(n) + slot256(kSpmvBlocks) + slot256(3 * (kVecBlocks > kSpmvBlocks ? kVecBlocks : kSpmvBlocks)) +
           slot256(S_COUNT + 2) + slot256(1);
}

// Fixed device workspace of mf_pcg_noalloc: 6 vectors of up to 2^20 rows and the
// partial sums (about 48 MiB, held by every GPU the library runs on until the process
// ends).  Host code reaches it only through the address hipGetSymbolAddress returns.
constexpr int64_t kNoAllocMaxRows = (int64_t)1 << 20;
constexpr int64_t kScratchDoubles = scratch_doubles_for(kNoAllocMaxRows);
__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
double* g_scratch_ptr[64] = {};

// Device address of this device's copy of `scratch` (looked up once per device, with
// the device current).
mf_status scratch_on_current_device(double** out)
{
    int dev = 0;
    MF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_error(MF_ERR_UNSUPPORTED, "device index %d", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        MF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_error(MF_ERR_HIP, "hipGetSymbolAddress returned NULL for the PCG workspace");
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return MF_OK;
}
}  // namespace

int64_t pcg_scratch_doubles(int64_t n) { return scratch_doubles_for(n); }

int64_t pcg_noalloc_max_rows() { return kNoAllocMaxRows; }

mf_status run_pcg_noalloc(const PcgArgs& a, mf_pcg_result* res)
{
    if (a.n > kNoAllocMaxRows)
        return set_error(MF_ERR_ARG, "n_rows %lld exceeds the fixed workspace of mf_pcg_noalloc (%lld rows)",
                         (long long)a.n, (long long)kNoAllocMaxRows);
    if (a.precond != MF_PRECOND_NONE && a.precond != MF_PRECOND_JACOBI)
        return set_error(MF_ERR_UNSUPPORTED, "mf_pcg_noalloc takes MF_PRECOND_NONE or MF_PRECOND_JACOBI");
    double* ws = nullptr;
    mf_status st = scratch_on_current_device(&ws);
    if (st != MF_OK) return st;
    return run_pcg(a, res, ws);
}

mf_status run_pcg(const PcgArgs& a, mf_pcg_result* res, double* scratch)
{
    const int n = (int)a.n;
    hipStream_t s = a.stream;
    res->iterations = 0;
    res->true_relres = 0.0;
    res->fallbacks = 0;
    res->restarts = 0;
    res->converged = 0;
    if (n == 0) {
        res->converged = 1;
        return MF_OK;
    }
    const int vec_blocks = (int)std::min<int64_t>(kVecBlocks, (n + kThreads - 1) / kThreads);
    const int spmv_blocks = spmv_blocks_for(n);
    const int nb = std::max(vec_blocks, spmv_blocks);

    // workspace: dinv r r_old z p q | pq partials | dot partials [3 nb] | scalars | flag
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
    double *dinv, *r, *r_old, *z, *p, *q, *pq_part, *partial, *sc;
    int* flag;
    if (scratch) {
        // caller-provided workspace of pcg_scratch_doubles(n) doubles (256-byte slots);
        // every value is written before it is read, so no clearing is needed
        auto slot = [](int64_t v) { return (v + 31) / 32 * 32; };
        double* w = scratch;
        auto take = [&](int64_t cnt) {
            double* t = w;
            w += slot(cnt);
            return t;
        };
        dinv = take(n);
        r = take(n);
        r_old = take(n);
        z = take(n);
        p = take(n);
        q = take(n);
        pq_part = take(kSpmvBlocks);
        partial = take(3 * (int64_t)std::max(kVecBlocks, kSpmvBlocks));
        sc = take(S_COUNT + 2);
        flag = (int*)take(1);
    } else {
        dinv = (double*)dalloc(sizeof(double) * n);
        r = (double*)dalloc(sizeof(double) * n);
        r_old = (double*)dalloc(sizeof(double) * n);
        z = (double*)dalloc(sizeof(double) * n);
        p = (double*)dalloc(sizeof(double) * n);
        q = (double*)dalloc(sizeof(double) * n);
        pq_part = (double*)dalloc(sizeof(double) * spmv_blocks);
        partial = (double*)dalloc(sizeof(double) * 3 * nb);
        sc = (double*)dalloc(sizeof(double) * (S_COUNT + 2));
        flag = (int*)dalloc(sizeof(int));
        if (!dinv || !r || !r_old || !z || !p || !q || !pq_part || !partial || !sc || !flag)
            return set_error(MF_ERR_OOM, "PCG workspace allocation failed");
    }

    bool external = a.precond == MF_PRECOND_EXTERNAL;  // false again after a restart
    const int jac = a.precond == MF_PRECOND_NONE ? 0 : 1;  // Jacobi z (also the external fallback)

    // ELL copy of K for the iterations when the padding stays small (not with a
    // caller-provided workspace: the copy is as large as K)
    int width = 0, nnz32 = 0;
    if (!scratch) {
        int* dmax = (int*)dalloc(sizeof(int));
        if (!dmax) return set_error(MF_ERR_OOM, "PCG workspace allocation failed");
        MF_HIP(hipMemsetAsync(dmax, 0, sizeof(int), s));
        k_max_row<<<vec_blocks, kThreads, 0, s>>>(n, a.row_ptr, dmax);
        MF_HIP(hipMemcpyAsync(&width, dmax, sizeof(int), hipMemcpyDeviceToHost, s));
        MF_HIP(hipMemcpyAsync(&nnz32, a.row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        MF_HIP(hipStreamSynchronize(s));
    }
    int32_t* ecol = nullptr;
    double* eval = nullptr;
    const int64_t nnz = nnz32;
    if (!scratch && width > 0 && (int64_t)width * n <= nnz + nnz / 2) {
        ecol = (int32_t*)dalloc(sizeof(int32_t) * (size_t)width * n);
        eval = (double*)dalloc(sizeof(double) * (size_t)width * n);
        if (ecol && eval) {
            k_to_ell<<<vec_blocks, kThreads, 0, s>>>(n, width, a.row_ptr, a.col_idx, a.values, ecol, eval);
        } else {
            (void)hipGetLastError();
            ecol = nullptr;
            eval = nullptr;
        }
    }
    auto spmv_pq = [&]() {
        if (ecol)
            k_spmv_ell_dot<<<spmv_blocks, kThreads, 0, s>>>(n, width, ecol, eval, p, q, p, pq_part);
        else
            k_spmv_dot<<<spmv_blocks, kThreads, 0, s>>>(n, a.row_ptr, a.col_idx, a.values, p, q, p, pq_part);
    };

    k_set<<<1, 64, 0, s>>>(sc, S_COUNT + 2, 0.0);
    k_init<<<vec_blocks, kThreads, 0, s>>>(n, a.row_ptr, a.col_idx, a.values, a.b, dinv, a.x, r, z, p, jac);
    if (external) {
        mf_status st = a.apply(a.apply_ctx, r, z, s);
        if (st != MF_OK) return st;
        k_dots<<<vec_blocks, kThreads, 0, s>>>(n, r, z, nullptr, partial);
        k_check_external<<<1, kThreads, 0, s>>>(partial, vec_blocks, sc, flag);
        k_jacobi_if<<<vec_blocks, kThreads, 0, s>>>(n, flag, dinv, r, z);
        MF_HIP(hipMemcpyAsync(p, z, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
    k_dots<<<vec_blocks, kThreads, 0, s>>>(n, r, z, nullptr, partial);
    k_reduce_beta<<<1, kThreads, 0, s>>>(partial, vec_blocks, sc, 0, 1);
    MF_HIP(hipGetLastError());

    // |b|
    double hb2[2] = {0, 0};
    k_true_res<<<spmv_blocks, kThreads, 0, s>>>(n, a.row_ptr, a.col_idx, a.values, a.x, a.b, partial);
    k_reduce2<<<1, kThreads, 0, s>>>(partial, spmv_blocks, sc + S_COUNT);
    MF_HIP(hipMemcpyAsync(hb2, sc + S_COUNT, sizeof(hb2), hipMemcpyDeviceToHost, s));
    MF_HIP(hipStreamSynchronize(s));
    const double bnorm = std::sqrt(hb2[1]);
    if (bnorm == 0.0) {
        res->converged = 1;
        return MF_OK;
    }

    auto iteration = [&]() -> mf_status {
        spmv_pq();
        k_reduce_alpha<<<1, kThreads, 0, s>>>(pq_part, spmv_blocks, sc);
        if (!external) {
            k_update_dots<<<vec_blocks, kThreads, 0, s>>>(n, sc, a.x, r, p, q, dinv, z, jac, partial);
            k_reduce_beta<<<1, kThreads, 0, s>>>(partial, vec_blocks, sc, 0, 0);
        } else {
            k_update_ext<<<vec_blocks, kThreads, 0, s>>>(n, sc, a.x, r, r_old, p, q);
            mf_status st = a.apply(a.apply_ctx, r, z, s);
            if (st != MF_OK) return st;
            k_dots<<<vec_blocks, kThreads, 0, s>>>(n, r, z, nullptr, partial);
            k_check_external<<<1, kThreads, 0, s>>>(partial, vec_blocks, sc, flag);
            k_jacobi_if<<<vec_blocks, kThreads, 0, s>>>(n, flag, dinv, r, z);
            k_dots<<<vec_blocks, kThreads, 0, s>>>(n, r, z, r_old, partial);
            k_reduce_beta<<<1, kThreads, 0, s>>>(partial, vec_blocks, sc, 1, 0);
        }
        k_dir<<<vec_blocks, kThreads, 0, s>>>(n, sc, z, p);
        return MF_OK;
    };

    const int chunk = a.check_every > 0 ? a.check_every : 8;
    // capture one chunk of iterations as a graph when the preconditioner allows it
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    bool use_graph = a.use_graph && !scratch && (!external || a.apply_graph_safe);
    if (use_graph) {
        hipStreamCaptureMode mode = hipStreamCaptureModeThreadLocal;
        if (hipStreamBeginCapture(s, mode) == hipSuccess) {
            mf_status st = MF_OK;
            for (int k = 0; k < chunk && st == MF_OK; ++k) st = iteration();
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

    // Stagnation: stall_iters iterations without the recurrence residual falling below
    // kStallDrop times its best (judged at the host checks), or a recurrence residual
    // below tol whose true residual is not.  Either restarts from the current x with the
    // true residual and a Jacobi (or no) preconditioner, at most kMaxRestarts times.
    constexpr int kMaxRestarts = 8;
    constexpr double kStallDrop = 0.9;
    const int stall_iters = a.stall_iters > 0 ? a.stall_iters : 512;
    double best = 1.0;
    int it = 0, it_best = 0;
    auto restart = [&]() -> mf_status {
        if (external) {  // the rest of the solve is Jacobi-PCG; the graph held the external step
            external = false;
            use_graph = false;
        }
        k_restart<<<spmv_blocks, kThreads, 0, s>>>(n, a.row_ptr, a.col_idx, a.values, a.x, a.b, dinv, jac, r, z, p);
        k_dots<<<vec_blocks, kThreads, 0, s>>>(n, r, z, nullptr, partial);
        k_reduce_beta<<<1, kThreads, 0, s>>>(partial, vec_blocks, sc, 0, 1);
        MF_HIP(hipGetLastError());
        ++res->restarts;
        it_best = it;
        best = 1.0;
        return MF_OK;
    };

    double h[S_COUNT];
    const double tol = a.tol;
    while (it < a.maxit) {
        const int todo = std::min(chunk, a.maxit - it);
        if (use_graph && todo == chunk) {
            MF_HIP(hipGraphLaunch(exec, s));
        } else {
            for (int k = 0; k < todo; ++k) {
                mf_status st = iteration();
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
        const double rel = std::sqrt(h[S_RR]) / bnorm;
        if (rel <= tol) {
            // true residual as judge
            k_true_res<<<spmv_blocks, kThreads, 0, s>>>(n, a.row_ptr, a.col_idx, a.values, a.x, a.b, partial);
            k_reduce2<<<1, kThreads, 0, s>>>(partial, spmv_blocks, sc + S_COUNT);
            MF_HIP(hipMemcpyAsync(hb2, sc + S_COUNT, sizeof(hb2), hipMemcpyDeviceToHost, s));
            MF_HIP(hipStreamSynchronize(s));
            res->true_relres = std::sqrt(hb2[0]) / bnorm;
            if (res->true_relres <= tol) {
                res->iterations = it;
                res->converged = 1;
                return MF_OK;
            }
            if (res->restarts < kMaxRestarts) {  // the recurrence drifted from b - K x
                mf_status st = restart();
                if (st != MF_OK) return st;
            }
            continue;
        }
        if (rel < kStallDrop * best) {
            best = rel;
            it_best = it;
        } else if (it - it_best >= stall_iters && res->restarts < kMaxRestarts) {
            mf_status st = restart();
            if (st != MF_OK) return st;
        }
    }
    k_true_res<<<spmv_blocks, kThreads, 0, s>>>(n, a.row_ptr, a.col_idx, a.values, a.x, a.b, partial);
    k_reduce2<<<1, kThreads, 0, s>>>(partial, spmv_blocks, sc + S_COUNT);
    MF_HIP(hipMemcpyAsync(hb2, sc + S_COUNT, sizeof(hb2), hipMemcpyDeviceToHost, s));
    MF_HIP(hipStreamSynchronize(s));
    res->true_relres = std::sqrt(hb2[0]) / bnorm;
    res->iterations = it;
    return set_error(MF_ERR_NOT_CONVERGED, "PCG reached maxit = %d (true relative residual %.3e)", a.maxit,
                     res->true_relres);
}


mf_status run_bicgstab(const PcgArgs& a, mf_pcg_result* res)
{
    const int n = (int)a.n;
    hipStream_t s = a.stream;
    res->iterations = 0;
    res->true_relres = 0.0;
    res->fallbacks = 0;
    res->restarts = 0;
    res->converged = 0;
    if (n == 0) {
        res->converged = 1;
        return MF_OK;
    }
    const int vec_blocks = (int)std::min<int64_t>(kVecBlocks, (n + kThreads - 1) / kThreads);
    const int spmv_blocks = spmv_blocks_for(n);
    const int nb = std::max(vec_blocks, spmv_blocks);

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
    double* rh = (double*)dalloc(sizeof(double) * n);
    double* p = (double*)dalloc(sizeof(double) * n);
    double* ph = (double*)dalloc(sizeof(double) * n);
    double* v = (double*)dalloc(sizeof(double) * n);
    double* sh = (double*)dalloc(sizeof(double) * n);
    double* t = (double*)dalloc(sizeof(double) * n);
    double* xbest = (double*)dalloc(sizeof(double) * n);  // iterate of the smallest residual seen
    double* rv_part = (double*)dalloc(sizeof(double) * spmv_blocks);
    double* partial = (double*)dalloc(sizeof(double) * 2 * nb);
    double* sc = (double*)dalloc(sizeof(double) * (B_COUNT + 2));
    if (!dinv || !r || !rh || !p || !ph || !v || !sh || !t || !xbest || !rv_part || !partial || !sc)
        return set_error(MF_ERR_OOM, "BiCGStab workspace allocation failed");
    const int jac = a.precond == MF_PRECOND_JACOBI ? 1 : 0;
    // an external preconditioner (multigrid) overwrites ph and sh after the kernels that
    // form p and s; D^-1 is then the identity
    const bool ext = a.precond == MF_PRECOND_EXTERNAL;
    if (ext && !a.apply) return set_error(MF_ERR_ARG, "external preconditioner without an apply function");
    mf_status apply_status = MF_OK;
    auto apply = [&](const double* in, double* out) {
        if (!ext) return;
        mf_status e = a.apply(a.apply_ctx, in, out, s);
        if (e != MF_OK && apply_status == MF_OK) apply_status = e;
    };

    // ELL copy of K when the padding stays small (as in run_pcg); none with the node graph
    int width = 0, nnz32 = 0;
    if (!a.node_ptr) {
        int* dmax = (int*)dalloc(sizeof(int));
        if (!dmax) return set_error(MF_ERR_OOM, "BiCGStab workspace allocation failed");
        MF_HIP(hipMemsetAsync(dmax, 0, sizeof(int), s));
        k_max_row<<<vec_blocks, kThreads, 0, s>>>(n, a.row_ptr, dmax);
        MF_HIP(hipMemcpyAsync(&width, dmax, sizeof(int), hipMemcpyDeviceToHost, s));
        MF_HIP(hipMemcpyAsync(&nnz32, a.row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        MF_HIP(hipStreamSynchronize(s));
    }
    int32_t* ecol = nullptr;
    double* eval = nullptr;
    if (width > 0 && (int64_t)width * n <= (int64_t)nnz32 + nnz32 / 2) {
        ecol = (int32_t*)dalloc(sizeof(int32_t) * (size_t)width * n);
        eval = (double*)dalloc(sizeof(double) * (size_t)width * n);
        if (ecol && eval) {
            k_to_ell<<<vec_blocks, kThreads, 0, s>>>(n, width, a.row_ptr, a.col_idx, a.values, ecol, eval);
        } else {
            (void)hipGetLastError();
            ecol = nullptr;
            eval = nullptr;
        }
    }
    auto spmv = [&](const double* x_in, double* y, const double* w, double* part) {
        if (a.node_ptr)
            k_spmv_nodes_dot<<<spmv_blocks, kThreads, 0, s>>>(n, a.node_ptr, a.node_nbr, a.values, x_in, y, w, part);
        else if (ecol)
            k_spmv_ell_dot<<<spmv_blocks, kThreads, 0, s>>>(n, width, ecol, eval, x_in, y, w, part);
        else
            k_spmv_dot<<<spmv_blocks, kThreads, 0, s>>>(n, a.row_ptr, a.col_idx, a.values, x_in, y, w, part);
    };

    k_set<<<1, 64, 0, s>>>(sc, B_COUNT + 2, 0.0);
    k_bcg_init<<<vec_blocks, kThreads, 0, s>>>(n, a.row_ptr, a.col_idx, a.values, a.b, dinv, a.x, r, rh, p, v, jac,
                                               partial);
    k_bcg_beta<<<1, kThreads, 0, s>>>(partial, vec_blocks, sc, 1);
    double h[B_COUNT];
    MF_HIP(hipGetLastError());
    MF_HIP(hipMemcpyAsync(h, sc, sizeof(h), hipMemcpyDeviceToHost, s));
    MF_HIP(hipStreamSynchronize(s));
    const double bnorm = std::sqrt(h[B_RR]);
    if (bnorm == 0.0) {
        res->converged = 1;
        return MF_OK;
    }

    // each iteration ends with the reduction of rh.r and r.r (rho and beta for the next
    // one), so the scalars hold the newest residual norm when a chunk ends
    auto iteration = [&]() {
        k_bcg_dir<<<vec_blocks, kThreads, 0, s>>>(n, sc, r, v, dinv, p, ph);
        apply(p, ph);
        spmv(ph, v, rh, rv_part);
        k_bcg_alpha<<<1, kThreads, 0, s>>>(rv_part, spmv_blocks, sc);
        k_bcg_s<<<vec_blocks, kThreads, 0, s>>>(n, sc, r, v, dinv, sh);
        apply(r, sh);
        spmv(sh, t, nullptr, nullptr);
        k_bcg_dots2<<<vec_blocks, kThreads, 0, s>>>(n, t, r, partial);
        k_bcg_omega<<<1, kThreads, 0, s>>>(partial, vec_blocks, sc);
        k_bcg_update<<<vec_blocks, kThreads, 0, s>>>(n, sc, a.x, r, t, ph, sh, rh, partial);
        k_bcg_beta<<<1, kThreads, 0, s>>>(partial, vec_blocks, sc, 0);
    };

    const int chunk = a.check_every > 0 ? a.check_every : 8;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    bool use_graph = a.use_graph != 0 && (!ext || a.apply_graph_safe);
    if (use_graph) {
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            for (int k = 0; k < chunk; ++k) iteration();
            hipError_t e = hipStreamEndCapture(s, &graph);
            if (e != hipSuccess || hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                use_graph = false;
                (void)hipGetLastError();
            }
        } else {
            use_graph = false;
            (void)hipGetLastError();
        }
        if (apply_status != MF_OK) return apply_status;
    }
    struct GraphFree {
        hipGraphExec_t* e;
        hipGraph_t* g;
        ~GraphFree() {
            if (*e) (void)hipGraphExecDestroy(*e);
            if (*g) (void)hipGraphDestroy(*g);
        }
    } gf{&exec, &graph};

    double hb2[2] = {0, 0};
    auto true_relres = [&]() -> mf_status {
        k_true_res<<<spmv_blocks, kThreads, 0, s>>>(n, a.row_ptr, a.col_idx, a.values, a.x, a.b, partial);
        k_reduce2<<<1, kThreads, 0, s>>>(partial, spmv_blocks, sc + B_COUNT);
        MF_HIP(hipMemcpyAsync(hb2, sc + B_COUNT, sizeof(hb2), hipMemcpyDeviceToHost, s));
        MF_HIP(hipStreamSynchronize(s));
        res->true_relres = std::sqrt(hb2[0]) / bnorm;
        return MF_OK;
    };
    // When the recurrence claims convergence that the true residual denies (rounding
    // after large intermediate residuals separates the two), or on a breakdown, the
    // method restarts with r = rh = b - Kx: from the current x, or from the iterate of the
    // smallest recurrence residual seen when the current one has drifted more than ten
    // times above it.  A solve that ends unconverged leaves whichever of the two has the
    // smaller true residual in x.
    constexpr int kMaxRestarts = 64;
    constexpr double kDrift = 10.0;
    int restarts = 0;
    int it = 0;
    double best_rec = 1.0;  // x0 = 0
    MF_HIP(hipMemcpyAsync(xbest, a.x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    auto finish_unconverged = [&]() -> mf_status {
        mf_status st = true_relres();
        if (st != MF_OK) return st;
        const double tx = res->true_relres;
        MF_HIP(hipMemcpyAsync(t, a.x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        MF_HIP(hipMemcpyAsync(a.x, xbest, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        st = true_relres();
        if (st != MF_OK) return st;
        if (!(res->true_relres < tx) && std::isfinite(tx)) {
            MF_HIP(hipMemcpyAsync(a.x, t, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            MF_HIP(hipStreamSynchronize(s));
            res->true_relres = tx;
        }
        return MF_OK;
    };
    while (it < a.maxit) {
        const int todo = std::min(chunk, a.maxit - it);
        if (use_graph && todo == chunk) {
            MF_HIP(hipGraphLaunch(exec, s));
        } else {
            for (int k = 0; k < todo; ++k) iteration();
            if (apply_status != MF_OK) return apply_status;
        }
        MF_HIP(hipGetLastError());
        it += todo;
        MF_HIP(hipMemcpyAsync(h, sc, sizeof(h), hipMemcpyDeviceToHost, s));
        MF_HIP(hipStreamSynchronize(s));
        const bool broke = h[B_BREAK] != 0.0 || !std::isfinite(h[B_RR]);
        const double rec = std::sqrt(h[B_RR]) / bnorm;
        if (!broke && rec < best_rec) {
            best_rec = rec;
            MF_HIP(hipMemcpyAsync(xbest, a.x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        }
        if (rec <= a.tol || broke) {
            mf_status st = true_relres();
            if (st != MF_OK) return st;
            if (res->true_relres <= a.tol) {
                res->iterations = it;
                res->converged = 1;
                return MF_OK;
            }
            if (!std::isfinite(res->true_relres) || ++restarts > kMaxRestarts) {
                res->iterations = it;
                st = finish_unconverged();
                if (st != MF_OK) return st;
                return set_error(MF_ERR_NONFINITE,
                                 "BiCGStab breakdown near iteration %d after %d restarts (true relative residual %.3e)",
                                 it, restarts - 1, res->true_relres);
            }
            res->restarts = restarts;
            if (res->true_relres > kDrift * best_rec)
                MF_HIP(hipMemcpyAsync(a.x, xbest, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            spmv(a.x, t, nullptr, nullptr);
            k_bcg_restart<<<vec_blocks, kThreads, 0, s>>>(n, a.b, t, r, rh, p, v, partial);
            k_bcg_beta<<<1, kThreads, 0, s>>>(partial, vec_blocks, sc, 1);
            MF_HIP(hipGetLastError());
        }
    }
    mf_status st = true_relres();
    if (st != MF_OK) return st;
    res->iterations = it;
    if (res->true_relres <= a.tol) {
        res->converged = 1;
        return MF_OK;
    }
    st = finish_unconverged();
    if (st != MF_OK) return st;
    if (res->true_relres <= a.tol) {
        res->converged = 1;
        return MF_OK;
    }
    return set_error(MF_ERR_NOT_CONVERGED, "BiCGStab reached maxit = %d (true relative residual %.3e)", a.maxit,
                     res->true_relres);
}

}  // namespace mf
