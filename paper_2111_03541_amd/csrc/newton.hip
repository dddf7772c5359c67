// Newton iteration for the steady flow form (Sec. 2.1: the update solves K dU = -R(U) with
// the tangent K = dR/dU and is repeated until the residual vanishes; form of Sec. 4.3).
// Each step: mf_assemble in FP64 at the current state (with the Dirichlet elimination,
// so d = -R is 0 on constrained rows), |d|_2 by fixed-order partial sums, mf_bicgstab
// (Jacobi, or a multigrid cycle rebuilt for each step's tangent) for dU, and the update
// state += dU mapped from the DOF numbering to the [4][n_nodes] state layout.  The linear solves are inexact: step k asks for a relative
// residual eta_k = max(lin_tol, min(0.1, |d_k| / |d_0|)), which tightens with the Newton
// residual and so keeps the convergence superlinear; a solve that stops short of eta_k
// (iteration limit or breakdown) but lowers the residual still gives its update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "mf_internal.h"
#include "pcg.h"

namespace mf {
namespace {

constexpr int kThreads = 256;
constexpr int kBlocks = 1024;

// state[f][node] += delta[dof(node, f)]
__global__ void __launch_bounds__(kThreads) k_state_update(int64_t n_rows, int64_t n_nodes, int nf, int field_major,
                                                           const double* __restrict__ delta, double* __restrict__ state)
{
    for (int64_t dof = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; dof < n_rows;
         dof += (int64_t)gridDim.x * blockDim.x) {
        const int64_t node = field_major ? dof % n_nodes : dof / nf;
        const int64_t f = field_major ? dof / n_nodes : dof % nf;
        state[f * n_nodes + node] += delta[dof];
    }
}

// partial[block] = sum of v^2 over a grid-stride share
__global__ void __launch_bounds__(kThreads) k_sumsq(int64_t n, const double* __restrict__ v, double* __restrict__ partial)
{
    __shared__ double sh[kThreads / 64];
    double a = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a = fma(v[i], v[i], a);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kThreads / 64; ++k) t += sh[k];
        partial[blockIdx.x] = t;
    }
}

// out = sum of the nb partials, in a fixed order
__global__ void k_sum_partials(const double* __restrict__ partial, int nb, double* __restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < nb; ++k) t += partial[k];
        *out = t;
    }
}

}  // namespace
}  // namespace mf

using namespace mf;

extern "C" mf_status mf_ns_newton(const mf_pattern_t* P, const mf_form* form, const double* coords, double* state,
                                  const uint8_t* dirichlet, const mf_quadrature* quad, const mf_newton_opts* opts,
                                  mf_newton_result* res, void* stream)
{
    return mf_ns_newton_ex(P, form, coords, state, dirichlet, nullptr, 0, quad, opts, res, stream);
}

// The Newton driver behind mf_ns_newton, mf_ns_newton_ex and mf_ns_newton_mg: with mgo,
// each step's solve is preconditioned by a multigrid cycle updated for that step's K.
static mf_status newton_run(const mf_pattern_t* P, const mf_form* form, const double* coords, double* state,
                            const uint8_t* dirichlet, const mf_bset* bsets, int32_t n_bsets, const mf_mg_opts* mgo,
                            const mf_quadrature* quad, const mf_newton_opts* opts, mf_newton_result* res,
                            void* stream)
{
    if (!P || !form || !quad || !opts || !res) return set_error(MF_ERR_ARG, "NULL pattern, form, quadrature, opts or res");
    if (n_bsets < 0 || (n_bsets > 0 && !bsets)) return set_error(MF_ERR_ARG, "n_bsets < 0 or bsets NULL");
    if (form->kind != MF_FORM_NS_SUPG) return set_error(MF_ERR_ARG, "mf_ns_newton needs the flow form");
    if (P->dim != 3 || P->nf != 4) return set_error(MF_ERR_ARG, "mf_ns_newton needs a 3D pattern with 4 fields");
    if (P->n_rows > 0 && (!coords || !state)) return set_error(MF_ERR_ARG, "coords or state is NULL");
    if (opts->max_steps < 0 || opts->max_steps >= MF_NEWTON_MAX_HISTORY)
        return set_error(MF_ERR_ARG, "max_steps must be in [0, %d)", MF_NEWTON_MAX_HISTORY);
    if (!(opts->rtol >= 0.0) || !(opts->atol >= 0.0) || !(opts->lin_tol > 0.0) || opts->lin_maxit < 0)
        return set_error(MF_ERR_ARG, "tolerances must be >= 0 (lin_tol > 0) and lin_maxit >= 0");
    hipStream_t s = (hipStream_t)stream;
    res->steps = 0;
    res->converged = 0;
    res->lin_iterations = 0;
    for (int k = 0; k < MF_NEWTON_MAX_HISTORY; ++k) res->res_norm[k] = 0.0;
    const int64_t n = P->n_rows, nnz = P->nnz;
    if (n == 0) {
        res->converged = 1;
        return MF_OK;
    }
    if (n >= ((int64_t)1 << 31)) return set_error(MF_ERR_OVERFLOW, "n_rows %lld", (long long)n);

    std::vector<void*> owned;
    auto dalloc = [&](size_t bytes) -> void* {
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        owned.push_back(p);
        return p;
    };
    struct Free {
        std::vector<void*>* v;
        hipStream_t s;
        ~Free() {
            (void)hipStreamSynchronize(s);
            for (void* p : *v) (void)hipFree(p);
        }
    } fr{&owned, s};
    mf_mg_t* mg = nullptr;
    struct MgFree {
        mf_mg_t** m;
        ~MgFree() { mf_mg_destroy(*m); }
    } mgf{&mg};
    if (mgo) {
        mf_status st = mf_mg_create(P, mgo, stream, &mg);
        if (st != MF_OK) return st;
    }
    const int nb = (int)std::min<int64_t>(kBlocks, (n + kThreads - 1) / kThreads);
    double* K = (double*)dalloc(sizeof(double) * (size_t)std::max<int64_t>(nnz, 1));
    double* d = (double*)dalloc(sizeof(double) * (size_t)n);
    double* du = (double*)dalloc(sizeof(double) * (size_t)n);
    double* partial = (double*)dalloc(sizeof(double) * nb);
    double* out = (double*)dalloc(sizeof(double));
    if (!K || !d || !du || !partial || !out) return set_error(MF_ERR_OOM, "Newton workspace allocation failed");

    mf_fields F{};
    F.lin_state = state;
    // with boundary forms the elimination comes after the faces are added
    F.dirichlet = n_bsets > 0 ? nullptr : dirichlet;
    AssembleArgs elim{};
    elim.P = P;
    elim.dirichlet = dirichlet;
    elim.prec = MF_F64;
    elim.K = K;
    elim.d = d;
    elim.stream = s;
    mf_csr A{n, P->row_ptr, P->col_idx, K};
    mf_pcg_opts lo{};
    lo.tol = opts->lin_tol;
    lo.maxit = opts->lin_maxit;
    lo.check_every = opts->check_every;
    lo.use_graph = opts->use_graph;
    lo.precond = MF_PRECOND_JACOBI;

    double d0 = 0.0;
    for (int k = 0;; ++k) {
        mf_status st = mf_assemble(P, form, coords, &F, quad, MF_F64, K, d, stream);
        if (st != MF_OK) return st;
        if (n_bsets > 0) {
            for (int b = 0; b < n_bsets; ++b) {
                const mf_bset& B = bsets[b];
                st = mf_assemble_boundary(P, &B.form, coords, B.n_faces, B.face_elem, B.face_id, state, B.target,
                                          MF_F64, K, d, stream);
                if (st != MF_OK) return st;
            }
            st = apply_dirichlet(elim);
            if (st != MF_OK) return st;
        }
        int64_t bad = -1;
        st = mf_status_poll(P, &bad);
        if (st != MF_OK) return st;
        k_sumsq<<<nb, kThreads, 0, s>>>(n, d, partial);
        k_sum_partials<<<1, 64, 0, s>>>(partial, nb, out);
        MF_HIP(hipGetLastError());
        double h = 0.0;
        MF_HIP(hipMemcpyAsync(&h, out, sizeof(double), hipMemcpyDeviceToHost, s));
        MF_HIP(hipStreamSynchronize(s));
        const double norm = std::sqrt(h);
        if (!std::isfinite(norm)) return set_error(MF_ERR_NONFINITE, "non-finite residual at Newton step %d", k);
        res->res_norm[k] = norm;
        if (k == 0) d0 = norm;
        if (norm <= std::max(opts->rtol * d0, opts->atol)) {
            res->converged = 1;
            return MF_OK;
        }
        if (k == opts->max_steps) break;
        if (mg) {
            mf_fields Fm{};
            Fm.lin_state = state;
            Fm.dirichlet = dirichlet;
            st = mf_mg_update_ex(mg, form, coords, &Fm, bsets, n_bsets, quad, K, stream);
            if (st != MF_OK) return st;
            lo.precond = MF_PRECOND_MG;
            lo.mg = mg;
        }
        mf_pcg_result lr{};
        // forcing term: the relative residual reached so far (at most 0.1), but no tighter
        // than half of what the final test still needs (target / |d_k|), so the last
        // steps do not ask the linear solver for accuracy the Newton test never uses
        const double target = std::max(opts->rtol * d0, opts->atol);
        lo.tol = std::max({opts->lin_tol, std::min(0.1, d0 > 0.0 ? norm / d0 : 0.1),
                           std::min(0.5, 0.5 * target / norm)});
        st = bicgstab_on_pattern(&A, P, d, du, &lo, &lr, stream);
        res->lin_iterations += lr.iterations;
        const bool usable = (st == MF_ERR_NOT_CONVERGED || st == MF_ERR_NONFINITE) &&
                            std::isfinite(lr.true_relres) && lr.true_relres < 1.0;
        if (st != MF_OK && !usable) return st;
        k_state_update<<<nb, kThreads, 0, s>>>(n, P->n_nodes, 4, P->numbering == MF_FIELD_MAJOR ? 1 : 0, du, state);
        MF_HIP(hipGetLastError());
        res->steps = k + 1;
    }
    return set_error(MF_ERR_NOT_CONVERGED, "Newton reached max_steps = %d (|d| %.3e from %.3e)", opts->max_steps,
                     res->res_norm[opts->max_steps], d0);
}

extern "C" mf_status mf_ns_newton_ex(const mf_pattern_t* P, const mf_form* form, const double* coords,
                                     double* state, const uint8_t* dirichlet, const mf_bset* bsets, int32_t n_bsets,
                                     const mf_quadrature* quad, const mf_newton_opts* opts, mf_newton_result* res,
                                     void* stream)
{
    return newton_run(P, form, coords, state, dirichlet, bsets, n_bsets, nullptr, quad, opts, res, stream);
}

extern "C" mf_status mf_ns_newton_mg(const mf_pattern_t* P, const mf_form* form, const double* coords,
                                     double* state, const uint8_t* dirichlet, const mf_bset* bsets, int32_t n_bsets,
                                     const mf_mg_opts* mg, const mf_quadrature* quad, const mf_newton_opts* opts,
                                     mf_newton_result* res, void* stream)
{
    if (!mg) return set_error(MF_ERR_ARG, "multigrid options are NULL");
    return newton_run(P, form, coords, state, dirichlet, bsets, n_bsets, mg, quad, opts, res, stream);
}
