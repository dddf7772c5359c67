// Transient thermal conduction, C dT/dt - div(k grad T) = s (the domain form of Sec. 4.1
// with its capacity term), stepped by the generalized-alpha scheme of Sec. 2.1 (dynamic
// extension of the Newton-Raphson update): per step the increments are linked by
//   dT = dt (u0 + b1 du),  T~ = T0 + c1 dT,  u~ = u0 + c2 du   (u = dT/dt),
// and the residual R(T~, u~) = M u~ + K T~ - F is driven to zero with the effective
// tangent c1 K + c2 / (b1 dt) M.  The problem is linear, so one solve per step:
//   (c1 K + c2/(b1 dt) M) dT = F - K T0 - (1 - c2/b1) M u0,
//   T1 = T0 + dT,  u1 = u0 + (dT/dt - u0) / b1.
// Parameters from the spectral radius at infinity rho (first-order systems):
//   c2 = alpha_m = (3 - rho) / (2 (1 + rho)),  c1 = alpha_f = 1 / (1 + rho),
//   b1 = gamma = 1/2 + alpha_m - alpha_f  (second order, unconditionally stable).
// M and K are assembled once (FP64, the library's mass and conduction forms); each step
// is two SpMVs, one combine-and-eliminate pass and a PCG solve, with Jacobi or (the _mg
// entry point) a multigrid cycle built once for the effective matrix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "mf_internal.h"
#include "pcg.h"

namespace mf {
namespace {

constexpr int kThreads = 256;
constexpr int kBlocks = 2048;

int blocks_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(kBlocks, (n + kThreads - 1) / kThreads)); }

// A = a K + b M (same pattern); Dirichlet rows become unit rows and their columns zero
__global__ void __launch_bounds__(kThreads) k_combine(int64_t n, const int32_t* __restrict__ rp,
                                                      const int32_t* __restrict__ ci, const double* __restrict__ K,
                                                      const double* __restrict__ M, double a, double b,
                                                      const uint8_t* __restrict__ mask, double* __restrict__ A)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const bool fixed = mask && mask[r];
        for (int64_t k = rp[r]; k < rp[r + 1]; ++k) {
            const int64_t c = ci[k];
            double v = fma(a, K[k], b * M[k]);
            if (mask) {
                if (fixed) v = (c == r) ? 1.0 : 0.0;
                else if (mask[c]) v = 0.0;
            }
            A[k] = v;
        }
    }
}

// rhs = F - KT - beta Mu (0 on fixed rows)
__global__ void __launch_bounds__(kThreads) k_rhs(int64_t n, const double* __restrict__ F,
                                                  const double* __restrict__ KT, const double* __restrict__ Mu,
                                                  double beta, const uint8_t* __restrict__ mask, double* __restrict__ rhs)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        rhs[i] = (mask && mask[i]) ? 0.0 : F[i] - KT[i] - beta * Mu[i];
}

// T += dT;  u = u + (dT / dt - u) / b1
__global__ void __launch_bounds__(kThreads) k_advance(int64_t n, const double* __restrict__ dT, double dt, double b1,
                                                      double* __restrict__ T, double* __restrict__ u)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double d = dT[i];
        T[i] += d;
        u[i] += (d / dt - u[i]) / b1;
    }
}

// u = x (the consistent initial rate), 0 on fixed rows
__global__ void __launch_bounds__(kThreads) k_copy_masked(int64_t n, const double* __restrict__ x,
                                                          const uint8_t* __restrict__ mask, double* __restrict__ u)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        u[i] = (mask && mask[i]) ? 0.0 : x[i];
}

}  // namespace
}  // namespace mf

using namespace mf;

// The driver behind mf_heat_transient and mf_heat_transient_mg: with mgo, the solves of
// the steps are preconditioned by a multigrid cycle built once for the effective matrix.
static mf_status transient_run(const mf_pattern_t* P, double capacity, double conductivity, const double* coords,
                               const double* elem_k, const double* source, const uint8_t* dirichlet,
                               const mf_mg_opts* mgo, const mf_quadrature* quad, const mf_transient_opts* opts,
                               double* T, double* Tdot, mf_transient_result* res, void* stream)
{
    if (!P || !quad || !opts || !res) return set_error(MF_ERR_ARG, "NULL pattern, quadrature, opts or res");
    if (P->nf != 1) return set_error(MF_ERR_ARG, "transient conduction needs a scalar pattern (1 field)");
    if (!(opts->dt > 0.0) || !(opts->rho_inf >= 0.0 && opts->rho_inf <= 1.0) || opts->n_steps < 0 ||
        !(opts->lin_tol > 0.0) || opts->lin_maxit < 0 || !(capacity > 0.0) || !(conductivity > 0.0))
        return set_error(MF_ERR_ARG, "need dt > 0, rho_inf in [0, 1], n_steps >= 0, lin_tol > 0, C > 0, k > 0");
    const int64_t n = P->n_rows, nnz = P->nnz;
    res->steps = 0;
    res->lin_iterations = 0;
    res->max_lin_relres = 0.0;
    if (n == 0) return MF_OK;
    if (!T || !Tdot || !coords) return set_error(MF_ERR_ARG, "T, Tdot or coords is NULL");
    hipStream_t s = (hipStream_t)stream;

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
    double* K = (double*)dalloc(sizeof(double) * nnz);
    double* M = (double*)dalloc(sizeof(double) * nnz);
    double* A = (double*)dalloc(sizeof(double) * nnz);
    double* F = (double*)dalloc(sizeof(double) * n);
    double* w1 = (double*)dalloc(sizeof(double) * n);
    double* w2 = (double*)dalloc(sizeof(double) * n);
    double* rhs = (double*)dalloc(sizeof(double) * n);
    double* dT = (double*)dalloc(sizeof(double) * n);
    if (!K || !M || !A || !F || !w1 || !w2 || !rhs || !dT) return set_error(MF_ERR_OOM, "transient workspace");

    // K and F = int N_a s (conduction form, nodal source), M (mass form with coefficient C)
    mf_form fk{};
    fk.kind = MF_FORM_POISSON;
    fk.coef = conductivity;
    mf_fields ff{};
    ff.elem_param = elem_k;
    ff.nodal_src = source;
    mf_status st = mf_assemble(P, &fk, coords, &ff, quad, MF_F64, K, F, stream);
    if (st != MF_OK) return st;
    mf_form fm{};
    fm.kind = MF_FORM_MASS;
    fm.coef = capacity;
    mf_fields fmf{};
    st = mf_assemble(P, &fm, coords, &fmf, quad, MF_F64, M, w1, stream);
    if (st != MF_OK) return st;

    const double rho = opts->rho_inf;
    const double am = (3.0 - rho) / (2.0 * (1.0 + rho)), af = 1.0 / (1.0 + rho), g = 0.5 + am - af;
    const double dt = opts->dt;
    mf_csr Kc{n, P->row_ptr, P->col_idx, K};
    mf_csr Mc{n, P->row_ptr, P->col_idx, M};
    mf_csr Ac{n, P->row_ptr, P->col_idx, A};
    mf_pcg_opts po{};
    po.tol = opts->lin_tol;
    po.maxit = opts->lin_maxit;
    po.check_every = 8;
    po.use_graph = stream != nullptr;
    po.precond = MF_PRECOND_JACOBI;
    const int nb = blocks_for(n);

    auto solve = [&](const mf_csr* Amat, const double* b, double* x) -> mf_status {
        mf_pcg_result pr{};
        mf_status r = mf_pcg(Amat, b, x, &po, &pr, stream);
        res->lin_iterations += pr.iterations;
        res->max_lin_relres = std::max(res->max_lin_relres, pr.true_relres);
        return r;
    };

    if (opts->init_rate) {
        // M u0 = F - K T0 on the free rows, u0 = 0 on fixed rows
        k_combine<<<nb, kThreads, 0, s>>>(n, P->row_ptr, P->col_idx, K, M, 0.0, 1.0, dirichlet, A);
        st = run_spmv(&Kc, T, w1, s);
        if (st != MF_OK) return st;
        k_rhs<<<nb, kThreads, 0, s>>>(n, F, w1, w1, 0.0, dirichlet, rhs);
        MF_HIP(hipGetLastError());
        st = solve(&Ac, rhs, dT);
        if (st != MF_OK) return st;
        k_copy_masked<<<nb, kThreads, 0, s>>>(n, dT, dirichlet, Tdot);
        MF_HIP(hipGetLastError());
    }
    if (opts->n_steps == 0) return MF_OK;
    k_combine<<<nb, kThreads, 0, s>>>(n, P->row_ptr, P->col_idx, K, M, af, am / (g * dt), dirichlet, A);
    MF_HIP(hipGetLastError());
    mf_mg_t* mg = nullptr;
    struct MgFree {
        mf_mg_t** m;
        ~MgFree() { mf_mg_destroy(*m); }
    } mgf{&mg};
    if (mgo) {
        // the effective matrix af K + am/(g dt) M on every level
        st = mf_mg_create(P, mgo, stream, &mg);
        if (st != MF_OK) return st;
        st = mg_update_combined(mg, &fk, elem_k, af, &fm, am / (g * dt), coords, dirichlet, quad, A, s);
        if (st != MF_OK) return st;
        po.precond = MF_PRECOND_MG;
        po.mg = mg;
        po.check_every = 4;
    }
    const double beta = 1.0 - am / g;
    for (int k = 0; k < opts->n_steps; ++k) {
        st = run_spmv(&Kc, T, w1, s);
        if (st != MF_OK) return st;
        st = run_spmv(&Mc, Tdot, w2, s);
        if (st != MF_OK) return st;
        k_rhs<<<nb, kThreads, 0, s>>>(n, F, w1, w2, beta, dirichlet, rhs);
        MF_HIP(hipGetLastError());
        st = solve(&Ac, rhs, dT);
        if (st != MF_OK) return st;
        k_advance<<<nb, kThreads, 0, s>>>(n, dT, dt, g, T, Tdot);
        MF_HIP(hipGetLastError());
        res->steps = k + 1;
    }
    return MF_OK;
}

extern "C" mf_status mf_heat_transient(const mf_pattern_t* P, double capacity, double conductivity,
                                       const double* coords, const double* elem_k, const double* source,
                                       const uint8_t* dirichlet, const mf_quadrature* quad,
                                       const mf_transient_opts* opts, double* T, double* Tdot,
                                       mf_transient_result* res, void* stream)
{
    return transient_run(P, capacity, conductivity, coords, elem_k, source, dirichlet, nullptr, quad, opts, T, Tdot,
                         res, stream);
}

extern "C" mf_status mf_heat_transient_mg(const mf_pattern_t* P, double capacity, double conductivity,
                                          const double* coords, const double* elem_k, const double* source,
                                          const uint8_t* dirichlet, const mf_mg_opts* mg, const mf_quadrature* quad,
                                          const mf_transient_opts* opts, double* T, double* Tdot,
                                          mf_transient_result* res, void* stream)
{
    if (!mg) return set_error(MF_ERR_ARG, "multigrid options are NULL");
    return transient_run(P, capacity, conductivity, coords, elem_k, source, dirichlet, mg, quad, opts, T, Tdot, res,
                         stream);
}
