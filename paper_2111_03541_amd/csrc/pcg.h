// Internal interface of the PCG driver (pcg.hip) used by the C ABI and by the learned
// preconditioner.
#pragma once

#include <hip/hip_runtime.h>

#include "mf.h"

namespace mf {

enum PcgPrecond { MF_PRECOND_INTERNAL_NONE = 0 };
constexpr int MF_PRECOND_EXTERNAL = 100;  // z = apply(r) supplied by the caller

// Writes z from r on the stream (no synchronisation).
typedef mf_status (*PcgApply)(void* ctx, const double* r, double* z, hipStream_t s);

struct PcgArgs {
    int64_t n;
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const double* values;
    const double* b;
    double* x;
    double tol;
    int maxit;
    int check_every;
    int use_graph;
    int precond;  // MF_PRECOND_NONE, MF_PRECOND_JACOBI or MF_PRECOND_EXTERNAL
    int stall_iters;  // iterations without progress that trigger a restart (0 = 512)
    PcgApply apply;
    void* apply_ctx;
    int apply_graph_safe;
    // BiCGStab only: the node graph (offsets [n/4 + 1], neighbours) of node-major rows of
    // four fully coupled fields, whose SpMV then reads the columns from it; null otherwise
    const int32_t* node_ptr;
    const int32_t* node_nbr;
    hipStream_t stream;
};

// scratch: null (the workspace is allocated per call), or a device workspace of at
// least pcg_scratch_doubles(n) doubles; with one, the solve allocates nothing, uses the
// CSR SpMV and launches eagerly (no graph)
mf_status run_pcg(const PcgArgs& a, mf_pcg_result* res, double* scratch = nullptr);
int64_t pcg_scratch_doubles(int64_t n);
// run_pcg on the library's fixed device workspace (at most pcg_noalloc_max_rows() rows,
// Jacobi or no preconditioner); allocates nothing
mf_status run_pcg_noalloc(const PcgArgs& a, mf_pcg_result* res);
int64_t pcg_noalloc_max_rows();
// BiCGStab with Jacobi, no or an external preconditioner (precond MF_PRECOND_JACOBI,
// MF_PRECOND_NONE or MF_PRECOND_EXTERNAL)
mf_status run_bicgstab(const PcgArgs& a, mf_pcg_result* res);
mf_status run_spmv(const mf_csr* A, const double* x, double* y, hipStream_t s);

}  // namespace mf
