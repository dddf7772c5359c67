// Host side of the C ABI declared in include/mf.h: argument validation, handle
// lifetime, strategy dispatch and error reporting.  No device arithmetic here.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "mf_internal.h"
#include "pcg.h"

namespace {
thread_local char g_err[512] = "";
}

namespace mf {

mf_status set_error(mf_status s, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

void clear_error() { g_err[0] = 0; }

mf_status hip_error(hipError_t e, const char* what)
{
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return set_error(MF_ERR_OOM, "%s: %s", what, hipGetErrorString(e));
    return set_error(MF_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace mf

using namespace mf;

static void free_pattern(mf_pattern_s* P)
{
    if (!P) return;
    (void)hipFree(P->conn);
    (void)hipFree(P->nbr_ptr);
    (void)hipFree(P->nbr);
    (void)hipFree(P->row_ptr);
    (void)hipFree(P->col_idx);
    (void)hipFree(P->rank);
    (void)hipFree(P->status);
    (void)hipFree(P->color_elems);
    (void)hipFree(P->elem_color);
    (void)hipFree(P->face_work);
    (void)hipFree(P->face_elem_work);
    delete P;
}

extern "C" {

const char* mf_last_error(void) { return g_err; }

// The assembly kernel revision is part of the string so that measurements taken on one
// revision (for example HBM byte counters) can be matched to it.
const char* mf_version(void) { return "metafem-mi 0.2 (gfx950; assembly column-4x2 r10; flow mfma-4x4 r3)"; }

mf_status mf_pattern(const mf_mesh* mesh, mf_elem_type type, int32_t order, const mf_dofs* dofs,
                     void* stream, mf_pattern_t** out)
{
    g_err[0] = 0;
    if (!out) return set_error(MF_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!mesh || !dofs) return set_error(MF_ERR_ARG, "mesh or dofs is NULL");
    if (type != MF_QUAD4 && type != MF_HEX8 && type != MF_HEX20 && type != MF_QUAD8 && type != MF_TET10)
        return set_error(MF_ERR_UNSUPPORTED, "element type %d", (int)type);
    const int elem_order = (type == MF_HEX20 || type == MF_QUAD8 || type == MF_TET10) ? 2 : 1;
    if (order != elem_order)
        return set_error(MF_ERR_UNSUPPORTED, "element order %d for element type %d", (int)order, (int)type);
    const int dim = (type == MF_QUAD4 || type == MF_QUAD8) ? 2 : 3;
    if (mesh->dim != dim) return set_error(MF_ERR_ARG, "mesh dim %d does not match the element", (int)mesh->dim);
    if (mesh->n_nodes < 0 || mesh->n_elems < 0) return set_error(MF_ERR_ARG, "negative mesh size");
    if (mesh->n_elems > 0 && !mesh->conn) return set_error(MF_ERR_ARG, "conn is NULL");
    if (dofs->n_fields < 1 || dofs->n_fields > 4) return set_error(MF_ERR_ARG, "n_fields %d not in 1..4", (int)dofs->n_fields);
    if (dofs->numbering != MF_NODE_MAJOR && dofs->numbering != MF_FIELD_MAJOR)
        return set_error(MF_ERR_ARG, "unknown numbering %d", (int)dofs->numbering);
    const int nen = type == MF_HEX20 ? 20 : type == MF_QUAD8 ? 8 : type == MF_TET10 ? 10 : 1 << dim;
    if ((int64_t)nen * nen * mesh->n_elems >= ((int64_t)1 << 31) || mesh->n_nodes * dofs->n_fields >= ((int64_t)1 << 31))
        return set_error(MF_ERR_OVERFLOW, "mesh too large for int32 indices");

    mf_pattern_s* P = new (std::nothrow) mf_pattern_s();
    if (!P) return set_error(MF_ERR_OOM, "host allocation failed");
    P->dim = dim;
    P->nen = nen;
    P->order = elem_order;
    P->nf = dofs->n_fields;
    P->numbering = dofs->numbering;
    P->n_nodes = mesh->n_nodes;
    P->n_elems = mesh->n_elems;
    P->n_rows = mesh->n_nodes * dofs->n_fields;
    bool full = true;
    for (int k = 0; k < P->nf * P->nf; ++k) {
        P->coupling[k] = dofs->coupling ? (dofs->coupling[k] ? 1 : 0) : 1;
        full = full && P->coupling[k];
    }
    for (int i = 0; i < P->nf; ++i) {
        bool any = false;
        for (int j = 0; j < P->nf; ++j) any = any || P->coupling[i * P->nf + j];
        if (!any) {
            delete P;
            return set_error(MF_ERR_ARG, "coupling row %d is empty", i);
        }
    }
    P->full_coupling = full;
    hipStream_t s = (hipStream_t)stream;
    mf_status st = build_pattern(P, mesh->conn, s);
    if (st != MF_OK) {
        (void)hipStreamSynchronize(s);
        free_pattern(P);
        return st;
    }
    st = reset_status(P, s);
    if (st == MF_OK) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_error(e, "hipStreamSynchronize");
    }
    if (st != MF_OK) {
        free_pattern(P);
        return st;
    }
    *out = P;
    return MF_OK;
}

mf_status mf_pattern_info(const mf_pattern_t* P, int64_t* n_rows, int64_t* nnz, const int32_t** row_ptr,
                          const int32_t** col_idx, const uint8_t** rank)
{
    if (!P) return set_error(MF_ERR_ARG, "pattern is NULL");
    if (n_rows) *n_rows = P->n_rows;
    if (nnz) *nnz = P->nnz;
    if (row_ptr) *row_ptr = P->row_ptr;
    if (col_idx) *col_idx = P->col_idx;
    if (rank) *rank = P->rank;
    return MF_OK;
}

mf_status mf_pattern_grid(const mf_pattern_t* P, int32_t* is_grid, int64_t* nx, int64_t* ny, int64_t* nz)
{
    if (!P) return set_error(MF_ERR_ARG, "pattern is NULL");
    if (is_grid) *is_grid = P->is_grid;
    if (nx) *nx = P->gx;
    if (ny) *ny = P->gy;
    if (nz) *nz = P->gz;
    return MF_OK;
}

void mf_pattern_destroy(mf_pattern_t* P)
{
    if (!P) return;
    if (P->last_stream) (void)hipStreamSynchronize(P->last_stream);
    free_pattern(P);
}

mf_status mf_assemble_ex(const mf_pattern_t* P, const mf_form* form, const double* coords,
                         const mf_fields* fields, const mf_quadrature* quad, mf_precision prec,
                         mf_scatter scatter, void* K, void* d, void* stream)
{
    g_err[0] = 0;
    if (!P || !form || !quad) return set_error(MF_ERR_ARG, "pattern, form or quadrature is NULL");
    const int want_q = P->nen == 10 && P->dim == 3 ? 4 : (P->order == 2 ? 3 : 2);
    if (quad->points_per_axis != want_q)
        return set_error(MF_ERR_UNSUPPORTED, "%d Gauss points per axis (this element takes %d)",
                         (int)quad->points_per_axis, want_q);
    if (prec != MF_F64 && prec != MF_F32) return set_error(MF_ERR_ARG, "unknown precision %d", (int)prec);
    int nf_form;
    switch (form->kind) {
        case MF_FORM_MASS:
        case MF_FORM_POISSON: nf_form = 1; break;
        case MF_FORM_ELASTICITY: nf_form = P->dim; break;
        case MF_FORM_NS_SUPG: nf_form = P->dim + 1; break;
        default: return set_error(MF_ERR_ARG, "unknown form kind %d", (int)form->kind);
    }
    if (nf_form != P->nf)
        return set_error(MF_ERR_ARG, "form needs %d fields, pattern has %d", nf_form, P->nf);
    if (!P->full_coupling)
        return set_error(MF_ERR_ARG, "the form couples every field pair; the pattern's coupling is partial");
    if (form->kind == MF_FORM_ELASTICITY && !(form->nu > -1.0 && form->nu < 0.5))
        return set_error(MF_ERR_ARG, "Poisson's ratio %g outside (-1, 0.5)", form->nu);
    if (P->n_elems > 0 && !coords) return set_error(MF_ERR_ARG, "coords is NULL");
    if ((P->nnz > 0 && !K) || (P->n_rows > 0 && !d)) return set_error(MF_ERR_ARG, "K or d is NULL");
    if (scatter != MF_SCATTER_AUTO && scatter != MF_SCATTER_ATOMIC && scatter != MF_SCATTER_GATHER)
        return set_error(MF_ERR_ARG, "unknown scatter strategy %d", (int)scatter);

    AssembleArgs A{};
    A.P = P;
    A.form = form;
    A.coords = coords;
    mf_fields none{};
    const mf_fields* F = fields ? fields : &none;
    A.elem_param = F->elem_param;
    A.nodal_src = F->nodal_src;
    A.lin_state = F->lin_state;
    A.dirichlet = F->dirichlet;
    A.prec = prec;
    A.K = K;
    A.d = d;
    A.stream = (hipStream_t)stream;
    const_cast<mf_pattern_s*>(P)->last_stream = A.stream;

    mf_status st;
    if (scatter == MF_SCATTER_AUTO && P->dim == 2 && P->order == 1) {
        // small 2D meshes: the whole call as one launch
        st = assemble_small(A);
        if (st != MF_ERR_UNSUPPORTED) return st;
    }
    st = reset_status(P, A.stream);
    if (st != MF_OK) return st;
    if (P->order == 2) {  // quadratic elements: colour by colour, one workgroup per element
        st = assemble_quadratic(A);
        if (st != MF_OK) return st;
        return apply_dirichlet(A);
    }
    // AUTO: the owner-computes gather on structured grids, else (and for forms without a
    // gather kernel) the element-parallel scatter colour by colour, whose sums do not
    // depend on the run; ATOMIC asks for the paper's atomic scatter explicitly.
    const bool auto_mode = scatter == MF_SCATTER_AUTO;
    if (auto_mode) scatter = P->is_grid ? MF_SCATTER_GATHER : MF_SCATTER_ATOMIC;
    // the coloured scatter: the flow form on 8-node bricks runs one workgroup per element
    // (geometry once per element), the other forms one thread per (element, row)
    auto coloured = [&]() -> mf_status {
        if (form->kind == MF_FORM_NS_SUPG && P->dim == 3) {
            mf_status s2 = assemble_quadratic(A);
            if (s2 != MF_ERR_UNSUPPORTED) return s2;
        }
        return assemble_atomic(A, true);
    };
    bool gathered = false;
    if (scatter == MF_SCATTER_GATHER) {
        st = assemble_column(A);  // applies the Dirichlet elimination while writing K
        gathered = st == MF_OK;
        if (st == MF_ERR_UNSUPPORTED) st = coloured();  // e.g. a form without a gather kernel
    } else {
        st = auto_mode ? coloured() : assemble_atomic(A, false);
    }
    if (st != MF_OK) return st;
    return gathered ? MF_OK : apply_dirichlet(A);
}

mf_status mf_assemble(const mf_pattern_t* P, const mf_form* form, const double* coords, const mf_fields* fields,
                      const mf_quadrature* quad, mf_precision prec, void* K, void* d, void* stream)
{
    return mf_assemble_ex(P, form, coords, fields, quad, prec, MF_SCATTER_AUTO, K, d, stream);
}

mf_status mf_status_poll(const mf_pattern_t* P, int64_t* first_bad_elem)
{
    if (!P) return set_error(MF_ERR_ARG, "pattern is NULL");
    unsigned long long v[3] = {0, 0, 0};
    if (P->last_stream) MF_HIP(hipStreamSynchronize(P->last_stream));
    MF_HIP(hipMemcpy(v, P->status, sizeof(v), hipMemcpyDeviceToHost));
    if (first_bad_elem) *first_bad_elem = v[0] != ~0ull ? (int64_t)v[0] : v[2] != ~0ull ? (int64_t)v[2] : -1;
    if (v[1] != ~0ull)
        return set_error(MF_ERR_ARG, "boundary face %lld: element id or local face out of range (skipped)",
                         (long long)v[1]);
    if (v[0] != ~0ull) return set_error(MF_ERR_BAD_JACOBIAN, "det J <= 0 in element %lld", (long long)v[0]);
    if (v[2] != ~0ull)
        return set_error(MF_ERR_NONFINITE, "non-finite input or coefficient in element %lld", (long long)v[2]);
    return MF_OK;
}

// Validates the arguments of mf_pcg / mf_pcg_noalloc and fills the solver arguments.
static mf_status pcg_args(const mf_csr* A, const double* b, double* x, const mf_pcg_opts* opts,
                          mf_pcg_result* res, void* stream, PcgArgs* a)
{
    if (!A || !opts || !res) return set_error(MF_ERR_ARG, "A, opts or res is NULL");
    if (A->n_rows < 0 || A->n_rows >= ((int64_t)1 << 31)) return set_error(MF_ERR_ARG, "n_rows out of range");
    if (A->n_rows > 0 && (!A->row_ptr || !A->col_idx || !A->values || !b || !x))
        return set_error(MF_ERR_ARG, "NULL matrix or vector");
    if (!(opts->tol > 0.0) || opts->maxit < 0) return set_error(MF_ERR_ARG, "tol must be > 0 and maxit >= 0");
    *a = PcgArgs{};
    a->n = A->n_rows;
    a->row_ptr = A->row_ptr;
    a->col_idx = A->col_idx;
    a->values = A->values;
    a->b = b;
    a->x = x;
    a->tol = opts->tol;
    a->maxit = opts->maxit;
    a->check_every = opts->check_every;
    a->use_graph = opts->use_graph && stream != nullptr;
    a->stream = (hipStream_t)stream;
    if (opts->stall_iters < 0) return set_error(MF_ERR_ARG, "stall_iters must be >= 0");
    a->stall_iters = opts->stall_iters;
    switch (opts->precond) {
        case MF_PRECOND_NONE: a->precond = MF_PRECOND_NONE; break;
        case MF_PRECOND_JACOBI: a->precond = MF_PRECOND_JACOBI; break;
        case MF_PRECOND_NN: {
            if (!opts->net) return set_error(MF_ERR_ARG, "MF_PRECOND_NN needs a network");
            return nn_bind_pcg(opts->net, A->n_rows, a);
        }
        case MF_PRECOND_MG: {
            if (!opts->mg) return set_error(MF_ERR_ARG, "MF_PRECOND_MG needs a multigrid cycle");
            return mg_bind_pcg(opts->mg, A->n_rows, A->values, a);
        }
        default: return set_error(MF_ERR_ARG, "unknown preconditioner %d", (int)opts->precond);
    }
    return MF_OK;
}

mf_status mf_pcg(const mf_csr* A, const double* b, double* x, const mf_pcg_opts* opts, mf_pcg_result* res,
                 void* stream)
{
    g_err[0] = 0;
    PcgArgs a;
    mf_status st = pcg_args(A, b, x, opts, res, stream, &a);
    if (st != MF_OK) return st;
    return run_pcg(a, res);
}

mf_status mf_pcg_noalloc(const mf_csr* A, const double* b, double* x, const mf_pcg_opts* opts,
                         mf_pcg_result* res, void* stream)
{
    g_err[0] = 0;
    if (opts && (opts->precond == MF_PRECOND_NN || opts->precond == MF_PRECOND_MG))
        return set_error(MF_ERR_UNSUPPORTED, "mf_pcg_noalloc takes MF_PRECOND_NONE or MF_PRECOND_JACOBI");
    PcgArgs a;
    mf_status st = pcg_args(A, b, x, opts, res, stream, &a);
    if (st != MF_OK) return st;
    return run_pcg_noalloc(a, res);
}

int64_t mf_pcg_noalloc_max_rows(void) { return pcg_noalloc_max_rows(); }

mf_status mf_bicgstab(const mf_csr* A, const double* b, double* x, const mf_pcg_opts* opts, mf_pcg_result* res,
                      void* stream)
{
    return bicgstab_on_pattern(A, nullptr, b, x, opts, res, stream);
}

mf_status mf_spmv(const mf_csr* A, const double* x, double* y, void* stream)
{
    if (!A) return set_error(MF_ERR_ARG, "A is NULL");
    if (A->n_rows > 0 && (!A->row_ptr || !A->col_idx || !A->values || !x || !y))
        return set_error(MF_ERR_ARG, "NULL matrix or vector");
    return run_spmv(A, x, y, (hipStream_t)stream);
}

}  // extern "C"

mf_status mf::bicgstab_on_pattern(const mf_csr* A, const mf_pattern_s* P, const double* b, double* x,
                                  const mf_pcg_opts* opts, mf_pcg_result* res, void* stream)
{
    g_err[0] = 0;
    if (!A || !opts || !res) return set_error(MF_ERR_ARG, "A, opts or res is NULL");
    if (A->n_rows < 0 || A->n_rows >= ((int64_t)1 << 31)) return set_error(MF_ERR_ARG, "n_rows out of range");
    if (A->n_rows > 0 && (!A->row_ptr || !A->col_idx || !A->values || !b || !x))
        return set_error(MF_ERR_ARG, "NULL matrix or vector");
    if (!(opts->tol > 0.0) || opts->maxit < 0) return set_error(MF_ERR_ARG, "tol must be > 0 and maxit >= 0");
    if (opts->precond != MF_PRECOND_NONE && opts->precond != MF_PRECOND_JACOBI && opts->precond != MF_PRECOND_MG)
        return set_error(MF_ERR_ARG, "BiCGStab takes MF_PRECOND_NONE, MF_PRECOND_JACOBI or MF_PRECOND_MG, not %d",
                         (int)opts->precond);
    PcgArgs a{};
    a.n = A->n_rows;
    a.row_ptr = A->row_ptr;
    a.col_idx = A->col_idx;
    a.values = A->values;
    a.b = b;
    a.x = x;
    a.tol = opts->tol;
    a.maxit = opts->maxit;
    a.check_every = opts->check_every;
    a.use_graph = opts->use_graph && stream != nullptr;
    a.stream = (hipStream_t)stream;
    a.precond = opts->precond;
    // A on P's CSR structure with node-major rows of four fully coupled fields (16 entries
    // per node pair): the SpMV reads the columns from the node graph
    if (P && A->row_ptr == P->row_ptr && A->col_idx == P->col_idx && A->n_rows == P->n_rows && P->nf == 4 &&
        P->numbering == MF_NODE_MAJOR && P->nnz == 16 * P->n_pairs) {
        a.node_ptr = P->nbr_ptr;
        a.node_nbr = P->nbr;
    }
    if (opts->precond == MF_PRECOND_MG) {
        if (!opts->mg) return set_error(MF_ERR_ARG, "MF_PRECOND_MG needs a multigrid cycle");
        mf_status st = mg_bind_pcg(opts->mg, A->n_rows, A->values, &a);
        if (st != MF_OK) return st;
    }
    return run_bicgstab(a, res);
}
