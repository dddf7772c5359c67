// Internal declarations shared by the host API and the HIP kernels of libmf.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mf.h"

// Library-owned state of one pattern (Sec. 2.2 Block B).
struct mf_pattern_s {
    int dim = 0, nen = 0, nf = 0;
    int order = 1;  // element order: 2 for the serendipity elements
    mf_numbering numbering = MF_NODE_MAJOR;
    int64_t n_nodes = 0, n_elems = 0, n_rows = 0, nnz = 0, n_pairs = 0;
    uint8_t coupling[16] = {0};
    bool full_coupling = false;
    // device arrays, all owned
    int32_t* conn = nullptr;     // [nen][n_elems] copy of the caller's connectivity
    int32_t* nbr_ptr = nullptr;  // [n_nodes+1] node graph offsets
    int32_t* nbr = nullptr;      // [n_pairs] sorted neighbours N(v)
    int32_t* row_ptr = nullptr;  // [n_rows+1]
    int32_t* col_idx = nullptr;  // [nnz]
    uint8_t* rank = nullptr;     // [nen*nen][n_elems]
    unsigned long long* status = nullptr;  // [3] first element with det J <= 0, first bad face, first element
                                           // with a non-finite input or coefficient (each ~0 when none)
    // element colouring (no two elements of one colour share a node), made on first use:
    // the elements of colour c are color_elems[color_ptr[c] .. color_ptr[c+1])
    int32_t* color_elems = nullptr;  // device [n_elems]
    int32_t* elem_color = nullptr;   // device [n_elems]: colour of each element
    std::vector<int64_t> color_ptr;
    // boundary-face buckets (boundary.hip): device workspace, grown on demand
    int32_t* face_work = nullptr;
    int64_t face_work_cap = 0;
    // 8-node hexahedra faces per element (boundary.hip): mask [n_elems], counts [6][n_elems]
    uint32_t* face_elem_work = nullptr;
    // structured lexicographic grid detection
    int is_grid = 0;
    int64_t gx = 0, gy = 0, gz = 0;
    hipStream_t last_stream = nullptr;
};

namespace mf {

mf_status set_error(mf_status s, const char* fmt, ...);
mf_status hip_error(hipError_t e, const char* what);
void clear_error();  // empties the thread's last-error message

#define MF_HIP(call)                                            \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return ::mf::hip_error(e_, #call); \
    } while (0)

// pattern.hip
mf_status build_pattern(mf_pattern_s* P, const int32_t* conn_in, hipStream_t s);
// greedy element colouring, cached in the pattern (sync on first call)
mf_status ensure_coloring(const mf_pattern_s* P, hipStream_t s);

struct PcgArgs;
// mf_bicgstab; with P (the pattern whose CSR structure A uses) the SpMV of node-major
// 4-field rows reads its columns from P's node graph
mf_status bicgstab_on_pattern(const mf_csr* A, const mf_pattern_s* P, const double* b, double* x,
                              const mf_pcg_opts* opts, mf_pcg_result* res, void* stream);
mf_status nn_bind_pcg(const mf_nn_t* net, int64_t n_rows, PcgArgs* a);
// multigrid.hip: one V-cycle as the external preconditioner of a solve on `values`
mf_status mg_bind_pcg(const mf_mg_t* mg, int64_t n_rows, const double* values, PcgArgs* a);
// the cycle for A = wa Ka + wb Kb (scalar forms; fa with elem_param) with the Dirichlet
// elimination on every level, A0 the level-0 operator (sync)
mf_status mg_update_combined(mf_mg_t* mg, const mf_form* fa, const double* elem_param, double wa,
                             const mf_form* fb, double wb, const double* coords, const uint8_t* dirichlet,
                             const mf_quadrature* quad, const double* A0, hipStream_t s);

// assemble.hip
struct AssembleArgs {
    const mf_pattern_s* P;
    const mf_form* form;
    const double* coords;
    const void* elem_param;
    const void* nodal_src;
    const void* lin_state;
    const uint8_t* dirichlet;
    mf_precision prec;
    void* K;
    void* d;
    hipStream_t stream;
};
// element-parallel scatter: hardware atomics, or colour by colour with plain adds
// (deterministic sums)
mf_status assemble_atomic(const AssembleArgs& a, bool coloured);
// small 2D meshes (at most 16 colours of at most 16k rows each): status reset, clear,
// coloured scatter and Dirichlet elimination in one single-workgroup launch; the same sums
// as assemble_atomic(a, true) + apply_dirichlet.  MF_ERR_UNSUPPORTED (nothing launched,
// no error recorded) for any other mesh.
mf_status assemble_small(const AssembleArgs& a);
mf_status assemble_quadratic(const AssembleArgs& a);  // assemble_quadratic.hip: MF_HEX20, MF_QUAD8
mf_status assemble_column(const AssembleArgs& a);
mf_status apply_dirichlet(const AssembleArgs& a);
mf_status reset_status(const mf_pattern_s* P, hipStream_t s);

// batched persistent launch (assemble_column.hip)
mf_status batch_check(const AssembleArgs& a);
// chunks[k]: problem k's columns are cut into that many work items along z (the tile
// height); xw[k]: their cross-section, 4 (4x2 nodes) or 2 (2x4); *dev_probs and
// *dev_status are allocated on the first call, reused after
mf_status batch_upload(const std::vector<AssembleArgs>& probs, const std::vector<int>& chunks,
                       const std::vector<int>& xw, void** dev_probs, void** dev_status);
int64_t batch_units_of(const mf_pattern_s* P, int chunks, int xw);
// items [0, n_first) belong to one kernel (elasticity when first_elastic), the rest to the
// other (mass and Poisson); counter holds two ints
mf_status batch_launch(const void* dev_probs, void* dev_status, int n_probs, const int2* items, int n_first,
                       int n_items, bool first_elastic, int* counter, int n_wg, mf_precision prec, bool masked,
                       hipStream_t s);
// workgroups per CU the batched kernel is built for
int batch_max_wg_per_cu(mf_precision prec);

inline unsigned blocks_for(int64_t n, int threads) {
    return (unsigned)((n + threads - 1) / threads);
}

}  // namespace mf
