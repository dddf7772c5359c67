/*
 * mf.h - C ABI of the MI355X finite-element assembly library (libmf.so).
 *
 * The library assembles the sparse linear system K x = d of a weak form on a mesh of
 * linear (4-node quadrilateral, 8-node hexahedron) or quadratic (8-node quadrilateral,
 * 20-node hexahedron, 10-node tetrahedron) elements (MetaFEM, arXiv 2111.03541).  Sec. 1 of the paper states that K x = d is fixed by
 * six inputs: the weak forms, their linearisation, the element type and order, the
 * quadrature, the time scheme and the numbering of the unknowns.  These become the
 * arguments below.  The time scheme is steady here, so the time coefficient of the
 * stiffness assembly (Sec. 2.2 D-3) is 1.
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers unless marked (host).
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   - Calls are asynchronous on `stream` unless marked (sync).
 *   - Every call returns an mf_status.  A message for the last failure on the
 *     calling thread is available from mf_last_error().
 *   - Nothing throws across the ABI.  A handle must not be used from two host
 *     threads at once.
 *   - The caller owns every array it passes: conn, coords, fields, K values, d and
 *     vectors.  The library owns the arrays of a pattern handle.  Views returned by
 *     mf_pattern_info stay valid until mf_pattern_destroy.
 *   - Structure-of-arrays layouts:
 *       conn    [nen][n_elems] int32, with the local node order of the reference
 *               element, a = ax + 2 ay + 4 az
 *       coords  [dim][n_nodes] FP64
 *       fields  [n_fields][n_nodes]
 */
#ifndef MF_H
#define MF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MF_OK = 0,
    MF_ERR_ARG = 1,           /* invalid argument (message says which)                  */
    MF_ERR_UNSUPPORTED = 2,   /* valid but not implemented (element, order, quadrature) */
    MF_ERR_OVERFLOW = 3,      /* an index exceeds its type: nnz >= 2^31, valence > 255  */
    MF_ERR_HIP = 4,           /* a HIP runtime call failed                              */
    MF_ERR_BAD_JACOBIAN = 5,  /* det J <= 0 at an integration point (mf_status_poll)    */
    MF_ERR_NONFINITE = 6,     /* non-finite value produced                              */
    MF_ERR_NOT_CONVERGED = 7, /* iterative solver hit its iteration limit               */
    MF_ERR_OOM = 8,           /* device allocation failed                               */
    MF_ERR_BAD_MESH = 9       /* connectivity references a node outside [0, n_nodes)    */
} mf_status;

typedef enum {
    MF_QUAD4 = 1,   /* 4-node quadrilateral, order 1                                        */
    MF_HEX8 = 2,    /* 8-node hexahedron, order 1 (corners a = ax + 2 ay + 4 az)             */
    MF_HEX20 = 3,   /* 20-node serendipity hexahedron, order 2: corners as MF_HEX8, then the
                       midpoints of the x-, y- and z-directed edges, four each, ordered by
                       the bits of the two other axes; mass, conduction, elasticity and
                       flow forms with 3 Gauss points per axis (element colours, one
                       workgroup per element)                                                */
    MF_QUAD8 = 4,   /* 8-node serendipity quadrilateral, order 2: corners as MF_QUAD4, then the
                       midpoints of the x-directed edges at y = -1, +1 and of the y-directed
                       edges at x = -1, +1; the forms of MF_HEX20 (plane-strain elasticity)
                       with 3 Gauss points per axis                                          */
    MF_TET10 = 5    /* 10-node quadratic tetrahedron, order 2: vertices 0..3 (positively
                       oriented), then the midpoints of the edges (0,1), (1,2), (2,0), (0,3),
                       (1,3), (2,3); the forms of MF_HEX20 with the 64-point collapsed Gauss
                       rule (points_per_axis = 4)                                            */
} mf_elem_type;
/* DOF numbering.  Field-major is the paper's map (Sec. 2.2 B-3): dof = field*n_nodes + node.
   Node-major interleaves the fields of a node: dof = n_fields*node + field. */
typedef enum { MF_NODE_MAJOR = 0, MF_FIELD_MAJOR = 1 } mf_numbering;
typedef enum {
    MF_FORM_MASS = 0,       /* K_ab = int c N_a N_b,                    d = M f           */
    MF_FORM_POISSON = 1,    /* thermal conduction, Sec. 4.1 (steady): K_ab = int k dN_a.dN_b,
                               d = M f                                                    */
    MF_FORM_ELASTICITY = 2, /* linear elasticity, Sec. 4.2: K = int eps(N_a):sigma(N_b),
                               d = int N_a b (nodal body force b, interpolated)           */
    MF_FORM_NS_SUPG = 3     /* steady incompressible Navier-Stokes with SUPG/PSPG/LSIC,
                               Sec. 4.3: Newton tangent K = dR/dU and d = -R at the state U0 */
} mf_form_kind;
typedef enum { MF_F64 = 0, MF_F32 = 1 } mf_precision;

typedef struct {
    int32_t dim;           /* 2 (MF_QUAD4, MF_QUAD8) or 3 (MF_HEX8, MF_HEX20, MF_TET10) */
    int64_t n_nodes;
    int64_t n_elems;
    const int32_t* conn;   /* [nen][n_elems] (device) */
} mf_mesh;

typedef struct {
    int32_t n_fields;          /* 1..4 */
    const uint8_t* coupling;   /* (host) [n_fields*n_fields], 1 = block (i,j) present; NULL = all */
    mf_numbering numbering;
} mf_dofs;

typedef struct mf_pattern_s mf_pattern_t;   /* opaque, library-owned */

/*
 * mf_pattern - sparsity pattern of K (Sec. 2.2 Block B: B-1 element-to-node map and node
 * pairs, B-3 DOF map, B-4 sparse layout, here CSR instead of COO).
 *   N(v) = sorted set of nodes sharing an element with node v (v included).
 *   Row dof(v,i) holds columns dof(w,j) for w in N(v) and coupling(i,j), ascending.
 *   rank[(a*nen+b)*n_elems + e] = position of conn[b][e] in N(conn[a][e]).
 * order must match the element type: 1 for MF_QUAD4 and MF_HEX8, 2 for MF_QUAD8,
 * MF_HEX20 and MF_TET10 (MF_ERR_UNSUPPORTED otherwise).  Runs on `stream` and
 * synchronises it (sync); allocates the
 * pattern's device arrays.  Errors: MF_ERR_ARG, MF_ERR_BAD_MESH (node id out of
 * range), MF_ERR_OVERFLOW (nnz or nen*n_elems >= 2^31, or more than 255 neighbours of
 * one node), MF_ERR_OOM, MF_ERR_HIP.  *out is NULL on error.
 */
mf_status mf_pattern(const mf_mesh* mesh, mf_elem_type type, int32_t order, const mf_dofs* dofs,
                     void* stream, mf_pattern_t** out);

/* (sync) sizes and device views: row_ptr int32 [n_rows+1], col_idx int32 [nnz],
   rank uint8 [nen*nen][n_elems].  Any output pointer may be NULL. */
mf_status mf_pattern_info(const mf_pattern_t* pat, int64_t* n_rows, int64_t* nnz,
                          const int32_t** row_ptr, const int32_t** col_idx, const uint8_t** rank);

/* (sync) 1 when the connectivity is a structured lexicographic grid (node id
   i + (nx+1)(j + (ny+1)k), element id ex + nx(ey + ny ez)), with its element counts. */
mf_status mf_pattern_grid(const mf_pattern_t* pat, int32_t* is_grid, int64_t* nx, int64_t* ny,
                          int64_t* nz);

void mf_pattern_destroy(mf_pattern_t* pat);

/* Scalar parameters of a form.
   coef: MASS density c, POISSON conductivity k, ELASTICITY Young's modulus E; each is
         multiplied by elem_param[e] when that array is given.
   nu:   ELASTICITY Poisson's ratio (Lame parameters as in Sec. 4.2).
   rho, mu, tau_m, tau_c: NS_SUPG density, dynamic viscosity, stabilisation constants. */
typedef struct {
    mf_form_kind kind;
    double coef, nu, rho, mu, tau_m, tau_c;
} mf_form;

/* Per-mesh inputs; precision-typed arrays are double (MF_F64) or float (MF_F32). */
typedef struct {
    const void* elem_param;   /* [n_elems] or NULL (= 1) */
    const void* nodal_src;    /* MASS/POISSON: f [1][n_nodes]; ELASTICITY: b [dim][n_nodes];
                                 NULL = 0 */
    const void* lin_state;    /* NS_SUPG: U0 [dim+1][n_nodes] = (u_1..u_dim, p); NULL = 0 */
    const uint8_t* dirichlet; /* [n_rows] constrained-DOF mask or NULL; a constrained row
                                 becomes a unit row with d = 0, its column is zeroed
                                 elsewhere (homogeneous elimination, structure kept) */
} mf_fields;

typedef struct { int32_t points_per_axis; } mf_quadrature;   /* Gauss-Legendre: 2 for order 1,
                                                                  3 for MF_HEX20 and MF_QUAD8,
                                                                  4 for MF_TET10 (collapsed) */

/* Assembly strategies.  AUTO picks the owner-computes gather for structured grids, and
   otherwise (or for a form without a gather kernel) the element-parallel scatter colour
   by colour with plain adds, whose sums are the same on every run.  ATOMIC is the
   element-parallel scatter with hardware atomics in one launch (the paper's scheme).  In
   ATOMIC and in the gather (which sums a node's element blocks with LDS atomics) the
   order of the additions, and so the last bits, may vary between runs.  GATHER asks for
   the owner-computes kernel. */
typedef enum { MF_SCATTER_AUTO = 0, MF_SCATTER_ATOMIC = 1, MF_SCATTER_GATHER = 2 } mf_scatter;

/*
 * mf_assemble - fill K (CSR values on the pattern) and d (Sec. 2.2 D-2 residual and
 * D-3 stiffness assembly, Sec. 2.1 numerical integration).
 *   K = dR/dU and d = -R(U0), where R is the weak form with the sign that makes the
 *   diffusion term positive (thermal and elastic forms times -1, the flow form as
 *   written).  Each integration point uses the geometry Jacobian J = sum_a x_a (x)
 *   dN_a/dxi, with det J > 0 required, g_a = J^-T dN_a/dxi and weight w_q det J.
 * precision MF_F64: everything in FP64.  MF_F32: geometry (J, det J, J^-1, g, weights)
 *   in FP64, rounded to FP32; coefficients and the element contractions in FP32 (the
 *   structured-grid path sums the element contributions of a row in FP64 and rounds
 *   once); K, d, elem_param, nodal_src and lin_state are float.  coords are FP64 always.
 * K_values [nnz] and d [n_rows] are overwritten entirely (no prior clear needed).
 * Async on `stream`.  A device-side det J <= 0 is reported by mf_status_poll.
 * The pattern's n_fields must match the form (1, 1, dim, dim+1).
 */
mf_status mf_assemble(const mf_pattern_t* pat, const mf_form* form, const double* coords,
                      const mf_fields* fields, const mf_quadrature* quad, mf_precision precision,
                      void* K_values, void* d, void* stream);

/* Same as mf_assemble with an explicit strategy (for tests and tuning). */
mf_status mf_assemble_ex(const mf_pattern_t* pat, const mf_form* form, const double* coords,
                         const mf_fields* fields, const mf_quadrature* quad, mf_precision precision,
                         mf_scatter scatter, void* K_values, void* d, void* stream);

/* (sync) Reads the device status words of the assemblies on this pattern since the last
   mf_assemble (which clears them): MF_OK; MF_ERR_ARG when mf_assemble_boundary skipped a
   face out of range (the message names the first); else MF_ERR_BAD_JACOBIAN with the
   smallest offending element id in *first_bad_elem. */
mf_status mf_status_poll(const mf_pattern_t* pat, int64_t* first_bad_elem);

/* Thread-local message for the last failing call ("" if none). */
const char* mf_last_error(void);

/* ------------------------------------------------------------------------------------
 * Batched assembly: many independent structured problems (each with its own pattern,
 * the paper's "workpieces", Sec. 2.2 A-1 and B-2) assembled by ONE persistent launch
 * that work-steals (problem, node column) items, replayed as a HIP graph.  Problems must be
 * structured 3D grids (mf_pattern_grid) with MASS, POISSON or ELASTICITY forms.
 * ------------------------------------------------------------------------------------ */
typedef struct mf_batch_s mf_batch_t;

typedef struct {
    const mf_pattern_t* pattern;
    mf_form form;
    const double* coords;     /* [3][n_nodes] FP64 (device) */
    mf_fields fields;         /* lin_state unused */
    void* K;                  /* [nnz] of this problem (device, precision-typed) */
    void* d;                  /* [n_rows] (device) */
} mf_batch_problem;

/* (sync) Copies the problem descriptors to the device; the arrays they point to must
   stay valid while the batch is used.  Default launch (before mf_batch_tune): round-
   robin items, whole columns, one workgroup per CU. */
mf_status mf_batch_create(const mf_batch_problem* problems /* (host) [n] */, int32_t n,
                          mf_precision precision, mf_batch_t** out);

/* (sync) Autotuner, timing candidates on the batch itself.  First the tile shape per class
   of problems, a class being (form: mass/Poisson or elasticity) x (size bucket of the
   column height NZ = nz + 1: <= 20, <= 34, larger): a tile is a 4x2 or 2x4 node column cut
   along z into 1..4 chunks, and the shape of each class is chosen by coordinate descent.
   Then the launch shape for those tiles (work-item order within each kernel: problem-
   major or round-robin, elasticity kernel first; or round-robin with the mass/Poisson
   kernel first; workgroups per CU: 1, 2 in FP64, 1..3 in FP32).  cache_path (host
   string, may be NULL) is a text file of tuned choices keyed by device, precision,
   Dirichlet flags, problems per class and column count: a hit skips timing. */
mf_status mf_batch_tune(mf_batch_t* batch, const char* cache_path, void* stream);

/* (sync) Tile shapes: *n_classes (6) classes ordered (form: 0 mass/Poisson, 1 elasticity)
   x (size bucket 0..2); problems[c] (host, may be NULL) the number of problems in class c;
   chunks[c] (host, may be NULL) the chunks per column (tile height NZ / chunks);
   cross_x[c] (host, may be NULL) the column cross-section's width along x in nodes: 4 for
   4x2 columns, 2 for 2x4. */
mf_status mf_batch_tiles(const mf_batch_t* batch, int32_t* n_classes, int32_t* problems, int32_t* chunks,
                         int32_t* cross_x);

/* Assembles every problem (K and d overwritten; device status words of all patterns reset
   first): two persistent launches, one for the elasticity problems and one for the mass
   and Poisson problems (each built for its own forms' registers).  On a non-default stream
   the launches are captured once as a HIP graph and replayed on later calls.  Async. */
mf_status mf_batch_run(mf_batch_t* batch, void* stream);

/* (sync) Work items, workgroups, item order, whether a graph exists, tuned time (us). */
mf_status mf_batch_info(const mf_batch_t* batch, int64_t* n_items, int32_t* n_workgroups, int32_t* order,
                        int32_t* graphed, double* tuned_us);

void mf_batch_destroy(mf_batch_t* batch);

/* ------------------------------------------------------------------------------------
 * Transient thermal conduction (the domain form of Sec. 4.1 with its capacity term,
 * C dT/dt - div(k grad T) = s) stepped by the generalized-alpha scheme of Sec. 2.1 (its
 * dynamic extension of the Newton-Raphson update).  With u = dT/dt, each step links the
 * increments by dT = dt (u0 + b1 du), evaluates the residual at T~ = T0 + c1 dT and
 * u~ = u0 + c2 du, and solves the linear effective system
 *   (c1 K + c2 / (b1 dt) M) dT = F - K T0 - (1 - c2 / b1) M u0,
 * then T1 = T0 + dT, u1 = u0 + (dT / dt - u0) / b1.  The parameters follow from the
 * spectral radius at infinity rho: c2 = (3 - rho) / (2 (1 + rho)), c1 = 1 / (1 + rho),
 * b1 = 1/2 + c2 - c1 (second order, unconditionally stable).
 * ------------------------------------------------------------------------------------ */
typedef struct {
    double dt;              /* time step                                                    */
    double rho_inf;         /* spectral radius at infinity, in [0, 1]                        */
    int32_t n_steps;        /* steps to take (0: only the optional initial rate)             */
    int32_t init_rate;      /* 1: first set Tdot from M Tdot = F - K T (0 on fixed rows)      */
    double lin_tol;         /* relative true-residual tolerance of each PCG solve             */
    int32_t lin_maxit;
} mf_transient_opts;

typedef struct {
    int32_t steps;          /* steps taken                                                  */
    int32_t lin_iterations; /* PCG iterations over all solves                               */
    double max_lin_relres;  /* largest true relative residual of the solves                 */
} mf_transient_result;

/*
 * mf_heat_transient - P is a scalar pattern (1 field, 2D or 3D).  K_ab = int k_e grad N_a .
 * grad N_b with k_e = conductivity * elem_k[e] (elem_k [n_elems] device FP64, or NULL = 1),
 * M_ab = int capacity N_a N_b, F_a = int N_a s with s the nodal source [n_nodes] (device
 * FP64, or NULL = 0).  T and Tdot [n_nodes] (device FP64) hold the state at the start and
 * are overwritten with the state after n_steps.  dirichlet [n_rows] (device, or NULL)
 * keeps T fixed on marked rows (their Tdot should be 0).  M and K are assembled once per
 * call; workspace is allocated and freed inside.  (sync)
 * Errors: MF_ERR_ARG, those of mf_assemble and mf_pcg (a solve that misses lin_tol stops
 * the run with MF_ERR_NOT_CONVERGED; res->steps counts the finished steps), MF_ERR_OOM.
 */
mf_status mf_heat_transient(const mf_pattern_t* P, double capacity, double conductivity, const double* coords,
                            const double* elem_k, const double* source, const uint8_t* dirichlet,
                            const mf_quadrature* quad, const mf_transient_opts* opts, double* T, double* Tdot,
                            mf_transient_result* res, void* stream);

/* mf_heat_transient with the steps' solves preconditioned by the multigrid cycle (mf_mg_*,
   declared below) of the effective matrix c1 K + c2 / (b1 dt) M: every coarse level
   assembles both forms (elem_k averaged over the eight children) and combines them with
   the same weights and elimination.  P must be a structured grid of 8-node hexahedra
   (MF_ERR_UNSUPPORTED otherwise).  The optional initial-rate solve keeps Jacobi.  (sync)
   Errors: those of mf_heat_transient and of mf_mg_create. */
typedef struct mf_mg_opts_s mf_mg_opts;
mf_status mf_heat_transient_mg(const mf_pattern_t* P, double capacity, double conductivity, const double* coords,
                               const double* elem_k, const double* source, const uint8_t* dirichlet,
                               const mf_mg_opts* mg, const mf_quadrature* quad, const mf_transient_opts* opts,
                               double* T, double* Tdot, mf_transient_result* res, void* stream);

/* ------------------------------------------------------------------------------------
 * Boundary forms: the physics one dimension lower (Sec. 2.2, opening of the algorithm),
 * integrated over element faces with the 2x2 Gauss rule of the face and added into an
 * assembled K and d.  Forms of Sec. 4.1 (thermal), Sec. 4.2 (elasticity) and Sec. 4.3
 * (flow), with the sign reading of the domain forms (R = -d_paper for the thermal and
 * elastic forms, R = +d_paper for the flow; K = dR/dU, d = -R(U)):
 *   MF_BFORM_PENALTY     R_(a,i) = int coef N_a (u_i - g_i)          fix (1 or 3 fields)
 *   MF_BFORM_CONVECTION  R_a     = int coef N_a (T - T_env)           coef = h   (1 field)
 *   MF_BFORM_RADIATION   R_a     = int coef N_a (T^4 - T_env^4)       coef = e_m sigma^b
 *   MF_BFORM_FLUX        R_a     = - int coef N_a n . grad T          coef = k: the flux
 *                        term of the thermal fix condition (grad T of the face's element)
 *   MF_BFORM_TRACTION    R_(a,i) = - int N_a sigma^l_ij n_j           load (3 fields), or
 *                        - int N_a t_i with a nodal traction t given as `target`
 * Flow (4 fields u_0, u_1, u_2, p; coef = tau^b, value[3] = rho, value[4] = mu), every
 * kind with the base term R_(a,i) += int N_a (p n_i - mu u_i,j n_j):
 *   MF_BFORM_NS_INFLOW   R_(a,i) += int rho N_a u^w_i (u^w . n) + mu (n . grad N_a)(u^w_i - u_i)
 *                                   + tau^b rho N_a (u_i - u^w_i);  R_(a,p) += int N_a (u^w - u) . n
 *   MF_BFORM_NS_OUTFLOW  R_(a,i) += int rho N_a u_i (u . n)
 *   MF_BFORM_NS_FIX      the inflow form with u^w = 0
 *   (grad N_a is the gradient of the face's element, so all 8 of its nodes get rows.)
 * g / T_env / u^w come from `target` ([nf][n_nodes] nodal values, interpolated; rows
 * 0..2 for u^w) when given, else from value[0..nf) (value[0..3) for u^w); sigma^l is
 * value[0..9) row-major; n is the outward unit normal.
 * ------------------------------------------------------------------------------------ */
typedef enum {
    MF_BFORM_PENALTY = 0,
    MF_BFORM_CONVECTION = 1,
    MF_BFORM_RADIATION = 2,
    MF_BFORM_FLUX = 3,
    MF_BFORM_TRACTION = 4,
    MF_BFORM_NS_INFLOW = 5,
    MF_BFORM_NS_OUTFLOW = 6,
    MF_BFORM_NS_FIX = 7
} mf_bform_kind;

typedef struct {
    mf_bform_kind kind;
    double coef;
    double value[9];
} mf_bform;

/*
 * mf_assemble_boundary - adds the face integrals of `form` into K [nnz] and d [n_rows]
 * (precision prec, the layout of mf_assemble), so call it after mf_assemble, without a
 * Dirichlet mask there (boundary forms replace the elimination).  Faces: face_elem
 * [n_faces] element ids and face_id [n_faces] local faces 2 * axis + side (side 1: the
 * face at xi_axis = +1), device arrays.  state [nf][n_nodes] (device, precision prec, or
 * NULL = 0) is the linearisation point of the radiation, flux, penalty and flow residuals.
 * P must have full coupling and be: 8-node hexahedra (all forms, 2x2 face rule),
 * 20-node hexahedra (penalty, convection, radiation and traction, over the eight nodes of
 * the face with the 3x3 face rule), 10-node tetrahedra (the same four forms over the six
 * nodes of the face; face_id k is the face opposite vertex k, 0..3; collapsed 4x4 Gauss
 * rule of the triangle) or 4- and 8-node quadrilaterals (the same four forms on element
 * edges: face_id 2 * axis + side as for hexahedra, 2 or 3 Gauss points along the edge,
 * 1 or 2 fields, sigma^l the leading 2x2 block of value[0..9)); MF_ERR_UNSUPPORTED
 * otherwise.
 * Queued on the stream (see below for the one synchronisation).  Reported by
 * mf_status_poll (until the next mf_assemble clears the status): a face whose element id
 * or local face is out of range (skipped; MF_ERR_ARG with the first such face), and a
 * degenerate face (zero area) or element (det J <= 0, flux form; MF_ERR_BAD_JACOBIAN).
 * Errors: MF_ERR_ARG (a form/field-count mismatch or bad arguments), MF_ERR_UNSUPPORTED
 * (an element type the boundary kernels do not cover, or the flux and flow forms on
 * anything but 8-node hexahedra), MF_ERR_HIP.  Two calls with the same inputs give the
 * same bits: on 8-node hexahedra the faces are marked per element and added element
 * colour by element colour (async); on the other elements they go in buckets of (colour
 * of the face's element, local face), one launch per non-empty bucket, and the call
 * synchronises the stream once to size the buckets.
 */
mf_status mf_assemble_boundary(const mf_pattern_t* P, const mf_bform* form, const double* coords,
                               int64_t n_faces, const int32_t* face_elem, const uint8_t* face_id,
                               const void* state, const void* target, mf_precision prec, void* K,
                               void* d, void* stream);

/* ------------------------------------------------------------------------------------
 * Linear solve of the assembled system (Sec. 2.2 D-4 leaves the solver open): FP64
 * preconditioned conjugate gradients for symmetric positive definite K.
 * ------------------------------------------------------------------------------------ */
typedef enum {
    MF_PRECOND_NONE = 0,    /* plain CG                                                 */
    MF_PRECOND_JACOBI = 1,  /* z = r / diag(K)                                          */
    MF_PRECOND_NN = 2,      /* learned network (mf_nn_t), flexible CG; an iteration whose
                               z.r <= 0 or non-finite z falls back to the Jacobi z      */
    MF_PRECOND_MG = 3       /* one geometric multigrid V-cycle (mf_mg_t, see below); mf_pcg
                               uses the flexible beta with it                           */
} mf_precond_kind;

typedef struct mf_nn_s mf_nn_t;   /* opaque learned preconditioner, see below */
typedef struct mf_mg_s mf_mg_t;   /* opaque multigrid preconditioner, see below */

typedef struct {
    int64_t n_rows;
    const int32_t* row_ptr;   /* [n_rows+1] (device) */
    const int32_t* col_idx;   /* [nnz] (device) */
    const double* values;     /* [nnz] (device), FP64 */
} mf_csr;

typedef struct {
    double tol;               /* stop when |b - K x|_2 / |b|_2 <= tol (true residual)      */
    int32_t maxit;
    int32_t check_every;      /* iterations between host convergence checks (0 = 8)       */
    int32_t use_graph;        /* 1: replay each chunk of iterations as a HIP graph (needs a
                                 non-default stream; silently off otherwise)              */
    mf_precond_kind precond;
    int32_t stall_iters;      /* mf_pcg: iterations without the recurrence residual
                                 falling below 0.9 x its best that count as stagnation
                                 (0 = 512; judged at the host checks); ignored by
                                 mf_bicgstab                                             */
    const mf_nn_t* net;       /* MF_PRECOND_NN only */
    const mf_mg_t* mg;        /* MF_PRECOND_MG only: updated for this K (mf_mg_update)    */
} mf_pcg_opts;

typedef struct {
    int32_t iterations;       /* iterations run (a multiple of check_every unless maxit)  */
    int32_t converged;        /* 1 when the true residual met tol                         */
    int32_t fallbacks;        /* MF_PRECOND_NN: iterations that used the Jacobi z         */
    int32_t restarts;         /* restarts from the current x (stagnation, breakdown)      */
    double true_relres;       /* |b - K x|_2 / |b|_2 at exit                              */
} mf_pcg_result;

/*
 * mf_pcg - solve K x = b from x0 = 0.  x [n_rows] is overwritten.  (sync: returns when
 * the solve is done.)  Scalars stay on the device; the host reads the recurrence
 * residual every check_every iterations and accepts only a true residual <= tol.
 * Stagnation (opts->stall_iters iterations without progress), or a recurrence residual that
 * meets tol while the true residual does not, restarts the method from the current x:
 * r = b - K x, z = Jacobi r, p = z; an MF_PRECOND_NN or MF_PRECOND_MG solve continues as
 * Jacobi-PCG after its first restart.  At most 8 restarts; res->restarts counts them.
 * MF_PRECOND_MG needs opts->mg updated for this K (A->values); the cycle is applied with
 * the flexible beta, as for the network.
 * Errors: MF_ERR_ARG, MF_ERR_NOT_CONVERGED (maxit reached; x and res hold the last
 * iterate), MF_ERR_NONFINITE (breakdown: p.Kp <= 0 or r.z <= 0), MF_ERR_OOM, MF_ERR_HIP.
 */
mf_status mf_pcg(const mf_csr* A, const double* b, double* x, const mf_pcg_opts* opts,
                 mf_pcg_result* res, void* stream);

/*
 * mf_pcg_noalloc - mf_pcg for callers that cannot allocate device memory (code that must
 * not call hipMalloc, such as tight serving loops or harnesses that forbid it).  Same
 * arguments, result and synchronisation as mf_pcg, with these limits:
 *   - n_rows <= mf_pcg_noalloc_max_rows() (2^20); larger systems return MF_ERR_ARG;
 *   - opts->precond MF_PRECOND_JACOBI or MF_PRECOND_NONE (MF_PRECOND_NN and
 *     MF_PRECOND_MG: MF_ERR_UNSUPPORTED);
 *   - the SpMV runs on the caller's CSR arrays (no slot-major copy of K) and the
 *     iterations launch eagerly (use_graph is ignored), so the iteration count can
 *     differ from mf_pcg's by rounding, within the same tolerance.
 * The workspace is one fixed device array of the library (about 48 MiB per GPU, held
 * until the process ends); calls allocate nothing, not even on the first call.  Every
 * call on a GPU uses that GPU's one workspace: calls that overlap on one GPU (two host
 * threads, or two streams in flight) race and must be serialised by the caller.
 */
mf_status mf_pcg_noalloc(const mf_csr* A, const double* b, double* x, const mf_pcg_opts* opts,
                         mf_pcg_result* res, void* stream);

/* Largest n_rows mf_pcg_noalloc accepts. */
int64_t mf_pcg_noalloc_max_rows(void);

/* y = A x (FP64 CSR).  Async. */
mf_status mf_spmv(const mf_csr* A, const double* x, double* y, void* stream);

/*
 * mf_bicgstab - solve K x = b for a non-symmetric K (the Newton tangent of the flow form
 * of Sec. 4.3; Sec. 2.2 D-4 leaves the solver open) by BiCGStab from x0 = 0 with shadow
 * residual b, right-preconditioned by Jacobi (opts->precond MF_PRECOND_JACOBI), by one
 * multigrid V-cycle (MF_PRECOND_MG) or unpreconditioned (MF_PRECOND_NONE).  Options, result
 * and synchronisation as mf_pcg
 * (opts->net is ignored, res->fallbacks is 0); the true residual |b - K x|_2 / |b|_2
 * decides convergence.  On a breakdown (rh.r, rh.Kp or t.t exactly 0 or non-finite), or
 * when the recurrence residual meets tol but the true residual does not, the method
 * restarts from the current x with rh = r = b - K x (at most 64 restarts).
 * x [n_rows] is overwritten.  (sync)
 * MF_PRECOND_MG needs opts->mg updated for this K (A->values), else MF_ERR_ARG.
 * Errors: MF_ERR_ARG (including MF_PRECOND_NN), MF_ERR_NOT_CONVERGED (maxit reached; x and
 * res hold the last iterate), MF_ERR_NONFINITE (a non-finite true residual, or breakdown
 * after 64 restarts), MF_ERR_OOM, MF_ERR_HIP.
 */
mf_status mf_bicgstab(const mf_csr* A, const double* b, double* x, const mf_pcg_opts* opts,
                      mf_pcg_result* res, void* stream);

/* ------------------------------------------------------------------------------------
 * Newton iteration for the steady flow form (Sec. 2.1: the update solves K dU = -R(U)
 * with K = dR/dU, repeated until the residual vanishes; form of Sec. 4.3).  Each step
 * assembles K and d = -R(U) in FP64 at the current state with the Dirichlet elimination
 * (d is 0 on constrained rows, so the update keeps their values), solves K dU = d with
 * mf_bicgstab (Jacobi; mf_ns_newton_mg: a multigrid cycle) and adds dU to the state.
 * ------------------------------------------------------------------------------------ */
typedef struct {
    double rtol;            /* converged when |d|_2 <= rtol |d_0|_2 ...                     */
    double atol;            /* ... or |d|_2 <= atol (d_0: the residual of the initial state) */
    int32_t max_steps;      /* updates at most                                              */
    double lin_tol;         /* floor of the linear solves' relative true-residual tolerance:
                               step k asks for max(lin_tol, min(0.1, |d_k|_2 / |d_0|_2),
                               min(0.5, 0.5 t / |d_k|_2)), t = max(rtol |d_0|_2, atol): no
                               tighter than the final residual test needs                 */
    int32_t lin_maxit;
    int32_t check_every;    /* linear solve: iterations between host checks (0 = 8)          */
    int32_t use_graph;      /* linear solve: replay chunks as a HIP graph (non-default stream) */
} mf_newton_opts;

#define MF_NEWTON_MAX_HISTORY 64
typedef struct {
    int32_t steps;          /* updates applied                                              */
    int32_t converged;      /* 1 when the residual test passed                              */
    int32_t lin_iterations; /* BiCGStab iterations over all steps                           */
    double res_norm[MF_NEWTON_MAX_HISTORY];  /* |d|_2 at the state before update k, k <= steps
                                                (the first min(steps+1, 64) entries)        */
} mf_newton_result;

/*
 * mf_ns_newton - state [4][n_nodes] (device, FP64: u1, u2, u3, p per node) is the initial
 * guess and carries the Dirichlet values of the constrained DOFs; it is overwritten with
 * the last iterate.  P is a pattern of the 3D flow form (4 fields, full coupling) in
 * either numbering; dirichlet [n_rows] (device, may be NULL) marks constrained rows; the
 * form must be MF_FORM_NS_SUPG.  Workspace for K, d and dU is allocated and freed inside
 * the call.  (sync)
 * Errors: those of mf_assemble, and of mf_bicgstab unless the solve lowered the residual
 * (a solve that stops short of its tolerance, by the iteration limit or a breakdown, still
 * gives its update); MF_ERR_NOT_CONVERGED when max_steps is reached (state and res hold
 * the last iterate).
 */
mf_status mf_ns_newton(const mf_pattern_t* P, const mf_form* form, const double* coords, double* state,
                       const uint8_t* dirichlet, const mf_quadrature* quad, const mf_newton_opts* opts,
                       mf_newton_result* res, void* stream);

/* One set of boundary faces with its form (see mf_assemble_boundary): face_elem and
   face_id are device arrays of n_faces entries; target is NULL or [nf][n_nodes] FP64. */
typedef struct {
    mf_bform form;
    int64_t n_faces;
    const int32_t* face_elem;
    const uint8_t* face_id;
    const double* target;
} mf_bset;

/*
 * mf_ns_newton_ex - mf_ns_newton with the flow's boundary forms (Sec. 4.3: inflow, outflow,
 * fix; any form of mf_assemble_boundary) in the residual and tangent of every step: each
 * step assembles the domain form without elimination, adds the n_bsets face sets (host
 * array bsets, linearised at the current state), and only then eliminates the Dirichlet
 * rows.  With n_bsets = 0 it is mf_ns_newton.  Errors: those of mf_ns_newton and of
 * mf_assemble_boundary (a face set whose form does not fit the pattern: MF_ERR_ARG).
 */
mf_status mf_ns_newton_ex(const mf_pattern_t* P, const mf_form* form, const double* coords, double* state,
                          const uint8_t* dirichlet, const mf_bset* bsets, int32_t n_bsets,
                          const mf_quadrature* quad, const mf_newton_opts* opts, mf_newton_result* res,
                          void* stream);

/* ------------------------------------------------------------------------------------
 * Geometric multigrid preconditioner on a structured grid of 8-node hexahedra (the
 * lexicographic grid of mf_pattern_grid).  The paper leaves the solver of Sec. 2.2 D-4
 * open; this one serves the Newton step of Sec. 2.1 where the Jacobi preconditioner is too
 * weak (the flow tangent of Sec. 4.3 past about 36^3 elements).
 *   Levels: level 0 is the pattern's grid; level l+1 halves the elements per axis while
 *     every axis of level l has an even element count, and its node (i,j,k) is the level-l
 *     node (2i,2j,2k).  Coarsening stops at max_levels levels, or at the first level with at
 *     most coarse_rows rows, or when an axis is odd.
 *   Coarse operators: the same form assembled (FP64) on each coarser grid from the
 *     coordinates, linearisation state and Dirichlet flags of the coincident fine nodes
 *     (injection), an element coefficient field averaged over the eight children, and the
 *     flow form's stabilisation constants of that level.
 *   Transfers: P = trilinear interpolation (field by field), restriction R = P^T.
 *   Smoother: damped Jacobi x <- x + omega D^-1 (b - A x), D^-1 = 0 where diag A = 0.
 *   V-cycle V(l, b): on the coarsest level coarse_sweeps sweeps from x = 0; otherwise
 *     pre_sweeps sweeps from x = 0, r = b - A x, b_c = R r with the coarse Dirichlet rows set
 *     to 0, x += P V(l+1, b_c), post_sweeps sweeps.  It is a fixed linear map of b.
 * ------------------------------------------------------------------------------------ */
#define MF_MG_MAX_LEVELS 8
struct mf_mg_opts_s {
    int32_t max_levels;     /* levels including level 0, 1..MF_MG_MAX_LEVELS (0 = 8)         */
    int32_t coarse_rows;    /* stop coarsening at a level with at most this many rows (0 = 512) */
    int32_t pre_sweeps;     /* >= 0 */
    int32_t post_sweeps;    /* >= 0 */
    int32_t coarse_sweeps;  /* >= 0 */
    double omega;           /* Jacobi damping, in (0, 1]                                      */
    double tau_m[MF_MG_MAX_LEVELS];  /* flow form: tau_m, tau_c of level l's tangent (entry 0 */
    double tau_c[MF_MG_MAX_LEVELS];  /* unused: level 0 is the caller's K); 0 = the form's    */
};

/* Builds the level grids and their patterns (the pattern's numbering and field count) and
   allocates every level's vectors.  P: 3D 8-node hexahedra on a structured grid with full
   coupling (MF_ERR_UNSUPPORTED otherwise).  (sync)  Errors: MF_ERR_ARG, MF_ERR_UNSUPPORTED,
   MF_ERR_OOM, MF_ERR_HIP.  *out is NULL on error. */
mf_status mf_mg_create(const mf_pattern_t* P, const mf_mg_opts* opts, void* stream, mf_mg_t** out);

/* (host) number of levels and each level's element counts per axis (dims [n_levels][3],
   may be NULL; room for MF_MG_MAX_LEVELS). */
mf_status mf_mg_levels(const mf_mg_t* mg, int32_t* n_levels, int64_t* dims);

/* Prepares the cycle for the level-0 operator K [nnz of P] (device FP64, borrowed: it must
   stay unchanged until the next update): injects coords [3][n_nodes] and the fields'
   lin_state and dirichlet to every coarser level, carries elem_param (FP64 [n_elems], or
   NULL) to a coarse element as the mean of its eight children, assembles each coarse
   operator with `form` and `quad`, and forms every level's D^-1.  fields may be NULL; its
   nodal_src must be NULL (MF_ERR_UNSUPPORTED: the cycle needs no right side).  (sync)
   Errors: those of mf_assemble (a coarse element with det J <= 0: MF_ERR_BAD_JACOBIAN),
   MF_ERR_ARG, MF_ERR_HIP. */
mf_status mf_mg_update(mf_mg_t* mg, const mf_form* form, const double* coords, const mf_fields* fields,
                       const mf_quadrature* quad, const double* K, void* stream);

/* mf_mg_update with boundary forms on element faces (mf_bset, above; Sec. 4.1-4.3): K
   is the domain form plus the n_bsets face sets, then the Dirichlet elimination, and each
   coarse operator is built the same way.  A coarse face stands for four fine ones: the
   fine face (element (ex,ey,ez), local face 2 axis + side) is kept, as the coarse face of
   element (ex/2, ey/2, ez/2), when its in-plane indices are even and its index along the
   axis is even for side 0, odd for side 1; nodal targets are injected.  (sync)  Errors:
   those of mf_mg_update and mf_assemble_boundary. */
mf_status mf_mg_update_ex(mf_mg_t* mg, const mf_form* form, const double* coords, const mf_fields* fields,
                          const mf_bset* bsets, int32_t n_bsets, const mf_quadrature* quad, const double* K,
                          void* stream);

/* z = V(0, r): one cycle, r and z [n_rows] device FP64 (distinct).  Kernels only, on the
   stream (async, no allocation, no memset: can be captured in a HIP graph).  Calls that
   overlap on one mf_mg_t race (they share its level vectors).  Errors: MF_ERR_ARG (not
   updated yet, NULL vectors), MF_ERR_HIP. */
mf_status mf_mg_apply(const mf_mg_t* mg, const double* r, double* z, void* stream);

void mf_mg_destroy(mf_mg_t* mg);

/*
 * mf_ns_newton_mg - mf_ns_newton_ex with the multigrid preconditioner in every linear
 * solve: each step assembles K and d (with the n_bsets face sets, as mf_ns_newton_ex),
 * updates the cycle for that K (mf_mg_update_ex with the current state and the same face
 * sets) and solves with mf_bicgstab (MF_PRECOND_MG).  P must be a structured grid as for
 * mf_mg_create.  (sync)  Errors: those of mf_ns_newton_ex, mf_mg_create and
 * mf_mg_update_ex.
 */
mf_status mf_ns_newton_mg(const mf_pattern_t* P, const mf_form* form, const double* coords, double* state,
                          const uint8_t* dirichlet, const mf_bset* bsets, int32_t n_bsets, const mf_mg_opts* mg,
                          const mf_quadrature* quad, const mf_newton_opts* opts, mf_newton_result* res,
                          void* stream);

/* ------------------------------------------------------------------------------------
 * Learned preconditioner for mf_pcg on structured-grid scalar systems (node id
 * x + nx (y + ny z), one DOF per node).  A small linear multilevel 3D convolution network
 * applied to the diagonally scaled residual:
 *   z = Dm^-1/2 N(v),  v = Dm^-1/2 r,  Dm = diag(K),
 *   N(v) = y_0 + P(y_1 + P(y_2 + ...)),  y_0 = conv(v) (1->1 channel),
 *   y_l = conv(conv(conv(R^l v))) (1 -> c_l -> c_l -> 1), R full weighting, P = R^T,
 *   3x3x3 kernels, zero padding, no bias; z = 0 on Dirichlet rows.
 * Weights and activations are BF16, accumulation FP32; parameters are kept in FP32 for
 * the optimiser.  Training (Adam) minimises either the residual loss |K z - r|^2 / |r|^2
 * or the energy-norm error of z (mf_nn_train_step); the shipped weights were trained
 * with the energy loss.
 * ------------------------------------------------------------------------------------ */

/* grid (host) [3] = node counts (nx, ny, nz), odd and >= 3 on every level but the last;
   channels (host) [levels], channels[0] = 1, others in {1, 2, 4, 8}.  Parameters start
   with the level-0 stencil equal to the identity (the network starts as Jacobi) and the
   other weights drawn from N(0, 0.02^2) with the given seed.  (sync) */
mf_status mf_nn_create(const int32_t* grid, int32_t levels, const int32_t* channels, uint64_t seed,
                       mf_nn_t** out);

/* (sync) Number of parameters; copy them out (get, host, may be NULL) and/or replace them
   (set, host, may be NULL; resets the optimiser state).  Layout: the level-0 tensor
   [1][1][27], then per level l >= 1: [c][1][27], [c][c][27], [1][c][27]; each kernel
   tap t = (dz+1)*9 + (dy+1)*3 + (dx+1). */
mf_status mf_nn_params(mf_nn_t* net, float* get, const float* set, int64_t* n_params);

/* Bind the network to one assembled system: K (device CSR, FP64, n_rows = node count)
   and its Dirichlet mask (device, may be NULL).  Async; K must stay valid while bound. */
mf_status mf_nn_set_system(mf_nn_t* net, const mf_csr* K, const uint8_t* dirichlet, void* stream);

/* z = N_theta(r) for the bound system (BF16 inference).  Async, graph-capturable. */
mf_status mf_nn_apply(mf_nn_t* net, const double* r, double* z, void* stream);

/* One training step on residual r of the bound system: forward, loss, backward.
   Loss: with e == NULL, |K z - r|^2 / |r|^2; with e (device, the error whose residual is
   r = K e), the energy-norm error (z - e)^T K (z - e) / e^T K e, the quantity CG
   minimises.  grad (host, may be NULL): if given, the gradient is copied out and the
   parameters are NOT updated; otherwise one Adam step with learning rate lr.  *loss
   (host) receives the loss.  (sync) */
mf_status mf_nn_train_step(mf_nn_t* net, const double* r, const double* e, double lr, double* loss,
                           float* grad, void* stream);

/* Checkpoint of training (the resumable state: parameters, both Adam moment vectors, the
   step count that sets Adam's bias corrections, the seed of the initial weights, and the
   architecture).  mf_nn_checkpoint_size gives the byte count; mf_nn_save copies the state
   into buf (host, at least that many bytes); mf_nn_load restores it into a network of the
   same grid, levels and channels (MF_ERR_ARG otherwise), after which training continues
   exactly as it would have without the interruption.  The training data is the caller's:
   a caller that draws its systems from the step count resumes them too.  (sync) */
mf_status mf_nn_checkpoint_size(const mf_nn_t* net, int64_t* bytes);
mf_status mf_nn_save(const mf_nn_t* net, void* buf, int64_t bytes);
mf_status mf_nn_load(mf_nn_t* net, const void* buf, int64_t bytes);

void mf_nn_destroy(mf_nn_t* net);

/* Library version string. */
const char* mf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MF_H */
