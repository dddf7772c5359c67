/*
 * Oracle for finite-element assembly of K x = d (MetaFEM, arXiv 2111.03541).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product (the HIP
 * library under paper_2111_03541_amd/) never calls it, and the two share no code.
 *
 * Plain, sequential, FP64 C.  Every routine is the textbook definition of what it
 * computes, written out element by element and scattered in element-id order; no
 * blocking, fusion or reordering.  One exception, for the timed CPU baseline only:
 * or_assemble_colored runs the same element routine on all host cores, one element
 * colour at a time (checked against or_assemble by the test suite).  Sections cited are those of the paper:
 *   Sec. 2.1        weak form as a sum of bilinear forms, numerical integration,
 *                   residual component d_a and tangent K = dd/dphi (Eqs. Newton-Raphson,
 *                   stiffness)
 *   Sec. 2.2 B-1..B-4  element-to-control-point map, control-point pairs, DOF map
 *   Sec. 2.2 D-2, D-3  residual and stiffness assembly by element loops
 *   Sec. 4.1        thermal conduction weak form
 *   Sec. 4.2        linear elasticity weak form, Lame parameters
 *   Sec. 4.3        steady incompressible Navier-Stokes with SUPG/PSPG/LSIC terms
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - sign: the exported K is dR/dU and d = -R(U0), where R is the paper's weak form
 *     times -1 for the thermal and elastic forms (written with negative leading
 *     terms) and times +1 for the flow form (written with +mu diffusion).  Then K is
 *     SPD for the two linear forms and K dU = d is the Newton step.
 *   - reference element [-1,1]^dim, local node a = ax + 2 ay + 4 az, corner signs
 *     s_{a,d} = 2 bit_d(a) - 1; Gauss-Legendre in tensor order q = qx + p qy + p^2 qz.
 *   - sources are nodal values interpolated with the element basis.
 *   - the flow residual drops -mu u_{i,kk} in Rm_i (zero for Q1 on affine cubes).
 *   - Dirichlet constraints: symmetric elimination keeping the sparsity structure.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXNEN 8
#define OR_MAXDIM 3
#define OR_MAXQ 27
#define OR_MAXNF 4

enum { OR_MASS = 0, OR_POISSON = 1, OR_ELASTICITY = 2, OR_NS_SUPG = 3 };
enum { OR_NODE_MAJOR = 0, OR_FIELD_MAJOR = 1 };
enum { OR_OK = 0, OR_ERR_ARG = 1, OR_ERR_BAD_JACOBIAN = 2, OR_ERR_PATTERN = 3, OR_ERR_OOM = 4 };

/* ------------------------------------------------------------------------- */
/* Quadrature and basis (numerical integration of a bilinear form, Sec. 2.1)  */
/* ------------------------------------------------------------------------- */

/* Gauss-Legendre rule on [-1,1] with p points (closed forms for p = 1, 2, 3). */
int or_gauss(int p, double* pts, double* wts)
{
    if (p == 1) { pts[0] = 0.0; wts[0] = 2.0; return 0; }
    if (p == 2) {
        double r = 1.0 / sqrt(3.0);
        pts[0] = -r; pts[1] = r; wts[0] = 1.0; wts[1] = 1.0; return 0;
    }
    if (p == 3) {
        double r = sqrt(3.0 / 5.0);
        pts[0] = -r; pts[1] = 0.0; pts[2] = r;
        wts[0] = 5.0 / 9.0; wts[1] = 8.0 / 9.0; wts[2] = 5.0 / 9.0; return 0;
    }
    return OR_ERR_ARG;
}

/* Q1 Lagrange basis on the reference cube: N_a(xi) = prod_d (1 + s_{a,d} xi_d) / 2.
   N[a], dN[a*dim + d] = dN_a / dxi_d. */
void or_basis(int dim, const double* xi, double* N, double* dN)
{
    int nen = 1 << dim;
    for (int a = 0; a < nen; ++a) {
        double f[OR_MAXDIM];
        double s[OR_MAXDIM];
        for (int d = 0; d < dim; ++d) {
            s[d] = ((a >> d) & 1) ? 1.0 : -1.0;
            f[d] = 0.5 * (1.0 + s[d] * xi[d]);
        }
        double prod = 1.0;
        for (int d = 0; d < dim; ++d) prod *= f[d];
        N[a] = prod;
        for (int d = 0; d < dim; ++d) {
            double g = 0.5 * s[d];
            for (int e = 0; e < dim; ++e)
                if (e != d) g *= f[e];
            dN[a * dim + d] = g;
        }
    }
}

/* Tensor-product quadrature: points xi[q*dim + d], weights w[q]. Returns Q. */
static int tensor_rule(int dim, int p, double* xi, double* w)
{
    double pts[3], wts[3];
    if (or_gauss(p, pts, wts)) return -1;
    int Q = 1;
    for (int d = 0; d < dim; ++d) Q *= p;
    for (int q = 0; q < Q; ++q) {
        int r = q;
        double wq = 1.0;
        for (int d = 0; d < dim; ++d) {
            int k = r % p;
            r /= p;
            xi[q * dim + d] = pts[k];
            wq *= wts[k];
        }
        w[q] = wq;
    }
    return Q;
}

/* ------------------------------------------------------------------------- */
/* Geometry at one integration point                                          */
/* ------------------------------------------------------------------------- */

/* J_ij = sum_a x_{a,i} dN_a/dxi_j; inverse by cofactors; g_{a,m} = dN_a/dx_m.
   Returns det J. */
static double geometry(int dim, int nen, const double x[OR_MAXNEN][OR_MAXDIM],
                       const double* dN, double g[OR_MAXNEN][OR_MAXDIM])
{
    double J[3][3] = {{0}}, Ji[3][3];
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
            double s = 0.0;
            for (int a = 0; a < nen; ++a) s += x[a][i] * dN[a * dim + j];
            J[i][j] = s;
        }
    double det;
    if (dim == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        Ji[0][0] = J[1][1] / det;  Ji[0][1] = -J[0][1] / det;
        Ji[1][0] = -J[1][0] / det; Ji[1][1] = J[0][0] / det;
    } else {
        double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        /* inverse = adjugate / det, adj = cofactor^T */
        Ji[0][0] = c00 / det;
        Ji[1][0] = c01 / det;
        Ji[2][0] = c02 / det;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    }
    /* dN_a/dx_m = sum_j dN_a/dxi_j * dxi_j/dx_m = sum_j dN[a][j] * Ji[j][m] */
    for (int a = 0; a < nen; ++a)
        for (int m = 0; m < dim; ++m) {
            double s = 0.0;
            for (int j = 0; j < dim; ++j) s += dN[a * dim + j] * Ji[j][m];
            g[a][m] = s;
        }
    return det;
}

/* ------------------------------------------------------------------------- */
/* Sparsity pattern (Sec. 2.2 B-1..B-4)                                       */
/* ------------------------------------------------------------------------- */

typedef struct {
    int dim, nen, nf, numbering;
    int64_t n_nodes, n_el, n_rows, nnz;
    uint8_t coupling[OR_MAXNF * OR_MAXNF];
    int64_t* nbr_ptr;   /* [n_nodes+1] node graph: N(a) = sorted unique neighbours */
    int32_t* nbr;
    int64_t* row_ptr64; /* [n_rows+1] */
    int32_t* col_idx;   /* [nnz] */
    uint8_t* rank;      /* [nen*nen][n_el]: position of conn[b][e] in N(conn[a][e]) */
    int32_t* conn;      /* copy of the element-to-node map [nen][n_el] */
} or_pattern;

static int cmp_i64(const void* a, const void* b)
{
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

static int64_t dof_of(const or_pattern* P, int64_t node, int field)
{
    return P->numbering == OR_NODE_MAJOR ? (int64_t)P->nf * node + field
                                         : (int64_t)field * P->n_nodes + node;
}

void or_pattern_free(void* h)
{
    or_pattern* P = (or_pattern*)h;
    if (!P) return;
    free(P->nbr_ptr); free(P->nbr); free(P->row_ptr64); free(P->col_idx); free(P->rank); free(P->conn);
    free(P);
}

/* Build the pattern.  Returns NULL on bad arguments or allocation failure. */
void* or_pattern_build(int dim, int64_t n_nodes, int64_t n_el, const int32_t* conn,
                       int nf, const uint8_t* coupling, int numbering)
{
    if (dim < 2 || dim > 3 || nf < 1 || nf > OR_MAXNF || n_nodes < 0 || n_el < 0) return NULL;
    int nen = 1 << dim;
    for (int64_t k = 0; k < (int64_t)nen * n_el; ++k)
        if (conn[k] < 0 || conn[k] >= n_nodes) return NULL;
    or_pattern* P = (or_pattern*)calloc(1, sizeof(or_pattern));
    if (!P) return NULL;
    P->dim = dim; P->nen = nen; P->nf = nf; P->numbering = numbering;
    P->n_nodes = n_nodes; P->n_el = n_el; P->n_rows = n_nodes * nf;
    for (int i = 0; i < nf * nf; ++i) P->coupling[i] = coupling ? (coupling[i] ? 1 : 0) : 1;
    P->conn = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nen * n_el + 1));
    memcpy(P->conn, conn, sizeof(int32_t) * (size_t)(nen * n_el));

    /* B-1: node -> incident elements */
    int64_t* inc_cnt = (int64_t*)calloc((size_t)n_nodes + 1, sizeof(int64_t));
    for (int a = 0; a < nen; ++a)
        for (int64_t e = 0; e < n_el; ++e) inc_cnt[conn[a * n_el + e] + 1]++;
    for (int64_t v = 0; v < n_nodes; ++v) inc_cnt[v + 1] += inc_cnt[v];
    int64_t* inc = (int64_t*)malloc(sizeof(int64_t) * (size_t)(inc_cnt[n_nodes] + 1));
    int64_t* fill = (int64_t*)calloc((size_t)n_nodes + 1, sizeof(int64_t));
    for (int64_t e = 0; e < n_el; ++e)
        for (int a = 0; a < nen; ++a) {
            int64_t v = conn[a * n_el + e];
            inc[inc_cnt[v] + fill[v]++] = e;
        }

    /* control-point pairs: N(v) = sorted unique nodes sharing an element with v */
    P->nbr_ptr = (int64_t*)calloc((size_t)n_nodes + 1, sizeof(int64_t));
    int64_t cap = 0;
    for (int64_t v = 0; v < n_nodes; ++v) cap += (inc_cnt[v + 1] - inc_cnt[v]) * nen;
    P->nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cap + 1));
    int64_t* tmp = (int64_t*)malloc(sizeof(int64_t) * 4096);
    int64_t pos = 0;
    for (int64_t v = 0; v < n_nodes; ++v) {
        int64_t cnt = 0;
        for (int64_t k = inc_cnt[v]; k < inc_cnt[v + 1]; ++k) {
            int64_t e = inc[k];
            for (int b = 0; b < nen; ++b) {
                if (cnt >= 4096) { free(tmp); free(inc); free(inc_cnt); free(fill);
                                   or_pattern_free(P); return NULL; }
                tmp[cnt++] = conn[b * n_el + e];
            }
        }
        qsort(tmp, (size_t)cnt, sizeof(int64_t), cmp_i64);
        P->nbr_ptr[v] = pos;
        for (int64_t k = 0; k < cnt; ++k)
            if (k == 0 || tmp[k] != tmp[k - 1]) P->nbr[pos++] = (int32_t)tmp[k];
    }
    P->nbr_ptr[n_nodes] = pos;

    /* B-4 (as CSR): row (v,i) holds dof(w,j) for w in N(v), coupling(i,j), ascending */
    P->row_ptr64 = (int64_t*)calloc((size_t)P->n_rows + 1, sizeof(int64_t));
    int64_t nnz = 0;
    for (int64_t v = 0; v < n_nodes; ++v)
        for (int i = 0; i < nf; ++i) {
            int ci = 0;
            for (int j = 0; j < nf; ++j) ci += P->coupling[i * nf + j];
            int64_t r = dof_of(P, v, i);
            P->row_ptr64[r + 1] = (P->nbr_ptr[v + 1] - P->nbr_ptr[v]) * ci;
        }
    for (int64_t r = 0; r < P->n_rows; ++r) P->row_ptr64[r + 1] += P->row_ptr64[r];
    nnz = P->row_ptr64[P->n_rows];
    P->nnz = nnz;
    P->col_idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz + 1));
    int64_t maxrow = 0;
    for (int64_t v = 0; v < n_nodes; ++v) {
        int64_t deg = P->nbr_ptr[v + 1] - P->nbr_ptr[v];
        if (deg * nf > maxrow) maxrow = deg * nf;
    }
    int64_t* row = (int64_t*)malloc(sizeof(int64_t) * (size_t)(maxrow + 1));
    for (int64_t v = 0; v < n_nodes; ++v)
        for (int i = 0; i < nf; ++i) {
            int64_t cnt = 0;
            for (int64_t k = P->nbr_ptr[v]; k < P->nbr_ptr[v + 1]; ++k)
                for (int j = 0; j < nf; ++j)
                    if (P->coupling[i * nf + j]) row[cnt++] = dof_of(P, P->nbr[k], j);
            qsort(row, (size_t)cnt, sizeof(int64_t), cmp_i64);
            int64_t r = dof_of(P, v, i);
            for (int64_t k = 0; k < cnt; ++k) P->col_idx[P->row_ptr64[r] + k] = (int32_t)row[k];
        }
    free(row);

    /* element -> neighbour-rank map */
    P->rank = (uint8_t*)malloc((size_t)nen * nen * (size_t)(n_el > 0 ? n_el : 1));
    for (int64_t e = 0; e < n_el; ++e)
        for (int a = 0; a < nen; ++a)
            for (int b = 0; b < nen; ++b) {
                int64_t va = conn[a * n_el + e], vb = conn[b * n_el + e];
                int64_t r = -1;
                for (int64_t k = P->nbr_ptr[va]; k < P->nbr_ptr[va + 1]; ++k)
                    if (P->nbr[k] == vb) { r = k - P->nbr_ptr[va]; break; }
                P->rank[(size_t)(a * nen + b) * n_el + e] = (uint8_t)(r < 0 ? 255 : r);
            }

    free(tmp); free(inc); free(inc_cnt); free(fill);
    return P;
}

void or_pattern_sizes(const void* h, int64_t* n_rows, int64_t* nnz, int64_t* n_pairs)
{
    const or_pattern* P = (const or_pattern*)h;
    *n_rows = P->n_rows;
    *nnz = P->nnz;
    *n_pairs = P->nbr_ptr[P->n_nodes];
}

void or_pattern_copy(const void* h, int64_t* row_ptr, int32_t* col_idx, uint8_t* rank,
                     int64_t* nbr_ptr, int32_t* nbr)
{
    const or_pattern* P = (const or_pattern*)h;
    if (row_ptr) memcpy(row_ptr, P->row_ptr64, sizeof(int64_t) * (size_t)(P->n_rows + 1));
    if (col_idx) memcpy(col_idx, P->col_idx, sizeof(int32_t) * (size_t)P->nnz);
    if (rank) memcpy(rank, P->rank, (size_t)P->nen * P->nen * (size_t)P->n_el);
    if (nbr_ptr) memcpy(nbr_ptr, P->nbr_ptr, sizeof(int64_t) * (size_t)(P->n_nodes + 1));
    if (nbr) memcpy(nbr, P->nbr, sizeof(int32_t) * (size_t)P->nbr_ptr[P->n_nodes]);
}

/* position of column c in CSR row r, or -1 */
static int64_t find_col(const or_pattern* P, int64_t r, int64_t c)
{
    int64_t lo = P->row_ptr64[r], hi = P->row_ptr64[r + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        int64_t v = P->col_idx[mid];
        if (v == c) return mid;
        if (v < c) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* ------------------------------------------------------------------------- */
/* Element residual and tangent of each weak form                             */
/* ------------------------------------------------------------------------- */

/* Scalar parameters of a form: [coef, nu, rho, mu, tau_m, tau_c]. */
typedef struct { double coef, nu, rho, mu, tau_m, tau_c; } or_params;

static int form_nf(int kind, int dim)
{
    if (kind == OR_ELASTICITY) return dim;
    if (kind == OR_NS_SUPG) return dim + 1;
    return 1;
}

/*
 * Element residual Re[(a,i)] = R restricted to element e, and tangent
 * Ke[(a,i),(b,j)] = dRe[(a,i)]/dU[(b,j)], at the element state U (nodal values
 * [nen][nf]); src are nodal sources [nen][nsrc].  Local dof index is a*nf + i.
 * want_K = 0 skips the tangent.
 */
static int element(int kind, int dim, const or_params* prm, double cparam,
                   const double x[OR_MAXNEN][OR_MAXDIM], const double* U, const double* src,
                   int qpa, double* Re, double* Ke, int want_K)
{
    int nen = 1 << dim, nf = form_nf(kind, dim), ne = nen * nf;
    double xi[OR_MAXQ * OR_MAXDIM], w[OR_MAXQ];
    int Q = tensor_rule(dim, qpa, xi, w);
    if (Q < 0) return OR_ERR_ARG;
    memset(Re, 0, sizeof(double) * ne);
    if (want_K) memset(Ke, 0, sizeof(double) * ne * ne);

    for (int q = 0; q < Q; ++q) {
        double N[OR_MAXNEN], dN[OR_MAXNEN * OR_MAXDIM], g[OR_MAXNEN][OR_MAXDIM];
        or_basis(dim, &xi[q * dim], N, dN);
        double det = geometry(dim, nen, x, dN, g);
        if (!(det > 0.0)) return OR_ERR_BAD_JACOBIAN;
        double W = w[q] * det;

        if (kind == OR_MASS || kind == OR_POISSON) {
            /* MASS:    R_a = int rho_c N_a (u - f)
               POISSON: R_a = int k grad N_a . grad u - N_a f   (Sec. 4.1, steady, times -1) */
            double u = 0.0, f = 0.0, gu[OR_MAXDIM] = {0};
            for (int b = 0; b < nen; ++b) {
                u += N[b] * U[b];
                f += N[b] * (src ? src[b] : 0.0);
                for (int m = 0; m < dim; ++m) gu[m] += g[b][m] * U[b];
            }
            double c = prm->coef * cparam;
            for (int a = 0; a < nen; ++a) {
                if (kind == OR_MASS) {
                    Re[a] += W * c * N[a] * (u - f);
                } else {
                    double s = 0.0;
                    for (int m = 0; m < dim; ++m) s += g[a][m] * gu[m];
                    Re[a] += W * (c * s - N[a] * f);
                }
            }
            if (want_K)
                for (int a = 0; a < nen; ++a)
                    for (int b = 0; b < nen; ++b) {
                        double v;
                        if (kind == OR_MASS) v = c * N[a] * N[b];
                        else {
                            v = 0.0;
                            for (int m = 0; m < dim; ++m) v += g[a][m] * g[b][m];
                            v *= c;
                        }
                        Ke[a * ne + b] += W * v;
                    }
        } else if (kind == OR_ELASTICITY) {
            /* Sec. 4.2: lambda, mu from E, nu; sigma = lambda delta eps_mm + 2 mu eps;
               R_(a,i) = int dN_a/dx_j sigma_ij(u) - N_a b_i   (domain form times -1) */
            double E = prm->coef * cparam, nu = prm->nu;
            double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
            double mu = E / (2.0 * (1.0 + nu));
            double gu[OR_MAXDIM][OR_MAXDIM] = {{0}}; /* gu[i][j] = du_i/dx_j */
            double bq[OR_MAXDIM] = {0};
            for (int b = 0; b < nen; ++b)
                for (int i = 0; i < dim; ++i) {
                    for (int j = 0; j < dim; ++j) gu[i][j] += U[b * nf + i] * g[b][j];
                    bq[i] += N[b] * (src ? src[b * dim + i] : 0.0);
                }
            double tr = 0.0;
            for (int m = 0; m < dim; ++m) tr += gu[m][m];
            double sig[OR_MAXDIM][OR_MAXDIM];
            for (int i = 0; i < dim; ++i)
                for (int j = 0; j < dim; ++j)
                    sig[i][j] = (i == j ? lam * tr : 0.0) + mu * (gu[i][j] + gu[j][i]);
            for (int a = 0; a < nen; ++a)
                for (int i = 0; i < dim; ++i) {
                    double s = 0.0;
                    for (int j = 0; j < dim; ++j) s += g[a][j] * sig[i][j];
                    Re[a * nf + i] += W * (s - N[a] * bq[i]);
                }
            if (want_K)
                for (int a = 0; a < nen; ++a)
                    for (int b = 0; b < nen; ++b) {
                        double gg = 0.0;
                        for (int m = 0; m < dim; ++m) gg += g[a][m] * g[b][m];
                        for (int i = 0; i < dim; ++i)
                            for (int j = 0; j < dim; ++j) {
                                double v = lam * g[a][i] * g[b][j] + mu * g[a][j] * g[b][i] +
                                           (i == j ? mu * gg : 0.0);
                                Ke[(a * nf + i) * ne + b * nf + j] += W * v;
                            }
                    }
        } else if (kind == OR_NS_SUPG) {
            /* Sec. 4.3, domain form NS_BASE + NS_SUPG with Rc = div u and
               Rm_i = rho u_k du_i/dx_k + dp/dx_i (second derivatives dropped).
               Test word -> shape function factor:
                 (u_{i,j}, .) -> dN_a/dx_j,  (u_{i,i}, .) -> dN_a/dx_i,
                 (p, .) -> N_a,  (p_{,i}, .) -> dN_a/dx_i. */
            double rho = prm->rho, mu = prm->mu, tm = prm->tau_m, tc = prm->tau_c;
            double u[OR_MAXDIM] = {0}, p = 0.0;
            double gu[OR_MAXDIM][OR_MAXDIM] = {{0}}; /* gu[i][k] = du_i/dx_k */
            double gp[OR_MAXDIM] = {0};
            for (int b = 0; b < nen; ++b) {
                for (int i = 0; i < dim; ++i) {
                    u[i] += N[b] * U[b * nf + i];
                    for (int k = 0; k < dim; ++k) gu[i][k] += g[b][k] * U[b * nf + i];
                }
                p += N[b] * U[b * nf + dim];
                for (int k = 0; k < dim; ++k) gp[k] += g[b][k] * U[b * nf + dim];
            }
            double div = 0.0;
            for (int i = 0; i < dim; ++i) div += gu[i][i];
            double Rm[OR_MAXDIM];
            for (int i = 0; i < dim; ++i) {
                double c = 0.0;
                for (int k = 0; k < dim; ++k) c += u[k] * gu[i][k];
                Rm[i] = rho * c + gp[i];
            }
            double adv[OR_MAXNEN];
            for (int a = 0; a < nen; ++a) {
                adv[a] = 0.0;
                for (int k = 0; k < dim; ++k) adv[a] += u[k] * g[a][k];
            }
            for (int a = 0; a < nen; ++a) {
                for (int i = 0; i < dim; ++i) {
                    double visc = 0.0;
                    for (int j = 0; j < dim; ++j) visc += g[a][j] * gu[i][j];
                    double r = -rho * adv[a] * u[i]      /* -rho (u_{i,j}, u_i u_j)      */
                               - g[a][i] * p             /* -(u_{i,i}, p)                */
                               + mu * visc               /* +mu (u_{i,j}, u_{i,j})       */
                               + tm * rho * adv[a] * Rm[i] /* tau_m rho (u_{i,j}, Rm_i u_j) */
                               + tc * g[a][i] * div;     /* tau_c (u_{i,i}, Rc)          */
                    Re[a * nf + i] += W * r;
                }
                double gRm = 0.0;
                for (int i = 0; i < dim; ++i) gRm += g[a][i] * Rm[i];
                Re[a * nf + dim] += W * (N[a] * div     /* (p, u_{i,i})                 */
                                         + tm * gRm);   /* tau_m (p_{,i}, Rm_i)         */
            }
            if (want_K)
                for (int a = 0; a < nen; ++a)
                    for (int b = 0; b < nen; ++b) {
                        double gg = 0.0;
                        for (int m = 0; m < dim; ++m) gg += g[a][m] * g[b][m];
                        /* momentum rows, velocity columns: d/du_{b,l} */
                        for (int i = 0; i < dim; ++i)
                            for (int l = 0; l < dim; ++l) {
                                double dil = (i == l) ? 1.0 : 0.0;
                                double v = -rho * dil * adv[a] * N[b]
                                           - rho * u[i] * g[a][l] * N[b]
                                           + mu * dil * gg
                                           + tm * rho * Rm[i] * g[a][l] * N[b]
                                           + tm * rho * rho * adv[a] * N[b] * gu[i][l]
                                           + tm * rho * rho * dil * adv[a] * adv[b]
                                           + tc * g[a][i] * g[b][l];
                                Ke[(a * nf + i) * ne + b * nf + l] += W * v;
                            }
                        /* momentum rows, pressure column */
                        for (int i = 0; i < dim; ++i) {
                            double v = -g[a][i] * N[b] + tm * rho * adv[a] * g[b][i];
                            Ke[(a * nf + i) * ne + b * nf + dim] += W * v;
                        }
                        /* continuity row, velocity columns */
                        for (int l = 0; l < dim; ++l) {
                            double s = 0.0;
                            for (int i = 0; i < dim; ++i) s += g[a][i] * gu[i][l];
                            double v = N[a] * g[b][l] + tm * rho * (N[b] * s + g[a][l] * adv[b]);
                            Ke[(a * nf + dim) * ne + b * nf + l] += W * v;
                        }
                        /* continuity row, pressure column */
                        Ke[(a * nf + dim) * ne + b * nf + dim] += W * tm * gg;
                    }
        } else {
            return OR_ERR_ARG;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Global assembly (Sec. 2.2 D-2 and D-3), sequential scatter in element order */
/* ------------------------------------------------------------------------- */

/*
 * params: [coef, nu, rho, mu, tau_m, tau_c]
 * coords [dim][n_nodes]; elem_param [n_el] or NULL (=1);
 * nodal_src [nsrc][n_nodes] or NULL (nsrc = 1 for MASS/POISSON, dim for ELASTICITY);
 * state [nf][n_nodes] or NULL (=0): the point of linearisation U0 (flow) or the
 * temperature/displacement at which R is evaluated;
 * dirichlet [n_rows] mask or NULL.
 * Outputs: K [nnz] = dR/dU at U0 (K may be NULL), d [n_rows] = -R(U0),
 * bad_elem = first element with det J <= 0 at some integration point, else -1.
 */
int or_assemble(void* h, int kind, const double* params, const double* coords,
                const double* elem_param, const double* nodal_src, const double* state,
                const uint8_t* dirichlet, int qpa, double* K, double* d, int64_t* bad_elem)
{
    const or_pattern* P = (const or_pattern*)h;
    int dim = P->dim, nen = P->nen, nf = form_nf(kind, dim), ne = nen * nf;
    int64_t nn = P->n_nodes, n_el = P->n_el;
    if (nf != P->nf) return OR_ERR_ARG;
    or_params prm = {params[0], params[1], params[2], params[3], params[4], params[5]};
    int nsrc = (kind == OR_ELASTICITY) ? dim : 1;
    double* Ke = (double*)malloc(sizeof(double) * ne * ne);
    if (!Ke) return OR_ERR_OOM;
    if (K) memset(K, 0, sizeof(double) * (size_t)P->nnz);
    memset(d, 0, sizeof(double) * (size_t)P->n_rows);
    *bad_elem = -1;
    int status = OR_OK;
    for (int64_t e = 0; e < n_el && status == OR_OK; ++e) {
        double x[OR_MAXNEN][OR_MAXDIM], U[OR_MAXNEN * OR_MAXNF], src[OR_MAXNEN * OR_MAXDIM];
        double Re[OR_MAXNEN * OR_MAXNF];
        int64_t node[OR_MAXNEN];
        for (int a = 0; a < nen; ++a) {
            node[a] = P->conn[a * n_el + e];
            for (int m = 0; m < dim; ++m) x[a][m] = coords[m * nn + node[a]];
            for (int i = 0; i < nf; ++i) U[a * nf + i] = state ? state[i * nn + node[a]] : 0.0;
            for (int s = 0; s < nsrc; ++s)
                src[a * nsrc + s] = nodal_src ? nodal_src[s * nn + node[a]] : 0.0;
        }
        double cp = elem_param ? elem_param[e] : 1.0;
        int rc = element(kind, dim, &prm, cp, x, U, nodal_src ? src : NULL, qpa, Re, Ke, K != NULL);
        if (rc == OR_ERR_BAD_JACOBIAN) { *bad_elem = e; status = rc; break; }
        if (rc) { status = rc; break; }
        for (int a = 0; a < nen; ++a)
            for (int i = 0; i < nf; ++i) {
                int64_t r = dof_of(P, node[a], i);
                d[r] -= Re[a * nf + i];
                if (!K) continue;
                for (int b = 0; b < nen; ++b)
                    for (int j = 0; j < nf; ++j) {
                        double v = Ke[(a * nf + i) * ne + b * nf + j];
                        int64_t c = dof_of(P, node[b], j);
                        int64_t pos = find_col(P, r, c);
                        if (pos < 0) {
                            if (v != 0.0) { status = OR_ERR_PATTERN; }
                            continue;
                        }
                        K[pos] += v;
                    }
            }
    }
    free(Ke);
    if (status != OR_OK) return status;
    /* Dirichlet elimination: constrained row r -> unit row, d_r = 0; constrained
       columns zeroed in the other rows (structure kept). */
    if (dirichlet) {
        for (int64_t r = 0; r < P->n_rows; ++r) {
            if (dirichlet[r]) d[r] = 0.0;
            if (!K) continue;
            for (int64_t k = P->row_ptr64[r]; k < P->row_ptr64[r + 1]; ++k) {
                int64_t c = P->col_idx[k];
                if (dirichlet[r]) K[k] = (c == r) ? 1.0 : 0.0;
                else if (dirichlet[c]) K[k] = 0.0;
            }
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* The same assembly on all host cores, for the timed CPU baseline            */
/* ------------------------------------------------------------------------- */

/*
 * Element colours: elements in id order, each taking the smallest colour that no
 * element sharing one of its nodes has taken.  Two elements of one colour touch
 * disjoint nodes, hence disjoint rows of K and d.  Returns the number of colours and
 * fills color [n_el], or -1 on allocation failure.
 */
static int color_elements(const or_pattern* P, int32_t* color)
{
    int64_t nn = P->n_nodes, n_el = P->n_el;
    int nen = P->nen;
    int64_t* inc_ptr = (int64_t*)calloc((size_t)nn + 1, sizeof(int64_t));
    int64_t* inc = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_el * nen + 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nn + 1));
    if (!inc_ptr || !inc || !fill) { free(inc_ptr); free(inc); free(fill); return -1; }
    for (int64_t e = 0; e < n_el; ++e)
        for (int a = 0; a < nen; ++a) ++inc_ptr[P->conn[a * n_el + e] + 1];
    for (int64_t v = 0; v < nn; ++v) inc_ptr[v + 1] += inc_ptr[v];
    memcpy(fill, inc_ptr, sizeof(int64_t) * (size_t)nn);
    for (int64_t e = 0; e < n_el; ++e)
        for (int a = 0; a < nen; ++a) inc[fill[P->conn[a * n_el + e]]++] = e;
    int n_colors = 0;
    for (int64_t e = 0; e < n_el; ++e) color[e] = -1;
    for (int64_t e = 0; e < n_el; ++e) {
        uint64_t used = 0; /* at most 64 colours (27 suffice for hexahedra) */
        for (int a = 0; a < nen; ++a) {
            int64_t v = P->conn[a * n_el + e];
            for (int64_t k = inc_ptr[v]; k < inc_ptr[v + 1]; ++k) {
                int32_t c = color[inc[k]];
                if (c >= 0) used |= (uint64_t)1 << c;
            }
        }
        int c = 0;
        while (c < 64 && ((used >> c) & 1)) ++c;
        if (c == 64) { free(inc_ptr); free(inc); free(fill); return -1; }
        color[e] = c;
        if (c + 1 > n_colors) n_colors = c + 1;
    }
    free(inc_ptr); free(inc); free(fill);
    return n_colors;
}

/*
 * or_assemble without constraints, on n_threads OpenMP threads: the elements of one
 * colour at a time, each element computed and scattered exactly as in or_assemble.
 * Within a colour no two elements share a row, so the adds need no synchronisation;
 * the sums differ from the sequential ones only in the order of the (at most 8)
 * element contributions to an entry.  Returns the status as or_assemble; *threads_used
 * receives the number of threads that ran.
 */
int or_assemble_colored(void* h, int kind, const double* params, const double* coords,
                        const double* elem_param, const double* nodal_src, const double* state,
                        int qpa, int n_threads, double* K, double* d, int64_t* bad_elem,
                        int* threads_used)
{
    const or_pattern* P = (const or_pattern*)h;
    int dim = P->dim, nen = P->nen, nf = form_nf(kind, dim), ne = nen * nf;
    int64_t nn = P->n_nodes, n_el = P->n_el;
    if (nf != P->nf || n_threads < 1) return OR_ERR_ARG;
    or_params prm = {params[0], params[1], params[2], params[3], params[4], params[5]};
    int nsrc = (kind == OR_ELASTICITY) ? dim : 1;
    int32_t* color = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_el + 1));
    if (!color) return OR_ERR_OOM;
    int n_colors = color_elements(P, color);
    if (n_colors < 0) { free(color); return OR_ERR_OOM; }
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_el + 1));
    int64_t* cptr = (int64_t*)calloc((size_t)n_colors + 1, sizeof(int64_t));
    if (!order || !cptr) { free(color); free(order); free(cptr); return OR_ERR_OOM; }
    for (int64_t e = 0; e < n_el; ++e) ++cptr[color[e] + 1];
    for (int c = 0; c < n_colors; ++c) cptr[c + 1] += cptr[c];
    {
        int64_t* at = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_colors + 1));
        if (!at) { free(color); free(order); free(cptr); return OR_ERR_OOM; }
        memcpy(at, cptr, sizeof(int64_t) * (size_t)n_colors);
        for (int64_t e = 0; e < n_el; ++e) order[at[color[e]]++] = e;
        free(at);
    }
    free(color);
    if (K) memset(K, 0, sizeof(double) * (size_t)P->nnz);
    memset(d, 0, sizeof(double) * (size_t)P->n_rows);
    *bad_elem = -1;
    int status = OR_OK;
    int used = 1;
    for (int c = 0; c < n_colors && status == OR_OK; ++c) {
        int64_t c0 = cptr[c], c1 = cptr[c + 1];
#pragma omp parallel num_threads(n_threads)
        {
#pragma omp single
            used = omp_get_num_threads();
            double* Ke = (double*)malloc(sizeof(double) * ne * ne);
            int st = Ke ? OR_OK : OR_ERR_OOM;
            int64_t bad = -1;
#pragma omp for schedule(static)
            for (int64_t k = c0; k < c1; ++k) {
                if (st != OR_OK) continue;
                int64_t e = order[k];
                double x[OR_MAXNEN][OR_MAXDIM], U[OR_MAXNEN * OR_MAXNF], src[OR_MAXNEN * OR_MAXDIM];
                double Re[OR_MAXNEN * OR_MAXNF];
                int64_t node[OR_MAXNEN];
                for (int a = 0; a < nen; ++a) {
                    node[a] = P->conn[a * n_el + e];
                    for (int m = 0; m < dim; ++m) x[a][m] = coords[m * nn + node[a]];
                    for (int i = 0; i < nf; ++i) U[a * nf + i] = state ? state[i * nn + node[a]] : 0.0;
                    for (int s2 = 0; s2 < nsrc; ++s2)
                        src[a * nsrc + s2] = nodal_src ? nodal_src[s2 * nn + node[a]] : 0.0;
                }
                double cp = elem_param ? elem_param[e] : 1.0;
                int rc = element(kind, dim, &prm, cp, x, U, nodal_src ? src : NULL, qpa, Re, Ke, K != NULL);
                if (rc) {
                    st = rc;
                    if (rc == OR_ERR_BAD_JACOBIAN && (bad < 0 || e < bad)) bad = e;
                    continue;
                }
                for (int a = 0; a < nen; ++a)
                    for (int i = 0; i < nf; ++i) {
                        int64_t r = dof_of(P, node[a], i);
                        d[r] -= Re[a * nf + i];
                        if (!K) continue;
                        for (int b = 0; b < nen; ++b)
                            for (int j = 0; j < nf; ++j) {
                                int64_t pos = find_col(P, r, dof_of(P, node[b], j));
                                if (pos >= 0) K[pos] += Ke[(a * nf + i) * ne + b * nf + j];
                            }
                    }
            }
            free(Ke);
            if (st != OR_OK) {
#pragma omp critical
                {
                    status = st;
                    if (bad >= 0 && (*bad_elem < 0 || bad < *bad_elem)) *bad_elem = bad;
                }
            }
        }
    }
    free(order);
    free(cptr);
    *threads_used = used;
    return status;
}

/* Residual R(U) of a form (no constraints), [n_rows]; the Newton tangent K is dR/dU. */
int or_residual(void* h, int kind, const double* params, const double* coords,
                const double* elem_param, const double* nodal_src, const double* state,
                int qpa, double* R, int64_t* bad_elem)
{
    const or_pattern* P = (const or_pattern*)h;
    int rc = or_assemble(h, kind, params, coords, elem_param, nodal_src, state, NULL, qpa,
                         NULL, R, bad_elem);
    for (int64_t r = 0; r < P->n_rows; ++r) R[r] = -R[r];
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Solver of D-4 (the paper leaves it open): Jacobi-preconditioned CG          */
/* ------------------------------------------------------------------------- */

/* y = A x for CSR (row_ptr64, col_idx, val) */
static void csr_mv(int64_t n, const int64_t* rp, const int32_t* ci, const double* v,
                   const double* x, double* y)
{
    for (int64_t r = 0; r < n; ++r) {
        double s = 0.0;
        for (int64_t k = rp[r]; k < rp[r + 1]; ++k) s += v[k] * x[ci[k]];
        y[r] = s;
    }
}

static double dot(int64_t n, const double* a, const double* b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/*
 * Preconditioned CG with z = diag(A)^-1 r, x0 = 0, stopping when the TRUE residual
 * |b - A x|_2 / |b|_2 <= tol (checked whenever the recurrence residual says so).
 * Returns the iteration count, or -1 when maxit is reached.
 */
int64_t or_pcg_jacobi(int64_t n, const int64_t* rp, const int32_t* ci, const double* v,
                      const double* b, double tol, int64_t maxit, double* x, double* relres)
{
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n),
           *p = malloc(sizeof(double) * n), *Ap = malloc(sizeof(double) * n),
           *dinv = malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; ++i) {
        double di = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] == i) di = v[k];
        dinv[i] = 1.0 / di;
        x[i] = 0.0;
        r[i] = b[i];
    }
    double bn = sqrt(dot(n, b, b));
    int64_t it = 0, result = -1;
    if (bn == 0.0) { *relres = 0.0; result = 0; goto done; }
    for (int64_t i = 0; i < n; ++i) { z[i] = dinv[i] * r[i]; p[i] = z[i]; }
    double rz = dot(n, r, z);
    for (it = 1; it <= maxit; ++it) {
        csr_mv(n, rp, ci, v, p, Ap);
        double alpha = rz / dot(n, p, Ap);
        for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * Ap[i]; }
        double rn = sqrt(dot(n, r, r));
        if (rn / bn <= tol) {
            /* true residual as judge */
            csr_mv(n, rp, ci, v, x, Ap);
            double s = 0.0;
            for (int64_t i = 0; i < n; ++i) { double t = b[i] - Ap[i]; s += t * t; }
            *relres = sqrt(s) / bn;
            if (*relres <= tol) { result = it; break; }
            for (int64_t i = 0; i < n; ++i) r[i] = b[i] - Ap[i];
        }
        for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
        double rz1 = dot(n, r, z);
        double beta = rz1 / rz;
        rz = rz1;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    if (result < 0) {
        csr_mv(n, rp, ci, v, x, Ap);
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) { double t = b[i] - Ap[i]; s += t * t; }
        *relres = sqrt(s) / bn;
    }
done:
    free(r); free(z); free(p); free(Ap); free(dinv);
    return result;
}
