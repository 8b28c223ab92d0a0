/*
 * fe_oracle.c -- plain, slow, FP64 reference implementation of the finite
 * element pipeline: Galerkin element matrices for the Poisson and isotropic
 * linear-elasticity bilinear forms on Lagrangian Q_k quadrilaterals and
 * hexahedra, strong Dirichlet elimination, CSR storage of the free-free
 * system, and a Jacobi-preconditioned conjugate-gradient solve.
 *
 * THIS FILE IS TEST INFRASTRUCTURE (the "oracle").  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant generator with the HIP library;
 * it is written directly from the definitions in the FEMPAR paper
 * (Badia, Martin, Principe, arXiv 1708.01773) and from textbook methods,
 * each function naming the passage it follows.  Single-threaded, no
 * blocking, fusion or reordering beyond what the definitions state.
 *
 * Conventions (the readings of the paper this oracle takes):
 *  - Reference cell [0,1]^d (Sect. 3.14, the polytope coordinates; Sect. 3.15
 *    equidistant nodes x_i = i/k).
 *  - Local node numbering lexicographic with x fastest:
 *    a = a0 + (k+1) a1 + (k+1)^2 a2 (Sect. 3.15 / Sect. 6 node numbering).
 *  - Vertex v of a cell = v0 + 2 v1 + 4 v2 with v_r in {0,1} (Sect. 3.14).
 *  - Geometry: the order-1 (bi/trilinear) map built from the 2^d vertices for
 *    every k (the geometry FE order is left open in Sect. 7.1).
 *  - Jacobian J_rs = d Phi_r / d xi_s; physical gradients are J^{-T} times
 *    the reference gradient (Sect. 3.7, eq. shape_grad, read in column form).
 *  - Quadrature: tensor Gauss-Legendre with k+1 points per direction
 *    (Sect. 3.7 and the footnote of Sect. 8.1).
 *  - Vector fields: Cartesian product of scalar spaces (Sect. 3.8), local
 *    DOF index ncomp*a + c, global DOF ncomp*node_rank + c.
 *  - Elasticity form (not printed in the paper): a(u,v) = int 2 mu eps(u):eps(v)
 *    + lambda div u div v.
 *  - Dirichlet: strong elimination of fixed DOFs with lifting into the
 *    right-hand side (Sect. 10.4, eq. dirichlet_bc_discrete_problem).  Free
 *    DOFs are ranked lexicographically over the global node lattice; fixed
 *    DOFs are encoded as -1 - fixed_rank.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXK 4
#define ORC_MAXQ1 16 /* max Gauss points per direction */

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rule on [0,1] (Sect. 3.7: tensor Gauss-Legendre rule,     */
/* exact to degree 2n-1).  Textbook construction: the nodes are the roots   */
/* of the Legendre polynomial P_n, located by Newton's method on the        */
/* three-term recurrence (m+1) P_{m+1} = (2m+1) t P_m - m P_{m-1}; on       */
/* [-1,1] the weight of root t is 2 / ((1 - t^2) P_n'(t)^2).  The rule is   */
/* then mapped affinely to [0,1] (weights halve, so they sum to 1).         */
/* Nodes are returned in ascending order.                                   */
/* ------------------------------------------------------------------------ */
int orc_gauss_legendre(int n, double *x, double *w)
{
    if (n < 1 || n > ORC_MAXQ1) return -1;
    for (int i = 0; i < n; i++) {
        /* initial guess: Chebyshev-like approximation of the i-th largest root */
        double t = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; it++) {
            double p_prev = 1.0, p = t;       /* P_0, P_1 */
            if (n == 1) { p_prev = 1.0; p = t; }
            for (int m = 1; m < n; m++) {
                double p_next = ((2.0 * m + 1.0) * t * p - m * p_prev) / (m + 1.0);
                p_prev = p;
                p = p_next;
            }
            /* p = P_n(t), p_prev = P_{n-1}(t);  P_n' = n (t P_n - P_{n-1}) / (t^2 - 1) */
            dp = n * (t * p - p_prev) / (t * t - 1.0);
            double dt = p / dp;
            t -= dt;
            if (fabs(dt) < 1e-17) break;
        }
        /* recompute the derivative at the converged root */
        {
            double p_prev = 1.0, p = t;
            for (int m = 1; m < n; m++) {
                double p_next = ((2.0 * m + 1.0) * t * p - m * p_prev) / (m + 1.0);
                p_prev = p;
                p = p_next;
            }
            dp = n * (t * p - p_prev) / (t * t - 1.0);
        }
        x[n - 1 - i] = 0.5 * (t + 1.0);
        w[n - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp); /* = (1/2) * 2/((1-t^2) P'^2) */
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 1D Lagrange basis of order k on the equidistant nodes xi_s = s/k          */
/* (Sect. 3.4, eq. lagbas; Sect. 3.15 equidistant nodes):                    */
/*   l_m(x) = prod_{s != m} (x - xi_s) / (xi_m - xi_s),                      */
/* and its derivative by the product rule.                                   */
/* ------------------------------------------------------------------------ */
void orc_lagrange_1d(int k, double x, double *val, double *der)
{
    for (int m = 0; m <= k; m++) {
        double xm = (double)m / k;
        double den = 1.0, num = 1.0;
        for (int s = 0; s <= k; s++) {
            if (s == m) continue;
            double xs = (double)s / k;
            den *= (xm - xs);
            num *= (x - xs);
        }
        double dnum = 0.0;
        for (int j = 0; j <= k; j++) {
            if (j == m) continue;
            double prod = 1.0;
            for (int s = 0; s <= k; s++) {
                if (s == m || s == j) continue;
                prod *= (x - (double)s / k);
            }
            dnum += prod;
        }
        val[m] = num / den;
        der[m] = dnum / den;
    }
}

/* ------------------------------------------------------------------------ */
/* Order-1 geometrical map of a cell (Sect. 3.2 map Phi_K, Sect. 8.3         */
/* cell_map): Phi(xi) = sum_v X_v N_v(xi), N_v(xi) = prod_r (v_r ? xi_r :    */
/* 1 - xi_r).  Returns Phi(xi) and J_rs = dPhi_r/dxi_s (row-major J[r*d+s]).  */
/* ------------------------------------------------------------------------ */
static void orc_geometry(int dim, const double *X, const double *xi, double *phys, double *J)
{
    int nv = 1 << dim;
    for (int r = 0; r < dim; r++) {
        phys[r] = 0.0;
        for (int s = 0; s < dim; s++) J[r * dim + s] = 0.0;
    }
    for (int v = 0; v < nv; v++) {
        double N = 1.0;
        double dN[3];
        for (int r = 0; r < dim; r++) {
            int vr = (v >> r) & 1;
            N *= vr ? xi[r] : 1.0 - xi[r];
        }
        for (int s = 0; s < dim; s++) {
            double g = 1.0;
            for (int r = 0; r < dim; r++) {
                int vr = (v >> r) & 1;
                if (r == s) g *= vr ? 1.0 : -1.0;
                else g *= vr ? xi[r] : 1.0 - xi[r];
            }
            dN[s] = g;
        }
        for (int r = 0; r < dim; r++) {
            phys[r] += X[v * dim + r] * N;
            for (int s = 0; s < dim; s++) J[r * dim + s] += X[v * dim + r] * dN[s];
        }
    }
}

/* determinant and inverse of a 2x2 or 3x3 matrix by cofactors */
static double orc_det_inv(int dim, const double *J, double *Ji)
{
    if (dim == 2) {
        double det = J[0] * J[3] - J[1] * J[2];
        Ji[0] = J[3] / det;
        Ji[1] = -J[1] / det;
        Ji[2] = -J[2] / det;
        Ji[3] = J[0] / det;
        return det;
    }
    double c00 = J[4] * J[8] - J[5] * J[7];
    double c01 = J[5] * J[6] - J[3] * J[8];
    double c02 = J[3] * J[7] - J[4] * J[6];
    double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
    Ji[0] = c00 / det;
    Ji[1] = (J[2] * J[7] - J[1] * J[8]) / det;
    Ji[2] = (J[1] * J[5] - J[2] * J[4]) / det;
    Ji[3] = c01 / det;
    Ji[4] = (J[0] * J[8] - J[2] * J[6]) / det;
    Ji[5] = (J[2] * J[3] - J[0] * J[5]) / det;
    Ji[6] = c02 / det;
    Ji[7] = (J[1] * J[6] - J[0] * J[7]) / det;
    Ji[8] = (J[0] * J[4] - J[1] * J[3]) / det;
    return det;
}

/* Evaluation data of one quadrature point: reference shape values, physical
 * gradients (Sect. 3.7, eqs. shfunx and shape_grad), w |det J| and the
 * physical point. */
typedef struct {
    double wdet;
    double detJ;
    double x[3];
} orc_qp;

static int ipow(int b, int e)
{
    int r = 1;
    for (int i = 0; i < e; i++) r *= b;
    return r;
}

/* Shape values phi[a] and physical gradients grad[a*dim+i] at reference point
 * xi for tensor-product Lagrange basis of order k (Sect. 3.4 eq. lagbasmd). */
static int orc_shape_at(int dim, int k, const double *X, const double *xi,
                        double *phi, double *grad, orc_qp *qp)
{
    double L[3][ORC_MAXK + 1], D[3][ORC_MAXK + 1];
    for (int r = 0; r < dim; r++) orc_lagrange_1d(k, xi[r], L[r], D[r]);
    double J[9], Ji[9];
    orc_geometry(dim, X, xi, qp->x, J);
    double det = orc_det_inv(dim, J, Ji);
    qp->detJ = det;
    int nn = ipow(k + 1, dim);
    for (int a = 0; a < nn; a++) {
        int ar[3] = {a % (k + 1), (a / (k + 1)) % (k + 1), a / ((k + 1) * (k + 1))};
        double gref[3];
        double val = 1.0;
        for (int r = 0; r < dim; r++) val *= L[r][ar[r]];
        for (int s = 0; s < dim; s++) {
            double g = 1.0;
            for (int r = 0; r < dim; r++) g *= (r == s) ? D[r][ar[r]] : L[r][ar[r]];
            gref[s] = g;
        }
        phi[a] = val;
        /* (grad phi_a)_i = sum_s (J^{-1})_{s i} dphi_a/dxi_s */
        for (int i = 0; i < dim; i++) {
            double g = 0.0;
            for (int s = 0; s < dim; s++) g += Ji[s * dim + i] * gref[s];
            grad[a * dim + i] = g;
        }
    }
    return det > 0.0 ? 0 : -1;
}

/* ------------------------------------------------------------------------ */
/* Element matrix (Sect. 3.7 eq. fematrix; the Poisson example of Sect. 8.5; */
/* cell-wise split of eq. assembly in Sect. 3.6).                            */
/*  problem 0 (Poisson):  A_ab = sum_q w_q coef |det J_q| grad phi_a . grad phi_b */
/*  problem 1 (elasticity, d = 3 or 2, ncomp = d):                           */
/*   A_(a,i),(b,j) = sum_q w_q |det J_q| [ lambda d_i phi_a d_j phi_b +       */
/*                   mu (delta_ij grad phi_a . grad phi_b + d_j phi_a d_i phi_b) ] */
/*   (coef multiplies both Lame parameters).                                 */
/* A is row-major nloc x nloc, nloc = nn * ncomp, local DOF = ncomp*a + c.   */
/* Returns -1 if det J <= 0 at some quadrature point.                        */
/* ------------------------------------------------------------------------ */
int orc_element_matrix(int dim, int k, int problem, const double *X, double coef,
                       double lambda, double mu, double *A)
{
    if (dim < 2 || dim > 3 || k < 1 || k > ORC_MAXK) return -2;
    int nq1 = k + 1;
    double gx[ORC_MAXQ1], gw[ORC_MAXQ1];
    orc_gauss_legendre(nq1, gx, gw);
    int nn = ipow(k + 1, dim);
    int ncomp = (problem == 1) ? dim : 1;
    int nloc = nn * ncomp;
    double *phi = (double *)malloc(sizeof(double) * nn);
    double *grad = (double *)malloc(sizeof(double) * nn * dim);
    memset(A, 0, sizeof(double) * nloc * nloc);
    int nq = ipow(nq1, dim);
    int bad = 0;
    for (int q = 0; q < nq; q++) {
        int qr[3] = {q % nq1, (q / nq1) % nq1, q / (nq1 * nq1)};
        double xi[3], w = 1.0;
        for (int r = 0; r < dim; r++) {
            xi[r] = gx[qr[r]];
            w *= gw[qr[r]];
        }
        orc_qp qp;
        if (orc_shape_at(dim, k, X, xi, phi, grad, &qp) != 0) bad = 1;
        double wd = w * fabs(qp.detJ) * coef;
        for (int a = 0; a < nn; a++) {
            for (int b = 0; b < nn; b++) {
                double dot = 0.0;
                for (int i = 0; i < dim; i++) dot += grad[a * dim + i] * grad[b * dim + i];
                if (problem == 0) {
                    A[a * nloc + b] += wd * dot;
                } else {
                    for (int i = 0; i < dim; i++) {
                        for (int j = 0; j < dim; j++) {
                            double v = lambda * grad[a * dim + i] * grad[b * dim + j]
                                     + mu * grad[a * dim + j] * grad[b * dim + i];
                            if (i == j) v += mu * dot;
                            A[(a * ncomp + i) * nloc + (b * ncomp + j)] += wd * v;
                        }
                    }
                }
            }
        }
    }
    free(phi);
    free(grad);
    return bad ? -1 : 0;
}

/* Body force f evaluated at physical point x for component c.
 *  kind 0: none; kind 1: constant vector src[c];
 *  kind 2: src[c] * d * pi^2 * prod_r sin(pi x_r) (the manufactured load of
 *          u = prod_r sin(pi x_r) for -Laplace u = f). */
static double orc_source(int kind, const double *src, int dim, const double *x, int c)
{
    if (kind == 1) return src[c];
    if (kind == 2) {
        double p = 1.0;
        for (int r = 0; r < dim; r++) p *= sin(M_PI * x[r]);
        return src[c] * dim * M_PI * M_PI * p;
    }
    return 0.0;
}

/* Element load vector f_(a,c) = sum_q w_q |det J_q| f_c(Phi(xi_q)) phi_a(xi_q)
 * (Sect. 3.6 eq. linear_system right-hand side, integrated as eq. fematrix). */
int orc_element_load(int dim, int k, int ncomp, const double *X, int source_kind,
                     const double *source, double *f)
{
    int nq1 = k + 1;
    double gx[ORC_MAXQ1], gw[ORC_MAXQ1];
    orc_gauss_legendre(nq1, gx, gw);
    int nn = ipow(k + 1, dim);
    double *phi = (double *)malloc(sizeof(double) * nn);
    double *grad = (double *)malloc(sizeof(double) * nn * dim);
    memset(f, 0, sizeof(double) * nn * ncomp);
    int nq = ipow(nq1, dim);
    int bad = 0;
    for (int q = 0; q < nq; q++) {
        int qr[3] = {q % nq1, (q / nq1) % nq1, q / (nq1 * nq1)};
        double xi[3], w = 1.0;
        for (int r = 0; r < dim; r++) {
            xi[r] = gx[qr[r]];
            w *= gw[qr[r]];
        }
        orc_qp qp;
        if (orc_shape_at(dim, k, X, xi, phi, grad, &qp) != 0) bad = 1;
        double wd = w * fabs(qp.detJ);
        for (int c = 0; c < ncomp; c++) {
            double fc = orc_source(source_kind, source, dim, qp.x, c);
            for (int a = 0; a < nn; a++) f[a * ncomp + c] += wd * fc * phi[a];
        }
    }
    free(phi);
    free(grad);
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Mesh access: structured brick of n0 x n1 (x n2) cells (Sect. 7.4, the     */
/* structured generator), vertices numbered lexicographically x fastest,     */
/* vertex coordinates given (AoS, dim per vertex).                           */
/* ------------------------------------------------------------------------ */
void orc_cell_vertices(int dim, const int *n, const double *vxyz, int64_t cell, double *X)
{
    int64_t c = cell;
    int64_t ci[3] = {0, 0, 0};
    ci[0] = c % n[0];
    c /= n[0];
    ci[1] = c % n[1];
    c /= n[1];
    if (dim == 3) ci[2] = c;
    int64_t nv0 = n[0] + 1, nv1 = n[1] + 1;
    for (int v = 0; v < (1 << dim); v++) {
        int64_t vi[3];
        for (int r = 0; r < 3; r++) vi[r] = ci[r] + ((v >> r) & 1);
        if (dim == 2) vi[2] = 0;
        int64_t vid = vi[0] + nv0 * (vi[1] + nv1 * vi[2]);
        for (int r = 0; r < dim; r++) X[v * dim + r] = vxyz[vid * dim + r];
    }
}

/* ------------------------------------------------------------------------ */
/* DOF numbering (reading of Sect. 10.3 / 10.4): every node of the global     */
/* lattice (n_r k + 1 per axis, lexicographic, x fastest) is fixed if it lies */
/* on a Dirichlet face (bit 2r: x_r = 0, bit 2r+1: x_r = 1), else free.      */
/* Free and fixed nodes are ranked separately in lexicographic order.        */
/* node_code[node] = free rank (>= 0) or -1 - fixed rank.                    */
/* ------------------------------------------------------------------------ */
void orc_number_nodes(int dim, const int *n, int k, unsigned faces, int64_t *node_code,
                      int64_t *nfree_out, int64_t *nfixed_out)
{
    int64_t N[3] = {1, 1, 1};
    for (int r = 0; r < dim; r++) N[r] = (int64_t)n[r] * k + 1;
    int64_t nfree = 0, nfixed = 0;
    int64_t id = 0;
    for (int64_t I2 = 0; I2 < N[2]; I2++)
        for (int64_t I1 = 0; I1 < N[1]; I1++)
            for (int64_t I0 = 0; I0 < N[0]; I0++, id++) {
                int64_t I[3] = {I0, I1, I2};
                int fixed = 0;
                for (int r = 0; r < dim; r++) {
                    if (I[r] == 0 && (faces >> (2 * r) & 1u)) fixed = 1;
                    if (I[r] == N[r] - 1 && (faces >> (2 * r + 1) & 1u)) fixed = 1;
                }
                node_code[id] = fixed ? -1 - nfixed++ : nfree++;
            }
    *nfree_out = nfree;
    *nfixed_out = nfixed;
}

/* Global node id of local node a of a cell (local lexicographic numbering). */
static int64_t orc_local_to_global_node(int dim, const int *n, int k, int64_t cell, int a)
{
    int64_t c = cell;
    int64_t ci[3] = {0, 0, 0};
    ci[0] = c % n[0];
    c /= n[0];
    ci[1] = c % n[1];
    c /= n[1];
    if (dim == 3) ci[2] = c;
    int ar[3] = {a % (k + 1), (a / (k + 1)) % (k + 1), a / ((k + 1) * (k + 1))};
    int64_t N0 = (int64_t)n[0] * k + 1, N1 = (int64_t)n[1] * k + 1;
    int64_t I[3] = {0, 0, 0};
    for (int r = 0; r < dim; r++) I[r] = ci[r] * k + ar[r];
    return I[0] + N0 * (I[1] + N1 * I[2]);
}

/* Local-to-global DOF map (Sect. 10.1 lst_dofs_gids, Sect. 3.6 equivalence
 * of local DOFs at coinciding nodes): cell_dofs[cell*nloc + ncomp*a + c] =
 * ncomp*free_rank + c, or -1 - (ncomp*fixed_rank + c) for fixed DOFs. */
void orc_cell_dofs(int dim, const int *n, int k, int ncomp, const int64_t *node_code,
                   int64_t ncells, int64_t *cell_dofs)
{
    int nn = ipow(k + 1, dim);
    int nloc = nn * ncomp;
    for (int64_t K = 0; K < ncells; K++)
        for (int a = 0; a < nn; a++) {
            int64_t code = node_code[orc_local_to_global_node(dim, n, k, K, a)];
            for (int c = 0; c < ncomp; c++) {
                int64_t g = code >= 0 ? ncomp * code + c : -1 - (ncomp * (-1 - code) + c);
                cell_dofs[K * nloc + a * ncomp + c] = g;
            }
        }
}

/* Physical position of local node a of a cell: Phi_K(a/k) (nodes of a
 * high-order cell are images of the reference lattice, Sect. 3.15). */
static void orc_node_position(int dim, int k, const double *X, int a, double *x)
{
    int ar[3] = {a % (k + 1), (a / (k + 1)) % (k + 1), a / ((k + 1) * (k + 1))};
    double xi[3] = {0, 0, 0}, J[9];
    for (int r = 0; r < dim; r++) xi[r] = (double)ar[r] / k;
    orc_geometry(dim, X, xi, x, J);
}

/* Dirichlet datum u_D,c(x) = aff[4c] + sum_r aff[4c+1+r] x_r (kind 1), else 0. */
static double orc_dirichlet_value(int kind, const double *aff, int dim, const double *x, int c)
{
    if (kind != 1) return 0.0;
    double v = aff[4 * c];
    for (int r = 0; r < dim; r++) v += aff[4 * c + 1 + r] * x[r];
    return v;
}

/* ------------------------------------------------------------------------ */
/* Symbolic CSR pattern of the free-free system (Sect. 11.1: COO build-up,   */
/* then compression where duplicates merge).  Every pair (row, col) of free  */
/* DOFs that share a cell is an entry (structural zeros are kept).  Plain    */
/* way: collect all pairs, sort, drop duplicates.                            */
/* rowptr has nfree+1 entries; *colind_out is malloc'ed (caller frees with   */
/* orc_free).                                                                */
/* ------------------------------------------------------------------------ */
static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

int64_t orc_csr_pattern(int64_t ncells, int nloc, const int64_t *cell_dofs, int64_t nfree,
                        int64_t *rowptr, int32_t **colind_out)
{
    int64_t npairs = 0;
    for (int64_t K = 0; K < ncells; K++) {
        int64_t f = 0;
        for (int a = 0; a < nloc; a++) f += cell_dofs[K * nloc + a] >= 0;
        npairs += f * f;
    }
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (npairs > 0 ? npairs : 1));
    int64_t p = 0;
    for (int64_t K = 0; K < ncells; K++)
        for (int a = 0; a < nloc; a++) {
            int64_t ga = cell_dofs[K * nloc + a];
            if (ga < 0) continue;
            for (int b = 0; b < nloc; b++) {
                int64_t gb = cell_dofs[K * nloc + b];
                if (gb < 0) continue;
                key[p++] = ga * nfree + gb;
            }
        }
    qsort(key, (size_t)npairs, sizeof(int64_t), cmp_i64);
    int64_t nnz = 0;
    for (int64_t i = 0; i < npairs; i++)
        if (i == 0 || key[i] != key[i - 1]) key[nnz++] = key[i];
    int32_t *colind = (int32_t *)malloc(sizeof(int32_t) * (nnz > 0 ? nnz : 1));
    for (int64_t r = 0; r <= nfree; r++) rowptr[r] = 0;
    for (int64_t i = 0; i < nnz; i++) {
        rowptr[key[i] / nfree + 1]++;
        colind[i] = (int32_t)(key[i] % nfree);
    }
    for (int64_t r = 0; r < nfree; r++) rowptr[r + 1] += rowptr[r];
    free(key);
    *colind_out = colind;
    return nnz;
}

void orc_free(void *p) { free(p); }

/* position of column col in the sorted column list of a row (binary search) */
static int64_t orc_find(const int64_t *rowptr, const int32_t *colind, int64_t row, int64_t col)
{
    int64_t lo = rowptr[row], hi = rowptr[row + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (colind[mid] == col) return mid;
        if (colind[mid] < col) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

/* Problem description shared by the assembly routines. */
typedef struct {
    int dim;
    int n[3];
    int k;
    int problem;          /* 0 Poisson, 1 elasticity */
    double lambda, mu;    /* elasticity Lame parameters */
    int source_kind;
    double source[3];
    int dirichlet_kind;   /* 0 zero, 1 affine */
    double dirichlet_affine[12];
} orc_problem;

/* ------------------------------------------------------------------------ */
/* Numeric assembly with strong Dirichlet elimination (Sect. 3.6 eq.         */
/* assembly; Sect. 10.4 eq. dirichlet_bc_discrete_problem): for each cell in */
/* ascending order, for each local row a (free), for each local column b:    */
/*   b free  -> A[g_a, g_b] += A^K_ab                                        */
/*   b fixed -> rhs[g_a]   -= A^K_ab * u_D(b)                                */
/* and rhs[g_a] += f^K_a.  Rows of fixed DOFs are not assembled.             */
/* values must have nnz entries, rhs nfree entries (both are overwritten).   */
/* Returns -1 if some cell has det J <= 0 at a quadrature point.             */
/* ------------------------------------------------------------------------ */
int orc_assemble(const orc_problem *P, const double *vxyz, const double *coef,
                 const int64_t *cell_dofs, int64_t nfree, const int64_t *rowptr,
                 const int32_t *colind, double *values, double *rhs)
{
    int dim = P->dim, k = P->k;
    int ncomp = P->problem == 1 ? dim : 1;
    int nn = ipow(k + 1, dim);
    int nloc = nn * ncomp;
    int64_t ncells = (int64_t)P->n[0] * P->n[1] * (dim == 3 ? P->n[2] : 1);
    double *A = (double *)malloc(sizeof(double) * nloc * nloc);
    double *f = (double *)malloc(sizeof(double) * nloc);
    double *uD = (double *)malloc(sizeof(double) * nloc);
    double X[24];
    memset(values, 0, sizeof(double) * rowptr[nfree]);
    memset(rhs, 0, sizeof(double) * nfree);
    int bad = 0;
    for (int64_t K = 0; K < ncells; K++) {
        orc_cell_vertices(dim, P->n, vxyz, K, X);
        double kc = coef ? coef[K] : 1.0;
        if (orc_element_matrix(dim, k, P->problem, X, kc, P->lambda, P->mu, A) != 0) bad = 1;
        orc_element_load(dim, k, ncomp, X, P->source_kind, P->source, f);
        for (int a = 0; a < nn; a++) {
            double x[3];
            orc_node_position(dim, k, X, a, x);
            for (int c = 0; c < ncomp; c++)
                uD[a * ncomp + c] = orc_dirichlet_value(P->dirichlet_kind, P->dirichlet_affine, dim, x, c);
        }
        const int64_t *g = cell_dofs + K * nloc;
        for (int a = 0; a < nloc; a++) {
            if (g[a] < 0) continue;
            for (int b = 0; b < nloc; b++) {
                if (g[b] >= 0) values[orc_find(rowptr, colind, g[a], g[b])] += A[a * nloc + b];
                else rhs[g[a]] -= A[a * nloc + b] * uD[b];
            }
            rhs[g[a]] += f[a];
        }
    }
    free(A);
    free(f);
    free(uD);
    return bad ? -1 : 0;
}

/* One row of the assembled system computed on its own: scan every cell, and
 * for each cell that holds the free DOF `row`, add that cell's contributions
 * (same rules as orc_assemble).  Columns are returned sorted ascending.
 * Returns the row length, or -1 if more than maxlen columns. */
int64_t orc_assemble_row(const orc_problem *P, const double *vxyz, const double *coef,
                         const int64_t *cell_dofs, int64_t row, int64_t maxlen,
                         int64_t *cols, double *vals, double *rhs_out)
{
    int dim = P->dim, k = P->k;
    int ncomp = P->problem == 1 ? dim : 1;
    int nn = ipow(k + 1, dim);
    int nloc = nn * ncomp;
    int64_t ncells = (int64_t)P->n[0] * P->n[1] * (dim == 3 ? P->n[2] : 1);
    double *A = (double *)malloc(sizeof(double) * nloc * nloc);
    double *f = (double *)malloc(sizeof(double) * nloc);
    double X[24];
    int64_t len = 0;
    double rhs = 0.0;
    for (int64_t K = 0; K < ncells; K++) {
        const int64_t *g = cell_dofs + K * nloc;
        int a = -1;
        for (int t = 0; t < nloc; t++)
            if (g[t] == row) a = t;
        if (a < 0) continue;
        orc_cell_vertices(dim, P->n, vxyz, K, X);
        double kc = coef ? coef[K] : 1.0;
        orc_element_matrix(dim, k, P->problem, X, kc, P->lambda, P->mu, A);
        orc_element_load(dim, k, ncomp, X, P->source_kind, P->source, f);
        rhs += f[a];
        for (int b = 0; b < nloc; b++) {
            if (g[b] < 0) {
                int node = b / ncomp, c = b % ncomp;
                double x[3];
                orc_node_position(dim, k, X, node, x);
                rhs -= A[a * nloc + b] * orc_dirichlet_value(P->dirichlet_kind, P->dirichlet_affine, dim, x, c);
                continue;
            }
            /* insert into the sorted column list */
            int64_t pos = 0;
            while (pos < len && cols[pos] < g[b]) pos++;
            if (pos < len && cols[pos] == g[b]) {
                vals[pos] += A[a * nloc + b];
            } else {
                if (len >= maxlen) {
                    free(A);
                    free(f);
                    return -1;
                }
                for (int64_t t = len; t > pos; t--) {
                    cols[t] = cols[t - 1];
                    vals[t] = vals[t - 1];
                }
                cols[pos] = g[b];
                vals[pos] = A[a * nloc + b];
                len++;
            }
        }
    }
    *rhs_out = rhs;
    free(A);
    free(f);
    return len;
}

/* ------------------------------------------------------------------------ */
/* CSR matrix-vector product y = A x (plain row loop).                       */
/* ------------------------------------------------------------------------ */
void orc_spmv(int64_t n, const int64_t *rowptr, const int32_t *colind, const double *val,
              const double *x, double *y)
{
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t j = rowptr[i]; j < rowptr[i + 1]; j++) s += val[j] * x[colind[j]];
        y[i] = s;
    }
}

static double orc_dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

/* ------------------------------------------------------------------------ */
/* Jacobi-preconditioned conjugate gradients (textbook PCG, Saad, Iterative   */
/* Methods for Sparse Linear Systems, Alg. 9.1, with M = diag(A)).  The       */
/* paper names CG among its iterative solvers (Sect. 12).  x holds x0 on      */
/* entry.  Stops when ||r_j||_2 <= rtol ||b||_2 (recursively updated r).      */
/* alphas/betas (length >= maxit, may be NULL) receive the CG coefficients    */
/* for Lanczos eigenvalue estimates.  Returns 0 if converged, 1 if maxit was  */
/* reached, 2 on breakdown (p.Ap <= 0 or not finite).                         */
/* ------------------------------------------------------------------------ */
int orc_pcg(int64_t n, const int64_t *rowptr, const int32_t *colind, const double *val,
            const double *b, double *x, double rtol, int maxit, int *iters_out,
            double *relres_out, double *alphas, double *betas)
{
    double *r = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *q = (double *)malloc(sizeof(double) * n);
    double *dinv = (double *)malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; i++) {
        double d = 0.0;
        for (int64_t j = rowptr[i]; j < rowptr[i + 1]; j++)
            if (colind[j] == i) d = val[j];
        dinv[i] = 1.0 / d;
    }
    orc_spmv(n, rowptr, colind, val, x, q);
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - q[i];
    double bnorm = sqrt(orc_dot(n, b, b));
    for (int64_t i = 0; i < n; i++) z[i] = dinv[i] * r[i];
    for (int64_t i = 0; i < n; i++) p[i] = z[i];
    double rho = orc_dot(n, r, z);
    double rnorm = sqrt(orc_dot(n, r, r));
    int it = 0, status = 1;
    if (rnorm <= rtol * bnorm) status = 0;
    while (status == 1 && it < maxit) {
        orc_spmv(n, rowptr, colind, val, p, q);
        double pq = orc_dot(n, p, q);
        if (!(pq > 0.0) || !isfinite(pq)) {
            status = 2;
            break;
        }
        double alpha = rho / pq;
        for (int64_t i = 0; i < n; i++) x[i] += alpha * p[i];
        for (int64_t i = 0; i < n; i++) r[i] -= alpha * q[i];
        for (int64_t i = 0; i < n; i++) z[i] = dinv[i] * r[i];
        double rho_new = orc_dot(n, r, z);
        double beta = rho_new / rho;
        rho = rho_new;
        for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
        if (alphas) alphas[it] = alpha;
        if (betas) betas[it] = beta;
        it++;
        rnorm = sqrt(orc_dot(n, r, r));
        if (rnorm <= rtol * bnorm) status = 0;
    }
    *iters_out = it;
    *relres_out = bnorm > 0 ? rnorm / bnorm : rnorm;
    free(r);
    free(z);
    free(p);
    free(q);
    free(dinv);
    return status;
}

/* ------------------------------------------------------------------------ */
/* L2 error ||u - u_h|| of a discrete solution (Sect. 10.6 FE functions:      */
/* u_h restricted to a cell is sum_a u_a phi_a with free values from x and   */
/* fixed values from u_D).  Integrated with kq Gauss points per direction.   */
/* exact kind 1: u_c = exact[c] * prod_r sin(pi x_r); kind 2: affine with    */
/* exact[12] laid out like the Dirichlet datum.                              */
/* ------------------------------------------------------------------------ */
double orc_l2_error(const orc_problem *P, const double *vxyz, const int64_t *cell_dofs,
                    const double *xfree, int kq, int exact_kind, const double *exact)
{
    int dim = P->dim, k = P->k;
    int ncomp = P->problem == 1 ? dim : 1;
    int nn = ipow(k + 1, dim);
    int nloc = nn * ncomp;
    int64_t ncells = (int64_t)P->n[0] * P->n[1] * (dim == 3 ? P->n[2] : 1);
    double gx[ORC_MAXQ1], gw[ORC_MAXQ1];
    orc_gauss_legendre(kq, gx, gw);
    double *phi = (double *)malloc(sizeof(double) * nn);
    double *grad = (double *)malloc(sizeof(double) * nn * dim);
    double *uloc = (double *)malloc(sizeof(double) * nloc);
    double X[24];
    double err2 = 0.0;
    int nq = ipow(kq, dim);
    for (int64_t K = 0; K < ncells; K++) {
        orc_cell_vertices(dim, P->n, vxyz, K, X);
        const int64_t *g = cell_dofs + K * nloc;
        for (int a = 0; a < nn; a++) {
            double x[3];
            orc_node_position(dim, k, X, a, x);
            for (int c = 0; c < ncomp; c++) {
                int64_t gd = g[a * ncomp + c];
                uloc[a * ncomp + c] = gd >= 0 ? xfree[gd]
                    : orc_dirichlet_value(P->dirichlet_kind, P->dirichlet_affine, dim, x, c);
            }
        }
        for (int q = 0; q < nq; q++) {
            int qr[3] = {q % kq, (q / kq) % kq, q / (kq * kq)};
            double xi[3], w = 1.0;
            for (int r = 0; r < dim; r++) {
                xi[r] = gx[qr[r]];
                w *= gw[qr[r]];
            }
            orc_qp qp;
            orc_shape_at(dim, k, X, xi, phi, grad, &qp);
            for (int c = 0; c < ncomp; c++) {
                double uh = 0.0;
                for (int a = 0; a < nn; a++) uh += uloc[a * ncomp + c] * phi[a];
                double ue;
                if (exact_kind == 1) {
                    ue = exact[c];
                    for (int r = 0; r < dim; r++) ue *= sin(M_PI * qp.x[r]);
                } else {
                    ue = orc_dirichlet_value(1, exact, dim, qp.x, c);
                }
                err2 += w * fabs(qp.detJ) * (ue - uh) * (ue - uh);
            }
        }
    }
    free(phi);
    free(grad);
    free(uloc);
    return sqrt(err2);
}

/* Values of the Dirichlet datum at every fixed DOF, indexed by fixed rank
 * (used to reconstruct full nodal fields in tests). */
void orc_fixed_values(const orc_problem *P, const double *vxyz, const int64_t *cell_dofs,
                      int64_t nfixed_dofs, double *ufixed)
{
    int dim = P->dim, k = P->k;
    int ncomp = P->problem == 1 ? dim : 1;
    int nn = ipow(k + 1, dim);
    int nloc = nn * ncomp;
    int64_t ncells = (int64_t)P->n[0] * P->n[1] * (dim == 3 ? P->n[2] : 1);
    double X[24];
    for (int64_t i = 0; i < nfixed_dofs; i++) ufixed[i] = 0.0;
    for (int64_t K = 0; K < ncells; K++) {
        orc_cell_vertices(dim, P->n, vxyz, K, X);
        const int64_t *g = cell_dofs + K * nloc;
        for (int a = 0; a < nn; a++) {
            double x[3];
            orc_node_position(dim, k, X, a, x);
            for (int c = 0; c < ncomp; c++) {
                int64_t gd = g[a * ncomp + c];
                if (gd < 0)
                    ufixed[-1 - gd] = orc_dirichlet_value(P->dirichlet_kind, P->dirichlet_affine, dim, x, c);
            }
        }
    }
}

/* ======================================================================== */
/* Interior-penalty discontinuous Galerkin for -Laplace(u) = f (Sect. 3.12,  */
/* eq. ip_dg_formulations; the facet matrices of eq. local_to_face_matrix).  */
/* ======================================================================== */
/* Readings: tau = 1 (the symmetric member of the family; then the two ways  */
/* of placing the jump and the mean in the printed facet matrix coincide);   */
/* the penalty |F|^-1 read as h_F^-1 with h_F = |F|^(1/(d-1)) (the facet      */
/* length in 2D, as printed; its square root in 3D, so the penalty scales    */
/* like 1/h in every dimension); coefficient 1; Dirichlet data imposed       */
/* weakly on every boundary facet.  No DOF is shared: DOF(K, a) = K nn + a.  */
/* Facet quadrature: Gauss-Legendre with k+1 points per tangential direction */
/* on the reference face, mapped by the cell's order-1 geometry from either  */
/* side (the brick's neighbouring faces coincide point by point).            */

/* Cells that share the facet of cell K on side (r, +): K + stride(r), if any */
static int64_t orc_dg_neighbour(const int *n, int dim, int64_t K, int r, int side)
{
    int64_t ci[3] = {K % n[0], (K / n[0]) % n[1], dim == 3 ? K / ((int64_t)n[0] * n[1]) : 0};
    int64_t st[3] = {1, n[0], (int64_t)n[0] * n[1]};
    int64_t c = ci[r] + (side ? 1 : -1);
    if (c < 0 || c >= n[r]) return -1;
    return K + (side ? st[r] : -st[r]);
}

/* Pattern: row K nn + a has the columns of K and of its facet neighbours,  */
/* ascending.  rowptr has nn ncells + 1 entries; *colind_out malloc'ed.     */
int64_t orc_dg_pattern(const orc_problem *P, int64_t *rowptr, int32_t **colind_out)
{
    int dim = P->dim, k = P->k;
    int nn = ipow(k + 1, dim);
    int64_t ncells = (int64_t)P->n[0] * P->n[1] * (dim == 3 ? P->n[2] : 1);
    int64_t nnz = 0;
    rowptr[0] = 0;
    int64_t *cells = (int64_t *)malloc(sizeof(int64_t) * 8);
    for (int64_t K = 0; K < ncells; K++) {
        int nc = 0;
        cells[nc++] = K;
        for (int r = 0; r < dim; r++)
            for (int side = 0; side < 2; side++) {
                int64_t L = orc_dg_neighbour(P->n, dim, K, r, side);
                if (L >= 0) cells[nc++] = L;
            }
        for (int a = 0; a < nn; a++) rowptr[K * nn + a + 1] = rowptr[K * nn + a] + (int64_t)nc * nn;
        nnz += (int64_t)nc * nn * nn;
    }
    int32_t *colind = (int32_t *)malloc(sizeof(int32_t) * (nnz > 0 ? nnz : 1));
    for (int64_t K = 0; K < ncells; K++) {
        int nc = 0;
        cells[nc++] = K;
        for (int r = 0; r < dim; r++)
            for (int side = 0; side < 2; side++) {
                int64_t L = orc_dg_neighbour(P->n, dim, K, r, side);
                if (L >= 0) cells[nc++] = L;
            }
        qsort(cells, (size_t)nc, sizeof(int64_t), cmp_i64);
        for (int a = 0; a < nn; a++) {
            int64_t p = rowptr[K * nn + a];
            for (int c = 0; c < nc; c++)
                for (int b = 0; b < nn; b++) colind[p++] = (int32_t)(cells[c] * nn + b);
        }
    }
    free(cells);
    *colind_out = colind;
    return nnz;
}

/* One side of a facet at reference point xi of cell X: shape values,       */
/* physical gradients, the physical point, and the area-weighted normal     */
/* det(J) J^-T e_r (outward for the face xi_r = 1, inward for xi_r = 0).    */
static int orc_face_side(int dim, int k, const double *X, const double *xi, int r, double *phi, double *grad,
                         double *x, double *nvec)
{
    orc_qp qp;
    int bad = orc_shape_at(dim, k, X, xi, phi, grad, &qp);
    double J[9], Ji[9], tmp[3];
    orc_geometry(dim, X, xi, tmp, J);
    double det = orc_det_inv(dim, J, Ji);
    for (int i = 0; i < dim; i++) {
        x[i] = qp.x[i];
        nvec[i] = det * Ji[r * dim + i];
    }
    return bad;
}

static double orc_dot_d(int dim, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < dim; i++) s += a[i] * b[i];
    return s;
}

/* Adds v to the entry (row, col) of the DG system. */
static void orc_dg_add(const int64_t *rowptr, const int32_t *colind, double *values, int64_t row, int64_t col,
                       double v)
{
    values[orc_find(rowptr, colind, row, col)] += v;
}

/* The facet of cell K on side (r, side) with the tensor rule of k+1 points  */
/* per tangential direction: for every point, the reference coordinates on   */
/* K (xi_r = side) and on the neighbour (xi_r = 1 - side), and the weight.   */
static int orc_face_points(int dim, int k, int r, int side, double (*xiK)[3], double (*xiL)[3], double *wq)
{
    double gx[ORC_MAXQ1], gw[ORC_MAXQ1];
    orc_gauss_legendre(k + 1, gx, gw);
    int tang[2], nt = 0;
    for (int s = 0; s < dim; s++)
        if (s != r) tang[nt++] = s;
    int np = dim == 3 ? (k + 1) * (k + 1) : k + 1;
    for (int q = 0; q < np; q++) {
        int q0 = q % (k + 1), q1 = q / (k + 1);
        for (int s = 0; s < 3; s++) xiK[q][s] = xiL[q][s] = 0.0;
        xiK[q][tang[0]] = xiL[q][tang[0]] = gx[q0];
        wq[q] = gw[q0];
        if (nt == 2) {
            xiK[q][tang[1]] = xiL[q][tang[1]] = gx[q1];
            wq[q] *= gw[q1];
        }
        xiK[q][r] = side ? 1.0 : 0.0;
        xiL[q][r] = side ? 0.0 : 1.0;
    }
    return np;
}

/* DG system of -Laplace(u) = f with weak Dirichlet data on the whole        */
/* boundary (values and rhs overwritten).  Volume terms: the Poisson element */
/* matrix with coefficient 1 and the load of the problem.  Interior facet    */
/* between K- (this cell) and K+ = its neighbour on side (r, +), unit normal */
/* n outward of K-, sigma = gamma / h_F; with s(K-) = +1, s(K+) = -1 the    */
/* jump of phi from side i is s_i phi n and the mean of grad phi is half of  */
/* it, so test row a of side i, trial column b of side j get                 */
/*   sum_q W_q [ -s_i phi_a (n.grad phi_b)/2 - tau s_j phi_b (n.grad phi_a)/2 */
/*               + sigma s_i s_j phi_a phi_b ].                              */
/* Boundary facet of K with outward unit normal n:                           */
/*   A_ab += sum W [ -phi_a n.grad phi_b - tau phi_b n.grad phi_a + sigma phi_a phi_b ] */
/*   rhs_a += sum W [ -tau u_D n.grad phi_a + sigma u_D phi_a ].             */
/* Order: cells ascending (volume), then every cell's interior facets on    */
/* its + sides (axis ascending), then the boundary facets (cell ascending,  */
/* face 2r + side).  Returns -1 if a det J <= 0 was met.                     */
int orc_dg_assemble(const orc_problem *P, const double *vxyz, double gamma, double tau, const int64_t *rowptr,
                    const int32_t *colind, double *values, double *rhs)
{
    int dim = P->dim, k = P->k;
    int nn = ipow(k + 1, dim);
    int64_t ncells = (int64_t)P->n[0] * P->n[1] * (dim == 3 ? P->n[2] : 1);
    int64_t nrows = ncells * nn;
    double *A = (double *)malloc(sizeof(double) * nn * nn);
    double *f = (double *)malloc(sizeof(double) * nn);
    double *phiK = (double *)malloc(sizeof(double) * nn), *phiL = (double *)malloc(sizeof(double) * nn);
    double *gK = (double *)malloc(sizeof(double) * nn * dim), *gL = (double *)malloc(sizeof(double) * nn * dim);
    double (*xiK)[3] = malloc(sizeof(double[3]) * ORC_MAXQ1 * ORC_MAXQ1);
    double (*xiL)[3] = malloc(sizeof(double[3]) * ORC_MAXQ1 * ORC_MAXQ1);
    double *wq = (double *)malloc(sizeof(double) * ORC_MAXQ1 * ORC_MAXQ1);
    double X[24], XL[24];
    int bad = 0;
    memset(values, 0, sizeof(double) * rowptr[nrows]);
    memset(rhs, 0, sizeof(double) * nrows);
    for (int64_t K = 0; K < ncells; K++) {
        orc_cell_vertices(dim, P->n, vxyz, K, X);
        if (orc_element_matrix(dim, k, 0, X, 1.0, 0.0, 0.0, A) != 0) bad = 1;
        orc_element_load(dim, k, 1, X, P->source_kind, P->source, f);
        for (int a = 0; a < nn; a++) {
            for (int b = 0; b < nn; b++) orc_dg_add(rowptr, colind, values, K * nn + a, K * nn + b, A[a * nn + b]);
            rhs[K * nn + a] += f[a];
        }
    }
    /* interior facets */
    for (int64_t K = 0; K < ncells; K++)
        for (int r = 0; r < dim; r++) {
            int64_t L = orc_dg_neighbour(P->n, dim, K, r, 1);
            if (L < 0) continue;
            orc_cell_vertices(dim, P->n, vxyz, K, X);
            orc_cell_vertices(dim, P->n, vxyz, L, XL);
            int np = orc_face_points(dim, k, r, 1, xiK, xiL, wq);
            double area = 0.0;
            for (int q = 0; q < np; q++) {
                double x[3], nv[3];
                orc_face_side(dim, k, X, xiK[q], r, phiK, gK, x, nv);
                area += wq[q] * sqrt(orc_dot_d(dim, nv, nv));
            }
            double hF = dim == 3 ? sqrt(area) : area;
            double sigma = gamma / hF;
            for (int q = 0; q < np; q++) {
                double xK[3], xL[3], nvK[3], nvL[3];
                if (orc_face_side(dim, k, X, xiK[q], r, phiK, gK, xK, nvK)) bad = 1;
                if (orc_face_side(dim, k, XL, xiL[q], r, phiL, gL, xL, nvL)) bad = 1;
                double dS = sqrt(orc_dot_d(dim, nvK, nvK));
                double n[3] = {0, 0, 0};
                for (int i = 0; i < dim; i++) n[i] = nvK[i] / dS;
                double W = wq[q] * dS;
                /* sides: 0 = K (s = +1), 1 = L (s = -1) */
                const double *ph[2] = {phiK, phiL}, *gr[2] = {gK, gL};
                int64_t base[2] = {K * nn, L * nn};
                double sg[2] = {1.0, -1.0};
                for (int i = 0; i < 2; i++)
                    for (int j = 0; j < 2; j++)
                        for (int a = 0; a < nn; a++) {
                            double dna = orc_dot_d(dim, n, gr[i] + a * dim);
                            for (int b = 0; b < nn; b++) {
                                double dnb = orc_dot_d(dim, n, gr[j] + b * dim);
                                double v = -sg[i] * ph[i][a] * dnb * 0.5 - tau * sg[j] * ph[j][b] * dna * 0.5 +
                                           sigma * sg[i] * sg[j] * ph[i][a] * ph[j][b];
                                orc_dg_add(rowptr, colind, values, base[i] + a, base[j] + b, W * v);
                            }
                        }
            }
        }
    /* boundary facets */
    for (int64_t K = 0; K < ncells; K++)
        for (int r = 0; r < dim; r++)
            for (int side = 0; side < 2; side++) {
                if (orc_dg_neighbour(P->n, dim, K, r, side) >= 0) continue;
                orc_cell_vertices(dim, P->n, vxyz, K, X);
                int np = orc_face_points(dim, k, r, side, xiK, xiL, wq);
                double area = 0.0;
                for (int q = 0; q < np; q++) {
                    double x[3], nv[3];
                    orc_face_side(dim, k, X, xiK[q], r, phiK, gK, x, nv);
                    area += wq[q] * sqrt(orc_dot_d(dim, nv, nv));
                }
                double hF = dim == 3 ? sqrt(area) : area;
                double sigma = gamma / hF;
                for (int q = 0; q < np; q++) {
                    double x[3], nv[3];
                    if (orc_face_side(dim, k, X, xiK[q], r, phiK, gK, x, nv)) bad = 1;
                    double dS = sqrt(orc_dot_d(dim, nv, nv));
                    double n[3] = {0, 0, 0};
                    for (int i = 0; i < dim; i++) n[i] = (side ? 1.0 : -1.0) * nv[i] / dS;  /* outward */
                    double W = wq[q] * dS;
                    double uD = orc_dirichlet_value(P->dirichlet_kind, P->dirichlet_affine, dim, x, 0);
                    for (int a = 0; a < nn; a++) {
                        double dna = orc_dot_d(dim, n, gK + a * dim);
                        for (int b = 0; b < nn; b++) {
                            double dnb = orc_dot_d(dim, n, gK + b * dim);
                            double v = -phiK[a] * dnb - tau * phiK[b] * dna + sigma * phiK[a] * phiK[b];
                            orc_dg_add(rowptr, colind, values, K * nn + a, K * nn + b, W * v);
                        }
                        rhs[K * nn + a] += W * (-tau * uD * dna + sigma * uD * phiK[a]);
                    }
                }
            }
    free(A);
    free(f);
    free(phiK);
    free(phiL);
    free(gK);
    free(gL);
    free(xiK);
    free(xiL);
    free(wq);
    return bad ? -1 : 0;
}

/* ======================================================================== */
/* Taylor-Hood Stokes (the Stokes example of Sect. 3.1; Q_{k+1}^d x Q_k, the */
/* mixed pair of Sect. 3.8).  Readings: viscous term mu eps(u):eps(v), which  */
/* is the elasticity element matrix of orc_element_matrix with lambda = 0    */
/* and its mu set to mu / 2; the continuity equation multiplied by -1, so     */
/* that the system [[A, B^T], [B, 0]] is symmetric (same solution), with      */
/* b(v, q) = - int q div v.                                                  */
/* ======================================================================== */
/* Divergence block of one cell: B[a * nlu + dim * b + c] =                  */
/*   - sum_q w_q |det J_q| psi_a(q) d_c phi_b(q)                             */
/* for the (k+1)^d pressure nodes a (order k) and the (k+2)^d velocity nodes */
/* b (order k+1), nlu = dim (k+2)^d, on the velocity order's Gauss rule      */
/* ((k+2)^d points: exact for psi d_c phi on affine cells).  Also            */
/* md[a] = sum_q w_q |det J_q| psi_a(q)^2, the pressure mass diagonal.       */
/* Returns -1 if det J <= 0 at a quadrature point, -2 for a bad order.       */
int orc_stokes_b_element(int dim, int k, const double *X, double *B, double *md)
{
    int ku = k + 1, nq1 = ku + 1;
    if (dim < 2 || dim > 3 || k < 1 || ku > ORC_MAXK) return -2;
    int nnp = ipow(k + 1, dim), nnu = ipow(ku + 1, dim), nlu = nnu * dim;
    double gx[ORC_MAXQ1], gw[ORC_MAXQ1];
    orc_gauss_legendre(nq1, gx, gw);
    double *phiu = (double *)malloc(sizeof(double) * nnu), *gu = (double *)malloc(sizeof(double) * nnu * dim);
    double *psi = (double *)malloc(sizeof(double) * nnp), *gp = (double *)malloc(sizeof(double) * nnp * dim);
    memset(B, 0, sizeof(double) * (size_t)nnp * nlu);
    memset(md, 0, sizeof(double) * (size_t)nnp);
    int nq = ipow(nq1, dim), bad = 0;
    for (int q = 0; q < nq; q++) {
        int qi[3] = {q % nq1, (q / nq1) % nq1, q / (nq1 * nq1)};
        double xi[3] = {0, 0, 0}, w = 1.0;
        for (int r = 0; r < dim; r++) {
            xi[r] = gx[qi[r]];
            w *= gw[qi[r]];
        }
        orc_qp qu, qpp;
        if (orc_shape_at(dim, ku, X, xi, phiu, gu, &qu)) bad = 1;
        orc_shape_at(dim, k, X, xi, psi, gp, &qpp);
        double wd = w * fabs(qu.detJ);
        for (int a = 0; a < nnp; a++) {
            md[a] += wd * psi[a] * psi[a];
            for (int b = 0; b < nnu; b++)
                for (int c = 0; c < dim; c++) B[a * nlu + dim * b + c] -= wd * psi[a] * gu[b * dim + c];
        }
    }
    free(phiu);
    free(gu);
    free(psi);
    free(gp);
    return bad ? -1 : 0;
}

/* Lagrangian P_k on simplicial meshes (same oracle, same translation unit). */
#include "fe_oracle_simplex.c"
