/*
 * fe_oracle_simplex.c -- the oracle's Lagrangian P_k elements on simplices
 * (triangles, tetrahedra) over a general simplicial mesh given by vertex
 * coordinates and cell-to-vertex connectivity.
 *
 * THIS FILE IS TEST INFRASTRUCTURE (part of the oracle; compiled into the
 * same library by inclusion at the end of fe_oracle.c, whose Gauss-Legendre
 * rule, 3x3 inverse, load function, Dirichlet datum, CSR pattern and
 * binary search it uses).  Plain, slow, FP64.
 *
 * What it follows:
 *  - Reference simplex {xi_r >= 0, sum_r xi_r <= 1}, vertex 0 at the origin
 *    and vertex r at the unit vector e_r (Sect. 3.14: simplices as polytopes).
 *  - Local space P_k: polynomials of total degree <= k (Sect. 3.3, the
 *    truncated space); nodes the points s/k of the lattice N^{k1} with
 *    |s| <= k (the truncated node set of Sect. 3.3), taken in the order of
 *    the n-cube lattice (x fastest) with the points of |s| > k skipped.
 *  - Shape functions by the change of basis of Sect. 3.5: pre-basis the
 *    monomials xi^alpha, |alpha| <= k (Sect. 3.8 / 6: the truncated tensor
 *    product of 1D monomials), in the same multi-index order;
 *    C_ab = sigma_a(psi_b) = psi_b(x_a) and Phi^T = C^{-1}, so
 *    phi_a = sum_b (C^{-1})_{ba} psi_b.
 *  - Quadrature (Sect. 3.7): a tensor Gauss-Legendre rule with
 *    n = k + ceil(d/2) points per direction on [0,1]^d, carried onto the
 *    simplex by the collapsed (Duffy) transformation
 *      xi_0 = u_0, xi_1 = (1 - u_0) u_1, xi_2 = (1 - u_0)(1 - u_1) u_2,
 *    whose Jacobian (1 - u_0)^{d-1} (1 - u_1)^{d-2} multiplies the weights.
 *  - Geometry: the affine map x = v_0 + sum_r (v_r - v_0) xi_r of the cell's
 *    d+1 vertices in the order the connectivity gives (J_rs = v_{s+1,r} -
 *    v_{0,r}); |det J| in the integrals, det J = 0 an error.
 *  - Global nodes (Sect. 3.6: local DOFs at the same node are one global
 *    DOF; Sect. 10.3 numbering by a sweep over the cells): local node s of
 *    cell K sits at barycentric weights (k - |s|, s_0, .., s_{d-1}) / k on
 *    the cell's vertices; two local nodes are one global node when their sets
 *    {(vertex, weight) : weight > 0} are equal.  Global node ids in order of
 *    first appearance over (cell ascending, local node ascending).
 *  - Boundary: a facet (d vertices) that belongs to one cell only; every node
 *    of a boundary facet is fixed when Dirichlet data are imposed.  Free and
 *    fixed nodes ranked separately in global node order; cell_dofs as in the
 *    brick oracle (ncomp*rank + c, fixed -1 - (ncomp*fixed_rank + c)).
 *  - Forms, loads, lifting and the assembly order as in the brick oracle.
 */

#define ORC_SX_MAXK 4
#define ORC_SX_MAXNN 35 /* (k+1)(k+2)(k+3)/6 at k = 4 */

/* Local nodes of P_k on the d-simplex: s[3a + r] = s_r of node a.
 * Returns the number of nodes. */
int orc_sx_nodes(int dim, int k, int *s)
{
    int nn = 0;
    int top2 = dim == 3 ? k : 0;
    for (int s2 = 0; s2 <= top2; s2++)
        for (int s1 = 0; s1 <= k; s1++)
            for (int s0 = 0; s0 <= k; s0++)
                if (s0 + s1 + s2 <= k) {
                    s[3 * nn] = s0;
                    s[3 * nn + 1] = s1;
                    s[3 * nn + 2] = s2;
                    nn++;
                }
    return nn;
}

static double sx_pow(double x, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; i++) r *= x;
    return r;
}

/* Inverse of an n x n matrix by Gauss-Jordan elimination with partial
 * pivoting (textbook).  Returns -1 if the matrix is singular. */
static int sx_invert(int n, const double *A, double *Ainv)
{
    double M[ORC_SX_MAXNN][2 * ORC_SX_MAXNN];
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            M[i][j] = A[i * n + j];
            M[i][n + j] = i == j ? 1.0 : 0.0;
        }
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int i = c + 1; i < n; i++)
            if (fabs(M[i][c]) > fabs(M[p][c])) p = i;
        if (M[p][c] == 0.0) return -1;
        if (p != c)
            for (int j = 0; j < 2 * n; j++) {
                double t = M[c][j];
                M[c][j] = M[p][j];
                M[p][j] = t;
            }
        double piv = M[c][c];
        for (int j = 0; j < 2 * n; j++) M[c][j] /= piv;
        for (int i = 0; i < n; i++) {
            if (i == c) continue;
            double f = M[i][c];
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * n; j++) M[i][j] -= f * M[c][j];
        }
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) Ainv[i * n + j] = M[i][n + j];
    return 0;
}

/* The change of basis of Sect. 3.5: Phi[a*nn + b], phi_a = sum_b Phi_ab psi_b
 * with psi_b = xi^(alpha_b).  Returns nn, or -1. */
int orc_sx_basis(int dim, int k, double *Phi)
{
    if (dim < 2 || dim > 3 || k < 1 || k > ORC_SX_MAXK) return -1;
    int s[3 * ORC_SX_MAXNN];
    int nn = orc_sx_nodes(dim, k, s);
    double C[ORC_SX_MAXNN * ORC_SX_MAXNN], Ci[ORC_SX_MAXNN * ORC_SX_MAXNN];
    for (int a = 0; a < nn; a++)
        for (int b = 0; b < nn; b++) {
            /* sigma_a(psi_b): the monomial b at node a, x_a = s_a / k */
            double v = 1.0;
            for (int r = 0; r < dim; r++) v *= sx_pow((double)s[3 * a + r] / k, s[3 * b + r]);
            C[a * nn + b] = v;
        }
    if (sx_invert(nn, C, Ci) != 0) return -1;
    for (int a = 0; a < nn; a++)
        for (int b = 0; b < nn; b++) Phi[a * nn + b] = Ci[b * nn + a];
    return nn;
}

/* Reference shape values phi[a] and reference gradients dphi[a*dim + r] at
 * xi, from the monomials and the change-of-basis matrix. */
static void sx_shape_ref(int dim, int nn, const int *s, const double *Phi, const double *xi, double *phi,
                         double *dphi)
{
    double psi[ORC_SX_MAXNN], dpsi[ORC_SX_MAXNN * 3];
    for (int b = 0; b < nn; b++) {
        double v = 1.0;
        for (int r = 0; r < dim; r++) v *= sx_pow(xi[r], s[3 * b + r]);
        psi[b] = v;
        for (int r = 0; r < dim; r++) {
            int e = s[3 * b + r];
            double g = e == 0 ? 0.0 : e * sx_pow(xi[r], e - 1);
            for (int t = 0; t < dim; t++)
                if (t != r) g *= sx_pow(xi[t], s[3 * b + t]);
            dpsi[b * 3 + r] = g;
        }
    }
    for (int a = 0; a < nn; a++) {
        double v = 0.0, g[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < nn; b++) {
            v += Phi[a * nn + b] * psi[b];
            for (int r = 0; r < dim; r++) g[r] += Phi[a * nn + b] * dpsi[b * 3 + r];
        }
        phi[a] = v;
        for (int r = 0; r < dim; r++) dphi[a * dim + r] = g[r];
    }
}

/* Shape values at xi on the reference simplex (for tests). */
int orc_sx_shape(int dim, int k, const double *xi, double *phi, double *dphi)
{
    double Phi[ORC_SX_MAXNN * ORC_SX_MAXNN];
    int s[3 * ORC_SX_MAXNN];
    int nn = orc_sx_basis(dim, k, Phi);
    if (nn < 0) return -1;
    orc_sx_nodes(dim, k, s);
    sx_shape_ref(dim, nn, s, Phi, xi, phi, dphi);
    return nn;
}

/* Collapsed Gauss rule on the reference simplex: n^dim points, u_0 fastest.
 * xi[3q + r], w[q].  Returns the number of points. */
int orc_sx_quadrature(int dim, int n, double *xi, double *w)
{
    double gx[ORC_MAXQ1], gw[ORC_MAXQ1];
    if (n < 1 || n > ORC_MAXQ1) return -1;
    orc_gauss_legendre(n, gx, gw);
    int nq = ipow(n, dim);
    for (int q = 0; q < nq; q++) {
        int i0 = q % n, i1 = (q / n) % n, i2 = q / (n * n);
        double u0 = gx[i0], u1 = gx[i1];
        xi[3 * q] = u0;
        xi[3 * q + 1] = (1.0 - u0) * u1;
        xi[3 * q + 2] = 0.0;
        double jac = 1.0 - u0, wq = gw[i0] * gw[i1];
        if (dim == 3) {
            double u2 = gx[i2];
            xi[3 * q + 2] = (1.0 - u0) * (1.0 - u1) * u2;
            jac = (1.0 - u0) * (1.0 - u0) * (1.0 - u1);
            wq *= gw[i2];
        }
        w[q] = wq * jac;
    }
    return nq;
}

/* number of Gauss points per direction: k + ceil(d/2) */
static int sx_rule_points(int dim, int k) { return k + (dim + 1) / 2; }

/* Affine geometry of a cell: J[r*dim + s] = X_{s+1,r} - X_{0,r}. */
static double sx_jacobian(int dim, const double *X, double *J, double *Ji)
{
    for (int r = 0; r < dim; r++)
        for (int s = 0; s < dim; s++) J[r * dim + s] = X[(s + 1) * dim + r] - X[r];
    return orc_det_inv(dim, J, Ji);
}

/* Element matrix of the Poisson (problem 0) or elasticity (problem 1) form
 * on a simplex (the integrals of the brick oracle's orc_element_matrix, on
 * the collapsed rule).  X: (dim+1) x dim vertex coordinates.  A row-major
 * nloc x nloc.  Returns -1 if det J = 0. */
int orc_sx_element_matrix(int dim, int k, int problem, const double *X, double coef, double lambda, double mu,
                          double *A)
{
    double Phi[ORC_SX_MAXNN * ORC_SX_MAXNN];
    int s[3 * ORC_SX_MAXNN];
    int nn = orc_sx_basis(dim, k, Phi);
    if (nn < 0) return -2;
    orc_sx_nodes(dim, k, s);
    int ncomp = problem == 1 ? dim : 1, nloc = nn * ncomp;
    int n = sx_rule_points(dim, k);
    int nq = ipow(n, dim);
    double *qx = (double *)malloc(sizeof(double) * 3 * nq), *qw = (double *)malloc(sizeof(double) * nq);
    orc_sx_quadrature(dim, n, qx, qw);
    double J[9], Ji[9];
    double det = sx_jacobian(dim, X, J, Ji);
    memset(A, 0, sizeof(double) * nloc * nloc);
    double phi[ORC_SX_MAXNN], dref[ORC_SX_MAXNN * 3], grad[ORC_SX_MAXNN * 3];
    for (int q = 0; q < nq; q++) {
        sx_shape_ref(dim, nn, s, Phi, qx + 3 * q, phi, dref);
        /* physical gradient (grad phi_a)_i = sum_r (J^-1)_{r i} d phi_a / d xi_r */
        for (int a = 0; a < nn; a++)
            for (int i = 0; i < dim; i++) {
                double g = 0.0;
                for (int r = 0; r < dim; r++) g += Ji[r * dim + i] * dref[a * dim + r];
                grad[a * dim + i] = g;
            }
        double wd = qw[q] * fabs(det) * coef;
        for (int a = 0; a < nn; a++)
            for (int b = 0; b < nn; b++) {
                double dot = 0.0;
                for (int i = 0; i < dim; i++) dot += grad[a * dim + i] * grad[b * dim + i];
                if (problem == 0) {
                    A[a * nloc + b] += wd * dot;
                } else {
                    for (int i = 0; i < dim; i++)
                        for (int j = 0; j < dim; j++) {
                            double v = lambda * grad[a * dim + i] * grad[b * dim + j] +
                                       mu * grad[a * dim + j] * grad[b * dim + i];
                            if (i == j) v += mu * dot;
                            A[(a * ncomp + i) * nloc + (b * ncomp + j)] += wd * v;
                        }
                }
            }
    }
    free(qx);
    free(qw);
    return det == 0.0 ? -1 : 0;
}

/* Element load f_(a,c) = sum_q w_q |det J| f_c(x(xi_q)) phi_a(xi_q). */
int orc_sx_element_load(int dim, int k, int ncomp, const double *X, int source_kind, const double *source, double *f)
{
    double Phi[ORC_SX_MAXNN * ORC_SX_MAXNN];
    int s[3 * ORC_SX_MAXNN];
    int nn = orc_sx_basis(dim, k, Phi);
    if (nn < 0) return -2;
    orc_sx_nodes(dim, k, s);
    int n = sx_rule_points(dim, k);
    int nq = ipow(n, dim);
    double *qx = (double *)malloc(sizeof(double) * 3 * nq), *qw = (double *)malloc(sizeof(double) * nq);
    orc_sx_quadrature(dim, n, qx, qw);
    double J[9], Ji[9];
    double det = sx_jacobian(dim, X, J, Ji);
    memset(f, 0, sizeof(double) * nn * ncomp);
    double phi[ORC_SX_MAXNN], dref[ORC_SX_MAXNN * 3];
    for (int q = 0; q < nq; q++) {
        sx_shape_ref(dim, nn, s, Phi, qx + 3 * q, phi, dref);
        double x[3] = {0.0, 0.0, 0.0};
        for (int r = 0; r < dim; r++) {
            x[r] = X[r];
            for (int t = 0; t < dim; t++) x[r] += J[r * dim + t] * qx[3 * q + t];
        }
        double wd = qw[q] * fabs(det);
        for (int c = 0; c < ncomp; c++) {
            double fc = orc_source(source_kind, source, dim, x, c);
            for (int a = 0; a < nn; a++) f[a * ncomp + c] += phi[a] * fc * wd;
        }
    }
    free(qx);
    free(qw);
    return det == 0.0 ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Global numbering                                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t v[4]; /* support vertices, ascending; unused slots INT32_MAX */
    int32_t w[4]; /* their barycentric weights (times k) */
    int64_t cell;
    int32_t a;
} sx_occ;

static int sx_occ_cmp(const void *pa, const void *pb)
{
    const sx_occ *x = (const sx_occ *)pa, *y = (const sx_occ *)pb;
    for (int i = 0; i < 4; i++) {
        if (x->v[i] != y->v[i]) return x->v[i] < y->v[i] ? -1 : 1;
        if (x->w[i] != y->w[i]) return x->w[i] < y->w[i] ? -1 : 1;
    }
    if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
    return (x->a > y->a) - (x->a < y->a);
}

typedef struct {
    int64_t first; /* cell * nn + a of the first appearance */
    int64_t group; /* index of the group's first sorted record */
} sx_first;

static int sx_first_cmp(const void *pa, const void *pb)
{
    const sx_first *x = (const sx_first *)pa, *y = (const sx_first *)pb;
    return (x->first > y->first) - (x->first < y->first);
}

typedef struct {
    int32_t v[3]; /* facet vertices, ascending */
    int64_t cell;
    int32_t j; /* local vertex opposite the facet */
} sx_facet;

static int sx_facet_cmp(const void *pa, const void *pb)
{
    const sx_facet *x = (const sx_facet *)pa, *y = (const sx_facet *)pb;
    for (int i = 0; i < 3; i++)
        if (x->v[i] != y->v[i]) return x->v[i] < y->v[i] ? -1 : 1;
    if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
    return (x->j > y->j) - (x->j < y->j);
}

static void sx_sort_small(int32_t *v, int32_t *w, int m)
{
    for (int i = 1; i < m; i++)
        for (int j = i; j > 0 && v[j - 1] > v[j]; j--) {
            int32_t t = v[j];
            v[j] = v[j - 1];
            v[j - 1] = t;
            if (w) {
                t = w[j];
                w[j] = w[j - 1];
                w[j - 1] = t;
            }
        }
}

/* Numbering of the nodes of P_k on a simplicial mesh.
 *  node_of[K*nn + a]  global node id of local node a of cell K
 *  node_code[node]    free rank, or -1 - fixed rank (array of >= ncells*nn)
 * dirichlet != 0 fixes every node on a boundary facet.
 * Returns 0, -1 on bad input, -2 if a facet is shared by more than two cells. */
int orc_sx_number(int dim, int k, int64_t nverts, int64_t ncells, const int32_t *cells, int dirichlet,
                  int64_t *node_of, int64_t *node_code, int64_t *nnodes_out, int64_t *nfree_out, int64_t *nfixed_out)
{
    if (dim < 2 || dim > 3 || k < 1 || k > ORC_SX_MAXK) return -1;
    int s[3 * ORC_SX_MAXNN];
    int nn = orc_sx_nodes(dim, k, s);
    int nv = dim + 1;
    for (int64_t t = 0; t < ncells * nv; t++)
        if (cells[t] < 0 || cells[t] >= nverts) return -1;
    int64_t nocc = ncells * nn;
    sx_occ *occ = (sx_occ *)malloc(sizeof(sx_occ) * (nocc > 0 ? nocc : 1));
    for (int64_t K = 0; K < ncells; K++)
        for (int a = 0; a < nn; a++) {
            sx_occ *o = occ + K * nn + a;
            int lam[4];
            lam[0] = k;
            for (int r = 0; r < dim; r++) {
                lam[r + 1] = s[3 * a + r];
                lam[0] -= s[3 * a + r];
            }
            int m = 0;
            for (int j = 0; j < nv; j++)
                if (lam[j] > 0) {
                    o->v[m] = cells[K * nv + j];
                    o->w[m] = lam[j];
                    m++;
                }
            sx_sort_small(o->v, o->w, m);
            for (int i = m; i < 4; i++) {
                o->v[i] = INT32_MAX;
                o->w[i] = 0;
            }
            o->cell = K;
            o->a = a;
        }
    qsort(occ, nocc, sizeof(sx_occ), sx_occ_cmp);
    /* groups of equal keys; the first record of a group is its first appearance */
    sx_first *grp = (sx_first *)malloc(sizeof(sx_first) * (nocc > 0 ? nocc : 1));
    int64_t ng = 0;
    for (int64_t t = 0; t < nocc; t++) {
        int same = t > 0 && memcmp(occ[t].v, occ[t - 1].v, sizeof(occ[t].v)) == 0 &&
                   memcmp(occ[t].w, occ[t - 1].w, sizeof(occ[t].w)) == 0;
        if (!same) {
            grp[ng].first = occ[t].cell * nn + occ[t].a;
            grp[ng].group = t;
            ng++;
        }
    }
    qsort(grp, ng, sizeof(sx_first), sx_first_cmp);
    for (int64_t g = 0; g < ng; g++) {
        int64_t t = grp[g].group;
        do {
            node_of[occ[t].cell * nn + occ[t].a] = g;
            t++;
        } while (t < nocc && memcmp(occ[t].v, occ[t - 1].v, sizeof(occ[t].v)) == 0 &&
                 memcmp(occ[t].w, occ[t - 1].w, sizeof(occ[t].w)) == 0);
    }
    free(grp);
    free(occ);
    /* boundary facets: facets of exactly one cell */
    int64_t nfac = ncells * nv;
    sx_facet *fac = (sx_facet *)malloc(sizeof(sx_facet) * (nfac > 0 ? nfac : 1));
    for (int64_t K = 0; K < ncells; K++)
        for (int j = 0; j < nv; j++) {
            sx_facet *f = fac + K * nv + j;
            int m = 0;
            for (int i = 0; i < nv; i++)
                if (i != j) f->v[m++] = cells[K * nv + i];
            sx_sort_small(f->v, NULL, m);
            if (m < 3) f->v[2] = INT32_MAX;
            f->cell = K;
            f->j = j;
        }
    qsort(fac, nfac, sizeof(sx_facet), sx_facet_cmp);
    char *bnd = (char *)calloc(ng > 0 ? ng : 1, 1);
    int bad = 0;
    for (int64_t t = 0; t < nfac;) {
        int64_t u = t + 1;
        while (u < nfac && memcmp(fac[u].v, fac[t].v, sizeof(fac[t].v)) == 0) u++;
        if (u - t > 2) bad = 1;
        if (u - t == 1) {
            int64_t K = fac[t].cell;
            int j = fac[t].j;
            for (int a = 0; a < nn; a++) {
                int lj = k;
                if (j == 0)
                    for (int r = 0; r < dim; r++) lj -= s[3 * a + r];
                else
                    lj = s[3 * a + j - 1];
                if (lj == 0) bnd[node_of[K * nn + a]] = 1;
            }
        }
        t = u;
    }
    free(fac);
    int64_t nfree = 0, nfixed = 0;
    for (int64_t g = 0; g < ng; g++) node_code[g] = (dirichlet && bnd[g]) ? -1 - nfixed++ : nfree++;
    free(bnd);
    *nnodes_out = ng;
    *nfree_out = nfree;
    *nfixed_out = nfixed;
    return bad ? -2 : 0;
}

/* cell_dofs[K*nloc + a*ncomp + c] from the node numbering. */
void orc_sx_cell_dofs(int dim, int k, int ncomp, int64_t ncells, const int64_t *node_of, const int64_t *node_code,
                      int64_t *cell_dofs)
{
    int s[3 * ORC_SX_MAXNN];
    int nn = orc_sx_nodes(dim, k, s), nloc = nn * ncomp;
    for (int64_t K = 0; K < ncells; K++)
        for (int a = 0; a < nn; a++) {
            int64_t code = node_code[node_of[K * nn + a]];
            for (int c = 0; c < ncomp; c++)
                cell_dofs[K * nloc + a * ncomp + c] = code >= 0 ? ncomp * code + c : -1 - (ncomp * (-1 - code) + c);
        }
}

/* Physical position of local node a of a cell (affine image of s_a / k). */
static void sx_node_position(int dim, int k, const double *X, const int *s, int a, double *x)
{
    for (int r = 0; r < dim; r++) {
        x[r] = X[r];
        for (int t = 0; t < dim; t++) x[r] += (X[(t + 1) * dim + r] - X[r]) * s[3 * a + t] / k;
    }
}

/* Node positions of every global node (for tests): xyz[node*dim + r]. */
void orc_sx_node_positions(int dim, int k, int64_t ncells, const int32_t *cells, const double *vxyz,
                           const int64_t *node_of, double *xyz)
{
    int s[3 * ORC_SX_MAXNN];
    int nn = orc_sx_nodes(dim, k, s), nv = dim + 1;
    double X[12];
    for (int64_t K = 0; K < ncells; K++) {
        for (int j = 0; j < nv; j++)
            for (int r = 0; r < dim; r++) X[j * dim + r] = vxyz[(int64_t)cells[K * nv + j] * dim + r];
        for (int a = 0; a < nn; a++) sx_node_position(dim, k, X, s, a, xyz + node_of[K * nn + a] * dim);
    }
}

typedef struct {
    int dim, k, problem;
    double lambda, mu;
    int source_kind;
    double source[3];
    int dirichlet_kind; /* 0 zero, 1 affine */
    double dirichlet_affine[12];
} orc_sx_problem;

static void sx_cell_vertices(int dim, const int32_t *cells, const double *vxyz, int64_t K, double *X)
{
    int nv = dim + 1;
    for (int j = 0; j < nv; j++)
        for (int r = 0; r < dim; r++) X[j * dim + r] = vxyz[(int64_t)cells[K * nv + j] * dim + r];
}

/* Numeric assembly with strong Dirichlet elimination, cells in ascending
 * order (the brick oracle's orc_assemble on the simplex element routines).
 * coef: per-cell coefficient or NULL (1).  Returns -1 if a cell has
 * det J = 0. */
int orc_sx_assemble(const orc_sx_problem *P, const double *vxyz, int64_t ncells, const int32_t *cells,
                    const double *coef, const int64_t *cell_dofs, int64_t nfree, const int64_t *rowptr,
                    const int32_t *colind, double *values, double *rhs)
{
    int dim = P->dim, k = P->k;
    int s[3 * ORC_SX_MAXNN];
    int nn = orc_sx_nodes(dim, k, s);
    int ncomp = P->problem == 1 ? dim : 1, nloc = nn * ncomp;
    memset(values, 0, sizeof(double) * rowptr[nfree]);
    memset(rhs, 0, sizeof(double) * nfree);
    double *A = (double *)malloc(sizeof(double) * nloc * nloc);
    double *f = (double *)malloc(sizeof(double) * nloc);
    double *ud = (double *)malloc(sizeof(double) * nloc);
    double X[12];
    int bad = 0;
    for (int64_t K = 0; K < ncells; K++) {
        sx_cell_vertices(dim, cells, vxyz, K, X);
        double c = coef ? coef[K] : 1.0;
        if (orc_sx_element_matrix(dim, k, P->problem, X, c, P->lambda, P->mu, A) != 0) bad = 1;
        orc_sx_element_load(dim, k, ncomp, X, P->source_kind, P->source, f);
        for (int a = 0; a < nn; a++) {
            double x[3];
            sx_node_position(dim, k, X, s, a, x);
            for (int cc = 0; cc < ncomp; cc++)
                ud[a * ncomp + cc] = orc_dirichlet_value(P->dirichlet_kind, P->dirichlet_affine, dim, x, cc);
        }
        const int64_t *g = cell_dofs + K * nloc;
        for (int i = 0; i < nloc; i++) {
            if (g[i] < 0) continue;
            rhs[g[i]] += f[i];
            for (int j = 0; j < nloc; j++) {
                if (g[j] >= 0) values[orc_find(rowptr, colind, g[i], g[j])] += A[i * nloc + j];
                else rhs[g[i]] -= A[i * nloc + j] * ud[j];
            }
        }
    }
    free(A);
    free(f);
    free(ud);
    return bad ? -1 : 0;
}

/* L2 error of the discrete field (free values xfree, Dirichlet values from
 * the problem's datum) against exact_kind 1 (exact[c] prod_r sin(pi x_r)) or
 * 2 (affine, exact[4c + ...] as the Dirichlet datum), on the collapsed rule
 * with nq1 points per direction. */
double orc_sx_l2_error(const orc_sx_problem *P, const double *vxyz, int64_t ncells, const int32_t *cells,
                       const int64_t *cell_dofs, const double *xfree, int nq1, int exact_kind, const double *exact)
{
    int dim = P->dim, k = P->k;
    double Phi[ORC_SX_MAXNN * ORC_SX_MAXNN];
    int s[3 * ORC_SX_MAXNN];
    int nn = orc_sx_basis(dim, k, Phi);
    orc_sx_nodes(dim, k, s);
    int ncomp = P->problem == 1 ? dim : 1, nloc = nn * ncomp;
    int nq = ipow(nq1, dim);
    double *qx = (double *)malloc(sizeof(double) * 3 * nq), *qw = (double *)malloc(sizeof(double) * nq);
    orc_sx_quadrature(dim, nq1, qx, qw);
    double *uloc = (double *)malloc(sizeof(double) * nloc);
    double phi[ORC_SX_MAXNN], dref[ORC_SX_MAXNN * 3], X[12], J[9], Ji[9];
    double err2 = 0.0;
    for (int64_t K = 0; K < ncells; K++) {
        sx_cell_vertices(dim, cells, vxyz, K, X);
        double det = sx_jacobian(dim, X, J, Ji);
        const int64_t *g = cell_dofs + K * nloc;
        for (int a = 0; a < nn; a++) {
            double x[3];
            sx_node_position(dim, k, X, s, a, x);
            for (int c = 0; c < ncomp; c++) {
                int64_t gd = g[a * ncomp + c];
                uloc[a * ncomp + c] =
                    gd >= 0 ? xfree[gd] : orc_dirichlet_value(P->dirichlet_kind, P->dirichlet_affine, dim, x, c);
            }
        }
        for (int q = 0; q < nq; q++) {
            sx_shape_ref(dim, nn, s, Phi, qx + 3 * q, phi, dref);
            double x[3] = {0.0, 0.0, 0.0};
            for (int r = 0; r < dim; r++) {
                x[r] = X[r];
                for (int t = 0; t < dim; t++) x[r] += J[r * dim + t] * qx[3 * q + t];
            }
            for (int c = 0; c < ncomp; c++) {
                double uh = 0.0;
                for (int a = 0; a < nn; a++) uh += uloc[a * ncomp + c] * phi[a];
                double ue;
                if (exact_kind == 1) {
                    ue = exact[c];
                    for (int r = 0; r < dim; r++) ue *= sin(M_PI * x[r]);
                } else {
                    ue = orc_dirichlet_value(1, exact, dim, x, c);
                }
                err2 += qw[q] * fabs(det) * (uh - ue) * (uh - ue);
            }
        }
    }
    free(qx);
    free(qw);
    free(uloc);
    double norm = sqrt(err2);
    return norm;
}
