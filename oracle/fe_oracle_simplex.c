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

/* ======================================================================== */
/* Vector elements on simplices (Sect. 3.9 div-conforming, Sect. 3.10        */
/* curl-conforming), shape functions by the change of basis of Sect. 3.5:   */
/*  family 1: Nedelec of the lowest order, [P_0]^d + {W x : W skew}, one    */
/*            tangential moment per edge (covariant Piola map);             */
/*  family 2: Raviart-Thomas of the lowest order, [P_0]^d + x P_0, one flux */
/*            moment per facet (contravariant Piola map);                   */
/*  family 3: Nedelec of the second order, [P_1]^d + S_2 with S_2 the       */
/*            homogeneous quadratic fields orthogonal to x, two moments per */
/*            edge (against 1 - t and t along it), two per face (against   */
/*            its two edge tangents, 3D) and two interior ones (2D).       */
/*                                                                          */
/* Moments on the reference simplex (the readings taken):                   */
/*  - edge (i, j), i < j local: int_0^1 v(x_i + t (x_j - x_i)) . (x_j - x_i) */
/*    q(t) dt, the tangent not normalized (the line integral, which the     */
/*    covariant map preserves); q = 1 (family 1) or 1 - t, t (family 3);   */
/*  - facet opposite local vertex j, its vertices i0 < i1 (< i2) local:     */
/*    family 2: int over the reference (d-1)-simplex of v(phi_F(s)) . N ds  */
/*    with N = (x_i1 - x_i0) x (x_i2 - x_i0) (2D: (t_y, -t_x)), the flux;   */
/*    family 3 (3D): int v(phi_F(s)) . t_m ds, t_0 = x_i1 - x_i0,           */
/*    t_1 = x_i2 - x_i0;                                                    */
/*  - family 3 in 2D: the interior moments int_K v . e_m on the reference   */
/*    cell (local to the cell).                                             */
/* Global orientation: an edge runs from its lower to its higher global     */
/* vertex id, a facet's frame is taken over its vertices in ascending      */
/* global id.  The cell's local moments are T times the global ones (T      */
/* block diagonal: a sign per DOF for families 1-2; for family 3 a 2 x 2    */
/* block per edge -- identity, or the two DOFs swapped and negated when the */
/* edge runs the other way -- and per face, the integer matrix expressing  */
/* the local tangents in the global ones); so the cell's basis functions in */
/* the global frame are T^T phi, its matrix T^T A T and its load T^T f.     */
/* Local DOF order: edges (0,1),(0,2),(1,2) [2D] or (0,1),(0,2),(0,3),(1,2), */
/* (1,3),(2,3) [3D] (two consecutive DOFs each for family 3), then faces by  */
/* their opposite vertex, then interior DOFs; facets by their opposite     */
/* vertex for family 2.                                                     */
/* ======================================================================== */
#define VX_MAXND 20

static int vx_ndof(int family, int dim)
{
    if (family == 1) return dim == 3 ? 6 : 3;
    if (family == 2) return dim + 1;
    if (family == 4) return dim == 3 ? 15 : 8;
    return dim == 3 ? 20 : 8;
}

static int vx_order(int family) { return family >= 3 ? 2 : 1; }

/* the H(div) families (contravariant map, divergence) */
static int vx_contra(int family) { return family == 2 || family == 4; }

static void vx_edge(int dim, int a, int *i, int *j)
{
    static const int e2[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    static const int e3[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    *i = dim == 3 ? e3[a][0] : e2[a][0];
    *j = dim == 3 ? e3[a][1] : e2[a][1];
}

/* vertex r of the reference simplex */
static void vx_ref_vertex(int dim, int r, double *x)
{
    for (int t = 0; t < dim; t++) x[t] = (r > 0 && t == r - 1) ? 1.0 : 0.0;
}

/* pre-basis function b at x: value v[dim], derivative dv[c*dim + r] = d v_c / d x_r */
static void vx_prebasis(int family, int dim, int b, const double *x, double *v, double *dv)
{
    for (int c = 0; c < dim; c++) {
        v[c] = 0.0;
        for (int r = 0; r < dim; r++) dv[c * dim + r] = 0.0;
    }
    if (family == 3) {
        if (b < dim * (dim + 1)) { /* [P_1]^d: component b / (d+1) times 1, x_0, .. */
            int c = b / (dim + 1), m = b % (dim + 1);
            v[c] = m == 0 ? 1.0 : x[m - 1];
            if (m > 0) dv[c * dim + m - 1] = 1.0;
            return;
        }
        int j = b - dim * (dim + 1);
        if (dim == 2) { /* x_m (-y, x) */
            int m = j;
            double R[2] = {-x[1], x[0]};
            v[0] = x[m] * R[0];
            v[1] = x[m] * R[1];
            dv[0 * 2 + m] += R[0];
            dv[1 * 2 + m] += R[1];
            dv[0 * 2 + 1] += -x[m];
            dv[1 * 2 + 0] += x[m];
            return;
        }
        /* x_jj (x cross e_i) for the pairs (i, jj) other than (2, 2) */
        int i = j / 3, jj = j % 3;
        double R[3] = {0, 0, 0}, dR[9] = {0};
        if (i == 0) { /* (0, z, -y) */
            R[1] = x[2];
            R[2] = -x[1];
            dR[1 * 3 + 2] = 1.0;
            dR[2 * 3 + 1] = -1.0;
        } else if (i == 1) { /* (-z, 0, x) */
            R[0] = -x[2];
            R[2] = x[0];
            dR[0 * 3 + 2] = -1.0;
            dR[2 * 3 + 0] = 1.0;
        } else { /* (y, -x, 0) */
            R[0] = x[1];
            R[1] = -x[0];
            dR[0 * 3 + 1] = 1.0;
            dR[1 * 3 + 0] = -1.0;
        }
        for (int c = 0; c < 3; c++) {
            v[c] = x[jj] * R[c];
            for (int r = 0; r < 3; r++) dv[c * 3 + r] = (r == jj ? R[c] : 0.0) + x[jj] * dR[c * 3 + r];
        }
        return;
    }
    if (family == 4) {
        if (b < dim * (dim + 1)) { /* [P_1]^d as family 3 */
            int c = b / (dim + 1), m = b % (dim + 1);
            v[c] = m == 0 ? 1.0 : x[m - 1];
            if (m > 0) dv[c * dim + m - 1] = 1.0;
            return;
        }
        int m = b - dim * (dim + 1); /* x times x_m */
        for (int c = 0; c < dim; c++) {
            v[c] = x[c] * x[m];
            dv[c * dim + c] += x[m];
            dv[c * dim + m] += x[c];
        }
        return;
    }
    if (b < dim) { /* constants e_b */
        v[b] = 1.0;
        return;
    }
    if (family == 2) { /* x */
        for (int c = 0; c < dim; c++) {
            v[c] = x[c];
            dv[c * dim + c] = 1.0;
        }
        return;
    }
    /* Nedelec: rotations W x.  2D: (-y, x).  3D: b = 3: (0, -z, y), 4: (z, 0, -x), 5: (-y, x, 0) */
    if (dim == 2) {
        v[0] = -x[1];
        v[1] = x[0];
        dv[0 * 2 + 1] = -1.0;
        dv[1 * 2 + 0] = 1.0;
        return;
    }
    int m = b - 3; /* rotation about axis m: v = e_m x x */
    int p = (m + 1) % 3, q = (m + 2) % 3;
    v[p] = -x[q];
    v[q] = x[p];
    dv[p * 3 + q] = -1.0;
    dv[q * 3 + p] = 1.0;
}

/* the vertices of the facet opposite local vertex a, ascending local order */
static int vx_facet(int dim, int a, int *iv)
{
    int m = 0;
    for (int r = 0; r <= dim; r++)
        if (r != a) iv[m++] = r;
    return m;
}

/* moment a of the pre-basis function b */
static double vx_moment(int family, int dim, int a, int b)
{
    double gx[ORC_MAXQ1], gw[ORC_MAXQ1];
    double v[3], dv[9], p[3], xi[3], xj[3];
    double s = 0.0;
    int nedges = dim == 3 ? 6 : 3;
    if (family == 1 || (family == 3 && a < 2 * nedges)) {
        int e = family == 1 ? a : a / 2, slot = family == 1 ? -1 : a % 2;
        int i, j;
        vx_edge(dim, e, &i, &j);
        vx_ref_vertex(dim, i, xi);
        vx_ref_vertex(dim, j, xj);
        orc_gauss_legendre(3, gx, gw);
        for (int q = 0; q < 3; q++) {
            for (int t = 0; t < dim; t++) p[t] = xi[t] + gx[q] * (xj[t] - xi[t]);
            vx_prebasis(family, dim, b, p, v, dv);
            double d = 0.0;
            for (int t = 0; t < dim; t++) d += v[t] * (xj[t] - xi[t]);
            double qv = slot < 0 ? 1.0 : slot == 0 ? 1.0 - gx[q] : gx[q];
            s += gw[q] * d * qv;
        }
        return s;
    }
    if ((family == 3 && dim == 2) || (family == 4 && a >= dim * (dim + 1))) {
        /* interior moments: the components' integrals over the reference cell */
        int m = family == 3 ? a - 6 : a - dim * (dim + 1);
        double qx[3 * 27], qw[27];
        int nq = orc_sx_quadrature(dim, 3, qx, qw);
        for (int q = 0; q < nq; q++) {
            vx_prebasis(family, dim, b, qx + 3 * q, v, dv);
            s += qw[q] * v[m];
        }
        return s;
    }
    if (family == 4) { /* flux through facet a / d against the barycentric of its vertex a % d */
        int iv[3], k = a % dim;
        vx_facet(dim, a / dim, iv);
        double y[3][3] = {{0}};
        for (int t = 0; t < dim; t++) vx_ref_vertex(dim, iv[t], y[t]);
        double Nf[3] = {0, 0, 0};
        if (dim == 2) {
            Nf[0] = y[1][1] - y[0][1];
            Nf[1] = y[0][0] - y[1][0];
        } else {
            double e1[3], e2[3];
            for (int t = 0; t < 3; t++) {
                e1[t] = y[1][t] - y[0][t];
                e2[t] = y[2][t] - y[0][t];
            }
            Nf[0] = e1[1] * e2[2] - e1[2] * e2[1];
            Nf[1] = e1[2] * e2[0] - e1[0] * e2[2];
            Nf[2] = e1[0] * e2[1] - e1[1] * e2[0];
        }
        double fx[3 * 9], fw[9];
        int nf;
        if (dim == 2) {
            orc_gauss_legendre(2, gx, gw);
            for (int q = 0; q < 2; q++) {
                fx[3 * q] = gx[q];
                fw[q] = gw[q];
            }
            nf = 2;
        } else {
            nf = orc_sx_quadrature(2, 3, fx, fw);
        }
        for (int q = 0; q < nf; q++) {
            /* barycentrics of the facet's vertices at the point */
            double lam[3];
            lam[1] = fx[3 * q];
            lam[2] = dim == 3 ? fx[3 * q + 1] : 0.0;
            lam[0] = 1.0 - lam[1] - lam[2];
            for (int t = 0; t < dim; t++) {
                p[t] = 0.0;
                for (int r = 0; r < dim; r++) p[t] += lam[r] * y[r][t];
            }
            vx_prebasis(family, dim, b, p, v, dv);
            double d = 0.0;
            for (int t = 0; t < dim; t++) d += v[t] * Nf[t];
            s += fw[q] * d * lam[k];
        }
        return s;
    }
    /* facet moments: family 2 (flux) or family 3 in 3D (tangents) */
    int f = family == 2 ? a : (a - 12) / 2, slot = family == 2 ? -1 : (a - 12) % 2;
    int iv[3];
    vx_facet(dim, f, iv);
    double x0[3], x1[3], x2[3] = {0, 0, 0}, N[3];
    vx_ref_vertex(dim, iv[0], x0);
    vx_ref_vertex(dim, iv[1], x1);
    if (dim == 3) vx_ref_vertex(dim, iv[2], x2);
    double t1[3] = {0, 0, 0}, t2[3] = {0, 0, 0};
    for (int t = 0; t < dim; t++) {
        t1[t] = x1[t] - x0[t];
        t2[t] = x2[t] - x0[t];
    }
    if (dim == 2) {
        N[0] = t1[1];
        N[1] = -t1[0];
    } else if (slot < 0) {
        N[0] = t1[1] * t2[2] - t1[2] * t2[1];
        N[1] = t1[2] * t2[0] - t1[0] * t2[2];
        N[2] = t1[0] * t2[1] - t1[1] * t2[0];
    } else {
        for (int t = 0; t < 3; t++) N[t] = slot == 0 ? t1[t] : t2[t];
    }
    if (dim == 2) {
        orc_gauss_legendre(2, gx, gw);
        for (int q = 0; q < 2; q++) {
            for (int t = 0; t < 2; t++) p[t] = x0[t] + gx[q] * (x1[t] - x0[t]);
            vx_prebasis(family, dim, b, p, v, dv);
            s += gw[q] * (v[0] * N[0] + v[1] * N[1]);
        }
        return s;
    }
    double sq[3 * 9], sw[9];
    int nq = orc_sx_quadrature(2, 3, sq, sw);
    for (int q = 0; q < nq; q++) {
        for (int t = 0; t < 3; t++) p[t] = x0[t] + sq[3 * q] * (x1[t] - x0[t]) + sq[3 * q + 1] * (x2[t] - x0[t]);
        vx_prebasis(family, dim, b, p, v, dv);
        s += sw[q] * (v[0] * N[0] + v[1] * N[1] + v[2] * N[2]);
    }
    return s;
}

/* Change-of-basis matrix Phi (nd x nd) of the family.  Returns nd or -1. */
int orc_vx_basis(int family, int dim, double *Phi)
{
    if (family < 1 || family > 4 || dim < 2 || dim > 3) return -1;
    int nd = vx_ndof(family, dim);
    double C[VX_MAXND * VX_MAXND], Ci[VX_MAXND * VX_MAXND];
    for (int a = 0; a < nd; a++)
        for (int b = 0; b < nd; b++) C[a * nd + b] = vx_moment(family, dim, a, b);
    if (sx_invert(nd, C, Ci) != 0) return -1;
    for (int a = 0; a < nd; a++)
        for (int b = 0; b < nd; b++) Phi[a * nd + b] = Ci[b * nd + a];
    return nd;
}

/* Shape functions phi_a = sum_b Phi_ab psi_b at xi from a change-of-basis
 * matrix: phi[a*dim + c], their curl (3D: curl[a*3 + c]; 2D: the scalar
 * curl[a]) and divergence div[a]. */
static void vx_shape_with(int family, int dim, int nd, const double *Phi, const double *xi, double *phi, double *curl,
                          double *div)
{
    for (int a = 0; a < nd; a++) {
        double v[3] = {0, 0, 0}, dv[9] = {0};
        for (int b = 0; b < nd; b++) {
            double pv[3], pdv[9];
            vx_prebasis(family, dim, b, xi, pv, pdv);
            for (int c = 0; c < dim; c++) v[c] += Phi[a * nd + b] * pv[c];
            for (int t = 0; t < dim * dim; t++) dv[t] += Phi[a * nd + b] * pdv[t];
        }
        for (int c = 0; c < dim; c++) phi[a * dim + c] = v[c];
        if (dim == 3) {
            curl[a * 3 + 0] = dv[2 * 3 + 1] - dv[1 * 3 + 2];
            curl[a * 3 + 1] = dv[0 * 3 + 2] - dv[2 * 3 + 0];
            curl[a * 3 + 2] = dv[1 * 3 + 0] - dv[0 * 3 + 1];
        } else {
            curl[a] = dv[1 * 2 + 0] - dv[0 * 2 + 1];
        }
        div[a] = 0.0;
        for (int c = 0; c < dim; c++) div[a] += dv[c * dim + c];
    }
}

/* Reference shape functions at xi (the family's basis; for tests). */
int orc_vx_shape(int family, int dim, const double *xi, double *phi, double *curl, double *div)
{
    double Phi[VX_MAXND * VX_MAXND];
    int nd = orc_vx_basis(family, dim, Phi);
    if (nd < 0) return -1;
    vx_shape_with(family, dim, nd, Phi, xi, phi, curl, div);
    return nd;
}

/* Orientation signs of the lowest-order families' local DOFs. */
static void vx_signs(int family, int dim, const int32_t *g, double *sgn)
{
    int nd = vx_ndof(family, dim);
    for (int a = 0; a < nd; a++) {
        if (family == 1) {
            int i, j;
            vx_edge(dim, a, &i, &j);
            sgn[a] = g[i] < g[j] ? 1.0 : -1.0;
        } else {
            int iv[3], m = 0;
            for (int r = 0; r <= dim; r++)
                if (r != a) iv[m++] = g[r];
            /* parity of the permutation sorting the facet's vertex ids */
            int inv = 0;
            for (int x = 0; x < m; x++)
                for (int y = x + 1; y < m; y++)
                    if (iv[x] > iv[y]) inv++;
            sgn[a] = (inv % 2) ? -1.0 : 1.0;
        }
    }
}

/* T (nd x nd, row-major): local moments = T global moments, from the cell's
 * global vertex ids. */
static void vx_transform(int family, int dim, const int32_t *g, double *T)
{
    int nd = vx_ndof(family, dim);
    memset(T, 0, sizeof(double) * nd * nd);
    if (family == 4) {
        /* a facet's moments: against the barycentric of each of its vertices,
         * flux with N over the vertices in ascending global id; a local moment
         * is the global one of the same vertex, times the parity of the
         * permutation that sorts the facet's ids (the orientation of N) */
        for (int f = 0; f <= dim; f++) {
            int iv[3], rank[3], inv = 0;
            vx_facet(dim, f, iv);
            for (int x = 0; x < dim; x++) {
                rank[x] = 0;
                for (int y = 0; y < dim; y++) {
                    if (g[iv[y]] < g[iv[x]]) rank[x]++;
                    if (y > x && g[iv[x]] > g[iv[y]]) inv++;
                }
            }
            for (int x = 0; x < dim; x++) T[(f * dim + x) * nd + f * dim + rank[x]] = (inv % 2) ? -1.0 : 1.0;
        }
        for (int a = dim * (dim + 1); a < nd; a++) T[a * nd + a] = 1.0; /* interior */
        return;
    }
    if (family != 3) {
        double sgn[6];
        vx_signs(family, dim, g, sgn);
        for (int a = 0; a < nd; a++) T[a * nd + a] = sgn[a];
        return;
    }
    int nedges = dim == 3 ? 6 : 3;
    for (int e = 0; e < nedges; e++) {
        int i, j, a = 2 * e;
        vx_edge(dim, e, &i, &j);
        if (g[i] < g[j]) {
            T[a * nd + a] = 1.0;
            T[(a + 1) * nd + a + 1] = 1.0;
        } else { /* reversed: the two moments swap ends and change sign */
            T[a * nd + a + 1] = -1.0;
            T[(a + 1) * nd + a] = -1.0;
        }
    }
    if (dim == 3) {
        for (int f = 0; f < 4; f++) {
            int iv[3], a = 12 + 2 * f;
            vx_facet(dim, f, iv);
            /* rank of each facet vertex in ascending global id */
            int rank[3];
            for (int x = 0; x < 3; x++) {
                rank[x] = 0;
                for (int y = 0; y < 3; y++)
                    if (g[iv[y]] < g[iv[x]]) rank[x]++;
            }
            /* position of facet vertex x in the global frame: 0 -> (0,0), 1 -> (1,0), 2 -> (0,1) */
            double P[3][2];
            for (int x = 0; x < 3; x++) {
                P[x][0] = rank[x] == 1 ? 1.0 : 0.0;
                P[x][1] = rank[x] == 2 ? 1.0 : 0.0;
            }
            for (int m = 0; m < 2; m++)
                for (int b = 0; b < 2; b++) T[(a + m) * nd + a + b] = P[m + 1][b] - P[0][b];
        }
    } else {
        T[6 * nd + 6] = 1.0;
        T[7 * nd + 7] = 1.0;
    }
}

/* The family's manufactured field m(x): Nedelec 3D (sin pi y sin pi z,
 * sin pi z sin pi x, sin pi x sin pi y), 2D (sin pi y, sin pi x);
 * Raviart-Thomas (sin pi x_r)_r. */
static void vx_field(int family, int dim, const double *x, double *m)
{
    double s[3] = {0.0, 0.0, 0.0};
    for (int r = 0; r < dim; r++) s[r] = sin(M_PI * x[r]);
    if (vx_contra(family)) {
        for (int r = 0; r < dim; r++) m[r] = s[r];
    } else if (dim == 2) {
        m[0] = s[1];
        m[1] = s[0];
    } else {
        m[0] = s[1] * s[2];
        m[1] = s[2] * s[0];
        m[2] = s[0] * s[1];
    }
}

/* load f_c(x): kind 1 constant source[c], kind 2 source[c] m_c(x), kind 3
 * affine: source[4c] + sum_r source[4c+1+r] x_r (source has 12 entries) */
static void vx_source(int family, int dim, int kind, const double *src, const double *x, double *f)
{
    double m[3] = {0, 0, 0};
    if (kind == 2) vx_field(family, dim, x, m);
    for (int c = 0; c < dim; c++) {
        if (kind == 3) {
            f[c] = src[4 * c];
            for (int r = 0; r < dim; r++) f[c] += src[4 * c + 1 + r] * x[r];
        } else {
            f[c] = kind == 1 ? src[c] : kind == 2 ? src[c] * m[c] : 0.0;
        }
    }
}

/* Element matrix and load of the form
 *   a(u, v) = int coef (curl u . curl v) + kappa u . v     (families 1, 3)
 *   a(u, v) = int coef (div u div v) + kappa u . v         (family 2)
 * on a simplex with vertices X and global vertex ids g (for the
 * orientation), by the collapsed rule with order + ceil(d/2) points per
 * direction; physical shape functions J^-T phi (curl J curl / det J in 3D,
 * curl / det J in 2D) or J phi / det J (div / det J).  Returned in the global
 * frame: T^T A T and T^T f.  A nd x nd, f nd. */
int orc_vx_element(int family, int dim, const double *X, const int32_t *g, double coef, double kappa,
                   int source_kind, const double *source, double *A, double *f)
{
    int nd = vx_ndof(family, dim);
    int n = vx_order(family) + (dim + 1) / 2;
    int nq = ipow(n, dim);
    double *qx = (double *)malloc(sizeof(double) * 3 * nq), *qw = (double *)malloc(sizeof(double) * nq);
    orc_sx_quadrature(dim, n, qx, qw);
    double J[9], Ji[9];
    double det = sx_jacobian(dim, X, J, Ji);
    double T[VX_MAXND * VX_MAXND], Phi[VX_MAXND * VX_MAXND], Al[VX_MAXND * VX_MAXND], fl[VX_MAXND];
    vx_transform(family, dim, g, T);
    orc_vx_basis(family, dim, Phi);
    memset(Al, 0, sizeof(double) * nd * nd);
    memset(fl, 0, sizeof(double) * nd);
    for (int q = 0; q < nq; q++) {
        double phi[3 * VX_MAXND], curl[3 * VX_MAXND], div[VX_MAXND];
        vx_shape_with(family, dim, nd, Phi, qx + 3 * q, phi, curl, div);
        double P[3 * VX_MAXND], Cp[3 * VX_MAXND], Dp[VX_MAXND]; /* physical values */
        for (int a = 0; a < nd; a++) {
            for (int c = 0; c < dim; c++) {
                double v = 0.0;
                for (int r = 0; r < dim; r++)
                    v += !vx_contra(family) ? Ji[r * dim + c] * phi[a * dim + r] : J[c * dim + r] * phi[a * dim + r] / det;
                P[a * dim + c] = v;
            }
            if (dim == 3) {
                for (int c = 0; c < 3; c++) {
                    double v = 0.0;
                    for (int r = 0; r < 3; r++) v += J[c * 3 + r] * curl[a * 3 + r];
                    Cp[a * 3 + c] = v / det;
                }
            } else {
                Cp[a] = curl[a] / det;
            }
            Dp[a] = div[a] / det;
        }
        double x[3] = {0, 0, 0};
        for (int r = 0; r < dim; r++) {
            x[r] = X[r];
            for (int t = 0; t < dim; t++) x[r] += J[r * dim + t] * qx[3 * q + t];
        }
        double fx[3];
        vx_source(family, dim, source_kind, source, x, fx);
        double wd = qw[q] * fabs(det);
        int nc = dim == 3 ? 3 : 1;
        for (int a = 0; a < nd; a++) {
            double fa = 0.0;
            for (int c = 0; c < dim; c++) fa += fx[c] * P[a * dim + c];
            fl[a] += wd * fa;
            for (int b = 0; b < nd; b++) {
                double st = 0.0, ms = 0.0;
                if (!vx_contra(family))
                    for (int c = 0; c < nc; c++) st += Cp[a * nc + c] * Cp[b * nc + c];
                else
                    st = Dp[a] * Dp[b];
                for (int c = 0; c < dim; c++) ms += P[a * dim + c] * P[b * dim + c];
                Al[a * nd + b] += wd * (coef * st + kappa * ms);
            }
        }
    }
    free(qx);
    free(qw);
    /* to the global frame: A = T^T Al T, f = T^T fl */
    for (int b = 0; b < nd; b++) {
        double s = 0.0;
        for (int a = 0; a < nd; a++) s += T[a * nd + b] * fl[a];
        f[b] = s;
        for (int d = 0; d < nd; d++) {
            double v = 0.0;
            for (int a = 0; a < nd; a++)
                for (int c = 0; c < nd; c++) v += T[a * nd + b] * Al[a * nd + c] * T[c * nd + d];
            A[b * nd + d] = v;
        }
    }
    return det == 0.0 ? -1 : 0;
}

/* Numbering of the DOFs (an edge's, a facet's, or -- family 3 in 2D -- a
 * cell's interior ones): a DOF is named by its entity's sorted vertex ids
 * and its slot in the entity's global frame; ids by first appearance over
 * (cell, local DOF); dirichlet != 0 fixes the DOFs of entities on the
 * boundary (facets of one cell, and their edges).  dof_of[K*nd + a],
 * code[dof] as orc_sx_number.  Returns 0, -1, -2. */
int orc_vx_number(int family, int dim, int64_t nverts, int64_t ncells, const int32_t *cells, int dirichlet,
                  int64_t *dof_of, int64_t *code, int64_t *nent_out, int64_t *nfree_out, int64_t *nfixed_out)
{
    if (family < 1 || family > 4 || dim < 2 || dim > 3) return -1;
    int nd = vx_ndof(family, dim), nv = dim + 1, nedges = dim == 3 ? 6 : 3;
    for (int64_t t = 0; t < ncells * nv; t++)
        if (cells[t] < 0 || cells[t] >= nverts) return -1;
    int64_t nrec = ncells * nd;
    sx_occ *rec = (sx_occ *)malloc(sizeof(sx_occ) * (nrec > 0 ? nrec : 1));
    for (int64_t K = 0; K < ncells; K++)
        for (int a = 0; a < nd; a++) {
            sx_occ *r = rec + K * nd + a;
            const int32_t *g = cells + K * nv;
            int m = 0, slot = 0;
            if (family == 1 || (family == 3 && a < 2 * nedges)) {
                int i, j;
                vx_edge(dim, family == 1 ? a : a / 2, &i, &j);
                r->v[m++] = g[i];
                r->v[m++] = g[j];
                slot = family == 1 ? 0 : a % 2;
            } else if ((family == 3 && dim == 2) || (family == 4 && a >= dim * (dim + 1))) {
                /* interior: the cell's vertices */
                for (int t = 0; t < nv; t++) r->v[m++] = g[t];
                slot = family == 3 ? a - 6 : a - dim * (dim + 1);
            } else if (family == 4) { /* facet a / d, slot a % d of its global frame */
                int iv[3];
                vx_facet(dim, a / dim, iv);
                for (int t = 0; t < dim; t++) r->v[m++] = g[iv[t]];
                slot = a % dim;
            } else {
                int iv[3];
                vx_facet(dim, family == 2 ? a : (a - 12) / 2, iv);
                for (int t = 0; t < dim; t++) r->v[m++] = g[iv[t]];
                slot = family == 2 ? 0 : (a - 12) % 2;
            }
            sx_sort_small(r->v, NULL, m);
            for (int t = m; t < 4; t++) r->v[t] = INT32_MAX;
            r->w[0] = slot;
            r->w[1] = r->w[2] = r->w[3] = 0;
            r->cell = K;
            r->a = a;
        }
    qsort(rec, nrec, sizeof(sx_occ), sx_occ_cmp);
    sx_first *first_of = (sx_first *)malloc(sizeof(sx_first) * (nrec > 0 ? nrec : 1));
    int64_t ng = 0;
    for (int64_t t = 0; t < nrec; t++)
        if (t == 0 || memcmp(rec[t].v, rec[t - 1].v, sizeof(rec[t].v)) != 0 || rec[t].w[0] != rec[t - 1].w[0]) {
            first_of[ng].first = rec[t].cell * nd + rec[t].a;
            first_of[ng].group = t;
            ng++;
        }
    qsort(first_of, ng, sizeof(sx_first), sx_first_cmp);
    for (int64_t g2 = 0; g2 < ng; g2++) {
        int64_t t = first_of[g2].group;
        do {
            dof_of[rec[t].cell * nd + rec[t].a] = g2;
            t++;
        } while (t < nrec && memcmp(rec[t].v, rec[t - 1].v, sizeof(rec[t].v)) == 0 && rec[t].w[0] == rec[t - 1].w[0]);
    }
    free(first_of);
    free(rec);
    /* boundary facets */
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
            for (int a = 0; a < nd; a++) {
                int on;
                if (family == 2) {
                    on = a == j;
                } else if (family == 4) {
                    on = a < dim * (dim + 1) && a / dim == j;
                } else if (family == 1 || a < 2 * nedges) {
                    int i1, j1;
                    vx_edge(dim, family == 1 ? a : a / 2, &i1, &j1);
                    on = i1 != j && j1 != j; /* the edge avoids the opposite vertex */
                } else if (dim == 3) {
                    on = (a - 12) / 2 == j;
                } else {
                    on = 0; /* interior */
                }
                if (on) bnd[dof_of[K * nd + a]] = 1;
            }
        }
        t = u;
    }
    free(fac);
    int64_t nfree = 0, nfixed = 0;
    for (int64_t g2 = 0; g2 < ng; g2++) code[g2] = (dirichlet && bnd[g2]) ? -1 - nfixed++ : nfree++;
    free(bnd);
    *nent_out = ng;
    *nfree_out = nfree;
    *nfixed_out = nfixed;
    return bad ? -2 : 0;
}

/* Assembly of the vector-element system (zero boundary data: fixed DOFs are
 * dropped), cells ascending, as orc_sx_assemble. */
int orc_vx_assemble(int family, int dim, const double *vxyz, int64_t ncells, const int32_t *cells, const double *coef,
                    double kappa, int source_kind, const double *source, const int64_t *cell_dofs, int64_t nfree,
                    const int64_t *rowptr, const int32_t *colind, double *values, double *rhs)
{
    int nd = vx_ndof(family, dim), nv = dim + 1;
    memset(values, 0, sizeof(double) * rowptr[nfree]);
    memset(rhs, 0, sizeof(double) * nfree);
    double A[VX_MAXND * VX_MAXND], f[VX_MAXND], X[12];
    int bad = 0;
    for (int64_t K = 0; K < ncells; K++) {
        sx_cell_vertices(dim, cells, vxyz, K, X);
        if (orc_vx_element(family, dim, X, cells + K * nv, coef ? coef[K] : 1.0, kappa, source_kind, source, A, f))
            bad = 1;
        const int64_t *g = cell_dofs + K * nd;
        for (int a = 0; a < nd; a++) {
            if (g[a] < 0) continue;
            rhs[g[a]] += f[a];
            for (int b = 0; b < nd; b++)
                if (g[b] >= 0) values[orc_find(rowptr, colind, g[a], g[b])] += A[a * nd + b];
        }
    }
    return bad ? -1 : 0;
}

/* L2 error of the discrete field (free DOF values x, fixed DOFs zero)
 * against scale * m(x), the family's manufactured field, on the collapsed
 * rule with nq1 points per direction. */
double orc_vx_l2_error(int family, int dim, const double *vxyz, int64_t ncells, const int32_t *cells,
                       const int64_t *cell_dofs, const double *x, double scale, int nq1)
{
    int nd = vx_ndof(family, dim), nv = dim + 1;
    int nq = ipow(nq1, dim);
    double *qx = (double *)malloc(sizeof(double) * 3 * nq), *qw = (double *)malloc(sizeof(double) * nq);
    orc_sx_quadrature(dim, nq1, qx, qw);
    double X[12], J[9], Ji[9], err2 = 0.0, Phi[VX_MAXND * VX_MAXND], T[VX_MAXND * VX_MAXND];
    orc_vx_basis(family, dim, Phi);
    for (int64_t K = 0; K < ncells; K++) {
        sx_cell_vertices(dim, cells, vxyz, K, X);
        double det = sx_jacobian(dim, X, J, Ji);
        double ug[VX_MAXND], u[VX_MAXND];
        vx_transform(family, dim, cells + K * nv, T);
        for (int a = 0; a < nd; a++) {
            int64_t gd = cell_dofs[K * nd + a];
            ug[a] = gd >= 0 ? x[gd] : 0.0;
        }
        /* local coefficients u = T ug */
        for (int a = 0; a < nd; a++) {
            double s = 0.0;
            for (int b = 0; b < nd; b++) s += T[a * nd + b] * ug[b];
            u[a] = s;
        }
        for (int q = 0; q < nq; q++) {
            double phi[3 * VX_MAXND], curl[3 * VX_MAXND], div[VX_MAXND], uh[3] = {0, 0, 0}, p[3], m[3];
            vx_shape_with(family, dim, nd, Phi, qx + 3 * q, phi, curl, div);
            for (int a = 0; a < nd; a++)
                for (int c = 0; c < dim; c++)
                    for (int r = 0; r < dim; r++) {
                        /* covariant J^-T phi, or contravariant J phi / det J */
                        double m1 = !vx_contra(family) ? Ji[r * dim + c] : J[c * dim + r] / det;
                        uh[c] += u[a] * m1 * phi[a * dim + r];
                    }
            for (int r = 0; r < dim; r++) {
                p[r] = X[r];
                for (int t = 0; t < dim; t++) p[r] += J[r * dim + t] * qx[3 * q + t];
            }
            vx_field(family, dim, p, m);
            for (int c = 0; c < dim; c++) err2 += qw[q] * fabs(det) * (uh[c] - scale * m[c]) * (uh[c] - scale * m[c]);
        }
    }
    free(qx);
    free(qw);
    double e = sqrt(err2);
    return e;
}
