/*
 * sanitize_check.c -- a driver that runs every routine of the oracle on small
 * inputs, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (host code only).  TEST INFRASTRUCTURE: it includes the oracle's source and
 * is built and run by tests/test_oracle_sanitized.py; it exits non-zero if a
 * check fails, and the sanitizers abort on any out-of-bounds access, use of
 * freed memory or undefined operation.
 *
 * Besides exercising the code it checks a few properties that hold exactly
 * (symmetry, zero row sums without Dirichlet data, agreement of PCG with the
 * right-hand side), so a run that only avoids crashing does not pass.
 */
#include <stdio.h>

#include "fe_oracle.c"

static int failures = 0;

static void check(int ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s\n", what);
        failures++;
    }
}

/* brick vertices, jittered deterministically (no RNG needed) */
static double *brick(int dim, const int *n)
{
    int nx = n[0] + 1, ny = n[1] + 1, nz = dim == 3 ? n[2] + 1 : 1;
    double *v = (double *)malloc(sizeof(double) * nx * ny * nz * dim);
    for (int l = 0; l < nz; l++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                int id = i + nx * (j + ny * l);
                int I[3] = {i, j, l};
                for (int r = 0; r < dim; r++) {
                    double x = (double)I[r] / n[r];
                    int interior = i > 0 && i < nx - 1 && j > 0 && j < ny - 1 && (dim == 2 || (l > 0 && l < nz - 1));
                    if (interior) x += 0.1 / n[r] * sin(1.7 * id + r);
                    v[id * dim + r] = x;
                }
            }
    return v;
}

static double max_abs_row_sum(int64_t n, const int64_t *rp, const double *val)
{
    double m = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t t = rp[i]; t < rp[i + 1]; t++) s += val[t];
        if (fabs(s) > m) m = fabs(s);
    }
    return m;
}

static void run_brick(int dim, int k, int problem)
{
    int n[3] = {3, 2, 2};
    orc_problem P;
    memset(&P, 0, sizeof(P));
    P.dim = dim;
    P.n[0] = n[0];
    P.n[1] = n[1];
    P.n[2] = dim == 3 ? n[2] : 1;
    P.k = k;
    P.problem = problem;
    P.lambda = 0.5;
    P.mu = 0.7;
    P.source_kind = 2;
    P.source[0] = P.source[1] = P.source[2] = 1.0;
    P.dirichlet_kind = 1;
    for (int t = 0; t < 12; t++) P.dirichlet_affine[t] = 0.1 * (t + 1);
    double *v = brick(dim, P.n);
    int64_t nnodes = 1;
    for (int r = 0; r < dim; r++) nnodes *= (int64_t)P.n[r] * k + 1;
    int64_t *code = (int64_t *)malloc(sizeof(int64_t) * nnodes), nfree, nfixed;
    unsigned faces = (1u << (2 * dim)) - 1u;
    orc_number_nodes(dim, P.n, k, faces, code, &nfree, &nfixed);
    int ncomp = problem == 1 ? dim : 1, nn = ipow(k + 1, dim), nloc = nn * ncomp;
    int64_t ncells = (int64_t)P.n[0] * P.n[1] * P.n[2];
    int64_t *cd = (int64_t *)malloc(sizeof(int64_t) * ncells * nloc);
    orc_cell_dofs(dim, P.n, k, ncomp, code, ncells, cd);
    int64_t nf = nfree * ncomp;
    int64_t *rp = (int64_t *)malloc(sizeof(int64_t) * (nf + 1));
    int32_t *ci = NULL;
    int64_t nnz = orc_csr_pattern(ncells, nloc, cd, nf, rp, &ci);
    double *val = (double *)malloc(sizeof(double) * (nnz > 0 ? nnz : 1)), *rhs = (double *)malloc(sizeof(double) * nf);
    check(orc_assemble(&P, v, NULL, cd, nf, rp, ci, val, rhs) == 0, "brick assembly");
    /* symmetry, relative to the largest entry (cancellation leaves entries near zero) */
    double vmax = 0.0;
    for (int64_t t = 0; t < nnz; t++) vmax = fmax(vmax, fabs(val[t]));
    int sym = 1;
    for (int64_t i = 0; i < nf; i++)
        for (int64_t t = rp[i]; t < rp[i + 1]; t++) {
            int64_t p = orc_find(rp, ci, ci[t], i);
            if (p < 0 || fabs(val[p] - val[t]) > 1e-13 * vmax) sym = 0;
        }
    check(sym, "brick matrix symmetric");
    double *x = (double *)calloc(nf, sizeof(double));
    int it = 0;
    double rr = 0.0;
    int st = orc_pcg(nf, rp, ci, val, rhs, x, 1e-10, 5000, &it, &rr, NULL, NULL);
    check(st == 0 && rr <= 1e-10, "brick pcg");
    (void)orc_l2_error(&P, v, cd, x, k + 2, 1, P.source);
    free(x);
    free(val);
    free(rhs);
    orc_free(ci);
    free(rp);
    free(cd);
    free(code);
    free(v);
}

static void run_dg(int dim, int k)
{
    orc_problem P;
    memset(&P, 0, sizeof(P));
    P.dim = dim;
    P.n[0] = 2;
    P.n[1] = 3;
    P.n[2] = dim == 3 ? 2 : 1;
    P.k = k;
    P.source_kind = 2;
    P.source[0] = 1.0;
    P.dirichlet_kind = 1;
    P.dirichlet_affine[0] = 0.3;
    P.dirichlet_affine[1] = 1.0;
    double *v = brick(dim, P.n);
    int64_t nn = ipow(k + 1, dim), nrows = nn * P.n[0] * P.n[1] * P.n[2];
    int64_t *rp = (int64_t *)malloc(sizeof(int64_t) * (nrows + 1));
    int32_t *ci = NULL;
    int64_t nnz = orc_dg_pattern(&P, rp, &ci);
    double *val = (double *)malloc(sizeof(double) * nnz), *rhs = (double *)malloc(sizeof(double) * nrows);
    check(orc_dg_assemble(&P, v, 4.0 * (k + 1) * (k + 1), 1.0, rp, ci, val, rhs) == 0, "dg assembly");
    double vmax = 0.0;
    for (int64_t t = 0; t < nnz; t++) vmax = fmax(vmax, fabs(val[t]));
    int sym = 1;
    for (int64_t i = 0; i < nrows; i++)
        for (int64_t t = rp[i]; t < rp[i + 1]; t++) {
            int64_t p = orc_find(rp, ci, ci[t], i);
            if (p < 0 || fabs(val[p] - val[t]) > 1e-13 * vmax) sym = 0;
        }
    check(sym, "dg matrix symmetric for tau = 1");
    free(val);
    free(rhs);
    orc_free(ci);
    free(rp);
    free(v);
}

/* Kuhn subdivision of an n^3 (n^2) brick */
static int32_t *kuhn(int dim, const int *n, int64_t *ncells_out)
{
    int nx = n[0] + 1, ny = n[1] + 1;
    int64_t nc = (int64_t)n[0] * n[1] * (dim == 3 ? n[2] : 1) * (dim == 3 ? 6 : 2);
    int32_t *c = (int32_t *)malloc(sizeof(int32_t) * nc * (dim + 1));
    static const int perm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    static const int perm2[2][2] = {{0, 1}, {1, 0}};
    int64_t t = 0;
    for (int l = 0; l < (dim == 3 ? n[2] : 1); l++)
        for (int j = 0; j < n[1]; j++)
            for (int i = 0; i < n[0]; i++) {
                int base = i + nx * (j + ny * l), stride[3] = {1, nx, nx * ny};
                for (int p = 0; p < (dim == 3 ? 6 : 2); p++) {
                    int off = 0;
                    c[t * (dim + 1)] = base;
                    for (int s = 0; s < dim; s++) {
                        off += stride[dim == 3 ? perm3[p][s] : perm2[p][s]];
                        c[t * (dim + 1) + s + 1] = base + off;
                    }
                    t++;
                }
            }
    *ncells_out = nc;
    return c;
}

static void run_simplex(int dim, int k, int problem)
{
    int n[3] = {2, 2, 2};
    double *v = brick(dim, n);
    int64_t nv = (int64_t)(n[0] + 1) * (n[1] + 1) * (dim == 3 ? n[2] + 1 : 1), nc;
    int32_t *c = kuhn(dim, n, &nc);
    int nn = (k + 1) * (k + 2) / 2;
    if (dim == 3) nn = nn * (k + 3) / 3;
    int ncomp = problem == 1 ? dim : 1, nloc = nn * ncomp;
    int64_t *node_of = (int64_t *)malloc(sizeof(int64_t) * nc * nn), *code = (int64_t *)malloc(sizeof(int64_t) * nc * nn);
    int64_t nnodes, nfree, nfixed;
    check(orc_sx_number(dim, k, nv, nc, c, 0, node_of, code, &nnodes, &nfree, &nfixed) == 0, "simplex numbering");
    int64_t *cd = (int64_t *)malloc(sizeof(int64_t) * nc * nloc);
    orc_sx_cell_dofs(dim, k, ncomp, nc, node_of, code, cd);
    int64_t nf = nfree * ncomp;
    int64_t *rp = (int64_t *)malloc(sizeof(int64_t) * (nf + 1));
    int32_t *ci = NULL;
    int64_t nnz = orc_csr_pattern(nc, nloc, cd, nf, rp, &ci);
    double *val = (double *)malloc(sizeof(double) * nnz), *rhs = (double *)malloc(sizeof(double) * nf);
    orc_sx_problem P;
    memset(&P, 0, sizeof(P));
    P.dim = dim;
    P.k = k;
    P.problem = problem;
    P.lambda = 0.4;
    P.mu = 0.6;
    P.source_kind = 1;
    P.source[0] = 1.0;
    check(orc_sx_assemble(&P, v, nc, c, NULL, cd, nf, rp, ci, val, rhs) == 0, "simplex assembly");
    if (problem == 0) check(max_abs_row_sum(nf, rp, val) < 1e-10, "simplex Laplacian row sums without Dirichlet data");
    double *xyz = (double *)malloc(sizeof(double) * nnodes * dim);
    orc_sx_node_positions(dim, k, nc, c, v, node_of, xyz);
    free(xyz);
    free(val);
    free(rhs);
    orc_free(ci);
    free(rp);
    free(cd);
    free(code);
    free(node_of);
    free(c);
    free(v);
}

static void run_vector(int family, int dim)
{
    int n[3] = {2, 2, 2};
    double *v = brick(dim, n);
    int64_t nv = (int64_t)(n[0] + 1) * (n[1] + 1) * (dim == 3 ? n[2] + 1 : 1), nc;
    int32_t *c = kuhn(dim, n, &nc);
    int nd = vx_ndof(family, dim);
    int64_t *dof_of = (int64_t *)malloc(sizeof(int64_t) * nc * nd), *code = (int64_t *)malloc(sizeof(int64_t) * nc * nd);
    int64_t nent, nfree, nfixed;
    check(orc_vx_number(family, dim, nv, nc, c, 1, dof_of, code, &nent, &nfree, &nfixed) == 0, "vector numbering");
    int64_t *cd = (int64_t *)malloc(sizeof(int64_t) * nc * nd);
    for (int64_t t = 0; t < nc * nd; t++) cd[t] = code[dof_of[t]];
    int64_t *rp = (int64_t *)malloc(sizeof(int64_t) * (nfree + 1));
    int32_t *ci = NULL;
    int64_t nnz = orc_csr_pattern(nc, nd, cd, nfree, rp, &ci);
    double *val = (double *)malloc(sizeof(double) * (nnz > 0 ? nnz : 1)), *rhs = (double *)malloc(sizeof(double) * (nfree > 0 ? nfree : 1));
    double src[3] = {1.0, 2.0, 3.0};
    check(orc_vx_assemble(family, dim, v, nc, c, NULL, 1.0, 2, src, cd, nfree, rp, ci, val, rhs) == 0, "vector assembly");
    double *x = (double *)calloc(nfree > 0 ? nfree : 1, sizeof(double));
    int it = 0;
    double rr = 0.0;
    check(orc_pcg(nfree, rp, ci, val, rhs, x, 1e-10, 5000, &it, &rr, NULL, NULL) == 0, "vector pcg");
    (void)orc_vx_l2_error(family, dim, v, nc, c, cd, x, 1.0, 3);
    free(x);
    free(val);
    free(rhs);
    orc_free(ci);
    free(rp);
    free(cd);
    free(code);
    free(dof_of);
    free(c);
    free(v);
}

int main(void)
{
    for (int dim = 2; dim <= 3; dim++)
        for (int k = 1; k <= 4; k++) {
            run_brick(dim, k, 0);
            if (k <= 3) run_brick(dim, k, 1);
            run_dg(dim, k);
            run_simplex(dim, k, 0);
            if (k <= 3) run_simplex(dim, k, 1);
        }
    for (int dim = 2; dim <= 3; dim++) {
        run_vector(1, dim);
        run_vector(2, dim);
        run_vector(3, dim);
        run_vector(4, dim);
    }
    for (int dim = 2; dim <= 3; dim++)
        for (int k = 1; k <= 3; k++) {
            double X[24], B[64 * 3 * 125], md[64]; /* (k+1)^d x d (k+2)^d at k = 3 */
            int nn = ipow(2, dim);
            for (int a = 0; a < nn; a++)
                for (int r = 0; r < dim; r++) X[a * dim + r] = ((a >> r) & 1) + 0.05 * sin(a + r);
            check(orc_stokes_b_element(dim, k, X, B, md) == 0, "stokes divergence block");
        }
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("sanitized oracle run: all checks passed\n");
    return 0;
}
