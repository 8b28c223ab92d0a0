/*
 * fe_oracle_omp.c -- the oracle on all host cores (OpenMP), for the CPU
 * baseline only.
 *
 * THIS FILE IS TEST INFRASTRUCTURE.  It includes the plain oracle
 * (fe_oracle.c) and adds parallel versions of its three timed phases.  Parity
 * runs never use it: they load the single-threaded build of fe_oracle.c.
 *
 *  - Symbolic phase: the incidence of every free DOF in the cells (row ->
 *    (cell, local index) in ascending cell order), then, row-parallel, the
 *    sorted distinct free columns of the row's cells (the same pattern as the
 *    serial COO sort-and-compress, Sect. 11.1).
 *  - Numeric phase: element matrices, loads and Dirichlet data of every cell
 *    in parallel into per-cell buffers; then, row-parallel, each row adds its
 *    contributions cell by cell in ascending order, local column by local
 *    column -- the order of the serial assembly, so values and rhs are
 *    bitwise the serial oracle's.
 *  - Jacobi-PCG (Saad, Alg. 9.1): row-parallel SpMV and vector updates; dot
 *    products summed over fixed chunks of rows whose partial sums are added
 *    in chunk order, so the result does not depend on the thread count.
 */
#include "fe_oracle.c"

#include <omp.h>

int orc_omp_threads(void) { return omp_get_max_threads(); }

/* row -> (cell * nloc + a) for every free local DOF, ascending cell order */
static int64_t *orc_incidence(int64_t ncells, int nloc, const int64_t *cell_dofs, int64_t nfree,
                              int64_t **inc_ptr_out, int64_t *maxinc_out)
{
    int64_t *ptr = (int64_t *)calloc((size_t)nfree + 1, sizeof(int64_t));
    for (int64_t K = 0; K < ncells; K++)
        for (int a = 0; a < nloc; a++) {
            int64_t g = cell_dofs[K * nloc + a];
            if (g >= 0) ptr[g + 1]++;
        }
    int64_t maxinc = 0;
    for (int64_t r = 0; r < nfree; r++) {
        if (ptr[r + 1] > maxinc) maxinc = ptr[r + 1];
        ptr[r + 1] += ptr[r];
    }
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)nfree + 1));
    memcpy(fill, ptr, sizeof(int64_t) * ((size_t)nfree + 1));
    int64_t *inc = (int64_t *)malloc(sizeof(int64_t) * (ptr[nfree] > 0 ? (size_t)ptr[nfree] : 1));
    for (int64_t K = 0; K < ncells; K++)
        for (int a = 0; a < nloc; a++) {
            int64_t g = cell_dofs[K * nloc + a];
            if (g >= 0) inc[fill[g]++] = K * nloc + a;
        }
    free(fill);
    *inc_ptr_out = ptr;
    *maxinc_out = maxinc;
    return inc;
}

/* the sorted distinct free columns of row r into buf; returns their count */
static int64_t orc_row_columns(const int64_t *inc, const int64_t *inc_ptr, int64_t r, int nloc,
                               const int64_t *cell_dofs, int64_t *buf)
{
    int64_t m = 0;
    for (int64_t t = inc_ptr[r]; t < inc_ptr[r + 1]; t++) {
        const int64_t *g = cell_dofs + (inc[t] / nloc) * nloc;
        for (int b = 0; b < nloc; b++)
            if (g[b] >= 0) buf[m++] = g[b];
    }
    qsort(buf, (size_t)m, sizeof(int64_t), cmp_i64);
    int64_t u = 0;
    for (int64_t i = 0; i < m; i++)
        if (i == 0 || buf[i] != buf[i - 1]) buf[u++] = buf[i];
    return u;
}

int64_t orc_omp_csr_pattern(int64_t ncells, int nloc, const int64_t *cell_dofs, int64_t nfree, int64_t *rowptr,
                            int32_t **colind_out)
{
    int64_t *inc_ptr, maxinc;
    int64_t *inc = orc_incidence(ncells, nloc, cell_dofs, nfree, &inc_ptr, &maxinc);
    rowptr[0] = 0;
#pragma omp parallel
    {
        int64_t *buf = (int64_t *)malloc(sizeof(int64_t) * (size_t)(maxinc * nloc + 1));
#pragma omp for schedule(dynamic, 256)
        for (int64_t r = 0; r < nfree; r++)
            rowptr[r + 1] = orc_row_columns(inc, inc_ptr, r, nloc, cell_dofs, buf);
        free(buf);
    }
    for (int64_t r = 0; r < nfree; r++) rowptr[r + 1] += rowptr[r];
    int64_t nnz = rowptr[nfree];
    int32_t *colind = (int32_t *)malloc(sizeof(int32_t) * (nnz > 0 ? (size_t)nnz : 1));
#pragma omp parallel
    {
        int64_t *buf = (int64_t *)malloc(sizeof(int64_t) * (size_t)(maxinc * nloc + 1));
#pragma omp for schedule(dynamic, 256)
        for (int64_t r = 0; r < nfree; r++) {
            int64_t m = orc_row_columns(inc, inc_ptr, r, nloc, cell_dofs, buf);
            for (int64_t i = 0; i < m; i++) colind[rowptr[r] + i] = (int32_t)buf[i];
        }
        free(buf);
    }
    free(inc);
    free(inc_ptr);
    *colind_out = colind;
    return nnz;
}

int orc_omp_assemble(const orc_problem *P, const double *vxyz, const double *coef, const int64_t *cell_dofs,
                     int64_t nfree, const int64_t *rowptr, const int32_t *colind, double *values, double *rhs)
{
    int dim = P->dim, k = P->k;
    int ncomp = P->problem == 1 ? dim : 1;
    int nn = ipow(k + 1, dim);
    int nloc = nn * ncomp;
    int64_t ncells = (int64_t)P->n[0] * P->n[1] * (dim == 3 ? P->n[2] : 1);
    double *E = (double *)malloc(sizeof(double) * (size_t)ncells * nloc * nloc);
    double *Fv = (double *)malloc(sizeof(double) * (size_t)ncells * nloc);
    double *U = (double *)malloc(sizeof(double) * (size_t)ncells * nloc);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
    for (int64_t K = 0; K < ncells; K++) {
        double X[24];
        orc_cell_vertices(dim, P->n, vxyz, K, X);
        double kc = coef ? coef[K] : 1.0;
        if (orc_element_matrix(dim, k, P->problem, X, kc, P->lambda, P->mu, E + K * nloc * nloc) != 0) bad = 1;
        orc_element_load(dim, k, ncomp, X, P->source_kind, P->source, Fv + K * nloc);
        for (int a = 0; a < nn; a++) {
            double x[3];
            orc_node_position(dim, k, X, a, x);
            for (int c = 0; c < ncomp; c++)
                U[K * nloc + a * ncomp + c] =
                    orc_dirichlet_value(P->dirichlet_kind, P->dirichlet_affine, dim, x, c);
        }
    }
    int64_t *inc_ptr, maxinc;
    int64_t *inc = orc_incidence(ncells, nloc, cell_dofs, nfree, &inc_ptr, &maxinc);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = 0; r < nfree; r++) {
        for (int64_t j = rowptr[r]; j < rowptr[r + 1]; j++) values[j] = 0.0;
        double s = 0.0;
        for (int64_t t = inc_ptr[r]; t < inc_ptr[r + 1]; t++) {
            int64_t K = inc[t] / nloc;
            int a = (int)(inc[t] % nloc);
            const int64_t *g = cell_dofs + K * nloc;
            const double *A = E + K * nloc * nloc;
            for (int b = 0; b < nloc; b++) {
                if (g[b] >= 0) values[orc_find(rowptr, colind, r, g[b])] += A[a * nloc + b];
                else s -= A[a * nloc + b] * U[K * nloc + b];
            }
            s += Fv[K * nloc + a];
        }
        rhs[r] = s;
    }
    free(inc);
    free(inc_ptr);
    free(E);
    free(Fv);
    free(U);
    return bad ? -1 : 0;
}

#define ORC_CHUNK 8192

static void orc_omp_spmv(int64_t n, const int64_t *rowptr, const int32_t *colind, const double *val,
                         const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t j = rowptr[i]; j < rowptr[i + 1]; j++) s += val[j] * x[colind[j]];
        y[i] = s;
    }
}

/* sum over fixed chunks of ORC_CHUNK rows, partials added in chunk order */
static double orc_omp_dot(int64_t n, const double *a, const double *b, double *part)
{
    int64_t nc = (n + ORC_CHUNK - 1) / ORC_CHUNK;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; c++) {
        double s = 0.0;
        int64_t e = (c + 1) * ORC_CHUNK < n ? (c + 1) * ORC_CHUNK : n;
        for (int64_t i = c * ORC_CHUNK; i < e; i++) s += a[i] * b[i];
        part[c] = s;
    }
    double s = 0.0;
    for (int64_t c = 0; c < nc; c++) s += part[c];
    return s;
}

int orc_omp_pcg(int64_t n, const int64_t *rowptr, const int32_t *colind, const double *val, const double *b,
                double *x, double rtol, int maxit, int *iters_out, double *relres_out)
{
    double *r = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *q = (double *)malloc(sizeof(double) * n);
    double *dinv = (double *)malloc(sizeof(double) * n);
    double *part = (double *)malloc(sizeof(double) * ((n + ORC_CHUNK - 1) / ORC_CHUNK + 1));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double d = 0.0;
        for (int64_t j = rowptr[i]; j < rowptr[i + 1]; j++)
            if (colind[j] == i) d = val[j];
        dinv[i] = 1.0 / d;
    }
    orc_omp_spmv(n, rowptr, colind, val, x, q);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        r[i] = b[i] - q[i];
        z[i] = dinv[i] * r[i];
        p[i] = z[i];
    }
    double bnorm = sqrt(orc_omp_dot(n, b, b, part));
    double rho = orc_omp_dot(n, r, z, part);
    double rnorm = sqrt(orc_omp_dot(n, r, r, part));
    int it = 0, status = 1;
    if (rnorm <= rtol * bnorm) status = 0;
    while (status == 1 && it < maxit) {
        orc_omp_spmv(n, rowptr, colind, val, p, q);
        double pq = orc_omp_dot(n, p, q, part);
        if (!(pq > 0.0) || !isfinite(pq)) {
            status = 2;
            break;
        }
        double alpha = rho / pq;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; i++) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
            z[i] = dinv[i] * r[i];
        }
        double rho_new = orc_omp_dot(n, r, z, part);
        double beta = rho_new / rho;
        rho = rho_new;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
        it++;
        rnorm = sqrt(orc_omp_dot(n, r, r, part));
        if (rnorm <= rtol * bnorm) status = 0;
    }
    *iters_out = it;
    *relres_out = bnorm > 0 ? rnorm / bnorm : rnorm;
    free(r);
    free(z);
    free(p);
    free(q);
    free(dinv);
    free(part);
    return status;
}
