// fe_setup.hip -- order-dependent set-up of a structured mesh: reference
// tables, the canonical DOF numbering (cell-to-DOF map), the CSR pattern of
// the free-free system and the explicit cell-to-nnz permutation.
//
// The pattern is the set of free DOF pairs that share a cell (the entries the
// COO build-up of Sect. 11.1 would create).  On a structured brick the
// pattern, and the position of every element entry inside it, factor into
// per-axis intervals (struct AxisTab), so the set-up is a handful of integer
// kernels instead of a sort of all element entries.
#include <cmath>
#include <vector>

#include "fe_internal.h"

namespace fe {

// ---------------------------------------------------------------------------
// Reference tables (Sect. 3.7 Gauss-Legendre rule; Sect. 3.4 eq. lagbas on the
// equidistant nodes of Sect. 3.15)
// ---------------------------------------------------------------------------
void gauss_legendre_01(int n, double *x, double *w)
{
    // Legendre roots by Newton's method from the cosine initial guess, then
    // mapped from [-1,1] to [0,1].
    for (int i = 0; i < n; i++) {
        double t = std::cos(M_PI * (4.0 * i + 3.0) / (4.0 * n + 2.0));
        double deriv = 1.0;
        for (int it = 0; it < 60; it++) {
            double pm1 = 1.0, p = t;
            for (int m = 2; m <= n; m++) {
                double pn = ((2 * m - 1) * t * p - (m - 1) * pm1) / m;
                pm1 = p;
                p = pn;
            }
            if (n == 1) { pm1 = 1.0; p = t; }
            deriv = n * (pm1 - t * p) / (1.0 - t * t);
            double step = p / deriv;
            t -= step;
            if (std::fabs(step) <= 1e-16 * std::fabs(t) + 1e-300) break;
        }
        double pm1 = 1.0, p = t;
        for (int m = 2; m <= n; m++) {
            double pn = ((2 * m - 1) * t * p - (m - 1) * pm1) / m;
            pm1 = p;
            p = pn;
        }
        deriv = n * (pm1 - t * p) / (1.0 - t * t);
        x[n - 1 - i] = 0.5 + 0.5 * t;
        w[n - 1 - i] = 1.0 / ((1.0 - t * t) * deriv * deriv);
    }
}

void lagrange_1d(int k, int i, double x, double &val, double &der)
{
    const double xi = double(i) / k;
    double den = 1.0;
    for (int s = 0; s <= k; s++)
        if (s != i) den *= xi - double(s) / k;
    double v = 1.0, d = 0.0;
    for (int s = 0; s <= k; s++) {
        if (s == i) continue;
        // product rule: d/dx prod (x - x_s) accumulated on the fly
        d = d * (x - double(s) / k) + v;
        v *= x - double(s) / k;
    }
    val = v / den;
    der = d / den;
}

void ref_tables(int k, RefTables &t)
{
    const int nq = k + 1;
    gauss_legendre_01(nq, t.gx, t.gw);
    for (int i = 0; i <= k; i++)
        for (int q = 0; q < nq; q++) lagrange_1d(k, i, t.gx[q], t.L[i * nq + q], t.D[i * nq + q]);
}

// ---------------------------------------------------------------------------
// Per-axis interval tables
// ---------------------------------------------------------------------------
static void axis_table(int64_t n, int64_t N, int k, bool lo_fixed, bool hi_fixed, std::vector<int64_t> &cl,
                       std::vector<int64_t> &w, std::vector<int64_t> &P, int64_t &lo, int64_t &f, int64_t &T)
{
    lo = lo_fixed ? 1 : 0;
    int64_t hi = hi_fixed ? N - 1 : N;
    f = hi >= lo ? hi - lo + 1 : 0;
    cl.assign(f, 0);
    w.assign(f, 0);
    P.assign(f, 0);
    T = 0;
    for (int64_t t = 0; t < f; t++) {
        int64_t i = lo + t, a, b;
        if (N == 0) {
            a = b = 0;
        } else if (i % k == 0) {
            a = i - k;
            b = i + k;
        } else {
            a = (i / k) * k;
            b = a + k;
        }
        if (a < lo) a = lo;
        if (b > hi) b = hi;
        if (b > N) b = N;
        cl[t] = a;
        w[t] = b - a + 1;
        P[t] = T;
        T += w[t];
    }
    (void)n;
}

fe_status build_space(fe_mesh mesh, int k, int ncomp, uint32_t faces, Space &sp, hipStream_t s)
{
    free_space(sp);
    SpaceArgs &a = sp.args;
    a.dim = mesh->dim;
    a.k = k;
    a.ncomp = ncomp;
    a.nn = 1;
    for (int r = 0; r < mesh->dim; r++) a.nn *= (k + 1);
    a.nloc = a.nn * ncomp;
    a.ncells = mesh->ncells;
    std::vector<int64_t> cl[3], w[3], P[3];
    int64_t total = 0;
    for (int r = 0; r < 3; r++) {
        AxisTab &t = a.ax[r];
        const bool active = r < mesh->dim;
        t.n = active ? mesh->n[r] : 1;
        t.N = active ? int64_t(mesh->n[r]) * k : 0;
        const bool lo_fixed = active && ((faces >> (2 * r)) & 1u);
        const bool hi_fixed = active && ((faces >> (2 * r + 1)) & 1u);
        axis_table(t.n, t.N, k, lo_fixed, hi_fixed, cl[r], w[r], P[r], t.lo, t.f, t.T);
        t.finv = t.f > 0 ? 1.0 / double(t.f) : 0.0;
        total += 3 * t.f;
    }
    int64_t nfree_nodes = a.ax[0].f * a.ax[1].f * a.ax[2].f;
    a.n_rows = nfree_nodes * ncomp;
    a.nnz = int64_t(ncomp) * ncomp * a.ax[0].T * a.ax[1].T * a.ax[2].T;
    if (a.n_rows >= (int64_t(1) << 31))
        return set_error(FE_EINVAL, "system has 2^31 or more rows; column indices are int32");
    std::vector<int64_t> host(total > 0 ? total : 1);
    int64_t off = 0;
    int64_t offs[3];
    for (int r = 0; r < 3; r++) {
        offs[r] = off;
        const int64_t f = a.ax[r].f;
        for (int64_t t = 0; t < f; t++) {
            host[off + t] = cl[r][t];
            host[off + f + t] = w[r][t];
            host[off + 2 * f + t] = P[r][t];
        }
        off += 3 * f;
    }
    FE_HIP(hipMalloc(&sp.d_axis, sizeof(int64_t) * host.size()));
    FE_HIP(hipMemcpyAsync(sp.d_axis, host.data(), sizeof(int64_t) * host.size(), hipMemcpyHostToDevice, s));
    for (int r = 0; r < 3; r++) {
        const int64_t f = a.ax[r].f;
        a.ax[r].cl = sp.d_axis + offs[r];
        a.ax[r].w = sp.d_axis + offs[r] + f;
        a.ax[r].P = sp.d_axis + offs[r] + 2 * f;
    }
    FE_HIP(hipMalloc(&sp.d_cell_dofs, sizeof(int32_t) * size_t(a.ncells) * a.nloc));
    MeshArgs ma{};
    ma.n0 = a.ax[0].n;
    ma.n1 = a.ax[1].n;
    ma.n2 = a.ax[2].n;
    fe_status st = launch_cell_dofs(a, ma, sp.d_cell_dofs, s);
    if (st != FE_OK) return st;
    // the host table above must outlive the copy
    FE_HIP(hipStreamSynchronize(s));
    sp.k = k;
    sp.ncomp = ncomp;
    sp.faces = faces;
    sp.valid = true;
    return FE_OK;
}

void space_sizes(int dim, const int32_t *n, int k, int ncomp, uint32_t faces, int64_t &n_rows, int64_t &nnz)
{
    std::vector<int64_t> cl, w, P;
    int64_t f[3] = {1, 1, 1}, T[3] = {1, 1, 1};
    for (int r = 0; r < dim; r++) {
        int64_t lo;
        axis_table(n[r], int64_t(n[r]) * k, k, (faces >> (2 * r)) & 1u, (faces >> (2 * r + 1)) & 1u, cl, w, P, lo,
                   f[r], T[r]);
    }
    n_rows = f[0] * f[1] * f[2] * ncomp;
    nnz = int64_t(ncomp) * ncomp * T[0] * T[1] * T[2];
}

void free_space(Space &sp)
{
    if (sp.d_axis) (void)hipFree(sp.d_axis);
    if (sp.d_cell_dofs) (void)hipFree(sp.d_cell_dofs);
    sp.d_axis = nullptr;
    sp.d_cell_dofs = nullptr;
    sp.valid = false;
}

// ---------------------------------------------------------------------------
// Device helpers: free-rank and DOF code of a lattice node
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool node_free(const SpaceArgs &s, const int64_t I[3])
{
    for (int r = 0; r < 3; r++) {
        const int64_t t = I[r] - s.ax[r].lo;
        if (t < 0 || t >= s.ax[r].f) return false;
    }
    return true;
}

// Number of free indices of axis r strictly below node index i.
__device__ __forceinline__ int64_t free_below(const AxisTab &t, int64_t i)
{
    int64_t v = i - t.lo;
    return v < 0 ? 0 : (v > t.f ? t.f : v);
}

// DOF code of component c of lattice node I: free DOF id, or -1 - fixed id.
// Free nodes are ranked lexicographically; a fixed node's rank is its
// lexicographic id minus the number of free nodes before it.
__device__ __forceinline__ int64_t dof_code(const SpaceArgs &s, const int64_t I[3], int c)
{
    const AxisTab &a0 = s.ax[0], &a1 = s.ax[1], &a2 = s.ax[2];
    if (node_free(s, I)) {
        const int64_t rank = (I[0] - a0.lo) + a0.f * ((I[1] - a1.lo) + a1.f * (I[2] - a2.lo));
        return rank * s.ncomp + c;
    }
    const int64_t id = I[0] + (a0.N + 1) * (I[1] + (a1.N + 1) * I[2]);
    // free nodes with lexicographic id below this node
    int64_t before = free_below(a2, I[2]) * a1.f * a0.f;
    const bool z_free = I[2] >= a2.lo && I[2] - a2.lo < a2.f;
    if (z_free) {
        before += free_below(a1, I[1]) * a0.f;
        const bool y_free = I[1] >= a1.lo && I[1] - a1.lo < a1.f;
        if (y_free) before += free_below(a0, I[0]);
    }
    const int64_t frank = id - before;
    return -1 - (frank * s.ncomp + c);
}

__global__ void cell_dofs_kernel(SpaceArgs s, int32_t *out)
{
    const int64_t total = s.ncells * s.nloc;
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t cell = t / s.nloc;
        const int l = int(t % s.nloc);
        const int a = l / s.ncomp, c = l % s.ncomp;
        const int k1 = s.k + 1;
        const int64_t e0 = cell % s.ax[0].n, e1 = (cell / s.ax[0].n) % s.ax[1].n,
                      e2 = cell / (int64_t(s.ax[0].n) * s.ax[1].n);
        int64_t I[3] = {e0 * s.k + a % k1, e1 * s.k + (a / k1) % k1, 0};
        if (s.dim == 3) I[2] = e2 * s.k + a / (k1 * k1);
        out[t] = int32_t(dof_code(s, I, c));
    }
}

fe_status launch_cell_dofs(const SpaceArgs &sa, const MeshArgs &, int32_t *out, hipStream_t s)
{
    const int64_t total = sa.ncells * sa.nloc;
    if (total == 0) return FE_OK;
    const int block = 256;
    int64_t grid = (total + block - 1) / block;
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(cell_dofs_kernel, dim3(grid), dim3(block), 0, s, sa, out);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

// ---------------------------------------------------------------------------
// Row start of DOF row (free node offsets t0,t1,t2; component c):
//   S = P2 T1 T0 + w2 P1 T0 + w2 w1 P0   (nodes in earlier rows)
//   rowptr = ncomp^2 S + c ncomp (w0 w1 w2)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t row_start(const SpaceArgs &s, int64_t t0, int64_t t1, int64_t t2, int c,
                                             int64_t &len_nodes)
{
    const AxisTab &a0 = s.ax[0], &a1 = s.ax[1], &a2 = s.ax[2];
    const int64_t w0 = a0.w[t0], w1 = a1.w[t1], w2 = a2.w[t2];
    const int64_t S = a2.P[t2] * a1.T * a0.T + w2 * a1.P[t1] * a0.T + w2 * w1 * a0.P[t0];
    len_nodes = w0 * w1 * w2;
    return int64_t(s.ncomp) * s.ncomp * S + int64_t(c) * s.ncomp * len_nodes;
}

__global__ void pattern_kernel(SpaceArgs s, int64_t *rowptr, int32_t *colind)
{
    const int64_t row = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (row > s.n_rows) return;
    if (row == s.n_rows) {
        rowptr[row] = s.nnz;
        return;
    }
    const int64_t R = row / s.ncomp;
    const int c = int(row % s.ncomp);
    const AxisTab &a0 = s.ax[0], &a1 = s.ax[1], &a2 = s.ax[2];
    const int64_t t0 = R % a0.f, t1 = (R / a0.f) % a1.f, t2 = R / (a0.f * a1.f);
    int64_t len;
    const int64_t start = row_start(s, t0, t1, t2, c, len);
    rowptr[row] = start;
    const int64_t c0 = a0.cl[t0] - a0.lo, c1 = a1.cl[t1] - a1.lo, c2 = a2.cl[t2] - a2.lo;
    const int64_t w0 = a0.w[t0], w1 = a1.w[t1], w2 = a2.w[t2];
    int64_t p = start;
    for (int64_t j2 = 0; j2 < w2; j2++)
        for (int64_t j1 = 0; j1 < w1; j1++) {
            const int64_t base = c0 + a0.f * ((c1 + j1) + a1.f * (c2 + j2));
            for (int64_t j0 = 0; j0 < w0; j0++)
                for (int cc = 0; cc < s.ncomp; cc++) colind[p++] = int32_t((base + j0) * s.ncomp + cc);
        }
}

fe_status launch_pattern(const SpaceArgs &sa, int64_t *rowptr, int32_t *colind, hipStream_t s)
{
    const int block = 256;
    const int64_t grid = (sa.n_rows + 1 + block - 1) / block;
    hipLaunchKernelGGL(pattern_kernel, dim3(grid), dim3(block), 0, s, sa, rowptr, colind);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

// ---------------------------------------------------------------------------
// Explicit cell-to-nnz permutation: for element entry (a, b) of cell c with
// both DOFs free, the CSR position is rowptr(row of a) + the position of b's
// column inside that row, a tensor product of per-axis offsets.
// ---------------------------------------------------------------------------
__global__ void permutation_kernel(SpaceArgs s, int64_t *perm)
{
    const int64_t nl2 = int64_t(s.nloc) * s.nloc;
    const int64_t total = s.ncells * nl2;
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < total;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t cell = t / nl2;
        const int64_t ab = t % nl2;
        const int la = int(ab / s.nloc), lb = int(ab % s.nloc);
        const int a = la / s.ncomp, ca = la % s.ncomp, b = lb / s.ncomp, cbc = lb % s.ncomp;
        const int k1 = s.k + 1;
        const int64_t e[3] = {cell % s.ax[0].n, (cell / s.ax[0].n) % s.ax[1].n,
                              cell / (int64_t(s.ax[0].n) * s.ax[1].n)};
        const int ar[3] = {a % k1, (a / k1) % k1, a / (k1 * k1)};
        const int br[3] = {b % k1, (b / k1) % k1, b / (k1 * k1)};
        int64_t I[3], J[3];
        for (int r = 0; r < 3; r++) {
            const bool act = r < s.dim;
            I[r] = act ? e[r] * s.k + ar[r] : 0;
            J[r] = act ? e[r] * s.k + br[r] : 0;
        }
        if (!node_free(s, I) || !node_free(s, J)) {
            perm[t] = -1;
            continue;
        }
        const int64_t t0 = I[0] - s.ax[0].lo, t1 = I[1] - s.ax[1].lo, t2 = I[2] - s.ax[2].lo;
        int64_t len;
        const int64_t start = row_start(s, t0, t1, t2, ca, len);
        const int64_t w0 = s.ax[0].w[t0], w1 = s.ax[1].w[t1];
        const int64_t pos = ((J[2] - s.ax[2].cl[t2]) * w1 + (J[1] - s.ax[1].cl[t1])) * w0 + (J[0] - s.ax[0].cl[t0]);
        perm[t] = start + pos * s.ncomp + cbc;
    }
}

fe_status launch_permutation(const SpaceArgs &sa, const MeshArgs &, int64_t *perm, hipStream_t s)
{
    const int64_t total = sa.ncells * int64_t(sa.nloc) * sa.nloc;
    if (total == 0) return FE_OK;
    const int block = 256;
    int64_t grid = (total + block - 1) / block;
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(permutation_kernel, dim3(grid), dim3(block), 0, s, sa, perm);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

}  // namespace fe
