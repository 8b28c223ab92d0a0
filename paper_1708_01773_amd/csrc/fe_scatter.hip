// fe_scatter.hip -- K5/K6: deterministic assembly of the element matrices
// and loads into the CSR values, right-hand side and Jacobi diagonal
// (Sect. 3.6 eq. assembly, restricted to free DOFs as in Sect. 10.4; the
// duplicates of the COO build-up of Sect. 11.1 are summed here).
//
// Every CSR entry is produced by exactly one lane, which gathers its
// contributions -- the entries (a, b) of the cells that contain both DOFs --
// in ascending cell order.  There are no atomics, so the values are bitwise
// reproducible.  The contributing (cell, a, b) of an entry are the tensor
// product of the (at most two) cells per axis shared by the row and column
// nodes, and the entry's CSR position is the tensor product of per-axis
// offsets (struct AxisTab): the cell-to-nnz permutation is evaluated, not
// stored, which saves its 4-8 bytes per element entry of HBM traffic.
//
// Two traversals, matched to the two element layouts written by K3:
//  * blocked layout (Q1 scalar, upper triangle packed, E[c/64][t(a,b)][c%64]):
//    one thread per row;
//    consecutive threads own consecutive rows, whose cells are consecutive,
//    so every element read of a wave is contiguous.  The cells around the
//    row's node and their local columns are unrolled at compile time into
//    register accumulators of the row's 3^d stencil; the rows are staged in
//    LDS and the wave writes its rows' CSR range contiguously.
//  * cell-major layout (E[c][a][b]): one wave per row, lanes over 64
//    consecutive CSR positions (two positions per lane and step); entries
//    along an x-run of columns come from consecutive b of the same cell, so
//    reads and writes are both contiguous.  The element-matrix index of an
//    entry is a sum of per-axis terms, tabulated per row in LDS, and every
//    contribution of an entry is loaded before any is added.
#include <algorithm>
#include <type_traits>

#include "fe_internal.h"

namespace fe {


struct RowGeom {
    int64_t I0, I1, I2;     // node indices of the row
    int64_t cl0, cl1, cl2;  // first column node per axis
    int32_t w0, w1, w2;     // column widths per axis
    int64_t start;          // CSR position of the row's first entry
    int32_t c;              // component of the row
    int32_t v0, v1, v2;     // I_r / k
    int32_t m0, m1, m2;     // I_r % k
};

// Cells along one axis shared by row node I (= v k + m) and column node J,
// from comparisons only: an element-interior node lies in cell v alone; a
// vertex node lies in cells v-1 (columns below it) and v (columns above), and
// its diagonal in both (clipped to the mesh).
__device__ __forceinline__ void axis_cells(int64_t I, int32_t v, int32_t m, int64_t J, int32_t n, int32_t &elo,
                                           int32_t &ehi)
{
    if (m != 0) {
        elo = ehi = v;
    } else if (J < I) {
        elo = ehi = v - 1;
    } else if (J > I) {
        elo = ehi = v;
    } else {
        elo = v > 0 ? v - 1 : 0;
        ehi = v < n - 1 ? v : n - 1;
    }
}

__device__ __forceinline__ RowGeom row_geom(const SpaceArgs &s, int64_t row)
{
    RowGeom g;
    const int nc = s.ncomp;
    const int64_t R = row / nc;
    g.c = int(row - R * nc);
    const AxisTab &A0 = s.ax[0], &A1 = s.ax[1], &A2 = s.ax[2];
    const int64_t t0 = R % A0.f, t1 = (R / A0.f) % A1.f, t2 = R / (A0.f * A1.f);
    g.I0 = A0.lo + t0;
    g.I1 = A1.lo + t1;
    g.I2 = A2.lo + t2;
    g.w0 = int32_t(A0.w[t0]);
    g.w1 = int32_t(A1.w[t1]);
    g.w2 = int32_t(A2.w[t2]);
    g.cl0 = A0.cl[t0];
    g.cl1 = A1.cl[t1];
    g.cl2 = A2.cl[t2];
    const int32_t k = s.k;
    g.v0 = int32_t(g.I0 / k);
    g.v1 = int32_t(g.I1 / k);
    g.v2 = int32_t(g.I2 / k);
    g.m0 = int32_t(g.I0 - int64_t(g.v0) * k);
    g.m1 = int32_t(g.I1 - int64_t(g.v1) * k);
    g.m2 = int32_t(g.I2 - int64_t(g.v2) * k);
    const int64_t S = A2.P[t2] * A1.T * A0.T + int64_t(g.w2) * A1.P[t1] * A0.T + int64_t(g.w2) * g.w1 * A0.P[t0];
    g.start = int64_t(nc) * nc * S + int64_t(g.c) * nc * (int64_t(g.w0) * g.w1 * g.w2);
    return g;
}

// ---------------------------------------------------------------------------
// Blocked layout: thread per row, rows staged in LDS, contiguous writes
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Q1 scalar: the 2^DIM cells around a row's node and the 2^DIM local columns
// of each are unrolled at compile time, so every element entry lands in a
// register accumulator of the row's 3^DIM stencil.  The cells are visited in
// ascending id, which is the summation order of every entry (as in the
// cell-major traversal); contributions to fixed columns are accumulated and
// dropped.
// Work units of the Q1 scatter: line-aligned chunks of at most 64 rows (a
// line of nodes along x holds ceil(f0 / 64) of them), taken in strips of
// kQ1Strip lines along y through every plane: strip, then plane, then line
// in the strip, then chunk in the line.  A cell plane's element matrices are
// read again by the next plane of nodes a strip later, not a whole plane of
// nodes later, so the second read finds them in L2.
constexpr int kQ1Strip = 16;
constexpr int kQ1Win = 864;  // staged output values per wave (half of 64 full 3D rows)

__host__ __device__ inline int64_t q1_chunks(const SpaceArgs &s)
{
    const int64_t f0 = s.ax[0].f;
    return f0 == 0 ? 0 : (s.n_rows / f0) * ((f0 + 63) / 64);
}

// First row and row count of chunk c < q1_chunks(s).
__device__ __forceinline__ void q1_chunk_rows(const SpaceArgs &s, int64_t c, int64_t &r0, int &nrows)
{
    const int64_t f0 = s.ax[0].f, f1 = s.ax[1].f, f2 = s.n_rows / f0 / f1;
    const int64_t cpl = (f0 + 63) / 64, full = kQ1Strip * f2 * cpl;
    const int64_t nstrip = (f1 + kQ1Strip - 1) / kQ1Strip;
    const int64_t st = c / full < nstrip - 1 ? c / full : nstrip - 1;
    const int64_t rem = c - st * full;
    const int64_t sy = st == nstrip - 1 ? f1 - st * kQ1Strip : kQ1Strip;  // lines of this strip
    const int64_t z = rem / (sy * cpl), rem2 = rem - z * (sy * cpl);
    const int64_t y = st * kQ1Strip + rem2 / cpl, part = rem2 - (rem2 / cpl) * cpl;
    r0 = (z * f1 + y) * f0 + part * 64;
    nrows = int(f0 - part * 64 < 64 ? f0 - part * 64 : 64);
}

template <int DIM, typename ET>
__device__ __forceinline__ void k5_q1_body(const SpaceArgs &s, const ET *__restrict__ E,
                                           const double *__restrict__ F, double *__restrict__ values,
                                           double *__restrict__ rhs, double *__restrict__ dinv, int64_t bid)
{
    constexpr int NN = 1 << DIM;                // nodes per cell
    constexpr int NT = NN * (NN + 1) / 2;       // stored entries per cell (upper triangle)
    constexpr int NS = DIM == 3 ? 27 : 9;       // stencil entries
    constexpr int CB = 64;                      // cells per block of E
    constexpr int WIN = DIM == 3 ? kQ1Win : 64 * NS;  // 2D: one window holds 64 rows
    __shared__ double stage[4][WIN];
    double *my = stage[threadIdx.x / 64];
    const int lane = threadIdx.x % 64;
    const int64_t chunk = bid * 4 + threadIdx.x / 64;
    if (chunk >= q1_chunks(s)) return;  // the whole wave leaves together
    int64_t r0;
    int nvalid;
    q1_chunk_rows(s, chunk, r0, nvalid);
    const int64_t row = r0 + lane;
    RowGeom g{};
    int len = 0;
    double acc[NS];
#pragma unroll
    for (int t = 0; t < NS; t++) acc[t] = 0.0;
    double fsum = 0.0;
    if (lane < nvalid) {
        g = row_geom(s, row);
        len = g.w0 * g.w1 * g.w2;
        const int64_t n0 = s.ax[0].n, n1 = s.ax[1].n, n2 = s.ax[2].n;
#pragma unroll
        for (int c = 0; c < NN; c++) {
            const int d0 = (c & 1) - 1, d1 = ((c >> 1) & 1) - 1, d2 = DIM == 3 ? ((c >> 2) & 1) - 1 : 0;
            const int64_t e0 = g.I0 + d0, e1 = g.I1 + d1, e2 = g.I2 + d2;
            if (e0 < 0 || e0 >= n0 || e1 < 0 || e1 >= n1 || e2 < 0 || e2 >= n2) continue;
            const int64_t cell = e0 + n0 * (e1 + n1 * e2);
            const int a = -d0 - 2 * d1 - 4 * d2;
            // packed upper triangle: entry (min(a, b), max(a, b))
            const ET *__restrict__ Ec = E + (cell / CB) * (NT * CB) + (cell % CB);
#pragma unroll
            for (int b = 0; b < NN; b++) {
                const int s0 = d0 + (b & 1) + 1, s1 = d1 + ((b >> 1) & 1) + 1;
                const int s2 = DIM == 3 ? d2 + ((b >> 2) & 1) + 1 : 0;
                const int lo = a < b ? a : b, hi = a < b ? b : a;
                const int t = lo * NN - lo * (lo - 1) / 2 + (hi - lo);
                acc[(s2 * 3 + s1) * 3 + s0] += double(Ec[t * CB]);
            }
            fsum += F[cell * NN + a];
        }
    }
    // the wave's rows are consecutive, so their CSR ranges are contiguous
    const int64_t base = __shfl(g.start, 0);
    const int64_t last_start = __shfl(g.start, nvalid - 1);
    const int last_len = __shfl(len, nvalid - 1);
    const int total = int(last_start - base) + last_len;
    const int o0 = int(g.cl0 - (g.I0 - 1)), o1 = int(g.cl1 - (g.I1 - 1));
    const int o2 = DIM == 3 ? int(g.cl2 - (g.I2 - 1)) : 0;
    if (lane < nvalid) {
        dinv[row] = 1.0 / acc[NS / 2];
        rhs[row] = fsum;
    }
    // the wave's output [base, base + total) goes out through windows of WIN
    // values: each row places the entries that fall in the window, then the
    // window is written contiguously
    for (int w = 0; w < total; w += WIN) {
        if (lane < nvalid) {
            const int rel = int(g.start - base) - w;
#pragma unroll
            for (int t = 0; t < NS; t++) {
                const int s0 = t % 3, s1 = (t / 3) % 3, s2 = t / 9;
                const int j0 = s0 - o0, j1 = s1 - o1, j2 = s2 - o2;
                const int pos = rel + (j2 * g.w1 + j1) * g.w0 + j0;
                if (j0 >= 0 && j0 < g.w0 && j1 >= 0 && j1 < g.w1 && j2 >= 0 && j2 < g.w2 && pos >= 0 &&
                    pos < WIN)
                    my[pos] = acc[t];
            }
        }
        wave_lds_fence();
        const int cnt = total - w < WIN ? total - w : WIN;
        for (int t = lane; t < cnt; t += 64) values[base + w + t] = my[t];
        wave_lds_fence();
    }
}

template <int DIM, typename ET>
__global__ __launch_bounds__(256) void k5_q1_kernel(SpaceArgs s, const ET *__restrict__ E, const double *__restrict__ F,
                                                    double *__restrict__ values, double *__restrict__ rhs,
                                                    double *__restrict__ dinv)
{
    k5_q1_body<DIM, ET>(s, E, F, values, rhs, dinv, xcd_block(blockIdx.x, gridDim.x));
}

template <int DIM, typename ET>
__global__ __launch_bounds__(256) void k5_q1_batch_kernel(const AsmJob *__restrict__ jobs,
                                                          const int32_t *__restrict__ boff, int njobs)
{
    int64_t lb, nb;
    const AsmJob &J = jobs[find_job(boff, njobs, lb, nb)];
    k5_q1_body<DIM, ET>(J.s, static_cast<const ET *>(J.E), J.F, J.values, J.rhs, J.dinv, lb);
}

// ---------------------------------------------------------------------------
// Cell-major layout: wave per row, lanes over consecutive CSR positions
// ---------------------------------------------------------------------------
// Per-axis address tables of a row.  Along axis r the column node J = cl_r + j
// (j < w_r <= 2k + 1) shares with the row node I one or two cells e (see
// axis_cells); the element-matrix index of entry (row, column) in cell
// (e0, e1, e2) is a sum of per-axis terms,
//   e_r cs_r nloc^2 + (I_r - e_r k) s_r nloc + (J_r - e_r k) s_r  (s_r = NC (k+1)^r,
//   cs_0 = 1, cs_1 = n0, cs_2 = n0 n1)
// plus c nloc + cc, so a row stores off[r][j][d] for its first (d = 0) and
// second (d = 1) cell along each axis and cnt[r][j] = 1 or 2.
constexpr int kAxMax = 9;  // 2k + 1 for k <= 4

struct RowTables {
    int64_t off[3][kAxMax][2];
    int32_t cnt[3][kAxMax];
};

// One axis of the tables (R compile time, so no field of the row's geometry
// or of the argument struct is indexed at run time, which would put them in
// private memory): lane j < w_R fills column j.
template <int R>
__device__ __forceinline__ void build_axis_table(const SpaceArgs &s, int64_t I, int32_t v, int32_t m, int64_t cl,
                                                 int32_t w, int nc, RowTables &t, int lane)
{
    if (lane < w) {
        const int k = s.k, nloc = s.nloc;
        const int64_t J = cl + lane;
        int32_t elo, ehi;
        axis_cells(I, v, m, J, s.ax[R].n, elo, ehi);
        const int64_t nl2 = int64_t(nloc) * nloc;
        const int64_t cs = R == 0 ? nl2 : (R == 1 ? nl2 * s.ax[0].n : nl2 * s.ax[0].n * s.ax[1].n);
        const int64_t sr = R == 0 ? nc : (R == 1 ? nc * (k + 1) : nc * (k + 1) * (k + 1));
#pragma unroll
        for (int d = 0; d < 2; d++) {
            const int64_t e = elo + (d <= ehi - elo ? d : 0);
            t.off[R][lane][d] = e * cs + (I - e * k) * sr * nloc + (J - e * k) * sr;
        }
        t.cnt[R][lane] = ehi - elo + 1;
    }
}

__device__ __forceinline__ void build_row_tables(const SpaceArgs &s, const RowGeom &g, int nc, RowTables &t,
                                                 int lane)
{
    build_axis_table<0>(s, g.I0, g.v0, g.m0, g.cl0, g.w0, nc, t, lane);
    build_axis_table<1>(s, g.I1, g.v1, g.m1, g.cl1, g.w1, nc, t, lane);
    build_axis_table<2>(s, g.I2, g.v2, g.m2, g.cl2, g.w2, nc, t, lane);
}

// Entry (row, position pos): contributions of cells u = d0 + 2 d1 + 4 d2
// (d_r < cnt_r) loaded together and summed in ascending u, which is
// ascending cell id, the summation order of every CSR entry.  RM bit r says
// whether the row node lies in two cells along axis r; a column shares at
// most the row node's cells, so u with d_r = 1 where bit r is clear are
// never loaded (the bit pattern is the same for the whole row, so each
// pattern is its own instantiation).
template <int NC, typename ET, int RM = 7>
__device__ __forceinline__ double entry_from_tables(const RowTables &t, const ET *__restrict__ E, int64_t base,
                                                    int j0, int j1, int j2)
{
    const int64_t a0 = t.off[0][j0][0], a1 = t.off[0][j0][1];
    const int64_t b0 = t.off[1][j1][0], b1 = t.off[1][j1][1];
    const int64_t c0 = t.off[2][j2][0], c1 = t.off[2][j2][1];
    const int n0 = t.cnt[0][j0], n1 = t.cnt[1][j1], n2 = t.cnt[2][j2];
    double sum = 0.0;
    if constexpr (sizeof(ET) == 4) {
        // FP32 entries: every load is issued unconditionally (a contribution
        // that does not exist reads the first one, which always does, and is
        // skipped in the sum).  Conditional 32-bit loads, widened or not,
        // were each waited for before the next was issued (Q4 elasticity
        // scatter 9.4 ms conditional, 11.5 ms as raw words, 8.1 ms like this).
        ET v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            if ((u & ~RM) != 0) continue;
            const int d0 = u & 1, d1 = (u >> 1) & 1, d2 = u >> 2;
            const bool ok = d0 < n0 && d1 < n1 && d2 < n2;
            v[u] = E[base + (ok ? (d0 ? a1 : a0) + (d1 ? b1 : b0) + (d2 ? c1 : c0) : a0 + b0 + c0)];
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
            if ((u & ~RM) != 0) continue;
            const int d0 = u & 1, d1 = (u >> 1) & 1, d2 = u >> 2;
            if (d0 < n0 && d1 < n1 && d2 < n2) sum += double(v[u]);
        }
    } else {
        // FP64 entries: only the contributions that exist are loaded (at
        // Q3-Q4 most entries have one or two of the eight; unconditional
        // loads took 11.3 instead of 6.9 ms at Q4 elasticity)
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int d0 = u & 1, d1 = (u >> 1) & 1, d2 = u >> 2;
            v[u] = 0.0;
            if (d0 < n0 && d1 < n1 && d2 < n2) v[u] = E[base + (d0 ? a1 : a0) + (d1 ? b1 : b0) + (d2 ? c1 : c0)];
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int d0 = u & 1, d1 = (u >> 1) & 1, d2 = u >> 2;
            if (d0 < n0 && d1 < n1 && d2 < n2) sum += v[u];
        }
    }
    return sum;
}

// Row geometry from the closed forms of the axis tables (no table loads);
// the fields of row_geom.
template <int NC>
__device__ __forceinline__ RowGeom row_geom_closed(const SpaceArgs &s, const AxisClosed (&A)[3], double kinv,
                                                   int64_t row)
{
    RowGeom g;
    const int32_t k = s.k;
    const int32_t r32 = int32_t(row);
    const int32_t R = r32 / NC;
    g.c = r32 - R * NC;
    const int32_t f0 = int32_t(s.ax[0].f), f1 = int32_t(s.ax[1].f);
    const int32_t q = div_exact(R, f0, s.ax[0].finv), t0 = R - q * f0;
    const int32_t t2 = div_exact(q, f1, s.ax[1].finv), t1 = q - t2 * f1;
    int32_t w0, w1, w2, cl0, cl1, cl2, P0, P1, P2;
    axis_row(A[0], k, kinv, A[0].lo + t0, w0, cl0, P0);
    axis_row(A[1], k, kinv, A[1].lo + t1, w1, cl1, P1);
    axis_row(A[2], k, kinv, A[2].lo + t2, w2, cl2, P2);
    g.I0 = A[0].lo + t0;
    g.I1 = A[1].lo + t1;
    g.I2 = A[2].lo + t2;
    g.w0 = w0;
    g.w1 = w1;
    g.w2 = w2;
    g.cl0 = cl0;
    g.cl1 = cl1;
    g.cl2 = cl2;
    g.v0 = div_exact(int32_t(g.I0), k, kinv);
    g.v1 = div_exact(int32_t(g.I1), k, kinv);
    g.v2 = div_exact(int32_t(g.I2), k, kinv);
    g.m0 = int32_t(g.I0) - g.v0 * k;
    g.m1 = int32_t(g.I1) - g.v1 * k;
    g.m2 = int32_t(g.I2) - g.v2 * k;
    const int64_t T0 = s.ax[0].T, T1 = s.ax[1].T;
    const int64_t S = int64_t(P2) * T1 * T0 + int64_t(w2) * P1 * T0 + int64_t(w2) * w1 * P0;
    g.start = int64_t(NC) * NC * S + int64_t(g.c) * NC * (int64_t(w0) * w1 * w2);
    return g;
}

template <int NC, typename ET>
__device__ __forceinline__ void k5_entries_body(const SpaceArgs &s, const ET *__restrict__ E,
                                                const double *__restrict__ F, double *__restrict__ values,
                                                double *__restrict__ rhs, double *__restrict__ dinv, int64_t lb,
                                                int64_t nb)
{
    __shared__ RowTables tabs[4];
    RowTables &t = tabs[threadIdx.x / 64];
    const int lane = threadIdx.x % 64;
    const int64_t nw = nb * 4;
    const int64_t lw = lb * 4 + threadIdx.x / 64;
    const int32_t k = s.k, k1 = k + 1;
    const double kinv = 1.0 / double(k);
    AxisClosed A[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
        A[r].lo = int32_t(s.ax[r].lo);
        A[r].hi = int32_t(s.ax[r].lo + s.ax[r].f - 1);
        A[r].N = int32_t(s.ax[r].N);
        A[r].swlo = A[r].lo * (k + 1) + k * ((A[r].lo + k - 1) / k);
    }
    // A wave takes a node: its NC rows share the geometry and the tables, and
    // their CSR values are one contiguous range of NC len positions (row c
    // starts at c len), streamed as one.
    const int64_t n_nodes = s.n_rows / NC;
    for (int64_t node = lw; node < n_nodes; node += nw) {
        const int64_t row0 = node * NC;
        const RowGeom g = row_geom_closed<NC>(s, A, kinv, row0);
        build_row_tables(s, g, NC, t, lane);
        int32_t e0lo, e0hi, e1lo, e1hi, e2lo, e2hi;  // the node's cells along each axis
        axis_cells(g.I0, g.v0, g.m0, g.I0, s.ax[0].n, e0lo, e0hi);
        axis_cells(g.I1, g.v1, g.m1, g.I1, s.ax[1].n, e1lo, e1hi);
        axis_cells(g.I2, g.v2, g.m2, g.I2, s.ax[2].n, e2lo, e2hi);
        // rhs: lane 8 c + u loads component c of the node's cell u = d0 + 2 d1 + 4 d2
        double fu = 0.0;
        bool fok = false;
        if (lane < 8 * NC) {
            const int u = lane % 8, c = lane / 8;
            const int32_t e0 = e0lo + (u & 1), e1 = e1lo + ((u >> 1) & 1), e2 = e2lo + (u >> 2);
            fok = e0 <= e0hi && e1 <= e1hi && e2 <= e2hi;
            if (fok) {
                const int64_t cell = e0 + int64_t(s.ax[0].n) * (e1 + int64_t(s.ax[1].n) * e2);
                const int la = (int(g.I0 - int64_t(e0) * k) +
                                k1 * (int(g.I1 - int64_t(e1) * k) + k1 * int(g.I2 - int64_t(e2) * k))) * NC + c;
                fu = F[cell * s.nloc + la];
            }
        }
        wave_lds_fence();
        const int wx = g.w0 * NC;   // entries per x-run
        const int len = wx * g.w1 * g.w2;
        // the diagonal node's position in a row (row c's diagonal at c len + pdn + c)
        const int pdn = ((int(g.I2 - g.cl2) * g.w1 + int(g.I1 - g.cl1)) * g.w0 + int(g.I0 - g.cl0)) * NC;
        // floor(p / d) = (p m) >> 20 for m in [2^20 / d, 2^20 / d + 8] (p < 2^12, d <= 27;
        // positions within a row are below len <= 27 * 9 * 9)
        const uint32_t mx = uint32_t(1048576.0f * __builtin_amdgcn_rcpf(float(wx))) + 2u;
        const uint32_t my = uint32_t(1048576.0f * __builtin_amdgcn_rcpf(float(g.w1))) + 2u;
        auto decode = [&](int P, int &c, int &j0, int &j1, int &j2, int &cc) {
            c = NC == 1 ? 0 : (P >= len ? 1 : 0) + (NC == 3 && P >= 2 * len ? 1 : 0);
            const int pos = P - c * len;
            const int q = int((uint32_t(pos) * mx) >> 20), x = pos - q * wx;
            j2 = int((uint32_t(q) * my) >> 20);
            j1 = q - j2 * g.w1;
            j0 = x / NC;
            cc = x - j0 * NC;
        };
        const int total = NC * len;
        // two entries per lane and step (positions P, P + 64), their loads in flight together
        auto entries = [&](auto rm) {
            constexpr int RM = decltype(rm)::value;
            for (int P = lane; P < total; P += 128) {
                int ca, a0, a1, a2, ac, cb = 0, b0 = 0, b1 = 0, b2 = 0, bc = 0;
                decode(P, ca, a0, a1, a2, ac);
                const bool hb = P + 64 < total;
                if (hb) decode(P + 64, cb, b0, b1, b2, bc);
                const double va = entry_from_tables<NC, ET, RM>(t, E, int64_t(ca) * s.nloc + ac, a0, a1, a2);
                const double vb =
                    hb ? entry_from_tables<NC, ET, RM>(t, E, int64_t(cb) * s.nloc + bc, b0, b1, b2) : 0.0;
                values[g.start + P] = va;
                if (P == ca * len + pdn + ca) dinv[row0 + ca] = 1.0 / va;
                if (hb) {
                    values[g.start + P + 64] = vb;
                    if (P + 64 == cb * len + pdn + cb) dinv[row0 + cb] = 1.0 / vb;
                }
            }
        };
        if constexpr (sizeof(ET) == 4) {
            // FP32 loads are unconditional: bound them by the node's cells
            const int rm = __builtin_amdgcn_readfirstlane((e0hi > e0lo ? 1 : 0) | (e1hi > e1lo ? 2 : 0) |
                                                          (e2hi > e2lo ? 4 : 0));
            switch (rm) {
                case 0: entries(std::integral_constant<int, 0>{}); break;
                case 1: entries(std::integral_constant<int, 1>{}); break;
                case 2: entries(std::integral_constant<int, 2>{}); break;
                case 3: entries(std::integral_constant<int, 3>{}); break;
                case 4: entries(std::integral_constant<int, 4>{}); break;
                case 5: entries(std::integral_constant<int, 5>{}); break;
                case 6: entries(std::integral_constant<int, 6>{}); break;
                default: entries(std::integral_constant<int, 7>{}); break;
            }
        } else {
            entries(std::integral_constant<int, 7>{});
        }
        // rhs of each row summed in ascending cell order
#pragma unroll
        for (int c = 0; c < NC; c++) {
            double f = 0.0;
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const double fv = __shfl(fu, 8 * c + u);
                const bool ok = __shfl(int(fok), 8 * c + u) != 0;
                if (ok) f += fv;
            }
            if (lane == 0) rhs[row0 + c] = f;
        }
        wave_lds_fence();
    }
}

template <int NC, typename ET>
__global__ __launch_bounds__(256) void k5_entries_kernel(SpaceArgs s, const ET *__restrict__ E,
                                                         const double *__restrict__ F, double *__restrict__ values,
                                                         double *__restrict__ rhs, double *__restrict__ dinv)
{
    k5_entries_body<NC, ET>(s, E, F, values, rhs, dinv, xcd_block(blockIdx.x, gridDim.x), gridDim.x);
}

template <int NC, typename ET>
__global__ __launch_bounds__(256) void k5_entries_batch_kernel(const AsmJob *__restrict__ jobs,
                                                               const int32_t *__restrict__ boff, int njobs)
{
    int64_t lb, nb;
    const AsmJob &J = jobs[find_job(boff, njobs, lb, nb)];
    k5_entries_body<NC, ET>(J.s, static_cast<const ET *>(J.E), J.F, J.values, J.rhs, J.dinv, lb, nb);
}

fe_status launch_scatter(const SpaceArgs &sa, const ElemLayout &el, const void *ws, double *values, double *rhs,
                         double *dinv, hipStream_t s)
{
    if (sa.n_rows == 0) return FE_OK;
    const double *F = reinterpret_cast<const double *>(static_cast<const char *>(ws) + el.f_offset);
    if (el.cb > 1) {
        // thread per row: 4 waves of one chunk each per block
        const int64_t grid = (q1_chunks(sa) + 3) / 4;
        if (el.cb != 64) return set_error(FE_EINVAL, "unexpected element layout");
#define FE_K5Q(D, T)                                                                                           \
    hipLaunchKernelGGL((k5_q1_kernel<D, T>), dim3(grid), dim3(256), 0, s, sa, static_cast<const T *>(ws), F, values, \
                       rhs, dinv)
        if (sa.dim == 3) {
            if (el.elem_bytes == 8) FE_K5Q(3, double);
            else FE_K5Q(3, float);
        } else {
            if (el.elem_bytes == 8) FE_K5Q(2, double);
            else FE_K5Q(2, float);
        }
#undef FE_K5Q
    } else {
        // wave per row, rows interleaved over a grid that fills the chip
        const int64_t grid = std::min<int64_t>((sa.n_rows / sa.ncomp + 3) / 4, 8192);
#define FE_K5E(NCV, T)                                                                                              \
    hipLaunchKernelGGL((k5_entries_kernel<NCV, T>), dim3(grid), dim3(256), 0, s, sa, static_cast<const T *>(ws), F, \
                       values, rhs, dinv)
        if (sa.ncomp == 1) {
            if (el.elem_bytes == 8) FE_K5E(1, double);
            else FE_K5E(1, float);
        } else if (sa.ncomp == 2) {
            if (el.elem_bytes == 8) FE_K5E(2, double);
            else FE_K5E(2, float);
        } else {
            if (el.elem_bytes == 8) FE_K5E(3, double);
            else FE_K5E(3, float);
        }
#undef FE_K5E
    }
    FE_HIP(hipGetLastError());
    return FE_OK;
}

// Workgroups of one problem in the batched scatter (same shapes as launch_scatter).
int64_t scatter_blocks(const SpaceArgs &sa, const ElemLayout &el)
{
    if (sa.n_rows == 0) return 0;
    if (el.cb > 1) return (q1_chunks(sa) + 3) / 4;
    return std::min<int64_t>((sa.n_rows / sa.ncomp + 3) / 4, 8192);
}

fe_status launch_scatter_batch(const AsmJob &h, const ElemLayout &el, const AsmJob *jobs, const int32_t *boff,
                               int njobs, int grid, hipStream_t s)
{
    if (grid == 0) return FE_OK;
    if (el.cb > 1) {
        if (el.cb != 64) return set_error(FE_EINVAL, "unexpected element layout");
        if (h.s.dim == 3) {
            if (el.elem_bytes == 8)
                hipLaunchKernelGGL((k5_q1_batch_kernel<3, double>), dim3(grid), dim3(256), 0, s, jobs, boff, njobs);
            else
                hipLaunchKernelGGL((k5_q1_batch_kernel<3, float>), dim3(grid), dim3(256), 0, s, jobs, boff, njobs);
        } else {
            if (el.elem_bytes == 8)
                hipLaunchKernelGGL((k5_q1_batch_kernel<2, double>), dim3(grid), dim3(256), 0, s, jobs, boff, njobs);
            else
                hipLaunchKernelGGL((k5_q1_batch_kernel<2, float>), dim3(grid), dim3(256), 0, s, jobs, boff, njobs);
        }
    } else {
#define FE_K5B(NCV, T) \
    hipLaunchKernelGGL((k5_entries_batch_kernel<NCV, T>), dim3(grid), dim3(256), 0, s, jobs, boff, njobs)
        if (h.s.ncomp == 1) {
            if (el.elem_bytes == 8) FE_K5B(1, double);
            else FE_K5B(1, float);
        } else if (h.s.ncomp == 2) {
            if (el.elem_bytes == 8) FE_K5B(2, double);
            else FE_K5B(2, float);
        } else {
            if (el.elem_bytes == 8) FE_K5B(3, double);
            else FE_K5B(3, float);
        }
#undef FE_K5B
    }
    FE_HIP(hipGetLastError());
    return FE_OK;
}

}  // namespace fe
