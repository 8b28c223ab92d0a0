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
//    consecutive CSR positions; entries along an x-run of columns come from
//    consecutive b of the same cell, so reads and writes are both contiguous.
#include <algorithm>

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

// Sum of the contributions to entry (row g, column node J, component cc) of
// the cell-major layout E[c][a][b], ascending in cell id.  NC components.
template <int NC, typename ET>
__device__ __forceinline__ double entry_sum(const SpaceArgs &s, const RowGeom &g, int64_t J0, int64_t J1, int64_t J2,
                                           int cc, const ET *__restrict__ E)
{
    const int k = s.k, k1 = k + 1, nloc = s.nloc;
    const int64_t nl2 = int64_t(nloc) * nloc;
    const int64_t n0 = s.ax[0].n, n1 = s.ax[1].n;
    int32_t e0lo, e0hi, e1lo, e1hi, e2lo, e2hi;
    axis_cells(g.I0, g.v0, g.m0, J0, s.ax[0].n, e0lo, e0hi);
    axis_cells(g.I1, g.v1, g.m1, J1, s.ax[1].n, e1lo, e1hi);
    axis_cells(g.I2, g.v2, g.m2, J2, s.ax[2].n, e2lo, e2hi);
    double sum = 0.0;
    for (int32_t e2 = e2lo; e2 <= e2hi; e2++) {
        const int a2 = int(g.I2 - int64_t(e2) * k), b2 = int(J2 - int64_t(e2) * k);
        for (int32_t e1 = e1lo; e1 <= e1hi; e1++) {
            const int a1 = int(g.I1 - int64_t(e1) * k), b1 = int(J1 - int64_t(e1) * k);
            for (int32_t e0 = e0lo; e0 <= e0hi; e0++) {
                const int a0 = int(g.I0 - int64_t(e0) * k), b0 = int(J0 - int64_t(e0) * k);
                const int64_t cell = e0 + n0 * (e1 + n1 * int64_t(e2));
                const int la = (a0 + k1 * (a1 + k1 * a2)) * NC + g.c;
                const int lb = (b0 + k1 * (b1 + k1 * b2)) * NC + cc;
                sum += double(E[cell * nl2 + int64_t(la) * nloc + lb]);
            }
        }
    }
    return sum;
}

// rhs of a row: loads (with lifting) of every cell holding the node.
__device__ __forceinline__ double row_rhs(const SpaceArgs &s, const RowGeom &g, const double *__restrict__ F)
{
    const int k = s.k, k1 = k + 1, nc = s.ncomp, nloc = s.nloc;
    const int64_t n0 = s.ax[0].n, n1 = s.ax[1].n;
    int32_t e0lo, e0hi, e1lo, e1hi, e2lo, e2hi;
    axis_cells(g.I0, g.v0, g.m0, g.I0, s.ax[0].n, e0lo, e0hi);
    axis_cells(g.I1, g.v1, g.m1, g.I1, s.ax[1].n, e1lo, e1hi);
    axis_cells(g.I2, g.v2, g.m2, g.I2, s.ax[2].n, e2lo, e2hi);
    double f = 0.0;
    for (int64_t e2 = e2lo; e2 <= e2hi; e2++)
        for (int64_t e1 = e1lo; e1 <= e1hi; e1++)
            for (int64_t e0 = e0lo; e0 <= e0hi; e0++) {
                const int64_t cell = e0 + n0 * (e1 + n1 * e2);
                const int la = (int(g.I0 - e0 * k) + k1 * (int(g.I1 - e1 * k) + k1 * int(g.I2 - e2 * k))) * nc + g.c;
                f += F[cell * nloc + la];
            }
    return f;
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
// ascending id, which is the summation order of every entry (as in
// entry_sum); contributions to fixed columns are accumulated and dropped.
template <int DIM, typename ET>
__device__ __forceinline__ void k5_q1_body(const SpaceArgs &s, const ET *__restrict__ E,
                                           const double *__restrict__ F, double *__restrict__ values,
                                           double *__restrict__ rhs, double *__restrict__ dinv, int64_t bid)
{
    constexpr int NN = 1 << DIM;                // nodes per cell
    constexpr int NT = NN * (NN + 1) / 2;       // stored entries per cell (upper triangle)
    constexpr int NS = DIM == 3 ? 27 : 9;       // stencil entries
    constexpr int CB = 64;                      // cells per block of E
    __shared__ double stage[4][64 * NS];
    double *my = stage[threadIdx.x / 64];
    const int lane = threadIdx.x % 64;
    const int64_t r0 = (bid * 4 + threadIdx.x / 64) * 64;
    if (r0 >= s.n_rows) return;  // the whole wave leaves together
    const int nvalid = int(s.n_rows - r0 < 64 ? s.n_rows - r0 : 64);
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
    if (lane < nvalid) {
        double *out = my + (g.start - base);
        const int o0 = int(g.cl0 - (g.I0 - 1)), o1 = int(g.cl1 - (g.I1 - 1));
        const int o2 = DIM == 3 ? int(g.cl2 - (g.I2 - 1)) : 0;
#pragma unroll
        for (int t = 0; t < NS; t++) {
            const int s0 = t % 3, s1 = (t / 3) % 3, s2 = t / 9;
            const int j0 = s0 - o0, j1 = s1 - o1, j2 = s2 - o2;
            if (j0 >= 0 && j0 < g.w0 && j1 >= 0 && j1 < g.w1 && j2 >= 0 && j2 < g.w2)
                out[(j2 * g.w1 + j1) * g.w0 + j0] = acc[t];
        }
        dinv[row] = 1.0 / acc[NS / 2];
        rhs[row] = fsum;
    }
    wave_lds_fence();
    for (int t = lane; t < total; t += 64) values[base + t] = my[t];
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
template <int NC, typename ET>
__device__ __forceinline__ void k5_entries_body(const SpaceArgs &s, const ET *__restrict__ E,
                                                const double *__restrict__ F, double *__restrict__ values,
                                                double *__restrict__ rhs, double *__restrict__ dinv, int64_t lb,
                                                int64_t nb)
{
    const int lane = threadIdx.x % 64;
    const int64_t nw = nb * 4;
    const int64_t lw = lb * 4 + threadIdx.x / 64;
    for (int64_t row = lw; row < s.n_rows; row += nw) {
        const RowGeom g = row_geom(s, row);
        const int wx = g.w0 * NC;   // entries per x-run
        const int len = wx * g.w1 * g.w2;
        // mixed-radix position (j2, j1, x) of this lane's entry, advanced by 64 per step
        int x = lane, j1 = 0, j2 = 0;
        while (x >= wx) {
            x -= wx;
            if (++j1 == g.w1) {
                j1 = 0;
                j2++;
            }
        }
        for (int pos = lane; pos < len; pos += 64) {
            const int j0 = x / NC, cc = x - j0 * NC;
            const int64_t J0 = g.cl0 + j0, J1 = g.cl1 + j1, J2 = g.cl2 + j2;
            const double v = entry_sum<NC>(s, g, J0, J1, J2, cc, E);
            values[g.start + pos] = v;
            if (J0 == g.I0 && J1 == g.I1 && J2 == g.I2 && cc == g.c) dinv[row] = 1.0 / v;
            x += 64;
            while (x >= wx) {
                x -= wx;
                if (++j1 == g.w1) {
                    j1 = 0;
                    j2++;
                }
            }
        }
        if (lane == 0) rhs[row] = row_rhs(s, g, F);
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
        // thread per row: 4 waves of 64 rows per block
        const int64_t grid = (sa.n_rows + 255) / 256;
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
        const int64_t grid = std::min<int64_t>((sa.n_rows + 3) / 4, 8192);
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
    if (el.cb > 1) return (sa.n_rows + 255) / 256;
    return std::min<int64_t>((sa.n_rows + 3) / 4, 8192);
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
