// fe_scatter.hip -- K5/K6: deterministic assembly of the element matrices
// and loads into the CSR values, right-hand side and Jacobi diagonal
// (Sect. 3.6 eq. assembly, restricted to free DOFs as in Sect. 10.4; the
// duplicates of the COO build-up of Sect. 11.1 are summed here).
//
// Every CSR entry is produced by exactly one thread, which gathers its
// contributions -- the entries (a, b) of the cells that contain both DOFs --
// in ascending cell order.  There are no atomics, so the values are bitwise
// reproducible.  The contributing (cell, a, b) of an entry are the tensor
// product of the (at most two) cells per axis shared by the row and column
// nodes, and the entry's CSR position is the tensor product of per-axis
// offsets (struct AxisTab): the cell-to-nnz permutation is evaluated, not
// stored, which saves its 4-8 bytes per element entry of HBM traffic.
#include "fe_internal.h"

namespace fe {

template <typename ET>
__global__ __launch_bounds__(256) void k5_scatter_kernel(SpaceArgs s, const ET *__restrict__ E, int cb,
                                                         const double *__restrict__ F, double *__restrict__ values,
                                                         double *__restrict__ rhs, double *__restrict__ dinv)
{
    const int64_t bid = xcd_block(blockIdx.x, gridDim.x);
    const int64_t row = bid * blockDim.x + threadIdx.x;
    if (row >= s.n_rows) return;
    const int nc = s.ncomp, k = s.k, k1 = k + 1, nloc = s.nloc;
    const int64_t nl2 = int64_t(nloc) * nloc;
    const int64_t R = row / nc;
    const int c = int(row % nc);
    const AxisTab &A0 = s.ax[0], &A1 = s.ax[1], &A2 = s.ax[2];
    const int64_t t0 = R % A0.f, t1 = (R / A0.f) % A1.f, t2 = R / (A0.f * A1.f);
    const int64_t I0 = A0.lo + t0, I1 = A1.lo + t1, I2 = A2.lo + t2;
    const int64_t w0 = A0.w[t0], w1 = A1.w[t1], w2 = A2.w[t2];
    const int64_t cl0 = A0.cl[t0], cl1 = A1.cl[t1], cl2 = A2.cl[t2];
    const int64_t S = A2.P[t2] * A1.T * A0.T + w2 * A1.P[t1] * A0.T + w2 * w1 * A0.P[t0];
    int64_t pos = int64_t(nc) * nc * S + int64_t(c) * nc * (w0 * w1 * w2);
    const int64_t n0 = A0.n, n1 = A1.n;
    for (int64_t J2 = cl2; J2 < cl2 + w2; J2++) {
        int64_t e2lo, e2hi;
        shared_cells(I2, J2, k, A2.n, e2lo, e2hi);
        for (int64_t J1 = cl1; J1 < cl1 + w1; J1++) {
            int64_t e1lo, e1hi;
            shared_cells(I1, J1, k, A1.n, e1lo, e1hi);
            for (int64_t J0 = cl0; J0 < cl0 + w0; J0++) {
                int64_t e0lo, e0hi;
                shared_cells(I0, J0, k, A0.n, e0lo, e0hi);
                for (int cc = 0; cc < nc; cc++) {
                    double sum = 0.0;
                    for (int64_t e2 = e2lo; e2 <= e2hi; e2++) {
                        const int a2 = int(I2 - e2 * k), b2 = int(J2 - e2 * k);
                        for (int64_t e1 = e1lo; e1 <= e1hi; e1++) {
                            const int a1 = int(I1 - e1 * k), b1 = int(J1 - e1 * k);
                            for (int64_t e0 = e0lo; e0 <= e0hi; e0++) {
                                const int a0 = int(I0 - e0 * k), b0 = int(J0 - e0 * k);
                                const int64_t cell = e0 + n0 * (e1 + n1 * e2);
                                const int la = (a0 + k1 * (a1 + k1 * a2)) * nc + c;
                                const int lb = (b0 + k1 * (b1 + k1 * b2)) * nc + cc;
                                const int64_t idx = ((cell / cb) * nl2 + int64_t(la) * nloc + lb) * cb + cell % cb;
                                sum += double(E[idx]);
                            }
                        }
                    }
                    values[pos++] = sum;
                    if (J0 == I0 && J1 == I1 && J2 == I2 && cc == c) dinv[row] = 1.0 / sum;
                }
            }
        }
    }
    // right-hand side: loads (with lifting) of every cell holding the node
    int64_t e2lo, e2hi, e1lo, e1hi, e0lo, e0hi;
    shared_cells(I2, I2, k, A2.n, e2lo, e2hi);
    shared_cells(I1, I1, k, A1.n, e1lo, e1hi);
    shared_cells(I0, I0, k, A0.n, e0lo, e0hi);
    double f = 0.0;
    for (int64_t e2 = e2lo; e2 <= e2hi; e2++)
        for (int64_t e1 = e1lo; e1 <= e1hi; e1++)
            for (int64_t e0 = e0lo; e0 <= e0hi; e0++) {
                const int64_t cell = e0 + n0 * (e1 + n1 * e2);
                const int la = (int(I0 - e0 * k) + k1 * (int(I1 - e1 * k) + k1 * int(I2 - e2 * k))) * nc + c;
                f += F[cell * nloc + la];
            }
    rhs[row] = f;
}

fe_status launch_scatter(const SpaceArgs &sa, const ElemLayout &el, const void *ws, double *values, double *rhs,
                         double *dinv, hipStream_t s)
{
    if (sa.n_rows == 0) return FE_OK;
    const double *F = reinterpret_cast<const double *>(static_cast<const char *>(ws) + el.f_offset);
    const int64_t grid = (sa.n_rows + 255) / 256;
    if (el.elem_bytes == 8)
        hipLaunchKernelGGL(k5_scatter_kernel<double>, dim3(grid), dim3(256), 0, s, sa,
                           static_cast<const double *>(ws), el.cb, F, values, rhs, dinv);
    else
        hipLaunchKernelGGL(k5_scatter_kernel<float>, dim3(grid), dim3(256), 0, s, sa,
                           static_cast<const float *>(ws), el.cb, F, values, rhs, dinv);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

}  // namespace fe
