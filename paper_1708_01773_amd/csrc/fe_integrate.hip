// fe_integrate.hip -- K3: cell-wise numerical integration of the Galerkin
// element matrices and loads (Sect. 3.7 eq. fematrix, the element loop of the
// Poisson example in Sect. 8.5), on the reference cell [0,1]^d with the
// order-1 geometry map and tensor Gauss-Legendre quadrature of k+1 points per
// direction.  Geometry (J, det J, J^-1) is always FP64.
//
// Poisson:    A_ab = sum_q w_q k_K |det J_q| grad phi_a . grad phi_b
// Elasticity: A_(a,i),(b,j) = sum_q w_q k_K |det J_q|
//               [lambda d_i phi_a d_j phi_b + mu (delta_ij grad phi_a . grad phi_b + d_j phi_a d_i phi_b)]
// Load:       F_(a,c) = sum_q w_q |det J_q| f_c(x_q) phi_a(xi_q)
// Lifting:    F_a -= sum_{b fixed} A_ab u_D(b)   (Sect. 10.4)
#include <cmath>
#include <type_traits>

#include "fe_geom.h"
#include "fe_internal.h"

namespace fe {

ElemLayout elem_layout(const SpaceArgs &sa, int precision)
{
    ElemLayout el{};
    const bool q1_scalar = sa.k == 1 && sa.ncomp == 1;
    el.cb = q1_scalar ? 64 : 1;
    el.packed = q1_scalar ? 1 : 0;
    el.ne = q1_scalar ? sa.nloc * (sa.nloc + 1) / 2 : sa.nloc * sa.nloc;
    el.elem_bytes = precision == FE_FP64 ? 8 : 4;
    const int64_t cells_pad = (sa.ncells + el.cb - 1) / el.cb * el.cb;
    el.e_bytes = (size_t(cells_pad) * el.ne * el.elem_bytes + 255) / 256 * 256;
    el.f_offset = el.e_bytes;
    el.total = el.f_offset + (size_t(sa.ncells) * sa.nloc * sizeof(double) + 255) / 256 * 256;
    return el;
}

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double source_value(const ProblemArgs &p, int dim, const double *x, int c)
{
    if (p.source_kind == FE_SOURCE_CONST) return p.source[c];
    if (p.source_kind == FE_SOURCE_SINPROD) {
        double s = 1.0;
        for (int r = 0; r < dim; r++) s *= sin(M_PI * x[r]);
        return p.source[c] * dim * (M_PI * M_PI) * s;
    }
    return 0.0;
}

// ---------------------------------------------------------------------------
// Q1 scalar kernel: one thread per cell, element matrix in registers (the 36
// upper-triangle entries in 3D), written in the blocked layout
// E[(c/64)][a*8+b][c%64] so that a wave's stores of one entry are 512
// contiguous bytes.  Q1 is HBM-bound (6 flop per byte of E) and its 8 x 8 x 24
// product would fill a quarter of a 16 x 16 matrix tile, so it runs on the
// vector units in every precision.  PREC > 0: the two GEMM operands (the
// gradients, and the gradients times w_q k |det J_q|) are rounded to FP32 /
// FP16 / BF16 and accumulated in FP32, the result stored as FP32; for FP16 /
// BF16 they are first scaled by per-cell powers of two (undone exactly).
// ---------------------------------------------------------------------------
template <int PREC>
__device__ __forceinline__ float round_in(double v)
{
    if (PREC == FE_FP16) return float(_Float16(float(v)));
    if (PREC == FE_BF16) return float(__bf16(float(v)));
    return float(v);
}

template <int DIM, int PREC>
__device__ __forceinline__ void k3_q1_body(const SpaceArgs &s, const MeshArgs &m, const ProblemArgs &p,
                                           const RefTables &rt, void *__restrict__ Ev, double *__restrict__ F,
                                           int64_t bid)
{
    constexpr int NN = 1 << DIM;
    constexpr int NT = NN * (NN + 1) / 2;
    using Acc = typename std::conditional<PREC == FE_FP64, double, float>::type;
    const int64_t cell = bid * blockDim.x + threadIdx.x;
    if (cell >= s.ncells) return;
    double X[NN][3];
    load_vertices<DIM>(m, cell, X);
    const double coef = m.coef ? m.coef[cell] : 1.0;
    // per-cell operand scaling for FP16 / BF16
    double alpha = 1.0, beta = 1.0;
    if (PREC == FE_FP16 || PREC == FE_BF16) {
        double wmax = 0.0, det0 = 0.0;
#pragma unroll
        for (int q = 0; q < NN; q++) {
            const int q0 = q & 1, q1 = (q >> 1) & 1, q2 = (q >> 2) & 1;
            const double xi[3] = {rt.gx[q0], rt.gx[q1], DIM == 3 ? rt.gx[q2] : 0.0};
            double J[9], Ji[9], xq[3];
            const double det = geometry<DIM>(X, xi, J, Ji, xq);
            if (q == 0) det0 = det;
            wmax = fmax(wmax, rt.gw[q0] * rt.gw[q1] * (DIM == 3 ? rt.gw[q2] : 1.0) * fabs(det) * coef);
        }
        const double h = DIM == 3 ? cbrt(fabs(det0)) : sqrt(fabs(det0));
        alpha = exp2(floor(log2(h > 0.0 ? h : 1.0)));
        beta = alpha * (wmax > 0.0 ? exp2(-floor(log2(wmax))) : 1.0);
    }
    Acc acc[NT];
#pragma unroll
    for (int t = 0; t < NT; t++) acc[t] = Acc(0);
    double fl[NN];
#pragma unroll
    for (int a = 0; a < NN; a++) fl[a] = 0.0;
    bool bad = false;
    // the points one at a time: unrolled, every point's operands stayed live
    // at once (366 VGPRs, one wave per SIMD; 224 and two waves this way)
#pragma unroll 1
    for (int q = 0; q < NN; q++) {
        const int q0 = q & 1, q1 = (q >> 1) & 1, q2 = (q >> 2) & 1;
        const double xi[3] = {rt.gx[q0], rt.gx[q1], DIM == 3 ? rt.gx[q2] : 0.0};
        const double w = rt.gw[q0] * rt.gw[q1] * (DIM == 3 ? rt.gw[q2] : 1.0);
        double J[9], Ji[9], xq[3];
        const double det = geometry<DIM>(X, xi, J, Ji, xq);
        bad |= !(det > 0.0);
        const double wdet = w * fabs(det);
        const double wd = wdet * coef;
        const double fq = source_value(p, DIM, xq, 0);
        // physical gradients of the 2^d shape functions (Sect. 3.7 eq. shape_grad)
        double g[NN][DIM];
#pragma unroll
        for (int a = 0; a < NN; a++) {
            const int a0 = a & 1, a1 = (a >> 1) & 1, a2 = (a >> 2) & 1;
            double gr[3];
            const double L0 = rt.L[a0 * 2 + q0], L1 = rt.L[a1 * 2 + q1];
            const double D0 = rt.D[a0 * 2 + q0], D1 = rt.D[a1 * 2 + q1];
            if (DIM == 3) {
                const double L2 = rt.L[a2 * 2 + q2], D2 = rt.D[a2 * 2 + q2];
                gr[0] = D0 * L1 * L2;
                gr[1] = L0 * D1 * L2;
                gr[2] = L0 * L1 * D2;
                fl[a] += wdet * fq * (L0 * L1 * L2);
            } else {
                gr[0] = D0 * L1;
                gr[1] = L0 * D1;
                fl[a] += wdet * fq * (L0 * L1);
            }
#pragma unroll
            for (int i = 0; i < DIM; i++) {
                double v = 0.0;
#pragma unroll
                for (int sd = 0; sd < DIM; sd++) v += Ji[sd * DIM + i] * gr[sd];
                g[a][i] = v;
            }
        }
        if (PREC == FE_FP64) {
            int t = 0;
#pragma unroll
            for (int a = 0; a < NN; a++)
#pragma unroll
                for (int b = a; b < NN; b++, t++) {
                    double dot = 0.0;
#pragma unroll
                    for (int i = 0; i < DIM; i++) dot += g[a][i] * g[b][i];
                    acc[t] += Acc(wd * dot);
                }
        } else {
            float ga[NN][DIM], hb[NN][DIM];
#pragma unroll
            for (int a = 0; a < NN; a++)
#pragma unroll
                for (int i = 0; i < DIM; i++) {
                    ga[a][i] = round_in<PREC>(g[a][i] * alpha);
                    hb[a][i] = round_in<PREC>(g[a][i] * wd * beta);
                }
            int t = 0;
#pragma unroll
            for (int a = 0; a < NN; a++)
#pragma unroll
                for (int b = a; b < NN; b++, t++)
#pragma unroll
                    for (int i = 0; i < DIM; i++) acc[t] = fmaf(ga[a][i], hb[b][i], float(acc[t]));
        }
    }
    if (bad) atomicOr(m.status, 1);
    const double unscale = 1.0 / (alpha * beta);
    const int64_t blk = cell / 64, lane = cell % 64;
    using Out = Acc;
    // packed upper triangle, entry t = (a, b), a <= b, in row-major order
    Out *Eb = static_cast<Out *>(Ev) + blk * (NT * 64) + lane;
#pragma unroll
    for (int t = 0; t < NT; t++) Eb[t * 64] = PREC == FE_FP64 ? acc[t] : Out(double(acc[t]) * unscale);
#pragma unroll
    for (int a = 0; a < NN; a++) F[cell * NN + a] = fl[a];
}

template <int DIM, int PREC>
__global__ __launch_bounds__(256) void k3_q1_kernel(SpaceArgs s, MeshArgs m, ProblemArgs p, RefTables rt,
                                                     void *__restrict__ Ev, double *__restrict__ F)
{
    k3_q1_body<DIM, PREC>(s, m, p, rt, Ev, F, xcd_block(blockIdx.x, gridDim.x));
}

template <int DIM, int PREC>
__global__ __launch_bounds__(256) void k3_q1_batch_kernel(const AsmJob *__restrict__ jobs,
                                                           const int32_t *__restrict__ boff, int njobs)
{
    int64_t lb, nb;
    const AsmJob &J = jobs[find_job(boff, njobs, lb, nb)];
    k3_q1_body<DIM, PREC>(J.s, J.m, J.p, J.rt, J.E, J.F, lb);
}

// ---------------------------------------------------------------------------
// Generic tiled kernel (any order, Poisson or elasticity, FP64): one
// workgroup computes a TILE x TILE block of one cell's element matrix.
// Quadrature points are processed in slabs of QS: the slab's geometry and the
// physical gradients of the tile's row and column shape functions are staged
// in LDS, then every thread accumulates an MT x MT register micro-tile.
// ---------------------------------------------------------------------------
template <int DIM, int PROB, int MT>
__global__ __launch_bounds__(256) void k3_tiled_kernel(SpaceArgs s, MeshArgs m, ProblemArgs p, RefTables rt,
                                                        int tiles, double *__restrict__ E, double *__restrict__ F)
{
    constexpr int TILE = 16 * MT;
    constexpr int QS = 8;
    constexpr int NV = 1 << DIM;
    constexpr int NC = PROB == 1 ? DIM : 1;
    const int k = s.k, k1 = k + 1, nn = s.nn, nloc = s.nloc;
    const int nq = DIM == 3 ? k1 * k1 * k1 : k1 * k1;
    const int64_t bid = xcd_block(blockIdx.x, gridDim.x);
    const int64_t cell = bid / (tiles * tiles);
    const int tile = int(bid % (tiles * tiles));
    const int r0 = (tile / tiles) * TILE, c0 = (tile % tiles) * TILE;
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;

    __shared__ double sX[NV][3];
    __shared__ double sW[QS], sWd[QS], sXq[QS][3], sJi[QS][9];
    __shared__ double sGr[QS][TILE / NC + 2][DIM];
    __shared__ double sGc[QS][TILE / NC + 2][DIM];
    __shared__ int sBad;

    if (tid < NV) {
        double Xv[NV][3];
        load_vertices<DIM>(m, cell, Xv);
        sX[tid][0] = Xv[tid][0];
        sX[tid][1] = Xv[tid][1];
        sX[tid][2] = Xv[tid][2];
    }
    if (tid == 0) sBad = 0;
    const double coef = m.coef ? m.coef[cell] : 1.0;
    const int rn0 = r0 / NC, cn0 = c0 / NC;
    const int rn1 = min((r0 + TILE - 1) / NC, nn - 1), cn1 = min((c0 + TILE - 1) / NC, nn - 1);
    const int nrn = rn1 - rn0 + 1, ncn = cn1 - cn0 + 1;
    const bool do_load = (c0 == 0);
    __syncthreads();

    double acc[MT][MT];
#pragma unroll
    for (int i = 0; i < MT; i++)
#pragma unroll
        for (int j = 0; j < MT; j++) acc[i][j] = 0.0;
    double facc = 0.0;

    for (int qs0 = 0; qs0 < nq; qs0 += QS) {
        if (tid < QS && qs0 + tid < nq) {
            const int q = qs0 + tid;
            const int q0 = q % k1, q1 = (q / k1) % k1, q2 = q / (k1 * k1);
            const double xi[3] = {rt.gx[q0], rt.gx[q1], DIM == 3 ? rt.gx[q2] : 0.0};
            const double w = rt.gw[q0] * rt.gw[q1] * (DIM == 3 ? rt.gw[q2] : 1.0);
            double Xl[NV][3];
            for (int v = 0; v < NV; v++)
                for (int r = 0; r < 3; r++) Xl[v][r] = sX[v][r];
            double J[9], Ji[9], xq[3];
            const double det = geometry<DIM>(Xl, xi, J, Ji, xq);
            if (!(det > 0.0)) sBad = 1;
            sWd[tid] = w * fabs(det);
            sW[tid] = w * fabs(det) * coef;
            for (int t = 0; t < 9; t++) sJi[tid][t] = Ji[t];
            for (int r = 0; r < 3; r++) sXq[tid][r] = xq[r];
        }
        __syncthreads();
        // physical gradients of the row and column nodes at the slab's points
        for (int idx = tid; idx < QS * (nrn + ncn); idx += blockDim.x) {
            const int q = idx / (nrn + ncn);
            const int rem = idx % (nrn + ncn);
            const bool is_row = rem < nrn;
            const int node = is_row ? rn0 + rem : cn0 + (rem - nrn);
            const int qq = qs0 + q;
            double g[DIM];
            if (qq < nq) {
                const int q0 = qq % k1, q1 = (qq / k1) % k1, q2 = qq / (k1 * k1);
                const int a0 = node % k1, a1 = (node / k1) % k1, a2 = node / (k1 * k1);
                double gr[3];
                const double L0 = rt.L[a0 * k1 + q0], L1 = rt.L[a1 * k1 + q1];
                const double D0 = rt.D[a0 * k1 + q0], D1 = rt.D[a1 * k1 + q1];
                if (DIM == 3) {
                    const double L2 = rt.L[a2 * k1 + q2], D2 = rt.D[a2 * k1 + q2];
                    gr[0] = D0 * L1 * L2;
                    gr[1] = L0 * D1 * L2;
                    gr[2] = L0 * L1 * D2;
                } else {
                    gr[0] = D0 * L1;
                    gr[1] = L0 * D1;
                    gr[2] = 0.0;
                }
                for (int i = 0; i < DIM; i++) {
                    double v = 0.0;
                    for (int sd = 0; sd < DIM; sd++) v += sJi[q][sd * DIM + i] * gr[sd];
                    g[i] = v;
                }
            } else {
                for (int i = 0; i < DIM; i++) g[i] = 0.0;
            }
            if (is_row)
                for (int i = 0; i < DIM; i++) sGr[q][rem][i] = g[i];
            else
                for (int i = 0; i < DIM; i++) sGc[q][rem - nrn][i] = g[i];
        }
        __syncthreads();
        const int qn = min(QS, nq - qs0);
        for (int q = 0; q < qn; q++) {
            const double wq = sW[q];
            double ga[MT][DIM], gb[MT][DIM];
#pragma unroll
            for (int i = 0; i < MT; i++) {
                const int row = min(r0 + ty + 16 * i, nloc - 1);
                const int col = min(c0 + tx + 16 * i, nloc - 1);
#pragma unroll
                for (int d = 0; d < DIM; d++) {
                    ga[i][d] = sGr[q][row / NC - rn0][d];
                    gb[i][d] = sGc[q][col / NC - cn0][d];
                }
            }
#pragma unroll
            for (int i = 0; i < MT; i++)
#pragma unroll
                for (int j = 0; j < MT; j++) {
                    double dot = 0.0;
#pragma unroll
                    for (int d = 0; d < DIM; d++) dot += ga[i][d] * gb[j][d];
                    if (PROB == 0) {
                        acc[i][j] += wq * dot;
                    } else {
                        const int ci = (r0 + ty + 16 * i) % NC, cj = (c0 + tx + 16 * j) % NC;
                        double v = p.lambda * ga[i][ci] * gb[j][cj] + p.mu * ga[i][cj] * gb[j][ci];
                        if (ci == cj) v += p.mu * dot;
                        acc[i][j] += wq * v;
                    }
                }
        }
        if (do_load && tid < TILE && r0 + tid < nloc) {
            const int row = r0 + tid, a = row / NC, c = row % NC;
            const int a0 = a % k1, a1 = (a / k1) % k1, a2 = a / (k1 * k1);
            for (int q = 0; q < qn; q++) {
                const int qq = qs0 + q;
                const int q0 = qq % k1, q1 = (qq / k1) % k1, q2 = qq / (k1 * k1);
                double phi = rt.L[a0 * k1 + q0] * rt.L[a1 * k1 + q1];
                if (DIM == 3) phi *= rt.L[a2 * k1 + q2];
                const double xq[3] = {sXq[q][0], sXq[q][1], sXq[q][2]};
                facc += sWd[q] * source_value(p, DIM, xq, c) * phi;
            }
        }
        __syncthreads();
    }
    if (tid == 0 && sBad) atomicOr(m.status, 1);
    double *Ec = E + cell * int64_t(nloc) * nloc;
#pragma unroll
    for (int i = 0; i < MT; i++) {
        const int row = r0 + ty + 16 * i;
        if (row >= nloc) continue;
#pragma unroll
        for (int j = 0; j < MT; j++) {
            const int col = c0 + tx + 16 * j;
            if (col < nloc) Ec[int64_t(row) * nloc + col] = acc[i][j];
        }
    }
    if (do_load && tid < TILE && r0 + tid < nloc) F[cell * nloc + r0 + tid] = facc;
}

// ---------------------------------------------------------------------------
// Dirichlet lifting for non-zero (affine) data: F_a -= sum_{b fixed} A_ab u_D(b)
// on every cell that has fixed DOFs (one wave per cell).
// ---------------------------------------------------------------------------
template <int DIM, typename ET>
__global__ __launch_bounds__(64) void k3_lift_kernel(SpaceArgs s, MeshArgs m, ProblemArgs p, const int32_t *cell_dofs,
                                                     int cb, int packed, int ne, const ET *__restrict__ E,
                                                     double *__restrict__ F)
{
    const int64_t cell = blockIdx.x;
    const int nloc = s.nloc, k = s.k, k1 = k + 1, nc = s.ncomp;
    const int32_t *g = cell_dofs + cell * nloc;
    bool any = false;
    for (int t = 0; t < nloc; t++) any |= g[t] < 0;
    if (!any) return;
    double X[1 << DIM][3];
    load_vertices<DIM>(m, cell, X);
    for (int a = threadIdx.x; a < nloc; a += blockDim.x) {
        if (g[a] < 0) continue;
        double lift = 0.0;
        for (int b = 0; b < nloc; b++) {
            if (g[b] >= 0) continue;
            const int node = b / nc, c = b % nc;
            const double xi[3] = {double(node % k1) / k, double((node / k1) % k1) / k,
                                  DIM == 3 ? double(node / (k1 * k1)) / k : 0.0};
            double J[9], Ji[9], xb[3];
            geometry<DIM>(X, xi, J, Ji, xb);
            double u = p.aff[4 * c];
            for (int r = 0; r < DIM; r++) u += p.aff[4 * c + 1 + r] * xb[r];
            lift += double(E[elem_index(cell, a, b, nloc, cb, packed, ne)]) * u;
        }
        F[cell * nloc + a] -= lift;
    }
}

// ---------------------------------------------------------------------------
// Launch
// ---------------------------------------------------------------------------
template <int DIM, int PROB>
static fe_status launch_tiled(const SpaceArgs &sa, const MeshArgs &ma, const ProblemArgs &pa, const RefTables &rt,
                              double *E, double *F, hipStream_t s)
{
    const int nloc = sa.nloc;
    int mt = (nloc + 15) / 16;
    if (mt > 8) mt = 8;
    if (mt == 3) mt = 4;
    if (mt == 5) mt = 6;
    if (mt == 7) mt = 8;
    const int tile = 16 * mt;
    const int tiles = (nloc + tile - 1) / tile;
    const int64_t grid = sa.ncells * tiles * tiles;
    if (grid == 0) return FE_OK;
#define FE_TILED_CASE(MTV)                                                                                          \
    case MTV:                                                                                                       \
        hipLaunchKernelGGL((k3_tiled_kernel<DIM, PROB, MTV>), dim3(grid), dim3(256), 0, s, sa, ma, pa, rt, tiles, E, \
                           F);                                                                                      \
        break;
    switch (mt) {
        FE_TILED_CASE(1)
        FE_TILED_CASE(2)
        FE_TILED_CASE(4)
        FE_TILED_CASE(6)
        FE_TILED_CASE(8)
        default:
            return set_error(FE_EINVAL, "unsupported element size");
    }
#undef FE_TILED_CASE
    FE_HIP(hipGetLastError());
    return FE_OK;
}

fe_status launch_integrate(const SpaceArgs &sa, const MeshArgs &ma, const ProblemArgs &pa, const RefTables &rt,
                           const ElemLayout &el, void *ws, hipStream_t s)
{
    double *E = static_cast<double *>(ws);
    double *F = reinterpret_cast<double *>(static_cast<char *>(ws) + el.f_offset);
    if (sa.ncells == 0) return FE_OK;
    if (sa.dim == 3 && sa.k >= 2) return launch_integrate_mfma(sa, ma, pa, rt, ws, F, s);
    fe_status st = FE_OK;
    if (sa.k == 1 && sa.ncomp == 1) {
        const int64_t grid = (sa.ncells + 255) / 256;
#define FE_Q1(D, P) hipLaunchKernelGGL((k3_q1_kernel<D, P>), dim3(grid), dim3(256), 0, s, sa, ma, pa, rt, ws, F)
        if (sa.dim == 3) {
            switch (pa.precision) {
                case FE_FP64: FE_Q1(3, FE_FP64); break;
                case FE_FP32: FE_Q1(3, FE_FP32); break;
                case FE_FP16: FE_Q1(3, FE_FP16); break;
                default: FE_Q1(3, FE_BF16); break;
            }
        } else {
            switch (pa.precision) {
                case FE_FP64: FE_Q1(2, FE_FP64); break;
                case FE_FP32: FE_Q1(2, FE_FP32); break;
                case FE_FP16: FE_Q1(2, FE_FP16); break;
                default: FE_Q1(2, FE_BF16); break;
            }
        }
#undef FE_Q1
        FE_HIP(hipGetLastError());
    } else if (pa.precision != FE_FP64) {
        return set_error(FE_EINVAL, "reduced-precision integration needs 3D hexahedra (any order) or scalar Q1");
    } else if (sa.dim == 3) {
        st = pa.problem == 1 ? launch_tiled<3, 1>(sa, ma, pa, rt, E, F, s) : launch_tiled<3, 0>(sa, ma, pa, rt, E, F, s);
    } else {
        st = pa.problem == 1 ? launch_tiled<2, 1>(sa, ma, pa, rt, E, F, s) : launch_tiled<2, 0>(sa, ma, pa, rt, E, F, s);
    }
    return st;
}

fe_status launch_lift(const SpaceArgs &sa, const MeshArgs &ma, const ProblemArgs &pa, const int32_t *cell_dofs,
                      const ElemLayout &el, void *ws, hipStream_t s)
{
    if (pa.dirichlet_kind != FE_DIRICHLET_AFFINE || sa.ncells == 0) return FE_OK;
    double *F = reinterpret_cast<double *>(static_cast<char *>(ws) + el.f_offset);
    if (el.elem_bytes == 8) {
        const double *E = static_cast<const double *>(ws);
        if (sa.dim == 3)
            hipLaunchKernelGGL((k3_lift_kernel<3, double>), dim3(sa.ncells), dim3(64), 0, s, sa, ma, pa, cell_dofs,
                               el.cb, el.packed, el.ne, E, F);
        else
            hipLaunchKernelGGL((k3_lift_kernel<2, double>), dim3(sa.ncells), dim3(64), 0, s, sa, ma, pa, cell_dofs,
                               el.cb, el.packed, el.ne, E, F);
    } else {
        const float *E = static_cast<const float *>(ws);
        if (sa.dim == 3)
            hipLaunchKernelGGL((k3_lift_kernel<3, float>), dim3(sa.ncells), dim3(64), 0, s, sa, ma, pa, cell_dofs,
                               el.cb, el.packed, el.ne, E, F);
        else
            hipLaunchKernelGGL((k3_lift_kernel<2, float>), dim3(sa.ncells), dim3(64), 0, s, sa, ma, pa, cell_dofs,
                               el.cb, el.packed, el.ne, E, F);
    }
    FE_HIP(hipGetLastError());
    return FE_OK;
}

// ---------------------------------------------------------------------------
// Batched launches (one launch per kernel class, jobs in a device table)
// ---------------------------------------------------------------------------
bool integrate_batchable(const SpaceArgs &sa, const ProblemArgs &pa)
{
    return (sa.k == 1 && sa.ncomp == 1) || (sa.dim == 3 && sa.k >= 2);
}

int64_t integrate_blocks(const SpaceArgs &sa, const ProblemArgs &pa, int32_t &parts)
{
    parts = 1;
    if (sa.dim == 3 && sa.k >= 2) return mfma_blocks(sa, pa, parts);
    return (sa.ncells + 255) / 256;
}

fe_status launch_integrate_batch(const AsmJob &h, const AsmJob *jobs, const int32_t *boff, int njobs, int grid,
                                 hipStream_t s)
{
    if (grid == 0) return FE_OK;
    const SpaceArgs &sa = h.s;
    if (sa.dim == 3 && sa.k >= 2) return launch_mfma_batch(h, jobs, boff, njobs, grid, s);
    if (!(sa.k == 1 && sa.ncomp == 1)) return set_error(FE_EINVAL, "no batched kernel for this class");
#define FE_Q1B(D, P) hipLaunchKernelGGL((k3_q1_batch_kernel<D, P>), dim3(grid), dim3(256), 0, s, jobs, boff, njobs)
    if (sa.dim == 3) {
        switch (h.p.precision) {
            case FE_FP64: FE_Q1B(3, FE_FP64); break;
            case FE_FP32: FE_Q1B(3, FE_FP32); break;
            case FE_FP16: FE_Q1B(3, FE_FP16); break;
            default: FE_Q1B(3, FE_BF16); break;
        }
    } else {
        switch (h.p.precision) {
            case FE_FP64: FE_Q1B(2, FE_FP64); break;
            case FE_FP32: FE_Q1B(2, FE_FP32); break;
            case FE_FP16: FE_Q1B(2, FE_FP16); break;
            default: FE_Q1B(2, FE_BF16); break;
        }
    }
#undef FE_Q1B
    FE_HIP(hipGetLastError());
    return FE_OK;
}

}  // namespace fe
