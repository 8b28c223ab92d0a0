// fe_simplex.hip -- Lagrangian P_k elements on simplicial meshes: triangles
// and tetrahedra of a general mesh given by vertex coordinates and
// cell-to-vertex connectivity (Sect. 3.3 truncated polynomial spaces and
// node sets, Sect. 3.5 shape functions by a change of basis, Sect. 3.7
// quadrature on simplices through the collapsed (Duffy) map; Sect. 3.6 and
// 10.3 global DOFs; Sect. 11.1 a pattern built once and reused).
//
// Set-up on the host, once per mesh and order:
//  * the reference element: nodes s/k with |s| <= k (x fastest), shape
//    functions from the monomial pre-basis by the change of basis, the
//    collapsed Gauss rule with k + ceil(d/2) points per direction and the
//    reference gradient tensor S^{rs}_ab = int d_r phi_a d_s phi_b on it;
//  * global nodes: a local node is named by the sub-simplex its barycentric
//    support spans (vertex, edge, face or the cell) and its weights there;
//    edges and faces are found by sorting their vertex keys, so the cells
//    around a node name it alike whatever their local vertex order.  Global
//    ids by first appearance over (cell, local node); boundary facets are the
//    facets of one cell only; free and fixed ranks; the cell-to-DOF map;
//  * the stored pattern and permutation: each free row's columns (the free
//    nodes of the cells around it, ascending) and, per entry, its element
//    contributions in ascending cell order (the gather map).
// Numeric phase on the device:
//  * sx_element_kernel: per cell the affine geometry, then each entry of the
//    element matrix's upper triangle as a contraction of the cell's
//    coefficient tensor (|det J| J^-1 J^-T, or its elasticity analogue) with
//    the reference tensor -- the map is affine, so the quadrature sum does not
//    depend on the cell and is carried out once on the reference element --
//    and the load vector (with Dirichlet lifting) on the collapsed rule;
//  * gathers: each CSR entry sums its contributions in list order, each rhs
//    entry the loads of its node's occurrences; dinv from the diagonal.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "fe_internal.h"

namespace fe {

constexpr int kSxMaxK = 4;
constexpr int kSxMaxNN = 35;  // P4 on the tetrahedron

struct SxArgs {
    int32_t problem, source_kind, dirichlet_kind;
    double lambda, mu;
    double source[3];
    double aff[12];
    int64_t ncells;
    int8_t s[3 * kSxMaxNN];  // lattice point of every local node
};

__host__ __device__ constexpr int sx_nn(int dim, int k)
{
    return dim == 2 ? (k + 1) * (k + 2) / 2 : (k + 1) * (k + 2) * (k + 3) / 6;
}

template <int DIM, int K, int PROB>
struct SxShape {
    static constexpr int NN = sx_nn(DIM, K);
    static constexpr int NC = PROB == FE_ELASTICITY ? DIM : 1;
    static constexpr int NLOC = NN * NC;
    static constexpr int NTRI = NLOC * (NLOC + 1) / 2;
    // per-cell coefficients: the symmetric DIM x DIM tensor (Poisson) or
    // C^{ij}_{rs} (elasticity)
    static constexpr int NP = PROB == FE_ELASTICITY ? DIM * DIM * DIM * DIM : DIM * (DIM + 1) / 2;
    // reference table: per coefficient pair, every upper-triangle entry
    // (Poisson), or S^{rs}_{ab} over the full nn x nn (elasticity)
    static constexpr int NTAB = PROB == FE_ELASTICITY ? DIM * DIM * NN * NN : NP * NTRI;
    static constexpr int NQ1 = K + (DIM + 1) / 2;
    static constexpr int NQ = DIM == 3 ? NQ1 * NQ1 * NQ1 : NQ1 * NQ1;
    static constexpr int CPB = NTRI <= 16 ? 64 : NTRI <= 64 ? 32 : NTRI <= 256 ? 8 : 4;
};

// One workgroup per CPB consecutive cells.  Writes the upper triangle of
// every element matrix, E[K ntri + t] with t = I nloc - I (I - 1) / 2 + (J - I)
// for I <= J, and the load with lifting, F[K nloc + I].
template <int DIM, int K, int PROB>
__global__ __launch_bounds__(256) void sx_element_kernel(SxArgs sa, const double *__restrict__ vxyz,
                                                         const int32_t *__restrict__ cells,
                                                         const double *__restrict__ coef,
                                                         const int32_t *__restrict__ cell_dofs,
                                                         const double *__restrict__ tab, const int32_t *__restrict__ tri,
                                                         const double *__restrict__ phiq,
                                                         const double *__restrict__ qxw, double *__restrict__ E,
                                                         double *__restrict__ F)
{
    using S = SxShape<DIM, K, PROB>;
    constexpr int NV = DIM + 1;
    __shared__ double sTab[S::NTAB];
    __shared__ int32_t sTri[S::NTRI];
    __shared__ double sC[S::CPB][S::NP];
    __shared__ double sX[S::CPB][NV * DIM];
    __shared__ double sG[S::CPB][S::NQ];
    __shared__ double sDet[S::CPB];
    __shared__ int32_t sDofs[S::CPB * S::NLOC];
    const int tid = threadIdx.x;
    const int64_t K0 = xcd_block(blockIdx.x, gridDim.x) * S::CPB;
    const int ncl = sa.ncells - K0 < S::CPB ? int(sa.ncells - K0) : S::CPB;
    for (int t = tid; t < S::NTAB; t += blockDim.x) sTab[t] = tab[t];
    for (int t = tid; t < S::NTRI; t += blockDim.x) sTri[t] = tri[t];
    if (sa.dirichlet_kind == FE_DIRICHLET_AFFINE)
        for (int t = tid; t < ncl * S::NLOC; t += blockDim.x) sDofs[t] = cell_dofs[K0 * S::NLOC + t];
    // geometry and coefficients of the block's cells
    for (int c = tid; c < ncl; c += blockDim.x) {
        const int64_t Kc = K0 + c;
        double X[NV][DIM];
#pragma unroll
        for (int j = 0; j < NV; j++) {
            const int64_t v = cells[Kc * NV + j];
#pragma unroll
            for (int r = 0; r < DIM; r++) X[j][r] = vxyz[v * DIM + r];
        }
        double J[DIM][DIM], Ji[DIM][DIM], det;
#pragma unroll
        for (int r = 0; r < DIM; r++)
#pragma unroll
            for (int s = 0; s < DIM; s++) J[r][s] = X[s + 1][r] - X[0][r];
        if constexpr (DIM == 2) {
            det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            const double id = 1.0 / det;
            Ji[0][0] = J[1][1] * id;
            Ji[0][1] = -J[0][1] * id;
            Ji[1][0] = -J[1][0] * id;
            Ji[1][1] = J[0][0] * id;
        } else {
            const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
            const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
            const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
            det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
            const double id = 1.0 / det;
            Ji[0][0] = c00 * id;
            Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
            Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
            Ji[1][0] = c01 * id;
            Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
            Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
            Ji[2][0] = c02 * id;
            Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
            Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
        }
        const double ad = fabs(det);
        const double w = ad * (coef ? coef[Kc] : 1.0);
        if constexpr (PROB == FE_ELASTICITY) {
            // C^{ij}_{rs} = w [lambda Ji_ri Ji_sj + mu Ji_rj Ji_si + mu delta_ij sum_l Ji_rl Ji_sl]
#pragma unroll
            for (int i = 0; i < DIM; i++)
#pragma unroll
                for (int j = 0; j < DIM; j++)
#pragma unroll
                    for (int r = 0; r < DIM; r++)
#pragma unroll
                        for (int s = 0; s < DIM; s++) {
                            double v = sa.lambda * Ji[r][i] * Ji[s][j] + sa.mu * Ji[r][j] * Ji[s][i];
                            if (i == j) {
                                double g = 0.0;
#pragma unroll
                                for (int l = 0; l < DIM; l++) g += Ji[r][l] * Ji[s][l];
                                v += sa.mu * g;
                            }
                            sC[c][((i * DIM + j) * DIM + r) * DIM + s] = w * v;
                        }
        } else {
            // (J^-1 J^-T)_{rs}, r <= s, pairs in the order (0,0),(0,1),..,(1,1),..
            int p = 0;
#pragma unroll
            for (int r = 0; r < DIM; r++)
#pragma unroll
                for (int s = r; s < DIM; s++) {
                    double g = 0.0;
#pragma unroll
                    for (int l = 0; l < DIM; l++) g += Ji[r][l] * Ji[s][l];
                    sC[c][p++] = w * g;
                }
        }
#pragma unroll
        for (int j = 0; j < NV; j++)
#pragma unroll
            for (int r = 0; r < DIM; r++) sX[c][j * DIM + r] = X[j][r];
        sDet[c] = ad;
    }
    __syncthreads();
    // load weights at the quadrature points, w_q |det J| f(x_q) (the
    // component factor source[c] is applied below), over (cell, point) pairs
    if (sa.source_kind != FE_SOURCE_NONE)
        for (int e = tid; e < ncl * S::NQ; e += blockDim.x) {
            const int c = e / S::NQ, q = e - c * S::NQ;
            double g = 1.0;
            if (sa.source_kind == FE_SOURCE_SINPROD) {
                g = DIM * M_PI * M_PI;
#pragma unroll
                for (int r = 0; r < DIM; r++) {
                    double x = sX[c][r];
#pragma unroll
                    for (int t = 0; t < DIM; t++) x += (sX[c][(t + 1) * DIM + r] - sX[c][r]) * qxw[q * (DIM + 1) + t];
                    g *= sin(M_PI * x);
                }
            }
            sG[c][q] = g * qxw[q * (DIM + 1) + DIM] * sDet[c];
        }
    __syncthreads();
    // element matrices: contiguous over the block's cells
    for (int e = tid; e < ncl * S::NTRI; e += blockDim.x) {
        const int c = e / S::NTRI, t = e - c * S::NTRI;
        double v = 0.0;
        if (PROB == FE_ELASTICITY) {
            const int IJ = sTri[t], I = IJ >> 16, Jx = IJ & 0xffff;
            const int a = I / S::NC, i = I % S::NC, b = Jx / S::NC, j = Jx % S::NC;
#pragma unroll
            for (int rs = 0; rs < DIM * DIM; rs++)
                v = __fma_rn(sC[c][(i * DIM + j) * DIM * DIM + rs], sTab[rs * S::NN * S::NN + a * S::NN + b], v);
        } else {
#pragma unroll
            for (int p = 0; p < S::NP; p++) v = __fma_rn(sC[c][p], sTab[p * S::NTRI + t], v);
        }
        E[(K0 + c) * S::NTRI + t] = v;
    }
    // loads and lifting
    for (int e = tid; e < ncl * S::NLOC; e += blockDim.x) {
        const int c = e / S::NLOC, I = e - c * S::NLOC;
        const int a = I / S::NC, i = I % S::NC;
        const int64_t Kc = K0 + c;
        double f = 0.0;
        if (sa.source_kind != FE_SOURCE_NONE) {
#pragma unroll 4
            for (int q = 0; q < S::NQ; q++) f = __fma_rn(sG[c][q], phiq[q * S::NN + a], f);
            f *= sa.source[i];
        }
        if (sa.dirichlet_kind == FE_DIRICHLET_AFFINE) {
            for (int Jx = 0; Jx < S::NLOC; Jx++) {
                if (sDofs[c * S::NLOC + Jx] >= 0) continue;
                const int b = Jx / S::NC, j = Jx % S::NC;
                // entry (I, Jx) of the element matrix
                double A = 0.0;
                if (PROB == FE_ELASTICITY) {
#pragma unroll
                    for (int rs = 0; rs < DIM * DIM; rs++)
                        A = __fma_rn(sC[c][(i * DIM + j) * DIM * DIM + rs], sTab[rs * S::NN * S::NN + a * S::NN + b], A);
                } else {
                    const int lo = I < Jx ? I : Jx, hi = I < Jx ? Jx : I;
                    const int t = lo * S::NLOC - lo * (lo - 1) / 2 + (hi - lo);
#pragma unroll
                    for (int p = 0; p < S::NP; p++) A = __fma_rn(sC[c][p], sTab[p * S::NTRI + t], A);
                }
                // u_D,j at the node: x_b = X_0 + sum_t (X_{t+1} - X_0) s_t / k
                double u = sa.aff[4 * j];
#pragma unroll
                for (int r = 0; r < DIM; r++) {
                    double x = sX[c][r];
#pragma unroll
                    for (int t = 0; t < DIM; t++)
                        x += (sX[c][(t + 1) * DIM + r] - sX[c][r]) * (double(sa.s[3 * b + t]) / K);
                    u += sa.aff[4 * j + 1 + r] * x;
                }
                f -= A * u;
            }
        }
        F[Kc * S::NLOC + I] = f;
    }
}


// ---------------------------------------------------------------------------
// Lowest-order vector elements on simplices (Sect. 3.9, 3.10): family 1
// Nedelec (a DOF per edge, covariant map J^-T), family 2 Raviart-Thomas (a
// DOF per facet, contravariant map J / det J).  The form is
//   int coef curl u . curl v + kappa u . v   (Nedelec)
//   int coef div u div v + kappa u . v       (Raviart-Thomas)
// and for an affine map each term is a contraction of a per-cell symmetric
// tensor with reference products: curl curl (3D) coef/|det J| J^T J, (2D)
// coef/|det J|; div div coef/|det J|; mass kappa |det J| J^-1 J^-T
// (Nedelec) or kappa/|det J| J^T J (Raviart-Thomas).  Entries and loads are
// multiplied by the orientation signs of the cell's DOFs (edges run from the
// lower to the higher global vertex id; a facet's normal is taken over its
// vertices in ascending global id).
template <int DIM, int FAM>
struct SxvShape {
    static constexpr int ND = FAM == 1 ? (DIM == 3 ? 6 : 3) : DIM + 1;
    static constexpr int NTRI = ND * (ND + 1) / 2;
    static constexpr int NPS = (FAM == 1 && DIM == 3) ? 6 : 1;
    static constexpr int NPM = DIM * (DIM + 1) / 2;
    static constexpr int NP = NPS + NPM;
    static constexpr int NQ1 = 1 + (DIM + 1) / 2;
    static constexpr int NQ = DIM == 3 ? NQ1 * NQ1 * NQ1 : NQ1 * NQ1;
    static constexpr int CPB = 64;
};

template <int DIM, int FAM>
__global__ __launch_bounds__(256) void sx_vector_kernel(SxArgs sa, double kappa, const double *__restrict__ vxyz,
                                                        const int32_t *__restrict__ cells,
                                                        const double *__restrict__ coef, const double *__restrict__ tab,
                                                        const int32_t *__restrict__ tri,
                                                        const double *__restrict__ phq, const double *__restrict__ qxw,
                                                        double *__restrict__ E, double *__restrict__ F)
{
    using S = SxvShape<DIM, FAM>;
    constexpr int NV = DIM + 1;
    __shared__ double sTab[S::NP * S::NTRI];
    __shared__ int32_t sTri[S::NTRI];
    __shared__ double sC[S::CPB][S::NP];
    __shared__ double sSg[S::CPB][S::ND];
    __shared__ double sX[S::CPB][NV * DIM];
    __shared__ double sM[S::CPB][DIM * DIM];  // pull-back of the load: J^-1 or J^T / det J
    __shared__ double sDet[S::CPB];
    __shared__ double sG[S::CPB][S::NQ][DIM];
    __shared__ double sPh[S::NQ * S::ND * DIM];  // reference shape functions at the rule's points
    const int tid = threadIdx.x;
    const int64_t K0 = xcd_block(blockIdx.x, gridDim.x) * S::CPB;
    const int ncl = sa.ncells - K0 < S::CPB ? int(sa.ncells - K0) : S::CPB;
    for (int t = tid; t < S::NP * S::NTRI; t += blockDim.x) sTab[t] = tab[t];
    for (int t = tid; t < S::NTRI; t += blockDim.x) sTri[t] = tri[t];
    for (int t = tid; t < S::NQ * S::ND * DIM; t += blockDim.x) sPh[t] = phq[t];
    for (int c = tid; c < ncl; c += blockDim.x) {
        const int64_t Kc = K0 + c;
        int32_t g[NV];
        double X[NV][DIM];
#pragma unroll
        for (int j = 0; j < NV; j++) {
            g[j] = cells[Kc * NV + j];
#pragma unroll
            for (int r = 0; r < DIM; r++) X[j][r] = vxyz[int64_t(g[j]) * DIM + r];
        }
        double J[DIM][DIM], Ji[DIM][DIM], det;
#pragma unroll
        for (int r = 0; r < DIM; r++)
#pragma unroll
            for (int s = 0; s < DIM; s++) J[r][s] = X[s + 1][r] - X[0][r];
        if constexpr (DIM == 2) {
            det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            const double id = 1.0 / det;
            Ji[0][0] = J[1][1] * id;
            Ji[0][1] = -J[0][1] * id;
            Ji[1][0] = -J[1][0] * id;
            Ji[1][1] = J[0][0] * id;
        } else {
            const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
            const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
            const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
            det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
            const double id = 1.0 / det;
            Ji[0][0] = c00 * id;
            Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
            Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
            Ji[1][0] = c01 * id;
            Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
            Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
            Ji[2][0] = c02 * id;
            Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
            Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
        }
        const double ad = fabs(det), k = coef ? coef[Kc] : 1.0;
        // stiffness coefficients
        if constexpr (FAM == 1 && DIM == 3) {
            int p = 0;
#pragma unroll
            for (int r = 0; r < DIM; r++)
#pragma unroll
                for (int s = r; s < DIM; s++) {
                    double v = 0.0;
#pragma unroll
                    for (int l = 0; l < DIM; l++) v += J[l][r] * J[l][s];
                    sC[c][p++] = k / ad * v;
                }
        } else {
            sC[c][0] = k / ad;
        }
        // mass coefficients
        int p = S::NPS;
#pragma unroll
        for (int r = 0; r < DIM; r++)
#pragma unroll
            for (int s = r; s < DIM; s++) {
                double v = 0.0;
#pragma unroll
                for (int l = 0; l < DIM; l++) v += FAM == 1 ? Ji[r][l] * Ji[s][l] : J[l][r] * J[l][s];
                sC[c][p++] = FAM == 1 ? kappa * ad * v : kappa / ad * v;
            }
        // orientation signs
        if constexpr (FAM == 1) {
#pragma unroll
            for (int a = 0; a < S::ND; a++) {
                const int i = DIM == 3 ? (a < 3 ? 0 : a < 5 ? 1 : 2) : (a < 2 ? 0 : 1);
                const int j = DIM == 3 ? (a < 3 ? a + 1 : a < 5 ? a - 1 : 3) : (a < 2 ? a + 1 : 2);
                sSg[c][a] = g[i] < g[j] ? 1.0 : -1.0;
            }
        } else {
#pragma unroll
            for (int a = 0; a < S::ND; a++) {
                int32_t f[3];
                int m = 0;
#pragma unroll
                for (int r = 0; r < NV; r++)
                    if (r != a) f[m++] = g[r];
                int inv = f[0] > f[1];
                if (DIM == 3) inv += (f[0] > f[2]) + (f[1] > f[2]);
                sSg[c][a] = (inv & 1) ? -1.0 : 1.0;
            }
        }
#pragma unroll
        for (int r = 0; r < DIM; r++)
#pragma unroll
            for (int s = 0; s < DIM; s++) sM[c][r * DIM + s] = FAM == 1 ? Ji[r][s] : J[s][r] / det;
#pragma unroll
        for (int j = 0; j < NV; j++)
#pragma unroll
            for (int r = 0; r < DIM; r++) sX[c][j * DIM + r] = X[j][r];
        sDet[c] = ad;
    }
    __syncthreads();
    // pulled-back load weights at the rule's points: w_q |det J| M f(x_q)
    if (sa.source_kind != FE_SOURCE_NONE)
        for (int e = tid; e < ncl * S::NQ; e += blockDim.x) {
            const int c = e / S::NQ, q = e - c * S::NQ;
            double x[DIM], f[DIM];
#pragma unroll
            for (int r = 0; r < DIM; r++) {
                x[r] = sX[c][r];
#pragma unroll
                for (int t = 0; t < DIM; t++) x[r] += (sX[c][(t + 1) * DIM + r] - sX[c][r]) * qxw[q * (DIM + 1) + t];
            }
            if (sa.source_kind == FE_SOURCE_SINPROD) {
                double sn[DIM];
#pragma unroll
                for (int r = 0; r < DIM; r++) sn[r] = sin(M_PI * x[r]);
                double m[DIM];
                if constexpr (FAM == 2) {
#pragma unroll
                    for (int r = 0; r < DIM; r++) m[r] = sn[r];
                } else if constexpr (DIM == 2) {
                    m[0] = sn[1];
                    m[1] = sn[0];
                } else {
                    m[0] = sn[1] * sn[2];
                    m[1] = sn[2] * sn[0];
                    m[2] = sn[0] * sn[1];
                }
#pragma unroll
                for (int r = 0; r < DIM; r++) f[r] = sa.source[r] * m[r];
            } else {
#pragma unroll
                for (int r = 0; r < DIM; r++) f[r] = sa.source[r];
            }
            const double w = qxw[q * (DIM + 1) + DIM] * sDet[c];
#pragma unroll
            for (int r = 0; r < DIM; r++) {
                double v = 0.0;
#pragma unroll
                for (int t = 0; t < DIM; t++) v += sM[c][r * DIM + t] * f[t];
                sG[c][q][r] = w * v;
            }
        }
    __syncthreads();
    for (int e = tid; e < ncl * S::NTRI; e += blockDim.x) {
        const int c = e / S::NTRI, t = e - c * S::NTRI;
        const int a = sTri[t] >> 16, b = sTri[t] & 0xffff;
        double v = 0.0;
#pragma unroll
        for (int p = 0; p < S::NP; p++) v = __fma_rn(sC[c][p], sTab[p * S::NTRI + t], v);
        E[(K0 + c) * S::NTRI + t] = sSg[c][a] * sSg[c][b] * v;
    }
    for (int e = tid; e < ncl * S::ND; e += blockDim.x) {
        const int c = e / S::ND, a = e - c * S::ND;
        double f = 0.0;
        // (unrolled over all points the loop held every operand: 256 VGPRs, two waves per SIMD)
        if (sa.source_kind != FE_SOURCE_NONE)
#pragma unroll 3
            for (int q = 0; q < S::NQ; q++)
#pragma unroll
                for (int r = 0; r < DIM; r++) f = __fma_rn(sG[c][q][r], sPh[(q * S::ND + a) * DIM + r], f);
        F[(K0 + c) * S::ND + a] = sSg[c][a] * f;
    }
}


// ---------------------------------------------------------------------------
// Second-order Nedelec elements (family 3): two DOFs per edge (moments
// against 1 - t and t), two per face (against the face's two edge
// tangents, 3D) and two interior ones (2D).  The cell's local moments are T
// times the moments in the global frame (edges from the lower to the higher
// global vertex id, faces over their vertices in ascending id): a 2 x 2 block
// per edge (identity, or the two DOFs swapped and negated) and per face (the
// local tangents expressed in the global ones).  The cell's matrix in the
// global frame is T^T A T and its load T^T f; A's entries are contractions
// of the cell's stiffness and mass tensors with the reference products, as
// for the lowest order, so every global entry is a sum of at most four.
template <int DIM>
struct Sxn2Shape {
    static constexpr int ND = DIM == 3 ? 20 : 8;
    static constexpr int NB = ND / 2;  // 2 x 2 blocks
    static constexpr int NTRI = ND * (ND + 1) / 2;
    static constexpr int NPS = DIM == 3 ? 6 : 1;
    static constexpr int NPM = DIM * (DIM + 1) / 2;
    static constexpr int NP = NPS + NPM;
    static constexpr int NQ1 = 2 + (DIM + 1) / 2;
    static constexpr int NQ = DIM == 3 ? NQ1 * NQ1 * NQ1 : NQ1 * NQ1;
    static constexpr int CPB = DIM == 3 ? 8 : 32;
};

template <int DIM>
__global__ __launch_bounds__(256) void sx_nedelec2_kernel(SxArgs sa, double kappa, const double *__restrict__ vxyz,
                                                          const int32_t *__restrict__ cells,
                                                          const double *__restrict__ coef,
                                                          const double *__restrict__ tab,
                                                          const int32_t *__restrict__ tri,
                                                          const double *__restrict__ phq,
                                                          const double *__restrict__ qxw, double *__restrict__ E,
                                                          double *__restrict__ F)
{
    using S = Sxn2Shape<DIM>;
    constexpr int NV = DIM + 1;
    __shared__ double sTab[S::NP * S::NTRI];
    __shared__ int32_t sTri[S::NTRI];
    __shared__ double sC[S::CPB][S::NP];
    __shared__ double sT[S::CPB][S::NB][4];  // block entries T(2B + x, 2B + y) at [x * 2 + y]
    __shared__ double sX[S::CPB][NV * DIM];
    __shared__ double sM[S::CPB][DIM * DIM];
    __shared__ double sDet[S::CPB];
    __shared__ double sG[S::CPB][S::NQ][DIM];
    const int tid = threadIdx.x;
    const int64_t K0 = xcd_block(blockIdx.x, gridDim.x) * S::CPB;
    const int ncl = sa.ncells - K0 < S::CPB ? int(sa.ncells - K0) : S::CPB;
    for (int t = tid; t < S::NP * S::NTRI; t += blockDim.x) sTab[t] = tab[t];
    for (int t = tid; t < S::NTRI; t += blockDim.x) sTri[t] = tri[t];
    for (int c = tid; c < ncl; c += blockDim.x) {
        const int64_t Kc = K0 + c;
        int32_t g[NV];
        double X[NV][DIM];
#pragma unroll
        for (int j = 0; j < NV; j++) {
            g[j] = cells[Kc * NV + j];
#pragma unroll
            for (int r = 0; r < DIM; r++) X[j][r] = vxyz[int64_t(g[j]) * DIM + r];
        }
        double J[DIM][DIM], Ji[DIM][DIM], det;
#pragma unroll
        for (int r = 0; r < DIM; r++)
#pragma unroll
            for (int s = 0; s < DIM; s++) J[r][s] = X[s + 1][r] - X[0][r];
        if constexpr (DIM == 2) {
            det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            const double id = 1.0 / det;
            Ji[0][0] = J[1][1] * id;
            Ji[0][1] = -J[0][1] * id;
            Ji[1][0] = -J[1][0] * id;
            Ji[1][1] = J[0][0] * id;
        } else {
            const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
            const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
            const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
            det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
            const double id = 1.0 / det;
            Ji[0][0] = c00 * id;
            Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
            Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
            Ji[1][0] = c01 * id;
            Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
            Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
            Ji[2][0] = c02 * id;
            Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
            Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
        }
        const double ad = fabs(det), k = coef ? coef[Kc] : 1.0;
        if constexpr (DIM == 3) {
            int p = 0;
#pragma unroll
            for (int r = 0; r < 3; r++)
#pragma unroll
                for (int s = r; s < 3; s++) {
                    double v = 0.0;
#pragma unroll
                    for (int l = 0; l < 3; l++) v += J[l][r] * J[l][s];
                    sC[c][p++] = k / ad * v;
                }
        } else {
            sC[c][0] = k / ad;
        }
        int p = S::NPS;
#pragma unroll
        for (int r = 0; r < DIM; r++)
#pragma unroll
            for (int s = r; s < DIM; s++) {
                double v = 0.0;
#pragma unroll
                for (int l = 0; l < DIM; l++) v += Ji[r][l] * Ji[s][l];
                sC[c][p++] = kappa * ad * v;
            }
        // frame blocks: edges
        constexpr int NE = DIM == 3 ? 6 : 3;
#pragma unroll
        for (int e = 0; e < NE; e++) {
            const int i = DIM == 3 ? (e < 3 ? 0 : e < 5 ? 1 : 2) : (e < 2 ? 0 : 1);
            const int j = DIM == 3 ? (e < 3 ? e + 1 : e < 5 ? e - 1 : 3) : (e < 2 ? e + 1 : 2);
            const bool fwd = g[i] < g[j];
            sT[c][e][0] = fwd ? 1.0 : 0.0;
            sT[c][e][1] = fwd ? 0.0 : -1.0;
            sT[c][e][2] = fwd ? 0.0 : -1.0;
            sT[c][e][3] = fwd ? 1.0 : 0.0;
        }
        if constexpr (DIM == 3) {
#pragma unroll
            for (int f = 0; f < 4; f++) {
                int iv[3], m = 0;
#pragma unroll
                for (int r = 0; r < 4; r++)
                    if (r != f) iv[m++] = r;
                double P[3][2];
#pragma unroll
                for (int x = 0; x < 3; x++) {
                    int rank = 0;
#pragma unroll
                    for (int y = 0; y < 3; y++) rank += g[iv[y]] < g[iv[x]];
                    P[x][0] = rank == 1 ? 1.0 : 0.0;
                    P[x][1] = rank == 2 ? 1.0 : 0.0;
                }
#pragma unroll
                for (int mm = 0; mm < 2; mm++)
#pragma unroll
                    for (int b = 0; b < 2; b++) sT[c][NE + f][mm * 2 + b] = P[mm + 1][b] - P[0][b];
            }
        } else {
            sT[c][NE][0] = 1.0;
            sT[c][NE][1] = 0.0;
            sT[c][NE][2] = 0.0;
            sT[c][NE][3] = 1.0;
        }
#pragma unroll
        for (int r = 0; r < DIM; r++)
#pragma unroll
            for (int s = 0; s < DIM; s++) sM[c][r * DIM + s] = Ji[r][s];
#pragma unroll
        for (int j = 0; j < NV; j++)
#pragma unroll
            for (int r = 0; r < DIM; r++) sX[c][j * DIM + r] = X[j][r];
        sDet[c] = ad;
    }
    __syncthreads();
    if (sa.source_kind != FE_SOURCE_NONE)
        for (int e = tid; e < ncl * S::NQ; e += blockDim.x) {
            const int c = e / S::NQ, q = e - c * S::NQ;
            double x[DIM], f[DIM];
#pragma unroll
            for (int r = 0; r < DIM; r++) {
                x[r] = sX[c][r];
#pragma unroll
                for (int t = 0; t < DIM; t++) x[r] += (sX[c][(t + 1) * DIM + r] - sX[c][r]) * qxw[q * (DIM + 1) + t];
            }
            if (sa.source_kind == FE_SOURCE_SINPROD) {
                double sn[DIM], m[DIM];
#pragma unroll
                for (int r = 0; r < DIM; r++) sn[r] = sin(M_PI * x[r]);
                if constexpr (DIM == 2) {
                    m[0] = sn[1];
                    m[1] = sn[0];
                } else {
                    m[0] = sn[1] * sn[2];
                    m[1] = sn[2] * sn[0];
                    m[2] = sn[0] * sn[1];
                }
#pragma unroll
                for (int r = 0; r < DIM; r++) f[r] = sa.source[r] * m[r];
            } else {
#pragma unroll
                for (int r = 0; r < DIM; r++) f[r] = sa.source[r];
            }
            const double w = qxw[q * (DIM + 1) + DIM] * sDet[c];
#pragma unroll
            for (int r = 0; r < DIM; r++) {
                double v = 0.0;
#pragma unroll
                for (int t = 0; t < DIM; t++) v += sM[c][r * DIM + t] * f[t];
                sG[c][q][r] = w * v;
            }
        }
    __syncthreads();
    auto local_entry = [&](int c, int a, int b) {
        const int lo = a < b ? a : b, hi = a < b ? b : a;
        const int t = lo * S::ND - lo * (lo - 1) / 2 + (hi - lo);
        double v = 0.0;
#pragma unroll
        for (int p = 0; p < S::NP; p++) v = __fma_rn(sC[c][p], sTab[p * S::NTRI + t], v);
        return v;
    };
    for (int e = tid; e < ncl * S::NTRI; e += blockDim.x) {
        const int c = e / S::NTRI, t = e - c * S::NTRI;
        const int I = sTri[t] >> 16, Jx = sTri[t] & 0xffff;
        const int bI = I >> 1, rI = I & 1, bJ = Jx >> 1, rJ = Jx & 1;
        double v = 0.0;
#pragma unroll
        for (int x = 0; x < 2; x++) {
            const double tI = sT[c][bI][x * 2 + rI];
            if (tI == 0.0) continue;
#pragma unroll
            for (int y = 0; y < 2; y++) {
                const double tJ = sT[c][bJ][y * 2 + rJ];
                if (tJ == 0.0) continue;
                v += tI * tJ * local_entry(c, 2 * bI + x, 2 * bJ + y);
            }
        }
        E[(K0 + c) * S::NTRI + t] = v;
    }
    for (int e = tid; e < ncl * S::ND; e += blockDim.x) {
        const int c = e / S::ND, I = e - c * S::ND;
        const int bI = I >> 1, rI = I & 1;
        double f = 0.0;
        if (sa.source_kind != FE_SOURCE_NONE)
#pragma unroll
            for (int x = 0; x < 2; x++) {
                const double tI = sT[c][bI][x * 2 + rI];
                if (tI == 0.0) continue;
                const int a = 2 * bI + x;
                double fl = 0.0;
                for (int q = 0; q < S::NQ; q++)
#pragma unroll
                    for (int r = 0; r < DIM; r++) fl = __fma_rn(sG[c][q][r], phq[(q * S::ND + a) * DIM + r], fl);
                f += tI * fl;
            }
        F[(K0 + c) * S::ND + I] = f;
    }
}


// ---------------------------------------------------------------------------
// Second-order Raviart-Thomas elements (family 4): per facet the fluxes
// against the barycentrics of its vertices, then the interior moments of the
// components.  A facet's global frame lists its vertices in ascending global
// id (N over them); the cell's moment against local vertex x is the global
// one of the same vertex times the parity of the facet's vertex order, so
// each global DOF I is one local DOF loc(I) with a sign: the cell's matrix in
// the global frame has entries s_I s_J A(loc(I), loc(J)) and loads
// s_I f(loc(I)).  A is the contraction of k / |det J| (div-div) and
// kappa / |det J| J^T J (mass, contravariant map) with the reference products.
template <int DIM>
struct SxRt2Shape {
    static constexpr int ND = DIM == 3 ? 15 : 8;
    static constexpr int NTRI = ND * (ND + 1) / 2;
    static constexpr int NPM = DIM * (DIM + 1) / 2;
    static constexpr int NP = 1 + NPM;
    static constexpr int NQ1 = 2 + (DIM + 1) / 2;
    static constexpr int NQ = DIM == 3 ? NQ1 * NQ1 * NQ1 : NQ1 * NQ1;
    static constexpr int CPB = DIM == 3 ? 16 : 32;
};

template <int DIM>
__global__ __launch_bounds__(256) void sx_rt2_kernel(SxArgs sa, double kappa, const double *__restrict__ vxyz,
                                                     const int32_t *__restrict__ cells,
                                                     const double *__restrict__ coef,
                                                     const double *__restrict__ tab,
                                                     const int32_t *__restrict__ tri,
                                                     const double *__restrict__ phq,
                                                     const double *__restrict__ qxw, double *__restrict__ E,
                                                     double *__restrict__ F)
{
    using S = SxRt2Shape<DIM>;
    constexpr int NV = DIM + 1;
    __shared__ double sTab[S::NP * S::NTRI];
    __shared__ int32_t sTri[S::NTRI];
    __shared__ double sC[S::CPB][S::NP];
    __shared__ int32_t sLoc[S::CPB][S::ND];  // local DOF of global-frame DOF I
    __shared__ double sSg[S::CPB][S::ND];    // and its sign
    __shared__ double sX[S::CPB][NV * DIM];
    __shared__ double sM[S::CPB][DIM * DIM];  // pull-back of the load: J^T / det J
    __shared__ double sDet[S::CPB];
    __shared__ double sG[S::CPB][S::NQ][DIM];
    const int tid = threadIdx.x;
    const int64_t K0 = xcd_block(blockIdx.x, gridDim.x) * S::CPB;
    const int ncl = sa.ncells - K0 < S::CPB ? int(sa.ncells - K0) : S::CPB;
    for (int t = tid; t < S::NP * S::NTRI; t += blockDim.x) sTab[t] = tab[t];
    for (int t = tid; t < S::NTRI; t += blockDim.x) sTri[t] = tri[t];
    for (int c = tid; c < ncl; c += blockDim.x) {
        const int64_t Kc = K0 + c;
        int32_t g[NV];
        double X[NV][DIM];
#pragma unroll
        for (int j = 0; j < NV; j++) {
            g[j] = cells[Kc * NV + j];
#pragma unroll
            for (int r = 0; r < DIM; r++) X[j][r] = vxyz[int64_t(g[j]) * DIM + r];
        }
        double J[DIM][DIM], det;
#pragma unroll
        for (int r = 0; r < DIM; r++)
#pragma unroll
            for (int s = 0; s < DIM; s++) J[r][s] = X[s + 1][r] - X[0][r];
        if constexpr (DIM == 2) {
            det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        } else {
            det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) + J[0][1] * (J[1][2] * J[2][0] - J[1][0] * J[2][2]) +
                  J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        }
        const double ad = fabs(det), k = coef ? coef[Kc] : 1.0;
        sC[c][0] = k / ad;
        int p = 1;
#pragma unroll
        for (int r = 0; r < DIM; r++)
#pragma unroll
            for (int s = r; s < DIM; s++) {
                double v = 0.0;
#pragma unroll
                for (int l = 0; l < DIM; l++) v += J[l][r] * J[l][s];
                sC[c][p++] = kappa / ad * v;
            }
        // facet frames: local vertex x of facet f -> global slot rank(x), sign the parity
#pragma unroll
        for (int f = 0; f < NV; f++) {
            int iv[DIM], m = 0;
#pragma unroll
            for (int r = 0; r < NV; r++)
                if (r != f) iv[m++] = r;
            int inv = 0;
#pragma unroll
            for (int x = 0; x < DIM; x++)
#pragma unroll
                for (int y = x + 1; y < DIM; y++) inv += g[iv[x]] > g[iv[y]];
            const double sg = (inv & 1) ? -1.0 : 1.0;
#pragma unroll
            for (int x = 0; x < DIM; x++) {
                int rank = 0;
#pragma unroll
                for (int y = 0; y < DIM; y++) rank += g[iv[y]] < g[iv[x]];
                sLoc[c][f * DIM + rank] = f * DIM + x;
                sSg[c][f * DIM + rank] = sg;
            }
        }
#pragma unroll
        for (int a = DIM * NV; a < S::ND; a++) {
            sLoc[c][a] = a;
            sSg[c][a] = 1.0;
        }
#pragma unroll
        for (int r = 0; r < DIM; r++)
#pragma unroll
            for (int s = 0; s < DIM; s++) sM[c][r * DIM + s] = J[s][r] / det;
#pragma unroll
        for (int j = 0; j < NV; j++)
#pragma unroll
            for (int r = 0; r < DIM; r++) sX[c][j * DIM + r] = X[j][r];
        sDet[c] = ad;
    }
    __syncthreads();
    if (sa.source_kind != FE_SOURCE_NONE)
        for (int e = tid; e < ncl * S::NQ; e += blockDim.x) {
            const int c = e / S::NQ, q = e - c * S::NQ;
            double x[DIM], f[DIM];
#pragma unroll
            for (int r = 0; r < DIM; r++) {
                x[r] = sX[c][r];
#pragma unroll
                for (int t = 0; t < DIM; t++) x[r] += (sX[c][(t + 1) * DIM + r] - sX[c][r]) * qxw[q * (DIM + 1) + t];
            }
#pragma unroll
            for (int r = 0; r < DIM; r++)
                f[r] = sa.source_kind == FE_SOURCE_SINPROD ? sa.source[r] * sin(M_PI * x[r]) : sa.source[r];
            const double w = qxw[q * (DIM + 1) + DIM] * sDet[c];
#pragma unroll
            for (int r = 0; r < DIM; r++) {
                double v = 0.0;
#pragma unroll
                for (int t = 0; t < DIM; t++) v += sM[c][r * DIM + t] * f[t];
                sG[c][q][r] = w * v;
            }
        }
    __syncthreads();
    for (int e = tid; e < ncl * S::NTRI; e += blockDim.x) {
        const int c = e / S::NTRI, t = e - c * S::NTRI;
        const int I = sTri[t] >> 16, Jx = sTri[t] & 0xffff;
        const int a = sLoc[c][I], b = sLoc[c][Jx];
        const int lo = a < b ? a : b, hi = a < b ? b : a;
        const int tl = lo * S::ND - lo * (lo - 1) / 2 + (hi - lo);
        double v = 0.0;
#pragma unroll
        for (int p = 0; p < S::NP; p++) v = __fma_rn(sC[c][p], sTab[p * S::NTRI + tl], v);
        E[(K0 + c) * S::NTRI + t] = sSg[c][I] * sSg[c][Jx] * v;
    }
    for (int e = tid; e < ncl * S::ND; e += blockDim.x) {
        const int c = e / S::ND, I = e - c * S::ND;
        const int a = sLoc[c][I];
        double f = 0.0;
        if (sa.source_kind != FE_SOURCE_NONE)
#pragma unroll 4
            for (int q = 0; q < S::NQ; q++)
#pragma unroll
                for (int r = 0; r < DIM; r++) f = __fma_rn(sG[c][q][r], phq[(q * S::ND + a) * DIM + r], f);
        F[(K0 + c) * S::ND + I] = sSg[c][I] * f;
    }
}

// values[j] = sum of E over the contributions of entry j, in list order.
__global__ __launch_bounds__(256) void sx_gather_kernel(int64_t nnz, const int64_t *__restrict__ gptr,
                                                        const uint32_t *__restrict__ gsrc,
                                                        const double *__restrict__ E, double *__restrict__ values)
{
    const int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (j >= nnz) return;
    const int64_t t0 = gptr[j], t1 = gptr[j + 1];
    double s = 0.0;
    for (int64_t t = t0; t < t1; t++) s += E[gsrc[t]];
    values[j] = s;
}

// rhs[row] = sum of the loads of the row's node occurrences (ascending cell);
// dinv[row] = 1 / values[diag[row]].
__global__ __launch_bounds__(256) void sx_rhs_kernel(int64_t n_rows, int ncomp, const int64_t *__restrict__ optr,
                                                     const uint32_t *__restrict__ oidx, const double *__restrict__ F,
                                                     const int64_t *__restrict__ diag,
                                                     const double *__restrict__ values, double *__restrict__ rhs,
                                                     double *__restrict__ dinv)
{
    const int64_t row = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (row >= n_rows) return;
    const int64_t node = row / ncomp;
    const int comp = int(row - node * ncomp);
    double s = 0.0;
    for (int64_t t = optr[node]; t < optr[node + 1]; t++) s += F[int64_t(oidx[t]) * ncomp + comp];
    if (rhs) rhs[row] = s;
    if (dinv) dinv[row] = 1.0 / values[diag[row]];
}

}  // namespace fe

using namespace fe;

struct fe_simplex_s {
    int dim = 0, k = 0, nn = 0, ncomp = 0, nloc = 0, ntri = 0;
    int family = 0;  // 0 Lagrange P_k, 1 Nedelec, 2 Raviart-Thomas
    double kappa = 0.0;
    bool fix_boundary = false;
    int64_t nverts = 0, ncells = 0, nnodes = 0, nfree_nodes = 0, n_rows = 0, nnz = 0, ncontrib = 0;
    SxArgs args{};
    std::vector<int64_t> h_rowptr;
    std::vector<int32_t> h_colind;
    double *vxyz = nullptr, *coef = nullptr, *tab = nullptr, *phiq = nullptr, *qxw = nullptr, *E = nullptr,
           *F = nullptr;
    int32_t *cells = nullptr, *cell_dofs = nullptr, *tri = nullptr;
    int64_t *gptr = nullptr, *diag = nullptr, *optr = nullptr;
    uint32_t *gsrc = nullptr, *oidx = nullptr;
};

namespace {

template <typename T>
fe_status sx_alloc(T *&p, size_t count)
{
    FE_HIP(hipMalloc(&p, sizeof(T) * std::max<size_t>(count, 1)));
    return FE_OK;
}

template <typename T>
fe_status sx_upload(T *&d, const T *h, size_t count)
{
    fe_status st = sx_alloc(d, count);
    if (st != FE_OK) return st;
    if (count) FE_HIP(hipMemcpy(d, h, sizeof(T) * count, hipMemcpyHostToDevice));
    return FE_OK;
}

void sx_free(fe_simplex S)
{
    void *ptrs[] = {S->vxyz, S->coef, S->tab, S->phiq, S->qxw, S->E,    S->F,    S->cells,
                    S->cell_dofs, S->tri, S->gptr, S->diag, S->optr, S->gsrc, S->oidx};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete S;
}

// ---------------------------------------------------------------------------
// Reference element (host)
// ---------------------------------------------------------------------------
struct SxRef {
    int nn = 0;
    std::vector<int> s;        // nn x 3 lattice points
    std::vector<double> Phi;   // nn x nn: phi_a = sum_b Phi_ab xi^(s_b)
};

void sx_lattice(int dim, int k, std::vector<int> &s)
{
    s.clear();
    for (int s2 = 0; s2 <= (dim == 3 ? k : 0); s2++)
        for (int s1 = 0; s1 <= k; s1++)
            for (int s0 = 0; s0 <= k; s0++)
                if (s0 + s1 + s2 <= k) {
                    s.push_back(s0);
                    s.push_back(s1);
                    s.push_back(s2);
                }
}

double ipowd(double x, int e)
{
    double r = 1.0;
    while (e-- > 0) r *= x;
    return r;
}

// The change of basis: C_ab = (s_a / k)^(s_b) (the pre-basis monomial b at
// node a); Phi = C^-T, by Gauss-Jordan elimination with partial pivoting.
bool sx_reference(int dim, int k, SxRef &R)
{
    sx_lattice(dim, k, R.s);
    const int n = int(R.s.size() / 3);
    R.nn = n;
    std::vector<double> M(static_cast<size_t>(n) * 2 * n, 0.0);
    for (int a = 0; a < n; a++) {
        for (int b = 0; b < n; b++) {
            double v = 1.0;
            for (int r = 0; r < dim; r++) v *= ipowd(double(R.s[3 * a + r]) / k, R.s[3 * b + r]);
            M[a * 2 * n + b] = v;
        }
        M[a * 2 * n + n + a] = 1.0;
    }
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int i = c + 1; i < n; i++)
            if (std::fabs(M[i * 2 * n + c]) > std::fabs(M[p * 2 * n + c])) p = i;
        if (M[p * 2 * n + c] == 0.0) return false;
        if (p != c)
            for (int j = 0; j < 2 * n; j++) std::swap(M[c * 2 * n + j], M[p * 2 * n + j]);
        const double piv = M[c * 2 * n + c];
        for (int j = 0; j < 2 * n; j++) M[c * 2 * n + j] /= piv;
        for (int i = 0; i < n; i++) {
            if (i == c) continue;
            const double f = M[i * 2 * n + c];
            if (f != 0.0)
                for (int j = 0; j < 2 * n; j++) M[i * 2 * n + j] -= f * M[c * 2 * n + j];
        }
    }
    R.Phi.assign(size_t(n) * n, 0.0);
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++) R.Phi[a * n + b] = M[b * 2 * n + n + a];  // (C^-1)_{ba}
    return true;
}

void sx_eval(int dim, const SxRef &R, const double *xi, double *phi, double *dphi)
{
    const int n = R.nn;
    std::vector<double> psi(n), dpsi(size_t(n) * 3);
    for (int b = 0; b < n; b++) {
        double v = 1.0;
        for (int r = 0; r < dim; r++) v *= ipowd(xi[r], R.s[3 * b + r]);
        psi[b] = v;
        for (int r = 0; r < dim; r++) {
            const int e = R.s[3 * b + r];
            double g = e == 0 ? 0.0 : e * ipowd(xi[r], e - 1);
            for (int t = 0; t < dim; t++)
                if (t != r) g *= ipowd(xi[t], R.s[3 * b + t]);
            dpsi[b * 3 + r] = g;
        }
    }
    for (int a = 0; a < n; a++) {
        double v = 0.0, g[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < n; b++) {
            v += R.Phi[a * n + b] * psi[b];
            for (int r = 0; r < dim; r++) g[r] += R.Phi[a * n + b] * dpsi[b * 3 + r];
        }
        phi[a] = v;
        for (int r = 0; r < dim; r++) dphi[a * dim + r] = g[r];
    }
}

// Collapsed Gauss rule: nq1 points per direction, u_0 fastest.  Output
// qxw[q (dim + 1) + r] = xi_r, qxw[q (dim + 1) + dim] = weight.
void sx_rule(int dim, int nq1, std::vector<double> &qxw)
{
    double gx[16], gw[16];
    gauss_legendre_01(nq1, gx, gw);
    const int nq = dim == 3 ? nq1 * nq1 * nq1 : nq1 * nq1;
    qxw.assign(size_t(nq) * (dim + 1), 0.0);
    for (int q = 0; q < nq; q++) {
        const int i0 = q % nq1, i1 = (q / nq1) % nq1, i2 = q / (nq1 * nq1);
        const double u0 = gx[i0], u1 = gx[i1];
        double *o = &qxw[size_t(q) * (dim + 1)];
        o[0] = u0;
        o[1] = (1.0 - u0) * u1;
        if (dim == 3) {
            o[2] = (1.0 - u0) * (1.0 - u1) * gx[i2];
            o[3] = gw[i0] * gw[i1] * gw[i2] * (1.0 - u0) * (1.0 - u0) * (1.0 - u1);
        } else {
            o[2] = gw[i0] * gw[i1] * (1.0 - u0);
        }
    }
}

// ---------------------------------------------------------------------------
// Global numbering (host)
// ---------------------------------------------------------------------------
struct Facet {
    std::array<int32_t, 3> v;  // ascending; v[2] = -1 for an edge
    int64_t cell;
    int32_t j;  // local vertex opposite (facets), or local edge index
};

bool facet_less(const Facet &x, const Facet &y)
{
    if (x.v != y.v) return x.v < y.v;
    if (x.cell != y.cell) return x.cell < y.cell;
    return x.j < y.j;
}

// Unique keys of the given records (sorted in place), and the multiplicity
// of each.
void unique_keys(std::vector<Facet> &rec, std::vector<std::array<int32_t, 3>> &keys, std::vector<int32_t> &count)
{
    std::sort(rec.begin(), rec.end(), facet_less);
    keys.clear();
    count.clear();
    for (size_t t = 0; t < rec.size(); t++) {
        if (t == 0 || rec[t].v != rec[t - 1].v) {
            keys.push_back(rec[t].v);
            count.push_back(0);
        }
        count.back()++;
    }
}

int64_t key_index(const std::vector<std::array<int32_t, 3>> &keys, const std::array<int32_t, 3> &k)
{
    return int64_t(std::lower_bound(keys.begin(), keys.end(), k) - keys.begin());
}

int worker_count(int64_t work)
{
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int64_t by_work = std::max<int64_t>(1, work / 4096);
    return int(std::min<int64_t>(std::min<unsigned>(hw, 16u), by_work));
}

template <typename Fn>
void parallel_chunks(int64_t n, Fn fn)
{
    const int nt = worker_count(n);
    if (nt <= 1) {
        fn(int64_t(0), n);
        return;
    }
    // interleaved chunks of 2048 for balance
    const int64_t chunk = 2048;
    std::vector<std::thread> th;
    for (int w = 0; w < nt; w++)
        th.emplace_back([&, w]() {
            for (int64_t lo = int64_t(w) * chunk; lo < n; lo += int64_t(nt) * chunk) fn(lo, std::min(n, lo + chunk));
        });
    for (auto &t : th) t.join();
}

struct Cand {
    int32_t cn;   // column node (free rank)
    int32_t a, b;
    int64_t K;
};

// The common tail of the set-up, given every (cell, local DOF)'s global
// entity id (pre, ids by first appearance), the entity count and the
// boundary flags: free / fixed ranks, the cell-to-DOF map, each free
// entity's occurrences, the pattern and the gather map.
fe_status sx_finish(fe_simplex S, std::vector<int64_t> &pre, int64_t nnodes, const std::vector<char> &bnd)
{
    const int nn = S->nn, nc = S->ncomp;
    const int64_t ncells = S->ncells;
    S->nnodes = nnodes;
    // free / fixed ranks
    std::vector<int64_t> code(static_cast<size_t>(nnodes));
    int64_t nfree = 0, nfixed = 0;
    for (int64_t g = 0; g < nnodes; g++) code[g] = bnd[g] ? -1 - nfixed++ : nfree++;
    S->nfree_nodes = nfree;
    S->n_rows = nfree * nc;
    if (S->n_rows >= (int64_t(1) << 31)) return set_error(FE_EINVAL, "2^31 or more free DOFs");
    // cell-to-DOF map
    std::vector<int32_t> cdofs(static_cast<size_t>(ncells) * S->nloc);
    for (int64_t K = 0; K < ncells; K++)
        for (int a = 0; a < nn; a++) {
            const int64_t cd = code[pre[K * nn + a]];
            for (int c = 0; c < nc; c++)
                cdofs[(K * nn + a) * nc + c] = int32_t(cd >= 0 ? nc * cd + c : -1 - (nc * (-1 - cd) + c));
        }
    // occurrences of the free nodes, ascending cell
    std::vector<int64_t> optr(static_cast<size_t>(nfree) + 1, 0);
    for (int64_t t = 0; t < ncells * nn; t++) {
        const int64_t cd = code[pre[t]];
        if (cd >= 0) optr[cd + 1]++;
    }
    for (int64_t r = 0; r < nfree; r++) optr[r + 1] += optr[r];
    std::vector<uint32_t> oidx(static_cast<size_t>(optr[nfree]));
    {
        std::vector<int64_t> fill(optr.begin(), optr.end() - 1);
        for (int64_t t = 0; t < ncells * nn; t++) {
            const int64_t cd = code[pre[t]];
            if (cd >= 0) oidx[fill[cd]++] = uint32_t(t);
        }
    }
    // pattern and gather map: per free node, the candidates (column node,
    // cell, a, b) sorted by (column node, cell)
    const int ntri = S->ntri, nloc = S->nloc;
    auto candidates = [&](int64_t r, std::vector<Cand> &cd) {
        cd.clear();
        for (int64_t t = optr[r]; t < optr[r + 1]; t++) {
            const int64_t K = oidx[t] / nn;
            const int a = int(oidx[t] % nn);
            for (int b = 0; b < nn; b++) {
                const int64_t cb = code[pre[K * nn + b]];
                if (cb >= 0) cd.push_back({int32_t(cb), a, b, K});
            }
        }
        std::sort(cd.begin(), cd.end(), [](const Cand &x, const Cand &y) {
            return x.cn != y.cn ? x.cn < y.cn : x.K < y.K;
        });
    };
    std::vector<int64_t> ncol(static_cast<size_t>(nfree)), ncand(static_cast<size_t>(nfree));
    parallel_chunks(nfree, [&](int64_t lo, int64_t hi) {
        std::vector<Cand> cd;
        for (int64_t r = lo; r < hi; r++) {
            candidates(r, cd);
            int64_t m = 0;
            for (size_t u = 0; u < cd.size(); u++)
                if (u == 0 || cd[u].cn != cd[u - 1].cn) m++;
            ncol[r] = m;
            ncand[r] = int64_t(cd.size());
        }
    });
    const int64_t nrows = S->n_rows;
    std::vector<int64_t> rowptr(static_cast<size_t>(nrows) + 1, 0), cbase(size_t(nrows) + 1, 0);
    for (int64_t r = 0; r < nfree; r++)
        for (int i = 0; i < nc; i++) {
            rowptr[r * nc + i + 1] = ncol[r] * nc;
            cbase[r * nc + i + 1] = ncand[r] * nc;
        }
    for (int64_t row = 0; row < nrows; row++) {
        rowptr[row + 1] += rowptr[row];
        cbase[row + 1] += cbase[row];
    }
    const int64_t nnz = rowptr[nrows], ncontrib = cbase[nrows];
    if (ncells * int64_t(ntri) >= (int64_t(1) << 32) || ncells * int64_t(nn) >= (int64_t(1) << 32))
        return set_error(FE_EINVAL, "element storage of 2^32 or more entries");
    std::vector<int32_t> colind(static_cast<size_t>(nnz));
    std::vector<int64_t> gptr(static_cast<size_t>(nnz) + 1), diag(size_t(nrows), -1);
    std::vector<uint32_t> gsrc(static_cast<size_t>(ncontrib));
    parallel_chunks(nfree, [&](int64_t lo, int64_t hi) {
        std::vector<Cand> cd;
        for (int64_t r = lo; r < hi; r++) {
            candidates(r, cd);
            for (int i = 0; i < nc; i++) {
                const int64_t row = r * nc + i;
                int64_t pos = rowptr[row], cpos = cbase[row];
                for (size_t u0 = 0; u0 < cd.size();) {
                    size_t u1 = u0 + 1;
                    while (u1 < cd.size() && cd[u1].cn == cd[u0].cn) u1++;
                    for (int j = 0; j < nc; j++) {
                        const int64_t col = int64_t(cd[u0].cn) * nc + j;
                        colind[pos] = int32_t(col);
                        gptr[pos] = cpos;
                        if (col == row) diag[row] = pos;
                        for (size_t u = u0; u < u1; u++) {
                            const int I = cd[u].a * nc + i, J = cd[u].b * nc + j;
                            const int lo2 = std::min(I, J), hi2 = std::max(I, J);
                            const int t = lo2 * nloc - lo2 * (lo2 - 1) / 2 + (hi2 - lo2);
                            gsrc[cpos++] = uint32_t(cd[u].K * ntri + t);
                        }
                        pos++;
                    }
                    u0 = u1;
                }
            }
        }
    });
    gptr[nnz] = ncontrib;
    S->nnz = nnz;
    S->ncontrib = ncontrib;
    S->h_rowptr.swap(rowptr);
    S->h_colind.swap(colind);
    // device copies
    fe_status st = sx_upload(S->cell_dofs, cdofs.data(), cdofs.size());
    if (st == FE_OK) st = sx_upload(S->gptr, gptr.data(), gptr.size());
    if (st == FE_OK) st = sx_upload(S->gsrc, gsrc.data(), gsrc.size());
    if (st == FE_OK) st = sx_upload(S->diag, diag.data(), diag.size());
    if (st == FE_OK) st = sx_upload(S->optr, optr.data(), optr.size());
    if (st == FE_OK) st = sx_upload(S->oidx, oidx.data(), oidx.size());
    return st;
}

fe_status sx_setup(fe_simplex S, const int32_t *cells, const double *vxyz)
{
    const int dim = S->dim, k = S->k, nn = S->nn, nv = dim + 1;
    const int64_t ncells = S->ncells;
    std::vector<int> sl;
    sx_lattice(dim, k, sl);
    // barycentric weights of every local node
    std::vector<std::array<int, 4>> beta(nn);
    for (int a = 0; a < nn; a++) {
        int sum = 0;
        for (int r = 0; r < dim; r++) {
            beta[a][r + 1] = sl[3 * a + r];
            sum += sl[3 * a + r];
        }
        beta[a][0] = k - sum;
        for (int r = dim + 1; r < 4; r++) beta[a][r] = 0;
    }
    // edges (3D: 6 per cell) and facets (2D: the 3 edges; 3D: the 4 faces)
    std::vector<Facet> frec(static_cast<size_t>(ncells) * nv);
    for (int64_t K = 0; K < ncells; K++)
        for (int j = 0; j < nv; j++) {
            Facet &f = frec[K * nv + j];
            int m = 0;
            for (int i = 0; i < nv; i++)
                if (i != j) f.v[m++] = cells[K * nv + i];
            std::sort(f.v.begin(), f.v.begin() + m);
            if (m == 2) f.v[2] = -1;
            f.cell = K;
            f.j = j;
        }
    std::vector<std::array<int32_t, 3>> fkeys, ekeys;
    std::vector<int32_t> fcount, ecount;
    unique_keys(frec, fkeys, fcount);
    for (int32_t c : fcount)
        if (c > 2) return set_error(FE_EMESH, "a facet is shared by more than two cells");
    if (dim == 3) {
        std::vector<Facet> erec(static_cast<size_t>(ncells) * 6);
        for (int64_t K = 0; K < ncells; K++) {
            int e = 0;
            for (int i = 0; i < 4; i++)
                for (int j = i + 1; j < 4; j++, e++) {
                    Facet &f = erec[K * 6 + e];
                    const int32_t x = cells[K * 4 + i], y = cells[K * 4 + j];
                    f.v = {std::min(x, y), std::max(x, y), -1};
                    f.cell = K;
                    f.j = e;
                }
        }
        unique_keys(erec, ekeys, ecount);
    }
    const std::vector<std::array<int32_t, 3>> &edges = dim == 3 ? ekeys : fkeys;
    // sub-simplex slot counts: nodes strictly inside an edge, face, tetrahedron
    const int64_t ne = int64_t(edges.size()), nf = dim == 3 ? int64_t(fkeys.size()) : 0;
    const int64_t se = k - 1, sf = int64_t(std::max(k - 2, 0)) * std::max(k - 2, 0),
                  sc = dim == 3 ? int64_t(std::max(k - 3, 0)) * std::max(k - 3, 0) * std::max(k - 3, 0) : sf;
    const int64_t base_e = S->nverts, base_f = base_e + ne * se, base_c = base_f + nf * sf;
    const int64_t nprelim = base_c + ncells * sc;
    // preliminary node names of every (cell, local node)
    std::vector<int64_t> pre(static_cast<size_t>(ncells) * nn);
    parallel_chunks(ncells, [&](int64_t lo, int64_t hi) {
        for (int64_t K = lo; K < hi; K++)
            for (int a = 0; a < nn; a++) {
                int32_t vv[4];
                int ww[4], m = 0;
                for (int j = 0; j < nv; j++)
                    if (beta[a][j] > 0) {
                        vv[m] = cells[K * nv + j];
                        ww[m] = beta[a][j];
                        m++;
                    }
                // ascending vertex ids
                for (int i = 1; i < m; i++)
                    for (int j = i; j > 0 && vv[j - 1] > vv[j]; j--) {
                        std::swap(vv[j - 1], vv[j]);
                        std::swap(ww[j - 1], ww[j]);
                    }
                int64_t p;
                if (m == 1) {
                    p = vv[0];
                } else if (m == 2) {
                    p = base_e + key_index(edges, {vv[0], vv[1], -1}) * se + (ww[1] - 1);
                } else if (m == 3 && dim == 3) {
                    p = base_f + key_index(fkeys, {vv[0], vv[1], vv[2]}) * sf + (ww[0] - 1) * (k - 2) + (ww[1] - 1);
                } else if (m == 3) {  // interior of a triangle
                    p = base_c + K * sc + (ww[0] - 1) * (k - 2) + (ww[1] - 1);
                } else {  // interior of a tetrahedron
                    p = base_c + K * sc + ((ww[0] - 1) * (k - 3) + (ww[1] - 1)) * (k - 3) + (ww[2] - 1);
                }
                pre[K * nn + a] = p;
            }
    });
    // global ids by first appearance
    std::vector<int64_t> gid(static_cast<size_t>(nprelim), -1);
    int64_t nnodes = 0;
    for (int64_t t = 0; t < ncells * nn; t++) {
        int64_t &g = gid[pre[t]];
        if (g < 0) g = nnodes++;
        pre[t] = g;
    }
    std::vector<int64_t>().swap(gid);
    S->nnodes = nnodes;
    // boundary nodes: the nodes of facets of one cell
    std::vector<char> bnd(static_cast<size_t>(nnodes), 0);
    if (S->fix_boundary) {
        for (size_t t = 0; t < frec.size();) {
            size_t u = t + 1;
            while (u < frec.size() && frec[u].v == frec[t].v) u++;
            if (u - t == 1) {
                const int64_t K = frec[t].cell;
                const int j = frec[t].j;
                for (int a = 0; a < nn; a++)
                    if (beta[a][j] == 0) bnd[pre[K * nn + a]] = 1;
            }
            t = u;
        }
    }
    std::vector<Facet>().swap(frec);
    return sx_finish(S, pre, nnodes, bnd);
}

// Local DOF a of a vector family: its entity kind (0 edge, 1 facet, 2 the
// cell's interior), the entity's local index and the DOF's slot in it.
void sxv_dof(int fam, int dim, int a, int &kind, int &ent, int &slot)
{
    const int ne = dim == 3 ? 6 : 3;
    if (fam == 1) {
        kind = 0, ent = a, slot = 0;
    } else if (fam == 2) {
        kind = 1, ent = a, slot = 0;
    } else if (fam == 4) {  // facet a / d, slot a % d (its vertices); then the interior
        if (a < dim * (dim + 1))
            kind = 1, ent = a / dim, slot = a % dim;
        else
            kind = 2, ent = 0, slot = a - dim * (dim + 1);
    } else if (a < 2 * ne) {
        kind = 0, ent = a / 2, slot = a % 2;
    } else if (dim == 3) {
        kind = 1, ent = (a - 12) / 2, slot = (a - 12) % 2;
    } else {
        kind = 2, ent = 0, slot = a - 6;
    }
}

void sxv_edge(int dim, int e, int &i, int &j)
{
    i = dim == 3 ? (e < 3 ? 0 : e < 5 ? 1 : 2) : (e < 2 ? 0 : 1);
    j = dim == 3 ? (e < 3 ? e + 1 : e < 5 ? e - 1 : 3) : (e < 2 ? e + 1 : 2);
}

// DOF entities of the vector families: a DOF is named by its entity's sorted
// vertex ids (an edge's, a facet's, or for the interior DOFs of a 2D cell the
// cell's) and its slot; ids by first appearance over (cell, local DOF);
// boundary DOFs are those of entities on a facet of one cell.
fe_status sxv_setup(fe_simplex S, const int32_t *cells)
{
    const int dim = S->dim, nv = dim + 1, nd = S->nn, fam = S->family;
    const int64_t ncells = S->ncells;
    struct DofRec {
        std::array<int32_t, 5> key;  // sorted vertex ids (up to a tetrahedron's four, padded with -1), slot
        int64_t cell;
        int32_t a;
    };
    std::vector<DofRec> rec(static_cast<size_t>(ncells) * nd);
    std::vector<Facet> frec(static_cast<size_t>(ncells) * nv);
    for (int64_t K = 0; K < ncells; K++) {
        for (int a = 0; a < nd; a++) {
            int kind, ent, slot;
            sxv_dof(fam, dim, a, kind, ent, slot);
            std::array<int32_t, 5> k{-1, -1, -1, -1, slot};
            int m = 0;
            if (kind == 0) {
                int i, j;
                sxv_edge(dim, ent, i, j);
                k[m++] = cells[K * nv + i];
                k[m++] = cells[K * nv + j];
            } else if (kind == 1) {
                for (int r = 0; r < nv; r++)
                    if (r != ent) k[m++] = cells[K * nv + r];
            } else {
                for (int r = 0; r < nv; r++) k[m++] = cells[K * nv + r];
            }
            std::sort(k.begin(), k.begin() + m);
            rec[K * nd + a] = DofRec{k, K, a};
        }
        for (int j = 0; j < nv; j++) {
            Facet &f = frec[K * nv + j];
            int m = 0;
            for (int r = 0; r < nv; r++)
                if (r != j) f.v[m++] = cells[K * nv + r];
            std::sort(f.v.begin(), f.v.begin() + m);
            for (int r = m; r < 3; r++) f.v[r] = -1;
            f.cell = K;
            f.j = j;
        }
    }
    std::vector<std::array<int32_t, 3>> fkeys;
    std::vector<int32_t> fcount;
    unique_keys(frec, fkeys, fcount);
    for (int32_t c : fcount)
        if (c > 2) return set_error(FE_EMESH, "a facet is shared by more than two cells");
    std::sort(rec.begin(), rec.end(), [](const DofRec &x, const DofRec &y) {
        if (x.key != y.key) return x.key < y.key;
        if (x.cell != y.cell) return x.cell < y.cell;
        return x.a < y.a;
    });
    // group id of every (cell, local DOF), then ids by first appearance
    std::vector<int64_t> pre(static_cast<size_t>(ncells) * nd);
    int64_t ngrp = 0;
    for (size_t t = 0; t < rec.size(); t++) {
        if (t > 0 && rec[t].key != rec[t - 1].key) ngrp++;
        pre[rec[t].cell * nd + rec[t].a] = ngrp;
    }
    if (!rec.empty()) ngrp++;
    std::vector<DofRec>().swap(rec);
    std::vector<int64_t> gid(static_cast<size_t>(ngrp), -1);
    int64_t nent = 0;
    for (int64_t t = 0; t < ncells * nd; t++) {
        int64_t &g = gid[pre[t]];
        if (g < 0) g = nent++;
        pre[t] = g;
    }
    std::vector<char> bnd(static_cast<size_t>(nent), 0);
    if (S->fix_boundary)
        for (size_t t = 0; t < frec.size();) {
            size_t u = t + 1;
            while (u < frec.size() && frec[u].v == frec[t].v) u++;
            if (u - t == 1) {
                const int64_t K = frec[t].cell;
                const int j = frec[t].j;
                for (int a = 0; a < nd; a++) {
                    int kind, ent, slot;
                    sxv_dof(fam, dim, a, kind, ent, slot);
                    bool on = false;
                    if (kind == 1) {
                        on = ent == j;
                    } else if (kind == 0) {
                        int i1, j1;
                        sxv_edge(dim, ent, i1, j1);
                        on = i1 != j && j1 != j;
                    }
                    if (on) bnd[pre[K * nd + a]] = 1;
                }
            }
            t = u;
        }
    return sx_finish(S, pre, nent, bnd);
}

// Pre-basis of the vector family at x: value v and Jacobian dv[c dim + r].
// Families 1-2: constants e_b first, then Nedelec rotations (2D (-y, x); 3D
// e_m x x) or the Raviart-Thomas field x.  Family 3: [P_1]^d (component
// b / (d+1) times 1, x_0, ..), then the quadratic fields orthogonal to x:
// 2D x_m (-y, x); 3D x_j (x cross e_i) for the pairs (i, j) but (2, 2).
void sxv_prebasis(int fam, int dim, int b, const double *x, double *v, double *dv)
{
    for (int c = 0; c < 3; c++) v[c] = 0.0;
    for (int t = 0; t < 9; t++) dv[t] = 0.0;
    if (fam == 4 && b >= dim * (dim + 1)) {  // x times x_m
        const int m = b - dim * (dim + 1);
        for (int c = 0; c < dim; c++) {
            v[c] = x[c] * x[m];
            dv[c * dim + c] += x[m];
            dv[c * dim + m] += x[c];
        }
        return;
    }
    if (fam == 3 || fam == 4) {
        if (b < dim * (dim + 1)) {
            const int c = b / (dim + 1), m = b % (dim + 1);
            v[c] = m == 0 ? 1.0 : x[m - 1];
            if (m > 0) dv[c * dim + m - 1] = 1.0;
            return;
        }
        const int q = b - dim * (dim + 1);
        if (dim == 2) {
            const double R[2] = {-x[1], x[0]};
            v[0] = x[q] * R[0];
            v[1] = x[q] * R[1];
            dv[q] += R[0];
            dv[2 + q] += R[1];
            dv[1] += -x[q];
            dv[2] += x[q];
            return;
        }
        const int i = q / 3, j = q % 3;
        double R[3] = {0, 0, 0}, dR[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        // x cross e_i = x_{i+2} e_{i+1} - x_{i+1} e_{i+2}, indices mod 3
        const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
        R[i1] = x[i2];
        R[i2] = -x[i1];
        dR[i1 * 3 + i2] = 1.0;
        dR[i2 * 3 + i1] = -1.0;
        for (int c = 0; c < 3; c++) {
            v[c] = x[j] * R[c];
            for (int r = 0; r < 3; r++) dv[c * 3 + r] = (r == j ? R[c] : 0.0) + x[j] * dR[c * 3 + r];
        }
        return;
    }
    if (b < dim) {
        v[b] = 1.0;
    } else if (fam == 2) {
        for (int c = 0; c < dim; c++) {
            v[c] = x[c];
            dv[c * dim + c] = 1.0;
        }
    } else if (dim == 2) {
        v[0] = -x[1];
        v[1] = x[0];
        dv[1] = -1.0;
        dv[2] = 1.0;
    } else {
        const int m = b - 3, p = (m + 1) % 3, q = (m + 2) % 3;
        v[p] = -x[q];
        v[q] = x[p];
        dv[p * 3 + q] = -1.0;
        dv[q * 3 + p] = 1.0;
    }
}

// Degrees of freedom on the reference simplex: along edge (i, j) the line
// integral of v with tangent x_j - x_i (family 3: weighted by 1 - t and t);
// on the facet opposite vertex a (vertices in ascending local order) the flux
// with N (family 2) or, family 3, the integrals of v against the tangents
// x_i1 - x_i0 and x_i2 - x_i0; family 3 in 2D: the interior moments of v's
// components on the reference triangle.
double sxv_moment(int fam, int dim, int a, int b)
{
    double gx[4], gw[4];
    gauss_legendre_01(3, gx, gw);
    auto vert = [dim](int r, double *x) {
        for (int t = 0; t < dim; t++) x[t] = (r > 0 && t == r - 1) ? 1.0 : 0.0;
    };
    int kind, ent, slot;
    sxv_dof(fam, dim, a, kind, ent, slot);
    double v[3], dv[9], p[3] = {0, 0, 0};
    double s = 0.0;
    if (kind == 0) {
        int i, j;
        sxv_edge(dim, ent, i, j);
        double xi[3], xj[3];
        vert(i, xi);
        vert(j, xj);
        for (int q = 0; q < 3; q++) {
            for (int t = 0; t < dim; t++) p[t] = xi[t] + gx[q] * (xj[t] - xi[t]);
            sxv_prebasis(fam, dim, b, p, v, dv);
            double d = 0.0;
            for (int t = 0; t < dim; t++) d += v[t] * (xj[t] - xi[t]);
            const double w = fam != 3 ? 1.0 : slot == 0 ? 1.0 - gx[q] : gx[q];
            s += gw[q] * d * w;
        }
        return s;
    }
    // a degree-4 rule on the reference triangle (the collapsed 3 x 3 Gauss rule)
    auto triangle = [&](auto &&f) {
        double acc = 0.0;
        for (int q0 = 0; q0 < 3; q0++)
            for (int q1 = 0; q1 < 3; q1++) {
                const double u0 = gx[q0], u1 = (1.0 - gx[q0]) * gx[q1];
                acc += gw[q0] * gw[q1] * (1.0 - gx[q0]) * f(u0, u1);
            }
        return acc;
    };
    if (kind == 2 && dim == 3) {  // interior moments on the reference tetrahedron (degree 5)
        std::vector<double> r;
        sx_rule(3, 3, r);
        for (size_t q = 0; q < r.size() / 4; q++) {
            sxv_prebasis(fam, dim, b, &r[q * 4], v, dv);
            s += r[q * 4 + 3] * v[slot];
        }
        return s;
    }
    if (kind == 2) {
        return triangle([&](double u0, double u1) {
            double x[3] = {u0, u1, 0.0};
            sxv_prebasis(fam, dim, b, x, v, dv);
            return v[slot];
        });
    }
    int iv[3], m = 0;
    for (int r = 0; r <= dim; r++)
        if (r != ent) iv[m++] = r;
    double x0[3] = {0, 0, 0}, x1[3] = {0, 0, 0}, x2[3] = {0, 0, 0}, N[3] = {0, 0, 0};
    vert(iv[0], x0);
    vert(iv[1], x1);
    if (dim == 3) vert(iv[2], x2);
    if (dim == 2) {
        N[0] = x1[1] - x0[1];
        N[1] = x0[0] - x1[0];
        for (int q = 0; q < 3; q++) {
            for (int t = 0; t < 2; t++) p[t] = x0[t] + gx[q] * (x1[t] - x0[t]);
            sxv_prebasis(fam, dim, b, p, v, dv);
            // family 4: against the barycentric of the facet's vertex `slot`
            const double lam = fam != 4 ? 1.0 : slot == 0 ? 1.0 - gx[q] : gx[q];
            s += gw[q] * (v[0] * N[0] + v[1] * N[1]) * lam;
        }
        return s;
    }
    double t1[3], t2[3];
    for (int t = 0; t < 3; t++) {
        t1[t] = x1[t] - x0[t];
        t2[t] = x2[t] - x0[t];
    }
    if (fam == 2 || fam == 4) {
        N[0] = t1[1] * t2[2] - t1[2] * t2[1];
        N[1] = t1[2] * t2[0] - t1[0] * t2[2];
        N[2] = t1[0] * t2[1] - t1[1] * t2[0];
    } else {
        for (int t = 0; t < 3; t++) N[t] = slot == 0 ? t1[t] : t2[t];
    }
    return triangle([&](double u0, double u1) {
        for (int t = 0; t < 3; t++) p[t] = x0[t] + u0 * t1[t] + u1 * t2[t];
        sxv_prebasis(fam, dim, b, p, v, dv);
        const double lam = fam != 4 ? 1.0 : slot == 0 ? 1.0 - u0 - u1 : slot == 1 ? u0 : u1;
        return (v[0] * N[0] + v[1] * N[1] + v[2] * N[2]) * lam;
    });
}

fe_status sxv_tables(fe_simplex S)
{
    const int dim = S->dim, fam = S->family, nd = S->nn, ntri = S->ntri;
    // change of basis: C_ab = sigma_a(psi_b), Phi = C^-T (Gauss-Jordan)
    std::vector<double> M(static_cast<size_t>(nd) * 2 * nd, 0.0);
    for (int a = 0; a < nd; a++) {
        for (int b = 0; b < nd; b++) M[a * 2 * nd + b] = sxv_moment(fam, dim, a, b);
        M[a * 2 * nd + nd + a] = 1.0;
    }
    for (int c = 0; c < nd; c++) {
        int p = c;
        for (int i = c + 1; i < nd; i++)
            if (std::fabs(M[i * 2 * nd + c]) > std::fabs(M[p * 2 * nd + c])) p = i;
        if (M[p * 2 * nd + c] == 0.0) return set_error(FE_EINVAL, "singular change of basis");
        if (p != c)
            for (int j = 0; j < 2 * nd; j++) std::swap(M[c * 2 * nd + j], M[p * 2 * nd + j]);
        const double piv = M[c * 2 * nd + c];
        for (int j = 0; j < 2 * nd; j++) M[c * 2 * nd + j] /= piv;
        for (int i = 0; i < nd; i++)
            if (i != c) {
                const double f = M[i * 2 * nd + c];
                if (f != 0.0)
                    for (int j = 0; j < 2 * nd; j++) M[i * 2 * nd + j] -= f * M[c * 2 * nd + j];
            }
    }
    auto Phi = [&](int a, int b) { return M[b * 2 * nd + nd + a]; };  // (C^-1)_{ba}
    auto shape = [&](const double *x, double *phi, double *cu, double *dvg) {
        for (int a = 0; a < nd; a++) {
            double v[3] = {0, 0, 0}, dv[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (int b = 0; b < nd; b++) {
                double pv[3], pdv[9];
                sxv_prebasis(fam, dim, b, x, pv, pdv);
                for (int c = 0; c < 3; c++) v[c] += Phi(a, b) * pv[c];
                for (int t = 0; t < 9; t++) dv[t] += Phi(a, b) * pdv[t];
            }
            for (int c = 0; c < dim; c++) phi[a * dim + c] = v[c];
            if (dim == 3) {
                cu[a * 3 + 0] = dv[7] - dv[5];
                cu[a * 3 + 1] = dv[2] - dv[6];
                cu[a * 3 + 2] = dv[3] - dv[1];
            } else {
                cu[a] = dv[2] - dv[1];
            }
            dvg[a] = dim == 3 ? dv[0] + dv[4] + dv[8] : dv[0] + dv[3];
        }
    };
    const int nq1 = (fam >= 3 ? 2 : 1) + (dim + 1) / 2;
    std::vector<double> qxw;
    sx_rule(dim, nq1, qxw);
    const int nq = int(qxw.size() / (dim + 1));
    const int ncu = dim == 3 ? 3 : 1;
    std::vector<double> phq(static_cast<size_t>(nq) * nd * dim), cuq(static_cast<size_t>(nq) * nd * ncu),
        dvq(static_cast<size_t>(nq) * nd);
    for (int q = 0; q < nq; q++)
        shape(&qxw[size_t(q) * (dim + 1)], &phq[size_t(q) * nd * dim], &cuq[size_t(q) * nd * ncu],
              &dvq[size_t(q) * nd]);
    const bool hdiv = fam == 2 || fam == 4;
    const int nps = (!hdiv && dim == 3) ? 6 : 1, npm = dim * (dim + 1) / 2;
    std::vector<int32_t> tri(ntri);
    {
        int t = 0;
        for (int I = 0; I < nd; I++)
            for (int J = I; J < nd; J++) tri[t++] = (I << 16) | J;
    }
    // reference products by the rule: stiffness (curl or divergence) then mass
    std::vector<double> tab(static_cast<size_t>(nps + npm) * ntri, 0.0);
    for (int t = 0; t < ntri; t++) {
        const int a = tri[t] >> 16, b = tri[t] & 0xffff;
        for (int q = 0; q < nq; q++) {
            const double w = qxw[size_t(q) * (dim + 1) + dim];
            const double *cu = &cuq[size_t(q) * nd * ncu], *ph = &phq[size_t(q) * nd * dim], *dg = &dvq[size_t(q) * nd];
            if (nps == 6) {
                int p = 0;
                for (int r = 0; r < 3; r++)
                    for (int s = r; s < 3; s++, p++) {
                        double v = cu[a * 3 + r] * cu[b * 3 + s];
                        if (s != r) v += cu[a * 3 + s] * cu[b * 3 + r];
                        tab[size_t(p) * ntri + t] += w * v;
                    }
            } else {
                tab[t] += w * (!hdiv ? cu[a] * cu[b] : dg[a] * dg[b]);
            }
            int p = nps;
            for (int r = 0; r < dim; r++)
                for (int s = r; s < dim; s++, p++) {
                    double pr = ph[a * dim + r] * ph[b * dim + s];
                    if (s != r) pr += ph[a * dim + s] * ph[b * dim + r];
                    tab[size_t(p) * ntri + t] += w * pr;
                }
        }
    }
    fe_status st = sx_upload(S->tab, tab.data(), tab.size());
    if (st == FE_OK) st = sx_upload(S->tri, tri.data(), tri.size());
    if (st == FE_OK) st = sx_upload(S->phiq, phq.data(), phq.size());
    if (st == FE_OK) st = sx_upload(S->qxw, qxw.data(), qxw.size());
    return st;
}

// Reference tables for the element kernel: the coefficient-pair table and the
// entry table, the shape values at the rule's points and the rule itself.
fe_status sx_tables(fe_simplex S)
{
    const int dim = S->dim, k = S->k, nn = S->nn, nc = S->ncomp, nloc = S->nloc, ntri = S->ntri;
    SxRef R;
    if (!sx_reference(dim, k, R) || R.nn != nn) return set_error(FE_EINVAL, "singular change of basis");
    const int nq1 = k + (dim + 1) / 2;
    std::vector<double> qxw;
    sx_rule(dim, nq1, qxw);
    const int nq = int(qxw.size() / (dim + 1));
    std::vector<double> phiq(static_cast<size_t>(nq) * nn), dphi(size_t(nq) * nn * dim);
    for (int q = 0; q < nq; q++) sx_eval(dim, R, &qxw[size_t(q) * (dim + 1)], &phiq[size_t(q) * nn], &dphi[size_t(q) * nn * dim]);
    // S^{rs}_ab = sum_q w_q d_r phi_a d_s phi_b
    std::vector<double> Sg(static_cast<size_t>(dim) * dim * nn * nn, 0.0);
    for (int q = 0; q < nq; q++) {
        const double w = qxw[size_t(q) * (dim + 1) + dim];
        const double *g = &dphi[size_t(q) * nn * dim];
        for (int r = 0; r < dim; r++)
            for (int s = 0; s < dim; s++)
                for (int a = 0; a < nn; a++)
                    for (int b = 0; b < nn; b++)
                        Sg[((size_t(r) * dim + s) * nn + a) * nn + b] += w * g[a * dim + r] * g[b * dim + s];
    }
    std::vector<double> tab;
    std::vector<int32_t> tri(ntri);
    {
        int t = 0;
        for (int I = 0; I < nloc; I++)
            for (int J = I; J < nloc; J++) tri[t++] = (I << 16) | J;
    }
    if (S->args.problem == FE_ELASTICITY) {
        tab = Sg;
    } else {
        const int np = dim * (dim + 1) / 2;
        tab.assign(size_t(np) * ntri, 0.0);
        int p = 0;
        for (int r = 0; r < dim; r++)
            for (int s = r; s < dim; s++, p++)
                for (int t = 0; t < ntri; t++) {
                    const int a = tri[t] >> 16, b = tri[t] & 0xffff;
                    double v = Sg[((size_t(r) * dim + s) * nn + a) * nn + b];
                    if (s != r) v += Sg[((size_t(s) * dim + r) * nn + a) * nn + b];
                    tab[size_t(p) * ntri + t] = v;
                }
    }
    (void)nc;
    fe_status st = sx_upload(S->tab, tab.data(), tab.size());
    if (st == FE_OK) st = sx_upload(S->tri, tri.data(), tri.size());
    if (st == FE_OK) st = sx_upload(S->phiq, phiq.data(), phiq.size());
    if (st == FE_OK) st = sx_upload(S->qxw, qxw.data(), qxw.size());
    return st;
}

template <int DIM, int K, int PROB>
fe_status launch_sx_elements(fe_simplex S, hipStream_t s)
{
    using Sh = SxShape<DIM, K, PROB>;
    const int64_t nb = (S->ncells + Sh::CPB - 1) / Sh::CPB;
    if (nb == 0) return FE_OK;
    hipLaunchKernelGGL((sx_element_kernel<DIM, K, PROB>), dim3(unsigned(nb)), dim3(256), 0, s, S->args, S->vxyz,
                       S->cells, S->coef, S->cell_dofs, S->tab, S->tri, S->phiq, S->qxw, S->E, S->F);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

template <int DIM, int FAM>
fe_status launch_sx_vector(fe_simplex S, hipStream_t s)
{
    using Sh = SxvShape<DIM, FAM>;
    const int64_t nb = (S->ncells + Sh::CPB - 1) / Sh::CPB;
    if (nb == 0) return FE_OK;
    hipLaunchKernelGGL((sx_vector_kernel<DIM, FAM>), dim3(unsigned(nb)), dim3(256), 0, s, S->args, S->kappa, S->vxyz,
                       S->cells, S->coef, S->tab, S->tri, S->phiq, S->qxw, S->E, S->F);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

template <int DIM>
fe_status launch_sx_nedelec2(fe_simplex S, hipStream_t s)
{
    using Sh = Sxn2Shape<DIM>;
    const int64_t nb = (S->ncells + Sh::CPB - 1) / Sh::CPB;
    if (nb == 0) return FE_OK;
    hipLaunchKernelGGL((sx_nedelec2_kernel<DIM>), dim3(unsigned(nb)), dim3(256), 0, s, S->args, S->kappa, S->vxyz,
                       S->cells, S->coef, S->tab, S->tri, S->phiq, S->qxw, S->E, S->F);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

template <int DIM>
fe_status launch_sx_rt2(fe_simplex S, hipStream_t s)
{
    using Sh = SxRt2Shape<DIM>;
    const int64_t nb = (S->ncells + Sh::CPB - 1) / Sh::CPB;
    if (nb == 0) return FE_OK;
    hipLaunchKernelGGL((sx_rt2_kernel<DIM>), dim3(unsigned(nb)), dim3(256), 0, s, S->args, S->kappa, S->vxyz, S->cells,
                       S->coef, S->tab, S->tri, S->phiq, S->qxw, S->E, S->F);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

fe_status launch_elements(fe_simplex S, hipStream_t s)
{
    if (S->family == 3) return S->dim == 3 ? launch_sx_nedelec2<3>(S, s) : launch_sx_nedelec2<2>(S, s);
    if (S->family == 4) return S->dim == 3 ? launch_sx_rt2<3>(S, s) : launch_sx_rt2<2>(S, s);
    if (S->family == 1) return S->dim == 3 ? launch_sx_vector<3, 1>(S, s) : launch_sx_vector<2, 1>(S, s);
    if (S->family == 2) return S->dim == 3 ? launch_sx_vector<3, 2>(S, s) : launch_sx_vector<2, 2>(S, s);
    const bool el = S->args.problem == FE_ELASTICITY;
#define FE_SXL(D, KK)                                                                              \
    return el ? launch_sx_elements<D, KK, FE_ELASTICITY>(S, s) : launch_sx_elements<D, KK, FE_POISSON>(S, s)
    if (S->dim == 2) {
        switch (S->k) {
            case 1: FE_SXL(2, 1);
            case 2: FE_SXL(2, 2);
            case 3: FE_SXL(2, 3);
            default: return launch_sx_elements<2, 4, FE_POISSON>(S, s);
        }
    }
    switch (S->k) {
        case 1: FE_SXL(3, 1);
        case 2: FE_SXL(3, 2);
        case 3: FE_SXL(3, 3);
        default: return launch_sx_elements<3, 4, FE_POISSON>(S, s);
    }
#undef FE_SXL
}

// Mesh checks shared by the create calls (host only): sizes, vertex ids in
// range, no degenerate cell (either orientation is accepted).
fe_status sx_validate(const fe_simplex_desc *desc)
{
    const int dim = desc->dim;
    if (desc->nverts < 0 || desc->ncells < 0) return set_error(FE_EINVAL, "negative sizes");
    if (desc->ncells > 0 && (!desc->cells || !desc->vertex_xyz)) return set_error(FE_EINVAL, "null mesh arrays");
    if (desc->nverts >= (int64_t(1) << 31)) return set_error(FE_EINVAL, "2^31 or more vertices");
    const int nv = dim + 1;
    for (int64_t t = 0; t < desc->ncells * nv; t++)
        if (desc->cells[t] < 0 || desc->cells[t] >= desc->nverts) return set_error(FE_EMESH, "vertex id out of range");
    // degenerate cells (det J = 0) are rejected; either orientation is accepted
    for (int64_t K = 0; K < desc->ncells; K++) {
        double J[3][3];
        const double *x0 = desc->vertex_xyz + int64_t(desc->cells[K * nv]) * dim;
        for (int s = 0; s < dim; s++) {
            const double *xs = desc->vertex_xyz + int64_t(desc->cells[K * nv + s + 1]) * dim;
            for (int r = 0; r < dim; r++) J[r][s] = xs[r] - x0[r];
        }
        const double det = dim == 2 ? J[0][0] * J[1][1] - J[0][1] * J[1][0]
                                    : J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                          J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                          J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        if (!(det != 0.0) || !std::isfinite(det)) return set_error(FE_EMESH, "degenerate simplex (det J = 0)");
    }
    return FE_OK;
}

// Device copies of the mesh and the element storage.
fe_status sx_upload_mesh(fe_simplex S, const fe_simplex_desc *desc)
{
    fe_status st = sx_upload(S->vxyz, desc->vertex_xyz, size_t(desc->nverts) * S->dim);
    if (st == FE_OK) st = sx_upload(S->cells, desc->cells, size_t(desc->ncells) * (S->dim + 1));
    if (st == FE_OK && desc->cell_coeff) st = sx_upload(S->coef, desc->cell_coeff, size_t(desc->ncells));
    if (st == FE_OK) st = sx_alloc(S->E, size_t(S->ncells) * S->ntri);
    if (st == FE_OK) st = sx_alloc(S->F, size_t(S->ncells) * S->nloc);
    return st;
}

unsigned blocks_of(int64_t n) { return unsigned(std::max<int64_t>(1, (n + 255) / 256)); }

}  // namespace

extern "C" {

fe_status fe_simplex_create(const fe_simplex_desc *desc, int32_t order, const fe_coeff *coeff, fe_simplex *out)
{
    if (!desc || !coeff || !out) return set_error(FE_EINVAL, "null argument");
    *out = nullptr;
    const int dim = desc->dim;
    if (dim != 2 && dim != 3) return set_error(FE_EINVAL, "dim must be 2 or 3");
    if (order < 1 || order > kSxMaxK) return set_error(FE_EINVAL, "order must be in 1..4");
    if (coeff->problem != FE_POISSON && coeff->problem != FE_ELASTICITY)
        return set_error(FE_EINVAL, "unknown problem");
    if (coeff->problem == FE_ELASTICITY && order > 3)
        return set_error(FE_EINVAL, "elasticity on simplices supports orders 1..3");
    if (coeff->precision != FE_FP64) return set_error(FE_EINVAL, "simplices integrate in FP64 only");
    if (coeff->source_kind < FE_SOURCE_NONE || coeff->source_kind > FE_SOURCE_SINPROD)
        return set_error(FE_EINVAL, "unknown source kind");
    if (coeff->dirichlet_kind != FE_DIRICHLET_ZERO && coeff->dirichlet_kind != FE_DIRICHLET_AFFINE)
        return set_error(FE_EINVAL, "unknown Dirichlet kind");
    fe_status vst = sx_validate(desc);
    if (vst != FE_OK) return vst;
    fe_simplex S = new fe_simplex_s();
    S->dim = dim;
    S->k = order;
    S->nn = sx_nn(dim, order);
    S->ncomp = coeff->problem == FE_ELASTICITY ? dim : 1;
    S->nloc = S->nn * S->ncomp;
    S->ntri = S->nloc * (S->nloc + 1) / 2;
    S->nverts = desc->nverts;
    S->ncells = desc->ncells;
    SxArgs &a = S->args;
    a.problem = coeff->problem;
    a.source_kind = coeff->source_kind;
    a.dirichlet_kind = coeff->dirichlet_kind;
    for (int i = 0; i < 3; i++) a.source[i] = coeff->source[i];
    for (int i = 0; i < 12; i++) a.aff[i] = coeff->dirichlet_affine[i];
    if (coeff->problem == FE_ELASTICITY) {
        const double E = coeff->young, nu = coeff->poisson_ratio;
        if (!(nu > -1.0 && nu < 0.5)) {
            delete S;
            return set_error(FE_EINVAL, "poisson_ratio must be in (-1, 0.5)");
        }
        a.lambda = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
        a.mu = E / (2.0 * (1.0 + nu));
    }
    a.ncells = desc->ncells;
    {
        std::vector<int> sl;
        sx_lattice(dim, order, sl);
        for (size_t t = 0; t < sl.size(); t++) a.s[t] = int8_t(sl[t]);
    }
    // every node of a boundary facet is fixed when dirichlet_faces != 0
    S->fix_boundary = coeff->dirichlet_faces != 0;
    fe_status st = sx_setup(S, desc->cells, desc->vertex_xyz);
    if (st == FE_OK) st = sx_tables(S);
    if (st == FE_OK) st = sx_upload_mesh(S, desc);
    if (st != FE_OK) {
        sx_free(S);
        return st;
    }
    *out = S;
    return FE_OK;
}

fe_status fe_simplex_create_vector(const fe_simplex_desc *desc, int32_t family, double kappa, const fe_coeff *coeff,
                                   fe_simplex *out)
{
    if (!desc || !coeff || !out) return set_error(FE_EINVAL, "null argument");
    *out = nullptr;
    const int dim = desc->dim;
    if (dim != 2 && dim != 3) return set_error(FE_EINVAL, "dim must be 2 or 3");
    if (family != FE_NEDELEC && family != FE_RAVIART_THOMAS && family != FE_NEDELEC2 && family != FE_RAVIART_THOMAS2)
        return set_error(FE_EINVAL, "unknown element family");
    if (!(kappa >= 0.0) || !std::isfinite(kappa)) return set_error(FE_EINVAL, "kappa must be finite and >= 0");
    if (coeff->precision != FE_FP64) return set_error(FE_EINVAL, "simplices integrate in FP64 only");
    if (coeff->source_kind < FE_SOURCE_NONE || coeff->source_kind > FE_SOURCE_SINPROD)
        return set_error(FE_EINVAL, "unknown source kind");
    if (coeff->dirichlet_kind != FE_DIRICHLET_ZERO)
        return set_error(FE_EINVAL, "vector elements take zero boundary traces only");
    fe_status vst = sx_validate(desc);
    if (vst != FE_OK) return vst;
    fe_simplex S = new fe_simplex_s();
    S->dim = dim;
    S->k = 0;
    S->family = family;
    S->kappa = kappa;
    S->nn = family == FE_NEDELEC        ? (dim == 3 ? 6 : 3)
            : family == FE_NEDELEC2       ? (dim == 3 ? 20 : 8)
            : family == FE_RAVIART_THOMAS2 ? (dim == 3 ? 15 : 8)
                                           : dim + 1;
    S->ncomp = 1;
    S->nloc = S->nn;
    S->ntri = S->nloc * (S->nloc + 1) / 2;
    S->nverts = desc->nverts;
    S->ncells = desc->ncells;
    SxArgs &a = S->args;
    a.problem = -1;
    a.source_kind = coeff->source_kind;
    a.dirichlet_kind = FE_DIRICHLET_ZERO;
    for (int i = 0; i < 3; i++) a.source[i] = coeff->source[i];
    a.ncells = desc->ncells;
    S->fix_boundary = coeff->dirichlet_faces != 0;
    fe_status st = sxv_setup(S, desc->cells);
    if (st == FE_OK) st = sxv_tables(S);
    if (st == FE_OK) st = sx_upload_mesh(S, desc);
    if (st != FE_OK) {
        sx_free(S);
        return st;
    }
    *out = S;
    return FE_OK;
}

fe_status fe_simplex_destroy(fe_simplex S)
{
    if (!S) return set_error(FE_EINVAL, "null handle");
    (void)hipDeviceSynchronize();
    sx_free(S);
    return FE_OK;
}

fe_status fe_simplex_query(fe_simplex S, int64_t *n_rows, int64_t *nnz, int64_t *n_nodes, int64_t *n_contrib)
{
    if (!S) return set_error(FE_EINVAL, "null handle");
    if (n_rows) *n_rows = S->n_rows;
    if (nnz) *nnz = S->nnz;
    if (n_nodes) *n_nodes = S->nnodes;
    if (n_contrib) *n_contrib = S->ncontrib;
    return FE_OK;
}

fe_status fe_simplex_cell_dofs(fe_simplex S, int32_t *cell_dofs, fe_stream stream)
{
    if (!S || !cell_dofs) return set_error(FE_EINVAL, "null argument");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (S->ncells > 0)
        FE_HIP(hipMemcpyAsync(cell_dofs, S->cell_dofs, sizeof(int32_t) * size_t(S->ncells) * S->nloc,
                              hipMemcpyDeviceToDevice, s));
    return FE_OK;
}

fe_status fe_simplex_pattern(fe_simplex S, const fe_csr *A, fe_stream stream)
{
    if (!S || !A || !A->rowptr || (S->nnz > 0 && !A->colind)) return set_error(FE_EINVAL, "null argument");
    if (A->n_rows != S->n_rows || A->nnz != S->nnz) return set_error(FE_EINVAL, "CSR sizes do not match the space");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    FE_HIP(hipMemcpyAsync(A->rowptr, S->h_rowptr.data(), sizeof(int64_t) * S->h_rowptr.size(), hipMemcpyHostToDevice,
                          s));
    if (S->nnz > 0)
        FE_HIP(hipMemcpyAsync(A->colind, S->h_colind.data(), sizeof(int32_t) * S->h_colind.size(),
                              hipMemcpyHostToDevice, s));
    FE_HIP(hipStreamSynchronize(s));
    return FE_OK;
}

fe_status fe_simplex_assemble(fe_simplex S, const fe_csr *A, fe_stream stream)
{
    if (!S || !A || (S->nnz > 0 && !A->values) || (S->n_rows > 0 && (!A->rhs || !A->dinv)))
        return set_error(FE_EINVAL, "null argument");
    if (A->n_rows != S->n_rows || A->nnz != S->nnz) return set_error(FE_EINVAL, "CSR sizes do not match the space");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    fe_status st = launch_elements(S, s);
    if (st != FE_OK) return st;
    if (S->nnz > 0)
        hipLaunchKernelGGL(sx_gather_kernel, dim3(blocks_of(S->nnz)), dim3(256), 0, s, S->nnz, S->gptr, S->gsrc, S->E,
                           A->values);
    if (S->n_rows > 0)
        hipLaunchKernelGGL(sx_rhs_kernel, dim3(blocks_of(S->n_rows)), dim3(256), 0, s, S->n_rows, S->ncomp, S->optr,
                           S->oidx, S->F, S->diag, A->values, A->rhs, A->dinv);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

fe_status fe_simplex_elements(fe_simplex S, const double **E, const double **F)
{
    if (!S) return set_error(FE_EINVAL, "null handle");
    if (E) *E = S->E;
    if (F) *F = S->F;
    return FE_OK;
}

}  // extern "C"
