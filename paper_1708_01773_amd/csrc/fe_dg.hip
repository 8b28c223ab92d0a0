// fe_dg.hip -- interior-penalty discontinuous Galerkin for -Laplace(u) = f on
// the brick (Sect. 3.12 eq. ip_dg_formulations; the facet matrices of eq.
// local_to_face_matrix; facet integration of Sect. 3.13).
//
// Space: Q_k on every cell with no DOF shared between cells, DOF(K, a) =
// K nn + a (local node order of the conforming space).  The CSR row of
// DOF(K, a) holds the nn columns of K and of each facet neighbour of K, cells
// in ascending order, so the pattern is a closed form of the cell index.
//
// Assembly is a gather over cells, with no atomics: one workgroup per cell K
// writes every entry of K's nn rows.
//  - The volume block is the Poisson element matrix with coefficient 1 (the
//    integration kernels of fe_integrate*.hip).
//  - Each of the 2d facets of K adds its two facet matrices with K as the row
//    side: A^F_KK into the diagonal block and A^F_KL into the block of the
//    neighbour L.  The neighbour writes the other two, A^F_LL and A^F_LK, from
//    its own side.
//  - The facet form is unchanged when the two sides and the normal are
//    swapped, so every cell uses its own outward normal.
//  - The facet's measure, normal and penalty always come from the cell below
//    the facet (the lower index along the facet's axis).  Both cells then see
//    the same numbers, and for tau = 1 the blocks A^F_KL and A^F_LK are
//    transposes of each other to the last bit.
//  - The two sides of a brick facet carry the same quadrature points in the
//    same order: the point permutation between the sides is the identity.
//
// Trace structure used by the facet kernel.  The trace of the Lagrange basis
// on a facet is nonzero only for the (k+1)^(d-1) nodes on it.  Its value at
// a facet point is a product of 1D Lagrange values, the same on both sides.
// Per facet the kernel builds three small tables in LDS:
//   A[t][b] = sum_q W_q phi_t(q) (n . grad phi_b^K)(q)   (K's normal derivatives)
//   B[t][b] = sum_q W_q phi_t(q) (n . grad phi_b^L)(q)   (the neighbour's)
//   M[t][u] = sum_q W_q phi_t(q) phi_u(q)                 (facet mass)
// Here t and u run over facet nodes, b over the cell's nodes, n is K's
// outward unit normal and W_q = Gauss weight x facet measure.  Every facet
// entry is a signed combination of at most three table values.
#include <algorithm>
#include <cmath>

#include "fe_geom.h"
#include "fe_internal.h"

namespace fe {

struct DgArgs {
    int32_t dim, k;
    int32_t n[3];
    int64_t st[3];  // cell id strides 1, n0, n0 n1
    int64_t ncells, n_rows, nnz;
    double gamma, tau;
    // 1D tables: Gauss points and weights on [0,1]; Lagrange values and
    // derivatives at the Gauss points [i (k+1) + q] and at the ends [2 i + e]
    double gx[kMaxQ1], gw[kMaxQ1];
    double L[kMaxQ1 * kMaxQ1], D[kMaxQ1 * kMaxQ1];
    double Le[2 * kMaxQ1], De[2 * kMaxQ1];
};

__host__ __device__ __forceinline__ int64_t dg_prefix(const DgArgs &d, int64_t K)
{
    return dg_prefix_n(d.dim, d.n[0], d.n[1], d.n[2], K);
}

// Facet neighbours of K and their column slots.  Facet f = 2 r + side
// (side 1: x_r grows); nb[f] = -1 on the boundary.  Slots number the cells
// of K's row block in ascending id order: lower neighbours (far axis first),
// K itself, upper neighbours.
__host__ __device__ __forceinline__ void dg_cell_faces(const DgArgs &d, int64_t K, int64_t nb[6], int slot[6],
                                                       int &self, int &nc)
{
    const int64_t c[3] = {K % d.n[0], (K / d.n[0]) % d.n[1], d.dim == 3 ? K / (int64_t(d.n[0]) * d.n[1]) : 0};
    int s = 0;
    for (int r = 2; r >= 0; r--) {
        if (r >= d.dim) continue;
        const bool has = c[r] > 0;
        nb[2 * r] = has ? K - d.st[r] : -1;
        slot[2 * r] = has ? s++ : -1;
    }
    self = s++;
    for (int r = 0; r < d.dim; r++) {
        const bool has = c[r] < d.n[r] - 1;
        nb[2 * r + 1] = has ? K + d.st[r] : -1;
        slot[2 * r + 1] = has ? s++ : -1;
    }
    nc = s;
}

// ---------------------------------------------------------------------------
// Pattern: one workgroup per cell writes the row pointers and columns of its
// nn rows (row a of K: nc nn columns, the nn DOFs of each cell of the block).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void dg_pattern_kernel(DgArgs d, int32_t nn, int64_t *__restrict__ rowptr,
                                                         int32_t *__restrict__ colind)
{
    __shared__ int64_t sCells[7];
    __shared__ int sNc;
    const int64_t K = xcd_block(blockIdx.x, gridDim.x);
    if (threadIdx.x == 0) {
        int64_t nb[6];
        int slot[6], self, nc;
        dg_cell_faces(d, K, nb, slot, self, nc);
        for (int f = 0; f < 2 * d.dim; f++)
            if (slot[f] >= 0) sCells[slot[f]] = nb[f];
        sCells[self] = K;
        sNc = nc;
    }
    __syncthreads();
    const int nc = sNc;
    const int64_t base = int64_t(nn) * nn * dg_prefix(d, K);
    const int rlen = nc * nn;
    for (int a = threadIdx.x; a < nn; a += blockDim.x) rowptr[K * nn + a] = base + int64_t(a) * rlen;
    if (K == d.ncells - 1 && threadIdx.x == 0) rowptr[d.n_rows] = d.nnz;
    for (int e = threadIdx.x; e < nn * rlen; e += blockDim.x) {
        const int pos = e % rlen;
        colind[base + e] = int32_t(sCells[pos / nn] * nn + pos % nn);
    }
}

// ---------------------------------------------------------------------------
// Facet kernel
// ---------------------------------------------------------------------------
template <int DIM, int KO>
struct DgShape {
    static constexpr int K1 = KO + 1;
    static constexpr int NN = DIM == 3 ? K1 * K1 * K1 : K1 * K1;  // nodes per cell
    static constexpr int NF = DIM == 3 ? K1 * K1 : K1;           // nodes per facet
    static constexpr int NP = NF;                                // facet points (k + 1 per direction)
    static constexpr int NFACE = 2 * DIM;
    // threads: enough for one entry of the nn x nn block each, up to 256
    static constexpr int BS = NN * NN <= 64 ? 64 : (NN * NN <= 128 ? 128 : 256);
    static constexpr int JD = (NN * NN + BS - 1) / BS;  // diagonal-block entries per thread
    static constexpr bool DREG = JD <= 16;              // diagonal block held in registers
    static constexpr int NIT = 2 * NFACE * NP;          // (facet, side, point) items
    static constexpr int IT = (NIT + BS - 1) / BS;      // items per thread
};

// Index of node a on facet (r, side) (tangential indices, first axis
// fastest), or -1 if a is not on it.
template <int DIM, int KO>
__device__ __forceinline__ int face_node(int a, int r, int side)
{
    constexpr int K1 = KO + 1;
    int rem = a, t = 0, mul = 1, ar = 0;
#pragma unroll
    for (int s = 0; s < DIM; s++) {
        const int as = rem % K1;
        rem /= K1;
        if (s == r) {
            ar = as;
        } else {
            t += as * mul;
            mul *= K1;
        }
    }
    return ar == (side ? KO : 0) ? t : -1;
}

// One workgroup per cell K.  Phases:
//  0. tables, neighbours, and the vertices of K and its neighbours into LDS;
//  1. the geometry of every (facet, side, point) at once: J^-1 on each side,
//     the facet normal from the cell below the facet, weights, Dirichlet
//     data, penalties;
//  2. per facet: the normal derivatives of both sides at the facet points,
//     the facet mass, the tables A and B in place, then the facet's entries.
// The diagonal block (volume + every facet) accumulates in registers when a
// thread holds at most 16 of its entries, else in the output (re-read by the
// thread that wrote it).
template <int DIM, int KO>
__global__ __launch_bounds__((DgShape<DIM, KO>::BS)) void dg_cell_kernel(
    DgArgs d, MeshArgs m, ProblemArgs p, ElemLayout el, const double *__restrict__ E, const double *__restrict__ F,
    const int64_t *__restrict__ rowptr, double *__restrict__ values, double *__restrict__ rhs,
    double *__restrict__ dinv)
{
    using S = DgShape<DIM, KO>;
    constexpr int K1 = S::K1, NN = S::NN, NF = S::NF, NP = S::NP, NFACE = S::NFACE, BS = S::BS, JD = S::JD;
    constexpr int NV = 1 << DIM;
    // per facet: normal derivatives of K's and the neighbour's basis at the
    // facet points, overwritten in place by the tables A and B; facet mass M
    __shared__ double sX[NP * NN], sY[NP * NN], sM[NF * NF];
    __shared__ double sL[K1 * K1], sD[K1 * K1], sLe[2 * K1], sDe[2 * K1];
    __shared__ double sV[1 + NFACE][NV][3];  // vertices of K (slot 0) and of the neighbour across facet f (1 + f)
    __shared__ double sNv[NFACE][NP][3];     // det J J^-T e_r of the cell below the facet
    __shared__ double sMv[NFACE][2][NP][3];  // J^-1 n on K's side and on the neighbour's, n = K's outward normal
    __shared__ double sW[NFACE][NP], sU[NFACE][NP], sSig[NFACE];
    __shared__ int sFK[NN], sFL[NN];  // facet index of each node on K's facet and on the neighbour's
    __shared__ int64_t sNb[6];
    __shared__ int sSlot[6], sSelf, sNc, sBad;

    const int64_t K = xcd_block(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x;
    for (int t = tid; t < K1 * K1; t += BS) {
        sL[t] = d.L[t];
        sD[t] = d.D[t];
    }
    for (int t = tid; t < 2 * K1; t += BS) {
        sLe[t] = d.Le[t];
        sDe[t] = d.De[t];
    }
    if (tid == 0) {
        int64_t nb[6];
        int slot[6], self, nc;
        dg_cell_faces(d, K, nb, slot, self, nc);
        for (int f = 0; f < NFACE; f++) {
            sNb[f] = nb[f];
            sSlot[f] = slot[f];
        }
        sSelf = self;
        sNc = nc;
        sBad = 0;
    }
    __syncthreads();
    for (int t = tid; t < (1 + NFACE) * NV; t += BS) {
        const int sl = t / NV, v = t % NV;
        const int64_t cell = sl == 0 ? K : sNb[sl - 1];
        if (cell < 0) continue;
        const int64_t e0 = cell % m.n0, e1 = (cell / m.n0) % m.n1, e2 = cell / (int64_t(m.n0) * m.n1);
        const int64_t vid = (e0 + (v & 1)) +
                            int64_t(m.n0 + 1) * ((e1 + ((v >> 1) & 1)) + int64_t(m.n1 + 1) * (DIM == 3 ? e2 + ((v >> 2) & 1) : 0));
        sV[sl][v][0] = m.x[vid];
        sV[sl][v][1] = m.y[vid];
        sV[sl][v][2] = DIM == 3 ? m.z[vid] : 0.0;
    }
    const int self = sSelf, nc = sNc;
    const int64_t row0 = rowptr[K * NN];
    const int64_t rlen = int64_t(nc) * NN;
    __syncthreads();

    // 1a. J^-1 at every facet point on both sides; the facet normal from the
    // cell below the facet (K on its upper facets and on the boundary)
    double Ji[S::IT][9];
#pragma unroll
    for (int it = 0; it < S::IT; it++) {
        const int i = tid + it * BS;
        if (i >= S::NIT) continue;
        const int f = i / (2 * NP), gs = (i / NP) & 1, q = i % NP;
        const int r = f >> 1, side = f & 1;
        const bool interior = sNb[f] >= 0;
        if (gs == 1 && !interior) continue;
        const int t0 = DIM == 2 ? 1 - r : (r == 0 ? 1 : 0), t1 = DIM == 2 ? -1 : (r == 2 ? 1 : 2);
        const int q0 = q % K1, q1 = q / K1;
        const double er = (gs == 0) == (side == 1) ? 1.0 : 0.0;  // reference coordinate along r
        double xi[3];
#pragma unroll
        for (int sx = 0; sx < 3; sx++) xi[sx] = sx == r ? er : (sx == t0 ? d.gx[q0] : (sx == t1 ? d.gx[q1] : 0.0));
        double X[NV][3], J[9], xq[3];
#pragma unroll
        for (int v = 0; v < NV; v++)
#pragma unroll
            for (int c = 0; c < 3; c++) X[v][c] = sV[gs == 0 ? 0 : 1 + f][v][c];
        const double det = geometry<DIM>(X, xi, J, Ji[it], xq);
        if (!(det > 0.0)) atomicOr(&sBad, 1);
        const bool owner = gs == 0 ? (side == 1 || !interior) : side == 0;
        if (owner) {
#pragma unroll
            for (int rr = 0; rr < DIM; rr++)
                if (rr == r) {
#pragma unroll
                    for (int c = 0; c < DIM; c++) sNv[f][q][c] = det * Ji[it][rr * DIM + c];
                }
        }
        if (gs == 0) {
            double u = 0.0;
            if (!interior && p.dirichlet_kind == FE_DIRICHLET_AFFINE) {
                u = p.aff[0];
#pragma unroll
                for (int c = 0; c < DIM; c++) u += p.aff[1 + c] * xq[c];
            }
            sU[f][q] = u;
        }
    }
    __syncthreads();
    // 1b. K's outward unit normal n, J^-1 n on each side, weights
#pragma unroll
    for (int it = 0; it < S::IT; it++) {
        const int i = tid + it * BS;
        if (i >= S::NIT) continue;
        const int f = i / (2 * NP), gs = (i / NP) & 1, q = i % NP;
        if (gs == 1 && sNb[f] < 0) continue;
        double nv[3] = {0.0, 0.0, 0.0}, nn2 = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; c++) {
            nv[c] = sNv[f][q][c];
            nn2 += nv[c] * nv[c];
        }
        const double dS = sqrt(nn2);
        const double sgn = (f & 1) ? 1.0 : -1.0;
        double n[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < DIM; c++) n[c] = sgn * (nv[c] / dS);
#pragma unroll
        for (int sx = 0; sx < 3; sx++) {
            double mv = 0.0;
            if (sx < DIM) {
#pragma unroll
                for (int c = 0; c < DIM; c++) mv += Ji[it][sx * DIM + c] * n[c];
            }
            sMv[f][gs][q][sx] = mv;
        }
        if (gs == 0) {
            const int q0 = q % K1, q1 = q / K1;
            sW[f][q] = (d.gw[q0] * (DIM == 3 ? d.gw[q1] : 1.0)) * dS;
        }
    }
    __syncthreads();
    if (tid < NFACE) {
        double area = 0.0;
        for (int q = 0; q < NP; q++) area += sW[tid][q];
        sSig[tid] = d.gamma / (DIM == 3 ? sqrt(area) : area);
    }

    // the diagonal block starts from the element matrix of K
    double dacc[S::DREG ? JD : 1];
#pragma unroll
    for (int j = 0; j < (S::DREG ? JD : 1); j++) dacc[j] = 0.0;
    if constexpr (S::DREG) {
#pragma unroll
        for (int j = 0; j < JD; j++) {
            const int e = tid + j * BS;
            if (e < NN * NN) dacc[j] = E[elem_index(K, e / NN, e % NN, NN, el.cb, el.packed, el.ne)];
        }
    } else {
        for (int e = tid; e < NN * NN; e += BS) {
            const int a = e / NN, b = e % NN;
            values[row0 + a * rlen + self * NN + b] = E[elem_index(K, a, b, NN, el.cb, el.packed, el.ne)];
        }
    }
    double racc = tid < NN ? F[K * NN + tid] : 0.0;

#pragma unroll 1
    for (int f = 0; f < NFACE; f++) {
        const int r = f >> 1, side = f & 1;
        const bool interior = sNb[f] >= 0;
        const int t0 = DIM == 2 ? 1 - r : (r == 0 ? 1 : 0);
        if (f > 0) __syncthreads();  // the previous facet's tables are no longer read
        for (int a = tid; a < NN; a += BS) {
            sFK[a] = face_node<DIM, KO>(a, r, side);
            sFL[a] = face_node<DIM, KO>(a, r, 1 - side);
        }
        // normal derivatives of both sides at the facet points, facet mass
        const int nside = interior ? 2 : 1;
        for (int e = tid; e < nside * NP * NN; e += BS) {
            const int sd = e / (NP * NN), e2 = e - sd * (NP * NN);
            const int q = e2 / NN, b = e2 % NN;
            const int es = sd == 0 ? side : 1 - side;  // reference coordinate along r on this side
            const int qi[2] = {q % K1, q / K1};
            const int bi[3] = {b % K1, (b / K1) % K1, DIM == 3 ? b / (K1 * K1) : 0};
            double v[3], g[3];
#pragma unroll
            for (int sx = 0; sx < DIM; sx++) {
                if (sx == r) {
                    v[sx] = sLe[2 * bi[sx] + es];
                    g[sx] = sDe[2 * bi[sx] + es];
                } else {
                    const int qs = sx == t0 ? qi[0] : qi[1];
                    v[sx] = sL[bi[sx] * K1 + qs];
                    g[sx] = sD[bi[sx] * K1 + qs];
                }
            }
            const double *mv = sMv[f][sd][q];
            double out = 0.0;
#pragma unroll
            for (int sx = 0; sx < DIM; sx++) {
                double gr = g[sx];
#pragma unroll
                for (int t = 0; t < DIM; t++)
                    if (t != sx) gr *= v[t];
                out += mv[sx] * gr;
            }
            (sd == 0 ? sX : sY)[e2] = out;
        }
        for (int e = tid; e < NF * NF; e += BS) {
            const int t = e / NF, u = e % NF;
            double sm = 0.0;
#pragma unroll
            for (int q = 0; q < NP; q++) {
                const double pt = DIM == 3 ? sL[(t % K1) * K1 + q % K1] * sL[(t / K1) * K1 + q / K1] : sL[t * K1 + q];
                const double pu = DIM == 3 ? sL[(u % K1) * K1 + q % K1] * sL[(u / K1) * K1 + q / K1] : sL[u * K1 + q];
                sm += sW[f][q] * (pt * pu);  // symmetric in (t, u) to the last bit
            }
            sM[e] = sm;
        }
        __syncthreads();
        const double sigma = sSig[f];
        // A (from sX) and B (from sY) in place, one thread per column b:
        // T[t][b] = sum_q W_q phi_t(q) DN[q][b], t over the facet nodes
        if (tid < nside * NN) {
            const int sd = tid / NN, b = tid - sd * NN;
            double *T = sd == 0 ? sX : sY;
            double col[NP];
#pragma unroll
            for (int q = 0; q < NP; q++) col[q] = T[q * NN + b];
            if (sd == 0 && !interior) {
                // weak Dirichlet data of row b: sum_q W u_D (-tau n.grad phi_b + sigma phi_b)
                const int bf = sFK[b];
                double sr = 0.0;
#pragma unroll
                for (int q = 0; q < NP; q++) {
                    double v = -d.tau * col[q];
                    if (bf >= 0) {
                        const double phi = DIM == 3 ? sL[(bf % K1) * K1 + q % K1] * sL[(bf / K1) * K1 + q / K1]
                                                    : sL[bf * K1 + q];
                        v += sigma * phi;
                    }
                    sr += sW[f][q] * sU[f][q] * v;
                }
                racc += sr;  // thread b holds the rhs of row b
            }
#pragma unroll 1
            for (int t = 0; t < NF; t++) {
                const int ta = t % K1, tb = t / K1;
                double sa = 0.0;
#pragma unroll
                for (int q = 0; q < NP; q++) {
                    const double phi = DIM == 3 ? sL[ta * K1 + q % K1] * sL[tb * K1 + q / K1] : sL[ta * K1 + q];
                    sa += sW[f][q] * phi * col[q];
                }
                T[t * NN + b] = sa;
            }
        }
        __syncthreads();
        const double *sA = sX, *sB = sY;
        const double cc = interior ? 0.5 : 1.0;
        // A^F_KK: the cross of K's facet rows and columns in the diagonal block
        auto cross = [&](int e) -> double {
            const int a = e / NN, b = e % NN;
            const int af = sFK[a], bf = sFK[b];
            double v = 0.0;
            if (af >= 0) v -= cc * sA[af * NN + b];
            if (bf >= 0) v -= cc * d.tau * sA[bf * NN + a];
            if (af >= 0 && bf >= 0) v += sigma * sM[af * NF + bf];
            return v;
        };
        if constexpr (S::DREG) {
#pragma unroll
            for (int j = 0; j < JD; j++) {
                const int e = tid + j * BS;
                if (e < NN * NN) dacc[j] += cross(e);
            }
        } else {
            for (int e = tid; e < NN * NN; e += BS) {
                const int a = e / NN, b = e % NN;
                if (sFK[a] >= 0 || sFK[b] >= 0) values[row0 + a * rlen + self * NN + b] += cross(e);
            }
        }
        // A^F_KL: the block of the neighbour
        if (interior) {
            const int64_t off = row0 + int64_t(sSlot[f]) * NN;
            for (int e = tid; e < NN * NN; e += BS) {
                const int a = e / NN, b = e % NN;
                const int af = sFK[a], bl = sFL[b];
                double v = 0.0;
                if (af >= 0) v -= 0.5 * sB[af * NN + b];
                if (bl >= 0) v += 0.5 * d.tau * sA[bl * NN + a];
                if (af >= 0 && bl >= 0) v -= sigma * sM[af * NF + bl];
                values[off + a * rlen + b] = v;
            }
        }
    }
    if (tid < NN) rhs[K * NN + tid] = racc;
    // the diagonal block, and 1 / its diagonal from the thread holding it
    if constexpr (S::DREG) {
#pragma unroll
        for (int j = 0; j < JD; j++) {
            const int e = tid + j * BS;
            if (e >= NN * NN) continue;
            const int a = e / NN, b = e % NN;
            values[row0 + a * rlen + self * NN + b] = dacc[j];
            if (a == b) dinv[K * NN + a] = 1.0 / dacc[j];
        }
    } else {
        for (int e = tid; e < NN * NN; e += BS) {
            const int a = e / NN, b = e % NN;
            if (a == b) dinv[K * NN + a] = 1.0 / values[row0 + a * rlen + self * NN + b];
        }
    }
    __syncthreads();
    if (tid == 0 && sBad) atomicOr(m.status, 1);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static DgArgs make_dg(int dim, const int32_t *n, int k, double gamma, double tau)
{
    DgArgs d{};
    d.dim = dim;
    d.k = k;
    d.n[0] = n[0];
    d.n[1] = n[1];
    d.n[2] = dim == 3 ? n[2] : 1;
    d.st[0] = 1;
    d.st[1] = d.n[0];
    d.st[2] = int64_t(d.n[0]) * d.n[1];
    d.ncells = d.st[2] * d.n[2];
    int nn = 1;
    for (int r = 0; r < dim; r++) nn *= k + 1;
    d.n_rows = d.ncells * nn;
    d.nnz = int64_t(nn) * nn * dg_prefix(d, d.ncells);
    d.gamma = gamma;
    d.tau = tau;
    RefTables rt;
    ref_tables(k, rt);
    for (int i = 0; i <= k; i++) {
        d.gx[i] = rt.gx[i];
        d.gw[i] = rt.gw[i];
        lagrange_1d(k, i, 0.0, d.Le[2 * i], d.De[2 * i]);
        lagrange_1d(k, i, 1.0, d.Le[2 * i + 1], d.De[2 * i + 1]);
    }
    for (int t = 0; t < (k + 1) * (k + 1); t++) {
        d.L[t] = rt.L[t];
        d.D[t] = rt.D[t];
    }
    return d;
}

void dg_sizes(int dim, const int32_t *n, int k, int64_t &n_rows, int64_t &nnz)
{
    const DgArgs d = make_dg(dim, n, k, 1.0, 1.0);
    n_rows = d.n_rows;
    nnz = d.nnz;
}

SpaceArgs dg_space(int dim, const int32_t *n, int k)
{
    const DgArgs d = make_dg(dim, n, k, 1.0, 1.0);
    SpaceArgs sa{};
    sa.dim = dim;
    sa.k = k;
    sa.ncomp = 1;
    sa.nn = int32_t(d.n_rows / (d.ncells > 0 ? d.ncells : 1));
    sa.nloc = sa.nn;
    for (int r = 0; r < 3; r++) sa.ax[r].n = d.n[r];
    sa.ncells = d.ncells;
    sa.n_rows = d.n_rows;
    sa.nnz = d.nnz;
    return sa;
}

fe_status launch_dg_pattern(int dim, const int32_t *n, int k, int64_t *rowptr, int32_t *colind, hipStream_t s)
{
    const DgArgs d = make_dg(dim, n, k, 1.0, 1.0);
    if (d.ncells == 0) return FE_OK;
    const int32_t nn = int32_t(d.n_rows / d.ncells);
    hipLaunchKernelGGL(dg_pattern_kernel, dim3(d.ncells), dim3(256), 0, s, d, nn, rowptr, colind);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

fe_status launch_dg_facets(int dim, const int32_t *n, int k, double gamma, double tau, const MeshArgs &ma,
                           const ProblemArgs &pa, const ElemLayout &el, const void *ws, const int64_t *rowptr,
                           double *values, double *rhs, double *dinv, hipStream_t s)
{
    const DgArgs d = make_dg(dim, n, k, gamma, tau);
    if (d.ncells == 0) return FE_OK;
    const double *E = static_cast<const double *>(ws);
    const double *F = reinterpret_cast<const double *>(static_cast<const char *>(ws) + el.f_offset);
#define FE_DGK(D, KO)                                                                                  \
    hipLaunchKernelGGL((dg_cell_kernel<D, KO>), dim3(d.ncells), dim3((DgShape<D, KO>::BS)), 0, s, d, ma, pa, el, E, \
                       F, rowptr, values, rhs, dinv)
    if (dim == 3) {
        switch (k) {
            case 1: FE_DGK(3, 1); break;
            case 2: FE_DGK(3, 2); break;
            case 3: FE_DGK(3, 3); break;
            default: FE_DGK(3, 4); break;
        }
    } else {
        switch (k) {
            case 1: FE_DGK(2, 1); break;
            case 2: FE_DGK(2, 2); break;
            case 3: FE_DGK(2, 3); break;
            default: FE_DGK(2, 4); break;
        }
    }
#undef FE_DGK
    FE_HIP(hipGetLastError());
    return FE_OK;
}

}  // namespace fe
