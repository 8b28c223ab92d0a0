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

// Cells K' < K whose index along an axis of stride st and extent n equals v.
__host__ __device__ __forceinline__ int64_t dg_count_at(int64_t K, int64_t st, int64_t n, int64_t v)
{
    const int64_t P = st * n, q = K / P, rem = K % P;
    int64_t t = rem - v * st;
    t = t < 0 ? 0 : (t > st ? st : t);
    return q * st + t;
}

// Sum over cells K' < K of the cells in the row blocks of K' (K' and its
// facet neighbours): (2d + 1) K minus the missing neighbours on the boundary.
__host__ __device__ __forceinline__ int64_t dg_prefix(const DgArgs &d, int64_t K)
{
    int64_t s = (2 * d.dim + 1) * K;
    for (int r = 0; r < d.dim; r++)
        s -= dg_count_at(K, d.st[r], d.n[r], 0) + dg_count_at(K, d.st[r], d.n[r], d.n[r] - 1);
    return s;
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

template <int DIM, int KO>
__global__ __launch_bounds__(256) void dg_cell_kernel(DgArgs d, MeshArgs m, ProblemArgs p, ElemLayout el,
                                                      const double *__restrict__ E, const double *__restrict__ F,
                                                      const int64_t *__restrict__ rowptr, double *__restrict__ values,
                                                      double *__restrict__ rhs, double *__restrict__ dinv)
{
    using S = DgShape<DIM, KO>;
    constexpr int K1 = S::K1, NN = S::NN, NF = S::NF, NP = S::NP;
    // per facet: normal derivatives of K's and the neighbour's basis at the
    // facet points, overwritten in place by the tables A and B; facet mass M
    __shared__ double sX[NP * NN], sY[NP * NN], sM[NF * NF];
    __shared__ double sL[K1 * K1], sD[K1 * K1], sLe[2 * K1], sDe[2 * K1], sGw[K1];
    __shared__ double sW[NP], sU[NP], sMK[NP][3], sML[NP][3], sNv[NP][3];
    __shared__ double sSigma;
    __shared__ int sFK[NN], sFL[NN];  // facet index of each node on K's facet and on the neighbour's
    __shared__ int sBad;

    const int64_t K = xcd_block(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int t = tid; t < K1 * K1; t += nt) {
        sL[t] = d.L[t];
        sD[t] = d.D[t];
    }
    for (int t = tid; t < 2 * K1; t += nt) {
        sLe[t] = d.Le[t];
        sDe[t] = d.De[t];
    }
    if (tid < K1) sGw[tid] = d.gw[tid];
    if (tid == 0) sBad = 0;

    __shared__ int64_t sNb[6];
    __shared__ int sSlot[6], sSelf, sNc;
    if (tid == 0) {
        int64_t nb[6];
        int slot[6], self, nc;
        dg_cell_faces(d, K, nb, slot, self, nc);
        for (int f = 0; f < 2 * DIM; f++) {
            sNb[f] = nb[f];
            sSlot[f] = slot[f];
        }
        sSelf = self;
        sNc = nc;
    }
    __syncthreads();
    const int self = sSelf, nc = sNc;
    const int64_t row0 = rowptr[K * NN];
    const int64_t rlen = int64_t(nc) * NN;

    // volume block: the element matrix of K
    for (int e = tid; e < NN * NN; e += nt) {
        const int a = e / NN, b = e % NN;
        values[row0 + a * rlen + self * NN + b] = E[elem_index(K, a, b, NN, el.cb, el.packed, el.ne)];
    }
    double racc = tid < NN ? F[K * NN + tid] : 0.0;

#pragma unroll 1
    for (int f = 0; f < 2 * DIM; f++) {
        const int r = f >> 1, side = f & 1;
        const int64_t Lc = sNb[f];
        const bool interior = Lc >= 0;
        const int t0 = DIM == 2 ? 1 - r : (r == 0 ? 1 : 0), t1 = DIM == 2 ? -1 : (r == 2 ? 1 : 2);
        __syncthreads();  // the previous facet's tables are no longer read
        // facet points, one thread per (side, point): side 0 is K, side 1 the
        // neighbour.  Weights, K's outward unit normal n, J^-1 n on each side.
        for (int a = tid; a < NN; a += nt) {
            sFK[a] = face_node<DIM, KO>(a, r, side);
            sFL[a] = face_node<DIM, KO>(a, r, 1 - side);
        }
        const int gs = tid / NP, gq = tid % NP;
        const bool gact = tid < (interior ? 2 : 1) * NP;
        double Ji[9], xq[3];
        if (gact) {
            const int q0 = gq % K1, q1 = gq / K1;
            const double er = (gs == 0) == (side == 1) ? 1.0 : 0.0;  // reference coordinate along r
            double xi[3];
#pragma unroll
            for (int sx = 0; sx < 3; sx++)
                xi[sx] = sx == r ? er : (sx == t0 ? d.gx[q0] : (sx == t1 ? d.gx[q1] : 0.0));
            double X[1 << DIM][3], J[9];
            load_vertices<DIM>(m, gs == 0 ? K : Lc, X);
            const double det = geometry<DIM>(X, xi, J, Ji, xq);
            if (!(det > 0.0)) atomicOr(&sBad, 1);
            // the facet's normal det J J^-T e_r comes from the cell below it:
            // K on its upper facets and on the boundary, else the neighbour
            const bool owner = gs == 0 ? (side == 1 || !interior) : side == 0;
            if (owner) {
#pragma unroll
                for (int rr = 0; rr < DIM; rr++)
                    if (rr == r) {
#pragma unroll
                        for (int i = 0; i < DIM; i++) sNv[gq][i] = det * Ji[rr * DIM + i];
                    }
            }
        }
        __syncthreads();
        if (gact) {
            double nv[3] = {0.0, 0.0, 0.0}, nn2 = 0.0;
#pragma unroll
            for (int i = 0; i < DIM; i++) {
                nv[i] = sNv[gq][i];
                nn2 += nv[i] * nv[i];
            }
            const double dS = sqrt(nn2);
            const double sgn = side ? 1.0 : -1.0;
            double n[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < DIM; i++) n[i] = sgn * (nv[i] / dS);
            // n . grad phi = (J^-1 n) . grad_ref phi
            double(*dst)[3] = gs == 0 ? sMK : sML;
#pragma unroll
            for (int sx = 0; sx < 3; sx++) {
                double mv = 0.0;
                if (sx < DIM) {
#pragma unroll
                    for (int i = 0; i < DIM; i++) mv += Ji[sx * DIM + i] * n[i];
                }
                dst[gq][sx] = mv;
            }
            if (gs == 0) {
                const int q0 = gq % K1, q1 = gq / K1;
                sW[gq] = (d.gw[q0] * (DIM == 3 ? d.gw[q1] : 1.0)) * dS;
                double u = 0.0;
                if (!interior && p.dirichlet_kind == FE_DIRICHLET_AFFINE) {
                    u = p.aff[0];
#pragma unroll
                    for (int i = 0; i < DIM; i++) u += p.aff[1 + i] * xq[i];
                }
                sU[gq] = u;
            }
        }
        __syncthreads();
        // normal derivatives of both sides at the facet points (sX: K, sY:
        // the neighbour), the facet mass and the penalty
        if (tid == 0) {
            double area = 0.0;
            for (int q = 0; q < NP; q++) area += sW[q];
            sSigma = d.gamma / (DIM == 3 ? sqrt(area) : area);
        }
        const int nside = interior ? 2 : 1;
        for (int e = tid; e < nside * NP * NN; e += nt) {
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
            const double *mv = sd == 0 ? sMK[q] : sML[q];
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
        for (int e = tid; e < NF * NF; e += nt) {
            const int t = e / NF, u = e % NF;
            double sm = 0.0;
#pragma unroll
            for (int q = 0; q < NP; q++) {
                const double pt = DIM == 3 ? sL[(t % K1) * K1 + q % K1] * sL[(t / K1) * K1 + q / K1] : sL[t * K1 + q];
                const double pu = DIM == 3 ? sL[(u % K1) * K1 + q % K1] * sL[(u / K1) * K1 + q / K1] : sL[u * K1 + q];
                sm += sW[q] * (pt * pu);  // symmetric in (t, u) to the last bit
            }
            sM[e] = sm;
        }
        __syncthreads();
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
                        v += sSigma * phi;
                    }
                    sr += sW[q] * sU[q] * v;
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
                    sa += sW[q] * phi * col[q];
                }
                T[t * NN + b] = sa;
            }
        }
        __syncthreads();
        const double *sA = sX, *sB = sY;
        const double sigma = sSigma;
        const double cc = interior ? 0.5 : 1.0;
        // A^F_KK: the cross of K's facet rows and columns in the diagonal block
        for (int e = tid; e < NN * NN; e += nt) {
            const int a = e / NN, b = e % NN;
            const int af = sFK[a], bf = sFK[b];
            if (af < 0 && bf < 0) continue;
            double v = 0.0;
            if (af >= 0) v -= cc * sA[af * NN + b];
            if (bf >= 0) v -= cc * d.tau * sA[bf * NN + a];
            if (af >= 0 && bf >= 0) v += sigma * sM[af * NF + bf];
            values[row0 + a * rlen + self * NN + b] += v;
        }
        // A^F_KL: the block of the neighbour
        if (interior) {
            const int64_t off = row0 + int64_t(sSlot[f]) * NN;
            for (int e = tid; e < NN * NN; e += nt) {
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
    // each thread reads back only the diagonal entries it wrote itself
    for (int e = tid; e < NN * NN; e += nt) {
        const int a = e / NN, b = e % NN;
        if (a == b) dinv[K * NN + a] = 1.0 / values[row0 + a * rlen + self * NN + b];
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
    const int nn = int(d.n_rows / d.ncells);
    // enough threads for one entry of the nn x nn block each, up to 256
    const int bs = nn * nn <= 64 ? 64 : (nn * nn <= 128 ? 128 : 256);
#define FE_DGK(D, KO)                                                                                        \
    hipLaunchKernelGGL((dg_cell_kernel<D, KO>), dim3(d.ncells), dim3(bs), 0, s, d, ma, pa, el, E, F, rowptr, \
                       values, rhs, dinv)
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
