// fe_stokes.hip -- Taylor-Hood Stokes on the brick (the Stokes example of
// Sect. 3.1; the mixed pair Q_{k+1}^d x Q_k built from the scalar spaces of
// Sect. 3.8): velocity with zero Dirichlet data on the whole boundary,
// pressure with every node free.
//
//  [ A  B^T ] [u]   [f]     A: mu eps(u):eps(v), the library's elasticity
//  [ B   0  ] [p] = [0],       assembly of order k+1 with lambda = 0;
//                           B: b(v, q) = -int q div v.
//
// The continuity equation is taken with the sign that makes the system
// symmetric (the solution is unchanged).  B and B^T are assembled by a
// per-cell kernel (the element blocks on the velocity order's Gauss rule)
// followed by deterministic gathers: every CSR entry sums its element
// contributions in ascending cell order through a map built once on the host
// at set-up (the stored form of the cell-to-nnz permutation).  The system is
// solved by MINRES (a Lanczos process on the preconditioned operator with
// Givens rotations) preconditioned by the diagonal of A on the velocity and
// the pressure mass diagonal over mu on the pressure.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fe_geom.h"
#include "fe_internal.h"

namespace fe {

struct StokesArgs {
    int32_t dim, kp;  // pressure order; the velocity order is kp + 1
    double gx[kMaxQ1], gw[kMaxQ1];
    double Lu[kMaxQ1 * kMaxQ1], Du[kMaxQ1 * kMaxQ1];  // velocity basis at the Gauss points [i nq1 + q]
    double Lp[kMaxQ1 * kMaxQ1];                       // pressure basis at the Gauss points [i nq1 + q]
};

// One workgroup per cell: the divergence block
//   eb[(K nnp + a) nlu + dim b + c] = -sum_q w_q |det J_q| psi_a(q) (d_c phi_b)(q)
// and the pressure mass diagonal md[K nnp + a] = sum_q w_q |det J_q| psi_a(q)^2,
// on the (kp + 2)^d Gauss points of the velocity order.
template <int DIM, int KP>
__global__ __launch_bounds__(256) void stokes_b_kernel(StokesArgs sa, MeshArgs m, double *__restrict__ eb,
                                                       double *__restrict__ md)
{
    constexpr int KU = KP + 1, NQ1 = KU + 1, P1 = KP + 1, U1 = KU + 1;
    constexpr int NQ = DIM == 3 ? NQ1 * NQ1 * NQ1 : NQ1 * NQ1;
    constexpr int NNP = DIM == 3 ? P1 * P1 * P1 : P1 * P1;
    constexpr int NNU = DIM == 3 ? U1 * U1 * U1 : U1 * U1;
    constexpr int NLU = DIM * NNU;
    __shared__ double sJi[NQ][DIM * DIM], sW[NQ];
    __shared__ double sLu[U1 * NQ1], sDu[U1 * NQ1], sLp[P1 * NQ1];
    __shared__ int sBad;
    const int64_t K = xcd_block(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x;
    for (int t = tid; t < U1 * NQ1; t += blockDim.x) {
        sLu[t] = sa.Lu[t];
        sDu[t] = sa.Du[t];
    }
    for (int t = tid; t < P1 * NQ1; t += blockDim.x) sLp[t] = sa.Lp[t];
    if (tid == 0) sBad = 0;
    for (int q = tid; q < NQ; q += blockDim.x) {
        const int q0 = q % NQ1, q1 = (q / NQ1) % NQ1, q2 = DIM == 3 ? q / (NQ1 * NQ1) : 0;
        const double xi[3] = {sa.gx[q0], sa.gx[q1], DIM == 3 ? sa.gx[q2] : 0.0};
        double X[1 << DIM][3], J[9], Ji[9], xq[3];
        load_vertices<DIM>(m, K, X);
        const double det = geometry<DIM>(X, xi, J, Ji, xq);
        if (!(det > 0.0)) atomicOr(&sBad, 1);
#pragma unroll
        for (int t = 0; t < DIM * DIM; t++) sJi[q][t] = Ji[t];
        sW[q] = sa.gw[q0] * sa.gw[q1] * (DIM == 3 ? sa.gw[q2] : 1.0) * fabs(det);
    }
    __syncthreads();
    for (int e = tid; e < NNP * NLU; e += blockDim.x) {
        const int a = e / NLU, jb = e % NLU, b = jb / DIM, c = jb % DIM;
        const int ai[3] = {a % P1, (a / P1) % P1, DIM == 3 ? a / (P1 * P1) : 0};
        const int bi[3] = {b % U1, (b / U1) % U1, DIM == 3 ? b / (U1 * U1) : 0};
        double s = 0.0;
        for (int q = 0; q < NQ; q++) {
            const int qi[3] = {q % NQ1, (q / NQ1) % NQ1, DIM == 3 ? q / (NQ1 * NQ1) : 0};
            double psi = 1.0, v[3], g[3];
#pragma unroll
            for (int r = 0; r < DIM; r++) {
                psi *= sLp[ai[r] * NQ1 + qi[r]];
                v[r] = sLu[bi[r] * NQ1 + qi[r]];
                g[r] = sDu[bi[r] * NQ1 + qi[r]];
            }
            // (d_c phi_b) = sum_s (J^-1)_{s c} (d phi_b / d xi_s)
            double dc = 0.0;
#pragma unroll
            for (int sd = 0; sd < DIM; sd++) {
                double gr = g[sd];
#pragma unroll
                for (int r = 0; r < DIM; r++)
                    if (r != sd) gr *= v[r];
                dc += sJi[q][sd * DIM + c] * gr;
            }
            s -= sW[q] * psi * dc;
        }
        eb[(K * NNP + a) * NLU + jb] = s;
    }
    for (int a = tid; a < NNP; a += blockDim.x) {
        const int ai[3] = {a % P1, (a / P1) % P1, DIM == 3 ? a / (P1 * P1) : 0};
        double s = 0.0;
        for (int q = 0; q < NQ; q++) {
            const int qi[3] = {q % NQ1, (q / NQ1) % NQ1, DIM == 3 ? q / (NQ1 * NQ1) : 0};
            double psi = 1.0;
#pragma unroll
            for (int r = 0; r < DIM; r++) psi *= sLp[ai[r] * NQ1 + qi[r]];
            s += sW[q] * psi * psi;
        }
        md[K * NNP + a] = s;
    }
    __syncthreads();
    if (tid == 0 && sBad) atomicOr(m.status, 1);
}

// out[i] = sum over t in [ptr[i], ptr[i+1]) of src[idx[t]], in list order.
__global__ __launch_bounds__(256) void gather_sum_kernel(int64_t n, const int64_t *__restrict__ ptr,
                                                         const int64_t *__restrict__ idx, const double *__restrict__ src,
                                                         double *__restrict__ out)
{
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        double s = 0.0;
        for (int64_t t = ptr[i]; t < ptr[i + 1]; t++) s += src[idx[t]];
        out[i] = s;
    }
}

// Preconditioner diagonal: 1 / A_ii on the velocity, mu / md_i on the pressure.
__global__ __launch_bounds__(256) void stokes_minv_kernel(int64_t nu, int64_t np, const double *__restrict__ dinv,
                                                          const double *__restrict__ md, double mu,
                                                          double *__restrict__ minv)
{
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < nu + np;
         i += int64_t(gridDim.x) * blockDim.x)
        minv[i] = i < nu ? dinv[i] : mu / md[i - nu];
}

// ---------------------------------------------------------------------------
// MINRES vector kernels.  Dot products: per-block partials over a fixed grid,
// then one block sums them in a fixed order (bitwise reproducible).
// ---------------------------------------------------------------------------
constexpr int kMinresGrid = 512;

__device__ __forceinline__ double block_reduce_256(double v)
{
    __shared__ double red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    return red[0];
}

__global__ __launch_bounds__(256) void minres_sum_kernel(int np, const double *__restrict__ part,
                                                         double *__restrict__ out)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
    s = block_reduce_256(s);
    if (threadIdx.x == 0) *out = s;
}

__global__ __launch_bounds__(256) void minres_scale2_kernel(int64_t n, double s, const double *__restrict__ x,
                                                            double *__restrict__ y, const double *__restrict__ z,
                                                            double *__restrict__ w)
{
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        y[i] = s * x[i];
        w[i] = s * z[i];
    }
}

__global__ __launch_bounds__(256) void minres_axpy_kernel(int64_t n, double a, const double *__restrict__ x,
                                                          double *__restrict__ y)
{
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        y[i] += a * x[i];
}

// r = b - y (b: rhs; y: K x), z = minv r, partials of r.z
// ---------------------------------------------------------------------------
// MINRES with its scalars on the device.  The Givens state of the QR of the
// Lanczos tridiagonal lives in two slots (read one, write the other, by
// iteration parity); every block of a kernel sums the partials it needs in
// the fixed order of minres_sum_kernel, so all blocks hold the same scalars
// and the host never waits inside an iteration.  ctrl[0] is the iteration
// count at which the solve stopped (-1 while running), ctrl[1] the reason
// (0 converged, 1 breakdown, 2 maxit); kernels queued after a stop return at
// once, so x is never touched again.
struct MinresScalars {
    double beta, c_old, s_old, c, sn, eta;
};

__device__ __forceinline__ double sum_partials(int np, const double *__restrict__ part)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
    s = block_reduce_256(s);
    __syncthreads();  // every thread has read the sum before the buffer is reused
    return s;
}

__global__ __launch_bounds__(256) void minres_dot_dev_kernel(int64_t n, const double *__restrict__ a,
                                                             const double *__restrict__ b, double *__restrict__ part,
                                                             const int *__restrict__ ctrl)
{
    if (ctrl[0] >= 0) return;
    double s = 0.0;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        s += a[i] * b[i];
    s = block_reduce_256(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// w -= alpha v + beta vold; z = minv w; partial sums of w.z
__global__ __launch_bounds__(256) void minres_lanczos_dev_kernel(int64_t n, int np,
                                                                 const double *__restrict__ part_dot,
                                                                 const MinresScalars *__restrict__ sc,
                                                                 const double *__restrict__ v,
                                                                 const double *__restrict__ vold,
                                                                 double *__restrict__ w, const double *__restrict__ minv,
                                                                 double *__restrict__ z, double *__restrict__ part_bn,
                                                                 const int *__restrict__ ctrl)
{
    if (ctrl[0] >= 0) return;
    const double alpha = sum_partials(np, part_dot);
    const double beta = sc->beta;
    double s = 0.0;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const double pi = w[i] - alpha * v[i] - beta * vold[i];
        const double zi = minv[i] * pi;
        w[i] = pi;
        z[i] = zi;
        s += pi * zi;
    }
    s = block_reduce_256(s);
    if (threadIdx.x == 0) part_bn[blockIdx.x] = s;
}

// Givens step and the vector updates of iteration it:
//   d_new = (zv - delta d - eps d_old) / gamma   (written over d_old)
//   x += tau d_new; v_next = w / beta_new (over v_old); zv = z / beta_new
__global__ __launch_bounds__(256) void minres_update_dev_kernel(
    int64_t n, int64_t nu, int np, const double *__restrict__ part_dot, const double *__restrict__ part_bn,
    const MinresScalars *__restrict__ sc_in, MinresScalars *__restrict__ sc_out, double stop_tol, int it, int maxit,
    int *__restrict__ ctrl, const double *__restrict__ w, const double *__restrict__ z, double *__restrict__ zv,
    const double *__restrict__ d, double *__restrict__ dold_dnew, double *__restrict__ vold_vnext,
    double *__restrict__ xu, double *__restrict__ xp)
{
    if (ctrl[0] >= 0) return;
    const double alpha = sum_partials(np, part_dot);
    const double bn2 = sum_partials(np, part_bn);
    const MinresScalars S = *sc_in;
    const double beta_new = sqrt(bn2 > 0.0 ? bn2 : 0.0);
    const double eps = S.s_old * S.beta;
    const double t = S.c_old * S.beta;
    const double delta = S.c * t + S.sn * alpha;
    const double gbar = -S.sn * t + S.c * alpha;
    const double gamma = sqrt(gbar * gbar + beta_new * beta_new);
    const bool bad = !(bn2 >= 0.0) || !isfinite(bn2) || !isfinite(alpha) || !(gamma > 0.0);
    if (bad) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ctrl[0] = it;
            ctrl[1] = 1;
        }
        return;
    }
    const double c2 = gbar / gamma, sn2 = beta_new / gamma;
    const double tau = c2 * S.eta, eta2 = -sn2 * S.eta;
    const double ginv = 1.0 / gamma, bscale = beta_new > 0.0 ? 1.0 / beta_new : 0.0;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const double di = (zv[i] - delta * d[i] - eps * dold_dnew[i]) * ginv;
        dold_dnew[i] = di;
        if (i < nu) xu[i] += tau * di;
        else xp[i - nu] += tau * di;
        vold_vnext[i] = bscale * w[i];
        zv[i] = bscale * z[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *sc_out = MinresScalars{beta_new, S.c, S.sn, c2, sn2, eta2};
        if (fabs(eta2) <= stop_tol) {
            ctrl[0] = it + 1;
            ctrl[1] = 0;
        } else if (it + 1 >= maxit) {
            ctrl[0] = it + 1;
            ctrl[1] = 2;
        }
    }
}

__global__ __launch_bounds__(256) void minres_init_kernel(int64_t n, const double *__restrict__ b,
                                                          const double *__restrict__ y, const double *__restrict__ minv,
                                                          double *__restrict__ r, double *__restrict__ z,
                                                          double *__restrict__ part)
{
    double s = 0.0;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const double ri = b[i] - y[i];
        const double zi = minv[i] * ri;
        r[i] = ri;
        z[i] = zi;
        s += ri * zi;
    }
    s = block_reduce_256(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

}  // namespace fe

using namespace fe;

struct fe_stokes_s {
    fe_mesh mesh = nullptr;
    int32_t k = 0;
    double mu = 1.0;
    fe_coeff cu{};  // the velocity block's problem: elasticity, Young mu, Poisson 0, every face clamped
    Space su, sp;   // velocity (order k + 1, dim components) and pressure (order k, scalar, no fixed node)
    int64_t nu = 0, np = 0, nnz_a = 0, nnz_b = 0, nc_b = 0;
    ElemLayout el{};
    char *ws_a = nullptr;
    int64_t *a_rowptr = nullptr;
    int32_t *a_colind = nullptr;
    double *a_values = nullptr, *rhs = nullptr, *dinv = nullptr;
    int64_t *b_rowptr = nullptr, *bt_rowptr = nullptr;
    int32_t *b_colind = nullptr, *bt_colind = nullptr;
    double *b_values = nullptr, *bt_values = nullptr;
    int64_t *gb_ptr = nullptr, *gb_idx = nullptr, *gbt_ptr = nullptr, *gbt_idx = nullptr;
    int64_t *gm_ptr = nullptr, *gm_idx = nullptr;
    double *eb = nullptr, *mdb = nullptr, *md = nullptr, *minv = nullptr;
    double *mv = nullptr;    // MINRES vectors: 8 of n = nu + np
    double *part = nullptr;  // partials (kMinresGrid) and the scalar
    double *mr = nullptr;    // device MINRES: dot and w.z partials, two scalar slots, control word
    int *ctrl_host = nullptr; // pinned copies of the control word (two)
};

namespace {

template <typename T>
fe_status dmalloc(T *&p, size_t count)
{
    FE_HIP(hipMalloc(&p, sizeof(T) * std::max<size_t>(count, 1)));
    return FE_OK;
}

void stokes_free(fe_stokes S)
{
    void *ptrs[] = {S->ws_a,   S->a_rowptr, S->a_colind, S->a_values, S->rhs,     S->dinv,    S->b_rowptr,
                    S->bt_rowptr, S->b_colind, S->bt_colind, S->b_values, S->bt_values, S->gb_ptr,  S->gb_idx,
                    S->gbt_ptr,  S->gbt_idx,  S->gm_ptr,   S->gm_idx,   S->eb,      S->mdb,     S->md,
                    S->minv,     S->mv,       S->part,     S->mr};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (S->ctrl_host) (void)hipHostFree(S->ctrl_host);
    free_space(S->su);
    free_space(S->sp);
    delete S;
}

// CSR of the pairs (row, col) over the element contributions src, each entry
// keeping its contributions in ascending src order (src grows with the cell).
struct Contribution {
    int64_t row, col, src;
};

void build_gather(std::vector<Contribution> &c, int64_t nrows, std::vector<int64_t> &rowptr,
                  std::vector<int32_t> &colind, std::vector<int64_t> &gptr, std::vector<int64_t> &gidx)
{
    std::sort(c.begin(), c.end(), [](const Contribution &x, const Contribution &y) {
        if (x.row != y.row) return x.row < y.row;
        if (x.col != y.col) return x.col < y.col;
        return x.src < y.src;
    });
    rowptr.assign(nrows + 1, 0);
    colind.clear();
    gptr.clear();
    gidx.resize(c.size());
    for (size_t t = 0; t < c.size(); t++) {
        gidx[t] = c[t].src;
        if (t == 0 || c[t].row != c[t - 1].row || c[t].col != c[t - 1].col) {
            colind.push_back(int32_t(c[t].col));
            gptr.push_back(int64_t(t));
            rowptr[c[t].row + 1]++;
        }
    }
    gptr.push_back(int64_t(c.size()));
    for (int64_t r = 0; r < nrows; r++) rowptr[r + 1] += rowptr[r];
}

template <typename T>
fe_status upload(T *&d, const std::vector<T> &h)
{
    fe_status st = dmalloc(d, h.size());
    if (st != FE_OK) return st;
    if (!h.empty()) FE_HIP(hipMemcpy(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
    return FE_OK;
}

StokesArgs stokes_args(int dim, int kp)
{
    StokesArgs a{};
    a.dim = dim;
    a.kp = kp;
    RefTables rt;
    ref_tables(kp + 1, rt);  // Gauss points of the velocity order and its basis there
    const int nq1 = kp + 2;
    for (int q = 0; q < nq1; q++) {
        a.gx[q] = rt.gx[q];
        a.gw[q] = rt.gw[q];
    }
    for (int t = 0; t < nq1 * nq1; t++) {
        a.Lu[t] = rt.L[t];
        a.Du[t] = rt.D[t];
    }
    for (int i = 0; i <= kp; i++)
        for (int q = 0; q < nq1; q++) {
            double der;
            lagrange_1d(kp, i, rt.gx[q], a.Lp[i * nq1 + q], der);
        }
    return a;
}

MeshArgs stokes_mesh_args(const fe_mesh m)
{
    MeshArgs a{};
    a.x = m->d_xyz;
    a.y = m->d_xyz + m->nverts;
    a.z = m->dim == 3 ? m->d_xyz + 2 * m->nverts : nullptr;
    a.coef = nullptr;
    a.n0 = m->n[0];
    a.n1 = m->n[1];
    a.n2 = m->dim == 3 ? m->n[2] : 1;
    a.status = m->d_status;
    return a;
}

fe_status launch_stokes_b(const fe_stokes S, hipStream_t s)
{
    const StokesArgs sa = stokes_args(S->mesh->dim, S->k);
    const MeshArgs ma = stokes_mesh_args(S->mesh);
    const int64_t nc = S->mesh->ncells;
    if (nc == 0) return FE_OK;
#define FE_SB(D, KP) \
    hipLaunchKernelGGL((stokes_b_kernel<D, KP>), dim3(nc), dim3(256), 0, s, sa, ma, S->eb, S->mdb)
    if (S->mesh->dim == 3) {
        switch (S->k) {
            case 1: FE_SB(3, 1); break;
            case 2: FE_SB(3, 2); break;
            default: FE_SB(3, 3); break;
        }
    } else {
        switch (S->k) {
            case 1: FE_SB(2, 1); break;
            case 2: FE_SB(2, 2); break;
            default: FE_SB(2, 3); break;
        }
    }
#undef FE_SB
    FE_HIP(hipGetLastError());
    return FE_OK;
}

int grid_of(int64_t n) { return int(std::max<int64_t>(1, std::min<int64_t>(kMinresGrid, (n + 255) / 256))); }

}  // namespace

extern "C" {

fe_status fe_stokes_create(fe_mesh mesh, int32_t order, double mu, const fe_coeff *force, fe_stokes *out)
{
    if (!mesh || !out) return set_error(FE_EINVAL, "null argument");
    if (order < 1 || order + 1 > kMaxOrder) return set_error(FE_EINVAL, "pressure order must be in 1..3");
    if (!(mu > 0.0) || !std::isfinite(mu)) return set_error(FE_EINVAL, "mu must be positive and finite");
    fe_stokes S = new fe_stokes_s();
    S->mesh = mesh;
    S->k = order;
    S->mu = mu;
    S->cu.problem = FE_ELASTICITY;
    S->cu.precision = FE_FP64;
    S->cu.young = mu;
    S->cu.poisson_ratio = 0.0;
    if (force) {
        if (force->source_kind < FE_SOURCE_NONE || force->source_kind > FE_SOURCE_SINPROD) {
            delete S;
            return set_error(FE_EINVAL, "unknown source kind");
        }
        S->cu.source_kind = force->source_kind;
        for (int i = 0; i < 3; i++) S->cu.source[i] = force->source[i];
    }
    S->cu.dirichlet_faces = (1u << (2 * mesh->dim)) - 1u;
    S->cu.dirichlet_kind = FE_DIRICHLET_ZERO;
    const int dim = mesh->dim;
    fe_status st = build_space(mesh, order + 1, dim, S->cu.dirichlet_faces, S->su, nullptr);
    if (st == FE_OK) st = build_space(mesh, order, 1, 0u, S->sp, nullptr);
    if (st != FE_OK) {
        stokes_free(S);
        return st;
    }
    const SpaceArgs &au = S->su.args, &ap = S->sp.args;
    S->nu = au.n_rows;
    S->np = ap.n_rows;
    S->nnz_a = au.nnz;
    if (S->nu + S->np >= (int64_t(1) << 31)) {
        stokes_free(S);
        return set_error(FE_EINVAL, "system has 2^31 or more rows");
    }
    // cell-to-DOF maps on the host, then the contributions of every element entry
    const int64_t nc = mesh->ncells;
    const int nlu = au.nloc, nnp = ap.nloc;
    std::vector<int32_t> cdu(size_t(nc) * nlu), cdp(size_t(nc) * nnp);
    if (nc > 0) {
        if (hipMemcpy(cdu.data(), S->su.d_cell_dofs, sizeof(int32_t) * cdu.size(), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(cdp.data(), S->sp.d_cell_dofs, sizeof(int32_t) * cdp.size(), hipMemcpyDeviceToHost) != hipSuccess) {
            stokes_free(S);
            return set_error(FE_EDEVICE, "copy of the cell-to-DOF maps failed");
        }
    }
    std::vector<Contribution> cb, cm;
    cb.reserve(size_t(nc) * nnp * nlu);
    cm.reserve(size_t(nc) * nnp);
    for (int64_t K = 0; K < nc; K++)
        for (int a = 0; a < nnp; a++) {
            const int64_t row = cdp[K * nnp + a];
            cm.push_back({row, 0, K * nnp + a});
            for (int jb = 0; jb < nlu; jb++) {
                const int32_t col = cdu[K * nlu + jb];
                if (col >= 0) cb.push_back({row, col, (K * nnp + a) * nlu + jb});
            }
        }
    S->nc_b = int64_t(cb.size());
    std::vector<int64_t> rp, gp, gi;
    std::vector<int32_t> ci;
    std::vector<Contribution> cbt(cb.size());
    for (size_t t = 0; t < cb.size(); t++) cbt[t] = {cb[t].col, cb[t].row, cb[t].src};
    build_gather(cb, S->np, rp, ci, gp, gi);
    S->nnz_b = int64_t(ci.size());
    st = upload(S->b_rowptr, rp);
    if (st == FE_OK) st = upload(S->b_colind, ci);
    if (st == FE_OK) st = upload(S->gb_ptr, gp);
    if (st == FE_OK) st = upload(S->gb_idx, gi);
    if (st == FE_OK) {
        build_gather(cbt, S->nu, rp, ci, gp, gi);
        st = upload(S->bt_rowptr, rp);
    }
    if (st == FE_OK) st = upload(S->bt_colind, ci);
    if (st == FE_OK) st = upload(S->gbt_ptr, gp);
    if (st == FE_OK) st = upload(S->gbt_idx, gi);
    if (st == FE_OK) {
        std::vector<int32_t> unused;
        build_gather(cm, S->np, rp, unused, gp, gi);
        st = upload(S->gm_ptr, gp);
    }
    if (st == FE_OK) st = upload(S->gm_idx, gi);
    // device storage of the system and the solver
    S->el = elem_layout(au, FE_FP64);
    const int64_t n = S->nu + S->np;
    if (st == FE_OK) st = dmalloc(S->ws_a, S->el.total);
    if (st == FE_OK) st = dmalloc(S->a_rowptr, size_t(S->nu) + 1);
    if (st == FE_OK) st = dmalloc(S->a_colind, size_t(S->nnz_a));
    if (st == FE_OK) st = dmalloc(S->a_values, size_t(S->nnz_a));
    if (st == FE_OK) st = dmalloc(S->rhs, size_t(n));
    if (st == FE_OK) st = dmalloc(S->dinv, size_t(S->nu));
    if (st == FE_OK) st = dmalloc(S->b_values, size_t(S->nnz_b));
    if (st == FE_OK) st = dmalloc(S->bt_values, size_t(S->nnz_b));
    if (st == FE_OK) st = dmalloc(S->eb, size_t(nc) * nnp * nlu);
    if (st == FE_OK) st = dmalloc(S->mdb, size_t(nc) * nnp);
    if (st == FE_OK) st = dmalloc(S->md, size_t(S->np));
    if (st == FE_OK) st = dmalloc(S->minv, size_t(n));
    if (st == FE_OK) st = dmalloc(S->mv, 8 * size_t(n));
    if (st == FE_OK) st = dmalloc(S->part, kMinresGrid + 8);
    if (st == FE_OK) st = dmalloc(S->mr, 2 * kMinresGrid + 16);
    if (st == FE_OK && hipHostMalloc(&S->ctrl_host, 8 * sizeof(int)) != hipSuccess) {
        S->ctrl_host = nullptr;
        st = set_error(FE_ENOMEM, "pinned control word");
    }
    if (st == FE_OK) st = launch_pattern(au, S->a_rowptr, S->a_colind, nullptr);
    if (st == FE_OK && hipDeviceSynchronize() != hipSuccess) st = set_error(FE_EDEVICE, "stokes set-up failed");
    if (st != FE_OK) {
        stokes_free(S);
        return st;
    }
    *out = S;
    return FE_OK;
}

fe_status fe_stokes_destroy(fe_stokes S)
{
    if (!S) return set_error(FE_EINVAL, "null handle");
    (void)hipDeviceSynchronize();
    stokes_free(S);
    return FE_OK;
}

fe_status fe_stokes_query(fe_stokes S, int64_t *n_u, int64_t *n_p, int64_t *nnz_a, int64_t *nnz_b)
{
    if (!S) return set_error(FE_EINVAL, "null handle");
    if (n_u) *n_u = S->nu;
    if (n_p) *n_p = S->np;
    if (nnz_a) *nnz_a = S->nnz_a;
    if (nnz_b) *nnz_b = S->nnz_b;
    return FE_OK;
}

fe_status fe_stokes_assemble(fe_stokes S, fe_stream stream)
{
    if (!S) return set_error(FE_EINVAL, "null handle");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const SpaceArgs &au = S->su.args;
    RefTables rt;
    ref_tables(S->k + 1, rt);
    ProblemArgs pa{};
    pa.problem = FE_ELASTICITY;
    pa.precision = FE_FP64;
    pa.lambda = 0.0;
    pa.mu = S->mu / 2.0;  // 2 mu' eps:eps = mu eps:eps
    pa.source_kind = S->cu.source_kind;
    for (int i = 0; i < 3; i++) pa.source[i] = S->cu.source[i];
    pa.dirichlet_kind = FE_DIRICHLET_ZERO;
    const MeshArgs ma = stokes_mesh_args(S->mesh);
    S->mesh->last_stream = s;
    fe_status st = launch_integrate(au, ma, pa, rt, S->el, S->ws_a, s);
    if (st == FE_OK) st = launch_scatter(au, S->el, S->ws_a, S->a_values, S->rhs, S->dinv, s);
    if (st == FE_OK) st = launch_stokes_b(S, s);
    if (st != FE_OK) return st;
    if (S->nnz_b > 0) {
        hipLaunchKernelGGL(gather_sum_kernel, dim3(grid_of(S->nnz_b)), dim3(256), 0, s, S->nnz_b, S->gb_ptr, S->gb_idx,
                           S->eb, S->b_values);
        hipLaunchKernelGGL(gather_sum_kernel, dim3(grid_of(S->nnz_b)), dim3(256), 0, s, S->nnz_b, S->gbt_ptr,
                           S->gbt_idx, S->eb, S->bt_values);
    }
    if (S->np > 0)
        hipLaunchKernelGGL(gather_sum_kernel, dim3(grid_of(S->np)), dim3(256), 0, s, S->np, S->gm_ptr, S->gm_idx,
                           S->mdb, S->md);
    const int64_t n = S->nu + S->np;
    if (n > 0) {
        hipLaunchKernelGGL(stokes_minv_kernel, dim3(grid_of(n)), dim3(256), 0, s, S->nu, S->np, S->dinv, S->md, S->mu,
                           S->minv);
        // the pressure rows of the right-hand side are zero
        if (S->np > 0) FE_HIP(hipMemsetAsync(S->rhs + S->nu, 0, sizeof(double) * S->np, s));
    }
    FE_HIP(hipGetLastError());
    return FE_OK;
}

fe_status fe_stokes_system(fe_stokes S, fe_csr *A, fe_csr *B, fe_csr *Bt, const double **md, const double **rhs)
{
    if (!S) return set_error(FE_EINVAL, "null handle");
    if (A) *A = fe_csr{S->nu, S->nnz_a, S->a_rowptr, S->a_colind, S->a_values, S->rhs, S->dinv};
    if (B) *B = fe_csr{S->np, S->nnz_b, S->b_rowptr, S->b_colind, S->b_values, nullptr, nullptr};
    if (Bt) *Bt = fe_csr{S->nu, S->nnz_b, S->bt_rowptr, S->bt_colind, S->bt_values, nullptr, nullptr};
    if (md) *md = S->md;
    if (rhs) *rhs = S->rhs;
    return FE_OK;
}

// y = K x for x = (xu | xp) and y = (yu | yp); t: a scratch of nu
static fe_status stokes_apply(fe_stokes S, const double *xu, const double *xp, double *yu, double *yp, double *t,
                              hipStream_t s)
{
    fe_status st = launch_spmv_struct(S->su.args, S->a_values, xu, yu, s);
    if (st == FE_OK && S->nnz_b > 0) st = launch_spmv(S->nu, S->bt_rowptr, S->bt_colind, S->bt_values, xp, t, S->nnz_b, s);
    if (st == FE_OK && S->nnz_b > 0) st = launch_spmv(S->np, S->b_rowptr, S->b_colind, S->b_values, xu, yp, S->nnz_b, s);
    if (st != FE_OK) return st;
    if (S->nnz_b > 0)
        hipLaunchKernelGGL(minres_axpy_kernel, dim3(grid_of(S->nu)), dim3(256), 0, s, S->nu, 1.0, t, yu);
    else if (S->np > 0)
        FE_HIP(hipMemsetAsync(yp, 0, sizeof(double) * S->np, s));
    FE_HIP(hipGetLastError());
    return FE_OK;
}

static fe_status read_scalar(const fe_stokes S, int np, hipStream_t s, double &v)
{
    hipLaunchKernelGGL(minres_sum_kernel, dim3(1), dim3(256), 0, s, np, S->part, S->part + kMinresGrid);
    FE_HIP(hipGetLastError());
    FE_HIP(hipMemcpyAsync(&v, S->part + kMinresGrid, sizeof(double), hipMemcpyDeviceToHost, s));
    FE_HIP(hipStreamSynchronize(s));
    return FE_OK;
}

fe_status fe_stokes_solve(fe_stokes S, double rtol, int32_t maxit, double *u, double *p, fe_solve_info *info,
                          fe_stream stream)
{
    if (!S || !u || !p || !info) return set_error(FE_EINVAL, "null argument");
    if (!(rtol >= 0.0) || maxit < 0) return set_error(FE_EINVAL, "bad rtol/maxit");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::memset(info, 0, sizeof(*info));
    const int64_t n = S->nu + S->np, nu = S->nu;
    if (n == 0) return FE_OK;
    double *v = S->mv, *vold = v + n, *zv = vold + n, *w = zv + n, *z = w + n, *d = z + n, *dold = d + n,
           *dnew = dold + n;
    const int g = grid_of(n);
    // r0 = b - K x0 (v), z0 = M^-1 r0 (z), beta1 = sqrt(r0 . z0)
    fe_status st = stokes_apply(S, u, p, w, w + nu, dnew, s);
    if (st != FE_OK) return st;
    hipLaunchKernelGGL(minres_init_kernel, dim3(g), dim3(256), 0, s, n, S->rhs, w, S->minv, v, z, S->part);
    double b2 = 0.0;
    if ((st = read_scalar(S, g, s, b2)) != FE_OK) return st;
    // ||b||_{M^-1} for the relative stop test: b - 0 into scratch vectors
    FE_HIP(hipMemsetAsync(dold, 0, sizeof(double) * n, s));
    hipLaunchKernelGGL(minres_init_kernel, dim3(g), dim3(256), 0, s, n, S->rhs, dold, S->minv, w, dnew, S->part);
    double bb = 0.0;
    if ((st = read_scalar(S, g, s, bb)) != FE_OK) return st;
    if (!(b2 >= 0.0) || !std::isfinite(b2) || !(bb >= 0.0)) {
        info->status = FE_EBREAKDOWN;
        return set_error(FE_EBREAKDOWN, "minres: preconditioner not positive");
    }
    const double beta = std::sqrt(b2);
    const double bnorm = std::sqrt(std::max(bb, 0.0));
    FE_HIP(hipMemsetAsync(vold, 0, sizeof(double) * n, s));
    FE_HIP(hipMemsetAsync(d, 0, sizeof(double) * n, s));
    FE_HIP(hipMemsetAsync(dold, 0, sizeof(double) * n, s));
    if (beta > 0.0)
        hipLaunchKernelGGL(minres_scale2_kernel, dim3(g), dim3(256), 0, s, n, 1.0 / beta, v, v, z, zv);
    // device state: dot partials, w.z partials, two scalar slots, the control word
    double *part_dot = S->mr, *part_bn = S->mr + kMinresGrid;
    MinresScalars *slot = reinterpret_cast<MinresScalars *>(S->mr + 2 * kMinresGrid);
    int *ctrl = reinterpret_cast<int *>(S->mr + 2 * kMinresGrid + 12);
    const MinresScalars s0{beta, 1.0, 0.0, 1.0, 0.0, beta};  // |eta| = ||r||_{M^-1}
    const int ctrl0[2] = {-1, 0};
    FE_HIP(hipMemcpyAsync(slot, &s0, sizeof(s0), hipMemcpyHostToDevice, s));
    FE_HIP(hipMemcpyAsync(ctrl, ctrl0, sizeof(ctrl0), hipMemcpyHostToDevice, s));
    const double stop_tol = rtol * bnorm;
    int iters = 0, reason = 0;
    if (beta <= stop_tol || !(beta > 0.0)) {
        reason = 0;  // converged at x0
    } else if (maxit == 0) {
        reason = 2;
    } else {
        // iterations are queued in chunks; the host reads the control word of
        // chunk c (copied asynchronously) only after chunk c+1 is queued, so
        // the device never waits for it
        constexpr int kChunk = 8;
        hipEvent_t ev[2];
        FE_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
        FE_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
        int chunk = 0;
        bool stopped = false;
        for (int it = 0; it < maxit && !stopped; chunk++) {
            const int end = std::min(maxit, it + kChunk);
            for (; it < end; it++) {
                // Lanczos: w = K zv - alpha v - beta vold; z = M^-1 w; beta_new = sqrt(w . z)
                if ((st = stokes_apply(S, zv, zv + nu, w, w + nu, dnew, s)) != FE_OK) break;
                hipLaunchKernelGGL(minres_dot_dev_kernel, dim3(g), dim3(256), 0, s, n, zv, w, part_dot, ctrl);
                hipLaunchKernelGGL(minres_lanczos_dev_kernel, dim3(g), dim3(256), 0, s, n, g, part_dot, slot + (it & 1),
                                   v, vold, w, S->minv, z, part_bn, ctrl);
                hipLaunchKernelGGL(minres_update_dev_kernel, dim3(g), dim3(256), 0, s, n, nu, g, part_dot, part_bn,
                                   slot + (it & 1), slot + ((it + 1) & 1), stop_tol, it, maxit, ctrl, w, z, zv, d,
                                   dold, vold, u, p);
                // the new direction was written over dold, the new v over vold
                std::swap(d, dold);
                std::swap(v, vold);
            }
            if (st != FE_OK) break;
            FE_HIP(hipGetLastError());
            int *hc = S->ctrl_host + 2 * (chunk & 1);
            FE_HIP(hipMemcpyAsync(hc, ctrl, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
            FE_HIP(hipEventRecord(ev[chunk & 1], s));
            if (chunk > 0) {
                FE_HIP(hipEventSynchronize(ev[(chunk - 1) & 1]));
                stopped = S->ctrl_host[2 * ((chunk - 1) & 1)] >= 0;
            }
        }
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
        if (st != FE_OK) return st;
        int hc[2];
        FE_HIP(hipMemcpyAsync(hc, ctrl, sizeof(hc), hipMemcpyDeviceToHost, s));
        FE_HIP(hipStreamSynchronize(s));
        iters = hc[0] >= 0 ? hc[0] : maxit;
        reason = hc[0] >= 0 ? hc[1] : 2;
    }
    MinresScalars fin{};
    FE_HIP(hipMemcpyAsync(&fin, slot + (iters & 1), sizeof(fin), hipMemcpyDeviceToHost,
                          s));
    FE_HIP(hipStreamSynchronize(s));
    const double eta = fin.eta;
    const fe_status status = reason == 0 ? FE_OK : reason == 1 ? FE_EBREAKDOWN : FE_ENOTCONV;
    info->iters = iters;
    info->status = status;
    info->relres = bnorm > 0.0 ? std::fabs(eta) / bnorm : std::fabs(eta);
    // the true residual in the same norm
    if ((st = stokes_apply(S, u, p, w, w + nu, dnew, s)) != FE_OK) return st;
    hipLaunchKernelGGL(minres_init_kernel, dim3(g), dim3(256), 0, s, n, S->rhs, w, S->minv, v, z, S->part);
    double r2 = 0.0;
    if ((st = read_scalar(S, g, s, r2)) != FE_OK) return st;
    info->true_relres = bnorm > 0.0 ? std::sqrt(std::max(r2, 0.0)) / bnorm : std::sqrt(std::max(r2, 0.0));
    if (status == FE_ENOTCONV) return set_error(FE_ENOTCONV, "minres reached maxit");
    if (status == FE_EBREAKDOWN) return set_error(FE_EBREAKDOWN, "minres breakdown");
    return FE_OK;
}

}  // extern "C"
