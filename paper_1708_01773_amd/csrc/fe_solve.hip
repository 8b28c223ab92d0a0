// fe_solve.hip -- K7/K8: FP64 CSR SpMV and Jacobi-preconditioned conjugate
// gradients (the CG the paper lists among its iterative solvers, Sect. 12;
// the preconditioner M = diag(A)).
//
// Per iteration three kernels run: q = A p with the partial sums of p.q,
// x/r updates with the partial sums of r.z and r.r (z = M^-1 r is never
// stored), and p = z + beta p.  Every reduction is two-stage and
// deterministic: a fixed grid writes one partial per block (wave shuffles,
// then LDS, in a fixed order), and the last block to finish -- detected with
// an integer counter, never a float atomic -- sums the partials in index
// order and updates the solver state in device memory.  A device-side "done"
// flag makes the remaining kernels of a chunk exit at once, so the host reads
// the state only once per chunk of iterations.
#include <cmath>
#include <cstring>
#include <vector>

#include "fe_internal.h"

namespace fe {

constexpr int kBlock = 256;
constexpr int kMaxBlocks = 2048;
constexpr int kHist = 4096;  // CG coefficients kept for the Lanczos estimates

struct PcgState {
    double rho, pq, alpha, beta, rr, bb, rtol2, true_rr;
    int32_t iter, done, status, maxit;
    uint32_t counter[4];
};

struct PcgWs {
    PcgState *st;
    double *part;  // 3 * kMaxBlocks partial sums
    double *hist;  // 2 * kHist (alpha, beta)
    double *r, *p, *q;
};

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

size_t pcg_ws_bytes(int64_t n)
{
    return align256(sizeof(PcgState)) + align256(3 * kMaxBlocks * sizeof(double)) +
           align256(2 * kHist * sizeof(double)) + 3 * align256(size_t(n) * sizeof(double));
}

static PcgWs carve(void *ws, int64_t n)
{
    char *p = static_cast<char *>(ws);
    PcgWs w;
    w.st = reinterpret_cast<PcgState *>(p);
    p += align256(sizeof(PcgState));
    w.part = reinterpret_cast<double *>(p);
    p += align256(3 * kMaxBlocks * sizeof(double));
    w.hist = reinterpret_cast<double *>(p);
    p += align256(2 * kHist * sizeof(double));
    w.r = reinterpret_cast<double *>(p);
    p += align256(size_t(n) * sizeof(double));
    w.p = reinterpret_cast<double *>(p);
    p += align256(size_t(n) * sizeof(double));
    w.q = reinterpret_cast<double *>(p);
    return w;
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of v over the block, in a fixed order; valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (&out)[NV])
{
    __shared__ double sh[NV][kBlock / 64];
    const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
#pragma unroll
    for (int t = 0; t < NV; t++) {
        const double s = wave_sum(v[t]);
        if (lane == 0) sh[t][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int t = 0; t < NV; t++) {
            double s = 0.0;
            for (int w = 0; w < kBlock / 64; w++) s += sh[t][w];
            out[t] = s;
        }
    }
}

// Writes the block's partials, and returns true in every thread of the last
// block to finish; then `tot` (valid in thread 0) holds the grand totals,
// summed over the blocks in index order.
template <int NV>
__device__ bool grid_sum(double (&v)[NV], double *part, uint32_t *counter, double (&tot)[NV])
{
    __shared__ bool last;
    double bs[NV];
    block_sum<NV>(v, bs);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int t = 0; t < NV; t++) part[t * kMaxBlocks + blockIdx.x] = bs[t];
        __threadfence();
        const uint32_t prev = atomicAdd(counter, 1u);
        last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return false;
    __threadfence();
    double acc[NV];
#pragma unroll
    for (int t = 0; t < NV; t++) {
        acc[t] = 0.0;
        for (int b = threadIdx.x; b < int(gridDim.x); b += kBlock)
            acc[t] += static_cast<volatile double *>(part)[t * kMaxBlocks + b];
    }
    __syncthreads();
    block_sum<NV>(acc, tot);
    if (threadIdx.x == 0) *counter = 0u;
    return true;
}

// ---------------------------------------------------------------------------
// Row dot product of a CSR row with L lanes (deterministic butterfly)
// ---------------------------------------------------------------------------
template <int L>
__device__ __forceinline__ double row_dot(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ colind,
                                          const double *__restrict__ val, const double *__restrict__ x, int64_t row,
                                          int lane)
{
    const int64_t b = rowptr[row], e = rowptr[row + 1];
    double s = 0.0;
    for (int64_t j = b + lane; j < e; j += L) s += val[j] * x[colind[j]];
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, L);
    return s;
}

// Rows [lo, hi) of logical block `lb` out of `nb` blocks.
__device__ __forceinline__ void block_rows(int64_t n, int64_t lb, int64_t nb, int64_t &lo, int64_t &hi)
{
    const int64_t chunk = (n + nb - 1) / nb;
    lo = lb * chunk;
    hi = lo + chunk < n ? lo + chunk : n;
    if (lo > n) lo = n;
}

template <int L>
__global__ __launch_bounds__(kBlock) void spmv_kernel(int64_t n, const int64_t *__restrict__ rowptr,
                                                       const int32_t *__restrict__ colind,
                                                       const double *__restrict__ val, const double *__restrict__ x,
                                                       double *__restrict__ y)
{
    constexpr int G = kBlock / L;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    int64_t lo, hi;
    block_rows(n, lb, gridDim.x, lo, hi);
    const int lane = threadIdx.x % L, grp = threadIdx.x / L;
    for (int64_t r0 = lo; r0 < hi; r0 += G) {
        const int64_t row = r0 + grp;
        double s = 0.0;
        if (row < hi) s = row_dot<L>(rowptr, colind, val, x, row, lane);
        if (row < hi && lane == 0) y[row] = s;
    }
}

// r = b - A x; z = dinv r; p = z; sums r.z, r.r, b.b
template <int L>
__global__ __launch_bounds__(kBlock) void pcg_init_kernel(int64_t n, const int64_t *__restrict__ rowptr,
                                                           const int32_t *__restrict__ colind,
                                                           const double *__restrict__ val,
                                                           const double *__restrict__ dinv,
                                                           const double *__restrict__ b, const double *__restrict__ x,
                                                           PcgWs w)
{
    constexpr int G = kBlock / L;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    int64_t lo, hi;
    block_rows(n, lb, gridDim.x, lo, hi);
    const int lane = threadIdx.x % L, grp = threadIdx.x / L;
    double v[3] = {0.0, 0.0, 0.0};
    for (int64_t r0 = lo; r0 < hi; r0 += G) {
        const int64_t row = r0 + grp;
        if (row < hi) {
            const double ax = row_dot<L>(rowptr, colind, val, x, row, lane);
            if (lane == 0) {
                const double r = b[row] - ax;
                const double z = dinv[row] * r;
                w.r[row] = r;
                w.p[row] = z;
                v[0] += r * z;
                v[1] += r * r;
                v[2] += b[row] * b[row];
            }
        }
    }
    double tot[3];
    if (grid_sum<3>(v, w.part, &w.st->counter[0], tot) && threadIdx.x == 0) {
        PcgState *st = w.st;
        st->rho = tot[0];
        st->rr = tot[1];
        st->bb = tot[2];
        st->iter = 0;
        st->status = FE_OK;
        st->done = (tot[1] <= st->rtol2 * tot[2]) ? 1 : 0;
        if (!st->done && st->maxit <= 0) {
            st->done = 1;
            st->status = FE_ENOTCONV;
        }
    }
}

// q = A p; sum p.q; alpha = rho / p.q
template <int L>
__global__ __launch_bounds__(kBlock) void pcg_spmv_kernel(int64_t n, const int64_t *__restrict__ rowptr,
                                                           const int32_t *__restrict__ colind,
                                                           const double *__restrict__ val, PcgWs w)
{
    if (w.st->done) return;
    constexpr int G = kBlock / L;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    int64_t lo, hi;
    block_rows(n, lb, gridDim.x, lo, hi);
    const int lane = threadIdx.x % L, grp = threadIdx.x / L;
    double v[1] = {0.0};
    for (int64_t r0 = lo; r0 < hi; r0 += G) {
        const int64_t row = r0 + grp;
        if (row < hi) {
            const double s = row_dot<L>(rowptr, colind, val, w.p, row, lane);
            if (lane == 0) {
                w.q[row] = s;
                v[0] += w.p[row] * s;
            }
        }
    }
    double tot[1];
    if (grid_sum<1>(v, w.part, &w.st->counter[1], tot) && threadIdx.x == 0) {
        PcgState *st = w.st;
        st->pq = tot[0];
        if (!(tot[0] > 0.0) || !isfinite(tot[0])) {
            st->done = 1;
            st->status = FE_EBREAKDOWN;
        } else {
            st->alpha = st->rho / tot[0];
        }
    }
}

// x += alpha p; r -= alpha q; sums r.z (z = dinv r) and r.r; beta; convergence
__global__ __launch_bounds__(kBlock) void pcg_update_kernel(int64_t n, const double *__restrict__ dinv,
                                                             double *__restrict__ x, PcgWs w)
{
    if (w.st->done) return;
    const double alpha = w.st->alpha;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    int64_t lo, hi;
    block_rows(n, lb, gridDim.x, lo, hi);
    double v[2] = {0.0, 0.0};
    for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
        x[i] += alpha * w.p[i];
        const double r = w.r[i] - alpha * w.q[i];
        w.r[i] = r;
        v[0] += r * (dinv[i] * r);
        v[1] += r * r;
    }
    double tot[2];
    if (grid_sum<2>(v, w.part, &w.st->counter[2], tot) && threadIdx.x == 0) {
        PcgState *st = w.st;
        const double beta = tot[0] / st->rho;
        const int it = st->iter;
        if (it < kHist) {
            w.hist[it] = st->alpha;
            w.hist[kHist + it] = beta;
        }
        st->beta = beta;
        st->rho = tot[0];
        st->rr = tot[1];
        st->iter = it + 1;
        if (tot[1] <= st->rtol2 * st->bb) {
            st->done = 1;
            st->status = FE_OK;
        } else if (it + 1 >= st->maxit) {
            st->done = 1;
            st->status = FE_ENOTCONV;
        }
    }
}

// p = dinv r + beta p
__global__ __launch_bounds__(kBlock) void pcg_dir_kernel(int64_t n, const double *__restrict__ dinv, PcgWs w)
{
    if (w.st->done) return;
    const double beta = w.st->beta;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    int64_t lo, hi;
    block_rows(n, lb, gridDim.x, lo, hi);
    for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) w.p[i] = dinv[i] * w.r[i] + beta * w.p[i];
}

// sum over rows of (b - A x)^2
template <int L>
__global__ __launch_bounds__(kBlock) void resid_kernel(int64_t n, const int64_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ colind,
                                                        const double *__restrict__ val, const double *__restrict__ b,
                                                        const double *__restrict__ x, PcgWs w)
{
    constexpr int G = kBlock / L;
    const int64_t lb = xcd_block(blockIdx.x, gridDim.x);
    int64_t lo, hi;
    block_rows(n, lb, gridDim.x, lo, hi);
    const int lane = threadIdx.x % L, grp = threadIdx.x / L;
    double v[1] = {0.0};
    for (int64_t r0 = lo; r0 < hi; r0 += G) {
        const int64_t row = r0 + grp;
        if (row < hi) {
            const double ax = row_dot<L>(rowptr, colind, val, x, row, lane);
            if (lane == 0) v[0] += (b[row] - ax) * (b[row] - ax);
        }
    }
    double tot[1];
    if (grid_sum<1>(v, w.part, &w.st->counter[3], tot) && threadIdx.x == 0) w.st->true_rr = tot[0];
}

__global__ void pcg_state_init_kernel(PcgState *st, double rtol2, int maxit)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->rho = st->pq = st->alpha = st->beta = st->rr = st->bb = st->true_rr = 0.0;
        st->rtol2 = rtol2;
        st->iter = 0;
        st->done = 0;
        st->status = FE_OK;
        st->maxit = maxit;
        for (int i = 0; i < 4; i++) st->counter[i] = 0u;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int lanes_for(double nnz_per_row)
{
    int L = 2;
    while (L < 64 && 2 * L <= nnz_per_row / 2.0) L *= 2;
    return L;
}

static int grid_for(int64_t n, int L)
{
    const int64_t per = kBlock / L;
    int64_t g = (n + per - 1) / per;
    if (g > kMaxBlocks) g = kMaxBlocks;
    if (g < 1) g = 1;
    return int(g);
}

#define FE_LANES_DISPATCH(L, CALL) \
    switch (L) {                   \
        case 2: CALL(2); break;    \
        case 4: CALL(4); break;    \
        case 8: CALL(8); break;    \
        case 16: CALL(16); break;  \
        case 32: CALL(32); break;  \
        default: CALL(64); break;  \
    }

fe_status launch_spmv(int64_t n, const int64_t *rowptr, const int32_t *colind, const double *val, const double *x,
                      double *y, double nnz_per_row, hipStream_t s)
{
    if (n == 0) return FE_OK;
    const int L = lanes_for(nnz_per_row);
    const int grid = grid_for(n, L);
#define FE_SPMV(LV) hipLaunchKernelGGL(spmv_kernel<LV>, dim3(grid), dim3(kBlock), 0, s, n, rowptr, colind, val, x, y)
    FE_LANES_DISPATCH(L, FE_SPMV)
#undef FE_SPMV
    FE_HIP(hipGetLastError());
    return FE_OK;
}

// Smallest / largest eigenvalue of the symmetric tridiagonal (d, e) by
// bisection on Sturm sequence counts.
static int sturm_count(const std::vector<double> &d, const std::vector<double> &e, double x)
{
    int cnt = 0;
    double q = 1.0;
    for (size_t i = 0; i < d.size(); i++) {
        const double off = i > 0 ? e[i - 1] * e[i - 1] : 0.0;
        q = d[i] - x - (i > 0 ? off / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0) cnt++;
    }
    return cnt;
}

static void tridiag_extremes(const std::vector<double> &d, const std::vector<double> &e, double &lmin, double &lmax)
{
    const size_t m = d.size();
    double lo = d[0], hi = d[0];
    for (size_t i = 0; i < m; i++) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(e[i]) : 0.0);
        lo = std::fmin(lo, d[i] - r);
        hi = std::fmax(hi, d[i] + r);
    }
    auto kth = [&](int k) {
        double a = lo, b = hi;
        for (int it = 0; it < 200 && b - a > 1e-14 * std::fmax(std::fabs(a), std::fabs(b)); it++) {
            const double mid = 0.5 * (a + b);
            if (sturm_count(d, e, mid) >= k) b = mid;
            else a = mid;
        }
        return 0.5 * (a + b);
    };
    lmin = kth(1);
    lmax = kth(int(m));
}

struct PinnedState {
    PcgState *h = nullptr;
    ~PinnedState()
    {
        if (h) (void)hipHostFree(h);
    }
};

fe_status pcg_solve(const fe_csr *A, const double *b, double *x, double rtol, int maxit, void *ws, size_t ws_bytes,
                    fe_solve_info *info, hipStream_t s)
{
    const int64_t n = A->n_rows;
    if (ws_bytes < pcg_ws_bytes(n)) return set_error(FE_EINVAL, "pcg workspace too small");
    static thread_local PinnedState pin;
    if (!pin.h) FE_HIP(hipHostMalloc(reinterpret_cast<void **>(&pin.h), sizeof(PcgState), hipHostMallocDefault));
    PcgWs w = carve(ws, n);
    std::memset(info, 0, sizeof(*info));
    if (n == 0) {
        info->status = FE_OK;
        return FE_OK;
    }
    const double npr = double(A->nnz) / double(n);
    const int L = lanes_for(npr);
    const int gs = grid_for(n, L);                       // SpMV-shaped kernels
    const int gv = int(std::min<int64_t>(kMaxBlocks, (n + kBlock - 1) / kBlock));  // vector kernels
    hipLaunchKernelGGL(pcg_state_init_kernel, dim3(1), dim3(64), 0, s, w.st, rtol * rtol, maxit);
#define FE_INIT(LV) \
    hipLaunchKernelGGL(pcg_init_kernel<LV>, dim3(gs), dim3(kBlock), 0, s, n, A->rowptr, A->colind, A->values, A->dinv, b, x, w)
    FE_LANES_DISPATCH(L, FE_INIT)
#undef FE_INIT
    FE_HIP(hipGetLastError());
    int chunk = 8;
    int launched = 0;
    while (true) {
        for (int i = 0; i < chunk && launched < maxit; i++, launched++) {
#define FE_SPMVK(LV) \
    hipLaunchKernelGGL(pcg_spmv_kernel<LV>, dim3(gs), dim3(kBlock), 0, s, n, A->rowptr, A->colind, A->values, w)
            hipEvent_t t0 = timing_begin(s);
            FE_LANES_DISPATCH(L, FE_SPMVK)
            timing_end(t0, kTimeSpmv, s);
#undef FE_SPMVK
            hipLaunchKernelGGL(pcg_update_kernel, dim3(gv), dim3(kBlock), 0, s, n, A->dinv, x, w);
            hipLaunchKernelGGL(pcg_dir_kernel, dim3(gv), dim3(kBlock), 0, s, n, A->dinv, w);
        }
        FE_HIP(hipGetLastError());
        FE_HIP(hipMemcpyAsync(pin.h, w.st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
        FE_HIP(hipStreamSynchronize(s));
        if (pin.h->done || launched >= maxit) break;
        if (chunk < 128) chunk *= 2;
    }
#define FE_RES(LV) \
    hipLaunchKernelGGL(resid_kernel<LV>, dim3(gs), dim3(kBlock), 0, s, n, A->rowptr, A->colind, A->values, b, x, w)
    FE_LANES_DISPATCH(L, FE_RES)
#undef FE_RES
    FE_HIP(hipGetLastError());
    FE_HIP(hipMemcpyAsync(pin.h, w.st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    FE_HIP(hipStreamSynchronize(s));
    const PcgState st = *pin.h;
    info->iters = st.iter;
    info->status = st.done ? st.status : FE_ENOTCONV;
    const double bn = std::sqrt(st.bb);
    info->relres = bn > 0 ? std::sqrt(st.rr) / bn : std::sqrt(st.rr);
    info->true_relres = bn > 0 ? std::sqrt(st.true_rr) / bn : std::sqrt(st.true_rr);
    const int m = std::min(st.iter, kHist);
    if (m > 0) {
        std::vector<double> h(2 * kHist);
        FE_HIP(hipMemcpy(h.data(), w.hist, sizeof(double) * 2 * kHist, hipMemcpyDeviceToHost));
        std::vector<double> d(m), e(m > 1 ? m - 1 : 1);
        for (int j = 0; j < m; j++) {
            const double a = h[j], bprev = j > 0 ? h[kHist + j - 1] : 0.0, aprev = j > 0 ? h[j - 1] : 1.0;
            d[j] = 1.0 / a + (j > 0 ? bprev / aprev : 0.0);
            if (j + 1 < m) e[j] = std::sqrt(h[kHist + j]) / a;
        }
        tridiag_extremes(d, e, info->lambda_min_est, info->lambda_max_est);
    }
    if (info->status == FE_ENOTCONV) set_error(FE_ENOTCONV, "pcg reached maxit");
    if (info->status == FE_EBREAKDOWN) set_error(FE_EBREAKDOWN, "pcg breakdown: p.Ap <= 0 or not finite");
    return fe_status(info->status);
}

}  // namespace fe
