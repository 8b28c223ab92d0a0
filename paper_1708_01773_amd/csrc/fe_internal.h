// fe_internal.h -- internal declarations of the HIP finite element library.
// Not part of the ABI (the ABI is include/fe.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/fe.h"

namespace fe {

constexpr int kMaxOrder = 4;
constexpr int kMaxQ1 = kMaxOrder + 1;  // Gauss points per direction (k + 1)

// ---------------------------------------------------------------------------
// Error handling (thread-local text behind fe_last_error)
// ---------------------------------------------------------------------------
fe_status set_error(fe_status st, const std::string &msg);
fe_status hip_error(hipError_t e, const char *what);

#define FE_HIP(call)                                                   \
    do {                                                               \
        hipError_t _e = (call);                                        \
        if (_e != hipSuccess) return ::fe::hip_error(_e, #call);       \
    } while (0)

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// ---------------------------------------------------------------------------
// One axis of the structured node lattice of order k.
// Node indices run over 0..N (N = n k).  Free indices are [lo, hi] (a
// Dirichlet face removes the end node).  For every free index i the columns
// of its row are the node interval [cl, cl + w) clipped to the free range;
// P is the prefix sum of w over free indices below i.  These three numbers
// are all the cell-to-nnz map needs along one axis: the sparsity pattern and
// every element entry's position are tensor products of them.
// ---------------------------------------------------------------------------
struct AxisTab {
    const int64_t *cl;  // device, f entries (absolute node index)
    const int64_t *w;   // device, f entries
    const int64_t *P;   // device, f entries
    int64_t lo, f, N, T;  // first free index, number of free indices, last node index, sum of w
    int32_t n;            // cells along the axis
    double finv;          // 1 / f (0 when f = 0)
};

// Everything kernels need about a (mesh, order, problem, Dirichlet faces).
struct SpaceArgs {
    int32_t dim, k, ncomp, nn, nloc;
    AxisTab ax[3];
    int64_t ncells;
    int64_t n_rows, nnz;
};

// Device-side view of the mesh.
struct MeshArgs {
    const double *x, *y, *z;  // vertex coordinates (SoA)
    const double *coef;       // per cell (nullptr: 1 on every cell)
    int32_t n0, n1, n2;       // cells per axis (n2 = 1 in 2D)
    int32_t *status;          // device status word (bit 0: det J <= 0 seen)
};

// Problem parameters used inside kernels.
struct ProblemArgs {
    int32_t problem;  // 0 Poisson, 1 elasticity
    int32_t precision;
    double lambda, mu;
    int32_t source_kind;
    double source[3];
    int32_t dirichlet_kind;
    double aff[12];
};

// 1D reference data: Gauss points/weights on [0,1] and Lagrange values /
// derivatives of the equidistant basis at those points, table[i * nq1 + q].
struct RefTables {
    double gx[kMaxQ1], gw[kMaxQ1];
    double L[kMaxQ1 * kMaxQ1], D[kMaxQ1 * kMaxQ1];
};

// Layout of the element workspace written by K3 and read by K5.
struct ElemLayout {
    int32_t cb;          // cells per block of the blocked layout
    int32_t packed;      // 1: only the upper triangle a <= b is stored (Q1 scalar)
    int32_t ne;          // entries stored per cell (nloc^2, or nloc (nloc + 1) / 2 when packed)
    int32_t elem_bytes;  // 8 (double) or 4 (float)
    size_t e_bytes;      // bytes of E (padded to 256)
    size_t f_offset;     // byte offset of F
    size_t total;        // bytes of the whole workspace
};

// One problem of a batched assembly launch (device table entry).
struct AsmJob {
    SpaceArgs s;
    MeshArgs m;
    ProblemArgs p;
    RefTables rt;
    void *E;      // element matrices (layout of elem_layout)
    double *F;    // element load vectors
    double *values, *rhs, *dinv;
    int32_t parts;  // matrix-core workgroups per cell
};

// Cached order-dependent set-up of a mesh.
struct Space {
    int32_t k = 0, ncomp = 0;
    uint32_t faces = 0xffffffffu;
    SpaceArgs args{};
    int64_t *d_axis = nullptr;     // 3 axes x {cl, w, P} device buffer
    int32_t *d_cell_dofs = nullptr;
    bool valid = false;
};

}  // namespace fe

struct fe_mesh_s {
    int32_t dim = 0;
    int32_t n[3] = {1, 1, 1};
    int64_t ncells = 0, nverts = 0;
    double *d_xyz = nullptr;  // SoA: x | y | z
    double *d_coef = nullptr;
    int32_t *d_status = nullptr;
    int32_t device = 0;
    hipStream_t last_stream = nullptr;
    fe::Space space;
};

namespace fe {

// Set-up (fe_setup.hip)
fe_status build_space(fe_mesh mesh, int k, int ncomp, uint32_t faces, Space &sp, hipStream_t s);
// Rows and nonzeros of a structured space, from the axis tables on the host.
void space_sizes(int dim, const int32_t *n, int k, int ncomp, uint32_t faces, int64_t &n_rows, int64_t &nnz);
// Validates (mesh, order, coeff) and builds the cached space on stream s.
fe_status prepare_space(fe_mesh m, int32_t order, const fe_coeff *c, hipStream_t s);
void free_space(Space &sp);
fe_status launch_pattern(const SpaceArgs &sa, int64_t *rowptr, int32_t *colind, hipStream_t s);
fe_status launch_cell_dofs(const SpaceArgs &sa, const MeshArgs &ma, int32_t *out, hipStream_t s);
fe_status launch_permutation(const SpaceArgs &sa, const MeshArgs &ma, int64_t *perm, hipStream_t s);
void ref_tables(int k, RefTables &t);
// Gauss-Legendre rule of n points on [0,1] (nodes ascending).
void gauss_legendre_01(int n, double *x, double *w);
// Value and derivative at x of the 1D Lagrange polynomial of node i/k of the
// equidistant order-k basis on [0,1] (Sect. 3.4 eq. lagbas).
void lagrange_1d(int k, int i, double x, double &val, double &der);
// Interior-penalty DG (fe_dg.hip): sizes, the space the volume integration
// runs on (scalar, nloc = nn, no shared DOFs), pattern and facet kernels.
void dg_sizes(int dim, const int32_t *n, int k, int64_t &n_rows, int64_t &nnz);
SpaceArgs dg_space(int dim, const int32_t *n, int k);
fe_status launch_dg_pattern(int dim, const int32_t *n, int k, int64_t *rowptr, int32_t *colind, hipStream_t s);
fe_status launch_dg_facets(int dim, const int32_t *n, int k, double gamma, double tau, const MeshArgs &ma,
                           const ProblemArgs &pa, const ElemLayout &el, const void *ws, const int64_t *rowptr,
                           double *values, double *rhs, double *dinv, hipStream_t s);

// Integration (fe_integrate.hip)
ElemLayout elem_layout(const SpaceArgs &sa, int precision);
fe_status launch_integrate(const SpaceArgs &sa, const MeshArgs &ma, const ProblemArgs &pa, const RefTables &rt,
                           const ElemLayout &el, void *ws, hipStream_t s);
fe_status launch_integrate_mfma(const SpaceArgs &sa, const MeshArgs &ma, const ProblemArgs &pa, const RefTables &rt,
                                void *E, double *F, hipStream_t s);
fe_status launch_lift(const SpaceArgs &sa, const MeshArgs &ma, const ProblemArgs &pa, const int32_t *cell_dofs,
                      const ElemLayout &el, void *ws, hipStream_t s);

// Batched launches: every job of one launch shares the kernel class named by
// the host job h (dimension, order, problem, precision); grid = boff[njobs].
bool integrate_batchable(const SpaceArgs &sa, const ProblemArgs &pa);
int64_t integrate_blocks(const SpaceArgs &sa, const ProblemArgs &pa, int32_t &parts);
int64_t mfma_blocks(const SpaceArgs &sa, const ProblemArgs &pa, int32_t &parts);
fe_status integrate_autotune(const SpaceArgs &sa, const MeshArgs &ma, const ProblemArgs &pa, const RefTables &rt,
                             void *E, double *F, int reps, fe_k3_plan *tried, int max_tried, int *n_tried,
                             fe_k3_plan *chosen, hipStream_t s);
void integrate_plan_of(const SpaceArgs &sa, const ProblemArgs &pa, fe_k3_plan *plan);
void integrate_tuning_reset();
fe_status launch_mfma_batch(const AsmJob &h, const AsmJob *jobs, const int32_t *boff, int njobs, int grid,
                            hipStream_t s);
fe_status launch_integrate_batch(const AsmJob &h, const AsmJob *jobs, const int32_t *boff, int njobs, int grid,
                                 hipStream_t s);
int64_t scatter_blocks(const SpaceArgs &sa, const ElemLayout &el);
fe_status launch_scatter_batch(const AsmJob &h, const ElemLayout &el, const AsmJob *jobs, const int32_t *boff,
                               int njobs, int grid, hipStream_t s);

// Scatter (fe_scatter.hip)
fe_status launch_scatter(const SpaceArgs &sa, const ElemLayout &el, const void *ws, double *values, double *rhs,
                         double *dinv, hipStream_t s);

// Solver (fe_solve.hip)
size_t pcg_ws_bytes(int64_t n);

// PCG engine over a set of problems (fe_solve.hip).  A job's ws holds
// pcg_ws_bytes(n) bytes of its own state and vectors; the set's table lives
// in engine_table_bytes(number of jobs) bytes of device memory.  Jobs with
// n == 0 are left out of the set.
struct PcgJob {
    int64_t n, nnz;
    const int64_t *rowptr;
    const int32_t *colind;
    const void *val;
    bool fp32;  // values stored as float
    const double *dinv, *b;
    double *x;
    void *ws;
    fe_solve_info *info;  // filled by engine_finish (may be null)
    double rtol;
    int maxit;
    const SpaceArgs *sa = nullptr;  // structured pattern of a mesh-assembled system (FP32 values: block-staged), or null
    bool sym = false;               // val is the symmetric storage of a Q1 scalar system on sa
    bool dg = false;                // val holds a DG system on sa (pattern evaluated per cell)
};
struct EngineSet;
EngineSet *engine_create();
void engine_destroy(EngineSet *E);
size_t engine_table_bytes(int njobs);
fe_status engine_build(EngineSet &E, const PcgJob *jobs, int njobs, void *table, hipStream_t s);
int engine_size(const EngineSet &E);
const PcgJob &engine_job(const EngineSet &E, int t);  // t-th job of the sorted set
fe_status engine_init(EngineSet &E, hipStream_t s);
fe_status engine_iterate(EngineSet &E, int iters, hipStream_t s);
fe_status engine_states(EngineSet &E, hipStream_t s);  // synchronizes
bool engine_done(const EngineSet &E, int t);           // from the last engine_states / engine_finish
fe_status engine_finish(EngineSet &E, hipStream_t s);  // true residuals + infos; synchronizes
fe_status launch_spmv(int64_t n, const int64_t *rowptr, const int32_t *colind, const double *val, const double *x,
                      double *y, int64_t nnz, hipStream_t s);
size_t pcg_solve_ws_bytes(int64_t n);
fe_status pcg_solve(const fe_csr *A, const double *b, double *x, double rtol, int maxit, void *ws, size_t ws_bytes,
                    fe_solve_info *info, hipStream_t s);
size_t pcg_noalloc_bytes();
fe_status pcg_solve_noalloc(const fe_csr *A, const double *b, double *x, double rtol, int maxit, fe_solve_info *info,
                            hipStream_t s);
size_t pcg_batch_ws_bytes(int nprob, const int64_t *n_rows);
// sas: per system, the space whose closed-form pattern the SpMV evaluates
// instead of reading column indices (null array or entry: generic CSR).
fe_status pcg_solve_batch(int nprob, const fe_csr *A, const double *const *b, double *const *x, double rtol,
                          int maxit, void *ws, size_t ws_bytes, fe_solve_info *infos, hipStream_t s,
                          const SpaceArgs *const *sas = nullptr);
fe_status pcg_solve_mesh(const fe_csr *A, const SpaceArgs &sa, const double *b, double *x, double rtol, int maxit,
                         void *ws, size_t ws_bytes, fe_solve_info *info, hipStream_t s);
fe_status launch_spmv_struct(const SpaceArgs &sa, const double *val, const double *x, double *y, hipStream_t s);
// DG systems (pattern of fe_dg_pattern evaluated from the cell index; sa from dg_space)
fe_status launch_spmv_dg(const SpaceArgs &sa, const double *val, const double *x, double *y, hipStream_t s);
fe_status pcg_solve_dg(const fe_csr *A, const SpaceArgs &sa, const double *b, double *x, double rtol, int maxit,
                       void *ws, size_t ws_bytes, fe_solve_info *info, hipStream_t s);
bool sym_supported(const SpaceArgs &sa);
size_t sym_bytes(const SpaceArgs &sa);
fe_status launch_sym_fill(const SpaceArgs &sa, const double *val, double *sym, hipStream_t s);
fe_status launch_sym_fill_fp32(const SpaceArgs &sa, const double *val, float *sym, hipStream_t s);
fe_status launch_spmv_sym(const SpaceArgs &sa, const double *sym, const double *x, double *y, hipStream_t s);
fe_status pcg_solve_sym(const fe_csr *A, const SpaceArgs &sa, const double *sym, const double *b, double *x,
                        double rtol, int maxit, void *ws, size_t ws_bytes, fe_solve_info *info, hipStream_t s);
size_t autotune_ws_bytes(int64_t n);
fe_status spmv_autotune(const fe_csr *A, int reps, void *ws, size_t ws_bytes, fe_spmv_plan *tried, int max_tried,
                        int *n_tried, fe_spmv_plan *chosen, hipStream_t s);
void spmv_tuning_reset();
void spmv_plan_of(int64_t n, int64_t nnz, fe_spmv_plan *plan, int32_t *cls);
fe_status spmv_plan_set(int64_t n, int64_t nnz, const fe_spmv_plan &plan);
fe_status spmv_autotune_struct(const SpaceArgs &sa, const double *values, int reps, void *ws, size_t ws_bytes,
                               fe_spmv_plan *tried, int max_tried, int *n_tried, fe_spmv_plan *chosen, hipStream_t s);
void spmv_plan_of_struct(const SpaceArgs &sa, fe_spmv_plan *plan, int32_t *cls);
fe_status spmv_plan_set_struct(const SpaceArgs &sa, const fe_spmv_plan &plan);
size_t refine_ws_bytes(int64_t n);
size_t refine_batch_ws_bytes(int nprob, const int64_t *n_rows);
fe_status refine_solve_batch(int nprob, const fe_csr *Ahi, const fe_csr *Alo, const double *const *b,
                             double *const *x, double rtol, double inner_rtol, int max_outer, int max_inner,
                             void *ws, size_t ws_bytes, fe_refine_info *infos, hipStream_t s,
                             const SpaceArgs *const *sas);
fe_status csr_to_fp32(const fe_csr *A, float *values32, hipStream_t s);
fe_status refine_solve(const fe_csr *Ahi, const fe_csr *Alo, const float *values32, const double *b, double *x,
                       double rtol, double inner_rtol, int max_outer, int max_inner, void *ws, size_t ws_bytes,
                       fe_refine_info *info, hipStream_t s, const SpaceArgs *sa = nullptr,
                       const float *sym32 = nullptr);

// Kernel timing (fe_set_timing / fe_get_timing): event pairs recorded on the
// launching stream around timed kernels.
enum TimedKind { kTimeIntegrate = 0, kTimeScatter = 1, kTimeSpmv = 2 };
bool timing_on();
hipEvent_t timing_begin(hipStream_t s);                    // nullptr when timing is off
void timing_end(hipEvent_t begin, TimedKind kind, hipStream_t s);
hipEvent_t timing_mark(hipStream_t s);                     // records a pooled event (nullptr when off)
void timing_commit(hipEvent_t a, hipEvent_t b, TimedKind kind);
void timing_release(hipEvent_t e);

// ---------------------------------------------------------------------------
// Device helpers shared by the kernels
// ---------------------------------------------------------------------------
// Cells along one axis that contain both node indices i and j (at most 2):
// e in [max(ceil(max(i,j)/k) - 1, 0), min(floor(min(i,j)/k), n - 1)].
__device__ __forceinline__ void shared_cells(int64_t i, int64_t j, int32_t k, int32_t n, int64_t &elo,
                                             int64_t &ehi)
{
    int64_t mx = i > j ? i : j, mn = i < j ? i : j;
    int64_t a = (mx + k - 1) / k - 1;
    elo = a > 0 ? a : 0;
    int64_t b = mn / k;
    ehi = b < n - 1 ? b : n - 1;
}

// Map a linear block id so that consecutive logical blocks run on the same
// XCD (the hardware dispatches block b to XCD b % 8).
__device__ __forceinline__ int64_t xcd_block(int64_t bid, int64_t nblocks)
{
    const int64_t nx = 8;
    if (nblocks < nx) return bid;
    int64_t per = nblocks / nx, rem = nblocks % nx;
    int64_t x = bid % nx, j = bid / nx;
    // XCD x owns logical blocks [start_x, start_x + per + (x < rem))
    int64_t start = x * per + (x < rem ? x : rem);
    return start + j;
}

// Position of element entry (a, b) of cell c in the element workspace.
__host__ __device__ __forceinline__ int64_t elem_index(int64_t c, int a, int b, int nloc, int cb, int packed, int ne)
{
    int e;
    if (packed) {
        const int lo = a < b ? a : b, hi = a < b ? b : a;
        e = lo * nloc - lo * (lo - 1) / 2 + (hi - lo);
    } else {
        e = a * nloc + b;
    }
    return ((c / cb) * int64_t(ne) + e) * cb + c % cb;
}

// Pattern of the interior-penalty DG system on a brick of n[0] x n[1] (x n[2])
// cells: the row block of cell K holds the columns of K and of its facet
// neighbours, cells in ascending id order.
// Cells K' < K whose index along an axis of stride st and extent n equals v.
__host__ __device__ __forceinline__ int64_t dg_count_at(int64_t K, int64_t st, int64_t n, int64_t v)
{
    const int64_t P = st * n, q = K / P, rem = K % P;
    int64_t t = rem - v * st;
    t = t < 0 ? 0 : (t > st ? st : t);
    return q * st + t;
}

// Sum over cells K' < K of the cells in the row block of K': (2d + 1) K minus
// the neighbours missing on the boundary.
__host__ __device__ __forceinline__ int64_t dg_prefix_n(int dim, int64_t n0, int64_t n1, int64_t n2, int64_t K)
{
    const int64_t nr[3] = {n0, n1, n2}, st[3] = {1, n0, n0 * n1};
    int64_t s = (2 * dim + 1) * K;
    for (int r = 0; r < dim; r++) s -= dg_count_at(K, st[r], nr[r], 0) + dg_count_at(K, st[r], nr[r], nr[r] - 1);
    return s;
}

// The cells of K's row block in ascending id order; returns their number.
__host__ __device__ __forceinline__ int dg_block_cells(int dim, int64_t n0, int64_t n1, int64_t n2, int64_t K,
                                                       int64_t cells[7])
{
    const int64_t c[3] = {K % n0, (K / n0) % n1, dim == 3 ? K / (n0 * n1) : 0};
    const int64_t nr[3] = {n0, n1, n2}, st[3] = {1, n0, n0 * n1};
    int m = 0;
    for (int r = 2; r >= 0; r--)
        if (r < dim && c[r] > 0) cells[m++] = K - st[r];
    cells[m++] = K;
    for (int r = 0; r < dim; r++)
        if (c[r] < nr[r] - 1) cells[m++] = K + st[r];
    return m;
}

// Job of block blockIdx.x in a launch whose job j owns the blocks
// [boff[j], boff[j+1]); lb = block index within the job, nb = its blocks.
__device__ __forceinline__ int find_job(const int32_t *__restrict__ boff, int njobs, int64_t &lb, int64_t &nb)
{
    int lo = 0, hi = njobs;  // boff[lo] <= b < boff[hi]
    const int b = int(blockIdx.x);
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (boff[mid] <= b) lo = mid;
        else hi = mid;
    }
    nb = boff[lo + 1] - boff[lo];
    lb = b - boff[lo];
    return lo;
}

// floor(a / d) for 0 <= a < 2^31, 0 < d, with inv = 1 / d: the double
// estimate is off by at most one and is corrected exactly.
__device__ __forceinline__ int32_t div_exact(int32_t a, int32_t d, double inv)
{
    int32_t q = int32_t((double(a) + 0.5) * inv);
    const int32_t r = a - q * d;
    q += r < 0 ? -1 : (r >= d ? 1 : 0);
    return q;
}

// Interval of columns of free node i along one axis and the prefix P(i) of
// the interval widths over the free nodes below i: closed forms of the axis
// tables built on the host (the unclipped interval of a vertex node is
// [i - k, i + k], of an element-interior node [k floor(i / k), + k]; the ends
// of the free range [lo, hi] clip them).  swlo = unclipped widths below lo.
struct AxisClosed {
    int32_t lo, hi, N, swlo;
};

__device__ __forceinline__ void axis_row(const AxisClosed &A, int32_t k, double kinv, int32_t i, int32_t &w,
                                         int32_t &cl, int32_t &P)
{
    if (A.N == 0) {  // the third axis of a 2D mesh
        w = 1;
        cl = 0;
        P = 0;
        return;
    }
    const int32_t m = i - div_exact(i, k, kinv) * k;
    const int32_t low = A.lo == 0 ? (i == 0 ? k : 0) : ((i >= 1 && i <= k) ? 1 : 0);
    const int32_t high = A.hi == A.N ? (i == A.N ? k : 0) : ((i >= A.N - k && i <= A.N - 1) ? 1 : 0);
    w = (m == 0 ? 2 * k + 1 : k + 1) - low - high;
    cl = (m == 0 ? i - k : i - m) + low;
    // unclipped widths of nodes 0..i-1: i (k + 1) + k ceil(i / k)
    P = i * (k + 1) + k * div_exact(i + k - 1, k, kinv) - A.swlo;
    P -= A.lo == 0 ? (i >= 1 ? k : 0) : max(0, min(i - 1, k));
    if (A.hi != A.N) P -= max(0, i - max(A.lo, A.N - k));
}

}  // namespace fe
