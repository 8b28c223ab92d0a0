// fe_solve.hip -- K7/K8: FP64 CSR SpMV and Jacobi-preconditioned conjugate
// gradients (the CG the paper lists among its iterative solvers, Sect. 12;
// the preconditioner M = diag(A)).
//
// Iteration j runs three kernels:
//   spmv(j):  q = A p                      partials of p.q
//   upd(j):   alpha = rho_j / p.q;  x += alpha p;  r -= alpha q
//                                          partials of r.z and r.r (z = M^-1 r, never stored)
//   dir(j):   beta = rho_{j+1} / rho_j;  stop if ||r|| <= rtol ||b||;  p = z + beta p
// Reductions are deterministic and use no atomics and no fences: every block
// writes one partial with a plain store, and every block of the *next* kernel
// sums all partials in index order (the kernel boundary makes them visible),
// so all blocks agree bit for bit on the scalar.  Scalars that outlive a
// kernel (rho, the stop flag) are written by block 0 into slots indexed by
// the iteration parity, which the host passes in, so no kernel reads a slot
// it also writes.  A device-side stop flag makes the remaining kernels of a
// chunk of iterations exit at once; the host reads the state once per chunk.
//
// SpMV: rows with few non-zeros use a wave-level CSR-stream scheme (a wave
// stages the products of a run of rows in LDS with coalesced loads, then
// L lanes per row sum them); long rows use one wave per row straight from
// memory.  A row is always summed in the same lane-strided order followed by
// the same butterfly, so the result does not depend on the path taken.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>
#include <vector>

#include "fe_internal.h"

namespace fe {

constexpr int kBlock = 512;
constexpr int kWaves = kBlock / 64;
constexpr int kGrid = 1024;     // most blocks of a CSR or lanes-per-row kernel (each owns a contiguous chunk)
constexpr int kPartMax = 32768; // most blocks of a row kernel of the Q1 traversal (one partial each)
constexpr int kGridE = 256;     // most blocks of the vector kernels (update, dir)
constexpr int kHist = 4096;     // CG coefficients kept for the Lanczos estimates
constexpr int kWaveCap = 256;   // products staged in LDS per wave (2 KB)

// Device pointers read from a problem table are generic pointers; naming
// them global lets the compiler use global loads and stores, which do not
// count against the LDS counter the way flat accesses do.
#define FE_GLOBAL __attribute__((address_space(1)))
typedef double fe_dpair __attribute__((ext_vector_type(2)));  // 16-byte access of two doubles
__device__ __forceinline__ bool pair_aligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
template <typename T>
__device__ __forceinline__ const FE_GLOBAL T *as_global(const T *p)
{
    return (const FE_GLOBAL T *)p;
}
// A pointer that is the same in every lane, moved to scalar registers, so
// loads take it as their base with a 32-bit offset per lane.  The builtin
// reads an int: both halves go back through uint32_t, or the low half would
// be sign-extended into the high one.
template <typename T>
__device__ __forceinline__ const FE_GLOBAL char *wave_base(const T *p)
{
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(a))));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(a >> 32))));
    return reinterpret_cast<const FE_GLOBAL char *>((uint64_t(hi) << 32) | uint64_t(lo));
}
template <typename T>
__device__ __forceinline__ FE_GLOBAL T *as_global(T *p)
{
    return (FE_GLOBAL T *)p;
}

struct PcgState {
    double rho[2];  // rho_j in slot j & 1
    double bb, rr, true_rr;
    double alpha;      // alpha_j, from the update kernel to the dir kernel (x += alpha p there)
    int32_t iter;      // current iteration j (advanced by the dir kernel)
    int32_t iter_upd;  // j as seen by the update kernel, read by the dir kernel
    int32_t done;      // stopped before any iteration, or by a breakdown
    int32_t stop_at;   // the iteration whose dir kernel stopped the solve (converged or maxit)
    int32_t status;
};

// The solve has stopped for kernels of iteration j: the dir kernel of an
// earlier iteration stopped it (the dir kernel of iteration j itself records
// stop_at = j, which its other blocks read as still running), or it stopped
// before the first iteration or at a breakdown.
__host__ __device__ inline bool pcg_stopped(const PcgState &s, int32_t j) { return s.done || s.stop_at < j; }

struct PcgWs {
    PcgState *st;
    double *p1;    // ps partials of p.q (one per block of the row kernel)
    double *p2;    // 2 x kGrid partials of r.z, r.r
    double *p3;    // 3 x ps partials of the initial r.z, r.r, b.b (and the final residual)
    int32_t ps;    // partial slots of the row kernels
    double *hist;  // 2 x kHist (alpha, beta)
    double *r, *p, *q;
};

// One problem of a (possibly batched) solve, as the kernels see it.
struct PcgProb {
    int64_t n, nnz;
    const int64_t *rowptr;
    const int32_t *colind;
    const void *val;
    const double *dinv, *b;
    double *x;
    PcgWs w;
    double rtol2;
    int32_t maxit;
    int32_t nbr, nbe;  // blocks of the row kernels / of the vector kernels
    SpaceArgs sa;      // pattern of a system assembled on a structured brick (mode 2)
};

// How a CSR matrix is traversed.
struct SpmvPlan {
    int mode;  // 0: wave-level CSR-stream, 1: wave per row, 2: structured (pattern evaluated),
               // 3: structured short rows, two lanes per row (rpb = longest row),
               // 4: structured Q1 scalar rows, values and x runs staged in LDS (rpb = longest row),
               // 5: mode 4 with one wave step per wave (launch form only),
               // 6: structured rows, x of a 32-row chunk's column box staged per block (rpb 8),
               // 7: Q1 scalar rows of a system in symmetric storage (rpb = longest row),
               // 8: mode 7 with one wave step per wave (launch form only)
    int nc = 1;  // components (mode 2)
    int rpb;   // rows per wave-iteration (stream mode)
    int lanes; // lanes per row
};


// Partial slots of the row kernels of an n-row system: kGrid, or one per
// block of the Q1 traversal (128 rows each) up to kPartMax.
static int32_t part_slots(int64_t n)
{
    // a multiple of 8: the symmetric Q1 traversal pads its grid to one
    return int32_t(std::max<int64_t>(kGrid, std::min<int64_t>(kPartMax, ((n + 127) / 128 + 7) / 8 * 8)));
}

size_t pcg_ws_bytes(int64_t n)
{
    const size_t ps = size_t(part_slots(n));
    return align256(sizeof(PcgState)) + 4 * align256(ps * sizeof(double)) + 2 * align256(kGrid * sizeof(double)) +
           align256(2 * kHist * sizeof(double)) + 3 * align256(size_t(n) * sizeof(double));
}

static PcgWs carve(void *ws, int64_t n)
{
    char *p = static_cast<char *>(ws);
    PcgWs w;
    w.st = reinterpret_cast<PcgState *>(p);
    p += align256(sizeof(PcgState));
    w.ps = part_slots(n);
    w.p1 = reinterpret_cast<double *>(p);
    p += align256(size_t(w.ps) * sizeof(double));
    w.p2 = reinterpret_cast<double *>(p);
    p += 2 * align256(kGrid * sizeof(double));
    w.p3 = reinterpret_cast<double *>(p);
    p += 3 * align256(size_t(w.ps) * sizeof(double));
    w.hist = reinterpret_cast<double *>(p);
    p += align256(2 * kHist * sizeof(double));
    w.r = reinterpret_cast<double *>(p);
    p += align256(size_t(n) * sizeof(double));
    w.p = reinterpret_cast<double *>(p);
    p += align256(size_t(n) * sizeof(double));
    w.q = reinterpret_cast<double *>(p);
    return w;
}

// Device slot for the problem table of a single-problem solve (inside its workspace).
// Wave-level plans (modes 0 and 1) by average row length.
static SpmvPlan stream_plan(double avg)
{
    SpmvPlan pl{};
    if (avg >= 96.0) {
        pl.mode = 1;
        pl.rpb = 1;
        pl.lanes = 64;
        return pl;
    }
    int rpw = 32;  // a run's rpw + 1 row pointers sit in one wave's lanes
    while (rpw > 1 && rpw * avg > double(kWaveCap)) rpw /= 2;
    pl.mode = 0;
    pl.rpb = rpw;
    pl.lanes = 64 / rpw;
    return pl;
}

// Plans measured by the autotuner, per class of average row length (half
// octaves of nnz / n).  A plan fixes the summation order of every row, so a
// matrix gets the same plan alone and in a batch as long as the table is not
// changed in between.
static std::mutex g_tune_mu;
static std::map<int, SpmvPlan> g_tuned;

// The default CSR plan: block tiles (mode 9) of R rows, R the largest power of
// two in [4, 256] with R avg <= kTileRowsTarget entries (three passes; the
// fastest tile sizes of the autotuner on the 128^3 Q1 and the Q2-Q4
// elasticity matrices, 27 to 611 entries per row, lie at 3000-9000 entries).
constexpr double kTileRowsTarget = 6144.0;
static SpmvPlan heuristic_plan(double avg)
{
    int R = 256;
    while (R > 4 && R * avg > kTileRowsTarget) R /= 2;
    SpmvPlan pl{};
    pl.mode = 9;
    pl.rpb = R;
    pl.lanes = 256 / R;
    return pl;
}

// Mode 9 loads column indices and values 16 bytes at a time; a matrix whose
// arrays are not 16-byte aligned takes the wave-level plan of its row length.
static SpmvPlan csr_launch_form(SpmvPlan pl, int64_t n, int64_t nnz, const int32_t *colind, const void *val)
{
    if (pl.mode == 9 && ((reinterpret_cast<uintptr_t>(colind) | reinterpret_cast<uintptr_t>(val)) & 15u))
        return stream_plan(n > 0 ? double(nnz) / double(n) : 1.0);
    return pl;
}

static int plan_class(int64_t n, int64_t nnz)
{
    const double avg = n > 0 ? double(nnz) / double(n) : 1.0;
    return int(std::floor(2.0 * std::log2(std::max(avg, 1.0))));
}

static SpmvPlan plan_for(int64_t n, int64_t nnz)
{
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(plan_class(n, nnz));
        if (it != g_tuned.end()) return it->second;
    }
    return heuristic_plan(n > 0 ? double(nnz) / double(n) : 1.0);
}

// ---------------------------------------------------------------------------
// Reductions
// ---------------------------------------------------------------------------
template <int W>
__device__ __forceinline__ double butterfly(double v)
{
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
    return v;
}

// Sum over a block of B threads in a fixed order; the result is returned in
// every thread.
template <int NV, int B = kBlock>
__device__ __forceinline__ void block_sum_all(double (&v)[NV])
{
    __shared__ double sh[NV][B / 64];
    __shared__ double res[NV];
    const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
#pragma unroll
    for (int t = 0; t < NV; t++) {
        const double s = butterfly<64>(v[t]);
        if (lane == 0) sh[t][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < B / 64; w++) s += sh[threadIdx.x][w];
        res[threadIdx.x] = s;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NV; t++) v[t] = res[t];
    __syncthreads();
}

// Block partials of v -> part[t * stride + blockIdx.x].
template <int NV, int B = kBlock>
__device__ __forceinline__ void write_partials(double (&v)[NV], double *part, int stride)
{
    block_sum_all<NV, B>(v);
    if (threadIdx.x == 0)
#pragma unroll
        for (int t = 0; t < NV; t++) part[t * stride + blockIdx.x] = v[t];
}

// Grand totals of partials part[t * stride + b], b < nparts, written by a
// previous kernel of `nparts` blocks; identical in every thread of every
// block.  A thread sums the pairs of partials b = tid + j kBlock into
// accumulator j mod 8 (eight pair loads in flight; an odd last partial goes
// to thread 0's last accumulator) and adds the eight in a fixed tree.
template <int NV>
__device__ __forceinline__ void reduce_partials(const double *gpart, int nparts, int stride, double (&tot)[NV])
{
    const FE_GLOBAL double *__restrict__ part = as_global(gpart);
#pragma unroll
    for (int t = 0; t < NV; t++) {
        const FE_GLOBAL double *__restrict__ pt = part + int64_t(t) * stride;
        double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        const int np2 = nparts / 2;
        // pair b (partials 2b, 2b + 1) goes to accumulator (b / kBlock) mod 8;
        // 16-byte loads when the array is 16-byte aligned, else two 8-byte
        // loads: the same sums either way (decided once, outside the loops)
        auto sum_pairs = [&](auto wide) {
            constexpr bool W = decltype(wide)::value;
            auto pair = [&](int b) -> double {
                if constexpr (W) {
                    const fe_dpair v = *reinterpret_cast<const FE_GLOBAL fe_dpair *>(pt + 2 * b);
                    return v.x + v.y;
                } else {
                    return pt[2 * b] + pt[2 * b + 1];
                }
            };
            int b = threadIdx.x;
            for (; b + 7 * kBlock < np2; b += 8 * kBlock) {
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; u++) v[u] = pair(b + u * kBlock);
#pragma unroll
                for (int u = 0; u < 8; u++) a[u] += v[u];
            }
            for (int u = 0; b < np2; b += kBlock, u++) a[u] += pair(b);
        };
        if (pair_aligned(gpart + int64_t(t) * stride)) sum_pairs(std::true_type{});
        else sum_pairs(std::false_type{});
        if ((nparts & 1) && threadIdx.x == 0) a[7] += pt[nparts - 1];
        tot[t] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
    block_sum_all<NV>(tot);
}

// ---------------------------------------------------------------------------
// Row traversal
// ---------------------------------------------------------------------------
template <int L, typename VT>
__device__ __forceinline__ double row_dot(const int64_t *__restrict__ growptr, const int32_t *__restrict__ gcolind,
                                          const VT *__restrict__ gval, const double *__restrict__ gx, int64_t row,
                                          int lane)
{
    const FE_GLOBAL int64_t *__restrict__ rowptr = as_global(growptr);
    const FE_GLOBAL int32_t *__restrict__ colind = as_global(gcolind);
    const FE_GLOBAL VT *__restrict__ val = as_global(gval);
    const FE_GLOBAL double *__restrict__ x = as_global(gx);
    const int64_t b = rowptr[row], e = rowptr[row + 1];
    double s = 0.0;
    int64_t j = b + lane;
    // four loads in flight per lane, summed in the same lane-strided order
    for (; j + 3 * L < e; j += 4 * L) {
        double v[4];
        int32_t c[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            v[u] = double(val[j + u * L]);
            c[u] = colind[j + u * L];
        }
#pragma unroll
        for (int u = 0; u < 4; u++) s += v[u] * x[c[u]];
    }
    for (; j < e; j += L) s += double(val[j]) * x[colind[j]];
    return butterfly<L>(s);
}

// LDS writes of a wave made visible to the other lanes of the same wave.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Calls f(row, A_row . x) once per row handled by this wave (in the first
// lane of the row's lane group).  Wave-level CSR-stream: the rows are cut
// into runs of RPW; run t is handled by logical wave t mod (number of waves),
// so the waves of a workgroup work on neighbouring rows and share the
// gathered entries of x in cache (a mapping of workgroups to XCDs measured
// 3% slower than the hardware's round robin, so none is applied).  A wave
// loads the run's RPW + 1 row pointers with one coalesced load, issues every
// load of the run's values and column indices before the first gather of x,
// stages the products in its own LDS slice, then LW = 64 / RPW lanes per row
// sum them.  A run longer than the slice is summed straight from memory in
// the same lane order.
// lb / nb: this block's index among the nb blocks working on the matrix.
template <int RPW, typename VT, typename Fn>
__device__ __forceinline__ void for_rows_wstream(int64_t n, const int64_t *__restrict__ growptr,
                                                 const int32_t *__restrict__ gcolind, const VT *__restrict__ gval,
                                                 const double *__restrict__ gx, int64_t lb, int64_t nb, Fn f)
{
    const FE_GLOBAL int64_t *__restrict__ rowptr = as_global(growptr);
    const FE_GLOBAL int32_t *__restrict__ colind = as_global(gcolind);
    const FE_GLOBAL VT *__restrict__ val = as_global(gval);
    const FE_GLOBAL double *__restrict__ x = as_global(gx);
    constexpr int LW = 64 / RPW;
    __shared__ double prod[kWaves][kWaveCap];
    double *my = prod[threadIdx.x / 64];
    const int lane = threadIdx.x % 64, grp = lane / LW, sub = lane % LW;
    const int64_t nw = nb * kWaves;
    const int64_t lw = lb * kWaves + threadIdx.x / 64;
    const int64_t runs = (n + RPW - 1) / RPW;
    for (int64_t run = lw; run < runs; run += nw) {
        const int64_t r0 = run * RPW;
        const int64_t r1 = std::min<int64_t>(r0 + RPW, n);
        const int64_t rp = (lane <= RPW && r0 + lane <= n) ? rowptr[r0 + lane] : 0;
        const int64_t base = __shfl(rp, 0), end = __shfl(rp, int(r1 - r0));
        const int64_t rb = __shfl(rp, grp), re = __shfl(rp, grp + 1);
        const int64_t row = r0 + grp;
        double s = 0.0;
        if (end - base <= kWaveCap) {
            // every load of the run is issued before the first gather
            constexpr int CH = kWaveCap / 64;
            int32_t c[CH];
            double a[CH], xv[CH];
#pragma unroll
            for (int u = 0; u < CH; u++) {
                const int64_t j = base + lane + 64 * u;
                const bool ok = j < end;
                c[u] = ok ? colind[j] : 0;
                a[u] = ok ? double(val[j]) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < CH; u++) xv[u] = x[c[u]];
#pragma unroll
            for (int u = 0; u < CH; u++) my[lane + 64 * u] = a[u] * xv[u];
            wave_lds_sync();
            if (row < r1)
                for (int64_t t = rb - base + sub; t < re - base; t += LW) s += my[t];
            s = butterfly<LW>(s);
            wave_lds_sync();
        } else if (row < r1) {
            for (int64_t j = rb + sub; j < re; j += LW) s += double(val[j]) * x[colind[j]];
            s = butterfly<LW>(s);
        }
        if (row < r1 && sub == 0) f(row, s);
    }
}

// One wave per row (long rows), 64 lanes.
template <typename VT, typename Fn>
__device__ __forceinline__ void for_rows_wave(int64_t n, const int64_t *__restrict__ rowptr,
                                              const int32_t *__restrict__ colind, const VT *__restrict__ val,
                                              const double *__restrict__ x, int64_t lb, int64_t nb, Fn f)
{
    const int64_t nw = nb * kWaves;
    const int64_t lw = lb * kWaves + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    for (int64_t row = lw; row < n; row += nw) {
        const double s = row_dot<64>(rowptr, colind, val, x, row, lane);
        if (lane == 0) f(row, s);
    }
}

// CSR rows in block tiles (plan mode 9; R rows per tile, 4 <= R <= 256).  A
// block of kTileThreads threads takes a tile of R consecutive rows and streams
// its entries in passes of kTileCap: each thread loads four consecutive
// column indices with one 16-byte load and their values with 16-byte loads
// (two groups of four per thread, every load of a pass issued before the
// first gather of x), multiplies and stages the products in LDS; then the
// LPR = kTileThreads / R lanes of each row sum its staged entries of the pass
// in lane order, and a butterfly over the LPR lanes ends the row.  The
// streamed range starts at the row pointer rounded down to a multiple of four
// entries (the lead is loaded and masked); the last group of the matrix, if
// it has fewer than four entries, is loaded element by element.  Tiles are
// dealt XCD-contiguously: block lb runs on XCD lb mod 8 (nb is a multiple of
// 8), and the blocks of XCD x take the tiles of [x T / 8, (x + 1) T / 8) in
// turn, so a tile and its neighbours -- which gather much of the same x -- run
// under one L2.  Needs colind and val 16-byte aligned (checked at launch).
constexpr int kTileThreads = 256;
constexpr int kTileCap = 2048;  // products staged per pass (16 KB of LDS)
constexpr int kTileGroups = kTileCap / (4 * kTileThreads);

template <int R, typename VT, typename Fn>
__device__ __forceinline__ void for_rows_tiles(int64_t n, int64_t nnz, const int64_t *__restrict__ growptr,
                                               const int32_t *__restrict__ gcolind, const VT *__restrict__ gval,
                                               const double *__restrict__ gx, int64_t lb, int64_t nb, Fn f)
{
    static_assert(R >= 4 && R <= kTileThreads && kTileThreads % R == 0, "rows per tile");
    constexpr int LPR = kTileThreads / R;
    typedef int32_t int4v __attribute__((ext_vector_type(4)));
    typedef float float4v __attribute__((ext_vector_type(4)));
    const FE_GLOBAL int64_t *__restrict__ rowptr = as_global(growptr);
    const FE_GLOBAL int32_t *__restrict__ colind = as_global(gcolind);
    const FE_GLOBAL VT *__restrict__ val = as_global(gval);
    const FE_GLOBAL double *__restrict__ x = as_global(gx);
    __shared__ double prod[kTileCap];
    __shared__ int64_t rp[R + 1];
    const int tid = threadIdx.x, lr = tid / LPR, sub = tid % LPR;
    const int64_t ntiles = (n + R - 1) / R;
    const int64_t xcd = lb % 8, per = nb / 8;
    const int64_t t_hi = (xcd + 1) * ntiles / 8;
    // the row pointers of a tile: thread tid < nr holds rowptr[r0 + tid],
    // thread 0 also the tile's end; the next tile's are loaded while this one
    // streams, so only a block's first tile waits for them
    int64_t pa = 0, pe = 0;
    auto fetch_rp = [&](int64_t t) {
        const int64_t q0 = t * R;
        const int m = int(n - q0 < R ? n - q0 : R);
        pa = tid < m ? rowptr[q0 + tid] : 0;
        pe = tid == 0 ? rowptr[q0 + m] : 0;
    };
    int64_t tile = xcd * ntiles / 8 + lb / 8;
    if (tile < t_hi) fetch_rp(tile);
    for (; tile < t_hi; tile += per) {
        const int64_t r0 = tile * R;
        const int nr = int(n - r0 < R ? n - r0 : R);
        __syncthreads();  // the previous tile's reads of rp and prod are done
        if (tid < nr) rp[tid] = pa;
        if (tid == 0) rp[nr] = pe;
        __syncthreads();
        if (tile + per < t_hi) fetch_rp(tile + per);
        const int64_t base = rp[0], end = rp[nr];
        const int64_t rb = lr < nr ? rp[lr] : end, re = lr < nr ? rp[lr + 1] : end;
        double acc = 0.0;
        for (int64_t p0 = base & ~int64_t(3); p0 < end; p0 += kTileCap) {
            int32_t c[kTileGroups][4];
            double a[kTileGroups][4];
#pragma unroll
            for (int g = 0; g < kTileGroups; g++) {
                const int64_t e = p0 + 4 * (tid + kTileThreads * g);
                if (e < end && e + 4 <= nnz) {
                    const int4v cv = *reinterpret_cast<const FE_GLOBAL int4v *>(colind + e);
                    c[g][0] = cv.x;
                    c[g][1] = cv.y;
                    c[g][2] = cv.z;
                    c[g][3] = cv.w;
                    if constexpr (sizeof(VT) == 8) {
                        const fe_dpair v0 = *reinterpret_cast<const FE_GLOBAL fe_dpair *>(val + e);
                        const fe_dpair v1 = *reinterpret_cast<const FE_GLOBAL fe_dpair *>(val + e + 2);
                        a[g][0] = v0.x;
                        a[g][1] = v0.y;
                        a[g][2] = v1.x;
                        a[g][3] = v1.y;
                    } else {
                        const float4v v = *reinterpret_cast<const FE_GLOBAL float4v *>(val + e);
                        a[g][0] = double(v.x);
                        a[g][1] = double(v.y);
                        a[g][2] = double(v.z);
                        a[g][3] = double(v.w);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const bool ok = e + j < end;
                        c[g][j] = ok ? colind[e + j] : 0;
                        a[g][j] = ok ? double(val[e + j]) : 0.0;
                    }
                }
            }
#pragma unroll
            for (int g = 0; g < kTileGroups; g++) {
                const int64_t e = p0 + 4 * (tid + kTileThreads * g);
                double pr[4];
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const bool in = e + j >= base && e + j < end;
                    pr[j] = in ? a[g][j] * x[c[g][j]] : 0.0;
                }
                reinterpret_cast<fe_dpair *>(prod)[2 * (tid + kTileThreads * g)] = fe_dpair{pr[0], pr[1]};
                reinterpret_cast<fe_dpair *>(prod)[2 * (tid + kTileThreads * g) + 1] = fe_dpair{pr[2], pr[3]};
            }
            __syncthreads();
            const int64_t s1 = re < p0 + kTileCap ? re : p0 + kTileCap;
            for (int64_t j = (rb > p0 ? rb : p0) + sub; j < s1; j += LPR) acc += prod[j - p0];
            __syncthreads();
        }
        acc = butterfly<LPR>(acc);
        if (lr < nr && sub == 0) f(r0 + lr, acc);
    }
}

// Dispatch on the plan (mode, rows per wave-iteration) at compile time.
#define FE_PLAN_CASE(M, R, N, BODY) { constexpr int kMode = M, kRpb = R, kNc = N; (void)kNc; BODY; } break;
#define FE_PLAN_DISPATCH(PL, BODY)                                 \
    do {                                                           \
        if ((PL).mode == 1) {                                      \
            constexpr int kMode = 1, kRpb = 1, kNc = 1;            \
            BODY;                                                  \
        } else if ((PL).mode == 9) {                               \
            switch ((PL).rpb) {                                    \
                case 256: FE_PLAN_CASE(9, 256, 1, BODY)            \
                case 128: FE_PLAN_CASE(9, 128, 1, BODY)            \
                case 64: FE_PLAN_CASE(9, 64, 1, BODY)              \
                case 32: FE_PLAN_CASE(9, 32, 1, BODY)              \
                case 16: FE_PLAN_CASE(9, 16, 1, BODY)              \
                case 8: FE_PLAN_CASE(9, 8, 1, BODY)                \
                default: FE_PLAN_CASE(9, 4, 1, BODY)               \
            }                                                      \
        } else {                                                   \
            switch ((PL).rpb) {                                    \
                case 32: FE_PLAN_CASE(0, 32, 1, BODY)              \
                case 16: FE_PLAN_CASE(0, 16, 1, BODY)              \
                case 8: FE_PLAN_CASE(0, 8, 1, BODY)                \
                case 4: FE_PLAN_CASE(0, 4, 1, BODY)                \
                case 2: FE_PLAN_CASE(0, 2, 1, BODY)                \
                default: FE_PLAN_CASE(0, 1, 1, BODY)               \
            }                                                      \
        }                                                          \
    } while (0)


// Rows of a system assembled on a structured brick, with the pattern
// evaluated instead of read.  Row (free node (t0, t1, t2), component c) has
// the columns of the node box [cl, cl + w) per axis, all components, in
// lexicographic order; its values start at the closed-form position of the
// scatter.  Position p of the row decodes as p = ((j2 w1 + j1) w0 + j0) NC + cc
// and its column is NC rank(cl + j) + cc.  Nothing but the values and x is
// loaded, so a lane's loads wait on no other load.
// RPW rows per wave step, LW = 64 / RPW lanes per row, two runs of four
// positions per lane in flight.  A wave takes its runs in batches of LW
// (64 rows): each lane
// evaluates the geometry of one row of the batch, and the lanes of a row
// receive it by shuffles.  Each row is summed in lane order (positions sub,
// sub + LW, ... per lane, then a butterfly over the LW lanes).
template <int RPW, int NC, typename Fn>
__device__ __forceinline__ void for_rows_struct(const SpaceArgs &s, const double *__restrict__ gval,
                                                const double *__restrict__ gx, int64_t lb, int64_t nb, Fn f)
{
    const FE_GLOBAL double *__restrict__ val = as_global(gval);
    const FE_GLOBAL double *__restrict__ x = as_global(gx);
    constexpr int LW = 64 / RPW;
    const int lane = threadIdx.x % 64, g = lane / LW, sub = lane % LW;
    const int64_t n = s.n_rows;
    const int64_t nw = nb * kWaves, lw = lb * kWaves + threadIdx.x / 64;
    const int64_t runs = (n + RPW - 1) / RPW;
    const int32_t k = s.k;
    const double kinv = 1.0 / double(k);
    AxisClosed A[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
        A[r].lo = int32_t(s.ax[r].lo);
        A[r].hi = int32_t(s.ax[r].lo + s.ax[r].f - 1);
        A[r].N = int32_t(s.ax[r].N);
        A[r].swlo = A[r].lo * (k + 1) + k * ((A[r].lo + k - 1) / k);
    }
    const int32_t f0 = int32_t(s.ax[0].f), f1 = int32_t(s.ax[1].f);
    const double f0inv = 1.0 / double(f0), f1inv = 1.0 / double(f1);
    const int64_t T0 = s.ax[0].T, T1 = s.ax[1].T;
    const int32_t sy = NC * f0, sz = NC * f0 * f1;  // column steps of one node in y / in z
    for (int64_t b0 = lw; b0 < runs; b0 += int64_t(LW) * nw) {
        // geometry of row (run b0 + (lane / RPW) nw, lane % RPW) in this lane
        int32_t gstart_lo = 0, gstart_hi = 0, gcol = 0, gshape = 0, glen = 0;
        {
            const int64_t row = (b0 + int64_t(lane / RPW) * nw) * RPW + lane % RPW;
            if (row < n) {
                const int32_t r32 = int32_t(row);
                const int32_t R = r32 / NC, c = r32 - R * NC;
                const int32_t q = div_exact(R, f0, f0inv), t0 = R - q * f0;
                const int32_t t2 = div_exact(q, f1, f1inv), t1 = q - t2 * f1;
                int32_t w0, w1, w2, cl0, cl1, cl2, P0, P1, P2;
                axis_row(A[0], k, kinv, A[0].lo + t0, w0, cl0, P0);
                axis_row(A[1], k, kinv, A[1].lo + t1, w1, cl1, P1);
                axis_row(A[2], k, kinv, A[2].lo + t2, w2, cl2, P2);
                const int64_t S = int64_t(P2) * T1 * T0 + int64_t(w2) * P1 * T0 + int64_t(w2 * w1) * P0;
                const int32_t wx = w0 * NC;
                glen = wx * w1 * w2;
                const int64_t start = int64_t(NC) * NC * S + int64_t(c) * glen;
                gstart_lo = int32_t(uint32_t(uint64_t(start)));
                gstart_hi = int32_t(uint32_t(uint64_t(start) >> 32));
                gcol = NC * ((cl0 - A[0].lo) + f0 * ((cl1 - A[1].lo) + f1 * (cl2 - A[2].lo)));
                gshape = wx | (w1 << 16);
            }
        }
        // two runs per step: eight positions per lane in flight
        for (int u = 0; u < LW; u += 2) {
            if (b0 + int64_t(u) * nw >= runs) break;
            int64_t start[2], row[2];
            int32_t len[2], colbase[2], wx[2], w1[2];
            uint32_t mx[2], my[2];
            double sum[2];
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const int src = (u + h) * RPW + g;
                row[h] = (b0 + int64_t(u + h) * nw) * RPW + g;
                len[h] = __shfl(glen, src);
                colbase[h] = __shfl(gcol, src);
                const int32_t shape = __shfl(gshape, src);
                start[h] = int64_t((uint64_t(uint32_t(__shfl(gstart_hi, src))) << 32) |
                                   uint64_t(uint32_t(__shfl(gstart_lo, src))));
                const bool live = row[h] < n;
                wx[h] = live ? (shape & 0xffff) : 1;
                w1[h] = live ? (shape >> 16) : 1;
                if (!live) len[h] = 0;
                // floor(p / d) = (p m) >> 20 for m in [2^20 / d, 2^20 / d + 8]: exact for
                // p < 2^12, d <= 27 (the approximate reciprocal is within 1e-6 relative)
                mx[h] = uint32_t(1048576.0f * __builtin_amdgcn_rcpf(float(wx[h]))) + 2u;
                my[h] = uint32_t(1048576.0f * __builtin_amdgcn_rcpf(float(w1[h]))) + 2u;
                sum[h] = 0.0;
            }
            auto chunk = [&](int h, int32_t p0, double (&a4)[4], double (&x4)[4]) {
#pragma unroll
                for (int t = 0; t < 4; t++) {
                    const int32_t pos = p0 + sub + t * LW;
                    const bool ok = pos < len[h];
                    const int32_t pc = ok ? pos : 0;
                    const int32_t qy = int32_t((uint32_t(pc) * mx[h]) >> 20);
                    const int32_t xx = pc - qy * wx[h];
                    const int32_t j2 = int32_t((uint32_t(qy) * my[h]) >> 20);
                    const int32_t j1 = qy - j2 * w1[h];
                    a4[t] = ok ? val[start[h] + pc] : 0.0;
                    x4[t] = x[colbase[h] + xx + sy * j1 + sz * j2];
                }
            };
            {
                double a0[4], x0[4], a1[4], x1[4];
                chunk(0, 0, a0, x0);
                chunk(1, 0, a1, x1);
#pragma unroll
                for (int t = 0; t < 4; t++) sum[0] += a0[t] * x0[t];
#pragma unroll
                for (int t = 0; t < 4; t++) sum[1] += a1[t] * x1[t];
            }
#pragma unroll
            for (int h = 0; h < 2; h++) {
                for (int32_t p0 = 4 * LW; p0 < len[h]; p0 += 4 * LW) {
                    double a4[4], x4[4];
                    chunk(h, p0, a4, x4);
#pragma unroll
                    for (int t = 0; t < 4; t++) sum[h] += a4[t] * x4[t];
                }
            }
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const double t = butterfly<LW>(sum[h]);
                if (row[h] < n && sub == 0) f(row[h], t);
            }
        }
    }
}

// Short rows (at most LMAX <= 32 entries): 32 rows per wave step and two
// lanes per row (lane l holds row l % 32 and the positions
// [h H, h H + H) of it, h = l / 32, H = (LMAX + 1) / 2).  The values of the
// step's rows, contiguous in CSR, are loaded with coalesced loads into the
// wave's LDS slice; the x loads of neighbouring rows at the same position are
// neighbours in memory, so they coalesce too.  A row is the sum of its two
// half sums, each taken in position order.
template <int LMAX, int NC, typename Fn>
__device__ __forceinline__ void for_rows_short(const SpaceArgs &s, const double *__restrict__ gval,
                                               const double *__restrict__ gx, int64_t lb, int64_t nb, Fn f)
{
    const FE_GLOBAL double *__restrict__ val = as_global(gval);
    const FE_GLOBAL double *__restrict__ x = as_global(gx);
    constexpr int RW = 32, H = (LMAX + 1) / 2, CAP = RW * LMAX, CH = (CAP + 63) / 64;
    __shared__ double stage[kWaves][CAP];
    double *my = stage[threadIdx.x / 64];
    const int lane = threadIdx.x % 64, rl = lane % RW, h = lane / RW;
    const int64_t n = s.n_rows;
    const int64_t nw = nb * kWaves, lw = lb * kWaves + threadIdx.x / 64;
    const int64_t runs = (n + RW - 1) / RW;
    const int32_t k = s.k;
    const double kinv = 1.0 / double(k);
    AxisClosed A[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
        A[r].lo = int32_t(s.ax[r].lo);
        A[r].hi = int32_t(s.ax[r].lo + s.ax[r].f - 1);
        A[r].N = int32_t(s.ax[r].N);
        A[r].swlo = A[r].lo * (k + 1) + k * ((A[r].lo + k - 1) / k);
    }
    const int32_t f0 = int32_t(s.ax[0].f), f1 = int32_t(s.ax[1].f);
    const double f0inv = 1.0 / double(f0), f1inv = 1.0 / double(f1);
    const int64_t T0 = s.ax[0].T, T1 = s.ax[1].T;
    const int32_t sy = NC * f0, sz = NC * f0 * f1;
    for (int64_t run = lw; run < runs; run += nw) {
        const int64_t row = run * RW + rl;
        const bool live = row < n;
        int64_t start = 0;
        int32_t len = 0, colbase = 0, wx = 1, w1 = 1;
        if (live) {
            const int32_t r32 = int32_t(row);
            const int32_t R = r32 / NC, c = r32 - R * NC;
            const int32_t q = div_exact(R, f0, f0inv), t0 = R - q * f0;
            const int32_t t2 = div_exact(q, f1, f1inv), t1 = q - t2 * f1;
            int32_t w0, w2, cl0, cl1, cl2, P0, P1, P2;
            axis_row(A[0], k, kinv, A[0].lo + t0, w0, cl0, P0);
            axis_row(A[1], k, kinv, A[1].lo + t1, w1, cl1, P1);
            axis_row(A[2], k, kinv, A[2].lo + t2, w2, cl2, P2);
            const int64_t S = int64_t(P2) * T1 * T0 + int64_t(w2) * P1 * T0 + int64_t(w2 * w1) * P0;
            wx = w0 * NC;
            len = wx * w1 * w2;
            start = int64_t(NC) * NC * S + int64_t(c) * len;
            colbase = NC * ((cl0 - A[0].lo) + f0 * ((cl1 - A[1].lo) + f1 * (cl2 - A[2].lo)));
        }
        const int nv = int(n - run * RW < RW ? n - run * RW : RW);
        const int64_t base = __shfl(start, 0);
        const int total = int(__shfl(start, nv - 1) - base) + __shfl(len, nv - 1);
        {
            double t4[CH];
#pragma unroll
            for (int u = 0; u < CH; u++) {
                const int t = lane + 64 * u;
                t4[u] = t < total ? val[base + t] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < CH; u++)
                if (lane + 64 * u < CAP) my[lane + 64 * u] = t4[u];
        }
        wave_lds_sync();
        // floor(p / d) = (p m) >> 20 for m in [2^20 / d, 2^20 / d + 8] (p < 32, d <= 27)
        const uint32_t mx = uint32_t(1048576.0f * __builtin_amdgcn_rcpf(float(wx))) + 2u;
        const uint32_t my1 = uint32_t(1048576.0f * __builtin_amdgcn_rcpf(float(w1))) + 2u;
        const int off = int(start - base);
        double a[H], xv[H];
#pragma unroll
        for (int t = 0; t < H; t++) {
            const int32_t pos = h * H + t;
            const bool ok = pos < len;
            const int32_t pc = ok ? pos : 0;
            const int32_t qy = int32_t((uint32_t(pc) * mx) >> 20);
            const int32_t xx = pc - qy * wx;
            const int32_t j2 = int32_t((uint32_t(qy) * my1) >> 20);
            const int32_t j1 = qy - j2 * w1;
            xv[t] = x[colbase + xx + sy * j1 + sz * j2];
            a[t] = ok ? my[off + pc] : 0.0;
        }
        double sum = 0.0;
#pragma unroll
        for (int t = 0; t < H; t++) sum += a[t] * xv[t];
        const double upper = __shfl(sum, (lane + RW) % 64);
        if (h == 0 && live) f(row, sum + upper);
        wave_lds_sync();
    }
}

// Rows of the lowest-order scalar pattern (Q1, one component; longest row
// 3^d): row r couples the free nodes of the 3^d box around its node, so its
// columns are r + dx + f0 dy + f0 f1 dz for the offsets d in {-1, 0, 1}^d that
// stay in the free range.  A wave step takes 32 consecutive rows.  Their
// values, contiguous in CSR, are loaded with 16-byte loads into the wave's LDS
// slice, and every entry of x they touch lies in 3^(d-1) runs of 34
// consecutive unknowns (the rows' own line of nodes and its neighbour lines in
// y and z, widened by one node each side), which are loaded into LDS too: a
// 3D step issues 7 + 5 wide loads instead of one load per entry.  Two lanes
// per row sum the two halves of its positions in position order and the row
// is lower half + upper half, the order of the short-row traversal, so both
// give bitwise the same products.  f(row, A_row . x), or f(row, A_row . x,
// x[row]) when f takes three arguments.  Blocks of kQ1Block threads.  Plan mode 4;
// mode 5 is its instantiation with one step per wave, used whenever the
// partial slots cover that many blocks.
constexpr int kQ1Block = 256, kQ1Waves = kQ1Block / 64;


template <int DIM>
struct Q1Step {
    static constexpr int L = DIM == 3 ? 27 : 9;  // longest row
    static constexpr int RW = 32;                // rows per wave step
    static constexpr int H = (L + 1) / 2;        // positions per lane
    static constexpr int CAP = RW * L;           // most values of a step
    static constexpr int PCAP = CAP / 2 + 1;     // 16-byte slots (the step may start at an odd index)
    static constexpr int PCH = (PCAP + 63) / 64;
    static constexpr int SEG = RW + 2;           // unknowns of one run of x
    static constexpr int NSEG = DIM == 3 ? 9 : 3;
    static constexpr int XS = NSEG * SEG;
    static constexpr int XCH = (XS + 63) / 64;
};

template <int DIM, bool ONE, typename Fn>
__device__ __forceinline__ void for_rows_q1(const SpaceArgs &s, const double *__restrict__ gval,
                                            const double *__restrict__ gx, int64_t lb, int64_t nb, Fn f)
{
    using S = Q1Step<DIM>;
    const FE_GLOBAL double *__restrict__ val = as_global(gval);
    const FE_GLOBAL double *__restrict__ x = as_global(gx);
    __shared__ __align__(16) double vst[kQ1Waves][2 * S::PCAP];
    __shared__ double xst[kQ1Waves][S::XS];
    double *mv = vst[threadIdx.x / 64];
    double *mx = xst[threadIdx.x / 64];
    const int lane = threadIdx.x % 64, rl = lane % S::RW, h = lane / S::RW;
    const int64_t n = s.n_rows;
    const int64_t nw = nb * kQ1Waves, lw = lb * kQ1Waves + threadIdx.x / 64;
    const int64_t runs = (n + S::RW - 1) / S::RW;
    AxisClosed A[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
        A[r].lo = int32_t(s.ax[r].lo);
        A[r].hi = int32_t(s.ax[r].lo + s.ax[r].f - 1);
        A[r].N = int32_t(s.ax[r].N);
        A[r].swlo = A[r].lo * 2 + A[r].lo;  // unclipped widths below lo (k = 1)
    }
    const int32_t f0 = int32_t(s.ax[0].f), f1 = int32_t(s.ax[1].f);
    const double f0inv = s.ax[0].finv, f1inv = s.ax[1].finv;
    const int64_t T0 = s.ax[0].T, T1 = s.ax[1].T;
    auto step = [&](int64_t run) {
        const int64_t r0 = run * S::RW, row = r0 + rl;
        const bool live = row < n;
        int64_t start = 0;
        int32_t len = 0, wx = 1, w1 = 1, e0 = 0, e1 = 0, e2 = 0;
        if (live) {
            const int32_t r32 = int32_t(row);
            const int32_t q = div_exact(r32, f0, f0inv), t0 = r32 - q * f0;
            const int32_t t2 = div_exact(q, f1, f1inv), t1 = q - t2 * f1;
            int32_t w0, w2, cl0, cl1, cl2, P0, P1, P2;
            axis_row(A[0], 1, 1.0, A[0].lo + t0, w0, cl0, P0);
            axis_row(A[1], 1, 1.0, A[1].lo + t1, w1, cl1, P1);
            axis_row(A[2], 1, 1.0, A[2].lo + t2, w2, cl2, P2);
            start = int64_t(P2) * T1 * T0 + int64_t(w2) * P1 * T0 + int64_t(w2 * w1) * P0;
            wx = w0;
            len = w0 * w1 * w2;
            // slot of the first column along each axis: offset of the box's low end + 1
            e0 = cl0 - (A[0].lo + t0) + 1;
            e1 = cl1 - (A[1].lo + t1) + 1;
            e2 = DIM == 3 ? cl2 - (A[2].lo + t2) + 1 : 0;
        }
        const int nv = int(n - r0 < S::RW ? n - r0 : S::RW);
        const int64_t base = __shfl(start, 0);
        const int total = int(__shfl(start, nv - 1) - base) + __shfl(len, nv - 1);
        double xs[S::XCH];
#pragma unroll
        for (int u = 0; u < S::XCH; u++) {
            // slot i: unknown r0 - 1 + kk + f0 dy + f0 f1 dz of run (dy, dz)
            const int i = lane + 64 * u;
            const int sg = i / S::SEG, kk = i - sg * S::SEG;
            const int dy = sg % 3 - 1, dz = sg / 3 - 1;
            int64_t a = r0 + kk - 1 + dy * f0 + (DIM == 3 ? int64_t(dz) * f0 * f1 : 0);
            a = a < 0 ? 0 : (a >= n ? n - 1 : a);  // slots past either end are never read
            xs[u] = x[a];
        }
        // values [base, base + total) from the even index at or below base
        const int64_t abase = base & ~int64_t(1);
        const int lead = int(base - abase), tot = lead + total;
        fe_dpair vv[S::PCH];
#pragma unroll
        for (int u = 0; u < S::PCH; u++) {
            const int i = lane + 64 * u;
            const int64_t e = abase + 2 * int64_t(i);
            if (2 * i + 1 < tot) vv[u] = *reinterpret_cast<const FE_GLOBAL fe_dpair *>(val + e);
            else if (2 * i < tot) vv[u] = fe_dpair{val[e], 0.0};
            else vv[u] = fe_dpair{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < S::XCH; u++)
            if (lane + 64 * u < S::XS) mx[lane + 64 * u] = xs[u];
#pragma unroll
        for (int u = 0; u < S::PCH; u++)
            if (lane + 64 * u < S::PCAP) reinterpret_cast<fe_dpair *>(mv)[lane + 64 * u] = vv[u];
        wave_lds_sync();
        // floor(p / d) = (p m) >> 20 for m in [2^20 / d, 2^20 / d + 8] (p < 32, d <= 3)
        const uint32_t m0 = uint32_t(1048576.0f * __builtin_amdgcn_rcpf(float(wx))) + 2u;
        const uint32_t m1 = uint32_t(1048576.0f * __builtin_amdgcn_rcpf(float(w1))) + 2u;
        const int off = int(start - base) + lead;
        double sum = 0.0;
#pragma unroll
        for (int t = 0; t < S::H; t++) {
            const int32_t pos = h * S::H + t;
            const bool ok = pos < len;
            const int32_t pc = ok ? pos : 0;
            const int32_t qy = int32_t((uint32_t(pc) * m0) >> 20);
            const int32_t j0 = pc - qy * wx;
            const int32_t j2 = int32_t((uint32_t(qy) * m1) >> 20);
            const int32_t j1 = qy - j2 * w1;
            const int32_t sg = DIM == 3 ? (e1 + j1) + 3 * (e2 + j2) : e1 + j1;
            sum += (ok ? mv[off + pc] : 0.0) * mx[sg * S::SEG + rl + e0 + j0];
        }
        const double upper = __shfl(sum, (lane + S::RW) % 64);
        // x[row] sits in the rows' own run (dy = dz = 0) at slot rl + 1
        if (h == 0 && live) {
            if constexpr (std::is_invocable_v<Fn, int64_t, double, double>)
                f(row, sum + upper, mx[(DIM == 3 ? 4 : 1) * S::SEG + rl + 1]);
            else
                f(row, sum + upper);
        }
        wave_lds_sync();
    };
    // ONE: the grid has a wave per step (a loop-free body keeps four waves
    // per SIMD without spills); else wave-strided steps
    if constexpr (ONE) {
        if (lw < runs) step(lw);
    } else {
        for (int64_t run = lw; run < runs; run += nw) step(run);
    }
}

// Symmetric storage of a Q1 scalar system (the paper's option of keeping
// only the upper triangle of a symmetric matrix): with g(d) = 9 (dz + 1) +
// 3 (dy + 1) + (dx + 1) the code of a neighbour offset, the columns of a row
// in ascending order are the offsets in ascending g, and those with g >= C
// (C = 13, or 4 in 2D; C is the row's own node) form the upper triangle.
// Slot s = g - C of row r holds A[r, r + off(d)] at sym[s * stride + r]
// (slot-major, stride = n rounded up to 64; slot 0 is the diagonal, an entry
// whose neighbour is not free holds 0 and is never read).  A lower entry
// A[r, r + off(d)], g < C, is the upper entry of row r + off(d) at slot C - g.
constexpr int sym_slots(int dim) { return dim == 3 ? 14 : 5; }
__host__ __device__ constexpr int64_t sym_stride(int64_t n) { return (n + 63) / 64 * 64; }

// Rows of a Q1 scalar system in symmetric storage (plan mode 7; mode 8 is
// its instantiation with one step per wave).  A wave step takes 64
// consecutive rows, one lane per row; x is staged in LDS as 3^(d-1) runs of
// 66 unknowns (as in the Q1 traversal, one run per neighbour line), loaded
// straight into LDS in the one-step form.  The value
// of the neighbour with code g sits at the row plus an offset that depends on
// g only (slot |g - C|, and the mirrored row for g < C), so each lane walks the
// 3^d codes with a mask of the free ones (per axis, the offsets inside the
// row's box) and issues all its value loads at once, with no position decode:
// for a code shared by the rows of a step the 64 loads are consecutive.  The
// row's columns in ascending order are its free codes in ascending order; the
// first H = (3^d + 1) / 2 are summed into one partial, the rest into another,
// and the row is their sum: the order in which the two-lane Q1 traversal sums
// a row, so both give bitwise the same row sums of a symmetric matrix.
template <int DIM, bool ONE, typename VT, typename Fn>
__device__ __forceinline__ void for_rows_q1sym(const SpaceArgs &s, const VT *__restrict__ gval,
                                               const double *__restrict__ gx, int64_t lb, int64_t nb, Fn f)
{
    constexpr int L = DIM == 3 ? 27 : 9, H = (L + 1) / 2, C = (L - 1) / 2;
    // x runs staged from the even index at or below their start (16-byte pairs):
    // SEG2 = 68 slots per run, the run's first unknown at slot lead (0 or 1)
    constexpr int RW = 64, SEG = RW + 2, NSEG = DIM == 3 ? 9 : 3, SEG2 = SEG + 2, NP = SEG2 / 2;
    constexpr int XS = NSEG * SEG2, XCH = (NSEG * NP + 63) / 64;
    const FE_GLOBAL VT *__restrict__ val = as_global(gval);
    const FE_GLOBAL char *__restrict__ vbase = wave_base(gval);
    const FE_GLOBAL double *__restrict__ x = as_global(gx);
    __shared__ __align__(16) double xst[kQ1Waves][XS];
    double *mx = xst[threadIdx.x / 64];
    const int lane = threadIdx.x % 64;
    const int64_t n = s.n_rows, ns = sym_stride(n);
    const int64_t nw = nb * kQ1Waves, lw = lb * kQ1Waves + threadIdx.x / 64;
    const int64_t runs = (n + RW - 1) / RW;
    AxisClosed A[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
        A[r].lo = int32_t(s.ax[r].lo);
        A[r].hi = int32_t(s.ax[r].lo + s.ax[r].f - 1);
        A[r].N = int32_t(s.ax[r].N);
        A[r].swlo = A[r].lo * 2 + A[r].lo;
    }
    const int32_t f0 = int32_t(s.ax[0].f), f1 = int32_t(s.ax[1].f);
    const double f0inv = s.ax[0].finv, f1inv = s.ax[1].finv;
    const int64_t plane = int64_t(f0) * f1;
    auto step = [&](int64_t run) {
        const int64_t r0 = run * RW, row = r0 + lane;
        const bool live = row < n;
        // slot of run sg's first unknown: 1 when it starts at an odd index
        auto lead = [&](int sgi) {
            const int dy = sgi % 3 - 1, dz = sgi / 3 - 1;
            return int((r0 - 1 + dy * f0 + (DIM == 3 ? dz * plane : 0)) & 1);
        };
        // allowed neighbour offsets o of the row per axis: bit o + 1 (none for a row past n)
        uint32_t mk0 = 0, mk1 = 0, mk2 = 0;
        if (live) {
            const int32_t r32 = int32_t(row);
            const int32_t q = div_exact(r32, f0, f0inv), t0 = r32 - q * f0;
            const int32_t t2 = div_exact(q, f1, f1inv), t1 = q - t2 * f1;
            int32_t w0, w1, w2, cl0, cl1, cl2, P0, P1, P2;
            axis_row(A[0], 1, 1.0, A[0].lo + t0, w0, cl0, P0);
            axis_row(A[1], 1, 1.0, A[1].lo + t1, w1, cl1, P1);
            axis_row(A[2], 1, 1.0, A[2].lo + t2, w2, cl2, P2);
            mk0 = ((1u << w0) - 1u) << (cl0 - (A[0].lo + t0) + 1);
            mk1 = ((1u << w1) - 1u) << (cl1 - (A[1].lo + t1) + 1);
            mk2 = DIM == 3 ? ((1u << w2) - 1u) << (cl2 - (A[2].lo + t2) + 1) : 2u;
        }
        const bool xw = pair_aligned(gx);
        // One-step form with x 16-byte aligned: each lane's pair goes from
        // memory straight to LDS (a load-to-LDS instruction writes lane l's 16
        // bytes at the wave's LDS base + 16 l, which is pair slot 64 u + l), so
        // no registers are held for x across the value loads (82 instead of 96
        // VGPRs).  A pair that would run past the vector's end (the last
        // unknown starting a pair, or a clamped lane) is written by the lane.
        const bool dma = ONE && xw;
        if (dma) {
#pragma unroll
            for (int u = 0; u < XCH; u++) {
                const int i = lane + 64 * u;
                if (i < NSEG * NP) {
                    const int sg = i / NP, kk = 2 * (i - sg * NP);
                    const int dy = sg % 3 - 1, dz = sg / 3 - 1;
                    const int64_t st = r0 - 1 + dy * f0 + (DIM == 3 ? dz * plane : 0);
                    int64_t a = (st & ~int64_t(1)) + kk;
                    a = a < 0 ? 0 : a;
                    if (a + 1 < n) {
                        __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void *)(x + a),
                                                         (__attribute__((address_space(3))) void *)(mx + 128 * u), 16,
                                                         0, 0);
                    } else {
                        const int64_t bb = a < n ? a : n - 1;
                        reinterpret_cast<fe_dpair *>(mx)[i] = fe_dpair{x[bb], x[bb]};
                    }
                }
            }
        }
        fe_dpair xs[XCH];
#pragma unroll
        for (int u = 0; u < XCH && !dma; u++) {
            const int i = lane + 64 * u;  // pair i of the staged runs
            const int sg = i / NP, kk = 2 * (i - sg * NP);
            const int dy = sg % 3 - 1, dz = sg / 3 - 1;
            const int64_t st = r0 - 1 + dy * f0 + (DIM == 3 ? dz * plane : 0);
            int64_t a = (st & ~int64_t(1)) + kk;
            // pairs past either end (and lanes past the staged pairs) are never
            // read: clamped into the vector; the last unknown may start a pair
            a = a < 0 ? 0 : a;
            if (xw && a + 1 < n) {
                xs[u] = *reinterpret_cast<const FE_GLOBAL fe_dpair *>(x + a);
            } else {
                const int64_t b = a < n ? a : n - 1, c = a + 1 < n ? a + 1 : n - 1;
                xs[u] = fe_dpair{x[b], x[c]};
            }
        }
        // code g = 9 (o2 + 1) + 3 (o1 + 1) + (o0 + 1): the value of a free
        // neighbour is the row plus an offset common to the wave
        auto code_ok = [&](int g) {
            const int o0 = g % 3 - 1, o1 = (g / 3) % 3 - 1, o2 = DIM == 3 ? g / 9 - 1 : 0;
            return ((mk0 >> (o0 + 1)) & (mk1 >> (o1 + 1)) & (mk2 >> (o2 + 1)) & 1u) != 0u;
        };
        if (ONE && !dma) {
            // x only 8-byte aligned: staged through registers before the value loads
#pragma unroll
            for (int u = 0; u < XCH; u++)
                if (lane + 64 * u < NSEG * NP) reinterpret_cast<fe_dpair *>(mx)[lane + 64 * u] = xs[u];
        }
        // kept in the storage's type until the product: a conversion at the load
        // would wait for each load in turn
        VT vv[L];
#pragma unroll
        for (int g = 0; g < L; g++) {
            const int o0 = g % 3 - 1, o1 = (g / 3) % 3 - 1, o2 = DIM == 3 ? g / 9 - 1 : 0;
            const int64_t k = g >= C ? int64_t(g - C) * ns
                                     : int64_t(C - g) * ns + o0 + int64_t(o1) * f0 + int64_t(o2) * plane;
            if constexpr (ONE) {
                // one step per wave (at most 8.4 M rows): byte offsets fit in 32 bits
                const uint32_t boff = uint32_t(row + k) * uint32_t(sizeof(VT));
                if constexpr (sizeof(VT) == 4) {
                    // FP32 storage: loaded unconditionally (a lane whose code is not
                    // free reads its own diagonal, in range for every lane of the step;
                    // the sums skip it), or the widening to FP64 is folded into a
                    // conditional load and waits for each load in turn
                    vv[g] = *reinterpret_cast<const FE_GLOBAL VT *>(vbase + (code_ok(g) ? boff : uint32_t(row) * 4u));
                } else {
                    vv[g] = code_ok(g) ? *reinterpret_cast<const FE_GLOBAL VT *>(vbase + boff) : VT(0);
                }
            } else {
                vv[g] = code_ok(g) ? val[row + k] : VT(0);
            }
        }
        if (!ONE) {
#pragma unroll
            for (int u = 0; u < XCH; u++)
                if (lane + 64 * u < NSEG * NP) reinterpret_cast<fe_dpair *>(mx)[lane + 64 * u] = xs[u];
        }
        // the load-to-LDS writes complete with the vector memory counter, which
        // the compiler does not wait on before LDS reads: wait for it here
        // (immediate 0x0F70: vmcnt 0, expcnt and lgkmcnt not waited on)
        if (dma) __builtin_amdgcn_s_waitcnt(0x0F70);
        wave_lds_sync();
        // the row's columns in ascending order are its free codes in ascending
        // order: the first H go to lo, the rest to hi
        double lo = 0.0, hi = 0.0;
        int c = 0;
#pragma unroll
        for (int g = 0; g < L; g++) {
            const int o0 = g % 3 - 1, o1 = (g / 3) % 3 - 1, o2 = DIM == 3 ? g / 9 - 1 : 0;
            const int sgi = DIM == 3 ? (o1 + 1) + 3 * (o2 + 1) : o1 + 1;
            const double xg = mx[sgi * SEG2 + lead(sgi) + o0 + 1 + lane];
            if (code_ok(g)) {
                if (c < H) lo += double(vv[g]) * xg;
                else hi += double(vv[g]) * xg;
                c++;
            }
        }
        if (live) {
            if constexpr (std::is_invocable_v<Fn, int64_t, double, double>)
                f(row, lo + hi, mx[(DIM == 3 ? 4 : 1) * SEG2 + lead(DIM == 3 ? 4 : 1) + lane + 1]);
            else
                f(row, lo + hi);
        }
        wave_lds_sync();
    };
    if constexpr (ONE) {
        if (lw < runs) step(lw);
    } else {
        for (int64_t run = lw; run < runs; run += nw) step(run);
    }
}

// sym = the upper triangle of a Q1 scalar system assembled on the mesh, in the
// symmetric storage above.  A wave takes 32 consecutive rows (of the slot
// stride): their values, contiguous in CSR, are loaded into LDS with
// coalesced loads; then each half-wave writes half of the slots, one row per
// lane (rows past n and neighbours that are not free get 0).
template <int DIM, typename OT>
__global__ __launch_bounds__(kQ1Block) void sym_fill_kernel(SpaceArgs s, const double *__restrict__ gval,
                                                            OT *__restrict__ gsym)
{
    using S = Q1Step<DIM>;
    constexpr int C = DIM == 3 ? 13 : 4, NS = C + 1, SH = (NS + 1) / 2;
    const FE_GLOBAL double *__restrict__ val = as_global(gval);
    FE_GLOBAL OT *__restrict__ sym = as_global(gsym);
    __shared__ double vst[kQ1Waves][S::CAP];
    double *mv = vst[threadIdx.x / 64];
    const int lane = threadIdx.x % 64, rl = lane % S::RW, h = lane / S::RW;
    const int64_t n = s.n_rows, ns = sym_stride(n);
    const int64_t run = int64_t(blockIdx.x) * kQ1Waves + threadIdx.x / 64;
    const int64_t r0 = run * S::RW, row = r0 + rl;
    if (r0 >= ns) return;
    AxisClosed A[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
        A[r].lo = int32_t(s.ax[r].lo);
        A[r].hi = int32_t(s.ax[r].lo + s.ax[r].f - 1);
        A[r].N = int32_t(s.ax[r].N);
        A[r].swlo = A[r].lo * 2 + A[r].lo;
    }
    const int32_t f0 = int32_t(s.ax[0].f), f1 = int32_t(s.ax[1].f);
    const int64_t T0 = s.ax[0].T, T1 = s.ax[1].T;
    const bool live = row < n;
    int64_t start = 0;
    int32_t len = 0, w[3] = {1, 1, 1}, e[3] = {0, 0, 0};
    if (live) {
        const int32_t r32 = int32_t(row);
        const int32_t q = r32 / f0, t0 = r32 - q * f0;
        const int32_t t2 = q / f1, t1 = q - t2 * f1;
        int32_t cl[3], P[3];
        axis_row(A[0], 1, 1.0, A[0].lo + t0, w[0], cl[0], P[0]);
        axis_row(A[1], 1, 1.0, A[1].lo + t1, w[1], cl[1], P[1]);
        axis_row(A[2], 1, 1.0, A[2].lo + t2, w[2], cl[2], P[2]);
        start = int64_t(P[2]) * T1 * T0 + int64_t(w[2]) * P[1] * T0 + int64_t(w[2] * w[1]) * P[0];
        len = w[0] * w[1] * w[2];
        e[0] = cl[0] - (A[0].lo + t0) + 1;
        e[1] = cl[1] - (A[1].lo + t1) + 1;
        e[2] = DIM == 3 ? cl[2] - (A[2].lo + t2) + 1 : 0;
    }
    const int nv = int(n - r0 <= 0 ? 0 : (n - r0 < S::RW ? n - r0 : S::RW));
    int64_t base = 0;
    int total = 0;
    if (nv > 0) {
        base = __shfl(start, 0);
        total = int(__shfl(start, nv - 1) - base) + __shfl(len, nv - 1);
    }
#pragma unroll
    for (int u = 0; u < (S::CAP + 63) / 64; u++) {
        const int i = lane + 64 * u;
        if (i < total) mv[i] = val[base + i];
    }
    wave_lds_sync();
    const int off = int(start - base);
#pragma unroll
    for (int t = 0; t < SH; t++) {
        const int sl = h * SH + t;
        if (sl >= NS) continue;
        const int g = C + sl;
        const int32_t o0 = g % 3 - 1, o1 = (g / 3) % 3 - 1, o2 = DIM == 3 ? g / 9 - 1 : 0;
        const int32_t j0 = o0 + 1 - e[0], j1 = o1 + 1 - e[1], j2 = DIM == 3 ? o2 + 1 - e[2] : 0;
        const bool ok = live && j0 >= 0 && j0 < w[0] && j1 >= 0 && j1 < w[1] && j2 >= 0 && j2 < w[2];
        sym[sl * ns + row] = OT(ok ? mv[off + (j2 * w[1] + j1) * w[0] + j0] : 0.0);
    }
}

// Rows of any evaluated pattern, x staged per block (plan mode 6).  A block
// takes a chunk of kXbRows consecutive rows of one line of nodes (t1, t2
// fixed): their column boxes share the y and z ranges, and their x ranges lie
// in the union [cl0(first node), cl0(last node) + w0(last node)).  The block
// loads x over that box -- w1 w2 runs of NC (xb - xa) consecutive unknowns,
// coalesced -- into LDS once; then each wave sums eight rows, eight lanes per
// row, values read from memory and x from LDS, in the order of the
// lanes-per-row traversal with eight rows per wave (bitwise the same
// products).  Chunks never cross a line of nodes.
constexpr int kXbRows = 32;   // rows per chunk: 4 waves x 8 rows
constexpr int kXbCap = 4864;  // staged doubles: (2k+1)^2 runs of NC (nodes of a chunk + 2k), k <= 4

// The staged box of a chunk: its kXbRows rows cover at most (kXbRows - 1) / NC + 2
// nodes of the line (a chunk may start inside a node's components), whose
// column boxes along x reach k nodes beyond each end, and (2k + 1)^2 node
// lines across; every supported component count and order must fit.
constexpr int xblock_staged_max(int nc, int k) { return nc * ((kXbRows - 1) / nc + 2 + 2 * k) * (2 * k + 1) * (2 * k + 1); }
static_assert(xblock_staged_max(1, 4) <= kXbCap && xblock_staged_max(2, 4) <= kXbCap &&
                  xblock_staged_max(3, 4) <= kXbCap,
              "the staged x box of a mode-6 chunk exceeds its LDS buffer");

template <int NC, typename VT, typename Fn>
__device__ __forceinline__ void for_rows_xblock(const SpaceArgs &s, const VT *__restrict__ gval,
                                                const double *__restrict__ gx, int64_t lb, int64_t nb, Fn f)
{
    constexpr int RPW = 8, LW = 64 / RPW;
    __shared__ double sx[kXbCap];
    const FE_GLOBAL VT *__restrict__ val = as_global(gval);
    const FE_GLOBAL double *__restrict__ x = as_global(gx);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, g = lane / LW, sub = lane % LW;
    const int32_t k = s.k;
    const double kinv = 1.0 / double(k);
    AxisClosed A[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
        A[r].lo = int32_t(s.ax[r].lo);
        A[r].hi = int32_t(s.ax[r].lo + s.ax[r].f - 1);
        A[r].N = int32_t(s.ax[r].N);
        A[r].swlo = A[r].lo * (k + 1) + k * ((A[r].lo + k - 1) / k);
    }
    const int32_t f0 = int32_t(s.ax[0].f), f1 = int32_t(s.ax[1].f);
    const int64_t T0 = s.ax[0].T, T1 = s.ax[1].T;
    const int64_t rpl = int64_t(NC) * f0;                      // rows per line of nodes
    const int64_t cpl = (rpl + kXbRows - 1) / kXbRows;         // chunks per line
    const int64_t nchunks = int64_t(f1) * s.ax[2].f * cpl;
    for (int64_t ch = lb; ch < nchunks; ch += nb) {
        const int64_t line = ch / cpl, q = ch - line * cpl;
        const int32_t t1 = int32_t(line % f1), t2 = int32_t(line / f1);
        const int64_t lr0 = q * kXbRows;                        // first row of the chunk within its line
        const int64_t lr1 = lr0 + kXbRows < rpl ? lr0 + kXbRows : rpl;
        int32_t wa, cla, Pa, wb, clb, Pb, w1, cl1, P1, w2, cl2, P2;
        axis_row(A[0], k, kinv, A[0].lo + int32_t(lr0 / NC), wa, cla, Pa);
        axis_row(A[0], k, kinv, A[0].lo + int32_t((lr1 - 1) / NC), wb, clb, Pb);
        axis_row(A[1], k, kinv, A[1].lo + t1, w1, cl1, P1);
        axis_row(A[2], k, kinv, A[2].lo + t2, w2, cl2, P2);
        const int32_t xa = cla, run = NC * (clb + wb - cla);    // staged nodes [xa, xb) along x
        const int32_t nst = run * w1 * w2;
        __syncthreads();  // the previous chunk's reads of sx are done
        for (int e = threadIdx.x; e < nst; e += 256) {
            const int rr = e / run, i = e - rr * run;
            const int jz = rr / w1, jy = rr - jz * w1;
            const int64_t col = int64_t(NC) * ((xa - A[0].lo) + int64_t(f0) * ((cl1 + jy - A[1].lo) +
                                                                               int64_t(f1) * (cl2 + jz - A[2].lo))) + i;
            sx[e] = x[col];
        }
        __syncthreads();
        const int64_t lrow = lr0 + RPW * wave + g;
        const bool live = lrow < lr1;
        const int64_t row = line * rpl + lrow;
        double sum = 0.0;
        if (live) {
            const int32_t t0 = int32_t(lrow / NC), c = int32_t(lrow - int64_t(t0) * NC);
            int32_t w0, cl0, P0;
            axis_row(A[0], k, kinv, A[0].lo + t0, w0, cl0, P0);
            const int64_t S = int64_t(P2) * T1 * T0 + int64_t(w2) * P1 * T0 + int64_t(w2 * w1) * P0;
            const int32_t wx = w0 * NC, len = wx * w1 * w2;
            const int64_t start = int64_t(NC) * NC * S + int64_t(c) * len;
            const int32_t xoff = NC * (cl0 - xa);
            // floor(p / d) = (p m) >> 20 for m in [2^20 / d, 2^20 / d + 8] (p < 2^12, d <= 27)
            const uint32_t mx = uint32_t(1048576.0f * __builtin_amdgcn_rcpf(float(wx))) + 2u;
            const uint32_t my = uint32_t(1048576.0f * __builtin_amdgcn_rcpf(float(w1))) + 2u;
            for (int32_t p0 = 0; p0 < len; p0 += 4 * LW) {
                double a4[4], x4[4];
#pragma unroll
                for (int t = 0; t < 4; t++) {
                    const int32_t pos = p0 + sub + t * LW;
                    const bool ok = pos < len;
                    const int32_t pc = ok ? pos : 0;
                    const int32_t qy = int32_t((uint32_t(pc) * mx) >> 20);
                    const int32_t xx = pc - qy * wx;
                    const int32_t j2 = int32_t((uint32_t(qy) * my) >> 20);
                    const int32_t j1 = qy - j2 * w1;
                    // pc = 0 is in the row: an unconditional load, so an FP32 value's widening
                    // does not make each load wait for the one before
                    const VT raw = val[start + pc];
                    a4[t] = ok ? double(raw) : 0.0;
                    x4[t] = sx[(j2 * w1 + j1) * run + xoff + xx];
                }
#pragma unroll
                for (int t = 0; t < 4; t++) sum += a4[t] * x4[t];
            }
        }
        const double t = butterfly<LW>(sum);
        if (live && sub == 0) f(row, t);
    }
}

// Dispatch on the plan at compile time: kMode, kRpb (rows per wave) and kNc
// (components, structured mode only).  FE_PLAN_DISPATCH_ALL adds the
// structured plans (FP64 values only).
#define FE_SPLAN_DISPATCH(PL, BODY)                                                            \
    switch ((PL).mode * 1000 + (PL).nc * 100 + (PL).rpb) {                                     \
        case 8127: FE_PLAN_CASE(8, 27, 1, BODY)                                                \
        case 8109: FE_PLAN_CASE(8, 9, 1, BODY)                                                 \
        case 7127: FE_PLAN_CASE(7, 27, 1, BODY)                                                \
        case 7109: FE_PLAN_CASE(7, 9, 1, BODY)                                                 \
        case 6108: FE_PLAN_CASE(6, 8, 1, BODY)                                                 \
        case 6208: FE_PLAN_CASE(6, 8, 2, BODY)                                                 \
        case 6308: FE_PLAN_CASE(6, 8, 3, BODY)                                                 \
        case 5127: FE_PLAN_CASE(5, 27, 1, BODY)                                                \
        case 5109: FE_PLAN_CASE(5, 9, 1, BODY)                                                 \
        case 4127: FE_PLAN_CASE(4, 27, 1, BODY)                                                \
        case 4109: FE_PLAN_CASE(4, 9, 1, BODY)                                                 \
        case 3127: FE_PLAN_CASE(3, 27, 1, BODY)                                                \
        case 3109: FE_PLAN_CASE(3, 9, 1, BODY)                                                 \
        case 3125: FE_PLAN_CASE(3, 25, 1, BODY)                                                \
        case 3218: FE_PLAN_CASE(3, 18, 2, BODY)                                                \
        case 2116: FE_PLAN_CASE(2, 16, 1, BODY)                                                 \
        case 2108: FE_PLAN_CASE(2, 8, 1, BODY)                                                  \
        case 2104: FE_PLAN_CASE(2, 4, 1, BODY)                                                  \
        case 2102: FE_PLAN_CASE(2, 2, 1, BODY)                                                  \
        case 2101: FE_PLAN_CASE(2, 1, 1, BODY)                                                  \
        case 2208: FE_PLAN_CASE(2, 8, 2, BODY)                                                  \
        case 2204: FE_PLAN_CASE(2, 4, 2, BODY)                                                  \
        case 2202: FE_PLAN_CASE(2, 2, 2, BODY)                                                  \
        case 2201: FE_PLAN_CASE(2, 1, 2, BODY)                                                  \
        case 2308: FE_PLAN_CASE(2, 8, 3, BODY)                                                 \
        case 2304: FE_PLAN_CASE(2, 4, 3, BODY)                                                 \
        case 2302: FE_PLAN_CASE(2, 2, 3, BODY)                                                 \
        default: FE_PLAN_CASE(2, 1, 3, BODY)                                                   \
    }
// Plans of FP32 values: the CSR plans and the symmetric-storage ones
#define FE_SYM_DISPATCH(PL, BODY)                                                              \
    switch ((PL).mode * 1000 + (PL).rpb) {                                                     \
        case 8027: FE_PLAN_CASE(8, 27, 1, BODY)                                                \
        case 8009: FE_PLAN_CASE(8, 9, 1, BODY)                                                 \
        case 7027: FE_PLAN_CASE(7, 27, 1, BODY)                                                \
        default: FE_PLAN_CASE(7, 9, 1, BODY)                                                   \
    }
#define FE_PLAN_DISPATCH_FP32(PL, BODY)                                                        \
    do {                                                                                       \
        if ((PL).mode == 7 || (PL).mode == 8) {                                                \
            FE_SYM_DISPATCH(PL, BODY)                                                          \
        } else if ((PL).mode == 6) {                                                           \
            switch ((PL).nc) {                                                                 \
                case 1: FE_PLAN_CASE(6, 8, 1, BODY)                                            \
                case 2: FE_PLAN_CASE(6, 8, 2, BODY)                                            \
                default: FE_PLAN_CASE(6, 8, 3, BODY)                                           \
            }                                                                                  \
        } else {                                                                               \
            FE_PLAN_DISPATCH(PL, BODY);                                                        \
        }                                                                                      \
    } while (0)
// DG systems: kRpb = nodes per cell, kNc = dimension
#define FE_DG_DISPATCH(PL, BODY)                                                               \
    switch ((PL).nc * 1000 + (PL).rpb) {                                                       \
        case 3008: FE_PLAN_CASE(10, 8, 3, BODY)                                                \
        case 3027: FE_PLAN_CASE(10, 27, 3, BODY)                                               \
        case 3064: FE_PLAN_CASE(10, 64, 3, BODY)                                               \
        case 3125: FE_PLAN_CASE(10, 125, 3, BODY)                                              \
        case 2004: FE_PLAN_CASE(10, 4, 2, BODY)                                                \
        case 2009: FE_PLAN_CASE(10, 9, 2, BODY)                                                \
        case 2016: FE_PLAN_CASE(10, 16, 2, BODY)                                               \
        default: FE_PLAN_CASE(10, 25, 2, BODY)                                                 \
    }
#define FE_PLAN_DISPATCH_ALL(PL, BODY)                                                         \
    do {                                                                                       \
        if ((PL).mode == 10) {                                                                 \
            FE_DG_DISPATCH(PL, BODY)                                                           \
        } else if ((PL).mode >= 2 && (PL).mode <= 8) {                                         \
            FE_SPLAN_DISPATCH(PL, BODY)                                                        \
        } else {                                                                               \
            FE_PLAN_DISPATCH(PL, BODY);                                                        \
        }                                                                                      \
    } while (0)

// Row class of the evaluated-pattern traversal: (longest row, components).
static int struct_class(const SpaceArgs &sa)
{
    int L = sa.ncomp;
    for (int r = 0; r < sa.dim; r++) L *= 2 * sa.k + 1;
    return L * 4 + sa.ncomp;
}

static std::map<int, SpmvPlan> g_stuned;  // evaluated-pattern plans measured by the autotuner

// The plan of an evaluated-pattern system: the autotuned one of its class,
// else short rows (at most 32 entries, instantiated lengths) two lanes per
// row, longer rows eight rows per wave step.
static SpmvPlan struct_plan_of_class(const SpaceArgs &sa)
{
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_stuned.find(struct_class(sa));
        if (it != g_stuned.end()) return it->second;
    }
    int L = sa.ncomp;
    for (int r = 0; r < sa.dim; r++) L *= 2 * sa.k + 1;
    SpmvPlan pl{};
    pl.nc = sa.ncomp;
    // the Q1 scalar pattern: values and the touched runs of x staged in LDS
    if (sa.ncomp == 1 && sa.k == 1) {
        pl.mode = 4;
        pl.rpb = L;
        pl.lanes = 2;
        return pl;
    }
    // rows of at most 32 entries with an instantiated length: two lanes per row
    if ((sa.ncomp == 1 && (L == 27 || L == 9 || L == 25)) || (sa.ncomp == 2 && L == 18)) {
        pl.mode = 3;
        pl.rpb = L;
        pl.lanes = 2;
        return pl;
    }
    // vector patterns and order 4: x of each 32-row chunk staged per block
    // (measured on 2.6-4.0 M-row systems: elasticity Q2 / Q3 / Q4 996 / 1769 /
    // 2889 us against 1033 / 1850 / 3080 us for the best lanes-per-row plan,
    // scalar Q4 1910 against 2073 us)
    if (sa.ncomp >= 2 || sa.k >= 4) {
        pl.mode = 6;
        pl.rpb = 8;
        pl.lanes = 8;
        return pl;
    }
    // scalar Q2-Q3: eight rows per wave step (8 lanes per row, the rest of a
    // long row in further steps of 32 positions), measured fastest (the
    // block-staged plan: 415 / 925 us against 358 / 862 us)
    pl.mode = 2;
    pl.rpb = 8;
    pl.lanes = 8;
    return pl;
}

// The launch form of a plan: mode 4 (7) becomes its one-step-per-wave
// instantiation, mode 5 (8), when the partial slots hold a block per 128
// (256) rows.
static SpmvPlan launch_form(SpmvPlan pl, int64_t n)
{
    if (pl.mode == 4 && (n + 127) / 128 <= part_slots(n)) pl.mode = 5;
    if (pl.mode == 7 && ((n + 255) / 256 + 7) / 8 * 8 <= part_slots(n)) pl.mode = 8;
    return pl;
}

// The plan an evaluated-pattern system is launched with.
static SpmvPlan struct_plan(const SpaceArgs &sa) { return launch_form(struct_plan_of_class(sa), sa.n_rows); }

// Modes 4 and 5 stage the values with 16-byte loads from 16-byte boundaries
// of the array; values not 16-byte aligned take mode 3, the same summation
// order without wide loads.
static SpmvPlan aligned_form(SpmvPlan pl, const void *values)
{
    if ((reinterpret_cast<uintptr_t>(values) & 15u) == 0) return pl;
    if (pl.mode == 4 || pl.mode == 5) return SpmvPlan{3, pl.nc, pl.rpb, 2};
    return pl;
}

// Rows of an interior-penalty DG system on the brick (plan mode 10), the
// pattern evaluated from the cell index: the nn rows of cell K are
// contiguous in the values, rlen = nc nn entries each (the nn columns of each
// cell of K's row block, cells ascending), starting at nn^2 times the prefix
// of block sizes over the cells before K.  Only the values and x are read.
// The block tiles of the CSR traversal (mode 9) with a cell as the tile: the
// block stages the x entries of K's row block in LDS, streams the cell's
// values in passes of kTileCap with 16-byte loads, stages the products in
// LDS (the column of an entry is its offset in its row, one division per four
// entries), and LPR lanes of each row sum its staged entries in lane order,
// then a butterfly.  Cells are dealt XCD-contiguously as tiles are in mode 9.
template <int DIM, int NN, typename Fn>
__device__ __forceinline__ void for_rows_dg(const SpaceArgs &s, const double *__restrict__ gval,
                                            const double *__restrict__ gx, int64_t lb, int64_t nb, Fn f)
{
    const FE_GLOBAL double *__restrict__ val = as_global(gval);
    const FE_GLOBAL double *__restrict__ x = as_global(gx);
    constexpr int RMAX = (2 * DIM + 1) * NN;  // longest row
    constexpr int LPR = NN <= 8 ? 32 : (NN <= 16 ? 16 : (NN <= 32 ? 8 : (NN <= 64 ? 4 : 2)));  // LPR NN <= 256
    static_assert(LPR * NN <= kTileThreads, "lanes per row");
    __shared__ double prod[kTileCap];
    __shared__ double xs[RMAX];
    const int tid = threadIdx.x, lr = tid / LPR, sub = tid % LPR;
    const int32_t n0 = int32_t(s.ax[0].n), n1 = int32_t(s.ax[1].n), n2 = DIM == 3 ? int32_t(s.ax[2].n) : 1;
    const int32_t nr[3] = {n0, n1, n2}, st[3] = {1, n0, n0 * n1};
    const int64_t ncells = s.ncells, nnz = s.nnz;
    const int64_t xcd = lb % 8, per = nb / 8;
    const int64_t c_hi = (xcd + 1) * ncells / 8;
    for (int64_t K64 = xcd * ncells / 8 + lb / 8; K64 < c_hi; K64 += per) {
        const int32_t K = int32_t(K64);
        // coordinates, block size and the prefix of block sizes (32-bit: fewer than 2^31 rows)
        int32_t c[3], prefix = (2 * DIM + 1) * K, nc = 1;
#pragma unroll
        for (int r = 0; r < DIM; r++) {
            const int32_t P = st[r] * nr[r], q = K / P, rem = K - q * P;
            c[r] = rem / st[r];
            const int32_t lo = min(max(rem, 0), st[r]), hi = min(max(rem - (nr[r] - 1) * st[r], 0), st[r]);
            prefix -= 2 * q * st[r] + lo + hi;
            nc += (c[r] > 0) + (c[r] < nr[r] - 1);
        }
        const int32_t rlen = nc * NN;
        const int64_t base = int64_t(NN) * NN * prefix, end = base + int64_t(NN) * rlen;
        __syncthreads();  // the previous cell's reads of xs and prod are done
        // x of the block's cells (slot j: lower neighbours far axis first, K, upper neighbours)
        for (int t = tid; t < rlen; t += kTileThreads) {
            int j = t / NN;
            int32_t cell = -1;
#pragma unroll
            for (int r = DIM - 1; r >= 0; r--)
                if (c[r] > 0 && j-- == 0) cell = K - st[r];
            if (cell < 0 && j-- == 0) cell = K;
#pragma unroll
            for (int r = 0; r < DIM; r++)
                if (cell < 0 && c[r] < nr[r] - 1 && j-- == 0) cell = K + st[r];
            xs[t] = x[int64_t(cell) * NN + t % NN];
        }
        __syncthreads();
        const int64_t rb = lr < NN ? base + int64_t(lr) * rlen : end, re = lr < NN ? rb + rlen : end;
        const float rinv = 1.0f / float(rlen);
        double acc = 0.0;
        for (int64_t p0 = base & ~int64_t(3); p0 < end; p0 += kTileCap) {
            double a[kTileGroups][4];
#pragma unroll
            for (int g = 0; g < kTileGroups; g++) {
                const int64_t e = p0 + 4 * (tid + kTileThreads * g);
                if (e < end && e + 4 <= nnz) {
                    const fe_dpair v0 = *reinterpret_cast<const FE_GLOBAL fe_dpair *>(val + e);
                    const fe_dpair v1 = *reinterpret_cast<const FE_GLOBAL fe_dpair *>(val + e + 2);
                    a[g][0] = v0.x;
                    a[g][1] = v0.y;
                    a[g][2] = v1.x;
                    a[g][3] = v1.y;
                } else {
#pragma unroll
                    for (int j = 0; j < 4; j++) a[g][j] = e + j < end ? val[e + j] : 0.0;
                }
            }
#pragma unroll
            for (int g = 0; g < kTileGroups; g++) {
                const int64_t e = p0 + 4 * (tid + kTileThreads * g);
                // column of entry e within its row: (e - base) mod rlen (a lead before base is masked)
                const int32_t pos = int32_t(e - base);
                int32_t q = int32_t(float(pos) * rinv);
                int32_t col = pos - q * rlen;
                if (col < 0) col += rlen;
                if (col >= rlen) col -= rlen;
                double pr[4];
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const bool in = e + j >= base && e + j < end;
                    pr[j] = in ? a[g][j] * xs[col] : 0.0;
                    col = col + 1 == rlen ? 0 : col + 1;
                }
                reinterpret_cast<fe_dpair *>(prod)[2 * (tid + kTileThreads * g)] = fe_dpair{pr[0], pr[1]};
                reinterpret_cast<fe_dpair *>(prod)[2 * (tid + kTileThreads * g) + 1] = fe_dpair{pr[2], pr[3]};
            }
            __syncthreads();
            const int64_t s1 = re < p0 + kTileCap ? re : p0 + kTileCap;
            for (int64_t j = (rb > p0 ? rb : p0) + sub; j < s1; j += LPR) acc += prod[j - p0];
            __syncthreads();
        }
        acc = butterfly<LPR>(acc);
        if (lr < NN && sub == 0) f(K64 * NN + lr, acc);
    }
}

template <int MODE, int RPW, typename VT, typename Fn>
__device__ __forceinline__ void for_rows(int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *colind,
                                         const VT *val, const double *x, int64_t lb, int64_t nb, Fn f)
{
    if constexpr (MODE == 9)
        for_rows_tiles<RPW, VT>(n, nnz, rowptr, colind, val, x, lb, nb, f);
    else if constexpr (MODE == 1)
        for_rows_wave(n, rowptr, colind, val, x, lb, nb, f);
    else
        for_rows_wstream<RPW, VT>(n, rowptr, colind, val, x, lb, nb, f);
}

// Row traversal of one problem of a PCG table.
template <int MODE, int RPB, int NC, typename VT, typename Fn>
__device__ __forceinline__ void for_rows_p(const PcgProb &P, const double *x, int64_t lb, int64_t nb, Fn f)
{
    if constexpr (MODE == 10)
        for_rows_dg<NC, RPB>(P.sa, static_cast<const double *>(P.val), x, lb, nb, f);
    else if constexpr (MODE == 7 || MODE == 8)
        for_rows_q1sym<RPB == 27 ? 3 : 2, MODE == 8>(P.sa, static_cast<const VT *>(P.val), x, lb, nb, f);
    else if constexpr (MODE == 6)
        for_rows_xblock<NC, VT>(P.sa, static_cast<const VT *>(P.val), x, lb, nb, f);
    else if constexpr (MODE == 4 || MODE == 5)
        for_rows_q1<RPB == 27 ? 3 : 2, MODE == 5>(P.sa, static_cast<const double *>(P.val), x, lb, nb, f);
    else if constexpr (MODE == 3)
        for_rows_short<RPB, NC>(P.sa, static_cast<const double *>(P.val), x, lb, nb, f);
    else if constexpr (MODE == 2)
        for_rows_struct<RPB, NC>(P.sa, static_cast<const double *>(P.val), x, lb, nb, f);
    else
        for_rows<MODE, RPB, VT>(P.n, P.nnz, P.rowptr, P.colind, static_cast<const VT *>(P.val), x, lb, nb, f);
}

// Problem of block blockIdx.x in a launch whose problem p owns blocks
// [boff[p], boff[p+1]); returns the block's index within its problem.
__device__ __forceinline__ int find_problem(const int32_t *__restrict__ boff, int nprob, int64_t &lb, int64_t &nb)
{
    int lo = 0, hi = nprob;  // boff[lo] <= b < boff[hi]
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

// Block order of the symmetric Q1 traversal (modes 7, 8; nb a multiple of 8):
// workgroups are dealt to the eight XCDs in turn, so block b runs on XCD
// b mod 8; b takes the logical block (b mod 8) nb / 8 + b / 8, which gives each
// XCD one contiguous slab of rows, taken in ascending order.  A row's lower
// entries are read from rows up to a plane of nodes back, which its own XCD
// read as upper entries shortly before: they are served by that XCD's L2.
// The partial of a block goes to its logical slot, so the slots hold what the
// blocks of the unpermuted order hold (and blocks past the rows add zeros).
template <int MODE>
__device__ __forceinline__ int64_t xcd_block(int64_t lb, int64_t nb)
{
    if constexpr (MODE == 7 || MODE == 8) return (lb % 8) * (nb / 8) + lb / 8;
    else return lb;
}

// Vector access in pairs of neighbours: W, 16-byte loads and stores (every
// vector of the kernel 16-byte aligned, the kernel decides once per block),
// else one element at a time (a caller's vector only 8-byte aligned); m = 2,
// or 1 for the last, odd element of a range.

template <bool W>
__device__ __forceinline__ void load_pair(const double *__restrict__ ga, int64_t i, int m, double (&o)[2])
{
    const FE_GLOBAL double *__restrict__ a = as_global(ga);
    if (W && m == 2) {
        const fe_dpair t = *reinterpret_cast<const FE_GLOBAL fe_dpair *>(a + i);
        o[0] = t.x;
        o[1] = t.y;
    } else {
        o[0] = a[i];
        o[1] = m == 2 ? a[i + 1] : 0.0;
    }
}

template <bool W>
__device__ __forceinline__ void store_pair(double *__restrict__ ga, int64_t i, int m, const double (&v)[2])
{
    FE_GLOBAL double *__restrict__ a = as_global(ga);
    if (W && m == 2) {
        *reinterpret_cast<FE_GLOBAL fe_dpair *>(a + i) = fe_dpair{v[0], v[1]};
    } else {
        a[i] = v[0];
        if (m == 2) a[i + 1] = v[1];
    }
}

// body(std::true_type) when every pointer is 16-byte aligned, else
// body(std::false_type).
template <typename Body>
__device__ __forceinline__ void with_pair_width(bool aligned, Body body)
{
    if (aligned) body(std::true_type{});
    else body(std::false_type{});
}

// Visits the pairs (i, i + 1) of [lo, hi) (lo even) owned by this thread:
// body(i, m) issues the pair's loads and returns the work that uses them, so
// that the loads of two pairs are in flight before either pair's work runs.
// The visiting order, and so every partial sum, is fixed.
template <typename Body>
__device__ __forceinline__ void for_pairs(int64_t lo, int64_t hi, Body body)
{
    for (int64_t i0 = lo + 2 * int64_t(threadIdx.x); i0 < hi; i0 += 4 * int64_t(kBlock)) {
        const int64_t i1 = i0 + 2 * int64_t(kBlock);
        const int m0 = hi - i0 >= 2 ? 2 : 1;
        auto w0 = body(i0, m0);
        if (i1 < hi) {
            const int m1 = hi - i1 >= 2 ? 2 : 1;
            auto w1 = body(i1, m1);
            w0();
            w1();
        } else {
            w0();
        }
    }
}

// Elements [lo, hi) of logical block lb of nb for the vector kernels.
__device__ __forceinline__ void owned_elems(int64_t n, int64_t lb, int64_t nb, int64_t &lo, int64_t &hi)
{
    const int64_t per = ((n + nb - 1) / nb + 1) / 2 * 2;
    lo = std::min<int64_t>(lb * per, n);
    hi = std::min<int64_t>(lo + per, n);
}

// Threads per block of the row kernels of a plan mode.
constexpr int rows_block(int mode) { return mode >= 4 ? kQ1Block : kBlock; }

// ---------------------------------------------------------------------------
// Kernels (every one serves any number of problems: problem p owns the blocks
// [boff[p], boff[p+1]) of the launch)
// ---------------------------------------------------------------------------
template <int MODE, int RPB, typename VT>
__global__ __launch_bounds__(rows_block(MODE)) void spmv_kernel(int64_t n, int64_t nnz,
                                                                 const int64_t *__restrict__ rowptr,
                                                                 const int32_t *__restrict__ colind,
                                                                 const VT *__restrict__ val,
                                                                 const double *__restrict__ x, double *__restrict__ y)
{
    for_rows<MODE, RPB, VT>(n, nnz, rowptr, colind, val, x, blockIdx.x, gridDim.x,
                            [&](int64_t row, double s) { y[row] = s; });
}

template <int MODE, int RPB, int NC>
__global__ __launch_bounds__(rows_block(MODE)) void spmv_struct_kernel(SpaceArgs sa, const double *__restrict__ val,
                                                                        const double *__restrict__ x,
                                                                        double *__restrict__ y)
{
    if constexpr (MODE == 10)
        for_rows_dg<NC, RPB>(sa, val, x, xcd_block<MODE>(blockIdx.x, gridDim.x), gridDim.x,
                             [&](int64_t row, double s) { y[row] = s; });
    else if constexpr (MODE == 7 || MODE == 8)
        for_rows_q1sym<RPB == 27 ? 3 : 2, MODE == 8>(sa, val, x, xcd_block<MODE>(blockIdx.x, gridDim.x), gridDim.x,
                                                     [&](int64_t row, double s) { y[row] = s; });
    else if constexpr (MODE == 6)
        for_rows_xblock<NC, double>(sa, val, x, blockIdx.x, gridDim.x, [&](int64_t row, double s) { y[row] = s; });
    else if constexpr (MODE == 4 || MODE == 5)
        for_rows_q1<RPB == 27 ? 3 : 2, MODE == 5>(sa, val, x, blockIdx.x, gridDim.x,
                                                  [&](int64_t row, double s) { y[row] = s; });
    else if constexpr (MODE == 3)
        for_rows_short<RPB, NC>(sa, val, x, blockIdx.x, gridDim.x, [&](int64_t row, double s) { y[row] = s; });
    else
        for_rows_struct<RPB, NC>(sa, val, x, blockIdx.x, gridDim.x, [&](int64_t row, double s) { y[row] = s; });
}

// r = b - A x; p = z = dinv r; partials of r.z, r.r, b.b
template <int MODE, int RPB, int NC, typename VT>
__global__ __launch_bounds__(rows_block(MODE)) void pcg_init_kernel(const PcgProb *__restrict__ probs,
                                                           const int32_t *__restrict__ boff, int nprob)
{
    int64_t lb, nb;
    const PcgProb &P = probs[find_problem(boff, nprob, lb, nb)];
    lb = xcd_block<MODE>(lb, nb);
    double v[3] = {0.0, 0.0, 0.0};
    const FE_GLOBAL double *__restrict__ b = as_global(P.b);
    const FE_GLOBAL double *__restrict__ dinv = as_global(P.dinv);
    FE_GLOBAL double *__restrict__ r = as_global(P.w.r);
    FE_GLOBAL double *__restrict__ pv = as_global(P.w.p);
    for_rows_p<MODE, RPB, NC, VT>(P, P.x, lb, nb, [&](int64_t row, double ax) {
                                const double rr = b[row] - ax;
                                const double z = dinv[row] * rr;
                                r[row] = rr;
                                pv[row] = z;
                                v[0] += rr * z;
                                v[1] += rr * rr;
                                v[2] += b[row] * b[row];
                            });
    double t[3] = {v[0], v[1], v[2]};
    block_sum_all<3, rows_block(MODE)>(t);
    if (threadIdx.x == 0)
        for (int i = 0; i < 3; i++) P.w.p3[i * P.w.ps + lb] = t[i];
}

// one block per problem: initial scalars and stop test
__global__ __launch_bounds__(kBlock) void pcg_init_finish_kernel(const PcgProb *__restrict__ probs)
{
    const PcgProb &P = probs[blockIdx.x];
    double t[3];
    reduce_partials<3>(P.w.p3, P.nbr, P.w.ps, t);
    if (threadIdx.x == 0) {
        PcgState *st = P.w.st;
        st->rho[0] = t[0];
        st->rr = t[1];
        st->bb = t[2];
        st->iter = 0;
        st->iter_upd = 0;
        st->status = FE_OK;
        st->done = 0;
        st->stop_at = INT32_MAX;
        st->alpha = 0.0;
        if (t[1] <= P.rtol2 * t[2]) {
            st->done = 1;
        } else if (P.maxit <= 0) {
            st->done = 1;
            st->status = FE_ENOTCONV;
        }
    }
}

// q = A p; partials of p.q
template <int MODE, int RPB, int NC, typename VT>
__global__ __launch_bounds__(rows_block(MODE)) void pcg_spmv_kernel(const PcgProb *__restrict__ probs,
                                                           const int32_t *__restrict__ boff, int nprob)
{
    int64_t lb, nb;
    const PcgProb &P = probs[find_problem(boff, nprob, lb, nb)];
    if (pcg_stopped(*P.w.st, P.w.st->iter)) return;
    lb = xcd_block<MODE>(lb, nb);
    double v = 0.0;
    const FE_GLOBAL double *__restrict__ p = as_global(P.w.p);
    FE_GLOBAL double *__restrict__ q = as_global(P.w.q);
    // the Q1 traversals (modes 4, 5, 7, 8) hand over p[row] from their LDS copy of p
    for_rows_p<MODE, RPB, NC, VT>(P, P.w.p, lb, nb, [&](int64_t row, double s, double prow = 0.0) {
                                q[row] = s;
                                v += (MODE == 4 || MODE == 5 || MODE == 7 || MODE == 8 ? prow : p[row]) * s;
                            });
    // block partial: wave sums, then wave 0's lane 0 adds them in wave order
    __shared__ double wsum[rows_block(MODE) / 64];
    const double t = butterfly<64>(v);
    if (threadIdx.x % 64 == 0) wsum[threadIdx.x / 64] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double u = 0.0;
        for (int w = 0; w < rows_block(MODE) / 64; w++) u += wsum[w];
        as_global(P.w.p1)[lb] = u;
    }
}

// alpha = rho_j / p.q; r -= alpha q; partials of r.z, r.r (x += alpha p is
// left to the dir kernel, which reads p anyway)
__global__ __launch_bounds__(kBlock) void pcg_update_kernel(const PcgProb *__restrict__ probs,
                                                             const int32_t *__restrict__ boff, int nprob)
{
    int64_t lb, nb;
    const PcgProb &P = probs[find_problem(boff, nprob, lb, nb)];
    PcgState *st = P.w.st;
    const int j = st->iter;
    // the dir kernel's iteration, also when this one has stopped
    if (lb == 0 && threadIdx.x == 0) st->iter_upd = j;
    if (pcg_stopped(*st, j)) return;
    double pq[1];
    reduce_partials<1>(P.w.p1, P.nbr, P.w.ps, pq);
    if (!(pq[0] > 0.0) || !isfinite(pq[0])) {
        if (lb == 0 && threadIdx.x == 0) {
            st->done = 1;
            st->status = FE_EBREAKDOWN;
        }
        return;
    }
    const double alpha = st->rho[j & 1] / pq[0];
    if (lb == 0 && threadIdx.x == 0) {
        st->alpha = alpha;
        if (j < kHist) P.w.hist[j] = alpha;
    }
    int64_t lo, hi;
    owned_elems(P.n, lb, nb, lo, hi);
    double v[2] = {0.0, 0.0};
    const double *__restrict__ q = P.w.q;
    const double *__restrict__ dinv = P.dinv;
    double *__restrict__ r = P.w.r;
    // vectors of the caller (dinv) and of its workspace (q, r) may each be only 8-byte aligned
    with_pair_width(pair_aligned(dinv) && pair_aligned(q) && pair_aligned(r), [&](auto wide) {
        constexpr bool W = decltype(wide)::value;
        for_pairs(lo, hi, [&](int64_t i, int m) {
            double qq[2], rr[2], dd[2];
            load_pair<W>(q, i, m, qq);
            load_pair<W>(r, i, m, rr);
            load_pair<W>(dinv, i, m, dd);
            return [=, &v]() {
                double rn[2];
#pragma unroll
                for (int e = 0; e < 2; e++) {
                    // explicit fused operations: every instantiation rounds alike
                    rn[e] = fma(-alpha, qq[e], rr[e]);
                    if (e < m) {
                        v[0] = fma(rn[e], dd[e] * rn[e], v[0]);
                        v[1] = fma(rn[e], rn[e], v[1]);
                    }
                }
                store_pair<W>(r, i, m, rn);
            };
        });
    });
    block_sum_all<2>(v);
    if (threadIdx.x == 0) {
        P.w.p2[lb] = v[0];
        P.w.p2[kGrid + lb] = v[1];
    }
}

// beta = rho_{j+1} / rho_j; stop test; x += alpha_j p; p = z + beta p
__global__ __launch_bounds__(kBlock) void pcg_dir_kernel(const PcgProb *__restrict__ probs,
                                                          const int32_t *__restrict__ boff, int nprob)
{
    int64_t lb, nb;
    const PcgProb &P = probs[find_problem(boff, nprob, lb, nb)];
    PcgState *st = P.w.st;
    const int j = st->iter_upd;
    if (pcg_stopped(*st, j)) return;
    double t[2];
    reduce_partials<2>(P.w.p2, P.nbe, kGrid, t);
    const double rho_old = st->rho[j & 1];
    const double beta = t[0] / rho_old;
    const bool conv = t[1] <= P.rtol2 * st->bb;
    if (lb == 0 && threadIdx.x == 0) {
        st->rho[(j + 1) & 1] = t[0];
        st->rr = t[1];
        st->iter = j + 1;
        if (j < kHist) P.w.hist[kHist + j] = beta;
        // stop_at, not done: the other blocks of this kernel still read the solve as running
        if (conv) {
            st->stop_at = j;
            st->status = FE_OK;
        } else if (j + 1 >= P.maxit) {
            st->stop_at = j;
            st->status = FE_ENOTCONV;
        }
    }
    const double alpha = st->alpha;
    int64_t lo, hi;
    owned_elems(P.n, lb, nb, lo, hi);
    const double *__restrict__ r = P.w.r;
    const double *__restrict__ dinv = P.dinv;
    double *__restrict__ p = P.w.p;
    double *__restrict__ x = P.x;
    // vectors of the caller (x, dinv) and of its workspace (p, r) may each be only 8-byte aligned
    with_pair_width(pair_aligned(x) && pair_aligned(dinv) && pair_aligned(r) && pair_aligned(p), [&](auto wide) {
        constexpr bool W = decltype(wide)::value;
        if (conv) {  // the last x update; p is no longer needed
            for_pairs(lo, hi, [&](int64_t i, int m) {
                double pp[2], xx[2];
                load_pair<W>(p, i, m, pp);
                load_pair<W>(x, i, m, xx);
                return [=]() {
                    double xn[2];
#pragma unroll
                    for (int e = 0; e < 2; e++) xn[e] = fma(alpha, pp[e], xx[e]);
                    store_pair<W>(x, i, m, xn);
                };
            });
            return;
        }
        for_pairs(lo, hi, [&](int64_t i, int m) {
            double rr[2], dd[2], pp[2], xx[2];
            load_pair<W>(r, i, m, rr);
            load_pair<W>(dinv, i, m, dd);
            load_pair<W>(p, i, m, pp);
            load_pair<W>(x, i, m, xx);
            return [=]() {
                double pn[2], xn[2];
#pragma unroll
                for (int e = 0; e < 2; e++) {
                    // explicit fused operations: every instantiation rounds alike
                    xn[e] = fma(alpha, pp[e], xx[e]);
                    pn[e] = fma(beta, pp[e], dd[e] * rr[e]);
                }
                store_pair<W>(x, i, m, xn);
                store_pair<W>(p, i, m, pn);
            };
        });
    });
}

// partials of (b - A x)^2
template <int MODE, int RPB, int NC, typename VT>
__global__ __launch_bounds__(rows_block(MODE)) void resid_kernel(const PcgProb *__restrict__ probs,
                                                        const int32_t *__restrict__ boff, int nprob)
{
    int64_t lb, nb;
    const PcgProb &P = probs[find_problem(boff, nprob, lb, nb)];
    lb = xcd_block<MODE>(lb, nb);
    double v[1] = {0.0};
    const FE_GLOBAL double *__restrict__ b = as_global(P.b);
    for_rows_p<MODE, RPB, NC, VT>(P, P.x, lb, nb, [&](int64_t row, double ax) {
                                const double d = b[row] - ax;
                                v[0] += d * d;
                            });
    block_sum_all<1, rows_block(MODE)>(v);
    if (threadIdx.x == 0) P.w.p3[lb] = v[0];
}

__global__ __launch_bounds__(kBlock) void resid_finish_kernel(const PcgProb *__restrict__ probs)
{
    const PcgProb &P = probs[blockIdx.x];
    double t[1];
    reduce_partials<1>(P.w.p3, P.nbr, P.w.ps, t);
    if (threadIdx.x == 0) P.w.st->true_rr = t[0];
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int grid_rows(int64_t n, const SpmvPlan &pl)
{
    if (pl.mode == 10) {  // DG: a block per cell, at most one per partial slot; a multiple of 8 (XCD-contiguous cells)
        const int64_t ncells = n / pl.rpb;
        const int64_t cap = part_slots(n) / 8 * 8;
        return int((std::max<int64_t>(1, std::min<int64_t>(cap, ncells)) + 7) / 8 * 8);
    }
    if (pl.mode == 9) {  // a block per tile, at most one per partial slot; a multiple of 8 (XCD-contiguous tiles)
        const int64_t tiles = (n + pl.rpb - 1) / pl.rpb;
        const int64_t cap = part_slots(n) / 8 * 8;
        return int((std::max<int64_t>(1, std::min<int64_t>(cap, tiles)) + 7) / 8 * 8);
    }
    const int rows_per_run = pl.mode >= 7 ? 64 : pl.mode >= 3 ? 32 : pl.rpb;  // mode 6: a block per 32-row chunk
    const int waves = pl.mode == 6 ? 1 : rows_block(pl.mode) / 64;
    const int64_t runs = (n + rows_per_run - 1) / rows_per_run;
    // the Q1 traversals: up to one block per partial slot (modes 5 and 8:
    // exactly one wave per step); the others: at most kGrid blocks
    const int64_t cap = pl.mode == 4 || pl.mode == 5 || pl.mode >= 7 ? part_slots(n) : kGrid;
    const int64_t g = std::max<int64_t>(1, std::min<int64_t>(cap, (runs + waves - 1) / waves));
    // modes 7, 8: a multiple of the XCD count (cap is one), see xcd_block
    return int(pl.mode >= 7 ? (g + 7) / 8 * 8 : g);
}

// Blocks of the vector kernels of an n-row problem: at most kGridE, since
// every block of the update kernel re-reads all partials of the SpMV before
// its first vector access (256 blocks measured 4% faster per C2 iteration
// than 1024 with one SpMV partial per 128 rows).
static int grid_elems(int64_t n)
{
    return int(std::max<int64_t>(1, std::min<int64_t>(kGridE, (n + kBlock - 1) / kBlock)));
}

fe_status launch_spmv(int64_t n, const int64_t *rowptr, const int32_t *colind, const double *val, const double *x,
                      double *y, int64_t nnz, hipStream_t s)
{
    if (n == 0) return FE_OK;
    const SpmvPlan pl = csr_launch_form(plan_for(n, nnz), n, nnz, colind, val);
    const int g = grid_rows(n, pl);
    FE_PLAN_DISPATCH(pl, (spmv_kernel<kMode, kRpb, double><<<dim3(g), dim3(rows_block(kMode)), 0, s>>>(n, nnz,
                                             rowptr, colind, val, x, y)));
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

// ---------------------------------------------------------------------------
// SpMV autotuner: times every plan on a matrix and keeps the fastest for the
// matrix's row-length class.
// ---------------------------------------------------------------------------
// {mode, nc, rows per wave, lanes per row}
static const SpmvPlan kCandidates[] = {{0, 1, 1, 64},   {0, 1, 2, 32},  {0, 1, 4, 16},  {0, 1, 8, 8},
                                       {0, 1, 16, 4},   {0, 1, 32, 2},  {1, 1, 1, 64},  {9, 1, 256, 1},
                                       {9, 1, 128, 2},  {9, 1, 64, 4},  {9, 1, 32, 8},  {9, 1, 16, 16},
                                       {9, 1, 8, 32},   {9, 1, 4, 64}};

size_t autotune_ws_bytes(int64_t n) { return 2 * align256(size_t(std::max<int64_t>(n, 1)) * sizeof(double)); }

fe_status spmv_autotune(const fe_csr *A, int reps, void *ws, size_t ws_bytes, fe_spmv_plan *tried, int max_tried,
                        int *n_tried, fe_spmv_plan *chosen, hipStream_t s)
{
    const int64_t n = A->n_rows;
    if (ws_bytes < autotune_ws_bytes(n)) return set_error(FE_EINVAL, "autotune workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) & 7u) return set_error(FE_EINVAL, "workspace not 8-byte aligned");
    double *x = static_cast<double *>(ws);
    double *y = reinterpret_cast<double *>(static_cast<char *>(ws) + align256(size_t(std::max<int64_t>(n, 1)) * 8));
    if (n_tried) *n_tried = 0;
    if (n == 0) return set_error(FE_EINVAL, "empty matrix");
    FE_HIP(hipMemsetAsync(x, 0, sizeof(double) * size_t(n), s));
    hipEvent_t e0, e1;
    FE_HIP(hipEventCreate(&e0));
    FE_HIP(hipEventCreate(&e1));
    int best = -1;
    double best_us = 0.0;
    const int ncand = int(sizeof(kCandidates) / sizeof(kCandidates[0]));
    fe_status st = FE_OK;
    for (int c = 0; c < ncand && st == FE_OK; c++) {
        const SpmvPlan pl = csr_launch_form(kCandidates[c], n, A->nnz, A->colind, A->values);
        const int g = grid_rows(n, pl);
        for (int r = -1; r < reps; r++) {
            if (r == 0 && hipEventRecord(e0, s) != hipSuccess) st = set_error(FE_EDEVICE, "event record failed");
            FE_PLAN_DISPATCH(pl, (spmv_kernel<kMode, kRpb, double><<<dim3(g), dim3(rows_block(kMode)), 0, s>>>(
                                     n, A->nnz, A->rowptr, A->colind, A->values, x, y)));
        }
        if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess) {
            st = set_error(FE_EDEVICE, "autotune launch failed");
            break;
        }
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = set_error(FE_EDEVICE, "event timing failed");
            break;
        }
        const double us = 1000.0 * double(ms) / double(reps);
        if (tried && c < max_tried) tried[c] = fe_spmv_plan{pl.mode, pl.rpb, us};
        if (n_tried) *n_tried = std::min(c + 1, max_tried);
        if (best < 0 || us < best_us) {
            best = c;
            best_us = us;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FE_OK) return st;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[plan_class(n, A->nnz)] = kCandidates[best];
    }
    if (chosen) *chosen = fe_spmv_plan{kCandidates[best].mode, kCandidates[best].rpb, best_us};
    return FE_OK;
}

void spmv_tuning_reset()
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
    g_stuned.clear();
}

fe_status spmv_plan_set(int64_t n, int64_t nnz, const fe_spmv_plan &plan)
{
    for (const SpmvPlan &c : kCandidates)
        if (c.mode == plan.mode && c.rpb == plan.rows_per_wave) {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tuned[plan_class(n, nnz)] = c;
            return FE_OK;
        }
    return set_error(FE_EINVAL, "not a CSR plan the autotuner times");
}

void spmv_plan_of(int64_t n, int64_t nnz, fe_spmv_plan *plan, int32_t *cls)
{
    const SpmvPlan pl = plan_for(n, nnz);
    if (plan) *plan = fe_spmv_plan{pl.mode, pl.rpb, 0.0};
    if (cls) *cls = plan_class(n, nnz);
}

// Evaluated-pattern plans: every rows-per-wave of the lanes-per-row traversal
// instantiated for the component count, and the short-row traversal where it
// exists for the row length.
static std::vector<SpmvPlan> struct_candidates(const SpaceArgs &sa)
{
    int L = sa.ncomp;
    for (int r = 0; r < sa.dim; r++) L *= 2 * sa.k + 1;
    std::vector<SpmvPlan> c;
    const int nc = sa.ncomp;
    const std::vector<int> rpws = nc == 1 ? std::vector<int>{16, 8, 4, 2, 1}
                                          : std::vector<int>{8, 4, 2, 1};
    for (int r : rpws) c.push_back(SpmvPlan{2, nc, r, 64 / r});
    if ((nc == 1 && (L == 27 || L == 9 || L == 25)) || (nc == 2 && L == 18)) c.push_back(SpmvPlan{3, nc, L, 2});
    if (nc == 1 && sa.k == 1) c.push_back(SpmvPlan{4, nc, L, 2});
    else c.push_back(SpmvPlan{6, nc, 8, 8});
    return c;
}

fe_status spmv_autotune_struct(const SpaceArgs &sa, const double *values, int reps, void *ws, size_t ws_bytes,
                               fe_spmv_plan *tried, int max_tried, int *n_tried, fe_spmv_plan *chosen, hipStream_t s)
{
    const int64_t n = sa.n_rows;
    if (n_tried) *n_tried = 0;
    if (n == 0) return set_error(FE_EINVAL, "empty system");
    if (ws_bytes < autotune_ws_bytes(n)) return set_error(FE_EINVAL, "autotune workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) & 7u) return set_error(FE_EINVAL, "workspace not 8-byte aligned");
    double *x = static_cast<double *>(ws);
    double *y = reinterpret_cast<double *>(static_cast<char *>(ws) + align256(size_t(n) * 8));
    FE_HIP(hipMemsetAsync(x, 0, sizeof(double) * size_t(n), s));
    const std::vector<SpmvPlan> cand = struct_candidates(sa);
    hipEvent_t e0, e1;
    FE_HIP(hipEventCreate(&e0));
    FE_HIP(hipEventCreate(&e1));
    int best = -1;
    double best_us = 0.0;
    fe_status st = FE_OK;
    for (size_t c = 0; c < cand.size() && st == FE_OK; c++) {
        const SpmvPlan pl = aligned_form(launch_form(cand[c], n), values);
        const int g = grid_rows(n, pl);
        for (int r = -1; r < reps; r++) {
            if (r == 0 && hipEventRecord(e0, s) != hipSuccess) st = set_error(FE_EDEVICE, "event record failed");
            FE_SPLAN_DISPATCH(pl, (spmv_struct_kernel<kMode, kRpb, kNc><<<dim3(g), dim3(rows_block(kMode)), 0, s>>>(sa, values, x, y)));
        }
        float ms = 0.0f;
        if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = set_error(FE_EDEVICE, "autotune launch failed");
            break;
        }
        const double us = 1000.0 * double(ms) / double(reps);
        if (tried && int(c) < max_tried) tried[c] = fe_spmv_plan{cand[c].mode, cand[c].rpb, us};
        if (n_tried) *n_tried = std::min(int(c) + 1, max_tried);
        if (best < 0 || us < best_us) {
            best = int(c);
            best_us = us;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FE_OK) return st;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_stuned[struct_class(sa)] = cand[best];
    }
    if (chosen) *chosen = fe_spmv_plan{cand[best].mode, cand[best].rpb, best_us};
    return FE_OK;
}

fe_status spmv_plan_set_struct(const SpaceArgs &sa, const fe_spmv_plan &plan)
{
    for (const SpmvPlan &c : struct_candidates(sa))
        if (c.mode == plan.mode && c.rpb == plan.rows_per_wave) {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_stuned[struct_class(sa)] = c;
            return FE_OK;
        }
    return set_error(FE_EINVAL, "not a plan of this system's row class");
}

void spmv_plan_of_struct(const SpaceArgs &sa, fe_spmv_plan *plan, int32_t *cls)
{
    const SpmvPlan pl = struct_plan_of_class(sa);
    if (plan) *plan = fe_spmv_plan{pl.mode, pl.rpb, 0.0};
    if (cls) *cls = struct_class(sa);
}

// ---------------------------------------------------------------------------
// PCG engine: any number of problems solved together.  Problems are grouped
// by SpMV plan and value type (template parameters of the row kernels); the
// vector kernels serve all problems in one launch.  Chunks of iterations are
// launched directly or replayed from a captured HIP graph.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void count_active_kernel(const PcgProb *__restrict__ probs, int nprob,
                                                               int32_t *active)
{
    __shared__ int32_t cnt[kBlock];
    int32_t c = 0;
    for (int i = threadIdx.x; i < nprob; i += kBlock) c += pcg_stopped(*probs[i].w.st, probs[i].w.st->iter) ? 0 : 1;
    cnt[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int i = 0; i < kBlock; i++) t += cnt[i];
        *active = t;
    }
}

__global__ __launch_bounds__(kBlock) void gather_states_kernel(const PcgProb *__restrict__ probs, int nprob,
                                                                PcgState *out)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < nprob; i += gridDim.x * kBlock) out[i] = *probs[i].w.st;
}

size_t engine_table_bytes(int nprob)
{
    return align256(sizeof(PcgProb) * size_t(std::max(nprob, 1))) +
           align256(sizeof(int32_t) * (3 * size_t(nprob) + 16)) +
           align256(sizeof(PcgState) * size_t(std::max(nprob, 1))) + 256;
}

struct Group {
    SpmvPlan pl;
    bool fp32;
    int first, count;  // problems [first, first + count) of the sorted table
    int32_t *d_boff;   // count + 1 block offsets of the row kernels
    int grid;
};

// A set of problems launched together: the device table is sorted by (SpMV
// plan, value type) so that each row-kernel instantiation is one launch; the
// vector kernels cover the whole table in one launch.
struct EngineSet {
    std::vector<PcgJob> jobs;   // sorted like the table
    std::vector<PcgProb> hp;
    std::vector<int32_t> hi;
    std::vector<Group> groups;
    std::vector<PcgState> hs;
    int np = 0, ge = 0;
    PcgProb *d_probs = nullptr;
    int32_t *d_ints = nullptr;
    PcgState *d_states = nullptr;
    int32_t *d_active = nullptr;
};

EngineSet *engine_create() { return new EngineSet(); }
void engine_destroy(EngineSet *E) { delete E; }
int engine_size(const EngineSet &E) { return E.np; }
const PcgJob &engine_job(const EngineSet &E, int t) { return E.jobs[t]; }

#define FE_ROWS_KERNELS(DISPATCH, VT)                                                                                \
    switch (which) {                                                                                                  \
        case 0:                                                                                                       \
            DISPATCH(g.pl, (pcg_init_kernel<kMode, kRpb, kNc, VT><<<dim3(g.grid), dim3(rows_block(kMode)), 0, s>>>(tp, g.d_boff, g.count))); \
            break;                                                                                                    \
        case 1:                                                                                                       \
            DISPATCH(g.pl, (pcg_spmv_kernel<kMode, kRpb, kNc, VT><<<dim3(g.grid), dim3(rows_block(kMode)), 0, s>>>(tp, g.d_boff, g.count))); \
            break;                                                                                                    \
        default:                                                                                                      \
            DISPATCH(g.pl, (resid_kernel<kMode, kRpb, kNc, VT><<<dim3(g.grid), dim3(rows_block(kMode)), 0, s>>>(tp, g.d_boff, g.count))); \
            break;                                                                                                    \
    }

static void launch_rows(int which, const Group &g, const PcgProb *probs, hipStream_t s)
{
    const PcgProb *tp = probs + g.first;
    if (g.fp32) {
        FE_ROWS_KERNELS(FE_PLAN_DISPATCH_FP32, float)
    } else {
        FE_ROWS_KERNELS(FE_PLAN_DISPATCH_ALL, double)
    }
}

fe_status engine_build(EngineSet &E, const PcgJob *jobs, int njobs, void *table, hipStream_t s)
{
    std::vector<int> order;
    std::vector<SpmvPlan> plans(njobs);
    for (int i = 0; i < njobs; i++) {
        if (jobs[i].dg)  // DG: the cell-block traversal
            plans[i] = SpmvPlan{10, jobs[i].sa->dim, jobs[i].sa->nn, 0};
        else if (jobs[i].sa && jobs[i].fp32 && !jobs[i].sym)  // FP32 values: the block-staged traversal
            plans[i] = SpmvPlan{6, jobs[i].sa->ncomp, 8, 8};
        else if (jobs[i].sym)
            plans[i] = launch_form(SpmvPlan{7, 1, jobs[i].sa->dim == 3 ? 27 : 9, 2}, jobs[i].n);
        else
            plans[i] = jobs[i].sa ? aligned_form(struct_plan(*jobs[i].sa), jobs[i].val)
                                  : csr_launch_form(plan_for(jobs[i].n, jobs[i].nnz), jobs[i].n, jobs[i].nnz,
                                                    jobs[i].colind, jobs[i].val);
        if (jobs[i].n > 0) order.push_back(i);
    }
    auto key = [&](int i) {
        return ((plans[i].mode * 1024 + plans[i].rpb) * 4 + plans[i].nc) * 2 + (jobs[i].fp32 ? 1 : 0);
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key(a) < key(b); });
    const int np = int(order.size());
    E.np = np;
    E.jobs.clear();
    E.hp.assign(np, PcgProb{});
    E.hi.assign(3 * size_t(np) + 16, 0);
    E.groups.clear();
    E.hs.assign(np, PcgState{});
    if (np == 0) return FE_OK;
    char *tb = static_cast<char *>(table);
    const size_t sp = align256(sizeof(PcgProb) * size_t(np));
    const size_t si = align256(sizeof(int32_t) * (3 * size_t(np) + 16));
    const size_t ss = align256(sizeof(PcgState) * size_t(np));
    E.d_probs = reinterpret_cast<PcgProb *>(tb);
    E.d_ints = reinterpret_cast<int32_t *>(tb + sp);
    E.d_states = reinterpret_cast<PcgState *>(tb + sp + si);
    E.d_active = reinterpret_cast<int32_t *>(tb + sp + si + ss);
    int32_t eoff = 0;
    for (int t = 0; t < np; t++) {
        const PcgJob &jb = jobs[order[t]];
        E.jobs.push_back(jb);
        PcgProb &P = E.hp[t];
        P.n = jb.n;
        P.nnz = jb.nnz;
        P.rowptr = jb.rowptr;
        P.colind = jb.colind;
        P.val = jb.val;
        P.dinv = jb.dinv;
        P.b = jb.b;
        P.x = jb.x;
        P.w = carve(jb.ws, jb.n);
        P.rtol2 = jb.rtol * jb.rtol;
        P.maxit = jb.maxit;
        if (jb.sa) P.sa = *jb.sa;
        const SpmvPlan &pl = plans[order[t]];
        P.nbr = grid_rows(jb.n, pl);
        P.nbe = grid_elems(jb.n);
        E.hi[t] = eoff;
        eoff += P.nbe;
        if (E.groups.empty() || key(order[E.groups.back().first]) != key(order[t])) {
            Group g{};
            g.pl = pl;
            g.fp32 = jb.fp32;
            g.first = t;
            g.count = 0;
            E.groups.push_back(g);
        }
        E.groups.back().count++;
    }
    E.hi[np] = eoff;
    E.ge = eoff;
    int pos = np + 1;
    for (Group &g : E.groups) {
        int32_t off = 0;
        for (int t = 0; t < g.count; t++) {
            E.hi[pos + t] = off;
            off += E.hp[g.first + t].nbr;
        }
        E.hi[pos + g.count] = off;
        g.grid = off;
        g.d_boff = E.d_ints + pos;
        pos += g.count + 1;
    }
    FE_HIP(hipMemcpyAsync(E.d_probs, E.hp.data(), sizeof(PcgProb) * size_t(np), hipMemcpyHostToDevice, s));
    FE_HIP(hipMemcpyAsync(E.d_ints, E.hi.data(), sizeof(int32_t) * size_t(pos), hipMemcpyHostToDevice, s));
    return FE_OK;
}

// r = b - A x, p = z, first scalars and stop test of every problem of the set
fe_status engine_init(EngineSet &E, hipStream_t s)
{
    if (E.np == 0) return FE_OK;
    for (const Group &g : E.groups) launch_rows(0, g, E.d_probs, s);
    hipLaunchKernelGGL(pcg_init_finish_kernel, dim3(E.np), dim3(kBlock), 0, s, E.d_probs);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

// One CG iteration of every problem still running; marks are event pairs
// around the SpMV launches when timing is requested.
static void engine_iteration(const EngineSet &E, hipStream_t q, std::vector<std::pair<hipEvent_t, hipEvent_t>> *marks)
{
    for (const Group &g : E.groups) {
        hipEvent_t t0 = marks ? timing_mark(q) : nullptr;
        launch_rows(1, g, E.d_probs, q);
        if (t0) marks->emplace_back(t0, timing_mark(q));
    }
    hipLaunchKernelGGL(pcg_update_kernel, dim3(E.ge), dim3(kBlock), 0, q, E.d_probs, E.d_ints, E.np);
    hipLaunchKernelGGL(pcg_dir_kernel, dim3(E.ge), dim3(kBlock), 0, q, E.d_probs, E.d_ints, E.np);
}

fe_status engine_iterate(EngineSet &E, int iters, hipStream_t s)
{
    if (E.np == 0) return FE_OK;
    for (int i = 0; i < iters; i++) engine_iteration(E, s, nullptr);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

// Copies every problem's state to E.hs (waits for the stream).
fe_status engine_states(EngineSet &E, hipStream_t s)
{
    if (E.np == 0) return FE_OK;
    hipLaunchKernelGGL(gather_states_kernel, dim3((E.np + kBlock - 1) / kBlock), dim3(kBlock), 0, s, E.d_probs, E.np,
                       E.d_states);
    FE_HIP(hipGetLastError());
    FE_HIP(hipMemcpyAsync(E.hs.data(), E.d_states, sizeof(PcgState) * size_t(E.np), hipMemcpyDeviceToHost, s));
    FE_HIP(hipStreamSynchronize(s));
    return FE_OK;
}

// True residuals of every problem of the set, then their states and infos.
fe_status engine_finish(EngineSet &E, hipStream_t s)
{
    if (E.np == 0) return FE_OK;
    for (const Group &g : E.groups) launch_rows(2, g, E.d_probs, s);
    hipLaunchKernelGGL(resid_finish_kernel, dim3(E.np), dim3(kBlock), 0, s, E.d_probs);
    FE_HIP(hipGetLastError());
    fe_status st = engine_states(E, s);
    if (st != FE_OK) return st;
    for (int t = 0; t < E.np; t++) {
        const PcgState &h = E.hs[t];
        fe_solve_info *info = E.jobs[t].info;
        if (!info) continue;
        info->iters = h.iter;
        info->status = pcg_stopped(h, h.iter) ? h.status : FE_ENOTCONV;
        const double bn = std::sqrt(h.bb);
        info->relres = bn > 0 ? std::sqrt(h.rr) / bn : std::sqrt(h.rr);
        info->true_relres = bn > 0 ? std::sqrt(h.true_rr) / bn : std::sqrt(h.true_rr);
    }
    return FE_OK;
}

bool engine_done(const EngineSet &E, int t) { return pcg_stopped(E.hs[t], E.hs[t].iter); }

// Stream on which iteration chunks are captured (one per thread and device):
// capture only records launches, and the caller's stream may be the null
// stream, which cannot be captured.  The graph is launched on the caller's
// stream.
static fe_status capture_stream(hipStream_t &out)
{
    static thread_local std::vector<hipStream_t> streams;
    int dev = 0;
    FE_HIP(hipGetDevice(&dev));
    if (int(streams.size()) <= dev) streams.resize(dev + 1, nullptr);
    if (!streams[dev]) FE_HIP(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking));
    out = streams[dev];
    return FE_OK;
}

// no_alloc: direct launches only (no graph, no timing events) and the stop
// counter read into pageable host memory, so the solve creates no device,
// pinned or graph resource of its own.
static fe_status pcg_engine(std::vector<PcgJob> &jobs, void *table, bool use_graph, hipStream_t s,
                            bool no_alloc = false)
{
    for (PcgJob &jb : jobs) {
        std::memset(jb.info, 0, sizeof(fe_solve_info));
        if (jb.n == 0) jb.info->status = FE_OK;
    }
    EngineSet E;
    fe_status st = engine_build(E, jobs.data(), int(jobs.size()), table, s);
    if (st != FE_OK) return st;
    const int np = E.np;
    if (np == 0) return FE_OK;
    st = engine_init(E, s);
    if (st != FE_OK) return st;
    int maxit = 0;
    for (const PcgJob &jb : E.jobs) maxit = std::max(maxit, jb.maxit);

    static thread_local PinnedState pin;
    int32_t pageable_active = 0;
    int32_t *h_active = &pageable_active;
    if (no_alloc) {
        use_graph = false;
    } else {
        if (!pin.h) FE_HIP(hipHostMalloc(reinterpret_cast<void **>(&pin.h), sizeof(PcgState), hipHostMallocDefault));
        h_active = reinterpret_cast<int32_t *>(pin.h);
    }
    const bool timed = timing_on() && !use_graph && !no_alloc && np == 1;
    // SpMV launches timed: every kTimeEvery-th iteration (an event pair costs a
    // few microseconds of device time, which around every launch lengthened
    // the solve by about 6%); marks[i] belongs to iteration mark_iter[i]
    constexpr int kTimeEvery = 16;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> marks;
    std::vector<int> mark_iter;
    struct GraphHold {
        hipGraph_t g = nullptr;
        hipGraphExec_t e = nullptr;
        ~GraphHold()
        {
            if (e) (void)hipGraphExecDestroy(e);
            if (g) (void)hipGraphDestroy(g);
        }
    } hold;
    const int gchunk = 16;
    if (use_graph && maxit > 0) {
        hipStream_t cs = nullptr;
        st = capture_stream(cs);
        if (st != FE_OK) return st;
        FE_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < gchunk; i++) engine_iteration(E, cs, nullptr);
        hipLaunchKernelGGL(count_active_kernel, dim3(1), dim3(kBlock), 0, cs, E.d_probs, np, E.d_active);
        if (hipStreamEndCapture(cs, &hold.g) != hipSuccess) return set_error(FE_EDEVICE, "graph capture failed");
        if (hipGraphInstantiate(&hold.e, hold.g, nullptr, nullptr, 0) != hipSuccess)
            return set_error(FE_EDEVICE, "graph instantiation failed");
    }
    int j = 0, chunk = 8;
    while (j < maxit) {
        if (hold.e) {
            FE_HIP(hipGraphLaunch(hold.e, s));
            j += gchunk;
        } else {
            for (int i = 0; i < chunk && j < maxit; i++, j++) {
                const bool mark = timed && j % kTimeEvery == 0;
                engine_iteration(E, s, mark ? &marks : nullptr);
                mark_iter.resize(marks.size(), j);
            }
            hipLaunchKernelGGL(count_active_kernel, dim3(1), dim3(kBlock), 0, s, E.d_probs, np, E.d_active);
            if (chunk < 128) chunk *= 2;
        }
        FE_HIP(hipGetLastError());
        FE_HIP(hipMemcpyAsync(h_active, E.d_active, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        FE_HIP(hipStreamSynchronize(s));
        if (*h_active == 0) break;
    }
    st = engine_finish(E, s);
    if (st != FE_OK) return st;
    for (size_t i = 0; i < marks.size(); i++) {
        if (mark_iter[i] < E.hs[0].iter) {
            timing_commit(marks[i].first, marks[i].second, kTimeSpmv);
        } else {
            timing_release(marks[i].first);
            timing_release(marks[i].second);
        }
    }
    fe_status worst = FE_OK;
    for (int t = 0; t < np; t++) {
        const int stt = E.jobs[t].info->status;
        if (stt != FE_OK && worst == FE_OK) worst = fe_status(stt);
    }
    // Lanczos estimates from the CG coefficients (single problem)
    if (np == 1) {
        fe_solve_info *info = E.jobs[0].info;
        const int m = std::min(E.hs[0].iter, kHist);
        if (m > 0) {
            std::vector<double> h(2 * kHist);
            FE_HIP(hipMemcpy(h.data(), E.hp[0].w.hist, sizeof(double) * 2 * kHist, hipMemcpyDeviceToHost));
            std::vector<double> d(m), e(m > 1 ? m - 1 : 1);
            for (int i = 0; i < m; i++) {
                const double a = h[i];
                d[i] = 1.0 / a + (i > 0 ? h[kHist + i - 1] / h[i - 1] : 0.0);
                if (i + 1 < m) e[i] = std::sqrt(h[kHist + i]) / a;
            }
            tridiag_extremes(d, e, info->lambda_min_est, info->lambda_max_est);
        }
    }
    if (worst == FE_ENOTCONV) set_error(FE_ENOTCONV, "pcg reached maxit");
    if (worst == FE_EBREAKDOWN) set_error(FE_EBREAKDOWN, "pcg breakdown: p.Ap <= 0 or not finite");
    return worst;
}

template <typename VT>
static fe_status pcg_run(int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *colind, const VT *val,
                         const double *dinv, const double *b, double *x, double rtol, int maxit, void *ws,
                         size_t ws_bytes, fe_solve_info *info, hipStream_t s, const SpaceArgs *sa = nullptr,
                         bool sym = false, bool dg = false)
{
    if (ws_bytes < pcg_ws_bytes(n) + engine_table_bytes(1)) return set_error(FE_EINVAL, "pcg workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) & 7u) return set_error(FE_EINVAL, "workspace not 8-byte aligned");
    std::vector<PcgJob> jobs(1);
    jobs[0] = PcgJob{n, nnz, rowptr, colind, val, std::is_same<VT, float>::value, dinv, b, x, ws, info, rtol, maxit, sa,
                     sym, dg};
    void *table = static_cast<char *>(ws) + pcg_ws_bytes(n);
    // small systems are launch-bound: replay the iterations from a HIP graph
    const bool graph = n < (int64_t(1) << 18);
    return pcg_engine(jobs, table, graph, s);
}

fe_status pcg_solve(const fe_csr *A, const double *b, double *x, double rtol, int maxit, void *ws, size_t ws_bytes,
                    fe_solve_info *info, hipStream_t s)
{
    return pcg_run<double>(A->n_rows, A->nnz, A->rowptr, A->colind, A->values, A->dinv, b, x, rtol, maxit, ws,
                           ws_bytes, info, s);
}

// ---------------------------------------------------------------------------
// Jacobi-PCG without allocation: the workspace of fe_pcg_solve lives in a
// file-scope device array, one copy per device, instead of the caller's
// buffer.  Host code reaches it only through the address hipGetSymbolAddress
// returns for the current device (the array's name is a host-side stand-in).
// Every call on a device shares its copy: overlapping calls on one device
// race.  Nothing in the workspace has to start at zero (the init kernels write
// every state field before it is read), so the previous call's contents are
// harmless.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static std::vector<void *> g_scratch_ptr;  // per device: the array's device address

static fe_status scratch_address(void *&out)
{
    int dev = 0;
    FE_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (int(g_scratch_ptr.size()) <= dev) g_scratch_ptr.resize(size_t(dev) + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(FE_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    out = g_scratch_ptr[dev];
    return FE_OK;
}

size_t pcg_noalloc_bytes() { return kScratchBytes; }

fe_status pcg_solve_noalloc(const fe_csr *A, const double *b, double *x, double rtol, int maxit, fe_solve_info *info,
                            hipStream_t s)
{
    const int64_t n = A->n_rows;
    if (pcg_ws_bytes(n) + engine_table_bytes(1) > kScratchBytes)
        return set_error(FE_EINVAL, "system too large for the allocation-free solve (at most 2,700,000 rows)");
    void *ws = nullptr;
    const fe_status st = scratch_address(ws);
    if (st != FE_OK) return st;
    std::vector<PcgJob> jobs(1);
    jobs[0] = PcgJob{n, A->nnz, A->rowptr, A->colind, A->values, false, A->dinv, b, x, ws, info, rtol, maxit,
                     nullptr, false};
    return pcg_engine(jobs, static_cast<char *>(ws) + pcg_ws_bytes(n), false, s, true);
}

fe_status pcg_solve_mesh(const fe_csr *A, const SpaceArgs &sa, const double *b, double *x, double rtol, int maxit,
                         void *ws, size_t ws_bytes, fe_solve_info *info, hipStream_t s)
{
    return pcg_run<double>(A->n_rows, A->nnz, A->rowptr, A->colind, A->values, A->dinv, b, x, rtol, maxit, ws,
                           ws_bytes, info, s, &sa);
}

bool sym_supported(const SpaceArgs &sa) { return sa.k == 1 && sa.ncomp == 1 && (sa.dim == 2 || sa.dim == 3); }

size_t sym_bytes(const SpaceArgs &sa)
{
    return size_t(sym_slots(sa.dim)) * size_t(sym_stride(sa.n_rows)) * sizeof(double);
}

template <typename OT>
static fe_status sym_fill(const SpaceArgs &sa, const double *val, OT *sym, hipStream_t s)
{
    const int64_t ns = sym_stride(sa.n_rows);
    if (ns == 0) return FE_OK;
    const dim3 grid(unsigned((ns / 32 + kQ1Waves - 1) / kQ1Waves));  // a wave per 32 rows of the stride
    if (sa.dim == 3) hipLaunchKernelGGL((sym_fill_kernel<3, OT>), grid, dim3(kQ1Block), 0, s, sa, val, sym);
    else hipLaunchKernelGGL((sym_fill_kernel<2, OT>), grid, dim3(kQ1Block), 0, s, sa, val, sym);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

fe_status launch_sym_fill(const SpaceArgs &sa, const double *val, double *sym, hipStream_t s)
{
    return sym_fill(sa, val, sym, s);
}

fe_status launch_sym_fill_fp32(const SpaceArgs &sa, const double *val, float *sym, hipStream_t s)
{
    return sym_fill(sa, val, sym, s);
}

fe_status launch_spmv_sym(const SpaceArgs &sa, const double *sym, const double *x, double *y, hipStream_t s)
{
    if (sa.n_rows == 0) return FE_OK;
    const SpmvPlan pl = launch_form(SpmvPlan{7, 1, sa.dim == 3 ? 27 : 9, 2}, sa.n_rows);
    const int g = grid_rows(sa.n_rows, pl);
    FE_SPLAN_DISPATCH(pl, (spmv_struct_kernel<kMode, kRpb, kNc><<<dim3(g), dim3(rows_block(kMode)), 0, s>>>(sa, sym, x, y)));
    FE_HIP(hipGetLastError());
    return FE_OK;
}

fe_status pcg_solve_sym(const fe_csr *A, const SpaceArgs &sa, const double *sym, const double *b, double *x,
                        double rtol, int maxit, void *ws, size_t ws_bytes, fe_solve_info *info, hipStream_t s)
{
    return pcg_run<double>(A->n_rows, A->nnz, A->rowptr, A->colind, sym, A->dinv, b, x, rtol, maxit, ws, ws_bytes,
                           info, s, &sa, true);
}

fe_status launch_spmv_struct(const SpaceArgs &sa, const double *val, const double *x, double *y, hipStream_t s)
{
    if (sa.n_rows == 0) return FE_OK;
    const SpmvPlan pl = aligned_form(struct_plan(sa), val);
    const int g = grid_rows(sa.n_rows, pl);
    FE_SPLAN_DISPATCH(pl, (spmv_struct_kernel<kMode, kRpb, kNc><<<dim3(g), dim3(rows_block(kMode)), 0, s>>>(sa, val, x, y)));
    FE_HIP(hipGetLastError());
    return FE_OK;
}

fe_status launch_spmv_dg(const SpaceArgs &sa, const double *val, const double *x, double *y, hipStream_t s)
{
    if (sa.n_rows == 0) return FE_OK;
    const SpmvPlan pl{10, sa.dim, sa.nn, 0};
    const int g = grid_rows(sa.n_rows, pl);
    FE_DG_DISPATCH(pl, (spmv_struct_kernel<kMode, kRpb, kNc><<<dim3(g), dim3(rows_block(kMode)), 0, s>>>(sa, val, x, y)));
    FE_HIP(hipGetLastError());
    return FE_OK;
}

fe_status pcg_solve_dg(const fe_csr *A, const SpaceArgs &sa, const double *b, double *x, double rtol, int maxit,
                       void *ws, size_t ws_bytes, fe_solve_info *info, hipStream_t s)
{
    return pcg_run<double>(A->n_rows, A->nnz, A->rowptr, A->colind, A->values, A->dinv, b, x, rtol, maxit, ws, ws_bytes,
                           info, s, &sa, false, true);
}

size_t pcg_solve_ws_bytes(int64_t n) { return pcg_ws_bytes(n) + engine_table_bytes(1); }

fe_status pcg_solve_batch(int nprob, const fe_csr *A, const double *const *b, double *const *x, double rtol,
                          int maxit, void *ws, size_t ws_bytes, fe_solve_info *infos, hipStream_t s,
                          const SpaceArgs *const *sas)
{
    size_t need = engine_table_bytes(nprob);
    for (int i = 0; i < nprob; i++) need += pcg_ws_bytes(A[i].n_rows);
    if (ws_bytes < need) return set_error(FE_EINVAL, "batch pcg workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) & 7u) return set_error(FE_EINVAL, "workspace not 8-byte aligned");
    std::vector<PcgJob> jobs(nprob);
    char *p = static_cast<char *>(ws) + engine_table_bytes(nprob);
    for (int i = 0; i < nprob; i++) {
        jobs[i] = PcgJob{A[i].n_rows, A[i].nnz, A[i].rowptr, A[i].colind, A[i].values, false, A[i].dinv,
                         b[i], x[i], p, &infos[i], rtol, maxit, sas ? sas[i] : nullptr};
        p += pcg_ws_bytes(A[i].n_rows);
    }
    return pcg_engine(jobs, ws, true, s);
}

size_t pcg_batch_ws_bytes(int nprob, const int64_t *n_rows)
{
    size_t need = engine_table_bytes(nprob);
    for (int i = 0; i < nprob; i++) need += pcg_ws_bytes(n_rows[i]);
    return need;
}

// ---------------------------------------------------------------------------
// Iterative refinement (precision form): outer residual in FP64 with the FP64
// matrix, inner Jacobi-PCG on a lower-precision operator, x += correction.
// ---------------------------------------------------------------------------
// r = b - A x; partials of r.r
template <int MODE, int RPB>
__global__ __launch_bounds__(rows_block(MODE)) void resid_vec_kernel(int64_t n, int64_t nnz,
                                                                      const int64_t *__restrict__ rowptr,
                                                            const int32_t *__restrict__ colind,
                                                            const double *__restrict__ val,
                                                            const double *__restrict__ b, const double *__restrict__ x,
                                                            double *__restrict__ r, PcgWs w)
{
    double v[2] = {0.0, 0.0};
    for_rows<MODE, RPB, double>(n, nnz, rowptr, colind, val, x, blockIdx.x, gridDim.x,
                                [&](int64_t row, double ax) {
        const double d = b[row] - ax;
        r[row] = d;
        v[0] += d * d;
        v[1] += b[row] * b[row];
    });
    write_partials<2, rows_block(MODE)>(v, w.p3, w.ps);
}

__global__ __launch_bounds__(kBlock) void resid_vec_finish_kernel(PcgWs w, int nparts)
{
    double t[2];
    reduce_partials<2>(w.p3, nparts, w.ps, t);
    if (threadIdx.x == 0) {
        w.st->true_rr = t[0];
        w.st->bb = t[1];
    }
}

__global__ __launch_bounds__(kBlock) void axpy_kernel(int64_t n, const double *__restrict__ d, double *__restrict__ x)
{
    for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) x[i] += d[i];
}

__global__ __launch_bounds__(kBlock) void demote_kernel(int64_t nnz, const double *__restrict__ v, float *__restrict__ o)
{
    for (int64_t i = blockIdx.x * int64_t(kBlock) + threadIdx.x; i < nnz; i += int64_t(gridDim.x) * kBlock)
        o[i] = float(v[i]);
}

size_t refine_ws_bytes(int64_t n)
{
    return pcg_ws_bytes(n) + engine_table_bytes(1) + 2 * align256(size_t(n) * sizeof(double));
}

// Batched refinement: per problem its inner PCG workspace, r and d; plus the
// inner engine's table, the residual norms and a device array of state pointers.
size_t refine_batch_ws_bytes(int nprob, const int64_t *n_rows)
{
    const size_t np = size_t(std::max(nprob, 1));
    size_t b = engine_table_bytes(nprob) + align256(2 * np * sizeof(double)) + align256(np * sizeof(PcgState *));
    for (int i = 0; i < nprob; i++) b += pcg_ws_bytes(n_rows[i]) + 2 * align256(size_t(n_rows[i]) * sizeof(double));
    return b;
}

__global__ __launch_bounds__(kBlock) void refine_norms_kernel(PcgState *const *__restrict__ st, int np,
                                                               double *__restrict__ out)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < np; i += gridDim.x * kBlock) {
        out[2 * i] = st[i]->bb;
        out[2 * i + 1] = st[i]->true_rr;
    }
}

// Iterative refinement of many systems at once, each step as fe_refine_solve
// takes it for one system (the FP64 residual through the CSR of A_hi, the
// inner Jacobi-PCG on A_lo's FP64 values): the residuals of the running
// systems are formed and their norms read back together, and their
// corrections solved by one batched PCG (the engine solves each system as it
// would alone, so every result is bitwise that of the one-system call).
fe_status refine_solve_batch(int nprob, const fe_csr *Ahi, const fe_csr *Alo, const double *const *b,
                             double *const *x, double rtol, double inner_rtol, int max_outer, int max_inner,
                             void *ws, size_t ws_bytes, fe_refine_info *infos, hipStream_t s,
                             const SpaceArgs *const *sas)
{
    std::vector<int64_t> nr(nprob);
    for (int i = 0; i < nprob; i++) {
        nr[i] = Ahi[i].n_rows;
        std::memset(&infos[i], 0, sizeof(fe_refine_info));
        infos[i].status = nr[i] == 0 ? FE_OK : FE_ENOTCONV;
        if (Alo[i].n_rows != nr[i] || Alo[i].nnz != Ahi[i].nnz)
            return set_error(FE_EINVAL, "A_lo must have the pattern of A_hi");
    }
    if (ws_bytes < refine_batch_ws_bytes(nprob, nr.data())) return set_error(FE_EINVAL, "refinement workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) & 7u) return set_error(FE_EINVAL, "workspace not 8-byte aligned");
    if (nprob == 0) return FE_OK;
    char *p = static_cast<char *>(ws);
    void *table = p;
    p += engine_table_bytes(nprob);
    double *d_norms = reinterpret_cast<double *>(p);
    p += align256(2 * size_t(nprob) * sizeof(double));
    PcgState **d_st = reinterpret_cast<PcgState **>(p);
    p += align256(size_t(nprob) * sizeof(PcgState *));
    std::vector<void *> pws(nprob);
    std::vector<double *> r(nprob), d(nprob);
    std::vector<PcgState *> hst(nprob);
    for (int i = 0; i < nprob; i++) {
        pws[i] = p;
        hst[i] = carve(p, nr[i]).st;
        p += pcg_ws_bytes(nr[i]);
        r[i] = reinterpret_cast<double *>(p);
        p += align256(size_t(nr[i]) * sizeof(double));
        d[i] = reinterpret_cast<double *>(p);
        p += align256(size_t(nr[i]) * sizeof(double));
    }
    FE_HIP(hipMemcpyAsync(d_st, hst.data(), sizeof(PcgState *) * size_t(nprob), hipMemcpyHostToDevice, s));
    std::vector<int> active;
    for (int i = 0; i < nprob; i++)
        if (nr[i] > 0) active.push_back(i);
    std::vector<double> hn(2 * size_t(nprob));
    std::vector<fe_solve_info> inner(nprob);
    fe_status worst = FE_OK;
    for (int it = 0; it <= max_outer && !active.empty(); it++) {
        for (int i : active) {
            const int64_t n = nr[i];
            const SpmvPlan pl = csr_launch_form(plan_for(n, Ahi[i].nnz), n, Ahi[i].nnz, Ahi[i].colind, Ahi[i].values);
            const int gr = grid_rows(n, pl);
            const PcgWs w = carve(pws[i], n);
            FE_PLAN_DISPATCH(pl, (resid_vec_kernel<kMode, kRpb><<<dim3(gr), dim3(rows_block(kMode)), 0, s>>>(
                                     n, Ahi[i].nnz, Ahi[i].rowptr, Ahi[i].colind, Ahi[i].values, b[i], x[i], r[i], w)));
            hipLaunchKernelGGL(resid_vec_finish_kernel, dim3(1), dim3(kBlock), 0, s, w, gr);
        }
        hipLaunchKernelGGL(refine_norms_kernel, dim3((nprob + kBlock - 1) / kBlock), dim3(kBlock), 0, s, d_st, nprob,
                           d_norms);
        FE_HIP(hipGetLastError());
        FE_HIP(hipMemcpyAsync(hn.data(), d_norms, sizeof(double) * 2 * size_t(nprob), hipMemcpyDeviceToHost, s));
        FE_HIP(hipStreamSynchronize(s));
        std::vector<int> next;
        for (int i : active) {
            const double bn = std::sqrt(hn[2 * size_t(i)]), rn = std::sqrt(hn[2 * size_t(i) + 1]);
            infos[i].relres = bn > 0 ? rn / bn : rn;
            if (infos[i].relres <= rtol) infos[i].status = FE_OK;
            else if (it < max_outer) next.push_back(i);
        }
        if (next.empty()) break;
        std::vector<PcgJob> jobs;
        for (int i : next) {
            FE_HIP(hipMemsetAsync(d[i], 0, sizeof(double) * size_t(nr[i]), s));
            jobs.push_back(PcgJob{nr[i], Alo[i].nnz, Alo[i].rowptr, Alo[i].colind, Alo[i].values, false, Alo[i].dinv,
                                  r[i], d[i], pws[i], &inner[i], inner_rtol, max_inner, sas ? sas[i] : nullptr,
                                  false});
        }
        const fe_status st = pcg_engine(jobs, table, true, s);
        if (st == FE_EDEVICE || st == FE_EINVAL) return st;
        active.clear();
        for (int i : next) {
            infos[i].inner_iters += inner[i].iters;
            infos[i].outer_iters = it + 1;
            if (inner[i].status == FE_EBREAKDOWN) {
                infos[i].status = FE_EBREAKDOWN;
                worst = FE_EBREAKDOWN;
                continue;
            }
            hipLaunchKernelGGL(axpy_kernel, dim3(grid_elems(nr[i])), dim3(kBlock), 0, s, nr[i], d[i], x[i]);
            active.push_back(i);
        }
        FE_HIP(hipGetLastError());
    }
    FE_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < nprob; i++)
        if (infos[i].status == FE_ENOTCONV && worst == FE_OK) worst = FE_ENOTCONV;
    if (worst == FE_ENOTCONV) set_error(FE_ENOTCONV, "iterative refinement reached max_outer");
    if (worst == FE_EBREAKDOWN) set_error(FE_EBREAKDOWN, "inner pcg breakdown");
    return worst;
}

fe_status csr_to_fp32(const fe_csr *A, float *values32, hipStream_t s)
{
    if (A->nnz == 0) return FE_OK;
    const int64_t grid = std::min<int64_t>((A->nnz + kBlock - 1) / kBlock, 8192);
    hipLaunchKernelGGL(demote_kernel, dim3(grid), dim3(kBlock), 0, s, A->nnz, A->values, values32);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

fe_status refine_solve(const fe_csr *Ahi, const fe_csr *Alo, const float *values32, const double *b, double *x,
                       double rtol, double inner_rtol, int max_outer, int max_inner, void *ws, size_t ws_bytes,
                       fe_refine_info *info, hipStream_t s, const SpaceArgs *sa, const float *sym32)
{
    const int64_t n = Ahi->n_rows;
    std::memset(info, 0, sizeof(*info));
    if (ws_bytes < refine_ws_bytes(n)) return set_error(FE_EINVAL, "refinement workspace too small");
    if (reinterpret_cast<uintptr_t>(ws) & 7u) return set_error(FE_EINVAL, "workspace not 8-byte aligned");
    if (Alo->n_rows != n || Alo->nnz != Ahi->nnz) return set_error(FE_EINVAL, "A_lo must have the pattern of A_hi");
    if (n == 0) return FE_OK;
    static thread_local PinnedState pin;
    if (!pin.h) FE_HIP(hipHostMalloc(reinterpret_cast<void **>(&pin.h), sizeof(PcgState), hipHostMallocDefault));
    char *base = static_cast<char *>(ws);
    void *pws = base;
    const size_t inner_bytes = pcg_ws_bytes(n) + engine_table_bytes(1);
    double *r = reinterpret_cast<double *>(base + inner_bytes);
    double *d = reinterpret_cast<double *>(base + inner_bytes + align256(size_t(n) * sizeof(double)));
    PcgWs w = carve(pws, n);
    const SpmvPlan pl = csr_launch_form(plan_for(n, Ahi->nnz), n, Ahi->nnz, Ahi->colind, Ahi->values);
    const int gr = grid_rows(n, pl);
    const int ge = grid_elems(n);
    info->status = FE_ENOTCONV;
    for (int it = 0; it <= max_outer; it++) {
        FE_PLAN_DISPATCH(pl, (resid_vec_kernel<kMode, kRpb><<<dim3(gr), dim3(rows_block(kMode)), 0, s>>>(
                                 n, Ahi->nnz, Ahi->rowptr, Ahi->colind, Ahi->values, b, x, r, w)));
        hipLaunchKernelGGL(resid_vec_finish_kernel, dim3(1), dim3(kBlock), 0, s, w, gr);
        FE_HIP(hipGetLastError());
        FE_HIP(hipMemcpyAsync(pin.h, w.st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
        FE_HIP(hipStreamSynchronize(s));
        const double bn = std::sqrt(pin.h->bb), rn = std::sqrt(pin.h->true_rr);
        info->relres = bn > 0 ? rn / bn : rn;
        if (info->relres <= rtol) {
            info->status = FE_OK;
            break;
        }
        if (it == max_outer) break;
        // correction: A_lo d = r, from d = 0
        FE_HIP(hipMemsetAsync(d, 0, sizeof(double) * size_t(n), s));
        fe_solve_info inner;
        fe_status st;
        if (sym32)
            st = pcg_run<float>(n, Alo->nnz, Alo->rowptr, Alo->colind, sym32, Alo->dinv, r, d, inner_rtol,
                                max_inner, pws, inner_bytes, &inner, s, sa, true);
        else if (values32)
            st = pcg_run<float>(n, Alo->nnz, Alo->rowptr, Alo->colind, values32, Alo->dinv, r, d, inner_rtol,
                                max_inner, pws, inner_bytes, &inner, s, sa);
        else
            st = pcg_run<double>(n, Alo->nnz, Alo->rowptr, Alo->colind, Alo->values, Alo->dinv, r, d, inner_rtol,
                                 max_inner, pws, inner_bytes, &inner, s, sa);
        info->inner_iters += inner.iters;
        info->outer_iters = it + 1;
        if (st == FE_EBREAKDOWN || st == FE_EDEVICE || st == FE_EINVAL) {
            info->status = st;
            return st;
        }
        hipLaunchKernelGGL(axpy_kernel, dim3(ge), dim3(kBlock), 0, s, n, d, x);
        FE_HIP(hipGetLastError());
    }
    if (info->status == FE_ENOTCONV) return set_error(FE_ENOTCONV, "iterative refinement reached max_outer");
    return FE_OK;
}

}  // namespace fe
