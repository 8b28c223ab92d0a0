// fe_integrate_mfma.hip -- K3 on the matrix cores: element matrices of Q_k
// hexahedra (k >= 2) as small GEMMs on MFMA (Sect. 3.7 eq. fematrix; the
// Poisson element loop of Sect. 8.5 written as a contraction).
//
// With G[(c,q)][a] = (grad phi_a)_c at quadrature point q (physical, FP64
// geometry) and w_q = w_q k_K |det J_q|:
//   Poisson     A[a][b]        = sum_(c,q) G[(c,q)][a] w_q G[(c,q)][b]          (K = d nq)
//   Elasticity  M_ij[a][b]     = sum_q G[(i,q)][a] w_q G[(j,q)][b]              (9 Gram blocks, K = nq)
//               A[(a,i)][(b,j)] = lambda M_ij + mu (M_ji + delta_ij sum_l M_ll)  (combined per lane)
// FP64 (v_mfma_f64_16x16x4) and FP32 (v_mfma_f32_16x16x4): a workgroup owns
// one cell (or a part of its tile pairs); it stages the physical gradients of
// a slab of quadrature points in LDS, then every wave accumulates its
// node-tile pairs (ta <= tb, 16 x 16 each) with MFMA; the lower triangle is
// written as the mirror of the upper one.  FP16 / BF16 inputs with FP32
// accumulation (v_mfma_f32_16x16x32) run the whole-cell kernel further down.
// The gradients are always computed in FP64 and rounded to the input type.
#include <cmath>
#include <map>
#include <mutex>
#include <type_traits>
#include <vector>

#include "fe_internal.h"

namespace fe {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef __bf16 b8_t __attribute__((ext_vector_type(8)));

struct PolF64 {
    using S = double;
    using Acc = d4_t;
    using Out = double;
    static constexpr int KM = 4;
    static constexpr bool ROW_INTERLEAVED = true;  // D register r of lane l is row 4 r + l / 16
    __device__ static Acc zero() { return Acc{0.0, 0.0, 0.0, 0.0}; }
    __device__ static Acc mma(S a, S b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};

struct PolF32 {
    using S = float;
    using Acc = f4_t;
    using Out = float;
    static constexpr int KM = 4;
    static constexpr bool ROW_INTERLEAVED = false;  // row 4 (l / 16) + r
    __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
    __device__ static Acc mma(S a, S b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

// FP64 to FP16, correctly rounded, by round-to-odd (Boldo and Melquiond):
// FP32 to nearest even, moved one unit toward zero where that rounded away
// from zero and its last bit set where inexact (rounding to odd), then FP32
// to FP16 to nearest even in hardware; FP32 carries 13 more bits than FP16,
// so the second rounding gives the correctly rounded result.
__device__ __forceinline__ _Float16 f64_to_f16(double x)
{
    const float t = float(x);
    const double back = double(t);
    uint32_t u = __float_as_uint(t);
    if (back != x) {
        if (fabs(back) > fabs(x)) u -= 1u;
        u |= 1u;
    }
    return _Float16(__uint_as_float(u));
}

struct PolF16 {
    using S = _Float16;
    using V = h8_t;
    using Acc = f4_t;
    using Out = float;
    static constexpr int KM = 32;  // a lane reads 8 consecutive points
    __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
    __device__ static Acc mma(V a, V b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
    __device__ static S cvt(double x) { return f64_to_f16(x); }
};

struct PolBF16 {
    using S = __bf16;
    using V = b8_t;
    using Acc = f4_t;
    using Out = float;
    static constexpr int KM = 32;
    __device__ static Acc zero() { return Acc{0.f, 0.f, 0.f, 0.f}; }
    __device__ static Acc mma(V a, V b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
    __device__ static S cvt(double x) { return S(x); }
};

template <int DIM>
__device__ __forceinline__ double geometry_mf(const double X[][3], const double xi[3], double Ji[9], double xq[3])
{
    double J[9];
    for (int t = 0; t < 9; t++) J[t] = 0.0;
    xq[0] = xq[1] = xq[2] = 0.0;
    for (int v = 0; v < (1 << DIM); v++) {
        double Nv = 1.0, dN[3];
        for (int r = 0; r < DIM; r++) Nv *= ((v >> r) & 1) ? xi[r] : 1.0 - xi[r];
        for (int sd = 0; sd < DIM; sd++) {
            double g = 1.0;
            for (int r = 0; r < DIM; r++)
                g *= (r == sd) ? (((v >> r) & 1) ? 1.0 : -1.0) : (((v >> r) & 1) ? xi[r] : 1.0 - xi[r]);
            dN[sd] = g;
        }
        for (int r = 0; r < DIM; r++) {
            xq[r] += X[v][r] * Nv;
            for (int sd = 0; sd < DIM; sd++) J[r * DIM + sd] += X[v][r] * dN[sd];
        }
    }
    const double c00 = J[4] * J[8] - J[5] * J[7];
    const double c01 = J[5] * J[6] - J[3] * J[8];
    const double c02 = J[3] * J[7] - J[4] * J[6];
    const double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
    const double id = 1.0 / det;
    Ji[0] = c00 * id;
    Ji[1] = (J[2] * J[7] - J[1] * J[8]) * id;
    Ji[2] = (J[1] * J[5] - J[2] * J[4]) * id;
    Ji[3] = c01 * id;
    Ji[4] = (J[0] * J[8] - J[2] * J[6]) * id;
    Ji[5] = (J[2] * J[3] - J[0] * J[5]) * id;
    Ji[6] = c02 * id;
    Ji[7] = (J[1] * J[6] - J[0] * J[7]) * id;
    Ji[8] = (J[0] * J[4] - J[1] * J[3]) * id;
    return det;
}

__device__ __forceinline__ double source_value_mf(const ProblemArgs &p, const double *x, int c)
{
    if (p.source_kind == FE_SOURCE_CONST) return p.source[c];
    if (p.source_kind == FE_SOURCE_SINPROD) {
        const double s = sin(M_PI * x[0]) * sin(M_PI * x[1]) * sin(M_PI * x[2]);
        return p.source[c] * 3.0 * (M_PI * M_PI) * s;
    }
    return 0.0;
}

// (ta, tb) of pair p in the upper-triangle enumeration of NT x NT tiles.
__device__ __forceinline__ void pair_tiles(int p, int NT, int &ta, int &tb)
{
    ta = 0;
    while (p >= NT - ta) {
        p -= NT - ta;
        ta++;
    }
    tb = ta + p;
}

// Elasticity entry from the accumulated products: lambda a12 + mu a21, plus
// mu tr on the diagonal of a component block.  The roundings are fixed by
// explicit fused multiply-adds, so that every tile shape's instantiation
// gives the same bits (contraction left to the compiler can differ between
// instantiations).
__device__ __forceinline__ double el_value(double lambda, double mu, double a12, double a21, double tr, bool cdiag)
{
    const double v = __fma_rn(lambda, a12, mu * a21);
    return cdiag ? __fma_rn(mu, tr, v) : v;
}

// One workgroup = 4 waves = (cell, part).  NNP = padded node count (multiple
// of 16), PPW = max node-tile pairs per wave, QS = quadrature points per slab.
template <class Pol, int PROB, int NNP, int PPW, int QS>
__device__ __forceinline__ void k3_mfma_body(const SpaceArgs &s, const MeshArgs &m, const ProblemArgs &p,
                                             const RefTables &rt, int parts, typename Pol::Out *__restrict__ E,
                                             double *__restrict__ F, int64_t bid)
{
    constexpr int DIM = 3;
    constexpr int NT = NNP / 16;
    constexpr int NP = NT * (NT + 1) / 2;
    constexpr int NC = PROB == 1 ? DIM : 1;        // DOF components
    constexpr int NCP = PROB == 1 ? DIM * DIM : 1;  // accumulator tiles per pair
    constexpr int NW = 4;
    using S = typename Pol::S;
    using Acc = typename Pol::Acc;
    using Out = typename Pol::Out;

    // nodes per direction (compile time: the padded node count fixes the order)
    constexpr int K1 = NNP == 32 ? 3 : (NNP == 64 ? 4 : 5);
    constexpr int NQ = K1 * K1 * K1;  // quadrature points = nodes
    constexpr int TPQ = 256 / QS;     // threads per quadrature point in the gradient stage
    constexpr int NPT = NNP / TPQ;    // nodes per thread in the gradient stage
    static_assert(256 % QS == 0 && NNP % TPQ == 0, "gradient stage shape");
    const int nn = NQ, nloc = s.nloc;
    const int64_t cell = bid / parts;
    const int part = int(bid % parts);
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;

    __shared__ double sX[8][3];
    __shared__ double sL[K1 * K1], sD[K1 * K1];
    // geometry of every quadrature point of the cell
    __shared__ double sJi[NQ][9];
    __shared__ double sW[NQ], sGf[NQ][NC];
    __shared__ int sBad;
    // gradients of a slab of points, and their weights
    __shared__ __attribute__((aligned(16))) S sG[DIM][QS][NNP];
    __shared__ S sWs[QS];

    if (tid < 8) {
        const int64_t e0 = cell % m.n0, e1 = (cell / m.n0) % m.n1, e2 = cell / (int64_t(m.n0) * m.n1);
        const int64_t vid = (e0 + (tid & 1)) + int64_t(m.n0 + 1) * ((e1 + ((tid >> 1) & 1)) + int64_t(m.n1 + 1) * (e2 + ((tid >> 2) & 1)));
        sX[tid][0] = m.x[vid];
        sX[tid][1] = m.y[vid];
        sX[tid][2] = m.z[vid];
    }
    if (tid < K1 * K1) {
        sL[tid] = rt.L[tid];
        sD[tid] = rt.D[tid];
    }
    if (tid == 0) sBad = 0;
    const double coef = m.coef ? m.coef[cell] : 1.0;
    __syncthreads();
    for (int q = tid; q < NQ; q += 256) {
        const int a0 = q % K1, a1 = (q / K1) % K1, a2 = q / (K1 * K1);
        const double xi[3] = {rt.gx[a0], rt.gx[a1], rt.gx[a2]};
        double Xl[8][3], Ji[9], xq[3];
        for (int v = 0; v < 8; v++)
            for (int r = 0; r < 3; r++) Xl[v][r] = sX[v][r];
        const double det = geometry_mf<DIM>(Xl, xi, Ji, xq);
        if (!(det > 0.0)) sBad = 1;
        const double wd = rt.gw[a0] * rt.gw[a1] * rt.gw[a2] * fabs(det);
        sW[q] = wd * coef;
        for (int t = 0; t < 9; t++) sJi[q][t] = Ji[t];
        for (int c = 0; c < NC; c++) sGf[q][c] = wd * source_value_mf(p, xq, c);
    }
    __syncthreads();

    // tile pairs of this wave
    int pta[PPW], ptb[PPW];
    bool pok[PPW];
#pragma unroll
    for (int t = 0; t < PPW; t++) {
        const int pidx = (part * NW + wave) + t * (parts * NW);
        pok[t] = pidx < NP;
        pair_tiles(pok[t] ? pidx : 0, NT, pta[t], ptb[t]);
    }
    Acc acc[PPW][NCP];
#pragma unroll
    for (int t = 0; t < PPW; t++)
#pragma unroll
        for (int c = 0; c < NCP; c++) acc[t][c] = Pol::zero();
    const bool do_load = (part == 0);
    double facc[(NNP * NC + 255) / 256];
#pragma unroll
    for (int t = 0; t < (NNP * NC + 255) / 256; t++) facc[t] = 0.0;

    const int i16 = lane % 16, g4 = lane / 16;
    // gradient stage: thread -> (point qq of the slab, nodes sub, sub + TPQ, ...)
    const int gq = tid / TPQ, gsub = tid % TPQ;
    for (int q0s = 0; q0s < NQ; q0s += QS) {
        const int qn = min(QS, NQ - q0s);
        {
            const int q = q0s + gq;
            const bool live = gq < qn;
            double Ji[9];
            int b0 = 0, b1 = 0, b2 = 0;
            double w = 0.0;
            if (live) {
#pragma unroll
                for (int t = 0; t < 9; t++) Ji[t] = sJi[q][t];
                b0 = q % K1;
                b1 = (q / K1) % K1;
                b2 = q / (K1 * K1);
                w = sW[q];
            }
#pragma unroll
            for (int j = 0; j < NPT; j++) {
                const int node = gsub + TPQ * j;
                double g[3] = {0.0, 0.0, 0.0};
                if (live && node < nn) {
                    const int n0 = node % K1, n1 = (node / K1) % K1, n2 = node / (K1 * K1);
                    const double L0 = sL[n0 * K1 + b0], L1 = sL[n1 * K1 + b1], L2 = sL[n2 * K1 + b2];
                    const double gr[3] = {sD[n0 * K1 + b0] * L1 * L2, L0 * sD[n1 * K1 + b1] * L2,
                                          L0 * L1 * sD[n2 * K1 + b2]};
#pragma unroll
                    for (int c = 0; c < 3; c++) g[c] = Ji[0 * 3 + c] * gr[0] + Ji[1 * 3 + c] * gr[1] + Ji[2 * 3 + c] * gr[2];
                }
#pragma unroll
                for (int c = 0; c < 3; c++) sG[c][gq][node] = S(g[c]);
            }
            if (gsub == 0) sWs[gq] = S(w);
        }
        __syncthreads();
        // MFMA over the slab
#pragma unroll
        for (int t = 0; t < PPW; t++) {
            if (!pok[t]) continue;
            const int ra = pta[t] * 16 + i16, rb = ptb[t] * 16 + i16;
            for (int k0 = 0; k0 < QS; k0 += Pol::KM) {
                const int kq = k0 + g4;
                const S wk = sWs[kq];
                S av[DIM], bv[DIM];
#pragma unroll
                for (int c = 0; c < DIM; c++) {
                    av[c] = sG[c][kq][ra];
                    bv[c] = wk * sG[c][kq][rb];
                }
                if (PROB == 0) {
#pragma unroll
                    for (int c = 0; c < DIM; c++) acc[t][0] = Pol::mma(av[c], bv[c], acc[t][0]);
                } else {
#pragma unroll
                    for (int c1 = 0; c1 < DIM; c1++)
#pragma unroll
                        for (int c2 = 0; c2 < DIM; c2++)
                            acc[t][c1 * DIM + c2] = Pol::mma(av[c1], bv[c2], acc[t][c1 * DIM + c2]);
                }
            }
        }
        // load vector (FP64, VALU) on the part-0 workgroup
        if (do_load) {
#pragma unroll
            for (int t = 0; t < (NNP * NC + 255) / 256; t++) {
                const int row = tid + 256 * t;
                if (row < nloc) {
                    const int a = row / NC, c = row % NC;
                    const int n0 = a % K1, n1 = (a / K1) % K1, n2 = a / (K1 * K1);
                    for (int qq = 0; qq < qn; qq++) {
                        const int q = q0s + qq;
                        const int b0 = q % K1, b1 = (q / K1) % K1, b2 = q / (K1 * K1);
                        const double phi = sL[n0 * K1 + b0] * sL[n1 * K1 + b1] * sL[n2 * K1 + b2];
                        facc[t] = __fma_rn(sGf[q][c], phi, facc[t]);
                    }
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0 && sBad) atomicOr(m.status, 1);
    Out *Ec = E + cell * int64_t(nloc) * nloc;
#pragma unroll
    for (int t = 0; t < PPW; t++) {
        if (!pok[t]) continue;
        const int col = ptb[t] * 16 + i16;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int row = pta[t] * 16 + (Pol::ROW_INTERLEAVED ? 4 * r + g4 : 4 * g4 + r);
            if (row >= nn || col >= nn) continue;
            // on a diagonal tile only the upper triangle is taken, and mirrored,
            // so the element matrix is exactly symmetric in every precision
            const bool diag = pta[t] == ptb[t];
            if (diag && row > col) continue;
            if (PROB == 0) {
                const Out v = Out(double(acc[t][0][r]));
                Ec[int64_t(row) * nloc + col] = v;
                if (row != col) Ec[int64_t(col) * nloc + row] = v;
            } else {
                double tr = 0.0;
#pragma unroll
                for (int l = 0; l < DIM; l++) tr += double(acc[t][l * DIM + l][r]);
#pragma unroll
                for (int c1 = 0; c1 < DIM; c1++)
#pragma unroll
                    for (int c2 = 0; c2 < DIM; c2++) {
                        if (row == col && c1 > c2) continue;
                        const double v = el_value(p.lambda, p.mu, double(acc[t][c1 * DIM + c2][r]),
                                                  double(acc[t][c2 * DIM + c1][r]), tr, c1 == c2);
                        const Out o = Out(v);
                        Ec[int64_t(row * NC + c1) * nloc + col * NC + c2] = o;
                        if (row != col || c1 != c2) Ec[int64_t(col * NC + c2) * nloc + row * NC + c1] = o;
                    }
            }
        }
    }
    if (do_load) {
#pragma unroll
        for (int t = 0; t < (NNP * NC + 255) / 256; t++) {
            const int row = tid + 256 * t;
            if (row < nloc) F[cell * nloc + row] = facc[t];
        }
    }
}

template <class Pol, int PROB, int NNP, int PPW, int QS>
__global__ __launch_bounds__(256, 2) void k3_mfma_kernel(SpaceArgs s, MeshArgs m, ProblemArgs p, RefTables rt, int parts,
                                                      typename Pol::Out *__restrict__ E, double *__restrict__ F)
{
    k3_mfma_body<Pol, PROB, NNP, PPW, QS>(s, m, p, rt, parts, E, F, xcd_block(blockIdx.x, gridDim.x));
}

template <class Pol, int PROB, int NNP, int PPW, int QS>
__global__ __launch_bounds__(256, 2) void k3_mfma_batch_kernel(const AsmJob *__restrict__ jobs,
                                                             const int32_t *__restrict__ boff, int njobs)
{
    int64_t lb, nb;
    const AsmJob &J = jobs[find_job(boff, njobs, lb, nb)];
    k3_mfma_body<Pol, PROB, NNP, PPW, QS>(J.s, J.m, J.p, J.rt, J.parts, static_cast<typename Pol::Out *>(J.E), J.F,
                                          lb);
}

// ---------------------------------------------------------------------------
// FP16 / BF16 operands: one workgroup per cell.  With the operand
// sqrt(w_q) G[(c,q)][a] both GEMM operands are the same array, so the scaled
// gradients of all the cell's points fit in LDS at once (Q4: 3 x 128 nodes x
// 128 points x 2 bytes, rows padded by 16 bytes so that the 16 rows a
// quarter-wave reads sit in distinct banks).  They are computed once per cell;
// then each wave takes whole node-tile pairs in turn, accumulates the pair's
// blocks over all points and stores them, so no accumulator outlives its pair
// and no workgroup repeats another's gradients.  A pair's block goes out
// through a per-wave LDS chunk of 8 node rows (16 for Poisson), written as
// rows of the block and of its mirror, consecutive lanes on consecutive
// addresses: stored straight from the accumulators, one store instruction
// touches up to 32 rows and makes some 28 write requests to L2, which then
// bounds the kernel.  The operand is scaled by a
// power of two per cell (~ h / sqrt(max_q w_q)) so that it sits near 1; the
// product is unscaled exactly.  The load vector is the FP64 sum of the slab
// kernel, in the same order.
template <int NNP>
struct Cell16Shape {
    static constexpr int K1 = NNP == 32 ? 3 : (NNP == 64 ? 4 : 5);
    static constexpr int NQ = K1 * K1 * K1;
    static constexpr int NQP = (NQ + 31) / 32 * 32;  // points padded to the MFMA depth
    static constexpr int PITCH = NQP + 8;            // LDS row pitch (elements)
    static constexpr int NTH = NNP == 128 ? 512 : 256;
    static constexpr int WPE = NNP == 32 ? 4 : NNP == 64 ? 3 : 1;  // waves per SIMD the registers must allow
};

template <class Pol, int PROB, int NNP>
__device__ __forceinline__ void k3_cell16_body(const SpaceArgs &s, const MeshArgs &m, const ProblemArgs &p,
                                               const RefTables &rt, typename Pol::Out *__restrict__ E,
                                               double *__restrict__ F, int64_t cell)
{
    constexpr int DIM = 3;
    using Sh = Cell16Shape<NNP>;
    constexpr int K1 = Sh::K1, NQ = Sh::NQ, NQP = Sh::NQP, PITCH = Sh::PITCH, NTH = Sh::NTH, NW = NTH / 64;
    constexpr int NT = NNP / 16;
    constexpr int NP = NT * (NT + 1) / 2;
    constexpr int NC = PROB == 1 ? DIM : 1;
    constexpr int NCP = PROB == 1 ? DIM * DIM : 1;
    constexpr int TPQ = NTH / NQP;  // threads per point in the gradient stage
    static_assert(NTH % NQP == 0 && NNP % TPQ == 0, "gradient stage shape");
    constexpr int CH = PROB == 1 ? 8 : 16;        // node rows per output chunk
    constexpr int BC = 16 * NC, BP = BC + 1;      // block columns, staging pitch
    constexpr int CHR = CH * NC;                  // block rows per chunk
    constexpr int RPI = 64 / BC, MPI = 64 / CHR;  // rows per store instruction (block, mirror)
    static_assert(CHR % RPI == 0 && BC % MPI == 0, "output chunk shape");
    using S = typename Pol::S;
    using V = typename Pol::V;
    using Acc = typename Pol::Acc;
    using Out = typename Pol::Out;
    const int nn = NQ, nloc = s.nloc;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;

    __shared__ double sX[8][3];
    __shared__ double sL[K1 * K1], sD[K1 * K1];
    __shared__ double sJi[NQ][9];
    __shared__ double sW[NQ], sGf[NQ][NC];
    __shared__ double sDet0, sAlpha;
    __shared__ int sBad;
    __shared__ __attribute__((aligned(16))) S sG[DIM][NNP][PITCH];
    __shared__ Out sStage[NW][CHR * BP];

    if (tid < 8) {
        const int64_t e0 = cell % m.n0, e1 = (cell / m.n0) % m.n1, e2 = cell / (int64_t(m.n0) * m.n1);
        const int64_t vid = (e0 + (tid & 1)) + int64_t(m.n0 + 1) * ((e1 + ((tid >> 1) & 1)) + int64_t(m.n1 + 1) * (e2 + ((tid >> 2) & 1)));
        sX[tid][0] = m.x[vid];
        sX[tid][1] = m.y[vid];
        sX[tid][2] = m.z[vid];
    }
    if (tid < K1 * K1) {
        sL[tid] = rt.L[tid];
        sD[tid] = rt.D[tid];
    }
    if (tid == 0) sBad = 0;
    const double coef = m.coef ? m.coef[cell] : 1.0;
    __syncthreads();
    for (int q = tid; q < NQ; q += NTH) {
        const int a0 = q % K1, a1 = (q / K1) % K1, a2 = q / (K1 * K1);
        const double xi[3] = {rt.gx[a0], rt.gx[a1], rt.gx[a2]};
        double Xl[8][3], Ji[9], xq[3];
        for (int v = 0; v < 8; v++)
            for (int r = 0; r < 3; r++) Xl[v][r] = sX[v][r];
        const double det = geometry_mf<DIM>(Xl, xi, Ji, xq);
        if (!(det > 0.0)) sBad = 1;
        const double wd = rt.gw[a0] * rt.gw[a1] * rt.gw[a2] * fabs(det);
        sW[q] = wd * coef;
        for (int t = 0; t < 9; t++) sJi[q][t] = Ji[t];
        for (int c = 0; c < NC; c++) sGf[q][c] = wd * source_value_mf(p, xq, c);
        if (q == 0) sDet0 = det;
    }
    __syncthreads();
    if (wave == 0) {
        double wmax = 0.0;
        for (int q = lane; q < NQ; q += 64) wmax = fmax(wmax, sW[q]);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) wmax = fmax(wmax, __shfl_xor(wmax, off));
        if (lane == 0) {
            const double h = cbrt(fabs(sDet0) > 0.0 ? fabs(sDet0) : 1.0);
            sAlpha = wmax > 0.0 ? exp2(floor(log2(h / sqrt(wmax)))) : 1.0;
        }
    }
    __syncthreads();
    const double alpha = sAlpha;

    // scaled gradients of every point: thread -> (point gq, node lines u =
    // n1 + K1 n2 from gsub in steps of TPQ, each line K1 nodes along the
    // first axis, whose 1D values at the point stay in registers);
    // consecutive lanes write consecutive points of one node row
    {
        const int gq = tid % NQP, gsub = tid / NQP;
        const bool live = gq < NQ;
        double Ji[9] = {};
        double sw = 0.0;
        int b0 = 0, b1 = 0, b2 = 0;
        if (live) {
#pragma unroll
            for (int t = 0; t < 9; t++) Ji[t] = sJi[gq][t];
            b0 = gq % K1;
            b1 = (gq / K1) % K1;
            b2 = gq / (K1 * K1);
            sw = sqrt(sW[gq]) * alpha;
        }
        double La[K1], Da[K1];
#pragma unroll
        for (int n = 0; n < K1; n++) {
            La[n] = sL[n * K1 + b0];
            Da[n] = sD[n * K1 + b0];
        }
#pragma unroll 1
        for (int u = gsub; u < K1 * K1; u += TPQ) {
            const int n1 = u % K1, n2 = u / K1;
            const double L1 = sL[n1 * K1 + b1], D1 = sD[n1 * K1 + b1];
            const double L2 = sL[n2 * K1 + b2], D2 = sD[n2 * K1 + b2];
#pragma unroll
            for (int n0 = 0; n0 < K1; n0++) {
                const double L0 = La[n0];
                const double gr[3] = {Da[n0] * L1 * L2, L0 * D1 * L2, L0 * L1 * D2};
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    const double g = Ji[0 * 3 + c] * gr[0] + Ji[1 * 3 + c] * gr[1] + Ji[2 * 3 + c] * gr[2];
                    sG[c][n0 + K1 * u][gq] = Pol::cvt(live ? g * sw : 0.0);
                }
            }
        }
        // node rows past the last node are zero
        for (int node = nn + gsub; node < NNP; node += TPQ)
#pragma unroll
            for (int c = 0; c < 3; c++) sG[c][node][gq] = S(0.0);
    }
    __syncthreads();
    if (tid == 0 && sBad) atomicOr(m.status, 1);

    const int i16 = lane % 16, g4 = lane / 16;
    const double unscale = 1.0 / (alpha * alpha);
    Out *Ec = E + cell * int64_t(nloc) * nloc;
    for (int pidx = wave; pidx < NP; pidx += NW) {
        int ta, tb;
        pair_tiles(pidx, NT, ta, tb);
        const int ra = ta * 16 + i16, rb = tb * 16 + i16;
        Acc acc[NCP];
#pragma unroll
        for (int c = 0; c < NCP; c++) acc[c] = Pol::zero();
#pragma unroll
        for (int k0 = 0; k0 < NQP; k0 += Pol::KM) {
            V av[DIM], bv[DIM];
#pragma unroll
            for (int c = 0; c < DIM; c++) {
                av[c] = *reinterpret_cast<const V *>(&sG[c][ra][k0 + 8 * g4]);
                bv[c] = *reinterpret_cast<const V *>(&sG[c][rb][k0 + 8 * g4]);
            }
            if (PROB == 0) {
#pragma unroll
                for (int c = 0; c < DIM; c++) acc[0] = Pol::mma(av[c], bv[c], acc[0]);
            } else {
#pragma unroll
                for (int c1 = 0; c1 < DIM; c1++)
#pragma unroll
                    for (int c2 = 0; c2 < DIM; c2++)
                        acc[c1 * DIM + c2] = Pol::mma(av[c1], bv[c2], acc[c1 * DIM + c2]);
            }
        }
        // The staged chunk holds block rows (rl - ch0) NC + c1, columns
        // i16 NC + c2; on a diagonal tile only entries with block row <=
        // block column are computed (the upper triangle), the rest is their
        // mirror.  The wave's LDS operations run in order, so fences at
        // wavefront scope order the lanes' writes and reads.
        const int col = tb * 16 + i16;
        const bool diag = ta == tb;
        Out *stg = sStage[wave];
#pragma unroll
        for (int ch0 = 0; ch0 < 16; ch0 += CH) {
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int rl = 4 * g4 + r, row = ta * 16 + rl;
                if (rl < ch0 || rl >= ch0 + CH || row >= nn || col >= nn) continue;
                if (diag && row > col) continue;
                Out *st = stg + (rl - ch0) * NC * BP + i16 * NC;
                if (PROB == 0) {
                    st[0] = Out(double(acc[0][r]) * unscale);
                } else {
                    double tr = 0.0;
#pragma unroll
                    for (int l = 0; l < DIM; l++) tr += double(acc[l * DIM + l][r]);
#pragma unroll
                    for (int c1 = 0; c1 < DIM; c1++)
#pragma unroll
                        for (int c2 = 0; c2 < DIM; c2++) {
                            if (row == col && c1 > c2) continue;
                            const double v = el_value(p.lambda, p.mu, double(acc[c1 * DIM + c2][r]),
                                                      double(acc[c2 * DIM + c1][r]), tr, c1 == c2);
                            st[c1 * BP + c2] = Out(v * unscale);
                        }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // block rows: RPI rows per store instruction, a lane keeps its
            // column; mirror rows (block columns): MPI per instruction.  All
            // staged values are read first (lanes beyond RPI or MPI read row
            // or column 0 and store nothing), so the LDS reads are in flight
            // together and the stores wait on none of them one by one.
            const int I0 = (ta * 16 + ch0) * NC, J0 = tb * 16 * NC;
            const int rsub = lane / BC, rj = lane - rsub * BC, rs = rsub < RPI ? rsub : 0;
            const int msub = lane / CHR, mi = lane - msub * CHR, ms = msub < MPI ? msub : 0;
            Out vr[CHR / RPI], vm[BC / MPI];
#pragma unroll
            for (int it = 0; it < CHR / RPI; it++) vr[it] = stg[(it * RPI + rs) * BP + rj];
#pragma unroll
            for (int it = 0; it < BC / MPI; it++) vm[it] = stg[mi * BP + it * MPI + ms];
            {
                const int J = J0 + rj;
                if (rsub < RPI && J < nloc)
#pragma unroll
                    for (int it = 0; it < CHR / RPI; it++) {
                        const int I = I0 + it * RPI + rsub;
                        if (I < nloc && !(diag && J < I)) Ec[I * nloc + J] = vr[it];
                    }
            }
            {
                const int I = I0 + mi;
                if (msub < MPI && I < nloc)
#pragma unroll
                    for (int it = 0; it < BC / MPI; it++) {
                        const int J = J0 + it * MPI + msub;
                        if (J < nloc && !(diag && J <= I)) Ec[J * nloc + I] = vm[it];
                    }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    // load vector (FP64, VALU): the points in ascending order, each term
    // (w |det J| f_c(x_q)) phi_a(x_q) rounded as in the slab kernel; the
    // point factors were formed once per cell and a row keeps its 1D basis
    // values in registers.  Rows go first to the upper half of the waves,
    // which were given no more tile pairs than the lower half.
#pragma unroll 1
    for (int row = (tid + NTH / 2) % NTH; row < nloc; row += NTH) {
        const int a = row / NC, c = row % NC;
        const int n0 = a % K1, n1 = (a / K1) % K1, n2 = a / (K1 * K1);
        double L0[K1], L1[K1];
#pragma unroll
        for (int b = 0; b < K1; b++) {
            L0[b] = sL[n0 * K1 + b];
            L1[b] = sL[n1 * K1 + b];
        }
        double f = 0.0;
#pragma unroll 1
        for (int b2 = 0; b2 < K1; b2++) {
            const double L2 = sL[n2 * K1 + b2];
            const double *g = &sGf[K1 * K1 * b2][c];
#pragma unroll
            for (int b1 = 0; b1 < K1; b1++)
#pragma unroll
                for (int b0 = 0; b0 < K1; b0++) f = __fma_rn(g[(K1 * b1 + b0) * NC], L0[b0] * L1[b1] * L2, f);
        }
        F[cell * nloc + row] = f;
    }
}

template <class Pol, int PROB, int NNP>
__global__ __launch_bounds__(Cell16Shape<NNP>::NTH, Cell16Shape<NNP>::WPE) void k3_cell16_kernel(SpaceArgs s, MeshArgs m, ProblemArgs p,
                                                                            RefTables rt,
                                                                            typename Pol::Out *__restrict__ E,
                                                                            double *__restrict__ F)
{
    k3_cell16_body<Pol, PROB, NNP>(s, m, p, rt, E, F, xcd_block(blockIdx.x, gridDim.x));
}

template <class Pol, int PROB, int NNP>
__global__ __launch_bounds__(Cell16Shape<NNP>::NTH, Cell16Shape<NNP>::WPE) void k3_cell16_batch_kernel(const AsmJob *__restrict__ jobs,
                                                                                  const int32_t *__restrict__ boff,
                                                                                  int njobs)
{
    int64_t lb, nb;
    const AsmJob &J = jobs[find_job(boff, njobs, lb, nb)];
    k3_cell16_body<Pol, PROB, NNP>(J.s, J.m, J.p, J.rt, static_cast<typename Pol::Out *>(J.E), J.F, lb);
}

template <class Pol, int PROB, int NNP>
static fe_status launch_cell16_one(const SpaceArgs &sa, const MeshArgs &ma, const ProblemArgs &pa,
                                   const RefTables &rt, void *E, double *F, hipStream_t s)
{
    if (sa.ncells == 0) return FE_OK;
    hipLaunchKernelGGL((k3_cell16_kernel<Pol, PROB, NNP>), dim3(unsigned(sa.ncells)), dim3(Cell16Shape<NNP>::NTH), 0, s,
                       sa, ma, pa, rt, static_cast<typename Pol::Out *>(E), F);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

template <class Pol, int PROB, int NNP>
static fe_status launch_cell16_batch_one(const AsmJob *jobs, const int32_t *boff, int njobs, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((k3_cell16_batch_kernel<Pol, PROB, NNP>), dim3(grid), dim3(Cell16Shape<NNP>::NTH), 0, s, jobs,
                       boff, njobs);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

// Calls body.template operator()<PROB, NNP>() for (order, problem).
template <class Body>
static fe_status with_cell16(int k, bool el, Body body)
{
    switch (k * 2 + (el ? 1 : 0)) {
        case 2 * 2 + 0: return body.template operator()<0, 32>();
        case 2 * 2 + 1: return body.template operator()<1, 32>();
        case 3 * 2 + 0: return body.template operator()<0, 64>();
        case 3 * 2 + 1: return body.template operator()<1, 64>();
        case 4 * 2 + 0: return body.template operator()<0, 128>();
        case 4 * 2 + 1: return body.template operator()<1, 128>();
        default: return set_error(FE_EINVAL, "matrix-core integration needs order 2..4");
    }
}

template <class Pol>
struct Cell16Single {
    const SpaceArgs &sa;
    const MeshArgs &ma;
    const ProblemArgs &pa;
    const RefTables &rt;
    void *E;
    double *F;
    hipStream_t s;
    template <int PROB, int NNP>
    fe_status operator()() const
    {
        return launch_cell16_one<Pol, PROB, NNP>(sa, ma, pa, rt, E, F, s);
    }
};

template <class Pol>
struct Cell16Batch {
    const AsmJob *jobs;
    const int32_t *boff;
    int njobs, grid;
    hipStream_t s;
    template <int PROB, int NNP>
    fe_status operator()() const
    {
        return launch_cell16_batch_one<Pol, PROB, NNP>(jobs, boff, njobs, grid, s);
    }
};

// ---------------------------------------------------------------------------
// Launch shapes: node-tile pairs per wave (PPW; parts per cell follow) for
// (order, problem, precision).  Every shape sums each entry over the
// quadrature points in the same order, so the element matrices do not depend
// on it; the autotuner (fe_integrate_autotune) times the candidates of a
// class and keeps the fastest for the process.  Defaults measured on 32^3 Q3
// and 24^3 Q4 elasticity (Q3: 3.75 ms with one pair per wave against 5.57 ms
// with two).  FP64 Q4 elasticity runs one pair per wave (10.0 ms): two need
// more than 256 VGPRs and spill to private memory, and a variant of that
// kernel with more spills gave element matrices that differed from run to
// run, so no kernel here spills.  FP16 / BF16 have the one shape of the
// whole-cell kernel.
// ---------------------------------------------------------------------------
static std::mutex g_k3_mu;
static std::map<int, int> g_k3_tuned;  // class -> pairs per wave

static int k3_class(int k, bool el, int prec) { return (k * 2 + (el ? 1 : 0)) * 8 + prec; }

static bool whole_cell(int prec) { return prec == FE_FP16 || prec == FE_BF16; }

static int nnp_of(int k) { return k == 2 ? 32 : (k == 3 ? 64 : 128); }

// FP16 / BF16 run the whole-cell kernel, one shape per class: its waves take
// the node-tile pairs in turn (reported as the most pairs a wave takes).
static int cell16_ppw(int k)
{
    const int nt = nnp_of(k) / 16, np = nt * (nt + 1) / 2, nw = (k == 4 ? 512 : 256) / 64;
    return (np + nw - 1) / nw;
}

static std::vector<int> k3_candidates(int k, bool el, int prec)
{
    if (whole_cell(prec)) return {cell16_ppw(k)};
    if (k == 2) return {1};
    if (k == 3) return el ? std::vector<int>{1, 2} : std::vector<int>{1, 2, 3};
    if (el) return prec == FE_FP64 ? std::vector<int>{1} : std::vector<int>{1, 2};
    return {3, 5, 9};
}

static int k3_default(int k, bool el, int prec)
{
    if (whole_cell(prec)) return cell16_ppw(k);
    if (k == 3) return el ? 1 : 3;
    if (k == 4) return el ? (prec == FE_FP64 ? 1 : 2) : 9;
    return 1;
}

static int k3_ppw(int k, bool el, int prec)
{
    std::lock_guard<std::mutex> lk(g_k3_mu);
    auto it = g_k3_tuned.find(k3_class(k, el, prec));
    return it != g_k3_tuned.end() ? it->second : k3_default(k, el, prec);
}

static int parts_of(int k, int ppw)
{
    const int nt = nnp_of(k) / 16, np = nt * (nt + 1) / 2;
    return (np + 4 * ppw - 1) / (4 * ppw);
}

// Workgroups per cell of the shape (ppw) of a class.
static int parts_for(int k, int prec, int ppw) { return whole_cell(prec) ? 1 : parts_of(k, ppw); }

template <class Pol, int PROB, int NNP, int PPW, int QS>
static fe_status launch_one(const SpaceArgs &sa, const MeshArgs &ma, const ProblemArgs &pa, const RefTables &rt,
                            void *E, double *F, hipStream_t s)
{
    const int parts = parts_of(sa.k, PPW);
    const int64_t grid = sa.ncells * parts;
    if (grid == 0) return FE_OK;
    hipLaunchKernelGGL((k3_mfma_kernel<Pol, PROB, NNP, PPW, QS>), dim3(grid), dim3(256), 0, s, sa, ma, pa, rt, parts,
                       static_cast<typename Pol::Out *>(E), F);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

template <class Pol, int PROB, int NNP, int PPW, int QS>
static fe_status launch_batch_one(const AsmJob *jobs, const int32_t *boff, int njobs, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((k3_mfma_batch_kernel<Pol, PROB, NNP, PPW, QS>), dim3(grid), dim3(256), 0, s, jobs, boff,
                       njobs);
    FE_HIP(hipGetLastError());
    return FE_OK;
}

// Calls body.template operator()<PROB, NNP, PPW>() for the class's shape.
template <class Body>
static fe_status with_shape(int k, bool el, int ppw, Body body)
{
    switch ((k * 2 + (el ? 1 : 0)) * 16 + ppw) {
        case (2 * 2 + 0) * 16 + 1: return body.template operator()<0, 32, 1>();
        case (2 * 2 + 1) * 16 + 1: return body.template operator()<1, 32, 1>();
        case (3 * 2 + 0) * 16 + 1: return body.template operator()<0, 64, 1>();
        case (3 * 2 + 0) * 16 + 2: return body.template operator()<0, 64, 2>();
        case (3 * 2 + 0) * 16 + 3: return body.template operator()<0, 64, 3>();
        case (3 * 2 + 1) * 16 + 1: return body.template operator()<1, 64, 1>();
        case (3 * 2 + 1) * 16 + 2: return body.template operator()<1, 64, 2>();
        case (4 * 2 + 0) * 16 + 3: return body.template operator()<0, 128, 3>();
        case (4 * 2 + 0) * 16 + 5: return body.template operator()<0, 128, 5>();
        case (4 * 2 + 0) * 16 + 9: return body.template operator()<0, 128, 9>();
        case (4 * 2 + 1) * 16 + 1: return body.template operator()<1, 128, 1>();
        case (4 * 2 + 1) * 16 + 2: return body.template operator()<1, 128, 2>();
        default: return set_error(FE_EINVAL, "matrix-core integration needs order 2..4 and a candidate shape");
    }
}

// The shapes built for a precision: two pairs per wave at Q4 elasticity would
// need more than 256 VGPRs in FP64 (private-memory spills), so that shape is
// built for FP32 only.
template <class Pol, int PROB, int NNP, int PPW>
constexpr bool shape_built()
{
    return !(std::is_same<Pol, PolF64>::value && PROB == 1 && NNP == 128 && PPW == 2);
}

template <class Pol>
struct SingleLaunch {
    const SpaceArgs &sa;
    const MeshArgs &ma;
    const ProblemArgs &pa;
    const RefTables &rt;
    void *E;
    double *F;
    hipStream_t s;
    template <int PROB, int NNP, int PPW>
    fe_status operator()() const
    {
        if constexpr (shape_built<Pol, PROB, NNP, PPW>())
            return launch_one<Pol, PROB, NNP, PPW, 16>(sa, ma, pa, rt, E, F, s);
        else
            return set_error(FE_EINVAL, "tile shape not built for this precision");
    }
};

template <class Pol>
struct BatchLaunch {
    const AsmJob *jobs;
    const int32_t *boff;
    int njobs, grid;
    hipStream_t s;
    template <int PROB, int NNP, int PPW>
    fe_status operator()() const
    {
        if constexpr (shape_built<Pol, PROB, NNP, PPW>())
            return launch_batch_one<Pol, PROB, NNP, PPW, 16>(jobs, boff, njobs, grid, s);
        else
            return set_error(FE_EINVAL, "tile shape not built for this precision");
    }
};

static fe_status launch_with(const SpaceArgs &sa, const MeshArgs &ma, const ProblemArgs &pa, const RefTables &rt,
                             void *E, double *F, hipStream_t s, int ppw)
{
    const bool el = pa.problem == FE_ELASTICITY;
    if (sa.k < 2 || sa.k > 4) return set_error(FE_EINVAL, "matrix-core integration needs order 2..4");
    switch (pa.precision) {
        case FE_FP64: return with_shape(sa.k, el, ppw, SingleLaunch<PolF64>{sa, ma, pa, rt, E, F, s});
        case FE_FP32: return with_shape(sa.k, el, ppw, SingleLaunch<PolF32>{sa, ma, pa, rt, E, F, s});
        case FE_FP16: return with_cell16(sa.k, el, Cell16Single<PolF16>{sa, ma, pa, rt, E, F, s});
        default: return with_cell16(sa.k, el, Cell16Single<PolBF16>{sa, ma, pa, rt, E, F, s});
    }
}

fe_status launch_integrate_mfma(const SpaceArgs &sa, const MeshArgs &ma, const ProblemArgs &pa, const RefTables &rt,
                                void *E, double *F, hipStream_t s)
{
    return launch_with(sa, ma, pa, rt, E, F, s, k3_ppw(sa.k, pa.problem == FE_ELASTICITY, pa.precision));
}

// Batched: the class (precision, order, problem) is that of the host job h.
fe_status launch_mfma_batch(const AsmJob &h, const AsmJob *jobs, const int32_t *boff, int njobs, int grid,
                            hipStream_t s)
{
    const bool el = h.p.problem == FE_ELASTICITY;
    const int ppw = k3_ppw(h.s.k, el, h.p.precision);
    switch (h.p.precision) {
        case FE_FP64: return with_shape(h.s.k, el, ppw, BatchLaunch<PolF64>{jobs, boff, njobs, grid, s});
        case FE_FP32: return with_shape(h.s.k, el, ppw, BatchLaunch<PolF32>{jobs, boff, njobs, grid, s});
        case FE_FP16: return with_cell16(h.s.k, el, Cell16Batch<PolF16>{jobs, boff, njobs, grid, s});
        default: return with_cell16(h.s.k, el, Cell16Batch<PolBF16>{jobs, boff, njobs, grid, s});
    }
}

// Workgroups per cell of the matrix-core kernel (the shape launch_integrate_mfma uses now).
int64_t mfma_blocks(const SpaceArgs &sa, const ProblemArgs &pa, int32_t &parts)
{
    parts = parts_for(sa.k, pa.precision, k3_ppw(sa.k, pa.problem == FE_ELASTICITY, pa.precision));
    return sa.ncells * parts;
}

// Times every candidate shape of the class (reps launches after one warm-up)
// on this space and keeps the fastest.
fe_status integrate_autotune(const SpaceArgs &sa, const MeshArgs &ma, const ProblemArgs &pa, const RefTables &rt,
                             void *E, double *F, int reps, fe_k3_plan *tried, int max_tried, int *n_tried,
                             fe_k3_plan *chosen, hipStream_t s)
{
    if (sa.dim != 3 || sa.k < 2 || sa.k > 4) return set_error(FE_EINVAL, "no tile shapes to tune for this space");
    const bool el = pa.problem == FE_ELASTICITY;
    const std::vector<int> cand = k3_candidates(sa.k, el, pa.precision);
    hipEvent_t e0, e1;
    FE_HIP(hipEventCreate(&e0));
    FE_HIP(hipEventCreate(&e1));
    int best = -1;
    double best_us = 0.0;
    fe_status st = FE_OK;
    for (size_t c = 0; c < cand.size() && st == FE_OK; c++) {
        for (int r = -1; r < reps && st == FE_OK; r++) {
            if (r == 0 && hipEventRecord(e0, s) != hipSuccess) st = set_error(FE_EDEVICE, "event record failed");
            if (st == FE_OK) st = launch_with(sa, ma, pa, rt, E, F, s, cand[c]);
        }
        if (st != FE_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = set_error(FE_EDEVICE, "autotune timing failed");
            break;
        }
        const double us = 1000.0 * double(ms) / double(reps);
        if (tried && int(c) < max_tried) tried[c] = fe_k3_plan{cand[c], parts_for(sa.k, pa.precision, cand[c]), us};
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
        std::lock_guard<std::mutex> lk(g_k3_mu);
        g_k3_tuned[k3_class(sa.k, el, pa.precision)] = cand[best];
    }
    if (chosen) *chosen = fe_k3_plan{cand[best], parts_for(sa.k, pa.precision, cand[best]), best_us};
    return FE_OK;
}

void integrate_plan_of(const SpaceArgs &sa, const ProblemArgs &pa, fe_k3_plan *plan)
{
    const bool el = pa.problem == FE_ELASTICITY;
    const int ppw = (sa.dim == 3 && sa.k >= 2 && sa.k <= 4) ? k3_ppw(sa.k, el, pa.precision) : 0;
    *plan = fe_k3_plan{ppw, ppw ? parts_for(sa.k, pa.precision, ppw) : 0, 0.0};
}

void integrate_tuning_reset()
{
    std::lock_guard<std::mutex> lk(g_k3_mu);
    g_k3_tuned.clear();
}

}  // namespace fe
