// fe_geom.h -- device helpers for the order-1 cell geometry of the brick:
// the 2^d vertices of a cell and the map Phi, its Jacobian, determinant and
// inverse at a reference point (Sect. 3.7).  Used by the integration kernels
// and the facet kernels of the discontinuous Galerkin assembly.
#pragma once

#include "fe_internal.h"

namespace fe {

template <int DIM>
__device__ __forceinline__ void load_vertices(const MeshArgs &m, int64_t cell, double X[][3])
{
    const int64_t e0 = cell % m.n0, e1 = (cell / m.n0) % m.n1, e2 = cell / (int64_t(m.n0) * m.n1);
    const int64_t nx = m.n0 + 1, ny = m.n1 + 1;
#pragma unroll
    for (int v = 0; v < (1 << DIM); v++) {
        const int64_t vid = (e0 + (v & 1)) + nx * ((e1 + ((v >> 1) & 1)) + ny * (DIM == 3 ? e2 + ((v >> 2) & 1) : 0));
        X[v][0] = m.x[vid];
        X[v][1] = m.y[vid];
        X[v][2] = DIM == 3 ? m.z[vid] : 0.0;
    }
}

// J_rs = d Phi_r / d xi_s of the order-1 map, the physical point, det J and
// J^-1 (row-major) at reference point xi.
template <int DIM>
__device__ __forceinline__ double geometry(const double X[][3], const double xi[3], double J[9], double Ji[9],
                                           double xq[3])
{
#pragma unroll
    for (int t = 0; t < 9; t++) J[t] = 0.0;
    xq[0] = xq[1] = xq[2] = 0.0;
#pragma unroll
    for (int v = 0; v < (1 << DIM); v++) {
        double Nv = 1.0, dN[3];
#pragma unroll
        for (int r = 0; r < DIM; r++) Nv *= ((v >> r) & 1) ? xi[r] : 1.0 - xi[r];
#pragma unroll
        for (int sd = 0; sd < DIM; sd++) {
            double g = 1.0;
#pragma unroll
            for (int r = 0; r < DIM; r++)
                g *= (r == sd) ? (((v >> r) & 1) ? 1.0 : -1.0) : (((v >> r) & 1) ? xi[r] : 1.0 - xi[r]);
            dN[sd] = g;
        }
#pragma unroll
        for (int r = 0; r < DIM; r++) {
            xq[r] += X[v][r] * Nv;
#pragma unroll
            for (int sd = 0; sd < DIM; sd++) J[r * DIM + sd] += X[v][r] * dN[sd];
        }
    }
    double det;
    if (DIM == 2) {
        det = J[0] * J[3] - J[1] * J[2];
        const double id = 1.0 / det;
        Ji[0] = J[3] * id;
        Ji[1] = -J[1] * id;
        Ji[2] = -J[2] * id;
        Ji[3] = J[0] * id;
    } else {
        const double c00 = J[4] * J[8] - J[5] * J[7];
        const double c01 = J[5] * J[6] - J[3] * J[8];
        const double c02 = J[3] * J[7] - J[4] * J[6];
        det = J[0] * c00 + J[1] * c01 + J[2] * c02;
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
    }
    return det;
}

}  // namespace fe
