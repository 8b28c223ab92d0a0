"""Exact (rational) closed forms used to pin the oracle.

Nothing here calls the oracle or the HIP library.  1D Lagrange polynomials on
equidistant nodes are built as exact rational coefficient lists, products are
integrated exactly on [0,1], and element matrices of affine cells follow from
the chain rule as Kronecker products of the 1D matrices

    S_ij = int l_i' l_j',   M_ij = int l_i l_j,   C_ij = int l_i' l_j.
"""
from fractions import Fraction as Fr

import numpy as np


def polymul(p, q):
    out = [Fr(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def polyder(p):
    return [i * p[i] for i in range(1, len(p))] or [Fr(0)]


def int01(p):
    return sum(c / (i + 1) for i, c in enumerate(p))


def lagrange_polys(k):
    nodes = [Fr(s, k) for s in range(k + 1)]
    polys = []
    for m in range(k + 1):
        p = [Fr(1)]
        den = Fr(1)
        for s in range(k + 1):
            if s == m:
                continue
            p = polymul(p, [-nodes[s], Fr(1)])
            den *= nodes[m] - nodes[s]
        polys.append([c / den for c in p])
    return polys


def polyval(p, x):
    return sum(float(c) * x ** i for i, c in enumerate(p))


def matrices_1d(k):
    """(S, M, C) as float arrays, computed exactly."""
    L = lagrange_polys(k)
    D = [polyder(p) for p in L]
    n = k + 1
    S = np.array([[float(int01(polymul(D[i], D[j]))) for j in range(n)] for i in range(n)])
    M = np.array([[float(int01(polymul(L[i], L[j]))) for j in range(n)] for i in range(n)])
    C = np.array([[float(int01(polymul(D[i], L[j]))) for j in range(n)] for i in range(n)])
    return S, M, C


def kron_axes(factors):
    """Kronecker product over axes with x fastest: factors[0] is the x factor."""
    out = factors[0]
    for f in factors[1:]:
        out = np.kron(f, out)
    return out


def ref_gradient_grams(dim, k):
    """G[s][t][a][b] = int_{[0,1]^d} d_s phi_a d_t phi_b for the tensor basis."""
    S, M, C = matrices_1d(k)
    G = [[None] * dim for _ in range(dim)]
    for s in range(dim):
        for t in range(dim):
            fac = []
            for r in range(dim):
                if r == s and r == t:
                    fac.append(S)
                elif r == s:
                    fac.append(C)
                elif r == t:
                    fac.append(C.T)
                else:
                    fac.append(M)
            G[s][t] = kron_axes(fac)
    return G


def affine_cell_vertices(x0, B):
    """Vertices X_v = x0 + B v, v in {0,1}^d, vertex index v0 + 2 v1 + 4 v2."""
    dim = len(x0)
    X = np.zeros((1 << dim, dim))
    for v in range(1 << dim):
        e = np.array([(v >> r) & 1 for r in range(dim)], dtype=float)
        X[v] = np.asarray(x0) + np.asarray(B) @ e
    return X


def affine_element(dim, k, B, problem="poisson", coef=1.0, lam=0.0, mu=0.0):
    """Exact element matrix of the affine cell x = x0 + B xi."""
    B = np.asarray(B, dtype=float)
    Binv = np.linalg.inv(B)
    det = abs(np.linalg.det(B))
    G = ref_gradient_grams(dim, k)
    nn = (k + 1) ** dim
    # H[i][j] = int d_i phi_a d_j phi_b  (physical derivatives)
    H = [[sum(Binv[s, i] * Binv[t, j] * G[s][t] for s in range(dim) for t in range(dim))
          for j in range(dim)] for i in range(dim)]
    if problem == "poisson":
        return coef * det * sum(H[i][i] for i in range(dim))
    nloc = nn * dim
    A = np.zeros((nloc, nloc))
    tr = sum(H[l][l] for l in range(dim))
    for i in range(dim):
        for j in range(dim):
            blk = lam * H[i][j] + mu * H[j][i] + (mu * tr if i == j else 0.0)
            A[i::dim, j::dim] = coef * det * blk
    return A


def mass_1d_load(k):
    """int l_i over [0,1] (exact)."""
    return np.array([float(int01(p)) for p in lagrange_polys(k)])
