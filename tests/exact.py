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


def lagrange_end_values(k):
    """(l_i(0), l_i(1), l_i'(0), l_i'(1)) for the equidistant Lagrange basis, exact."""
    P = lagrange_polys(k)
    v0 = [polyval(p, Fr(0)) for p in P]
    v1 = [polyval(p, Fr(1)) for p in P]
    d0 = [polyval(polyder(p), Fr(0)) for p in P]
    d1 = [polyval(polyder(p), Fr(1)) for p in P]
    return v0, v1, d0, d1


def dg_box_matrix(dim, k, n, gamma, tau):
    """The symmetric-interior-penalty DG matrix of -Laplace on the Cartesian
    brick of n[r] equal cells per axis of [0,1]^d (cell sides h_r = 1/n_r),
    DOF K nn + a, assembled from exact per-axis factors: a facet term is the
    Kronecker product of h_s M over the tangential axes with, across the
    normal axis r, the 1D endpoint factor of the facet's three terms
      - s_i l_a(e_i) n.l_b'(e_j) / (2 h_r) - tau s_j l_b(e_j) n.l_a'(e_i) / (2 h_r)
      + sigma s_i s_j l_a(e_i) l_b(e_j),  sigma = gamma / h_F,
    e_i the end of cell i at the facet, s = +1 (lower cell) / -1 (upper cell),
    h_F = h_s (2D) or sqrt(h_s h_t) (3D); boundary facets take s = 1 and the
    outward sign of the normal derivative, without the halves."""
    S, M, C = matrices_1d(k)
    v0, v1, d0, d1 = [np.array([float(t) for t in arr]) for arr in lagrange_end_values(k)]
    h = [1.0 / n[r] for r in range(dim)]
    nn = (k + 1) ** dim
    ncells = int(np.prod(n[:dim]))
    A = np.zeros((ncells * nn, ncells * nn))

    def cell_index(ci):
        return ci[0] + n[0] * (ci[1] + (n[1] * ci[2] if dim == 3 else 0))

    def face_block(r, normal_factor):
        facs = []
        for s_ in range(dim):
            facs.append(normal_factor if s_ == r else h[s_] * M)
        return kron_axes(facs)

    def sigma(r):
        tang = [h[s_] for s_ in range(dim) if s_ != r]
        hF = tang[0] if dim == 2 else np.sqrt(tang[0] * tang[1])
        return gamma / hF

    for K in range(ncells):
        ci = [K % n[0], (K // n[0]) % n[1], K // (n[0] * n[1]) if dim == 3 else 0][:dim]
        # volume: sum over axes of (S / h_r^2) on axis r and M on the others, times the cell volume
        vol = np.zeros((nn, nn))
        for r in range(dim):
            facs = [(S / h[r] ** 2 if s_ == r else M) for s_ in range(dim)]
            vol += kron_axes(facs)
        A[K * nn:(K + 1) * nn, K * nn:(K + 1) * nn] += vol * np.prod(h)
        for r in range(dim):
            sg = sigma(r)
            # upper side of K along r: interior facet with the neighbour, or boundary
            if ci[r] + 1 < n[r]:
                cj = list(ci)
                cj[r] += 1
                L = cell_index(cj)
                ends = {0: (v1, d1), 1: (v0, d0)}  # K sees the facet at 1, L at 0
                sgn = {0: 1.0, 1: -1.0}
                idx = {0: K, 1: L}
                for i in (0, 1):
                    for j in (0, 1):
                        vi, di = ends[i]
                        vj, dj = ends[j]
                        fac = (-sgn[i] * np.outer(vi, dj) / (2 * h[r]) - tau * sgn[j] * np.outer(di, vj) / (2 * h[r])
                               + sg * sgn[i] * sgn[j] * np.outer(vi, vj))
                        A[idx[i] * nn:(idx[i] + 1) * nn, idx[j] * nn:(idx[j] + 1) * nn] += face_block(r, fac)
            else:
                fac = -np.outer(v1, d1) / h[r] - tau * np.outer(d1, v1) / h[r] + sg * np.outer(v1, v1)
                A[K * nn:(K + 1) * nn, K * nn:(K + 1) * nn] += face_block(r, fac)
            if ci[r] == 0:  # lower boundary: outward normal -e_r
                fac = np.outer(v0, d0) / h[r] + tau * np.outer(d0, v0) / h[r] + sg * np.outer(v0, v0)
                A[K * nn:(K + 1) * nn, K * nn:(K + 1) * nn] += face_block(r, fac)
    return A


def mixed_matrices_1d(kp, ku):
    """1D matrices between the order-kp basis (rows) and the order-ku basis
    (columns), computed exactly: Mx_ij = int l^kp_i l^ku_j and
    Gx_ij = int l^kp_i (l^ku_j)'."""
    Lp, Lu = lagrange_polys(kp), lagrange_polys(ku)
    Du = [polyder(p) for p in Lu]
    Mx = np.array([[float(int01(polymul(Lp[i], Lu[j]))) for j in range(ku + 1)] for i in range(kp + 1)])
    Gx = np.array([[float(int01(polymul(Lp[i], Du[j]))) for j in range(ku + 1)] for i in range(kp + 1)])
    return Mx, Gx


def stokes_box_b_element(dim, k, h):
    """Divergence block -int psi_a d_c phi_b of an axis-aligned box cell with
    sides h (pressure order k, velocity order k+1, local velocity DOF
    dim b + c), and the pressure mass diagonal, as Kronecker products of the
    exact 1D matrices: the derivative along c brings 1/h_c, the measure h_c."""
    Mx, Gx = mixed_matrices_1d(k, k + 1)
    _, Mp, _ = matrices_1d(k)
    kp1, ku1 = k + 1, k + 2
    nnp, nnu = kp1 ** dim, ku1 ** dim
    B = np.zeros((nnp, dim * nnu))
    md = np.zeros(nnp)
    for a in range(nnp):
        ai = [(a // kp1 ** r) % kp1 for r in range(dim)]
        md[a] = np.prod([h[r] * Mp[ai[r], ai[r]] for r in range(dim)])
        for b in range(nnu):
            bi = [(b // ku1 ** r) % ku1 for r in range(dim)]
            for c in range(dim):
                v = 1.0
                for r in range(dim):
                    v *= Gx[ai[r], bi[r]] if r == c else h[r] * Mx[ai[r], bi[r]]
                B[a, dim * b + c] = -v
    return B, md
