"""Pins of the oracle's interior-penalty DG assembly (Sect. 3.12), on the CPU.

* Box meshes: the whole matrix against an independent exact assembly from
  1D factors (tests/exact.py), for the symmetric method and two others (tau =
  0, -1), so the place of tau, the halves of the means, the signs of the
  normals and the penalty scale are all fixed.
* Jittered meshes: symmetric and positive definite (tau = 1, penalty large
  enough); the linear patch test (SIPG is consistent: an affine u_D with
  f = 0 is reproduced at every DOF, exactly up to rounding, since every
  integrand of an affine field is a polynomial the rules integrate exactly);
  O(h^(k+1)) L2 convergence of a smooth solution with weak Dirichlet data.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from fe_inputs import structured_vertices
from tests import exact as EX


def penalty(k):
    return 4.0 * (k + 1) ** 2


@pytest.mark.parametrize("dim,n,k", [(2, [2, 3], 1), (2, [3, 2], 3), (3, [2, 2, 1], 1), (3, [1, 2, 2], 2),
                                     (3, [2, 1, 1], 3), (2, [2, 2], 4)])
@pytest.mark.parametrize("tau", [1.0, 0.0, -1.0])
def test_dg_box_matrix_closed_form(dim, n, k, tau):
    P = O.Problem(dim, n, k)
    D = O.DGSystem(P, structured_vertices(dim, n), gamma=penalty(k), tau=tau)
    assert D.ok
    Ae = EX.dg_box_matrix(dim, k, n + [1] * (3 - len(n)), penalty(k), tau)
    Ao = D.dense()
    assert np.abs(Ao - Ae).max() <= 1e-13 * np.abs(Ae).max()
    # the pattern holds the blocks of a cell and of its facet neighbours: nn^2 (1 + neighbours) per cell
    nb = sum(1 + sum((c[r] > 0) + (c[r] < n[r] - 1) for r in range(dim))
             for c in (tuple(reversed(t)) for t in np.ndindex(*reversed(n))))
    assert D.nnz == nb * P.nn * P.nn


@pytest.mark.parametrize("dim,n,k", [(2, [4, 3], 1), (2, [3, 3], 2), (3, [3, 2, 2], 1), (3, [2, 2, 2], 2)])
def test_dg_symmetric_positive_definite_on_jittered_mesh(dim, n, k):
    P = O.Problem(dim, n, k, source_kind=1, source=(1.0,))
    D = O.DGSystem(P, structured_vertices(dim, n, jitter=0.2, seed=61), gamma=penalty(k))
    A = D.dense()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    np.linalg.cholesky(A)
    # a smaller penalty loses definiteness: the penalty is what makes it SPD
    D0 = O.DGSystem(P, structured_vertices(dim, n, jitter=0.2, seed=61), gamma=0.0)
    assert np.linalg.eigvalsh(D0.dense())[0] < 0


@pytest.mark.parametrize("dim,n,k", [(2, [3, 4], 1), (2, [3, 2], 3), (3, [2, 3, 2], 1), (3, [2, 2, 2], 2),
                                     (3, [2, 1, 2], 3)])
def test_dg_linear_patch_test(dim, n, k):
    aff = [0.3, 1.0, -2.0, 0.5]
    P = O.Problem(dim, n, k, source_kind=0, dirichlet_kind=1, dirichlet_affine=aff)
    v = structured_vertices(dim, n, jitter=0.2, seed=62)
    D = O.DGSystem(P, v, gamma=penalty(k))
    x = spla.spsolve(D.scipy().tocsc(), D.rhs)
    # every DOF (K, a) equals the affine field at its node Phi_K(a / k)
    for K in range(P.ncells):
        X = O.cell_vertices(dim, P.n, v, K)
        for a in range(P.nn):
            ar = [(a // (k + 1) ** r) % (k + 1) for r in range(dim)]
            t = np.array(ar) / k
            N = np.ones(1 << dim)
            for vv in range(1 << dim):
                for r in range(dim):
                    N[vv] *= t[r] if (vv >> r) & 1 else 1 - t[r]
            xn = N @ X
            ue = aff[0] + np.dot(aff[1:1 + dim], xn)
            assert abs(x[K * P.nn + a] - ue) <= 1e-11, (K, a, x[K * P.nn + a], ue)
    assert O.l2_error(P, v, D.cell_dofs, x, k + 3, 2, aff + [0.0] * 8) <= 1e-11


def _dg_rate(dim, k, ns, jitter=0.0):
    errs = []
    for n in ns:
        P = O.Problem(dim, [n] * dim, k, source_kind=2, source=(1.0,))
        v = structured_vertices(dim, n, jitter=jitter, seed=63 + n)
        D = O.DGSystem(P, v, gamma=penalty(k))
        x = spla.spsolve(D.scipy().tocsc(), D.rhs)
        errs.append(O.l2_error(P, v, D.cell_dofs, x, k + 3, 1, [1.0]))
    return errs, np.log(errs[-2] / errs[-1]) / np.log(ns[-1] / ns[-2])


@pytest.mark.parametrize("dim,k,ns,jitter", [(2, 1, [8, 16, 32], 0.0), (2, 2, [4, 8, 16], 0.2), (2, 3, [4, 8, 16], 0.0),
                                             (3, 1, [4, 8, 16], 0.0), (3, 2, [2, 4, 8], 0.2)])
def test_dg_l2_convergence_rate(dim, k, ns, jitter):
    errs, rate = _dg_rate(dim, k, ns, jitter)
    assert k + 1 - 0.2 <= rate <= k + 1 + 0.3, (errs, rate)
