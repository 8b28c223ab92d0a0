"""Pins of the oracle's Taylor-Hood Stokes system (the Stokes example of
Sect. 3.1, the Q_{k+1}^d x Q_k pair), on the CPU.

* The divergence block of an axis-aligned box cell against Kronecker products
  of exact 1D matrices (tests/exact.py), and its pressure mass diagonal.
* The assembled B annihilates constants: 1^T B = -int div v_h = 0 for every
  velocity that vanishes on the boundary (the pressure basis sums to one).
* Inf-sup on the brick: B has rank n_p - 1 (only the constant pressure mode
  in its left kernel), on uniform and jittered meshes.
* An exact solution: a constant body force f with zero velocity data is
  balanced by the pressure alone, u = 0 and p = f . x (up to a constant).
  The affine pressure lies in the mapped Q_k space and every integral
  involved is a polynomial the rule integrates exactly, so the discrete
  solution reproduces it to rounding on jittered meshes too.
"""
import numpy as np
import pytest

import oracle as O
from fe_inputs import structured_vertices
from tests import exact as EX


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_b_element_box_closed_form(dim, k):
    h = [0.5, 0.25, 0.2][:dim]
    X = np.array([[h[r] * ((v >> r) & 1) + 0.1 * r for r in range(dim)] for v in range(1 << dim)])
    B, md, ok = O.stokes_b_element(dim, k, X)
    Be, mde = EX.stokes_box_b_element(dim, k, h)
    assert ok
    assert np.abs(B - Be).max() <= 1e-14 * np.abs(Be).max()
    assert np.abs(md - mde).max() <= 1e-14 * np.abs(mde).max()


@pytest.mark.parametrize("dim,n,k,jit", [(2, [3, 4], 1, 0.2), (2, [3, 2], 2, 0.0), (3, [2, 2, 2], 1, 0.2),
                                         (3, [2, 3, 2], 2, 0.2)])
def test_assembled_b_annihilates_constants_and_is_inf_sup_stable(dim, n, k, jit):
    v = structured_vertices(dim, n, jitter=jit, seed=71)
    S = O.StokesSystem(dim, n, k, v)
    assert S.ok
    B = S.B.toarray()
    assert np.abs(np.ones(S.np) @ B).max() <= 1e-13 * np.abs(B).max()
    sv = np.linalg.svd(B, compute_uv=False)
    assert sv[-1] <= 1e-12 * sv[0]           # the constant mode
    assert sv[-2] >= 1e-4 * sv[0]            # and no other: rank n_p - 1


@pytest.mark.parametrize("dim,n,k", [(2, [3, 4], 1), (2, [3, 3], 2), (3, [2, 2, 2], 1), (3, [2, 2, 3], 2),
                                     (2, [2, 2], 3)])
def test_constant_force_is_balanced_by_an_affine_pressure(dim, n, k):
    f = [1.5, -0.75, 0.5][:dim]
    v = structured_vertices(dim, n, jitter=0.2, seed=72)
    S = O.StokesSystem(dim, n, k, v, mu=2.0, source_kind=1, source=f)
    u, p = S.solve()
    xp = S.pressure_nodes()
    pe = xp @ np.array(f)
    pe -= pe.mean()
    assert np.abs(u).max() <= 1e-11 * np.abs(pe).max()
    assert np.abs(p - pe).max() <= 1e-11 * np.abs(pe).max()


def test_sin_force_gives_a_nonzero_velocity_and_a_symmetric_system():
    v = structured_vertices(3, [2, 2, 2], jitter=0.2, seed=73)
    S = O.StokesSystem(3, [2, 2, 2], 1, v, source_kind=2, source=(1.0, -0.5, 0.25))
    K = S.matrix()
    assert abs(K - K.T).max() <= 1e-14 * abs(K).max()
    u, p = S.solve()
    r = K @ np.concatenate([u, p]) - S.rhs()
    assert np.abs(r).max() <= 1e-10 * np.abs(S.rhs()).max()
    assert np.abs(u).max() > 1e-3
