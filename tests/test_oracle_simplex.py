"""Pins of the oracle's P_k elements on simplices (Sect. 3.3 truncated spaces,
Sect. 3.5 change of basis, Sect. 3.7 collapsed quadrature) against what the
mathematics fixes independently of it:

* the basis against Silvester's closed form of the Lagrange basis on the
  simplex (products of k lambda_j - m over the barycentric coordinates), and
  P1 = the barycentric coordinates themselves;
* the collapsed Gauss rule against the exact simplex moments
  alpha! / (|alpha| + d)! up to the degree the rule claims;
* element matrices against an exact rational computation on the reference
  simplex (Silvester polynomials, exact monomial moments) carried to the cell
  by its Jacobian, P1 against the textbook |K| grad(lambda_a) . grad(lambda_b),
  energies of linear fields and the kernel of the elasticity form;
* the numbering against a brute-force numbering by node positions (first
  appearance over cells and local nodes) on lattice meshes, plain and
  shuffled, node counts (kn+1)^d, the boundary;
* the assembled system: the P1 Kuhn stiffness is the 5- / 7-point stencil,
  row sums and loads without Dirichlet data, the linear patch test on
  jittered and shuffled meshes, O(h^(k+1)) convergence, the L2 error's
  magnitude.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from fe_inputs import rng, simplex_mesh


# ---------------------------------------------------------------------------
# exact polynomials in xi (dict: exponent tuple -> Fraction)
# ---------------------------------------------------------------------------
def p_const(dim, c):
    return {(0,) * dim: Fraction(c)}


def p_var(dim, r):
    e = [0] * dim
    e[r] = 1
    return {tuple(e): Fraction(1)}


def p_add(p, q, s=1):
    out = dict(p)
    for e, c in q.items():
        out[e] = out.get(e, Fraction(0)) + s * c
    return {e: c for e, c in out.items() if c != 0}


def p_mul(p, q):
    out = {}
    for e1, c1 in p.items():
        for e2, c2 in q.items():
            e = tuple(a + b for a, b in zip(e1, e2))
            out[e] = out.get(e, Fraction(0)) + c1 * c2
    return {e: c for e, c in out.items() if c != 0}


def p_der(p, r):
    out = {}
    for e, c in p.items():
        if e[r] > 0:
            f = list(e)
            f[r] -= 1
            out[tuple(f)] = out.get(tuple(f), Fraction(0)) + c * e[r]
    return out


def p_int(p, dim):
    """Exact integral over the reference simplex: prod alpha_r! / (|alpha| + d)!"""
    s = Fraction(0)
    for e, c in p.items():
        s += c * Fraction(math.prod(math.factorial(a) for a in e), math.factorial(sum(e) + dim))
    return s


def p_eval(p, xi):
    return float(sum(float(c) * np.prod([x ** a for x, a in zip(xi, e)]) for e, c in p.items()))


def lattice(dim, k):
    """Local nodes: lattice points with |s| <= k, x fastest."""
    pts = []
    for s in itertools.product(range(k + 1), repeat=dim):
        s = s[::-1]
        if sum(s) <= k:
            pts.append(s)
    return pts


def silvester(dim, k):
    """Lagrange basis on the simplex in Silvester's product form."""
    lam = [p_add(p_const(dim, 1), {e: c for v in [p_var(dim, r) for r in range(dim)] for e, c in v.items()}, -1)]
    lam += [p_var(dim, r) for r in range(dim)]
    basis = []
    for s in lattice(dim, k):
        beta = [k - sum(s)] + list(s)
        phi = p_const(dim, 1)
        for j in range(dim + 1):
            for m in range(beta[j]):
                term = p_add({e: k * c for e, c in lam[j].items()}, p_const(dim, m), -1)
                phi = p_mul(phi, {e: c / (m + 1) for e, c in term.items()})
        basis.append(phi)
    return basis


_S_CACHE = {}


def exact_gradient_tensor(dim, k):
    """S[r][s][a][b] = int d_r phi_a d_s phi_b over the reference simplex (exact)."""
    key = (dim, k)
    if key not in _S_CACHE:
        B = silvester(dim, k)
        dB = [[p_der(p, r) for r in range(dim)] for p in B]
        nn = len(B)
        S = np.zeros((dim, dim, nn, nn))
        for a in range(nn):
            for b in range(nn):
                for r in range(dim):
                    for s in range(dim):
                        S[r, s, a, b] = float(p_int(p_mul(dB[a][r], dB[b][s]), dim))
        _S_CACHE[key] = S
    return _S_CACHE[key]


def random_simplex(dim, seed):
    g = rng(seed)
    while True:
        X = np.vstack([np.zeros(dim), np.eye(dim)]) + 0.3 * g.standard_normal((dim + 1, dim))
        J = (X[1:] - X[0]).T
        if abs(np.linalg.det(J)) > 0.2:
            return X


# ---------------------------------------------------------------------------
# basis and quadrature
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2), (3, 3), (3, 4)])
def test_local_nodes_and_basis_match_silvester(dim, k):
    s = O.simplex_nodes(dim, k)
    assert [tuple(r) for r in s] == lattice(dim, k)
    assert len(s) == O.simplex_nn(dim, k)
    B = silvester(dim, k)
    g = rng(7)
    for _ in range(6):
        xi = g.dirichlet(np.ones(dim + 1))[:dim]
        phi, dphi = O.simplex_shape(dim, k, xi)
        ref = np.array([p_eval(p, xi) for p in B])
        dref = np.array([[p_eval(p_der(p, r), xi) for r in range(dim)] for p in B])
        np.testing.assert_allclose(phi, ref, atol=1e-12)
        np.testing.assert_allclose(dphi, dref, atol=1e-10)
    # the delta property at the nodes
    for a, sa in enumerate(lattice(dim, k)):
        phi, _ = O.simplex_shape(dim, k, [v / k for v in sa])
        e = np.zeros(len(phi))
        e[a] = 1.0
        np.testing.assert_allclose(phi, e, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_p1_basis_is_barycentric(dim):
    g = rng(8)
    for _ in range(5):
        xi = g.dirichlet(np.ones(dim + 1))[:dim]
        phi, dphi = O.simplex_shape(dim, 1, xi)
        np.testing.assert_allclose(phi, [1 - xi.sum()] + list(xi), atol=1e-14)
        np.testing.assert_allclose(dphi, np.vstack([-np.ones(dim), np.eye(dim)]), atol=1e-14)


@pytest.mark.parametrize("dim,n", [(2, 1), (2, 2), (2, 4), (3, 2), (3, 3), (3, 5)])
def test_collapsed_rule_integrates_monomials_exactly(dim, n):
    xi, w = O.simplex_quadrature(dim, n)
    assert abs(w.sum() - 1.0 / math.factorial(dim)) < 1e-15
    assert np.all(xi >= 0) and np.all(xi.sum(axis=1) <= 1.0)
    # exact for total degree <= 2n - 1 - (d - 1): the Jacobian adds d - 1 to u_0's degree
    top = 2 * n - dim
    for e in itertools.product(range(top + 1), repeat=dim):
        if sum(e) > top:
            continue
        exact = math.prod(math.factorial(a) for a in e) / math.factorial(sum(e) + dim)
        got = float(np.sum(w * np.prod(xi ** np.array(e), axis=1)))
        assert abs(got - exact) <= 1e-14 * max(1.0, exact), (e, got, exact)


# ---------------------------------------------------------------------------
# element matrices and loads
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2), (3, 3)])
def test_poisson_element_matches_exact_reference_tensor(dim, k):
    S = exact_gradient_tensor(dim, k)
    for seed in (1, 2):
        X = random_simplex(dim, seed)
        J = (X[1:] - X[0]).T
        Ji = np.linalg.inv(J)
        M = Ji @ Ji.T * abs(np.linalg.det(J))
        ref = np.einsum("rs,rsab->ab", M, S) * 1.7
        A, ok = O.simplex_element_matrix(dim, k, X, coef=1.7)
        assert ok
        assert np.abs(A - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_elasticity_element_matches_exact_reference_tensor(dim, k):
    S = exact_gradient_tensor(dim, k)
    young, nu = 2.0, 0.3
    lam, mu = O.lame(young, nu)
    X = random_simplex(dim, 3)
    J = (X[1:] - X[0]).T
    Ji = np.linalg.inv(J)
    det = abs(np.linalg.det(J))
    # G[i][j][a][b] = int d_i phi_a d_j phi_b on the cell
    G = det * np.einsum("ri,sj,rsab->ijab", Ji, Ji, S)
    nn = S.shape[2]
    ref = np.zeros((nn * dim, nn * dim))
    for i in range(dim):
        for j in range(dim):
            blk = lam * G[i, j] + mu * G[j, i] + (mu * sum(G[l, l] for l in range(dim)) if i == j else 0.0)
            ref[i::dim, j::dim] = blk
    A, ok = O.simplex_element_matrix(dim, k, X, problem="elasticity", young=young, nu=nu)
    assert ok
    assert np.abs(A - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_p1_element_is_textbook(dim):
    X = random_simplex(dim, 4)
    T = np.hstack([np.ones((dim + 1, 1)), X])
    grads = np.linalg.inv(T)[1:].T  # row a: grad lambda_a
    vol = abs(np.linalg.det(T)) / math.factorial(dim)
    A, ok = O.simplex_element_matrix(dim, 1, X, coef=0.6)
    np.testing.assert_allclose(A, 0.6 * vol * grads @ grads.T, rtol=1e-12, atol=1e-14)


def _node_positions(dim, k, X):
    return np.array([X[0] + (X[1:] - X[0]).T @ (np.array(s) / k) for s in lattice(dim, k)])


@pytest.mark.parametrize("dim,k", [(2, 2), (3, 3), (3, 4)])
def test_energy_of_linear_fields_and_rigid_kernel(dim, k):
    X = random_simplex(dim, 5)
    vol = abs(np.linalg.det((X[1:] - X[0]).T)) / math.factorial(dim)
    P = _node_positions(dim, k, X)
    g = rng(6)
    b = g.standard_normal(dim)
    u = 0.4 + P @ b
    A, _ = O.simplex_element_matrix(dim, k, X)
    assert abs(u @ A @ u - vol * b @ b) <= 1e-12 * vol * (b @ b)
    assert np.abs(A @ np.ones(len(u))).max() <= 1e-12 * np.abs(A).max()
    young, nu = 1.5, 0.25
    lam, mu = O.lame(young, nu)
    Ae, _ = O.simplex_element_matrix(dim, k, X, problem="elasticity", young=young, nu=nu)
    Bm = g.standard_normal((dim, dim))
    ue = (P @ Bm.T + g.standard_normal(dim)).ravel()
    eps = 0.5 * (Bm + Bm.T)
    energy = vol * (2 * mu * np.sum(eps * eps) + lam * np.trace(eps) ** 2)
    assert abs(ue @ Ae @ ue - energy) <= 1e-11 * energy
    W = g.standard_normal((dim, dim))
    W = W - W.T
    ur = (P @ W.T + g.standard_normal(dim)).ravel()
    assert np.abs(Ae @ ur).max() <= 1e-11 * np.abs(Ae).max()


@pytest.mark.parametrize("dim,k", [(2, 3), (3, 2), (3, 3)])
def test_load_of_constant_source_is_exact_moment(dim, k):
    B = silvester(dim, k)
    moments = np.array([float(p_int(p, dim)) for p in B])
    X = random_simplex(dim, 9)
    det = abs(np.linalg.det((X[1:] - X[0]).T))
    f = O.simplex_element_load(dim, k, dim, X, 1, (0.5, -2.0, 1.25)[:dim])
    for c, v in enumerate((0.5, -2.0, 1.25)[:dim]):
        np.testing.assert_allclose(f[c::dim], v * det * moments, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------------------
# numbering and pattern
# ---------------------------------------------------------------------------
def brute_numbering(dim, k, n, verts, cells):
    """Nodes identified by their lattice position (exact on unjittered meshes),
    numbered by first appearance; boundary = a coordinate at 0 or 1."""
    scale = k * n
    ids, bnd, node_of = {}, [], np.zeros((len(cells), len(lattice(dim, k))), dtype=np.int64)
    for K, c in enumerate(cells):
        X = verts[c]
        for a, x in enumerate(_node_positions(dim, k, X)):
            key = tuple(int(round(v * scale)) for v in x)
            if key not in ids:
                ids[key] = len(ids)
                bnd.append(any(v == 0 or v == scale for v in key))
            node_of[K, a] = ids[key]
    return node_of, np.array(bnd)


@pytest.mark.parametrize("dim,k,n,shuffle", [(2, 1, 3, False), (2, 3, 3, True), (3, 1, 2, False), (3, 2, 2, True),
                                             (3, 3, 2, False), (3, 4, 2, True)])
def test_numbering_matches_brute_force_by_position(dim, k, n, shuffle):
    v, c = simplex_mesh(dim, n, shuffle=shuffle)
    node_of, code, nfree, nfixed = O.simplex_number(dim, k, len(v), c)
    ref, bnd = brute_numbering(dim, k, n, v, c)
    np.testing.assert_array_equal(node_of, ref)
    assert len(code) == (k * n + 1) ** dim
    assert nfree == (k * n - 1) ** dim and nfixed == len(code) - nfree
    np.testing.assert_array_equal(code < 0, bnd)
    # free and fixed ranks ascend with the node id
    np.testing.assert_array_equal(code[code >= 0], np.arange(nfree))
    np.testing.assert_array_equal(-1 - code[code < 0], np.arange(nfixed))


@pytest.mark.parametrize("dim,k,n", [(2, 2, [3, 2]), (3, 2, [2, 1, 2]), (3, 3, [1, 2, 1])])
def test_pattern_is_every_free_pair_sharing_a_cell(dim, k, n):
    v, c = simplex_mesh(dim, n, jitter=0.2, shuffle=True)
    S = O.SimplexSystem(dim, k, v, c, problem="elasticity")
    pairs = set()
    for row in S.cell_dofs:
        f = [d for d in row if d >= 0]
        pairs.update((i, j) for i in f for j in f)
    assert S.nnz == len(pairs)
    for i in range(S.nfree):
        cols = S.colind[S.rowptr[i]:S.rowptr[i + 1]]
        assert list(cols) == sorted(j for (r, j) in pairs if r == i)


# ---------------------------------------------------------------------------
# assembled systems
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_p1_kuhn_stiffness_is_the_finite_difference_stencil(dim):
    n = 4
    v, c = simplex_mesh(dim, n)
    S = O.SimplexSystem(dim, 1, v, c)
    A = S.dense()
    h = 1.0 / n
    P = S.node_positions()
    free_pos = np.zeros((S.nfree, dim))
    for g, code in enumerate(S.node_code):
        if code >= 0:
            free_pos[code] = P[g]
    scale = h ** (dim - 2)
    for i in range(S.nfree):
        for j in range(S.nfree):
            d = np.rint((free_pos[j] - free_pos[i]) / h).astype(int)
            if i == j:
                expect = 2 * dim * scale
            elif np.abs(d).sum() == 1:
                expect = -scale
            else:
                expect = 0.0
            assert abs(A[i, j] - expect) <= 1e-13, (i, j, d, A[i, j])


@pytest.mark.parametrize("dim,k", [(2, 2), (3, 2)])
def test_row_sums_and_load_without_dirichlet(dim, k):
    v, c = simplex_mesh(dim, 2, jitter=0.2, shuffle=True)
    S = O.SimplexSystem(dim, k, v, c, dirichlet=False, source_kind=1, source=(1.5,))
    A = S.scipy()
    assert np.abs(A @ np.ones(S.nfree)).max() <= 1e-12 * np.abs(S.values).max()
    assert abs(S.rhs.sum() - 1.5) <= 1e-13
    assert abs(A - A.T).max() <= 1e-14 * np.abs(S.values).max()


AFF = [0.3, 1.0, -2.0, 0.5, -0.7, 0.2, 0.4, 1.1, 0.9, -0.3, 0.6, -1.2]


@pytest.mark.parametrize("dim,k,problem,n", [(2, 1, "poisson", 4), (2, 4, "poisson", 2), (3, 1, "poisson", 3),
                                             (3, 3, "poisson", 2), (3, 2, "elasticity", 2), (2, 3, "elasticity", 3)])
def test_linear_patch_test(dim, k, problem, n):
    v, c = simplex_mesh(dim, n, jitter=0.2, shuffle=True)
    S = O.SimplexSystem(dim, k, v, c, problem=problem, dirichlet_kind=1, dirichlet_affine=AFF)
    x = S.solve()
    P = S.node_positions()
    nc = S.ncomp
    exact = np.zeros(S.nfree)
    for g, code in enumerate(S.node_code):
        if code >= 0:
            for comp in range(nc):
                exact[nc * code + comp] = AFF[4 * comp] + np.dot(AFF[4 * comp + 1:4 * comp + 1 + dim], P[g])
    assert np.abs(x - exact).max() <= 1e-10


@pytest.mark.parametrize("dim,k,ns", [(2, 1, (4, 8)), (2, 2, (4, 8)), (2, 3, (2, 4)), (3, 1, (4, 8)), (3, 2, (3, 6))])
def test_l2_convergence_rate(dim, k, ns):
    errs = []
    for n in ns:
        v, c = simplex_mesh(dim, n, jitter=0.15)
        S = O.SimplexSystem(dim, k, v, c, source_kind=2, source=(1.0,))
        errs.append(S.l2_error(S.solve(), 1, [1.0]))
    rate = math.log(errs[0] / errs[1]) / math.log(ns[1] / ns[0])
    assert k + 1 - 0.35 <= rate <= k + 1 + 0.6, (errs, rate)


@pytest.mark.parametrize("dim,k", [(2, 2), (3, 1)])
def test_l2_error_magnitude_closed_forms(dim, k):
    n = 4
    v, c = simplex_mesh(dim, n, jitter=0.2)
    S = O.SimplexSystem(dim, k, v, c)
    zero = np.zeros(S.nfree)
    # a zero field against prod sin(pi x_r): the norm of the sine product, 2^(-d/2)
    assert abs(S.l2_error(zero, 1, [1.0], nq1=k + 6) - 2.0 ** (-dim / 2)) <= 1e-7
    # against an affine field (a polynomial the rule integrates exactly)
    a = [0.5, 1.0, -1.0, 2.0][: dim + 1] + [0.0] * (12 - dim - 1)
    b = np.array(a[1:dim + 1])
    exact2 = a[0] ** 2 + a[0] * b.sum() + (b.sum() ** 2 - (b * b).sum()) / 4 + (b * b).sum() / 3
    assert abs(S.l2_error(zero, 2, a) - math.sqrt(exact2)) <= 1e-13
