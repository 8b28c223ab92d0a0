"""Pins of the oracle's lowest-order Nedelec (curl-conforming, Sect. 3.10) and
Raviart-Thomas (div-conforming, Sect. 3.9) elements on simplices, against
what the mathematics fixes independently of the change-of-basis code:

* the shape functions against the Whitney forms: lambda_i grad(lambda_j) -
  lambda_j grad(lambda_i) for the edge (i, j), and (d-1)! (x - p_j) / ((x_i0 -
  p_j) . N) for the facet opposite vertex j; their curls and divergences;
* element matrices (with the global orientation signs) on random cells
  against the same Whitney forms integrated exactly through barycentric
  moments;
* the de Rham complex on assembled meshes: the curl-curl matrix annihilates
  discrete gradients, the div-div matrix annihilates discrete curls (3D) and
  rotated gradients (2D) -- which holds only if every cell orients every
  shared edge and facet alike;
* patch tests (constant fields reproduced on jittered, shuffled meshes) and
  first-order L2 convergence to a manufactured solution.
"""
import math

import numpy as np
import pytest

import oracle as O
from fe_inputs import rng, simplex_mesh

EDGES = {2: [(0, 1), (0, 2), (1, 2)], 3: [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]}


def bary(X):
    """Barycentric gradients (rows) and volume of the simplex X ((d+1) x d)."""
    d = X.shape[1]
    T = np.hstack([np.ones((d + 1, 1)), X])
    return np.linalg.inv(T)[1:].T, abs(np.linalg.det(T)) / math.factorial(d)


def facet_normal(P):
    """N of a facet from its vertices in the given order."""
    if P.shape[1] == 2:
        t = P[1] - P[0]
        return np.array([t[1], -t[0]])
    return np.cross(P[1] - P[0], P[2] - P[0])


def whitney(family, X, x):
    """Whitney forms of the simplex X at the point x (local orientation)."""
    d = X.shape[1]
    G, _ = bary(X)
    lam = np.linalg.solve(np.hstack([np.ones((d + 1, 1)), X]).T, np.concatenate([[1.0], x]))
    if family == "nedelec":
        return np.array([lam[i] * G[j] - lam[j] * G[i] for i, j in EDGES[d]])
    out = []
    for j in range(d + 1):
        P = X[[r for r in range(d + 1) if r != j]]
        out.append(math.factorial(d - 1) * (x - X[j]) / ((P[0] - X[j]) @ facet_normal(P)))
    return np.array(out)


def crs(a, b):
    """Cross product; the scalar a_x b_y - a_y b_x for plane vectors."""
    if len(a) == 2:
        return a[0] * b[1] - a[1] * b[0]
    return np.cross(a, b)


def random_simplex(dim, seed):
    g = rng(seed)
    while True:
        X = np.vstack([np.zeros(dim), np.eye(dim)]) + 0.3 * g.standard_normal((dim + 1, dim))
        if abs(np.linalg.det(X[1:] - X[0])) > 0.2:
            return X


REF = {d: np.vstack([np.zeros(d), np.eye(d)]) for d in (2, 3)}


@pytest.mark.parametrize("family,dim", [("nedelec", 2), ("nedelec", 3), ("raviart_thomas", 2), ("raviart_thomas", 3)])
def test_shape_functions_are_whitney_forms(family, dim):
    g = rng(11)
    Gr, _ = bary(REF[dim])
    for _ in range(5):
        xi = g.dirichlet(np.ones(dim + 1))[:dim]
        phi, curl, div = O.vector_shape(family, dim, xi)
        np.testing.assert_allclose(phi, whitney(family, REF[dim], xi), atol=1e-13)
        if family == "nedelec":
            for a, (i, j) in enumerate(EDGES[dim]):
                c = 2 * crs(Gr[i], Gr[j])
                np.testing.assert_allclose(curl[a], c, atol=1e-13)
            np.testing.assert_allclose(div, 0.0, atol=1e-13)
        else:
            for j in range(dim + 1):
                P = REF[dim][[r for r in range(dim + 1) if r != j]]
                den = (P[0] - REF[dim][j]) @ facet_normal(P)
                assert abs(div[j] - math.factorial(dim) / den) <= 1e-13


def exact_element(family, X, gids, coef, kappa):
    """Whitney-form element matrix with the global orientation signs, from
    exact barycentric moments: int lam_i lam_j = |K| (1 + delta_ij) / ((d+1)(d+2))."""
    d = X.shape[1]
    G, vol = bary(X)
    M = vol * (np.ones((d + 1, d + 1)) + np.eye(d + 1)) / ((d + 1) * (d + 2))
    if family == "nedelec":
        E = EDGES[d]
        n = len(E)
        A = np.zeros((n, n))
        for a, (i, j) in enumerate(E):
            for b, (k, l) in enumerate(E):
                mass = (M[i, k] * G[j] @ G[l] - M[i, l] * G[j] @ G[k] - M[j, k] * G[i] @ G[l] + M[j, l] * G[i] @ G[k])
                ca, cb = 2 * crs(G[i], G[j]), 2 * crs(G[k], G[l])
                A[a, b] = coef * vol * np.dot(np.atleast_1d(ca), np.atleast_1d(cb)) + kappa * mass
        s = np.array([1.0 if gids[i] < gids[j] else -1.0 for i, j in E])
    else:
        n = d + 1
        A = np.zeros((n, n))
        den = []
        for j in range(n):
            P = X[[r for r in range(n) if r != j]]
            den.append((P[0] - X[j]) @ facet_normal(P))
        f = math.factorial(d - 1)
        for a in range(n):
            for b in range(n):
                # int (x - p_a) . (x - p_b) with x - p = sum_i lam_i (x_i - p)
                mass = sum(M[i, k] * (X[i] - X[a]) @ (X[k] - X[b]) for i in range(n) for k in range(n))
                A[a, b] = (coef * vol * (d * f) ** 2 + kappa * f * f * mass) / (den[a] * den[b])
        s = []
        for j in range(n):
            ids = [gids[r] for r in range(n) if r != j]
            inv = sum(1 for x in range(len(ids)) for y in range(x + 1, len(ids)) if ids[x] > ids[y])
            s.append(-1.0 if inv % 2 else 1.0)
        s = np.array(s)
    return A * np.outer(s, s)


@pytest.mark.parametrize("family,dim", [("nedelec", 2), ("nedelec", 3), ("raviart_thomas", 2), ("raviart_thomas", 3)])
def test_element_matrix_matches_exact_whitney_integrals(family, dim):
    for seed in (1, 2, 3):
        X = random_simplex(dim, seed)
        gids = rng(seed + 10).permutation(100)[: dim + 1].astype(np.int32)
        A, f, ok = O.vector_element(family, dim, X, gids, coef=1.3, kappa=0.7)
        assert ok
        ref = exact_element(family, X, gids, 1.3, 0.7)
        assert np.abs(A - ref).max() <= 1e-12 * np.abs(ref).max()


def _edge_vertices(S):
    """Global edge -> (lower, higher) global vertex id."""
    ev = np.zeros((S.nent, 2), dtype=np.int64)
    for K, row in enumerate(S.dof_of):
        for a, (i, j) in enumerate(EDGES[S.dim]):
            x, y = S.cells[K, i], S.cells[K, j]
            ev[row[a]] = (min(x, y), max(x, y))
    return ev


@pytest.mark.parametrize("dim", [2, 3])
def test_curl_curl_annihilates_discrete_gradients(dim):
    v, c = simplex_mesh(dim, 3, jitter=0.2, shuffle=True)
    S = O.VectorSystem("nedelec", dim, v, c, kappa=0.0, dirichlet=False)
    ev = _edge_vertices(S)
    Gd = np.zeros((S.nent, len(v)))
    Gd[np.arange(S.nent), ev[:, 1]] = 1.0
    Gd[np.arange(S.nent), ev[:, 0]] = -1.0
    A = S.scipy()
    assert S.nfree == S.nent
    res = A @ Gd
    assert np.abs(res).max() <= 1e-12 * np.abs(S.values).max()
    # with the mass term the kernel is gone (positive definite)
    S2 = O.VectorSystem("nedelec", dim, v, c, kappa=1.0, dirichlet=False)
    assert np.linalg.eigvalsh(S2.scipy().toarray()).min() > 0


def test_div_div_annihilates_discrete_curls_3d():
    v, c = simplex_mesh(3, 2, jitter=0.2, shuffle=True)
    N = O.VectorSystem("nedelec", 3, v, c, kappa=0.0, dirichlet=False)
    R = O.VectorSystem("raviart_thomas", 3, v, c, kappa=0.0, dirichlet=False)
    ev = _edge_vertices(N)
    eid = {tuple(e): k for k, e in enumerate(ev)}
    C = np.zeros((R.nent, N.nent))
    for K, row in enumerate(R.dof_of):
        for j in range(4):
            g0, g1, g2 = sorted(int(R.cells[K, r]) for r in range(4) if r != j)
            f = row[j]
            C[f, :] = 0.0
            C[f, eid[(g0, g1)]] = 1.0
            C[f, eid[(g1, g2)]] = 1.0
            C[f, eid[(g0, g2)]] = -1.0
    A = R.scipy()
    assert np.abs(A @ C).max() <= 1e-12 * np.abs(R.values).max()


def test_div_div_annihilates_rotated_gradients_2d():
    v, c = simplex_mesh(2, 4, jitter=0.2, shuffle=True)
    R = O.VectorSystem("raviart_thomas", 2, v, c, kappa=0.0, dirichlet=False)
    N = O.VectorSystem("nedelec", 2, v, c, kappa=0.0, dirichlet=False)
    ev = _edge_vertices(N)  # 2D facets are the edges; number them the RT way
    Gd = np.zeros((R.nent, len(v)))
    for K, row in enumerate(R.dof_of):
        for j in range(3):
            a, b = sorted(int(R.cells[K, r]) for r in range(3) if r != j)
            Gd[row[j]] = 0.0
            Gd[row[j], b] = 1.0
            Gd[row[j], a] = -1.0
    assert np.abs(R.scipy() @ Gd).max() <= 1e-12 * np.abs(R.values).max()


@pytest.mark.parametrize("family,dim", [("nedelec", 2), ("nedelec", 3), ("raviart_thomas", 2), ("raviart_thomas", 3)])
def test_constant_field_patch_test(family, dim):
    v, c = simplex_mesh(dim, 3, jitter=0.2, shuffle=True)
    cvec = np.array([0.7, -1.3, 0.4][:dim])
    kappa = 2.5
    S = O.VectorSystem(family, dim, v, c, kappa=kappa, source_kind=1, source=list(kappa * cvec), dirichlet=False)
    x = S.solve()
    exact = np.zeros(S.nent)
    for K, row in enumerate(S.dof_of):
        for a in range(S.nd):
            if family == "nedelec":
                i, j = EDGES[dim][a]
                lo, hi = sorted((int(c[K, i]), int(c[K, j])))
                exact[row[a]] = cvec @ (v[hi] - v[lo])
            else:
                ids = sorted(int(c[K, r]) for r in range(dim + 1) if r != a)
                exact[row[a]] = cvec @ facet_normal(v[ids]) / math.factorial(dim - 1)
    assert np.abs(x - exact).max() <= 1e-10 * np.abs(exact).max()


@pytest.mark.parametrize("family,dim,ns", [("nedelec", 2, (8, 16)), ("nedelec", 3, (4, 8)),
                                           ("raviart_thomas", 2, (8, 16)), ("raviart_thomas", 3, (4, 8))])
def test_l2_convergence_to_manufactured_field(family, dim, ns):
    kappa = 1.0
    lap = (2.0 if (family == "nedelec" and dim == 3) else 1.0) * math.pi ** 2
    scale = 1.0
    errs = []
    for n in ns:
        v, c = simplex_mesh(dim, n, jitter=0.15)
        S = O.VectorSystem(family, dim, v, c, kappa=kappa, source_kind=2, source=[(lap + kappa) * scale] * dim)
        errs.append(S.l2_error(S.solve(), scale, nq1=4))
    rate = math.log(errs[0] / errs[1]) / math.log(ns[1] / ns[0])
    assert 0.8 <= rate <= 1.4, (errs, rate)
    # the error is a fraction of the field's norm (each component's square integrates to 2^-(number of sines))
    sines = 2 if (family == "nedelec" and dim == 3) else 1
    norm = math.sqrt(dim * 0.5 ** sines)
    assert errs[1] < 0.25 * norm


@pytest.mark.parametrize("family,dim", [("nedelec", 3), ("raviart_thomas", 3)])
def test_boundary_dofs_and_definiteness(family, dim):
    n = 2
    v, c = simplex_mesh(dim, n)
    S = O.VectorSystem(family, dim, v, c, kappa=1.0)
    Sf = O.VectorSystem(family, dim, v, c, kappa=1.0, dirichlet=False)
    # Kuhn subdivision of the n^3 brick: boundary edges 3 per boundary square x 6 n^2 squares
    # + ... counted directly: a DOF is fixed iff all of its entity's vertices are on the boundary face set
    if family == "raviart_thomas":
        assert S.nfixed == 2 * 6 * n * n  # two triangles per boundary square
    assert S.nfree + S.nfixed == Sf.nfree
    A = S.scipy().toarray()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() > 0


# ---------------------------------------------------------------------------
# second-order Nedelec ("nedelec2"): two DOFs per edge and per face (3D), two
# interior DOFs (2D), local moments = T global moments with 2 x 2 blocks
# ---------------------------------------------------------------------------
def _gl(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 + 0.5 * x, 0.5 * w


def _tri_rule():
    """A degree-4 rule on the reference triangle (collapsed Gauss, numpy)."""
    x, w = _gl(4)
    pts, wts = [], []
    for i in range(4):
        for j in range(4):
            pts.append((x[i], (1 - x[i]) * x[j]))
            wts.append(w[i] * w[j] * (1 - x[i]))
    return np.array(pts), np.array(wts)


def edge_moments(u, xa, xb):
    """int_0^1 u(xa + t (xb - xa)) . (xb - xa) q_s(t) dt for q_0 = 1 - t, q_1 = t."""
    x, w = _gl(4)
    out = np.zeros(2)
    for t, wt in zip(x, w):
        d = u(xa + t * (xb - xa)) @ (xb - xa)
        out += wt * d * np.array([1 - t, t])
    return out


def face_moments(u, x0, x1, x2):
    """int over the reference triangle of u(x0 + s0 t0 + s1 t1) . t_m ds."""
    t0, t1 = x1 - x0, x2 - x0
    P, W = _tri_rule()
    out = np.zeros(2)
    for (s0, s1), w in zip(P, W):
        val = u(x0 + s0 * t0 + s1 * t1)
        out += w * np.array([val @ t0, val @ t1])
    return out


def reference_moments(u, dim):
    """The second-order Nedelec moments of u on the reference simplex in the
    local frame (edges, faces or interior, in the element's DOF order)."""
    X = REF[dim]
    out = []
    for i, j in EDGES[dim]:
        out += list(edge_moments(u, X[i], X[j]))
    if dim == 3:
        for f in range(4):
            iv = [r for r in range(4) if r != f]
            out += list(face_moments(u, X[iv[0]], X[iv[1]], X[iv[2]]))
    else:
        P, W = _tri_rule()
        out += list(sum(w * u(np.array(p)) for p, w in zip(P, W)))
    return np.array(out)


@pytest.mark.parametrize("dim", [2, 3])
def test_nedelec2_interpolates_its_space_exactly(dim):
    """The interpolant sum_a sigma_a(v) phi_a reproduces fields of the space:
    random affine fields ([P_1]^d) and the quadratic fields x_m (x x e_i)
    (3D) or x_m (-y, x) (2D) orthogonal to x."""
    g = rng(21)
    fields = []
    for _ in range(3):
        B, c = g.standard_normal((dim, dim)), g.standard_normal(dim)
        fields.append(lambda x, B=B, c=c: B @ x + c)
    if dim == 3:
        for i in range(3):
            for m in range(3):
                e = np.eye(3)[i]
                fields.append(lambda x, e=e, m=m: x[m] * np.cross(x, e))
    else:
        for m in range(2):
            fields.append(lambda x, m=m: x[m] * np.array([-x[1], x[0]]))
    for u in fields:
        sig = reference_moments(u, dim)
        for _ in range(4):
            xi = g.dirichlet(np.ones(dim + 1))[:dim]
            phi, _, _ = O.vector_shape("nedelec2", dim, xi)
            np.testing.assert_allclose(sig @ phi, u(xi), atol=1e-12)


def _global_moments(u, v, c, S, dim):
    """Global-frame DOF values of the field u on the mesh (fixed DOFs dropped):
    edges lower -> higher id, faces over their vertices in ascending id; the
    2D interior moments of the covariant pull-back J^T u on the reference cell."""
    vals = np.full(S.nent, np.nan)
    for K, row in enumerate(S.dof_of):
        gids = c[K]
        for e, (i, j) in enumerate(EDGES[dim]):
            lo, hi = sorted((int(gids[i]), int(gids[j])))
            vals[row[2 * e:2 * e + 2]] = edge_moments(u, v[lo], v[hi])
        if dim == 3:
            for f in range(4):
                ids = sorted(int(gids[r]) for r in range(4) if r != f)
                vals[row[12 + 2 * f:14 + 2 * f]] = face_moments(u, v[ids[0]], v[ids[1]], v[ids[2]])
        else:
            X = v[gids]
            J = (X[1:] - X[0]).T
            P, W = _tri_rule()
            vals[row[6:8]] = sum(w * (J.T @ u(X[0] + J @ np.array(p))) for p, w in zip(P, W))
    return vals


@pytest.mark.parametrize("dim,n", [(2, 3), (3, 2)])
def test_nedelec2_linear_curl_free_patch_test(dim, n):
    """u = B x + c with B symmetric has no curl, so curl curl u + kappa u =
    kappa u and the natural boundary condition holds: the discrete solution
    is u's interpolant, exactly, on jittered shuffled meshes."""
    v, c = simplex_mesh(dim, n, jitter=0.2, shuffle=True)
    g = rng(22)
    B = g.standard_normal((dim, dim))
    B = B + B.T
    cv = g.standard_normal(dim)
    kappa = 2.5
    aff = []
    for comp in range(dim):
        aff += [kappa * cv[comp]] + list(kappa * B[comp]) + [0.0] * (3 - dim)
    S = O.VectorSystem("nedelec2", dim, v, c, kappa=kappa, source_kind=3, source=aff, dirichlet=False)
    x = S.solve()
    exact = _global_moments(lambda p: B @ p + cv, v, c, S, dim)
    assert np.abs(x - exact).max() <= 1e-10 * np.abs(exact).max()


@pytest.mark.parametrize("dim,n", [(2, 3), (3, 2)])
def test_nedelec2_curl_curl_annihilates_gradients_of_p2(dim, n):
    """Gradients of the global P2 Lagrange functions lie in the second-order
    Nedelec space; the curl-curl matrix (kappa = 0, no boundary DOFs fixed)
    times the matrix of their global-frame moments vanishes -- only if every
    cell maps shared edge and face DOFs to the global frame alike."""
    v, c = simplex_mesh(dim, n, jitter=0.2, shuffle=True)
    S = O.VectorSystem("nedelec2", dim, v, c, kappa=0.0, dirichlet=False)
    node_of, code, _, _ = O.simplex_number(dim, 2, len(v), c, dirichlet=False)
    nnodes = len(code)
    G = np.zeros((S.nent, nnodes))
    for K in range(c.shape[0]):
        X = v[c[K]]
        J = (X[1:] - X[0]).T
        Ji = np.linalg.inv(J)
        for ln in range(node_of.shape[1]):
            def grad(p, ln=ln):
                xi = Ji @ (p - X[0])
                _, d = O.simplex_shape(dim, 2, xi)
                return Ji.T @ d[ln]
            col = _global_moments_cell(grad, v, c, S, dim, K)
            for pos, val in col.items():
                G[pos, node_of[K, ln]] = val
    A = S.scipy()
    assert np.abs(G).max() > 0.1 and np.abs(A @ np.ones(S.nent)).max() > 1e-3  # neither side is trivial
    assert np.abs(A @ G).max() <= 1e-10 * np.abs(S.values).max()


def _global_moments_cell(u, v, c, S, dim, K):
    """Global-frame moments of u over the edges and faces of cell K (the
    interior DOFs of a 2D cell: the pull-back moments on the reference cell)."""
    out = {}
    gids = c[K]
    row = S.dof_of[K]
    for e, (i, j) in enumerate(EDGES[dim]):
        lo, hi = sorted((int(gids[i]), int(gids[j])))
        m = edge_moments(u, v[lo], v[hi])
        out[row[2 * e]], out[row[2 * e + 1]] = m
    if dim == 3:
        for f in range(4):
            ids = sorted(int(gids[r]) for r in range(4) if r != f)
            m = face_moments(u, v[ids[0]], v[ids[1]], v[ids[2]])
            out[row[12 + 2 * f]], out[row[13 + 2 * f]] = m
    else:
        X = v[gids]
        J = (X[1:] - X[0]).T
        P, W = _tri_rule()
        m = sum(w * (J.T @ u(X[0] + J @ np.array(p))) for p, w in zip(P, W))
        out[row[6]], out[row[7]] = m
    return out


@pytest.mark.parametrize("dim,ns", [(2, (4, 8)), (3, (2, 4))])
def test_nedelec2_second_order_convergence(dim, ns):
    kappa = 1.0
    lap = (2.0 if dim == 3 else 1.0) * math.pi ** 2
    errs = []
    for n in ns:
        v, c = simplex_mesh(dim, n, jitter=0.15)
        S = O.VectorSystem("nedelec2", dim, v, c, kappa=kappa, source_kind=2, source=[lap + kappa] * dim)
        errs.append(S.l2_error(S.solve(), 1.0, nq1=5))
    rate = math.log(errs[0] / errs[1]) / math.log(ns[1] / ns[0])
    assert 1.7 <= rate <= 2.5, (errs, rate)


# ---------------------------------------------------------------------------
# second-order Raviart-Thomas ("raviart_thomas2"): per facet the flux against
# the barycentric of each of its vertices (N over the facet's vertices, in
# ascending global id in the global frame), the components' integrals inside;
# local moments = the global ones of the same vertex times the facet's parity
# ---------------------------------------------------------------------------
def _tet_rule():
    """A degree-5 rule on the reference tetrahedron (collapsed Gauss, numpy)."""
    x, w = _gl(4)
    pts, wts = [], []
    for i in range(4):
        for j in range(4):
            for k in range(4):
                a = x[i]
                b = (1 - a) * x[j]
                c = (1 - a) * (1 - x[j]) * x[k]
                pts.append((a, b, c))
                wts.append(w[i] * w[j] * w[k] * (1 - a) ** 2 * (1 - x[j]))
    return np.array(pts), np.array(wts)


def flux_moments(u, ys):
    """int over the facet with vertices ys (in the given order) of u . N times
    the barycentric of each vertex, in the facet's parameter measure; N the
    rotated edge (2D) or the cross product of the edges from ys[0] (3D)."""
    ys = [np.asarray(y, dtype=np.float64) for y in ys]
    if len(ys) == 2:
        t = ys[1] - ys[0]
        N = np.array([t[1], -t[0]])
        x, w = _gl(4)
        return sum(wt * (u(ys[0] + s * t) @ N) * np.array([1 - s, s]) for s, wt in zip(x, w))
    N = np.cross(ys[1] - ys[0], ys[2] - ys[0])
    P, W = _tri_rule()
    out = np.zeros(3)
    for (s0, s1), wt in zip(P, W):
        out += wt * (u(ys[0] + s0 * (ys[1] - ys[0]) + s1 * (ys[2] - ys[0])) @ N) * np.array([1 - s0 - s1, s0, s1])
    return out


def _cell_rule(dim):
    return _tri_rule() if dim == 2 else _tet_rule()


def rt2_reference_moments(u, dim):
    X = REF[dim]
    out = []
    for f in range(dim + 1):
        out += list(flux_moments(u, [X[r] for r in range(dim + 1) if r != f]))
    P, W = _cell_rule(dim)
    out += list(sum(w * u(np.array(p)) for p, w in zip(P, W)))
    return np.array(out)


@pytest.mark.parametrize("dim", [2, 3])
def test_rt2_interpolates_its_space_exactly(dim):
    """The interpolant sum_a sigma_a(v) phi_a reproduces fields of the space:
    random affine fields ([P_1]^d) and x x_m."""
    g = rng(31)
    fields = []
    for _ in range(3):
        B, c = g.standard_normal((dim, dim)), g.standard_normal(dim)
        fields.append(lambda x, B=B, c=c: B @ x + c)
    for m in range(dim):
        fields.append(lambda x, m=m: x * x[m])
    for u in fields:
        sig = rt2_reference_moments(u, dim)
        for _ in range(4):
            xi = g.dirichlet(np.ones(dim + 1))[:dim]
            phi, _, _ = O.vector_shape("raviart_thomas2", dim, xi)
            np.testing.assert_allclose(sig @ phi, u(xi), atol=1e-12)


def _rt2_global_moments(u, v, c, S, dim):
    """Global-frame DOF values of u: facets over their vertices in ascending
    id; a cell's interior moments of the contravariant pull-back
    det J J^-1 u on the reference cell."""
    vals = np.full(S.nent, np.nan)
    P, W = _cell_rule(dim)
    for K, row in enumerate(S.dof_of):
        gids = c[K]
        for f in range(dim + 1):
            ids = sorted(int(gids[r]) for r in range(dim + 1) if r != f)
            vals[row[f * dim:(f + 1) * dim]] = flux_moments(u, [v[i] for i in ids])
        X = v[gids]
        J = (X[1:] - X[0]).T
        pull = np.linalg.det(J) * np.linalg.inv(J)
        vals[row[dim * (dim + 1):]] = sum(w * (pull @ u(X[0] + J @ np.array(p))) for p, w in zip(P, W))
    return vals


@pytest.mark.parametrize("dim,n", [(2, 3), (3, 2)])
def test_rt2_divergence_free_affine_patch_test(dim, n):
    """u = B x + c with trace B = 0 has no divergence, so -grad(k div u) +
    kappa u = kappa u and the natural boundary term vanishes: the discrete
    solution is u's interpolant, exactly, on jittered shuffled meshes."""
    v, c = simplex_mesh(dim, n, jitter=0.2, shuffle=True)
    g = rng(32)
    B = g.standard_normal((dim, dim))
    B -= np.trace(B) / dim * np.eye(dim)
    cv = g.standard_normal(dim)
    kappa = 1.7
    aff = []
    for comp in range(dim):
        aff += [kappa * cv[comp]] + list(kappa * B[comp]) + [0.0] * (3 - dim)
    S = O.VectorSystem("raviart_thomas2", dim, v, c, kappa=kappa, source_kind=3, source=aff, dirichlet=False)
    x = S.solve()
    exact = _rt2_global_moments(lambda p: B @ p + cv, v, c, S, dim)
    assert np.abs(x - exact).max() <= 1e-10 * np.abs(exact).max()


@pytest.mark.parametrize("dim,n", [(2, [3, 2]), (3, [2, 1, 1])])
def test_rt2_div_div_kernel_is_the_discrete_curls(dim, n):
    """With no DOF fixed and kappa = 0, the div-div matrix's null space is the
    divergence-free part of the space, which the exact sequence makes the
    curls of the second-order Nedelec space (3D) or the rotated gradients of
    P2 (2D): its rank is #RT2 - (#N2 - (#P2 - 1)) (3D), #RT2 - (#P2 - 1) (2D).
    A facet whose two cells disagree on its orientation or vertex order breaks
    the count."""
    v, c = simplex_mesh(dim, n, jitter=0.2, shuffle=True)
    S = O.VectorSystem("raviart_thomas2", dim, v, c, kappa=0.0, dirichlet=False)
    _, code, _, _ = O.simplex_number(dim, 2, len(v), c, dirichlet=False)
    npk = len(code)
    if dim == 3:
        _, ncode, nfree, _ = O.vector_number("nedelec2", dim, len(v), c, dirichlet=False)
        kernel = nfree - (npk - 1)
    else:
        kernel = npk - 1
    ev = np.linalg.eigvalsh(S.scipy().toarray())
    rank = int((ev > 1e-9 * ev.max()).sum())
    assert rank == S.nent - kernel, (S.nent, kernel, rank)
    gap = ev[ev > 1e-9 * ev.max()].min() / ev.max()
    assert gap > 1e-6 and np.abs(ev[: S.nent - rank]).max() < 1e-12 * ev.max()


def test_rt2_div_div_annihilates_rotated_gradients_2d():
    """The rotated gradients (d_y phi, -d_x phi) of the global P2 Lagrange
    functions lie in the second-order Raviart-Thomas space; the div-div matrix
    times the matrix of their global-frame moments vanishes."""
    dim = 2
    v, c = simplex_mesh(dim, [3, 2], jitter=0.2, shuffle=True)
    S = O.VectorSystem("raviart_thomas2", dim, v, c, kappa=0.0, dirichlet=False)
    node_of, code, _, _ = O.simplex_number(dim, 2, len(v), c, dirichlet=False)
    G = np.zeros((S.nent, len(code)))
    P, W = _cell_rule(dim)
    for K in range(c.shape[0]):
        X = v[c[K]]
        J = (X[1:] - X[0]).T
        Ji = np.linalg.inv(J)
        pull = np.linalg.det(J) * Ji
        gids = c[K]
        row = S.dof_of[K]
        for ln in range(node_of.shape[1]):
            def rot(p, ln=ln):
                _, d = O.simplex_shape(dim, 2, Ji @ (p - X[0]))
                gr = Ji.T @ d[ln]
                return np.array([gr[1], -gr[0]])
            for f in range(3):
                ids = sorted(int(gids[r]) for r in range(3) if r != f)
                G[row[2 * f:2 * f + 2], node_of[K, ln]] = flux_moments(rot, [v[i] for i in ids])
            G[row[6:8], node_of[K, ln]] = sum(w * (pull @ rot(X[0] + J @ np.array(p))) for p, w in zip(P, W))
    A = S.scipy()
    assert np.abs(G).max() > 0.1 and np.abs(A @ np.ones(S.nent)).max() > 1e-3
    assert np.abs(A @ G).max() <= 1e-10 * np.abs(S.values).max()


@pytest.mark.parametrize("dim,ns", [(2, (4, 8)), (3, (2, 4))])
def test_rt2_second_order_convergence(dim, ns):
    kappa = 1.0
    errs = []
    for n in ns:
        v, c = simplex_mesh(dim, n, jitter=0.15)
        S = O.VectorSystem("raviart_thomas2", dim, v, c, kappa=kappa, source_kind=2,
                           source=[math.pi ** 2 + kappa] * dim)
        errs.append(S.l2_error(S.solve(), 1.0, nq1=5))
    rate = math.log(errs[0] / errs[1]) / math.log(ns[1] / ns[0])
    assert 1.7 <= rate <= 2.5, (errs, rate)
