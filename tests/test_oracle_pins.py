"""Pins of the oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check is a closed form,
an invariant, a library routine for a special case, brute force on a tiny
input, or a worked example printed in the paper.
"""
import itertools
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from fe_inputs import lognormal_coefficients, structured_vertices
from tests import exact as EX

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------
# Quadrature (Sect. 3.7: n Gauss points per direction integrate degree 2n-1)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", range(1, 13))
def test_gauss_legendre_matches_numpy_and_is_exact(n):
    x, w = O.gauss_legendre(n)
    t, v = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(x, (t + 1) / 2, rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, v / 2, rtol=0, atol=1e-15)
    assert abs(w.sum() - 1.0) < 1e-15
    for m in range(2 * n):
        assert abs((w * x ** m).sum() - 1.0 / (m + 1)) < 2e-15
    # degree 2n is not integrated exactly (the error shrinks fast with n)
    if n <= 6:
        assert abs((w * x ** (2 * n)).sum() - 1.0 / (2 * n + 1)) > 1e-8


# --------------------------------------------------------------------------
# 1D Lagrange basis (Sect. 3.4 eq. lagbas: l_m(x_l) = delta_ml)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_lagrange_delta_partition_and_exact_polynomials(k):
    for l in range(k + 1):
        v, _ = O.lagrange_1d(k, l / k)
        np.testing.assert_allclose(v, np.eye(k + 1)[l], atol=1e-14)
    polys = EX.lagrange_polys(k)
    for x in np.linspace(-0.1, 1.1, 13):
        v, d = O.lagrange_1d(k, x)
        assert abs(v.sum() - 1.0) < 1e-13
        assert abs(d.sum()) < 1e-12
        np.testing.assert_allclose(v, [EX.polyval(p, x) for p in polys], atol=1e-13)
        np.testing.assert_allclose(d, [EX.polyval(EX.polyder(p), x) for p in polys], atol=1e-12)


# --------------------------------------------------------------------------
# Worked example printed in the paper: bi-cubic quad local numbering and the
# DOFs owned by / lying on each n-face (Sect. 6.2 figure).
# --------------------------------------------------------------------------
def _golden_bicubic():
    rows = {}
    with open(os.path.join(HERE, "golden", "bicubic_quad_dofs.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            head, dofs = line.split(":")
            kind, where = head.split()
            rows[(kind, where)] = sorted(int(t) for t in dofs.split())
    return rows


def test_paper_bicubic_quad_numbering():
    g = _golden_bicubic()
    P = O.Problem(2, [1, 1], 3)
    face_bit = {"x0": 0, "x1": 1, "y0": 2, "y1": 3}
    closure = {}
    for where, bit in face_bit.items():
        code, nf, nx = O.number_nodes(2, [1, 1], 3, 1 << bit)
        cd = O.cell_dofs(P, code)[0]
        closure[where] = sorted(int(a) + 1 for a in np.nonzero(cd < 0)[0])
    # the DOFs lying on the closure of edge x = 1 (n-face 8)
    assert closure["x1"] == g[("closure", "x1")]
    # owned DOFs: edge interior = closure minus the two vertices; vertices are
    # intersections of two closures; the interior is never on a face
    verts = {"x0y0": ("x0", "y0"), "x1y0": ("x1", "y0"), "x0y1": ("x0", "y1"), "x1y1": ("x1", "y1")}
    vset = set()
    for name, (a, b) in verts.items():
        inter = sorted(set(closure[a]) & set(closure[b]))
        assert inter == g[("vertex", name)]
        vset |= set(inter)
    for e in face_bit:
        assert sorted(set(closure[e]) - vset) == g[("edge", e)]
    on_any = set().union(*closure.values())
    assert sorted(set(range(1, 17)) - on_any) == g[("interior", "-")]


# --------------------------------------------------------------------------
# Element matrices on affine cells against exact Kronecker closed forms
# --------------------------------------------------------------------------
def _random_affine(dim, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    B = np.eye(dim) * r.uniform(0.5, 1.5, dim) + r.uniform(-0.3, 0.3, (dim, dim))
    x0 = r.uniform(-1, 1, dim)
    return x0, B


@pytest.mark.parametrize("dim,k", [(d, k) for d in (2, 3) for k in (1, 2, 3, 4)])
def test_poisson_element_affine_closed_form(dim, k):
    for seed, diag_only in ((1, True), (2, False)):
        x0, B = _random_affine(dim, seed)
        if diag_only:
            B = np.diag(np.diag(B))
        X = EX.affine_cell_vertices(x0, B)
        A, ok = O.element_matrix(dim, k, X, coef=1.7)
        assert ok
        Ae = EX.affine_element(dim, k, B, coef=1.7)
        assert np.linalg.norm(A - Ae) <= 1e-13 * np.linalg.norm(Ae)


@pytest.mark.parametrize("dim,k", [(d, k) for d in (2, 3) for k in (1, 2, 3)] + [(3, 4)])
def test_elasticity_element_affine_closed_form(dim, k):
    x0, B = _random_affine(dim, 3)
    X = EX.affine_cell_vertices(x0, B)
    lam, mu = O.lame(1.0, 0.3)
    A, ok = O.element_matrix(dim, k, X, coef=0.8, problem="elasticity", young=1.0, nu=0.3)
    assert ok
    Ae = EX.affine_element(dim, k, B, problem="elasticity", coef=0.8, lam=lam, mu=mu)
    assert np.linalg.norm(A - Ae) <= 1e-13 * np.linalg.norm(Ae)


def test_q1_unit_cube_and_square_textbook_values():
    """Q1 Laplace stiffness of the unit cube: (1/12)*[4 on the diagonal, 0 for
    edge-adjacent, -1 for face-diagonal and body-diagonal vertex pairs]; unit
    square: (1/6)*[4, -1 edge-adjacent, -2 diagonal]."""
    for dim, scale, table in ((3, 12.0, {0: 4, 1: 0, 2: -1, 3: -1}), (2, 6.0, {0: 4, 1: -1, 2: -2})):
        X = EX.affine_cell_vertices(np.zeros(dim), np.eye(dim))
        A, ok = O.element_matrix(dim, 1, X)
        for u in range(1 << dim):
            for v in range(1 << dim):
                ham = bin(u ^ v).count("1")
                assert abs(A[u, v] * scale - table[ham]) < 1e-14
        # side h scales by h^(d-2)
        A2, _ = O.element_matrix(dim, 1, 0.5 * X)
        np.testing.assert_allclose(A2, A * 0.5 ** (dim - 2), atol=1e-15)


def test_energy_of_linear_fields():
    """u^T A u for a linear field equals the continuum energy on the cell:
    Poisson |c|^2 vol; elasticity vol (2 mu |sym B|^2 + lambda (tr B)^2)."""
    r = np.random.Generator(np.random.PCG64(7))
    for dim in (2, 3):
        for k in (1, 2, 3):
            x0, B = _random_affine(dim, 11 + k)
            X = EX.affine_cell_vertices(x0, B)
            vol = abs(np.linalg.det(B))
            nn = (k + 1) ** dim
            nodes = np.array([x0 + B @ (np.array([(a // (k + 1) ** r) % (k + 1) for r in range(dim)]) / k)
                              for a in range(nn)])
            c = r.standard_normal(dim)
            A, _ = O.element_matrix(dim, k, X)
            u = nodes @ c
            assert abs(u @ A @ u - vol * c @ c) < 1e-12 * max(1.0, vol * c @ c)
            G = r.standard_normal((dim, dim))
            lam, mu = O.lame(1.0, 0.3)
            Ae, _ = O.element_matrix(dim, k, X, problem="elasticity")
            U = (nodes @ G.T).reshape(-1)  # interleaved: node a, component c
            eps = 0.5 * (G + G.T)
            energy = vol * (2 * mu * (eps * eps).sum() + lam * np.trace(G) ** 2)
            assert abs(U @ Ae @ U - energy) < 1e-12 * energy


# --------------------------------------------------------------------------
# Invariants on jittered cells
# --------------------------------------------------------------------------
def _rigid_modes(dim, nodes):
    nn = len(nodes)
    modes = []
    for c in range(dim):
        m = np.zeros((nn, dim))
        m[:, c] = 1
        modes.append(m.reshape(-1))
    pairs = [(0, 1)] if dim == 2 else [(0, 1), (1, 2), (0, 2)]
    for i, j in pairs:
        m = np.zeros((nn, dim))
        m[:, i] = -nodes[:, j]
        m[:, j] = nodes[:, i]
        modes.append(m.reshape(-1))
    return np.array(modes)


@pytest.mark.parametrize("dim,k", [(2, 1), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_jittered_element_invariants(dim, k):
    v = structured_vertices(dim, 3, jitter=0.2, seed=99)
    cell = 13 if dim == 3 else 4  # the centre cell, all vertices jittered
    X = O.cell_vertices(dim, [3] * dim, v, cell)
    A, ok = O.element_matrix(dim, k, X, coef=2.5)
    assert ok
    nrm = np.linalg.norm(A)
    assert np.abs(A - A.T).max() <= 1e-13 * nrm
    assert np.abs(A @ np.ones(len(A))).max() <= 1e-13 * nrm
    ev = np.linalg.eigvalsh(A)
    assert (ev > 1e-10 * ev[-1]).sum() == len(A) - 1
    # elasticity: the rigid-body modes span the kernel
    Ae, ok = O.element_matrix(dim, k, X, problem="elasticity")
    nrm = np.linalg.norm(Ae)
    assert np.abs(Ae - Ae.T).max() <= 1e-13 * nrm
    nn = (k + 1) ** dim
    # node positions: image of the reference lattice under the bilinear map
    t = np.array([[(a // (k + 1) ** r) % (k + 1) / k for r in range(dim)] for a in range(nn)])
    N = np.ones((nn, 1 << dim))
    for vv in range(1 << dim):
        for r in range(dim):
            N[:, vv] *= t[:, r] if (vv >> r) & 1 else 1 - t[:, r]
    nodes = N @ X
    R = _rigid_modes(dim, nodes)
    assert np.abs(Ae @ R.T).max() <= 1e-12 * nrm
    ev = np.linalg.eigvalsh(Ae)
    nkern = 3 if dim == 2 else 6
    assert (ev > 1e-10 * ev[-1]).sum() == len(Ae) - nkern


def test_inverted_cell_is_flagged():
    X = EX.affine_cell_vertices(np.zeros(3), np.eye(3))
    X[[0, 1]] = X[[1, 0]]  # swap two vertices -> det J < 0 somewhere
    _, ok = O.element_matrix(3, 1, X)
    assert not ok


# --------------------------------------------------------------------------
# Global structure
# --------------------------------------------------------------------------
def _pairs_1d(n, k, lo_fixed=True, hi_fixed=True):
    """Brute-force count of (i, j) free node pairs of the 1D lattice that
    share a cell."""
    N = n * k
    free = [i for i in range(N + 1) if not ((i == 0 and lo_fixed) or (i == N and hi_fixed))]
    cells = [set(range(e * k, e * k + k + 1)) for e in range(n)]
    cnt = 0
    for i in free:
        for j in free:
            if any(i in c and j in c for c in cells):
                cnt += 1
    return cnt


@pytest.mark.parametrize("dim,n,k,prob", [(2, 4, 1, "poisson"), (2, 3, 3, "poisson"), (3, 3, 1, "poisson"),
                                          (3, 2, 2, "elasticity"), (3, 2, 3, "poisson"), (2, 3, 2, "elasticity")])
def test_pattern_nnz_closed_form_and_symmetry(dim, n, k, prob):
    P = O.Problem(dim, [n] * dim, k, problem=prob)
    v = structured_vertices(dim, n, jitter=0.2, seed=5)
    S = O.System(P, v)
    assert S.nnz == _pairs_1d(n, k) ** dim * P.ncomp ** 2
    M = S.scipy()
    pat = (M != 0).astype(int)  # values may be exactly zero, so compare the structure instead
    rows = np.repeat(np.arange(S.nfree), np.diff(S.rowptr))
    st = set(zip(rows.tolist(), S.colind.tolist()))
    assert all((c, r) in st for r, c in st)
    for r in range(S.nfree):
        cols = S.colind[S.rowptr[r]:S.rowptr[r + 1]]
        assert np.all(np.diff(cols) > 0)
    del pat


def test_uniform_q1_stencils():
    """Interior row of the uniform Q1 Laplacian: 3D centre 8h/3, face
    neighbours 0, edge neighbours -h/6, corner neighbours -h/12; 2D centre 8/3,
    the eight neighbours -1/3."""
    n = 4
    for dim in (2, 3):
        P = O.Problem(dim, [n] * dim, 1)
        S = O.System(P, structured_vertices(dim, n))
        h = 1.0 / n
        # the centre node (2,2[,2]) has free rank with the boundary removed
        rank = sum((2 - 1) * (n - 1) ** r for r in range(dim))
        cols = S.colind[S.rowptr[rank]:S.rowptr[rank + 1]]
        vals = S.values[S.rowptr[rank]:S.rowptr[rank + 1]]
        assert len(cols) == 3 ** dim
        for c, val in zip(cols, vals):
            off = [(c // (n - 1) ** r) % (n - 1) - 1 for r in range(dim)]
            m = sum(abs(o) for o in off)
            if dim == 3:
                expect = {0: 8 * h / 3, 1: 0.0, 2: -h / 6, 3: -h / 12}[m]
            else:
                expect = {0: 8 / 3, 1: -1 / 3, 2: -1 / 3}[m]
            assert abs(val - expect) < 1e-14


@pytest.mark.parametrize("dim,k,prob", [(2, 2, "poisson"), (3, 1, "poisson"), (3, 3, "poisson"),
                                        (3, 2, "elasticity"), (2, 3, "elasticity")])
def test_global_kernel_and_load_without_dirichlet(dim, k, prob):
    """With no Dirichlet faces: A 1 = 0 (Poisson), A r = 0 for rigid modes
    (elasticity); sum of rhs = int f over the (jittered) unit domain."""
    n = 3
    P = O.Problem(dim, [n] * dim, k, problem=prob, faces=0, source_kind=1, source=(1.0, -2.0, 0.5))
    v = structured_vertices(dim, n, jitter=0.2, seed=21)
    coef = lognormal_coefficients(P.ncells, seed=22)
    S = O.System(P, v, coef)
    M = S.scipy()
    nrm = abs(M).sum(axis=1).max()
    nnodes = S.nfree // P.ncomp
    # node coordinates of the global lattice (images of the reference lattice)
    coords = np.zeros((nnodes, dim))
    for K in range(P.ncells):
        X = O.cell_vertices(dim, P.n, v, K)
        t = np.array([[(a // (k + 1) ** r) % (k + 1) / k for r in range(dim)] for a in range(P.nn)])
        N = np.ones((P.nn, 1 << dim))
        for vv in range(1 << dim):
            for r in range(dim):
                N[:, vv] *= t[:, r] if (vv >> r) & 1 else 1 - t[:, r]
        coords[S.cell_dofs[K, ::P.ncomp] // P.ncomp] = N @ X
    if prob == "poisson":
        assert np.abs(M @ np.ones(S.nfree)).max() <= 1e-12 * nrm
        assert abs(S.rhs.sum() - 1.0) < 1e-13
    else:
        for m in _rigid_modes(dim, coords):
            assert np.abs(M @ m).max() <= 1e-12 * nrm
        for c in range(dim):
            assert abs(S.rhs[c::dim].sum() - P.source[c]) < 1e-13


def test_coo_compression_equals_csr():
    """The paper's COO build-up + compression (duplicates summed) gives the
    same CSR as the symbolic + numeric path."""
    P = O.Problem(3, [2, 3, 2], 2, faces=0b000011, source_kind=1, source=(1.0,))
    v = structured_vertices(3, [2, 3, 2], jitter=0.2, seed=4)
    coef = lognormal_coefficients(P.ncells, seed=8)
    S = O.System(P, v, coef)
    rows, cols, vals = [], [], []
    for K in range(P.ncells):
        A, _ = O.element_matrix(3, 2, O.cell_vertices(3, P.n, v, K), coef=coef[K])
        g = S.cell_dofs[K]
        for a in range(P.nloc):
            for b in range(P.nloc):
                if g[a] >= 0 and g[b] >= 0:
                    rows.append(g[a])
                    cols.append(g[b])
                    vals.append(A[a, b])
    rp, ci, vv = O.coo_compress(rows, cols, vals, S.nfree)
    np.testing.assert_array_equal(rp, S.rowptr)
    np.testing.assert_array_equal(ci, S.colind)
    np.testing.assert_allclose(vv, S.values, rtol=0, atol=1e-13 * np.abs(vv).max())


def test_assemble_row_matches_full_assembly():
    P = O.Problem(3, [3, 2, 2], 2, problem="elasticity", faces=0b000101, source_kind=1, source=(0, 0, -1),
                  dirichlet_kind=1, dirichlet_affine=[0.1, 0.2, 0, 0, 0, 0, 0.3, 0, -0.1, 0, 0, 0.2])
    v = structured_vertices(3, [3, 2, 2], jitter=0.2, seed=6)
    coef = lognormal_coefficients(P.ncells, seed=9)
    S = O.System(P, v, coef)
    for row in [0, 5, S.nfree // 2, S.nfree - 1]:
        cols, vals, rhs = O.assemble_row(P, v, coef, S.cell_dofs, row)
        np.testing.assert_array_equal(cols, S.colind[S.rowptr[row]:S.rowptr[row + 1]])
        np.testing.assert_allclose(vals, S.values[S.rowptr[row]:S.rowptr[row + 1]], rtol=0, atol=1e-14)
        assert abs(rhs - S.rhs[row]) < 1e-14


# --------------------------------------------------------------------------
# Linear patch test (exact) and convergence on a manufactured solution
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dim,k,n,prob", [(2, 1, 5, "poisson"), (2, 3, 3, "poisson"), (2, 4, 2, "poisson"),
                                          (3, 1, 4, "poisson"), (3, 2, 3, "poisson"), (3, 4, 2, "poisson"),
                                          (3, 1, 3, "elasticity"), (3, 2, 2, "elasticity"), (2, 3, 3, "elasticity")])
def test_linear_patch_test(dim, k, n, prob):
    r = np.random.Generator(np.random.PCG64(100 + 10 * dim + k))
    ncomp = dim if prob == "elasticity" else 1
    aff = np.zeros(12)
    for c in range(ncomp):
        aff[4 * c:4 * c + 1 + dim] = r.uniform(-1, 1, 1 + dim)
    P = O.Problem(dim, [n] * dim, k, problem=prob, dirichlet_kind=1, dirichlet_affine=aff)
    v = structured_vertices(dim, n, jitter=0.2, seed=31 + n)
    S = O.System(P, v, None)
    x = spla.spsolve(S.scipy().tocsc(), S.rhs)
    # exact nodal values of the affine field at every free node
    nnodes = S.nfree // ncomp
    coords = np.zeros((nnodes, dim))
    for K in range(P.ncells):
        X = O.cell_vertices(dim, P.n, v, K)
        t = np.array([[(a // (k + 1) ** rr) % (k + 1) / k for rr in range(dim)] for a in range(P.nn)])
        N = np.ones((P.nn, 1 << dim))
        for vv in range(1 << dim):
            for rr in range(dim):
                N[:, vv] *= t[:, rr] if (vv >> rr) & 1 else 1 - t[:, rr]
        g = S.cell_dofs[K, ::ncomp]
        free = g >= 0
        coords[g[free] // ncomp] = (N @ X)[free]
    for c in range(ncomp):
        ue = aff[4 * c] + coords @ aff[4 * c + 1:4 * c + 1 + dim]
        assert np.abs(x[c::ncomp] - ue).max() < 1e-12
    # the L2 error of the discrete solution is also zero
    err = O.l2_error(P, v, S.cell_dofs, x, k + 3, 2, aff)
    assert err < 1e-12


def _l2_rate(dim, k, ns, jitter=0.0):
    errs = []
    for n in ns:
        P = O.Problem(dim, [n] * dim, k, source_kind=2, source=(1.0,))
        v = structured_vertices(dim, n, jitter=jitter, seed=40 + n)
        S = O.System(P, v, None)
        x = spla.spsolve(S.scipy().tocsc(), S.rhs)
        errs.append(O.l2_error(P, v, S.cell_dofs, x, k + 3, 1, [1.0]))
    return errs, np.log(errs[-2] / errs[-1]) / np.log(ns[-1] / ns[-2])


@pytest.mark.parametrize("dim,k,ns", [(2, 1, [8, 16, 32]), (2, 2, [4, 8, 16]), (2, 3, [4, 8, 16]),
                                      (2, 4, [2, 4, 8]), (3, 1, [4, 8, 16]), (3, 2, [2, 4, 8])])
def test_l2_convergence_rate(dim, k, ns):
    # Q_k on shape-regular meshes converges at exactly O(h^{k+1}) in L2 for a
    # smooth solution: the rate is bounded on both sides (a squared or
    # unsquared norm would double or halve it)
    errs, rate = _l2_rate(dim, k, ns)
    assert k + 1 - 0.15 <= rate <= k + 1 + 0.15, (errs, rate)


def test_l2_convergence_rate_jittered():
    errs, rate = _l2_rate(2, 2, [8, 16, 32], jitter=0.2)
    assert 3 - 0.3 <= rate <= 3 + 0.3, (errs, rate)


def _l2_of_field(dim, k, n, jitter, problem, exact_kind, exact, xval=0.0, uD=None):
    """The oracle's L2 error of the discrete field that is ``xval`` at every
    free DOF and ``uD`` (affine datum, kind 1) or 0 at every fixed DOF."""
    P = O.Problem(dim, [n] * dim, k, problem=problem, dirichlet_kind=0 if uD is None else 1,
                  dirichlet_affine=uD)
    v = structured_vertices(dim, n, jitter=jitter, seed=70 + n + k)
    code, nfree_nodes, _ = O.number_nodes(dim, P.n, k, P.faces)
    cd = O.cell_dofs(P, code)
    x = np.full(nfree_nodes * P.ncomp, float(xval))
    return O.l2_error(P, v, cd, x, k + 3, exact_kind, exact)


def _affine_norm2(a, b):
    """Closed form of the integral of (a + b.x)^2 over the unit cube [0,1]^d:
    a^2 + a sum(b) + sum(b^2)/3 + sum_{r<s} b_r b_s / 2."""
    b = list(b)
    cross = sum(b[r] * b[s] for r in range(len(b)) for s in range(r + 1, len(b)))
    return a * a + a * sum(b) + sum(t * t for t in b) / 3.0 + cross / 2.0


@pytest.mark.parametrize("dim,k,n,jitter", [(2, 1, 8, 0.0), (2, 2, 6, 0.2), (2, 4, 4, 0.2),
                                            (3, 1, 5, 0.0), (3, 2, 4, 0.2), (3, 3, 3, 0.2)])
def test_l2_norm_of_sine_product_closed_form(dim, k, n, jitter):
    # A zero discrete field: the oracle's error is the L2 norm of
    # prod_r sin(pi x_r) over the unit square/cube, whose square is 2^-d
    # (each factor integrates sin^2 to 1/2).  Boundary vertices are fixed, so
    # the jittered mesh still tiles the unit cube exactly.
    err = _l2_of_field(dim, k, n, jitter, "poisson", 1, [1.0])
    assert abs(err - 2.0 ** (-dim / 2.0)) <= 1e-10 * 2.0 ** (-dim / 2.0), err


@pytest.mark.parametrize("dim,k,n,jitter", [(2, 1, 4, 0.2), (2, 3, 3, 0.2), (3, 1, 3, 0.2), (3, 2, 2, 0.2)])
def test_l2_norm_of_affine_field_is_exact(dim, k, n, jitter):
    # (a + b.x)^2 |det J| is a polynomial of degree <= 4 per reference
    # variable on a multilinear cell, so k+3 >= 4 Gauss points give the exact
    # integral: the closed form holds to rounding.
    a, b = 0.7, [1.5, -2.0, 0.25][:dim]
    ex = [a] + b + [0.0] * (3 - dim)
    err = _l2_of_field(dim, k, n, jitter, "poisson", 2, ex)
    assert abs(err - np.sqrt(_affine_norm2(a, b))) <= 1e-13, err
    # a nonzero discrete field: the constant c at every DOF (free values and an
    # affine Dirichlet datum with no slope), so u - u_h = (a - c) + b.x
    c = -0.4
    uD = [c] + [0.0] * 11
    err = _l2_of_field(dim, k, n, jitter, "poisson", 2, ex, xval=c, uD=uD)
    assert abs(err - np.sqrt(_affine_norm2(a - c, b))) <= 1e-13, err


def test_l2_norm_of_vector_field_sums_components():
    # a vector field's squared norm is the sum of its components' squared
    # norms: exact = (1, -2, 0.5) times the sine product, squared norm
    # (1 + 4 + 0.25) / 8 on the unit cube
    err = _l2_of_field(3, 2, 3, 0.2, "elasticity", 1, [1.0, -2.0, 0.5])
    ref = np.sqrt(5.25 / 8.0)
    assert abs(err - ref) <= 1e-8 * ref, err


# --------------------------------------------------------------------------
# Solver: PCG against a direct solve, SPD, Lanczos bounds
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dim,k,prob", [(2, 2, "poisson"), (3, 1, "poisson"), (3, 2, "elasticity")])
def test_pcg_matches_direct_solve_and_lanczos_bounds(dim, k, prob):
    n = 4 if dim == 3 else 8
    P = O.Problem(dim, [n] * dim, k, problem=prob, source_kind=1, source=(1.0, 0.0, -1.0))
    v = structured_vertices(dim, n, jitter=0.2, seed=50)
    coef = lognormal_coefficients(P.ncells, seed=51)
    S = O.System(P, v, coef)
    Ad = S.dense()
    np.linalg.cholesky(Ad)  # SPD after elimination
    xd = np.linalg.solve(Ad, S.rhs)
    res = O.pcg(S.rowptr, S.colind, S.values, S.rhs, 1e-13, 5000)
    assert res["status"] == 0
    assert np.linalg.norm(S.rhs - Ad @ res["x"]) <= 1e-12 * np.linalg.norm(S.rhs)
    dinv = 1.0 / np.sqrt(np.diag(Ad))
    ev = np.linalg.eigvalsh(Ad * dinv[:, None] * dinv[None, :])
    kappa = ev[-1] / ev[0]
    assert np.linalg.norm(res["x"] - xd) <= 10 * kappa * 1e-13 * np.linalg.norm(xd)
    lo, hi = O.lanczos_extremes(res["alphas"], res["betas"])
    assert ev[0] * (1 - 1e-8) <= lo <= hi <= ev[-1] * (1 + 1e-8)
    assert hi > 0.9 * ev[-1] and lo < 1.5 * ev[0]


def test_pcg_flags_breakdown_and_maxit():
    # indefinite matrix -> breakdown; maxit=1 on a real system -> not converged
    rowptr = np.array([0, 1, 2], dtype=np.int64)
    colind = np.array([0, 1], dtype=np.int32)
    res = O.pcg(rowptr, colind, np.array([1.0, -1.0]), np.array([1.0, 1.0]), 1e-12, 10)
    assert res["status"] == 2
    P = O.Problem(2, [6, 6], 1, source_kind=1, source=(1.0,))
    S = O.System(P, structured_vertices(2, 6))
    res = O.pcg(S.rowptr, S.colind, S.values, S.rhs, 1e-12, 1)
    assert res["status"] == 1 and res["iters"] == 1


# --------------------------------------------------------------------------
# The paper's owner-cell DOF numbering (Sect. 10.3) against the canonical
# lattice numbering: the same system up to a symmetric permutation
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dim,n,k,prob,faces", [(2, [3, 4], 1, "poisson", None), (2, [3, 2], 3, "poisson", 0b0101),
                                                (3, [2, 3, 2], 2, "poisson", None),
                                                (3, [2, 2, 3], 1, "elasticity", 0b000011),
                                                (3, [2, 2, 2], 2, "elasticity", None)])
def test_owner_cell_numbering_gives_the_same_system(dim, n, k, prob, faces):
    P = O.Problem(dim, n, k, problem=prob, source_kind=1, source=(1.0, -0.5, 2.0), faces=faces,
                  dirichlet_kind=1, dirichlet_affine=[0.3, 1.0, -2.0, 0.5, -0.1, 0.2, 0.7, -1.1, 0.4, 0.0, 0.9, 0.6])
    v = structured_vertices(dim, n, jitter=0.2, seed=90)
    coef = lognormal_coefficients(P.ncells, seed=91)
    S = O.System(P, v, coef)
    cd, nfree, nfixed = O.owner_cell_numbering(P)
    # the paper's numbering counts the same free and fixed DOFs
    assert (nfree, nfixed) == (S.nfree, S.nfixed)
    # it is a bijection of the canonical one, free onto free, fixed onto fixed
    perm = np.full(nfree, -1, dtype=np.int64)
    canon, own = S.cell_dofs.reshape(-1), cd.reshape(-1)
    assert np.array_equal(canon >= 0, own >= 0)
    free = canon >= 0
    perm[canon[free]] = own[free]
    pairs = set(zip(canon[free].tolist(), own[free].tolist()))
    assert len(pairs) == nfree and sorted(perm.tolist()) == list(range(nfree))
    if k >= 2:  # edge, face and cell nodes come before later vertices: a different order
        assert not np.array_equal(perm, np.arange(nfree))
    # the owner-numbered system, assembled by the same plain loops
    rp, ci = O.csr_pattern(cd, nfree)
    vals, rhs, ok = O.assemble(P, v, coef, cd, nfree, rp, ci)
    assert ok and rp[-1] == S.nnz
    A_own = np.zeros((nfree, nfree))
    for i in range(nfree):
        A_own[i, ci[rp[i]:rp[i + 1]]] = vals[rp[i]:rp[i + 1]]
    # contributions are summed in the same (cell, a, b) order: bitwise equal
    assert np.array_equal(A_own[np.ix_(perm, perm)], S.dense())
    assert np.array_equal(rhs[perm], S.rhs)


# --------------------------------------------------------------------------
# The all-cores build of the oracle (the CPU baseline's OpenMP leg) computes
# the same system as the serial oracle
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dim,n,k,prob", [(3, [5, 4, 3], 1, "poisson"), (3, [3, 2, 2], 2, "elasticity"),
                                          (2, [6, 5], 3, "poisson")])
def test_openmp_oracle_matches_serial_oracle(dim, n, k, prob):
    P = O.Problem(dim, n, k, problem=prob, source_kind=1, source=(1.0, -0.5, 0.25), faces=0b000101 if dim == 3
                  else 0b0101, dirichlet_kind=1, dirichlet_affine=[0.2, 1.0, -0.5, 0.3] * 3)
    v = structured_vertices(dim, n, jitter=0.2, seed=95)
    coef = lognormal_coefficients(P.ncells, seed=96)
    S = O.System(P, v, coef)
    rp, ci = O.omp_csr_pattern(S.cell_dofs, S.nfree)
    assert np.array_equal(rp, S.rowptr) and np.array_equal(ci, S.colind)
    vals, rhs, ok = O.omp_assemble(P, v, coef, S.cell_dofs, S.nfree, rp, ci)
    # same per-entry summation order: bitwise the serial assembly
    assert ok and np.array_equal(vals, S.values) and np.array_equal(rhs, S.rhs)
    res = O.omp_pcg(S.rowptr, S.colind, S.values, S.rhs, 1e-12, 20000)
    ref = O.pcg(S.rowptr, S.colind, S.values, S.rhs, 1e-12, 20000)
    assert res["status"] == 0 and abs(res["iters"] - ref["iters"]) <= 2
    assert np.linalg.norm(res["x"] - ref["x"]) <= 1e-9 * np.linalg.norm(ref["x"])
