"""GPU parity of Lagrangian P_k on simplicial meshes (Sect. 3.3, 3.5, 3.7)
against the oracle, through the C ABI.

* Small meshes (triangles and tetrahedra, orders 1-4, Poisson and
  elasticity, lognormal coefficients, zero and affine Dirichlet data, the
  Kuhn meshes as generated and with vertex labels, cell order and local
  vertex order shuffled): the cell-to-DOF map and the CSR pattern bit-exact;
  every element matrix (upper triangle) and load within 1e-12 of the
  oracle's; values, rhs and dinv within 1e-12 (relative Frobenius);
  repeated assembly bitwise equal.
* Jacobi-PCG on the assembled system against a direct solve of the oracle's.
* The 64^3 P2 workload the benchmark times (1,572,864 tetrahedra): the
  cell-to-DOF map bit-exact against the oracle's numbering of the whole mesh;
  sampled cells' element matrices and loads against the oracle; sampled rows
  (columns bit-exact, values and the CSR SpMV's products within 1e-12) built
  from the oracle's element matrices of the cells around each row; the
  solve's true residual.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import oracle as O
from fe_inputs import lognormal_coefficients, rng, simplex_mesh
from paper_1708_01773_amd import fe as F
from tests.gpu_util import MATRIX_RTOL, rel, say

pytestmark = pytest.mark.gpu

AFF = [0.3, 1.0, -2.0, 0.5, -0.7, 0.2, 0.4, 1.1, 0.9, -0.3, 0.6, -1.2]

CASES = [
    # dim, n, k, problem, shuffle, source_kind, dirichlet_kind
    (2, [3, 2], 1, "poisson", False, 2, 0),
    (2, [2, 3], 2, "poisson", True, 1, 1),
    (2, [2, 2], 3, "poisson", True, 2, 1),
    (2, [2, 2], 4, "poisson", False, 1, 0),
    (2, [2, 3], 2, "elasticity", True, 1, 1),
    (2, [2, 2], 3, "elasticity", False, 2, 0),
    (3, [2, 2, 1], 1, "poisson", True, 2, 1),
    (3, [2, 1, 2], 2, "poisson", False, 1, 0),
    (3, [1, 2, 2], 3, "poisson", True, 2, 1),
    (3, [1, 1, 2], 4, "poisson", True, 1, 1),
    (3, [2, 1, 1], 1, "elasticity", False, 1, 1),
    (3, [2, 1, 1], 2, "elasticity", True, 2, 1),
    (3, [1, 1, 1], 3, "elasticity", True, 1, 0),
]


def _ids(c):
    return f"{c[0]}d_{'x'.join(map(str, c[1]))}_p{c[2]}_{c[3][:4]}{'_shuf' if c[4] else ''}_f{c[5]}_d{c[6]}"


def build_pair(dim, n, k, problem, shuffle, source_kind, dirichlet_kind, seed=3):
    v, c = simplex_mesh(dim, n, jitter=0.2, shuffle=shuffle)
    coef = lognormal_coefficients(c.shape[0], seed=17081 + seed)
    src = (1.0, -0.5, 0.25)
    coeff = F.make_coeff(problem, "fp64", young=2.0, nu=0.3, source_kind=source_kind, source=src, dim=dim,
                         dirichlet_kind=dirichlet_kind, affine=AFF)
    G = F.Simplex(dim, v, c, k, coeff, cell_coeff=coef)
    G.assemble()
    torch.cuda.synchronize()
    S = O.SimplexSystem(dim, k, v, c, coef=coef, problem=problem, young=2.0, nu=0.3, source_kind=source_kind,
                        source=src, dirichlet_kind=dirichlet_kind, dirichlet_affine=AFF)
    assert S.ok
    return v, c, coef, G, S


def upper(A):
    n = A.shape[0]
    return A[np.triu_indices(n)]


@pytest.mark.parametrize("case", CASES, ids=[_ids(c) for c in CASES])
def test_simplex_system_matches_oracle(case):
    dim, n, k, problem, shuffle, sk, dk = case
    say(f"[simplex] {_ids(case)}")
    v, c, coef, G, S = build_pair(dim, n, k, problem, shuffle, sk, dk)
    assert (G.n_rows, G.nnz, G.n_nodes) == (S.nfree, S.nnz, S.nnodes)
    np.testing.assert_array_equal(G.cell_dofs().cpu().numpy(), S.cell_dofs)
    np.testing.assert_array_equal(G.rowptr.cpu().numpy(), S.rowptr)
    np.testing.assert_array_equal(G.colind[: G.nnz].cpu().numpy(), S.colind)
    # element matrices and loads, cell by cell
    E, Fl = G.elements()
    nc = dim if problem == "elasticity" else 1
    worst = 0.0
    for K in range(c.shape[0]):
        A, ok = O.simplex_element_matrix(dim, k, v[c[K]], coef=coef[K], problem=problem, young=2.0, nu=0.3)
        assert ok
        worst = max(worst, rel(E[K], upper(A)))
    assert worst <= MATRIX_RTOL, worst
    if dk == 0:
        for K in range(min(c.shape[0], 8)):
            f = O.simplex_element_load(dim, k, nc, v[c[K]], sk, (1.0, -0.5, 0.25))
            assert rel(Fl[K], f) <= MATRIX_RTOL
    ev = rel(G.values[: G.nnz].cpu().numpy(), S.values)
    er = rel(G.rhs[: G.n_rows].cpu().numpy(), S.rhs)
    ed = rel(G.dinv[: G.n_rows].cpu().numpy(), S.dinv)
    say(f"element {worst:.2e} values {ev:.2e} rhs {er:.2e} dinv {ed:.2e}")
    assert ev <= MATRIX_RTOL and er <= MATRIX_RTOL and ed <= MATRIX_RTOL
    # repeated assembly is bitwise the same
    v1 = G.values.clone()
    r1 = G.rhs.clone()
    G.assemble()
    torch.cuda.synchronize()
    assert torch.equal(v1, G.values) and torch.equal(r1, G.rhs)


@pytest.mark.parametrize("dim,n,k,problem", [(2, [6, 5], 2, "poisson"), (3, [3, 3, 2], 2, "poisson"),
                                             (3, [2, 2, 2], 3, "poisson"), (3, [3, 2, 2], 2, "elasticity")])
def test_simplex_pcg_matches_direct_solve_of_oracle(dim, n, k, problem):
    say(f"[simplex solve] dim={dim} n={n} k={k} {problem}")
    v, c, coef, G, S = build_pair(dim, n, k, problem, True, 2, 1)
    xo = S.solve()
    x = torch.zeros(G.n_rows, dtype=torch.float64, device="cuda")
    ws = torch.empty(F.pcg_query(G.n_rows), dtype=torch.uint8, device="cuda")
    info = F.pcg_solve(G.csr, G.rhs, x, 1e-12, 20000, ws)
    say(f"iters {info['iters']} true relres {info['true_relres']:.2e}")
    assert info["status"] == 0 and info["true_relres"] <= 1e-11
    assert rel(x.cpu().numpy(), xo) <= 1e-8


def test_simplex_meshes_without_free_dofs_and_with_one():
    # one tetrahedron: every P1..P3 node is on the boundary; P4 has one interior node
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    c = np.array([[0, 1, 2, 3]], dtype=np.int32)
    for k, rows in [(1, 0), (3, 0), (4, 1)]:
        coeff = F.make_coeff("poisson", "fp64", source_kind=1, source=(1.0,), dim=3)
        G = F.Simplex(3, v, c, k, coeff)
        assert G.n_rows == rows
        G.assemble()
        torch.cuda.synchronize()
        if rows:
            S = O.SimplexSystem(3, k, v, c, source_kind=1, source=(1.0,))
            assert rel(G.values[:1].cpu().numpy(), S.values) <= MATRIX_RTOL
            assert rel(G.rhs[:1].cpu().numpy(), S.rhs) <= MATRIX_RTOL


def test_simplex_rows_of_sampled_nodes_at_workload_size():
    """3D P2 on the Kuhn subdivision of the jittered 64^3 brick, lognormal
    coefficients, f = 1, u = 0 on the boundary: the system the benchmark's
    simplex form solves."""
    dim, n, k = 3, 64, 2
    say("[simplex workload] 64^3 Kuhn P2")
    v, c = simplex_mesh(dim, n, jitter=0.2)
    coef = lognormal_coefficients(c.shape[0])
    coeff = F.make_coeff("poisson", "fp64", source_kind=1, source=(1.0,), dim=dim)
    G = F.Simplex(dim, v, c, k, coeff, cell_coeff=coef)
    G.assemble()
    torch.cuda.synchronize()
    say(f"rows {G.n_rows} nnz {G.nnz} contributions {G.n_contrib}")
    assert G.n_rows == (k * n - 1) ** 3
    node_of, code, nfree, _ = O.simplex_number(dim, k, len(v), c)
    cd_o = code[node_of]  # scalar problem: the DOF is the node code
    cd = G.cell_dofs().cpu().numpy()
    np.testing.assert_array_equal(cd, cd_o)
    E, Fl = G.elements()
    g = rng(97)
    for K in list(g.integers(0, c.shape[0], size=24)) + [0, c.shape[0] - 1]:
        A, _ = O.simplex_element_matrix(dim, k, v[c[K]], coef=coef[K])
        assert rel(E[K], upper(A)) <= MATRIX_RTOL
        f = O.simplex_element_load(dim, k, 1, v[c[K]], 1, (1.0,))
        assert rel(Fl[K], f) <= MATRIX_RTOL
    rowptr = G.rowptr.cpu().numpy()
    x = g.standard_normal(G.n_rows)
    y = torch.full((G.n_rows,), np.nan, dtype=torch.float64, device="cuda")
    F.spmv(G.csr, torch.from_numpy(x).cuda(), y)
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    rows = list(g.integers(0, G.n_rows, size=30)) + [0, G.n_rows - 1]
    worst, worst_y = 0.0, 0.0
    for r in rows:
        Ks, As = np.nonzero(cd == r)
        acc = {}
        rhs = 0.0
        for K, a in zip(Ks, As):
            A, _ = O.simplex_element_matrix(dim, k, v[c[K]], coef=coef[K])
            f = O.simplex_element_load(dim, k, 1, v[c[K]], 1, (1.0,))
            rhs += f[a]
            for b in range(cd.shape[1]):
                if cd[K, b] >= 0:
                    acc[cd[K, b]] = acc.get(cd[K, b], 0.0) + A[a, b]
        cols = np.array(sorted(acc))
        vals = np.array([acc[j] for j in cols])
        r0, r1 = rowptr[r], rowptr[r + 1]
        np.testing.assert_array_equal(G.colind[r0:r1].cpu().numpy(), cols)
        worst = max(worst, rel(G.values[r0:r1].cpu().numpy(), vals), rel(G.rhs[r:r + 1].cpu().numpy(), [rhs]))
        worst_y = max(worst_y, abs(y[r] - vals @ x[cols]) / (np.abs(vals) @ np.abs(x[cols])))
    say(f"worst sampled-row rel err {worst:.2e}, SpMV {worst_y:.2e}")
    assert worst <= MATRIX_RTOL and worst_y <= 1e-12
    xs = torch.zeros(G.n_rows, dtype=torch.float64, device="cuda")
    ws = torch.empty(F.pcg_query(G.n_rows), dtype=torch.uint8, device="cuda")
    info = F.pcg_solve(G.csr, G.rhs, xs, 1e-8, 20000, ws)
    say(f"solve: iters {info['iters']} true relres {info['true_relres']:.2e}")
    assert info["status"] == 0 and info["true_relres"] <= 2e-8


# ---------------------------------------------------------------------------
# Nedelec (first and second order) and Raviart-Thomas elements (Sect. 3.9,
# 3.10)
# ---------------------------------------------------------------------------
VCASES = [
    # family, dim, n, shuffle, source_kind, dirichlet
    ("nedelec", 2, [3, 2], False, 1, True),
    ("nedelec", 2, [2, 3], True, 2, False),
    ("nedelec", 3, [2, 2, 1], True, 2, True),
    ("nedelec", 3, [2, 1, 2], False, 1, False),
    ("raviart_thomas", 2, [3, 2], True, 2, True),
    ("raviart_thomas", 2, [2, 2], False, 1, False),
    ("raviart_thomas", 3, [1, 2, 2], True, 1, True),
    ("raviart_thomas", 3, [2, 2, 2], True, 2, False),
    ("nedelec2", 2, [3, 2], True, 2, True),
    ("nedelec2", 2, [2, 3], False, 1, False),
    ("nedelec2", 3, [2, 2, 1], True, 2, True),
    ("nedelec2", 3, [1, 2, 2], True, 1, False),
    ("nedelec2", 3, [2, 1, 2], False, 2, False),
    ("raviart_thomas2", 2, [3, 2], True, 2, True),
    ("raviart_thomas2", 2, [2, 3], False, 1, False),
    ("raviart_thomas2", 3, [2, 2, 1], True, 2, True),
    ("raviart_thomas2", 3, [1, 2, 2], True, 1, False),
    ("raviart_thomas2", 3, [2, 1, 2], False, 2, False),
]


def _vids(c):
    return f"{c[0][:3]}{c[0][-1] if c[0][-1].isdigit() else ''}_{c[1]}d_{'x'.join(map(str, c[2]))}{'_shuf' if c[3] else ''}_f{c[4]}{'_dir' if c[5] else ''}"


def build_vector_pair(family, dim, n, shuffle, sk, dirichlet, kappa=0.8, seed=5):
    v, c = simplex_mesh(dim, n, jitter=0.2, shuffle=shuffle)
    coef = lognormal_coefficients(c.shape[0], seed=17081 + seed)
    src = (1.0, -0.5, 0.25)
    coeff = F.make_coeff("poisson", "fp64", source_kind=sk, source=src, dim=dim, faces=None if dirichlet else 0)
    G = F.Simplex(dim, v, c, 0, coeff, cell_coeff=coef, family=family, kappa=kappa)
    G.assemble()
    torch.cuda.synchronize()
    S = O.VectorSystem(family, dim, v, c, coef=coef, kappa=kappa, source_kind=sk, source=src, dirichlet=dirichlet)
    assert S.ok
    return v, c, coef, G, S


@pytest.mark.parametrize("case", VCASES, ids=[_vids(c) for c in VCASES])
def test_vector_element_system_matches_oracle(case):
    family, dim, n, shuffle, sk, dirichlet = case
    say(f"[vector] {_vids(case)}")
    v, c, coef, G, S = build_vector_pair(family, dim, n, shuffle, sk, dirichlet)
    assert (G.n_rows, G.nnz, G.n_nodes) == (S.nfree, S.nnz, S.nent)
    np.testing.assert_array_equal(G.cell_dofs().cpu().numpy(), S.cell_dofs)
    np.testing.assert_array_equal(G.rowptr.cpu().numpy(), S.rowptr)
    np.testing.assert_array_equal(G.colind[: G.nnz].cpu().numpy(), S.colind)
    E, Fl = G.elements()
    worst = 0.0
    for K in range(c.shape[0]):
        A, f, ok = O.vector_element(family, dim, v[c[K]], c[K], coef=coef[K], kappa=0.8, source_kind=sk,
                                    source=(1.0, -0.5, 0.25))
        assert ok
        worst = max(worst, rel(E[K], upper(A)), rel(Fl[K], f))
    ev = rel(G.values[: G.nnz].cpu().numpy(), S.values)
    er = rel(G.rhs[: G.n_rows].cpu().numpy(), S.rhs)
    ed = rel(G.dinv[: G.n_rows].cpu().numpy(), S.dinv)
    say(f"element {worst:.2e} values {ev:.2e} rhs {er:.2e} dinv {ed:.2e}")
    assert worst <= MATRIX_RTOL and ev <= MATRIX_RTOL and er <= MATRIX_RTOL and ed <= MATRIX_RTOL
    v1 = G.values.clone()
    G.assemble()
    torch.cuda.synchronize()
    assert torch.equal(v1, G.values)


@pytest.mark.parametrize("family", ["nedelec", "raviart_thomas", "nedelec2", "raviart_thomas2"])
@pytest.mark.parametrize("dim", [2, 3])
def test_vector_single_cell_with_and_without_free_dofs(family, dim):
    """One reference-shaped cell with its vertices listed out of order: with a
    zero trace every edge, facet and face DOF is fixed (the interior DOFs of
    the second-order triangle, and of second-order Raviart-Thomas, stay free);
    without, every DOF is free and the system is the cell's matrix in the
    global frame."""
    if dim == 3:
        v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64) * 0.7
        c = np.array([[2, 0, 3, 1]], dtype=np.int32)
    else:
        v = np.array([[0, 0], [1, 0], [0.2, 0.9]], dtype=np.float64)
        c = np.array([[1, 2, 0]], dtype=np.int32)
    say(f"[vector single cell] {family} dim={dim}")
    for dirichlet in (True, False):
        coeff = F.make_coeff("poisson", "fp64", source_kind=1, source=(1.0, -0.5, 0.25), dim=dim,
                             faces=None if dirichlet else 0)
        G = F.Simplex(dim, v, c, 0, coeff, cell_coeff=np.array([1.3]), family=family, kappa=0.8)
        G.assemble()
        torch.cuda.synchronize()
        S = O.VectorSystem(family, dim, v, c, coef=np.array([1.3]), kappa=0.8, source_kind=1,
                           source=(1.0, -0.5, 0.25), dirichlet=dirichlet)
        assert S.ok
        assert (G.n_rows, G.nnz, G.n_nodes) == (S.nfree, S.nnz, S.nent)
        np.testing.assert_array_equal(G.cell_dofs().cpu().numpy(), S.cell_dofs)
        if dirichlet:
            interior = {"nedelec2": 2 if dim == 2 else 0, "raviart_thomas2": dim}.get(family, 0)
            assert G.n_rows == interior
        else:
            assert G.n_rows == G.cell_dofs().shape[1]
        if G.n_rows:
            np.testing.assert_array_equal(G.rowptr.cpu().numpy(), S.rowptr)
            np.testing.assert_array_equal(G.colind[: G.nnz].cpu().numpy(), S.colind)
            assert rel(G.values[: G.nnz].cpu().numpy(), S.values) <= MATRIX_RTOL
            assert rel(G.rhs[: G.n_rows].cpu().numpy(), S.rhs) <= MATRIX_RTOL
            assert rel(G.dinv[: G.n_rows].cpu().numpy(), S.dinv) <= MATRIX_RTOL


@pytest.mark.parametrize("family,dim,n", [("nedelec", 3, [3, 3, 2]), ("raviart_thomas", 3, [3, 2, 2]),
                                          ("nedelec", 2, [6, 5]), ("nedelec2", 3, [2, 2, 2]),
                                          ("nedelec2", 2, [5, 4]), ("raviart_thomas2", 3, [2, 2, 2]),
                                          ("raviart_thomas2", 2, [5, 4])])
def test_vector_element_pcg_matches_direct_solve_of_oracle(family, dim, n):
    say(f"[vector solve] {family} dim={dim} n={n}")
    v, c, coef, G, S = build_vector_pair(family, dim, n, True, 2, True, kappa=1.0)
    xo = S.solve()
    x = torch.zeros(G.n_rows, dtype=torch.float64, device="cuda")
    ws = torch.empty(F.pcg_query(G.n_rows), dtype=torch.uint8, device="cuda")
    info = F.pcg_solve(G.csr, G.rhs, x, 1e-12, 20000, ws)
    say(f"iters {info['iters']} true relres {info['true_relres']:.2e}")
    assert info["status"] == 0 and info["true_relres"] <= 1e-11
    assert rel(x.cpu().numpy(), xo) <= 1e-8


def test_nedelec_rows_of_sampled_edges_at_workload_size():
    """Lowest-order Nedelec on the Kuhn subdivision of the jittered 64^3
    brick (the benchmark's vector workload): curl curl u + u = f with the
    manufactured field's load, zero tangential trace, lognormal coefficient."""
    dim, n = 3, 64
    say("[nedelec workload] 64^3 Kuhn")
    v, c = simplex_mesh(dim, n, jitter=0.2)
    coef = lognormal_coefficients(c.shape[0])
    lap = 2.0 * np.pi ** 2
    src = (lap + 1.0,) * 3
    coeff = F.make_coeff("poisson", "fp64", source_kind=2, source=src, dim=dim)
    G = F.Simplex(dim, v, c, 0, coeff, cell_coeff=coef, family="nedelec", kappa=1.0)
    G.assemble()
    torch.cuda.synchronize()
    say(f"rows {G.n_rows} nnz {G.nnz} contributions {G.n_contrib}")
    dof_of, code, nfree, _ = O.vector_number("nedelec", dim, len(v), c)
    cd = G.cell_dofs().cpu().numpy()
    np.testing.assert_array_equal(cd, code[dof_of])
    assert G.n_rows == nfree
    E, Fl = G.elements()
    g = rng(98)
    for K in list(g.integers(0, c.shape[0], size=24)) + [0, c.shape[0] - 1]:
        A, f, _ = O.vector_element("nedelec", dim, v[c[K]], c[K], coef=coef[K], kappa=1.0, source_kind=2, source=src)
        assert rel(E[K], upper(A)) <= MATRIX_RTOL and rel(Fl[K], f) <= MATRIX_RTOL
    rowptr = G.rowptr.cpu().numpy()
    x = g.standard_normal(G.n_rows)
    y = torch.full((G.n_rows,), np.nan, dtype=torch.float64, device="cuda")
    F.spmv(G.csr, torch.from_numpy(x).cuda(), y)
    torch.cuda.synchronize()
    y = y.cpu().numpy()
    worst, worst_y = 0.0, 0.0
    for r in list(g.integers(0, G.n_rows, size=30)) + [0, G.n_rows - 1]:
        Ks, As = np.nonzero(cd == r)
        acc, rhs = {}, 0.0
        for K, a in zip(Ks, As):
            A, f, _ = O.vector_element("nedelec", dim, v[c[K]], c[K], coef=coef[K], kappa=1.0, source_kind=2,
                                       source=src)
            rhs += f[a]
            for b in range(cd.shape[1]):
                if cd[K, b] >= 0:
                    acc[cd[K, b]] = acc.get(cd[K, b], 0.0) + A[a, b]
        cols = np.array(sorted(acc))
        vals = np.array([acc[j] for j in cols])
        r0, r1 = rowptr[r], rowptr[r + 1]
        np.testing.assert_array_equal(G.colind[r0:r1].cpu().numpy(), cols)
        worst = max(worst, rel(G.values[r0:r1].cpu().numpy(), vals), rel(G.rhs[r:r + 1].cpu().numpy(), [rhs]))
        worst_y = max(worst_y, abs(y[r] - vals @ x[cols]) / (np.abs(vals) @ np.abs(x[cols])))
    say(f"worst sampled-row rel err {worst:.2e}, SpMV {worst_y:.2e}")
    assert worst <= MATRIX_RTOL and worst_y <= 1e-12
    xs = torch.zeros(G.n_rows, dtype=torch.float64, device="cuda")
    ws = torch.empty(F.pcg_query(G.n_rows), dtype=torch.uint8, device="cuda")
    info = F.pcg_solve(G.csr, G.rhs, xs, 1e-8, 20000, ws)
    say(f"solve: iters {info['iters']} true relres {info['true_relres']:.2e}")
    assert info["status"] == 0 and info["true_relres"] <= 2e-8


def test_nedelec2_sampled_cells_numbering_and_solve_at_24():
    """Second-order Nedelec on the shuffled Kuhn subdivision of the jittered
    24^3 brick: the numbering bit-exact against the oracle's, sampled element
    matrices and loads in the global frame, then Jacobi-PCG to 1e-8."""
    dim, n = 3, 24
    say("[nedelec2] 24^3 shuffled Kuhn")
    v, c = simplex_mesh(dim, n, jitter=0.2, shuffle=True)
    coef = lognormal_coefficients(c.shape[0])
    lap = 2.0 * np.pi ** 2
    src = (lap + 1.0,) * 3
    coeff = F.make_coeff("poisson", "fp64", source_kind=2, source=src, dim=dim)
    G = F.Simplex(dim, v, c, 0, coeff, cell_coeff=coef, family="nedelec2", kappa=1.0)
    G.assemble()
    torch.cuda.synchronize()
    say(f"rows {G.n_rows} nnz {G.nnz} contributions {G.n_contrib}")
    dof_of, code, nfree, _ = O.vector_number("nedelec2", dim, len(v), c)
    np.testing.assert_array_equal(G.cell_dofs().cpu().numpy(), code[dof_of])
    assert G.n_rows == nfree
    E, Fl = G.elements()
    g = rng(99)
    for K in list(g.integers(0, c.shape[0], size=24)) + [0, c.shape[0] - 1]:
        A, f, _ = O.vector_element("nedelec2", dim, v[c[K]], c[K], coef=coef[K], kappa=1.0, source_kind=2,
                                   source=src)
        assert rel(E[K], upper(A)) <= MATRIX_RTOL and rel(Fl[K], f) <= MATRIX_RTOL
    xs = torch.zeros(G.n_rows, dtype=torch.float64, device="cuda")
    ws = torch.empty(F.pcg_query(G.n_rows), dtype=torch.uint8, device="cuda")
    # the curl-free fields are damped only by the mass term: Jacobi-PCG needs
    # a few 10^4 iterations here
    info = F.pcg_solve(G.csr, G.rhs, xs, 1e-8, 60000, ws)
    say(f"solve: iters {info['iters']} true relres {info['true_relres']:.2e}")
    assert info["status"] == 0 and info["true_relres"] <= 2e-8


def test_raviart_thomas2_sampled_cells_numbering_and_solve_at_24():
    """Second-order Raviart-Thomas on the shuffled Kuhn subdivision of the
    jittered 24^3 brick: -grad(k div u) + u = f with the manufactured field's
    load, zero normal trace; the numbering bit-exact against the oracle's,
    sampled element matrices and loads in the global frame, then Jacobi-PCG
    to 1e-8."""
    dim, n = 3, 24
    say("[raviart_thomas2] 24^3 shuffled Kuhn")
    v, c = simplex_mesh(dim, n, jitter=0.2, shuffle=True)
    coef = lognormal_coefficients(c.shape[0])
    src = (np.pi ** 2 + 1.0,) * 3
    coeff = F.make_coeff("poisson", "fp64", source_kind=2, source=src, dim=dim)
    G = F.Simplex(dim, v, c, 0, coeff, cell_coeff=coef, family="raviart_thomas2", kappa=1.0)
    G.assemble()
    torch.cuda.synchronize()
    say(f"rows {G.n_rows} nnz {G.nnz} contributions {G.n_contrib}")
    dof_of, code, nfree, _ = O.vector_number("raviart_thomas2", dim, len(v), c)
    np.testing.assert_array_equal(G.cell_dofs().cpu().numpy(), code[dof_of])
    assert G.n_rows == nfree
    E, Fl = G.elements()
    g = rng(97)
    for K in list(g.integers(0, c.shape[0], size=24)) + [0, c.shape[0] - 1]:
        A, f, _ = O.vector_element("raviart_thomas2", dim, v[c[K]], c[K], coef=coef[K], kappa=1.0, source_kind=2,
                                   source=src)
        assert rel(E[K], upper(A)) <= MATRIX_RTOL and rel(Fl[K], f) <= MATRIX_RTOL
    xs = torch.zeros(G.n_rows, dtype=torch.float64, device="cuda")
    ws = torch.empty(F.pcg_query(G.n_rows), dtype=torch.uint8, device="cuda")
    info = F.pcg_solve(G.csr, G.rhs, xs, 1e-8, 60000, ws)
    say(f"solve: iters {info['iters']} true relres {info['true_relres']:.2e}")
    assert info["status"] == 0 and info["true_relres"] <= 2e-8
