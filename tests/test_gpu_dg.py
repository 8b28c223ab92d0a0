"""GPU parity of the interior-penalty DG assembly (Sect. 3.12 eq.
ip_dg_formulations, the facet matrices of eq. local_to_face_matrix) against
the oracle, through the C ABI.

* Small meshes (2D and 3D, orders 1-4, every tau of the family, cells with
  one cell along an axis): pattern bit-exact; values, rhs and dinv within
  1e-12 relative (Frobenius) of the oracle; for tau = 1 the off-diagonal
  blocks of the two cells of every facet are transposes to the last bit.
* The cell-block SpMV (pattern evaluated from the cell index) against the
  oracle's CSR SpMV, element-wise within 1e-12 (|A| |x|), on every small case
  and on sampled rows of the workload.
* The solve: Jacobi-PCG on the GPU system (CSR SpMV, and the cell-block
  SpMV) against a direct solve of the oracle's system.
* The 48^3 Q2 workload the benchmark times: the rows of sampled cells
  (corners, edges, faces, interior, random) against the oracle run on the
  block of cells around each (the rows of a cell depend only on it and its
  facet neighbours), bit-exact columns, values within 1e-12.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import oracle as O
from fe_inputs import rng, structured_vertices
from paper_1708_01773_amd import fe as F
from tests.gpu_util import MATRIX_RTOL, rel, say

pytestmark = pytest.mark.gpu

AFF = [0.3, 1.0, -2.0, 0.5]


def penalty(k):
    return 4.0 * (k + 1) ** 2


def gpu_dg(dim, n, k, v, gamma, tau, source_kind=1, source=(1.0,), dirichlet_kind=1, affine=AFF):
    mesh = F.create_mesh(dim, n, v)
    coeff = F.make_coeff("poisson", "fp64", source_kind=source_kind, source=source, dim=dim,
                         dirichlet_kind=dirichlet_kind, affine=affine)
    A = F.DGAssembly(mesh, k, coeff, gamma, tau)
    A.assemble()
    torch.cuda.synchronize()
    assert F.get_status(mesh) == F.FE_OK
    return mesh, coeff, A


CASES = [
    # dim, n, k, tau
    (2, [3, 2], 1, 1.0),
    (2, [4, 3], 2, -1.0),
    (2, [2, 3], 3, 1.0),
    (2, [2, 2], 4, 0.0),
    (2, [1, 3], 2, 1.0),
    (3, [3, 2, 2], 1, 1.0),
    (3, [2, 3, 2], 2, 0.0),
    (3, [4, 3, 2], 2, 1.0),
    (3, [2, 2, 1], 3, -1.0),
    (3, [1, 2, 2], 4, 1.0),
]


@pytest.mark.parametrize("dim,n,k,tau", CASES, ids=[f"{c[0]}d_{'x'.join(map(str, c[1]))}_q{c[2]}_tau{c[3]:+.0f}"
                                                    for c in CASES])
def test_dg_system_matches_oracle(dim, n, k, tau):
    say(f"[dg] dim={dim} n={n} k={k} tau={tau}")
    v = structured_vertices(dim, n, jitter=0.2, seed=91)
    gamma = penalty(k)
    mesh, coeff, A = gpu_dg(dim, n, k, v, gamma, tau)
    P = O.Problem(dim, n, k, source_kind=1, source=(1.0,), dirichlet_kind=1, dirichlet_affine=AFF)
    D = O.DGSystem(P, v, gamma=gamma, tau=tau)
    assert D.ok
    assert (A.n_rows, A.nnz) == (D.nfree, D.nnz)
    np.testing.assert_array_equal(A.rowptr.cpu().numpy(), D.rowptr)
    np.testing.assert_array_equal(A.colind[: A.nnz].cpu().numpy(), D.colind)
    vals = A.values[: A.nnz].cpu().numpy()
    rhs = A.rhs[: A.n_rows].cpu().numpy()
    dinv = A.dinv[: A.n_rows].cpu().numpy()
    ev, er = rel(vals, D.values), rel(rhs, D.rhs)
    diag = np.diag(D.dense())
    ed = rel(dinv, 1.0 / diag)
    say(f"values rel {ev:.2e} rhs rel {er:.2e} dinv rel {ed:.2e}")
    assert ev <= MATRIX_RTOL and er <= MATRIX_RTOL and ed <= MATRIX_RTOL
    if tau == 1.0:
        import scipy.sparse as sp
        M = sp.csr_matrix((vals, D.colind, D.rowptr), shape=(D.nfree, D.nfree)).tocoo()
        nn = P.nn
        off = (M.row // nn) != (M.col // nn)
        T = sp.csr_matrix((vals, D.colind, D.rowptr), shape=(D.nfree, D.nfree)).T.tocsr()
        # every off-diagonal block entry equals its transpose partner bit for bit
        r, c = M.row[off], M.col[off]
        np.testing.assert_array_equal(M.data[off], np.asarray(T[r, c]).ravel())


@pytest.mark.parametrize("dim,n,k,tau", CASES, ids=[f"{c[0]}d_{'x'.join(map(str, c[1]))}_q{c[2]}" for c in CASES])
def test_dg_cell_block_spmv_matches_oracle(dim, n, k, tau):
    say(f"[dg spmv] dim={dim} n={n} k={k}")
    v = structured_vertices(dim, n, jitter=0.2, seed=94)
    mesh, coeff, A = gpu_dg(dim, n, k, v, penalty(k), tau)
    P = O.Problem(dim, n, k, source_kind=1, source=(1.0,), dirichlet_kind=1, dirichlet_affine=AFF)
    D = O.DGSystem(P, v, gamma=penalty(k), tau=tau)
    x = rng(95).standard_normal(A.n_rows)
    xd = torch.from_numpy(x).cuda()
    y = torch.full_like(xd, np.nan)
    A.spmv(xd, y)
    torch.cuda.synchronize()
    yo = O.spmv(D.rowptr, D.colind, D.values, x)
    scale = O.spmv(D.rowptr, D.colind, np.abs(D.values), np.abs(x))
    assert np.all(np.abs(y.cpu().numpy() - yo) <= 1e-12 * scale + 1e-300)


@pytest.mark.parametrize("dim,n,k", [(2, [6, 5], 2), (3, [4, 3, 3], 2), (3, [3, 3, 2], 3)])
def test_dg_pcg_solution_matches_direct_solve_of_oracle(dim, n, k):
    say(f"[dg solve] dim={dim} n={n} k={k}")
    v = structured_vertices(dim, n, jitter=0.2, seed=92)
    gamma = penalty(k)
    mesh, coeff, A = gpu_dg(dim, n, k, v, gamma, 1.0, source_kind=2, source=(1.0,), dirichlet_kind=1)
    P = O.Problem(dim, n, k, source_kind=2, source=(1.0,), dirichlet_kind=1, dirichlet_affine=AFF)
    D = O.DGSystem(P, v, gamma=gamma)
    xo = spla.spsolve(D.scipy().tocsc(), D.rhs)
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
    info = F.pcg_solve(A.csr, A.rhs, x, 1e-12, 20000, ws)
    say(f"iters {info['iters']} true relres {info['true_relres']:.2e}")
    assert info["status"] == 0 and info["true_relres"] <= 1e-11
    assert rel(x.cpu().numpy(), xo) <= 1e-8
    # the same solve with the cell-block SpMV
    x2 = torch.zeros_like(x)
    info2 = A.solve(x2, 1e-12, 20000, ws)
    say(f"cell-block SpMV: iters {info2['iters']} true relres {info2['true_relres']:.2e}")
    assert info2["status"] == 0 and info2["true_relres"] <= 1e-11 and abs(info2["iters"] - info["iters"]) <= 2
    assert rel(x2.cpu().numpy(), xo) <= 1e-8


def _block_around(dim, n, c):
    lo = [max(c[r] - 1, 0) for r in range(dim)]
    hi = [min(c[r] + 1, n[r] - 1) for r in range(dim)]
    return lo, [hi[r] - lo[r] + 1 for r in range(dim)]


def test_dg_rows_of_sampled_cells_at_workload_size():
    """48^3 Q2, gamma 36, tau 1, sinusoidal source, zero data on the boundary:
    the system the benchmark's DG form solves."""
    dim, n, k = 3, [48, 48, 48], 2
    say(f"[dg workload] n={n} k={k}")
    v = structured_vertices(dim, n, jitter=0.2)
    gamma = penalty(k)
    mesh, coeff, A = gpu_dg(dim, n, k, v, gamma, 1.0, source_kind=2, source=(1.0,), dirichlet_kind=0, affine=None)
    nn = (k + 1) ** dim
    g = rng(93)
    cells = [(0, 0, 0), (47, 47, 47), (0, 47, 0), (47, 0, 47), (5, 0, 9), (0, 17, 30), (23, 47, 2), (24, 24, 24)]
    cells += [tuple(int(x) for x in g.integers(0, 48, size=3)) for _ in range(8)]
    rowptr = A.rowptr.cpu().numpy()
    assert rowptr[-1] == A.nnz
    xs = rng(96).standard_normal(A.n_rows)
    yd = torch.full((A.n_rows,), np.nan, dtype=torch.float64, device="cuda")
    A.spmv(torch.from_numpy(xs).cuda(), yd)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    assert np.isfinite(y).all()
    worst = 0.0
    worst_spmv = 0.0
    for c in cells:
        K = c[0] + 48 * (c[1] + 48 * c[2])
        lo, m = _block_around(dim, n, c)
        # vertices of the block: global vertex (i, j, l) for i in lo .. lo + m
        ids = [(lo[0] + i) + 49 * ((lo[1] + j) + 49 * (lo[2] + l))
               for l in range(m[2] + 1) for j in range(m[1] + 1) for i in range(m[0] + 1)]
        P = O.Problem(dim, m, k, source_kind=2, source=(1.0,))
        D = O.DGSystem(P, v[ids], gamma=gamma)
        kl = (c[0] - lo[0]) + m[0] * ((c[1] - lo[1]) + m[1] * (c[2] - lo[2]))

        def glob(sub_cell):
            s0, s1, s2 = sub_cell % m[0], (sub_cell // m[0]) % m[1], sub_cell // (m[0] * m[1])
            return (lo[0] + s0) + 48 * ((lo[1] + s1) + 48 * (lo[2] + s2))
        r0, r1 = rowptr[K * nn], rowptr[(K + 1) * nn]
        cols = A.colind[r0:r1].cpu().numpy().astype(np.int64)
        vals = A.values[r0:r1].cpu().numpy()
        so, se = D.rowptr[kl * nn], D.rowptr[(kl + 1) * nn]
        ocols = D.colind[so:se].astype(np.int64)
        exp_cols = np.array([glob(cc // nn) * nn + cc % nn for cc in ocols])
        np.testing.assert_array_equal(cols, exp_cols)
        e = rel(vals, D.values[so:se])
        er = rel(A.rhs[K * nn:(K + 1) * nn].cpu().numpy(), D.rhs[kl * nn:(kl + 1) * nn])
        worst = max(worst, e, er)
        # the cell-block SpMV on these rows: the oracle's row values times x
        ov = D.values[so:se].reshape(nn, -1)
        xc = xs[exp_cols.reshape(nn, -1)]
        yo = (ov * xc).sum(axis=1)
        scale = (np.abs(ov) * np.abs(xc)).sum(axis=1)
        worst_spmv = max(worst_spmv, float(np.max(np.abs(y[K * nn:(K + 1) * nn] - yo) / scale)))
    say(f"worst sampled-row rel err {worst:.2e}, cell-block SpMV {worst_spmv:.2e}")
    assert worst <= MATRIX_RTOL and worst_spmv <= 1e-12
