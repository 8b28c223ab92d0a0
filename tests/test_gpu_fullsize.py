"""Parity at the full benchmark size (3D Poisson, 128^3 jittered Q1 hexes,
lognormal coefficients), in the configuration the benchmark times: sampled
element matrices and CSR rows are recomputed one by one by the oracle;
size-independent properties are checked on the whole system."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle as O
from paper_1708_01773_amd import fe as F
from tests.gpu_util import MATRIX_RTOL, Pair, element_matrices, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2():
    say("[fullsize] 3D Poisson 128^3 Q1 jittered lognormal, f = 1")
    pair = Pair(3, [128, 128, 128], 1, source=(1.0,))
    A = pair.gpu_assembly()
    code, nf, nx = O.number_nodes(3, pair.n, 1, pair.P.faces)
    cdofs = O.cell_dofs(pair.P, code)
    return pair, A, cdofs


def test_sizes(c2):
    pair, A, _ = c2
    assert A.n_rows == 127 ** 3 == 2048383
    assert A.nnz == 379 ** 3 == 54439939


def test_sampled_element_matrices(c2):
    pair, A, _ = c2
    cells = np.random.Generator(np.random.PCG64(1)).integers(0, pair.P.ncells, 200)
    Es, _ = element_matrices(pair, A, cells)
    worst = max(rel(E, pair.oracle_element(int(c))) for c, E in zip(cells, Es))
    say(f"worst sampled element rel err {worst:.2e}")
    assert worst <= MATRIX_RTOL


def test_sampled_rows(c2):
    pair, A, cdofs = c2
    rows = np.random.Generator(np.random.PCG64(2)).integers(0, A.n_rows, 40)
    rowptr = A.rowptr.cpu().numpy()
    for r in rows:
        cols, vals, rhs = O.assemble_row(pair.P, pair.v, pair.coef, cdofs, int(r))
        lo, hi = rowptr[r], rowptr[r + 1]
        np.testing.assert_array_equal(A.colind[lo:hi].cpu().numpy(), cols)
        assert rel(A.values[lo:hi].cpu().numpy(), vals) <= MATRIX_RTOL
        assert abs(A.rhs[r].item() - rhs) <= MATRIX_RTOL * abs(rhs)
        d = np.searchsorted(cols, r)
        assert A.dinv[r].item() == 1.0 / A.values[lo + d].item()


def test_whole_matrix_properties(c2):
    pair, A, _ = c2
    n = A.n_rows
    M = sp.csr_matrix((A.values.cpu().numpy(), A.colind.cpu().numpy(), A.rowptr.cpu().numpy()), shape=(n, n))
    # symmetric to rounding, and every diagonal positive
    D = M - M.T
    assert abs(D).max() <= 1e-13 * abs(M).max()
    assert (M.diagonal() > 0).all()
    # sum of the load over free rows is below the volume (f = 1, boundary rows removed)
    s = A.rhs.sum().item()
    assert 0.9 < s < 1.0


def test_symmetric_storage_at_full_size(c2):
    """The benchmark's operator: the upper triangle in symmetric storage, its
    SpMV in the one-step launch form and the PCG to rtol 1e-10.  Sampled rows
    of the storage and of y = A x against the oracle's rows; the whole matrix
    is bitwise symmetric; the solve's residual recomputed with the CSR SpMV."""
    pair, A, cdofs = c2
    n = A.n_rows
    M = sp.csr_matrix((A.values.cpu().numpy(), A.colind.cpu().numpy(), A.rowptr.cpu().numpy()), shape=(n, n))
    assert (M != M.T).nnz == 0
    nb = F.sym_query(pair.mesh, 1, pair.coeff)
    ns = (n + 63) // 64 * 64
    assert nb == 14 * ns * 8
    sym = torch.empty(nb // 8, dtype=torch.float64, device="cuda")
    F.sym_from_csr(pair.mesh, 1, pair.coeff, A.csr, sym)
    g = torch.Generator(device="cuda").manual_seed(3)
    x = torch.rand(n, dtype=torch.float64, device="cuda", generator=g) - 0.5
    y = torch.empty_like(x)
    F.spmv_sym(pair.mesh, 1, pair.coeff, sym, x, y)
    torch.cuda.synchronize()
    S = sym.cpu().numpy().reshape(14, ns)
    xh, yh = x.cpu().numpy(), y.cpu().numpy()
    f0 = f1 = 127
    rows = np.random.Generator(np.random.PCG64(4)).integers(0, n, 40)
    for r in rows:
        cols, vals, _ = O.assemble_row(pair.P, pair.v, pair.coef, cdofs, int(r))
        want = float(np.dot(vals, xh[cols]))
        scale = float(np.dot(np.abs(vals), np.abs(xh[cols])))
        assert abs(yh[r] - want) <= 1e-12 * scale
        for c, v in zip(cols, vals):
            if c < r:
                continue
            d = c - r
            dz, rem = divmod(d + f0 * f1 + f0 + 1, f0 * f1)
            dy, dx = divmod(rem, f0)
            gcode = 9 * dz + 3 * dy + dx  # offsets shifted by +1 per axis
            assert abs(S[gcode - 13, r] - v) <= MATRIX_RTOL * max(abs(v), np.abs(vals).max())
    ws = torch.empty(F.pcg_query(n), dtype=torch.uint8, device="cuda")
    u = torch.zeros(n, dtype=torch.float64, device="cuda")
    info = F.pcg_solve_sym(pair.mesh, 1, pair.coeff, A.csr, sym, A.rhs, u, 1e-10, 100000, ws)
    res = torch.empty_like(u)
    F.spmv(A.csr, u, res)
    torch.cuda.synchronize()
    tr = float(torch.linalg.vector_norm(A.rhs[:n] - res) / torch.linalg.vector_norm(A.rhs[:n]))
    say(f"   sym pcg iters {info['iters']} relres {info['relres']:.2e} true (CSR SpMV) {tr:.2e}")
    assert info["status"] == F.FE_OK and info["relres"] <= 1e-10
    assert tr <= 2e-10 and abs(tr - info["true_relres"]) <= 1e-12
