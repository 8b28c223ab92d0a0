"""GPU parity of set-up, element integration (K3) and scatter (K5) against
the oracle, through the C ABI.  FP64 matrices and vectors must agree to 1e-12
relative (Frobenius); integer outputs (cell-to-DOF map, CSR structure,
cell-to-nnz permutation) bit-exactly."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1708_01773_amd import fe as F
from tests.gpu_util import MATRIX_RTOL, Pair, element_matrices, rel, say

pytestmark = pytest.mark.gpu

AFF3 = [0.3, 1.0, -0.5, 0.25, -0.2, 0.1, 0.4, -0.3, 0.05, 0.2, -0.1, 0.6]

CASES = [
    # id, dim, n, k, problem, extra kwargs
    ("c1_2d_q1_32", 2, [32, 32], 1, "poisson", dict(lognormal=False, jitter=0.0, source_kind=2, source=(1.0,))),
    ("2d_q2_ragged", 2, [5, 3], 2, "poisson", {}),
    ("2d_q3", 2, [3, 4], 3, "poisson", dict(faces=0b0110)),
    ("2d_q4", 2, [2, 3], 4, "poisson", {}),
    ("3d_q1_ragged", 3, [6, 5, 4], 1, "poisson", {}),
    ("3d_q1_nodirichlet", 3, [4, 3, 5], 1, "poisson", dict(faces=0)),
    ("3d_q1_affine", 3, [4, 4, 3], 1, "poisson", dict(dirichlet_kind=1, affine=AFF3)),
    ("3d_q2", 3, [3, 4, 2], 2, "poisson", dict(faces=0b101101)),
    ("3d_q3", 3, [2, 3, 2], 3, "poisson", {}),
    ("3d_q4", 3, [2, 2, 2], 4, "poisson", dict(dirichlet_kind=1, affine=AFF3)),
    ("3d_el_q1", 3, [3, 3, 2], 1, "elasticity", dict(source=(0.0, 0.0, -1.0))),
    ("3d_el_q2", 3, [2, 2, 2], 2, "elasticity", dict(faces=0b000011, dirichlet_kind=1, affine=AFF3)),
    ("3d_el_q3", 3, [2, 2, 1], 3, "elasticity", {}),
    ("3d_el_q4", 3, [1, 1, 2], 4, "elasticity", dict(faces=0b010000)),
    ("2d_el_q2", 2, [3, 2], 2, "elasticity", dict(source=(1.0, -1.0))),
]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def built(request):
    name, dim, n, k, prob, kw = request.param
    say(f"[case {name}] dim={dim} n={n} k={k} {prob} {kw}")
    pair = Pair(dim, n, k, prob, **kw)
    A = pair.gpu_assembly()
    return pair, A


def test_cell_dofs_bit_exact(built):
    pair, A = built
    out = torch.empty(pair.P.ncells * pair.P.nloc, dtype=torch.int32, device="cuda")
    F.cell_dofs(pair.mesh, pair.k, pair.coeff, out)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy().reshape(pair.P.ncells, -1), pair.system.cell_dofs)


def test_pattern_bit_exact(built):
    pair, A = built
    S = pair.system
    assert A.n_rows == S.nfree and A.nnz == S.nnz
    np.testing.assert_array_equal(A.rowptr.cpu().numpy(), S.rowptr)
    np.testing.assert_array_equal(A.colind[: A.nnz].cpu().numpy(), S.colind)


def test_element_matrices_match_oracle(built):
    pair, A = built
    cells = list(range(pair.P.ncells))
    Es, Fl = element_matrices(pair, A, cells)
    worst = 0.0
    for c, E in zip(cells, Es):
        Eo = pair.oracle_element(c)
        worst = max(worst, rel(E, Eo))
    say(f"worst element-matrix rel err {worst:.2e}")
    assert worst <= MATRIX_RTOL


def test_values_rhs_dinv_match_oracle(built):
    pair, A = built
    S = pair.system
    vals = A.values[: A.nnz].cpu().numpy()
    rhs = A.rhs[: A.n_rows].cpu().numpy()
    ev, er = rel(vals, S.values), rel(rhs, S.rhs)
    say(f"values rel {ev:.2e} rhs rel {er:.2e}")
    assert ev <= MATRIX_RTOL and er <= MATRIX_RTOL
    if A.n_rows:
        diag = S.scipy().diagonal()
        np.testing.assert_array_equal(A.dinv[: A.n_rows].cpu().numpy(), 1.0 / vals[
            [int(S.rowptr[i] + np.searchsorted(S.colind[S.rowptr[i]:S.rowptr[i + 1]], i)) for i in range(A.n_rows)]])
        assert rel(1.0 / A.dinv[: A.n_rows].cpu().numpy(), diag) <= MATRIX_RTOL


def test_permutation_bit_exact(built):
    pair, A = built
    S = pair.system
    nl = pair.P.nloc
    perm = torch.empty(pair.P.ncells * nl * nl, dtype=torch.int64, device="cuda")
    F.permutation(pair.mesh, pair.k, pair.coeff, perm)
    torch.cuda.synchronize()
    perm = perm.cpu().numpy().reshape(pair.P.ncells, nl, nl)
    g = S.cell_dofs
    for c in range(pair.P.ncells):
        ga = g[c][:, None].repeat(nl, 1)
        gb = g[c][None, :].repeat(nl, 0)
        free = (ga >= 0) & (gb >= 0)
        expect = np.full((nl, nl), -1, dtype=np.int64)
        for a, b in zip(*np.nonzero(free)):
            r = ga[a, b]
            row = S.colind[S.rowptr[r]:S.rowptr[r + 1]]
            expect[a, b] = S.rowptr[r] + np.searchsorted(row, gb[a, b])
        np.testing.assert_array_equal(perm[c], expect)


def test_assembly_is_bitwise_reproducible(built):
    pair, A = built
    v1 = A.values.clone()
    r1 = A.rhs.clone()
    A.assemble()
    torch.cuda.synchronize()
    assert torch.equal(v1, A.values) and torch.equal(r1, A.rhs)


def test_empty_system():
    # one Q1 cell with all faces Dirichlet: no free DOF
    pair = Pair(3, [1, 1, 1], 1, jitter=0.0)
    A = pair.gpu_assembly()
    assert A.n_rows == 0 and A.nnz == 0
    assert A.rowptr.cpu().numpy().tolist() == [0]
    # one Q2 cell: exactly the centre node is free
    pair = Pair(3, [1, 1, 1], 2, jitter=0.0)
    A = pair.gpu_assembly()
    assert A.n_rows == 1 and A.nnz == 1
    assert abs(A.values[0].item() - pair.system.values[0]) <= 1e-14 * abs(pair.system.values[0])


def test_quadrature_point_status_is_clear():
    pair = Pair(3, [3, 3, 3], 2)
    pair.gpu_assembly()
    assert F.get_status(pair.mesh) == F.FE_OK
