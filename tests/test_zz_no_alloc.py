"""The allocation-free Jacobi-PCG (fe_pcg_solve_noalloc) against the
workspace solve (fe_pcg_solve): two calls in a row, the second on a smaller
system, so the second finds the first one's contents in the library's static
workspace.  Both run the same kernels in the same order with the same plan,
so solutions and infos must be bitwise the same; each is also checked against
a direct solve of the oracle's system."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

from paper_1708_01773_amd import fe as F
from tests.gpu_util import Pair, rel, say

pytestmark = pytest.mark.gpu


def _solve_both(pair):
    A = pair.gpu_assembly()
    ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
    xr = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    ir = F.pcg_solve(A.csr, A.rhs, xr, 1e-11, 20000, ws)
    xn = torch.zeros_like(xr)
    inn = F.pcg_solve_noalloc(A.csr, A.rhs, xn, 1e-11, 20000)
    torch.cuda.synchronize()
    say(f"   rows {A.n_rows} iters ws {ir['iters']} noalloc {inn['iters']}")
    return A, xr, ir, xn, inn


def test_noalloc_solve_matches_workspace_solve_on_two_calls():
    cases = [Pair(3, [14, 13, 12], 1, seed=71), Pair(3, [4, 3, 3], 2, "elasticity", seed=72,
                                                     source=(0.2, 0.0, -1.0))]
    for i, pair in enumerate(cases):
        say(f"[noalloc] call {i + 1}: n {pair.n} k {pair.k} {pair.prob}")
        A, xr, ir, xn, inn = _solve_both(pair)
        assert ir["status"] == inn["status"] == F.FE_OK
        assert inn == ir
        assert torch.equal(xn, xr)
        S = pair.system
        xd = spla.spsolve(S.scipy().tocsc(), S.rhs)
        kappa = inn["lambda_max_est"] / inn["lambda_min_est"]
        assert rel(xn.cpu().numpy(), xd) <= max(1e-9, 10 * kappa * 1e-11)


def test_noalloc_solve_refuses_oversized_systems():
    n = F.PCG_NOALLOC_MAX_ROWS + 1
    dummy = torch.zeros(8, dtype=torch.float64, device="cuda")
    rp = torch.zeros(8, dtype=torch.int64, device="cuda")
    ci = torch.zeros(8, dtype=torch.int32, device="cuda")
    csr = F.csr_struct(n, 8, rp, ci, dummy, dummy, dummy)
    with pytest.raises(F.FeError, match="2,700,000"):
        F.pcg_solve_noalloc(csr, dummy, dummy, 1e-8, 10)
