"""The tile-shape autotuner of the matrix-core element integration: every
candidate shape sums each entry over the quadrature points in the same order,
so the element matrices are bitwise the same whichever shape is tuned in; the
tuned shape is used by single and batched assembly alike."""
import numpy as np
import pytest
import torch

from paper_1708_01773_amd import fe as F
from tests.gpu_util import MATRIX_RTOL, Pair, element_matrices, rel, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k,prob,prec", [(3, "elasticity", "fp64"), (3, "poisson", "bf16"), (4, "elasticity", "fp16"),
                                         (4, "poisson", "fp32"), (2, "elasticity", "fp64")])
def test_tuned_shapes_leave_element_matrices_bitwise_unchanged(k, prob, prec):
    pair = Pair(3, [3, 2, 2], k, prob, precision=prec, seed=81, source=(0.5, 0.0, -1.0))
    F.spmv_tuning_reset()
    try:
        default = F.integrate_plan_of(pair.mesh, k, pair.coeff)
        A = pair.gpu_assembly()
        E0 = A.ws.clone()
        chosen, tried = F.integrate_autotune(pair.mesh, k, pair.coeff, A.ws, reps=2)
        say(f"[k3 tune] k={k} {prob} {prec}: default {default}, tried {tried}, chosen {chosen}")
        assert chosen["pairs_per_wave"] in [t["pairs_per_wave"] for t in tried]
        assert chosen["us"] == min(t["us"] for t in tried) and len(tried) >= 1
        # the workspace now holds the last candidate's element matrices
        torch.cuda.synchronize()
        assert torch.equal(A.ws, E0)
        assert F.integrate_plan_of(pair.mesh, k, pair.coeff)[0] == chosen["pairs_per_wave"]
        A.assemble()
        torch.cuda.synchronize()
        assert torch.equal(A.ws, E0)
        # and they are the oracle's
        cells = list(range(pair.P.ncells))
        Es, _ = element_matrices(pair, A, cells)
        if prec == "fp64":
            assert max(rel(E, pair.oracle_element(c)) for c, E in zip(cells, Es)) <= MATRIX_RTOL
    finally:
        F.spmv_tuning_reset()
    assert F.integrate_plan_of(pair.mesh, k, pair.coeff) == default


def test_integrate_autotune_refuses_spaces_without_tile_shapes():
    pair = Pair(3, [3, 3, 3], 1)
    A = pair.gpu_assembly()
    with pytest.raises(F.FeError):
        F.integrate_autotune(pair.mesh, 1, pair.coeff, A.ws)
    assert F.integrate_plan_of(pair.mesh, 1, pair.coeff) == (0, 0)
