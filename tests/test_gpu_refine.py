"""Mixed precision recovers FP64 accuracy by iterative refinement: the outer
residual uses the FP64 matrix, the inner Jacobi-PCG a lower-precision one
(FP32-stored values, or a matrix assembled with FP32 / FP16 / BF16 element
integration).  Compared with the plain FP64 solve on the same GPU at 1e-10
relative solution error."""
import numpy as np
import pytest
import torch

from paper_1708_01773_amd import fe as F
from tests.gpu_util import Pair, rel, say

pytestmark = pytest.mark.gpu


def _fp64_solution(A, rtol=1e-13):
    ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    info = F.pcg_solve(A.csr, A.rhs, x, rtol, 20000, ws)
    assert info["status"] == F.FE_OK
    return x, info


@pytest.mark.parametrize("k,prob,n,lo_prec,demote", [
    (1, "poisson", [12, 10, 8], "fp64", True),
    (1, "poisson", [12, 10, 8], "fp32", False),
    (2, "poisson", [5, 4, 4], "bf16", False),
    (2, "elasticity", [3, 3, 3], "fp16", True),
    (3, "poisson", [3, 3, 2], "fp32", True),
])
def test_refinement_recovers_fp64(k, prob, n, lo_prec, demote):
    say(f"[refine] k={k} {prob} n={n} A_lo integrated in {lo_prec}, FP32 storage={demote}")
    hi = Pair(3, n, k, prob, source=(1.0, 0.0, -1.0))
    A_hi = hi.gpu_assembly()
    lo = Pair(3, n, k, prob, source=(1.0, 0.0, -1.0), precision=lo_prec)
    A_lo = lo.gpu_assembly()
    v32 = None
    if demote:
        v32 = torch.empty(A_lo.nnz, dtype=torch.float32, device="cuda")
        F.csr_to_fp32(A_lo.csr, v32)
    ws = torch.empty(F.refine_query(A_hi.n_rows), dtype=torch.uint8, device="cuda")
    x = torch.zeros(A_hi.n_rows, dtype=torch.float64, device="cuda")
    info = F.refine_solve(A_hi.csr, A_lo.csr, A_hi.rhs, x, 1e-12, 1e-4, 50, 5000, ws, values32=v32)
    say(f"   {info}")
    assert info["status"] == F.FE_OK and info["relres"] <= 1e-12
    xr, _ = _fp64_solution(A_hi)
    e = rel(x.cpu().numpy(), xr.cpu().numpy())
    say(f"   |x_refined - x_fp64| / |x_fp64| = {e:.2e}")
    assert e <= 1e-10


def test_refinement_limits():
    pair = Pair(3, [6, 6, 6], 1)
    A = pair.gpu_assembly()
    ws = torch.empty(F.refine_query(A.n_rows), dtype=torch.uint8, device="cuda")
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    info = F.refine_solve(A.csr, A.csr, A.rhs, x, 1e-12, 1e-3, 0, 100, ws)
    assert info["status"] == F.FE_ENOTCONV and info["outer_iters"] == 0 and abs(info["relres"] - 1.0) < 1e-12
    # with the FP64 matrix itself as the inner operator one tight correction suffices
    info = F.refine_solve(A.csr, A.csr, A.rhs, x, 1e-10, 1e-12, 5, 2000, ws)
    assert info["status"] == F.FE_OK and info["outer_iters"] == 1


def test_refinement_on_fp32_symmetric_storage_with_wave_strided_steps():
    """Above 256 x 32768 rows the FP32 symmetric SpMV loops over steps (the
    looping form, mode 7): the refined solution against the refinement whose
    inner operator is the FP32 CSR of the same system."""
    n = 205  # 204^3 = 8.49M free nodes
    say("[refine sym32 strided] 205^3 Q1")
    hi = Pair(3, [n, n, n], 1, source=(1.0,), seed=13)  # a jitter draw that inverts no cell at 205^3
    A_hi = hi.gpu_assembly()
    lo = Pair(3, [n, n, n], 1, source=(1.0,), seed=13, precision="fp32")
    A_lo = lo.gpu_assembly()
    assert A_hi.n_rows > 256 * 32768
    nb = F.sym_query(lo.mesh, 1, lo.coeff)
    sym32 = torch.full((nb // 8,), float("nan"), dtype=torch.float32, device="cuda")
    F.sym_fp32_from_csr(lo.mesh, 1, lo.coeff, A_lo.csr, sym32)
    ws = torch.empty(F.refine_query(A_hi.n_rows), dtype=torch.uint8, device="cuda")
    x = torch.zeros(A_hi.n_rows, dtype=torch.float64, device="cuda")
    info = F.refine_solve_sym(hi.mesh, 1, hi.coeff, A_hi.csr, A_lo.csr, sym32, A_hi.rhs, x, 1e-10, 1e-4, 50, 20000,
                              ws)
    v32 = torch.empty(A_lo.nnz, dtype=torch.float32, device="cuda")
    F.csr_to_fp32(A_lo.csr, v32)
    xc = torch.zeros_like(x)
    infoc = F.refine_solve(A_hi.csr, A_lo.csr, A_hi.rhs, xc, 1e-10, 1e-4, 50, 20000, ws, values32=v32)
    torch.cuda.synchronize()
    say(f"   sym32 {info}  csr32 {infoc}")
    assert info["status"] == infoc["status"] == F.FE_OK and info["relres"] <= 1e-10
    assert abs(info["outer_iters"] - infoc["outer_iters"]) <= 1
    assert rel(x.cpu().numpy(), xc.cpu().numpy()) <= 1e-8


@pytest.mark.parametrize("dim,n,lo_prec,faces", [(3, [12, 10, 8], "fp32", None), (3, [9, 7, 11], "fp64", 0b011010),
                                                 (2, [40, 33], "fp32", None)])
def test_refinement_on_fp32_symmetric_storage(dim, n, lo_prec, faces):
    """The inner PCG on the FP32 symmetric storage of A_lo: the storage is the
    FP32 rounding of the FP64 one entry by entry, and the refined solution
    reaches FP64 accuracy like the CSR-stored FP32 inner solve."""
    say(f"[refine sym32] dim={dim} n={n} A_lo integrated in {lo_prec} faces={faces}")
    src = (1.0,)
    hi = Pair(dim, n, 1, source=src, faces=faces, seed=61)
    A_hi = hi.gpu_assembly()
    lo = Pair(dim, n, 1, source=src, faces=faces, seed=61, precision=lo_prec)
    A_lo = lo.gpu_assembly()
    nb = F.sym_query(lo.mesh, 1, lo.coeff)
    sym64 = torch.empty(nb // 8, dtype=torch.float64, device="cuda")
    sym32 = torch.full((nb // 8,), float("nan"), dtype=torch.float32, device="cuda")
    F.sym_from_csr(lo.mesh, 1, lo.coeff, A_lo.csr, sym64)
    F.sym_fp32_from_csr(lo.mesh, 1, lo.coeff, A_lo.csr, sym32)
    torch.cuda.synchronize()
    assert torch.equal(sym32, sym64.float())
    ws = torch.empty(F.refine_query(A_hi.n_rows), dtype=torch.uint8, device="cuda")
    x = torch.zeros(A_hi.n_rows, dtype=torch.float64, device="cuda")
    info = F.refine_solve_sym(hi.mesh, 1, hi.coeff, A_hi.csr, A_lo.csr, sym32, A_hi.rhs, x, 1e-12, 1e-4, 50, 5000, ws)
    x2 = torch.zeros_like(x)
    info2 = F.refine_solve_sym(hi.mesh, 1, hi.coeff, A_hi.csr, A_lo.csr, sym32, A_hi.rhs, x2, 1e-12, 1e-4, 50, 5000,
                               ws)
    v32 = torch.empty(A_lo.nnz, dtype=torch.float32, device="cuda")
    F.csr_to_fp32(A_lo.csr, v32)
    xc = torch.zeros_like(x)
    infoc = F.refine_solve(A_hi.csr, A_lo.csr, A_hi.rhs, xc, 1e-12, 1e-4, 50, 5000, ws, values32=v32)
    torch.cuda.synchronize()
    say(f"   sym32 {info}  csr32 {infoc}")
    assert info["status"] == infoc["status"] == F.FE_OK and info["relres"] <= 1e-12
    assert info2 == info and torch.equal(x, x2)
    assert abs(info["outer_iters"] - infoc["outer_iters"]) <= 1
    xr, _ = _fp64_solution(A_hi)
    assert rel(x.cpu().numpy(), xr.cpu().numpy()) <= 1e-10
    # a float buffer only 4-byte aligned is accepted; one too small is refused
    raw = torch.empty(nb // 8 + 1, dtype=torch.float32, device="cuda")
    F.sym_fp32_from_csr(lo.mesh, 1, lo.coeff, A_lo.csr, raw[1:])
    torch.cuda.synchronize()
    assert torch.equal(raw[1:], sym32)
    with pytest.raises(F.FeError, match="too small"):
        F.sym_fp32_from_csr(lo.mesh, 1, lo.coeff, A_lo.csr, raw[2:])


@pytest.mark.parametrize("k,prob,n,lo_prec,demote,faces", [
    (2, "elasticity", [4, 3, 3], "fp16", True, None),
    (3, "poisson", [3, 3, 2], "bf16", True, 0b101011),
    (4, "elasticity", [2, 2, 2], "fp32", True, None),
    (1, "poisson", [7, 6, 5], "fp32", True, None),
    (2, "elasticity", [3, 3, 3], "bf16", False, 0b000111),
    (1, "elasticity", [5, 4, 3], "fp64", True, None),
])
def test_refinement_with_the_evaluated_pattern_inner_solve(k, prob, n, lo_prec, demote, faces):
    """fe_refine_solve_mesh: the inner PCG evaluates the pattern (FP32 values
    through the block-staged traversal, or A_lo's FP64 values through the mesh
    plan); the refined solution must reach the FP64 solution as the CSR
    refinement does."""
    say(f"[refine mesh] k={k} {prob} n={n} faces={faces} A_lo {lo_prec}, FP32 storage={demote}")
    hi = Pair(3, n, k, prob, faces=faces, source=(1.0, 0.0, -1.0))
    A_hi = hi.gpu_assembly()
    lo = Pair(3, n, k, prob, faces=faces, source=(1.0, 0.0, -1.0), precision=lo_prec)
    A_lo = lo.gpu_assembly()
    v32 = None
    if demote:
        v32 = torch.empty(A_lo.nnz, dtype=torch.float32, device="cuda")
        F.csr_to_fp32(A_lo.csr, v32)
    ws = torch.empty(F.refine_query(A_hi.n_rows), dtype=torch.uint8, device="cuda")
    x = torch.zeros(A_hi.n_rows, dtype=torch.float64, device="cuda")
    info = F.refine_solve_mesh(hi.mesh, k, hi.coeff, A_hi.csr, A_lo.csr, A_hi.rhs, x, 1e-12, 1e-4, 50, 20000, ws,
                               values32=v32)
    xc = torch.zeros_like(x)
    infoc = F.refine_solve(A_hi.csr, A_lo.csr, A_hi.rhs, xc, 1e-12, 1e-4, 50, 20000, ws, values32=v32)
    say(f"   mesh {info}  csr {infoc}")
    assert info["status"] == F.FE_OK and info["relres"] <= 1e-12
    xr, _ = _fp64_solution(A_hi)
    e = rel(x.cpu().numpy(), xr.cpu().numpy())
    say(f"   |x_refined - x_fp64| / |x_fp64| = {e:.2e}")
    assert e <= 1e-10 and rel(x.cpu().numpy(), xc.cpu().numpy()) <= 1e-10
    # the same inner operator: the outer iteration counts agree closely
    assert abs(info["outer_iters"] - infoc["outer_iters"]) <= 1
    # a mesh that did not assemble A is refused
    other = Pair(3, [n[0] + 1] + n[1:], k, prob, faces=faces)
    with pytest.raises(F.FeError):
        F.refine_solve_mesh(other.mesh, k, other.coeff, A_hi.csr, A_lo.csr, A_hi.rhs, x, 1e-12, 1e-4, 5, 100, ws,
                            values32=v32)
