"""GPU parity of the CSR SpMV (K7) and Jacobi-PCG (K8) against the oracle."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import oracle as O
from paper_1708_01773_amd import fe as F
from tests.gpu_util import Pair, rel, say

pytestmark = pytest.mark.gpu


def _gpu_csr_from_oracle(S):
    rowptr = torch.from_numpy(S.rowptr).cuda()
    colind = torch.from_numpy(S.colind.astype(np.int32)).cuda()
    values = torch.from_numpy(S.values).cuda()
    diag = S.scipy().diagonal()
    dinv = torch.from_numpy(1.0 / diag).cuda()
    rhs = torch.from_numpy(S.rhs).cuda()
    return F.csr_struct(S.nfree, S.nnz, rowptr, colind, values, rhs, dinv), (rowptr, colind, values, rhs, dinv)


@pytest.mark.parametrize("dim,n,k,prob", [(2, [32, 32], 1, "poisson"), (3, [7, 6, 5], 1, "poisson"),
                                          (3, [3, 3, 2], 3, "poisson"), (3, [3, 2, 2], 2, "elasticity")])
def test_spmv_matches_oracle(dim, n, k, prob):
    say(f"[spmv] dim={dim} n={n} k={k} {prob}")
    pair = Pair(dim, n, k, prob)
    A = pair.gpu_assembly()
    x = np.random.Generator(np.random.PCG64(3)).standard_normal(A.n_rows)
    xd = torch.from_numpy(x).cuda()
    y = torch.empty_like(xd)
    F.spmv(A.csr, xd, y)
    torch.cuda.synchronize()
    S = pair.system
    yo = O.spmv(S.rowptr, S.colind, S.values, x)
    # same matrix (bit-exact structure, values to 1e-12), different summation order
    scale = O.spmv(S.rowptr, S.colind, np.abs(S.values), np.abs(x))
    assert np.all(np.abs(y.cpu().numpy() - yo) <= 1e-12 * scale + 1e-300)


def test_c1_solution_matches_oracle():
    """The small 2D case: Poisson, 32x32 Q1, k = 1, sin-product load, u = 0 on the
    boundary, FP64 CSR + Jacobi-PCG to rtol 1e-10; then both solved to
    stagnation (rtol 1e-14) must agree to 1e-12."""
    say("[pcg] C1")
    pair = Pair(2, [32, 32], 1, lognormal=False, jitter=0.0, source_kind=2, source=(1.0,))
    A = pair.gpu_assembly()
    S = pair.system
    ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    info = F.pcg_solve(A.csr, A.rhs, x, 1e-10, 1000, ws)
    say(info)
    assert info["status"] == F.FE_OK and info["relres"] <= 1e-10
    orc = O.pcg(S.rowptr, S.colind, S.values, S.rhs, 1e-10, 1000)
    assert abs(info["iters"] - orc["iters"]) <= 2
    xd = spla.spsolve(S.scipy().tocsc(), S.rhs)
    kappa = info["lambda_max_est"] / info["lambda_min_est"]
    assert rel(x.cpu().numpy(), xd) <= 10 * kappa * 1e-10
    x.zero_()
    info = F.pcg_solve(A.csr, A.rhs, x, 1e-14, 5000, ws)
    orc = O.pcg(S.rowptr, S.colind, S.values, S.rhs, 1e-14, 5000)
    assert info["status"] == F.FE_OK and orc["status"] == 0
    assert rel(x.cpu().numpy(), orc["x"]) <= 1e-12
    # discretisation error of the manufactured solution
    err = O.l2_error(pair.P, pair.v, S.cell_dofs, x.cpu().numpy(), 4, 1, [1.0])
    assert err < 2e-3


@pytest.mark.parametrize("dim,n,k,prob", [(3, [6, 5, 4], 1, "poisson"), (3, [3, 3, 3], 2, "poisson"),
                                          (3, [3, 2, 2], 2, "elasticity"), (2, [4, 3], 4, "poisson")])
def test_pcg_solution_matches_direct_solve(dim, n, k, prob):
    say(f"[pcg] dim={dim} n={n} k={k} {prob}")
    pair = Pair(dim, n, k, prob, source=(1.0, 0.5, -1.0))
    A = pair.gpu_assembly()
    S = pair.system
    ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    info = F.pcg_solve(A.csr, A.rhs, x, 1e-14, 20000, ws)
    say(info)
    assert info["status"] == F.FE_OK
    xd = spla.spsolve(S.scipy().tocsc(), S.rhs)
    kappa = info["lambda_max_est"] / info["lambda_min_est"]
    assert rel(x.cpu().numpy(), xd) <= max(1e-11, 100 * kappa * 1e-14)
    # Lanczos estimates lie inside the spectrum of D^-1/2 A D^-1/2
    Ad = S.dense()
    d = 1.0 / np.sqrt(np.diag(Ad))
    ev = np.linalg.eigvalsh(Ad * d[:, None] * d[None, :])
    assert ev[0] * (1 - 1e-8) <= info["lambda_min_est"] <= info["lambda_max_est"] <= ev[-1] * (1 + 1e-8)
    # the true residual is reported
    assert info["true_relres"] <= 1e-12


def test_pcg_is_deterministic_and_reports_failures():
    pair = Pair(3, [5, 5, 5], 1)
    A = pair.gpu_assembly()
    ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
    x1 = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    x2 = torch.zeros_like(x1)
    i1 = F.pcg_solve(A.csr, A.rhs, x1, 1e-12, 1000, ws)
    i2 = F.pcg_solve(A.csr, A.rhs, x2, 1e-12, 1000, ws)
    assert torch.equal(x1, x2) and i1["iters"] == i2["iters"]
    x1.zero_()
    i3 = F.pcg_solve(A.csr, A.rhs, x1, 1e-12, 3, ws)
    assert i3["status"] == F.FE_ENOTCONV and i3["iters"] == 3
    # an indefinite diagonal matrix breaks CG down
    rowptr = torch.tensor([0, 1, 2], dtype=torch.int64, device="cuda")
    colind = torch.tensor([0, 1], dtype=torch.int32, device="cuda")
    vals = torch.tensor([1.0, -1.0], dtype=torch.float64, device="cuda")
    dinv = torch.tensor([1.0, 1.0], dtype=torch.float64, device="cuda")
    b = torch.tensor([1.0, 1.0], dtype=torch.float64, device="cuda")
    csr = F.csr_struct(2, 2, rowptr, colind, vals, None, dinv)
    xb = torch.zeros(2, dtype=torch.float64, device="cuda")
    ws2 = torch.empty(F.pcg_query(2), dtype=torch.uint8, device="cuda")
    i4 = F.pcg_solve(csr, b, xb, 1e-12, 10, ws2)
    assert i4["status"] == F.FE_EBREAKDOWN
    # initial guess = exact solution: converged at iteration 0
    i5 = F.pcg_solve(A.csr, A.rhs, x2, 1e-10, 10, ws)
    assert i5["status"] == F.FE_OK and i5["iters"] == 0


MESH_CASES = [(2, [32, 32], 1, "poisson", None), (3, [7, 6, 5], 1, "poisson", None), (3, [3, 3, 2], 3, "poisson", None),
              (3, [3, 2, 2], 2, "elasticity", None), (3, [2, 2, 2], 4, "poisson", 0b101101),
              (2, [3, 4], 3, "elasticity", 0b0110), (3, [4, 3, 3], 2, "poisson", 0), (3, [2, 1, 2], 4, "elasticity", 3),
              (2, [5, 4], 4, "poisson", None), (3, [3, 3, 3], 1, "elasticity", None)]


@pytest.mark.parametrize("dim,n,k,prob,faces", MESH_CASES)
def test_spmv_with_evaluated_pattern_matches_oracle(dim, n, k, prob, faces):
    say(f"[spmv mesh] dim={dim} n={n} k={k} {prob} faces={faces}")
    pair = Pair(dim, n, k, prob, faces=faces)
    A = pair.gpu_assembly()
    x = np.random.Generator(np.random.PCG64(4)).standard_normal(A.n_rows)
    xd = torch.from_numpy(x).cuda()
    y = torch.empty_like(xd)
    F.spmv_mesh(pair.mesh, pair.k, pair.coeff, A.csr, xd, y)
    torch.cuda.synchronize()
    S = pair.system
    yo = O.spmv(S.rowptr, S.colind, S.values, x)
    scale = O.spmv(S.rowptr, S.colind, np.abs(S.values), np.abs(x))
    assert np.all(np.abs(y.cpu().numpy() - yo) <= 1e-12 * scale + 1e-300)


@pytest.mark.parametrize("dim,n,k,prob", [(3, [6, 5, 4], 1, "poisson"), (3, [3, 3, 3], 2, "poisson"),
                                          (3, [3, 2, 2], 2, "elasticity"), (2, [4, 3], 4, "poisson")])
def test_pcg_with_evaluated_pattern_matches_direct_solve(dim, n, k, prob):
    say(f"[pcg mesh] dim={dim} n={n} k={k} {prob}")
    pair = Pair(dim, n, k, prob, source=(1.0, 0.5, -1.0))
    A = pair.gpu_assembly()
    S = pair.system
    ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    info = A.solve(x, 1e-14, 20000, ws)
    say(info)
    assert info["status"] == F.FE_OK and info["true_relres"] <= 1e-12
    xd = spla.spsolve(S.scipy().tocsc(), S.rhs)
    kappa = info["lambda_max_est"] / info["lambda_min_est"]
    assert rel(x.cpu().numpy(), xd) <= max(1e-11, 100 * kappa * 1e-14)
    # the same iteration as the CSR path up to rounding: iteration counts agree closely
    x2 = torch.zeros_like(x)
    info2 = F.pcg_solve(A.csr, A.rhs, x2, 1e-14, 20000, ws)
    assert abs(info2["iters"] - info["iters"]) <= max(2, info["iters"] // 50)
    # deterministic
    x3 = torch.zeros_like(x)
    info3 = A.solve(x3, 1e-14, 20000, ws)
    assert torch.equal(x, x3) and info3["iters"] == info["iters"]


def test_mesh_solve_rejects_a_foreign_system():
    a = Pair(3, [3, 3, 3], 1)
    b = Pair(3, [3, 3, 2], 1)
    A = a.gpu_assembly()
    ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FeError):
        F.pcg_solve_mesh(b.mesh, 1, b.coeff, A.csr, A.rhs, x, 1e-8, 100, ws)


# The Q1 scalar class: the LDS-staged traversal (mode 4) sums every row in
# the order of the two-lane traversal (mode 3), so its products must be
# bitwise the same; PCG solves group the fused dot-product partials by block
# (blocks differ between the two), so they agree to rounding.
@pytest.mark.parametrize("dim,n,faces", [(3, [7, 6, 5], None), (3, [9, 4, 6], 0b011010), (2, [33, 17], None),
                                         (2, [5, 40], 0b0110)])
def test_q1_staged_traversal_is_bitwise_the_two_lane_traversal(dim, n, faces):
    pair = Pair(dim, n, 1, faces=faces, seed=11)
    A = pair.gpu_assembly()
    say(f"[q1 staged] dim {dim} n {n} faces {faces} rows {A.n_rows}")
    x = torch.from_numpy(np.random.Generator(np.random.PCG64(12)).standard_normal(A.n_rows)).cuda()
    ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
    ys, sols, infos = [], [], []
    F.spmv_tuning_reset()
    try:
        for mode in (3, 4):
            F.spmv_plan_set_mesh(pair.mesh, 1, pair.coeff, mode, 3 ** dim)
            assert F.spmv_plan_of_mesh(pair.mesh, 1, pair.coeff)[:2] == (mode, 3 ** dim)
            y = torch.empty_like(x)
            F.spmv_mesh(pair.mesh, 1, pair.coeff, A.csr, x, y)
            u = torch.zeros_like(x)
            infos.append(A.solve(u, 1e-10, 5000, ws))
            torch.cuda.synchronize()
            ys.append(y)
            sols.append(u)
        with pytest.raises(F.FeError):
            F.spmv_plan_set_mesh(pair.mesh, 1, pair.coeff, 3, 25)
    finally:
        F.spmv_tuning_reset()
    assert torch.equal(ys[0], ys[1])
    assert all(i["status"] == F.FE_OK for i in infos) and abs(infos[0]["iters"] - infos[1]["iters"]) <= 1
    assert float(torch.linalg.vector_norm(sols[0] - sols[1]) / torch.linalg.vector_norm(sols[0])) <= 1e-9
    S = pair.system
    yo = O.spmv(S.rowptr, S.colind, S.values, x.cpu().numpy())
    scale = O.spmv(S.rowptr, S.colind, np.abs(S.values), np.abs(x.cpu().numpy()))
    assert np.all(np.abs(ys[1].cpu().numpy() - yo) <= 1e-12 * scale + 1e-300)


def test_q1_staged_traversal_with_wave_strided_steps():
    """Above 128 x 32768 rows the traversal's blocks take several steps each
    (the one-step form needs a partial slot per 128 rows): compared row by row
    with the CSR traversal of the same matrix."""
    n = 163  # 162^3 = 4.25M free nodes
    pair = Pair(3, [n, n, n], 1, seed=13)
    A = pair.gpu_assembly()
    assert A.n_rows > 128 * 32768
    say(f"[q1 strided] rows {A.n_rows} nnz {A.nnz}")
    assert F.spmv_plan_of_mesh(pair.mesh, 1, pair.coeff)[0] == 4
    g = torch.Generator(device="cuda").manual_seed(14)
    x = torch.rand(A.n_rows, dtype=torch.float64, device="cuda", generator=g) + 1.0
    y = torch.empty_like(x)
    yc = torch.empty_like(x)
    F.spmv_mesh(pair.mesh, 1, pair.coeff, A.csr, x, y)
    F.spmv(A.csr, x, yc)
    absv = A.values.abs()
    Cabs = F.csr_struct(A.n_rows, A.nnz, A.rowptr, A.colind, absv, A.rhs, A.dinv)
    scale = torch.empty_like(x)
    F.spmv(Cabs, x, scale)
    torch.cuda.synchronize()
    assert bool(torch.all((y - yc).abs() <= 1e-13 * scale))
    # and a PCG solve through it converges like the CSR solve
    ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
    u = torch.zeros_like(x)
    info = A.solve(u, 1e-8, 20000, ws)
    uc = torch.zeros_like(x)
    infoc = F.pcg_solve(A.csr, A.rhs, uc, 1e-8, 20000, ws)
    torch.cuda.synchronize()
    say(f"   iters mesh {info['iters']} csr {infoc['iters']}")
    assert info["status"] == F.FE_OK and infoc["status"] == F.FE_OK
    assert abs(info["iters"] - infoc["iters"]) <= 2
    assert float(torch.linalg.vector_norm(u - uc) / torch.linalg.vector_norm(uc)) <= 1e-6


# Orders 2..4 and vector patterns: the block-staged traversal (mode 6) sums
# every row in the order of the lanes-per-row traversal with eight rows per
# wave (mode 2), so the products must be bitwise the same; also through a PCG
# solve.
@pytest.mark.parametrize("dim,n,k,prob,faces", [(3, [5, 4, 3], 2, "poisson", None), (3, [3, 3, 2], 3, "elasticity", None),
                                                (3, [2, 3, 2], 4, "poisson", 0b011001), (3, [4, 3, 3], 2, "elasticity", 0),
                                                (2, [9, 7], 3, "poisson", None), (2, [6, 5], 2, "elasticity", 0b0110),
                                                (3, [7, 6, 5], 1, "elasticity", None)])
def test_block_staged_traversal_is_bitwise_the_lanes_per_row_traversal(dim, n, k, prob, faces):
    pair = Pair(dim, n, k, prob, faces=faces, seed=31)
    A = pair.gpu_assembly()
    say(f"[xblock] dim {dim} n {n} k {k} {prob} faces {faces} rows {A.n_rows}")
    x = torch.from_numpy(np.random.Generator(np.random.PCG64(32)).standard_normal(A.n_rows)).cuda()
    ys = []
    F.spmv_tuning_reset()
    try:
        for mode in (2, 6):
            F.spmv_plan_set_mesh(pair.mesh, k, pair.coeff, mode, 8)
            y = torch.empty_like(x)
            F.spmv_mesh(pair.mesh, k, pair.coeff, A.csr, x, y)
            torch.cuda.synchronize()
            ys.append(y)
        # a PCG solve through the block-staged traversal (faces = 0 leaves the system singular: no solve)
        if faces != 0:
            ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
            u = torch.zeros_like(x)
            info = A.solve(u, 1e-10, 20000, ws)
            assert info["status"] == F.FE_OK
    finally:
        F.spmv_tuning_reset()
    assert torch.equal(ys[0], ys[1])
    S = pair.system
    yo = O.spmv(S.rowptr, S.colind, S.values, x.cpu().numpy())
    scale = O.spmv(S.rowptr, S.colind, np.abs(S.values), np.abs(x.cpu().numpy()))
    assert np.all(np.abs(ys[1].cpu().numpy() - yo) <= 1e-12 * scale + 1e-300)
    if faces != 0:
        xd = spla.spsolve(S.scipy().tocsc(), S.rhs)
        assert rel(u.cpu().numpy(), xd) <= 1e-8


@pytest.mark.parametrize("dim,n,k,prob", [(3, [7, 6, 5], 1, "poisson"), (2, [17, 9], 1, "poisson"),
                                          (3, [3, 3, 2], 2, "elasticity"), (3, [4, 3, 3], 3, "poisson")])
def test_mesh_traversals_accept_values_off_16_byte_boundaries(dim, n, k, prob):
    """The LDS-staged Q1 traversal stages values with 16-byte loads; values 8
    bytes off a 16-byte boundary run the two-lane traversal (same order)."""
    pair = Pair(dim, n, k, prob, seed=41)
    A = pair.gpu_assembly()
    say(f"[unaligned] dim {dim} n {n} k {k} {prob} rows {A.n_rows}")
    buf = torch.empty(A.nnz + 1, dtype=torch.float64, device="cuda")
    buf[1:] = A.values[: A.nnz]
    vals = buf[1:]
    assert vals.data_ptr() % 16 == 8
    C = F.csr_struct(A.n_rows, A.nnz, A.rowptr, A.colind, vals, A.rhs, A.dinv)
    x = torch.from_numpy(np.random.Generator(np.random.PCG64(42)).standard_normal(A.n_rows)).cuda()
    y = torch.empty_like(x)
    F.spmv_mesh(pair.mesh, k, pair.coeff, C, x, y)
    ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
    u = torch.zeros_like(x)
    info = F.pcg_solve_mesh(pair.mesh, k, pair.coeff, C, A.rhs, u, 1e-10, 20000, ws)
    torch.cuda.synchronize()
    S = pair.system
    yo = O.spmv(S.rowptr, S.colind, S.values, x.cpu().numpy())
    scale = O.spmv(S.rowptr, S.colind, np.abs(S.values), np.abs(x.cpu().numpy()))
    assert np.all(np.abs(y.cpu().numpy() - yo) <= 1e-12 * scale + 1e-300)
    assert info["status"] == F.FE_OK
    assert rel(u.cpu().numpy(), spla.spsolve(S.scipy().tocsc(), S.rhs)) <= 1e-8
    # solution and Jacobi diagonal 8 bytes off 16-byte boundaries: the vector
    # kernels fall back to single accesses, same arithmetic, bitwise the same
    ua = torch.zeros_like(x)
    ia = F.pcg_solve_mesh(pair.mesh, k, pair.coeff, A.csr, A.rhs, ua, 1e-10, 20000, ws)
    xb = torch.zeros(A.n_rows + 1, dtype=torch.float64, device="cuda")
    db = torch.empty(A.n_rows + 1, dtype=torch.float64, device="cuda")
    db[1:] = A.dinv[: A.n_rows]
    um, dm = xb[1:], db[1:]
    assert um.data_ptr() % 16 == 8 and dm.data_ptr() % 16 == 8
    Cm = F.csr_struct(A.n_rows, A.nnz, A.rowptr, A.colind, A.values, A.rhs, dm)
    im = F.pcg_solve_mesh(pair.mesh, k, pair.coeff, Cm, A.rhs, um, 1e-10, 20000, ws)
    ic = F.pcg_solve(Cm, A.rhs, torch.zeros_like(x), 1e-10, 20000, ws)
    torch.cuda.synchronize()
    assert ia["status"] == im["status"] == ic["status"] == F.FE_OK and ia["iters"] == im["iters"]
    assert torch.equal(ua, um)
    # workspace 8 bytes off a 16-byte boundary (its p, q, r with it): same
    # arithmetic, bitwise the same; 4 bytes off: refused before any launch
    wb = torch.empty(ws.numel() + 16, dtype=torch.uint8, device="cuda")
    w8 = wb[8 : 8 + ws.numel()]
    assert w8.data_ptr() % 16 == 8
    uw = torch.zeros_like(x)
    iw = F.pcg_solve_mesh(pair.mesh, k, pair.coeff, A.csr, A.rhs, uw, 1e-10, 20000, w8)
    torch.cuda.synchronize()
    assert iw["status"] == F.FE_OK and iw["iters"] == ia["iters"] and torch.equal(ua, uw)
    with pytest.raises(F.FeError, match="8-byte"):
        F.pcg_solve_mesh(pair.mesh, k, pair.coeff, A.csr, A.rhs, uw, 1e-10, 20000, wb[4 : 4 + ws.numel()])
