"""Batched Jacobi-PCG: many independent systems of different sizes and orders
solved by one engine pass (one launch per kernel type covering every system,
iterations replayed from a captured HIP graph).  Each system's result must be
bitwise that of the single-system solve, which is itself checked against the
oracle in the solve tests; here the batch is also checked against a direct
solve of the oracle's systems."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

from paper_1708_01773_amd import fe as F
from tests.gpu_util import Pair, rel, say

pytestmark = pytest.mark.gpu

# (dim, n, k, problem): uneven sizes, every SpMV plan class, one empty system
SYSTEMS = [(3, [6, 5, 4], 1, "poisson"), (3, [3, 3, 3], 2, "poisson"), (3, [2, 2, 3], 3, "poisson"),
           (2, [9, 7], 1, "poisson"), (3, [3, 2, 2], 2, "elasticity"), (3, [1, 1, 1], 1, "poisson"),
           (3, [12, 11, 10], 1, "poisson"), (3, [2, 2, 2], 4, "poisson")]


def _build(seed0=0):
    out = []
    for i, (dim, n, k, prob) in enumerate(SYSTEMS):
        pair = Pair(dim, n, k, prob, seed=seed0 + i, source=(1.0, 0.5, -1.0))
        out.append((pair, pair.gpu_assembly()))
    return out


def test_batch_matches_single_solves_bitwise():
    say(f"[batch pcg] {len(SYSTEMS)} systems")
    built = _build()
    assert built[5][1].n_rows == 0  # one cell, every face fixed: no unknowns
    singles = []
    for pair, A in built:
        x = torch.zeros(max(A.n_rows, 1), dtype=torch.float64, device="cuda")
        if A.n_rows:
            ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
            info = F.pcg_solve(A.csr, A.rhs, x, 1e-12, 5000, ws)
            assert info["status"] == F.FE_OK
        else:
            info = dict(iters=0, status=F.FE_OK)
        singles.append((x, info))
    xs = [torch.zeros(max(A.n_rows, 1), dtype=torch.float64, device="cuda") for _, A in built]
    ws = torch.empty(F.pcg_batch_query([A.n_rows for _, A in built]), dtype=torch.uint8, device="cuda")
    st, infos = F.pcg_solve_batch([A.csr for _, A in built], [A.rhs for _, A in built], xs, 1e-12, 5000, ws)
    assert st == F.FE_OK
    for i, ((pair, A), (xs1, i1), xb, ib) in enumerate(zip(built, singles, xs, infos)):
        say(f"   system {i}: n_rows {A.n_rows} iters single {i1['iters']} batch {ib['iters']}")
        assert ib["status"] == F.FE_OK and ib["iters"] == i1["iters"]
        assert torch.equal(xb, xs1), f"system {i} differs from its single solve"
    # against a direct solve of the oracle's systems
    for (pair, A), xb in zip(built, xs):
        if A.n_rows == 0 or A.n_rows > 4000:
            continue
        S = pair.system
        xd = spla.spsolve(S.scipy().tocsc(), S.rhs)
        assert rel(xb.cpu().numpy(), xd) <= 1e-9


def test_batch_is_deterministic_and_stops_per_system():
    built = _build(seed0=50)
    live = [(p, A) for p, A in built if A.n_rows]
    ws = torch.empty(F.pcg_batch_query([A.n_rows for _, A in live]), dtype=torch.uint8, device="cuda")
    runs = []
    for _ in range(2):
        xs = [torch.zeros(A.n_rows, dtype=torch.float64, device="cuda") for _, A in live]
        st, infos = F.pcg_solve_batch([A.csr for _, A in live], [A.rhs for _, A in live], xs, 1e-12, 5000, ws)
        assert st == F.FE_OK
        runs.append((xs, infos))
    for a, b in zip(runs[0][0], runs[1][0]):
        assert torch.equal(a, b)
    # an iteration cap below some systems' needs: those report FE_ENOTCONV at
    # exactly the cap, the others converge as before
    iters = [i["iters"] for i in runs[0][1]]
    cap = sorted(iters)[len(iters) // 2]
    xs = [torch.zeros(A.n_rows, dtype=torch.float64, device="cuda") for _, A in live]
    st, infos = F.pcg_solve_batch([A.csr for _, A in live], [A.rhs for _, A in live], xs, 1e-12, cap, ws)
    assert st == F.FE_ENOTCONV
    for full, capped, x_full, x_cap in zip(iters, infos, runs[0][0], xs):
        if full <= cap:
            assert capped["status"] == F.FE_OK and capped["iters"] == full
            assert torch.equal(x_full, x_cap)
        else:
            assert capped["status"] == F.FE_ENOTCONV and capped["iters"] == cap
    # empty batch
    st, infos = F.pcg_solve_batch([], [], [], 1e-12, 10, ws)
    assert st == F.FE_OK and infos == []


# (dim, n, k, problem, precision, dirichlet): every kernel class, the per-problem
# fallbacks (2D order >= 2, Q1 elasticity), an affine lifting and an empty system
ASM = [(3, [5, 4, 3], 1, "poisson", "fp64", 0), (3, [6, 3, 2], 1, "poisson", "fp32", 0),
       (3, [3, 2, 2], 2, "poisson", "fp32", 0), (3, [2, 3, 2], 3, "poisson", "fp64", 0),
       (3, [2, 2, 1], 4, "poisson", "fp16", 0), (3, [2, 2, 2], 2, "elasticity", "bf16", 0),
       (2, [5, 4], 1, "poisson", "fp64", 0), (2, [3, 2], 3, "poisson", "fp64", 0),
       (3, [2, 2, 2], 1, "elasticity", "fp64", 0), (3, [3, 3, 2], 2, "poisson", "fp64", 1),
       (3, [1, 1, 1], 1, "poisson", "fp64", 0), (3, [4, 4, 4], 1, "poisson", "fp32", 0)]


def _asm_pairs():
    pairs = []
    for i, (dim, n, k, prob, prec, dk) in enumerate(ASM):
        aff = None
        if dk:
            aff = [0.3, -0.2, 0.1, 0.5, 1.0, -0.5, 0.25, 0.0, 0.75, -1.0, 0.5, 0.2][: (1 if prob == "poisson" else dim) * (dim + 1)]
        pairs.append(Pair(dim, n, k, prob, precision=prec, seed=100 + i, dirichlet_kind=dk, affine=aff))
    return pairs


def test_batch_assembly_matches_single_bitwise():
    say(f"[batch assembly] {len(ASM)} problems")
    pairs = _asm_pairs()
    B = F.BatchAssembly([p.mesh for p in pairs], [p.k for p in pairs], [p.coeff for p in pairs])
    for rep in range(2):  # re-assembly reuses the pattern and the workspace
        B.assemble()
        torch.cuda.synchronize()
        for i, p in enumerate(pairs):
            A = p.gpu_assembly()
            assert (A.n_rows, A.nnz) == (B.n_rows[i], B.nnz[i])
            if A.n_rows == 0:
                continue
            assert torch.equal(A.rowptr, B.rowptr[i]) and torch.equal(A.colind[: A.nnz], B.colind[i][: A.nnz])
            assert torch.equal(A.values[: A.nnz], B.values[i][: A.nnz]), f"values of problem {i}"
            assert torch.equal(A.rhs[: A.n_rows], B.rhs[i][: A.n_rows]), f"rhs of problem {i}"
            assert torch.equal(A.dinv[: A.n_rows], B.dinv[i][: A.n_rows]), f"dinv of problem {i}"
    # FP64 problems against the oracle (structure bit-exact, values 1e-12)
    for i, p in enumerate(pairs):
        if ASM[i][4] != "fp64" or B.n_rows[i] == 0:
            continue
        S = p.system
        np.testing.assert_array_equal(B.rowptr[i].cpu().numpy(), S.rowptr)
        np.testing.assert_array_equal(B.colind[i][: S.nnz].cpu().numpy(), S.colind)
        assert rel(B.values[i][: S.nnz].cpu().numpy(), S.values) <= 1e-12
        assert rel(B.rhs[i][: S.nfree].cpu().numpy(), S.rhs) <= 1e-12
    # batched solve of the assembled batch
    st, infos = B.solve(1e-10, 5000)
    assert st == F.FE_OK and all(i["status"] == F.FE_OK for i in infos)


def test_batch_assembly_rejects_bad_batches():
    a = Pair(3, [2, 2, 2], 1)
    b = Pair(3, [2, 2, 2], 2)
    # one mesh twice with different orders
    with pytest.raises(F.FeError):
        F.assemble_batch_query([a.mesh, a.mesh], [1, 2], [a.coeff, a.coeff])
    # the same mesh twice with the same space is fine
    nr, nz, ws = F.assemble_batch_query([a.mesh, a.mesh], [1, 1], [a.coeff, a.coeff])
    assert nr[0] == nr[1] and nz[0] == nz[1] and ws > 0
    # workspace too small
    B = F.BatchAssembly([a.mesh, b.mesh], [1, 2], [a.coeff, b.coeff])
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(F.FeError):
        F.assemble_batch([a.mesh, b.mesh], [1, 2], [a.coeff, b.coeff], B.csrs, small)
    # empty batch
    nr, nz, _ = F.assemble_batch_query([], [], [])
    assert nr == [] and nz == []
    F.assemble_batch([], [], [], [], small)


def test_spmv_autotuner_picks_a_measured_plan_and_keeps_results():
    import oracle as O
    pair = Pair(3, [10, 9, 8], 2)
    A = pair.gpu_assembly()
    S = pair.system
    x = np.random.Generator(np.random.PCG64(5)).standard_normal(A.n_rows)
    xd = torch.from_numpy(x).cuda()
    yo = O.spmv(S.rowptr, S.colind, S.values, x)
    scale = O.spmv(S.rowptr, S.colind, np.abs(S.values), np.abs(x))
    F.spmv_tuning_reset()
    try:
        untuned = F.spmv_plan_of(A.n_rows, A.nnz)
        chosen, tried = F.spmv_autotune(A.csr, reps=5)
        say(f"[autotune] untuned {untuned} chosen {chosen}")
        assert len(tried) == 14 and all(t["us"] > 0 for t in tried)
        assert chosen["us"] == min(t["us"] for t in tried)
        mode, rpw, _ = F.spmv_plan_of(A.n_rows, A.nnz)
        assert (mode, rpw) == (chosen["mode"], chosen["rows_per_wave"])
        # every candidate plan computes the same product up to rounding
        y = torch.empty_like(xd)
        F.spmv(A.csr, xd, y)
        torch.cuda.synchronize()
        assert np.all(np.abs(y.cpu().numpy() - yo) <= 1e-12 * scale + 1e-300)
    finally:
        F.spmv_tuning_reset()
    assert F.spmv_plan_of(A.n_rows, A.nnz) == untuned


def test_batch_with_evaluated_pattern_matches_single_bitwise():
    built = _build(seed0=70)
    live = [(p, A) for p, A in built if A.n_rows]
    singles = []
    for pair, A in live:
        x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda")
        ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
        info = A.solve(x, 1e-12, 5000, ws)
        assert info["status"] == F.FE_OK
        singles.append((x, info))
    xs = [torch.zeros(A.n_rows, dtype=torch.float64, device="cuda") for _, A in live]
    ws = torch.empty(F.pcg_batch_query([A.n_rows for _, A in live]), dtype=torch.uint8, device="cuda")
    st, infos = F.pcg_solve_batch_mesh([p.mesh for p, _ in live], [p.k for p, _ in live], [p.coeff for p, _ in live],
                                       [A.csr for _, A in live], [A.rhs for _, A in live], xs, 1e-12, 5000, ws)
    assert st == F.FE_OK
    for (x1, i1), xb, ib in zip(singles, xs, infos):
        assert ib["iters"] == i1["iters"] and torch.equal(xb, x1)


def test_mesh_spmv_autotuner_picks_a_measured_plan_and_keeps_results():
    import oracle as O
    pair = Pair(3, [6, 5, 4], 2)
    A = pair.gpu_assembly()
    S = pair.system
    x = np.random.Generator(np.random.PCG64(6)).standard_normal(A.n_rows)
    xd = torch.from_numpy(x).cuda()
    yo = O.spmv(S.rowptr, S.colind, S.values, x)
    scale = O.spmv(S.rowptr, S.colind, np.abs(S.values), np.abs(x))
    F.spmv_tuning_reset()
    try:
        untuned = F.spmv_plan_of_mesh(pair.mesh, pair.k, pair.coeff)
        chosen, tried = F.spmv_autotune_mesh(pair.mesh, pair.k, pair.coeff, A.csr, reps=5)
        say(f"[autotune mesh] untuned {untuned} chosen {chosen}")
        assert len(tried) == 6 and chosen["us"] == min(t["us"] for t in tried)
        assert F.spmv_plan_of_mesh(pair.mesh, pair.k, pair.coeff)[:2] == (chosen["mode"], chosen["rows_per_wave"])
        y = torch.empty_like(xd)
        F.spmv_mesh(pair.mesh, pair.k, pair.coeff, A.csr, xd, y)
        torch.cuda.synchronize()
        assert np.all(np.abs(y.cpu().numpy() - yo) <= 1e-12 * scale + 1e-300)
        # the 3D Q1 class (27 entries) adds the two-lane and the LDS-staged traversals
        q1 = Pair(3, [5, 4, 4], 1)
        A1 = q1.gpu_assembly()
        ch1, tried1 = F.spmv_autotune_mesh(q1.mesh, 1, q1.coeff, A1.csr, reps=5)
        assert len(tried1) == 7 and {3, 4} <= {t["mode"] for t in tried1}
        y1 = torch.empty(A1.n_rows, dtype=torch.float64, device="cuda")
        x1 = torch.ones(A1.n_rows, dtype=torch.float64, device="cuda")
        F.spmv_mesh(q1.mesh, 1, q1.coeff, A1.csr, x1, y1)
        S1 = q1.system
        y1o = O.spmv(S1.rowptr, S1.colind, S1.values, np.ones(A1.n_rows))
        sc1 = O.spmv(S1.rowptr, S1.colind, np.abs(S1.values), np.ones(A1.n_rows))
        assert np.all(np.abs(y1.cpu().numpy() - y1o) <= 1e-12 * sc1 + 1e-300)
    finally:
        F.spmv_tuning_reset()
    assert F.spmv_plan_of_mesh(pair.mesh, pair.k, pair.coeff) == untuned


def test_batched_refinement_is_bitwise_the_single_refinement_and_reaches_fp64():
    """Batching with reduced-precision integration: every problem of the batch
    refined against its FP64 system gives bitwise the one-by-one refinement
    (fe_refine_solve_mesh) and lies within 1e-10 of the plain FP64 solve."""
    from paper_1708_01773_amd import batch as BT
    specs = [(5, 1), (3, 3), (4, 2), (6, 1), (2, 2), (3, 1), (4, 3)]
    for prec in ("fp32", "fp16"):
        run = BT.BatchRun(specs, precision=prec, budget=1 << 30, first_index=40)
        assert run.refine
        xb, xs, x64 = {}, {}, {}
        res = run.run(1e-12, 20000, keep=lambda i, x: xb.__setitem__(i, x.clone()))
        seq = BT.run_sequential(run.problems, 1e-12, 20000, keep=lambda i, x: xs.__setitem__(i, x.clone()),
                                coeffs_hi=run.coeffs_hi)
        plain = BT.run_sequential([(m, k, run.coeffs_hi[i]) for i, (m, k, _) in enumerate(run.problems)], 1e-12,
                                  20000, keep=lambda i, x: x64.__setitem__(i, x.clone()))
        say(f"[batch refine {prec}] " + ", ".join(f"{i['outer_iters']}/{i['inner_iters']}" for i in res["infos"]))
        assert res["status"] == F.FE_OK
        for i in range(len(specs)):
            bi, si = res["infos"][i], seq["infos"][i]
            assert bi == si, (i, bi, si)
            assert torch.equal(xb[i], xs[i]), i
            if x64[i].numel():
                assert rel(xb[i].cpu().numpy(), x64[i].cpu().numpy()) <= 1e-10, i
    # a correction limit stops the problems that need more
    run = BT.BatchRun(specs, precision="fp16", budget=1 << 30, first_index=40)
    res = run.run(1e-12, 20000, max_outer=1)
    assert res["status"] == F.FE_ENOTCONV
    assert all(i["outer_iters"] <= 1 for i in res["infos"])
