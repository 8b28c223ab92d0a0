"""Serving form: requests admitted by a device-memory budget and solved by
continuous batching.  Each result must be bitwise the same alone and in the
mix (the same kernels, plans and reduction order), the budget must hold, and
failures must stay with their request."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

from paper_1708_01773_amd import fe as F
from paper_1708_01773_amd.serve import request_inputs, run_stream, summarize
from tests.gpu_util import Pair, rel, say

pytestmark = pytest.mark.gpu

# (arrival, n, k, request index): a burst, so the requests overlap on the device
MIX = [(0.0, 6, 1, 0), (0.0, 4, 3, 1), (0.0, 9, 2, 2), (0.0, 3, 4, 3), (0.001, 12, 1, 4), (0.002, 5, 2, 5),
       (0.002, 2, 4, 6), (0.003, 7, 3, 7), (0.004, 1, 1, 8), (0.004, 10, 1, 9)]


def _alone(i, n, k, rtol, maxit):
    a = request_inputs(i, n, k)
    mesh = F.create_mesh(3, a["n"], a["vertices"], a["cell_coeff"])
    A = F.Assembly(mesh, k, a["coeff"])
    A.pattern()
    A.assemble()
    x = torch.zeros(max(A.n_rows, 1), dtype=torch.float64, device="cuda")
    if A.n_rows:
        ws = torch.empty(F.pcg_query(A.n_rows), dtype=torch.uint8, device="cuda")
        info = A.solve(x, rtol, maxit, ws)
    else:
        info = dict(iters=0, status=F.FE_OK)
    torch.cuda.synchronize()
    return x[: A.n_rows].clone(), info


def test_results_are_the_same_alone_and_in_the_mix():
    say(f"[serve] mix of {len(MIX)} requests")
    rtol, maxit = 1e-12, 20000
    srv = F.Server(2 << 30, max_active=64)
    sols = {}

    def keep(j, ticket, r):
        assert r["state"] == F.FE_REQ_DONE, r
        x = torch.empty(r["n_rows"], dtype=torch.float64, device="cuda")
        srv.solution(ticket, x)
        sols[j] = (x, r)

    results, makespan = run_stream(srv, MIX, rtol=rtol, maxit=maxit, on_done=keep)
    st = srv.stats()
    say(f"   {summarize(results, makespan)}")
    say(f"   stats {st}")
    assert st["peak_solving"] > 1, "the requests never overlapped"
    assert st["completed"] == len(MIX) and st["in_use"] == 0
    srv.close()
    # alone: the plain single-problem path, and the server with one slot
    solo = F.Server(2 << 30, max_active=1)
    for j, (_, n, k, i) in enumerate(MIX):
        x_mix, r = sols[j]
        x1, info = _alone(i, n, k, rtol, maxit)
        assert r["iters"] == info["iters"] and r["status"] == F.FE_OK
        assert torch.equal(x_mix, x1), f"request {j} differs from its plain solve"
        a = request_inputs(i, n, k)
        t = solo.submit(a["dim"], a["n"], k, a["coeff"], rtol, maxit, a["vertices"], a["cell_coeff"])
        r2 = solo.wait(t)
        x2 = torch.empty(r2["n_rows"], dtype=torch.float64, device="cuda")
        solo.solution(t, x2)
        solo.release(t)
        assert torch.equal(x_mix, x2), f"request {j} differs from the same request served alone"
    solo.close()
    # one request against a direct solve of the oracle's system
    _, n, k, i = MIX[2]
    a = request_inputs(i, n, k)
    import oracle as O
    P = O.Problem(3, [n] * 3, k, problem="poisson", source_kind=1, source=(1.0,))
    S = O.System(P, a["vertices"], a["cell_coeff"])
    xd = spla.spsolve(S.scipy().tocsc(), S.rhs)
    assert rel(sols[2][0].cpu().numpy(), xd) <= 1e-9


def test_admission_holds_the_budget():
    sizes = [(0.0, 16, 2, 20 + j) for j in range(6)]
    probe = F.Server(1 << 30, max_active=8)
    a = request_inputs(20, 16, 2)
    t = probe.submit(3, a["n"], 2, a["coeff"], 1e-8, 10000, a["vertices"], a["cell_coeff"])
    one = probe.wait(t)
    probe.release(t)
    probe.close()
    need = one["bytes"]
    # room for about two requests in the arena (the budget also holds a mesh reserve of budget / 8)
    budget = int(max(2.4 * need / 0.87, 64 << 20))
    say(f"[serve] request bytes {need}, budget {budget}")
    srv = F.Server(budget, max_active=8)
    results, _ = run_stream(srv, sizes, rtol=1e-8, maxit=10000)
    st = srv.stats()
    say(f"   stats {st}")
    assert all(r["state"] == F.FE_REQ_DONE and r["status"] == F.FE_OK for r in results)
    assert st["peak_in_use"] <= budget
    # six requests cannot all fit: the head of the queue had to wait for memory
    assert st["admission_waits"] > 0 and st["admitted"] == 6
    # a request that can never fit is refused at submission
    big = request_inputs(30, 40, 3)
    with pytest.raises(F.FeError) as e:
        srv.submit(3, big["n"], 3, big["coeff"], 1e-8, 100, big["vertices"], big["cell_coeff"])
    assert e.value.status == F.FE_ENOMEM
    assert srv.stats()["rejected"] == 1
    srv.close()


def test_failures_stay_with_their_request():
    srv = F.Server(1 << 30, max_active=8)
    good = request_inputs(40, 6, 2)
    tg = srv.submit(3, good["n"], 2, good["coeff"], 1e-10, 10000, good["vertices"], good["cell_coeff"])
    # elasticity with an invalid Poisson ratio fails at set-up
    bad_c = F.make_coeff("elasticity", "fp64", nu=0.7, source_kind=F.FE_SOURCE_CONST, source=(0, 0, -1), dim=3)
    tb = srv.submit(3, [2, 2, 2], 2, bad_c, 1e-8, 100)
    # an inverted cell fails at mesh creation
    v = np.array(good["vertices"]).copy()
    v[1 + 7 * (1 + 7 * 1)] = [0.9, 0.9, 0.9]
    ti = srv.submit(3, good["n"], 2, good["coeff"], 1e-8, 100, v, good["cell_coeff"])
    # an iteration cap ends a request with FE_ENOTCONV
    tc = srv.submit(3, good["n"], 2, good["coeff"], 1e-14, 3, good["vertices"], good["cell_coeff"])
    rg, rb, ri, rc = (srv.wait(t) for t in (tg, tb, ti, tc))
    say(f"[serve] good {rg['state']}/{rg['status']} bad {rb['state']}/{rb['status']} {rb['error']} "
        f"inverted {ri['state']}/{ri['status']} capped {rc['state']}/{rc['status']}")
    assert rg["state"] == F.FE_REQ_DONE and rg["status"] == F.FE_OK
    assert rb["state"] == F.FE_REQ_FAILED and rb["status"] == F.FE_EINVAL
    assert ri["state"] == F.FE_REQ_FAILED and ri["status"] == F.FE_EMESH
    assert rc["state"] == F.FE_REQ_DONE and rc["status"] == F.FE_ENOTCONV and rc["iters"] == 3
    x = torch.empty(rg["n_rows"], dtype=torch.float64, device="cuda")
    srv.solution(tg, x)
    x1, _ = _alone(40, 6, 2, 1e-10, 10000)
    assert torch.equal(x, x1)
    with pytest.raises(F.FeError):
        srv.solution(tb, x)
    for t in (tg, tb, ti, tc):
        srv.release(t)
    with pytest.raises(F.FeError):
        srv.release(tg)  # unknown ticket now
    assert srv.stats()["in_use"] == 0
    srv.close()


def test_stream_records_requests_refused_at_submission():
    """Every drawn request is submitted; one needing more than the whole budget
    is refused by the server's admission and recorded, the others are served."""
    srv = F.Server(1 << 30, max_active=8)
    stream = [(0.0, 6, 2, 50), (0.0, 80, 4, 51), (0.01, 5, 1, 52)]  # the second needs about 100 GB
    results, makespan = run_stream(srv, stream, rtol=1e-8, maxit=10000)
    say(f"[serve] refused: {results[1]}")
    assert results[1]["state"] == "rejected" and "budget" in results[1]["error"]
    assert results[0]["state"] == F.FE_REQ_DONE and results[2]["state"] == F.FE_REQ_DONE
    s = summarize(results, makespan)
    assert s["rejected_at_submission"] == 1 and s["served"] == 2 and s["converged"] == 2
    assert srv.stats()["rejected"] == 1
    srv.close()
