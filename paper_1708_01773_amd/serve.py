"""Serving form: a client that replays a seeded Poisson-process request stream
against the library's server (fe_server_*), and the latency statistics.

Each request is a 3D Poisson assemble-and-solve on an n^3 brick (interior
vertices jittered by +-0.2 h, lognormal per-cell coefficients, f = 1, u = 0 on
the boundary) of order k; request i draws its mesh from its own seeds.
"""
import sys
import threading
import time

from fe_inputs import lognormal_coefficients, problem_seeds, structured_vertices

from . import fe as F


def request_inputs(i, n, k):
    """Host arrays and coefficients of request i."""
    sj, sc = problem_seeds(i)
    v = structured_vertices(3, n, jitter=0.2, seed=sj)
    coef = lognormal_coefficients(n ** 3, seed=sc)
    coeff = F.make_coeff("poisson", "fp64", source_kind=F.FE_SOURCE_CONST, source=(1.0,), dim=3)
    return dict(dim=3, n=[n, n, n], order=k, coeff=coeff, vertices=v, cell_coeff=coef)


def percentile(values, q):
    """Nearest-rank percentile (q in [0, 100])."""
    if not values:
        return None
    s = sorted(values)
    r = max(1, int(-(-q * len(s) // 100)))  # ceil(q n / 100)
    return s[min(r, len(s)) - 1]


def run_stream(server, stream, rtol=1e-8, maxit=200000, time_scale=1.0, on_done=None, timeout=1200.0,
               progress=None):
    """Submits stream[j] = (arrival_s, n, k, index) at its arrival time
    (scaled by time_scale) from a client thread and waits for all results.
    on_done(j, ticket, result) runs before the request is released; with
    progress = m, a line on stderr after every m-th result.  A request the
    server refuses at submission (more device memory than its whole budget)
    gets the result dict(state="rejected", error=...).  Returns the
    per-request results and the makespan."""
    inputs = [request_inputs(i, n, k) for (_, n, k, i) in stream]
    if progress:
        print(f"[serve] inputs of {len(stream)} requests built", file=sys.stderr, flush=True)
    tickets = [None] * len(stream)
    errors = []
    submitted = threading.Event()

    def client():
        t0 = time.perf_counter()
        try:
            for j, (t, _, _, _) in enumerate(stream):
                delay = t * time_scale - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
                a = inputs[j]
                try:
                    tickets[j] = server.submit(a["dim"], a["n"], a["order"], a["coeff"], rtol, maxit,
                                               vertices=a["vertices"], cell_coeff=a["cell_coeff"])
                except F.FeError as e:
                    if e.status != F.FE_ENOMEM:
                        raise
                    tickets[j] = ("rejected", str(e))
        except Exception as e:  # reported by the caller
            errors.append(e)
        finally:
            submitted.set()

    c0 = server.clock()
    th = threading.Thread(target=client, daemon=True)
    th.start()
    results = [None] * len(stream)
    for j in range(len(stream)):
        while tickets[j] is None and not errors:
            time.sleep(0.0005)
        if errors:
            break
        if isinstance(tickets[j], tuple):
            results[j] = dict(state="rejected", error=tickets[j][1])
            continue
        r = server.wait(tickets[j], timeout)
        results[j] = r
        if on_done is not None:
            on_done(j, tickets[j], r)
        server.release(tickets[j])
        if progress and (j + 1) % progress == 0:
            print(f"[serve] {j + 1}/{len(stream)} results", file=sys.stderr, flush=True)
    th.join()
    if errors:
        raise errors[0]
    makespan = max((r["t_done"] for r in results if r["state"] != "rejected"), default=c0) - c0
    return results, makespan


def summarize(results, makespan):
    """Latency statistics over the served requests (queueing included);
    requests refused at submission are counted, not timed."""
    rejected = [r for r in results if r["state"] == "rejected"]
    results = [r for r in results if r["state"] != "rejected"]
    lat = [r["t_done"] - r["t_submit"] for r in results]
    queue = [r["t_admit"] - r["t_submit"] for r in results]
    setup = [r["t_ready"] - r["t_admit"] for r in results]
    ok = sum(1 for r in results if r["state"] == F.FE_REQ_DONE and r["status"] == F.FE_OK)
    return {"requests": len(results) + len(rejected), "served": len(results), "rejected_at_submission": len(rejected),
            "converged": ok, "makespan_s": makespan,
            "solves_per_s": ok / makespan if makespan > 0 else None,
            "p50_ms": percentile(lat, 50) * 1e3, "p99_ms": percentile(lat, 99) * 1e3,
            "max_ms": max(lat) * 1e3, "queue_p50_ms": percentile(queue, 50) * 1e3,
            "queue_p99_ms": percentile(queue, 99) * 1e3, "setup_p50_ms": percentile(setup, 50) * 1e3,
            "iters_max": max(r["iters"] for r in results),
            "dofs": sum(r["n_rows"] for r in results), "nnz": sum(r["nnz"] for r in results)}
