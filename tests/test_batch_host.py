"""Host logic of the batching form (no GPU): wave planning and problem sizes."""
import pytest

from fe_inputs import batch_specs
from paper_1708_01773_amd.batch import plan_waves, problem_bytes


def test_waves_fit_the_budget_and_keep_order():
    sizes = [5, 3, 7, 1, 9, 2, 2]
    waves = plan_waves(sizes, 10)
    assert [i for w in waves for i in w] == list(range(len(sizes)))
    assert all(sum(sizes[i] for i in w) <= 10 for w in waves)
    # greedy: the next problem would not have fit in the previous wave
    for a, b in zip(waves, waves[1:]):
        assert sum(sizes[i] for i in a) + sizes[b[0]] > 10
    assert plan_waves([], 10) == []
    assert plan_waves([10, 10], 10) == [[0], [1]]
    with pytest.raises(ValueError):
        plan_waves([3, 11], 10)


def test_batch_specs_follow_the_recipe():
    specs = batch_specs(512)
    assert len(specs) == 512 and specs == batch_specs(512)
    ns = [n for n, _ in specs]
    ks = [k for _, k in specs]
    assert min(ns) >= 8 and max(ns) <= 64 and set(ks) == {1, 2, 3}
    # uniform draws: every order and both halves of the size range are well represented
    assert all(ks.count(k) > 120 for k in (1, 2, 3))
    assert sum(n <= 36 for n in ns) > 200 and sum(n > 36 for n in ns) > 200


def test_problem_bytes_counts_csr_and_vectors():
    b = problem_bytes(1000, 27000, 4096)
    assert b >= 8 * 1001 + 12 * 27000 + 6 * 8 * 1000 + 4096


def test_serving_summary_counts_refused_requests_apart():
    from paper_1708_01773_amd import fe as F
    from paper_1708_01773_amd.serve import percentile, summarize
    done = lambda ts, ta, tr, td: dict(state=F.FE_REQ_DONE, status=F.FE_OK, t_submit=ts, t_admit=ta, t_ready=tr,
                                       t_done=td, iters=10, n_rows=5, nnz=25)
    res = [done(0.0, 0.0, 0.1, 1.0), dict(state="rejected", error="budget"), done(0.5, 0.6, 0.7, 3.5)]
    s = summarize(res, 3.5)
    assert s["requests"] == 3 and s["served"] == 2 and s["rejected_at_submission"] == 1 and s["converged"] == 2
    assert s["p50_ms"] == 1000.0 and s["p99_ms"] == 3000.0 and s["solves_per_s"] == 2 / 3.5
    assert percentile([5, 1, 3], 50) == 3 and percentile([1], 99) == 1
