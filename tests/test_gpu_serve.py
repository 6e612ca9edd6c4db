"""GPU: continuous batching.  Requests served together (arriving while others run, sharing the
device through the batched step) give exactly the results of the same requests served one at
a time with plain launches."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2006_06775_amd import serve  # noqa: E402


def test_served_results_equal_alone():
    print("case: serve mix vs alone", flush=True)
    trace = serve.make_trace(12, seed=3, rate=5000.0, n_min=1000, n_max=40000, s_min=3, s_max=9)
    srv = serve.Server(capacity=200_000, max_boxes=600_000, slots=6, keep_results=True)
    stats = srv.run(trace)
    s = stats.summary()
    assert s["requests"] == 12 and s["max_concurrent"] > 1
    _, alone = serve.run_plain(trace, keep_results=True)
    for r in trace:
        for k in ("x", "y", "z"):
            assert np.array_equal(srv.results[r.rid][k].view(np.uint64), alone[r.rid][k].view(np.uint64)), (r.rid, k)
    print(s, flush=True)


def test_server_without_graph_matches():
    print("case: serve eager", flush=True)
    trace = serve.make_trace(5, seed=4, rate=1000.0, n_min=2000, n_max=9000, s_min=2, s_max=5)
    a = serve.Server(capacity=60_000, max_boxes=200_000, slots=3, use_graph=False, keep_results=True)
    a.run(trace)
    b = serve.Server(capacity=60_000, max_boxes=200_000, slots=3, use_graph=True, keep_results=True)
    b.run(trace)
    for r in trace:
        assert np.array_equal(a.results[r.rid]["x"], b.results[r.rid]["x"])


def test_served_mixed_box_edges_equal_alone():
    """Requests of different sizes get different box edges from a plan; each served result still
    equals the same request served alone with its edge."""
    print("case: serve mixed box edges", flush=True)
    from paper_2006_06775_amd import tune
    plan = tune.BoxPlan(serve.D_HI, {1000: 1.0, 30000: 1.3})
    trace = serve.make_trace(8, seed=5, rate=5000.0, n_min=1000, n_max=40000, s_min=2, s_max=6)
    assert len({serve.box_edge(plan, r.n) for r in trace}) == 2
    srv = serve.Server(capacity=200_000, max_boxes=600_000, slots=4, box=plan, keep_results=True)
    srv.run(trace)
    _, alone = serve.run_plain(trace, box=plan, keep_results=True)
    for r in trace:
        for k in ("x", "y", "z"):
            assert np.array_equal(srv.results[r.rid][k], alone[r.rid][k]), (r.rid, k)


def test_tune_plan_measures():
    print("case: tune plan", flush=True)
    from paper_2006_06775_amd import tune
    plan = tune.plan(classes=(2000, 20000), factors=(1.0, 1.25), caps=(1024, 8192), steps=2)
    assert set(plan.best) == {2000, 20000} and set(plan.best.values()) <= {1.0, 1.25}
    assert all(t > 0 for row in plan.table.values() for t in row.values())
    assert set(plan.split_table) == {1024, 8192} and plan.grid_cap in (1024, 8192)


def test_work_split_changes_no_result():
    """The same requests served with different work splits (grid caps) give identical results."""
    print("case: serve work splits", flush=True)
    from paper_2006_06775_amd import tune
    trace = serve.make_trace(6, seed=6, rate=5000.0, n_min=2000, n_max=60000, s_min=2, s_max=5)
    res = []
    for cap in (64, 1024, 0):
        srv = serve.Server(capacity=200_000, max_boxes=600_000, slots=4, box=tune.fixed(1.0, cap),
                           keep_results=True)
        srv.run(trace)
        res.append(srv.results)
    for r in trace:
        for k in ("x", "y", "z"):
            assert np.array_equal(res[0][r.rid][k].view(np.uint64), res[1][r.rid][k].view(np.uint64))
            assert np.array_equal(res[0][r.rid][k].view(np.uint64), res[2][r.rid][k].view(np.uint64))
