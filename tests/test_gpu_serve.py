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
