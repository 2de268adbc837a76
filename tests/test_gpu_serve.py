"""GPU test of the continuous-batching server: every request's result is the
same when served in the mix as when run alone (bitwise: identical
populations give identical diagnostics), and the serial baseline agrees."""
import pytest

from paper_2303_08163_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("policy", ["fifo", "swf"])
def test_served_results_equal_alone(policy):
    import torch
    from paper_2303_08163_amd import lbm, serve
    trace = workloads.serving_trace(n_requests=14, rate=400.0, seed=11, d2_range=(64, 160), d3_range=(16, 40),
                                    steps_range=(20, 300))
    be = serve.PoolBackend(1 << 30, max_slots=5)
    try:
        kw = {"policy": "swf", "lookahead": 64, "saturate_bytes": 2e6} if policy == "swf" else {"policy": "fifo"}
        out = serve.Server(be, chunk_s=0.002, **kw).serve(trace)
    finally:
        be.close()
    assert sorted(r["id"] for r in out) == list(range(len(trace)))
    dev = torch.device("cuda:0")
    byid = {r["id"]: r for r in out}
    for req in trace:
        rho, u = serve.init_fields_device(req, dev)
        with lbm.Domain.from_device(rho, u, req["tau"], dtype="fp32_dev") as d:
            d.step(req["steps"])
            _, _, diag = d.moments(fields=False, raise_on_domain=False)
        assert diag == byid[req["id"]]["diag"], req
    base = {r["id"]: r for r in serve.serial_serve(trace[:5])}
    for i in range(5):
        assert base[i]["diag"] == byid[i]["diag"]
    s = serve.summarize(out)
    assert s["requests"] == len(trace) and s["p99_latency_s"] >= s["p50_latency_s"] > 0
