"""GPU tests of the continuous-batching server.

Every request's rho and u fields are bitwise the same when served in the mix
(pipelined runs, unsynchronised admissions, reads on the pool's second
stream) as when the request runs alone as a single domain; two served
requests also match the FP64 CPU oracle within the FP32 budget (normwise
1e-5); and the serial baseline returns the same diagnostics.  Four 1024^2
D2Q9 requests arrive together after the small ones, so that their class holds
2^22 nodes, the size at which the pool advances D2Q9 two steps per launch."""
import numpy as np
import pytest

import oracle
from paper_2303_08163_amd import workloads

pytestmark = pytest.mark.gpu


def _trace():
    trace = workloads.serving_trace(n_requests=14, rate=400.0, seed=11, d2_range=(64, 160), d3_range=(16, 40),
                                    steps_range=(20, 300))
    t_big = trace[-1]["arrival"] + 0.5
    big = [dict(id=14 + j, arrival=t_big, lattice=9, n=1024, init="shear_wave" if j % 2 else "taylor_green",
                u0=0.05 + 0.02 * j, tau=0.52 + 0.01 * j, steps=40) for j in range(4)]
    return trace + big


def _alone(req):
    import torch
    from paper_2303_08163_amd import lbm, serve
    rho, u = serve.init_fields_device(req, torch.device("cuda:0"))
    with lbm.Domain.from_device(rho, u, req["tau"], dtype="fp32_dev") as d:
        d.step(req["steps"])
        return d.moments(raise_on_domain=False)


def rel_err(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


@pytest.mark.parametrize("policy", ["fifo", "swf"])
def test_served_fields_equal_alone_and_oracle(policy):
    from paper_2303_08163_amd import serve
    trace = _trace()
    be = serve.PoolBackend(1 << 30, max_slots=8)
    try:
        kw = {"policy": "swf", "lookahead": 64, "saturate_bytes": 400e6} if policy == "swf" else {"policy": "fifo"}
        out = serve.Server(be, chunk_s=0.002, keep_fields=True, **kw).serve(trace)
        assert be.pool.stats()["used_slots"] == 0
    finally:
        be.close()
    assert sorted(r["id"] for r in out) == list(range(len(trace)))
    byid = {r["id"]: r for r in out}
    for req in trace:
        rho, u, diag = _alone(req)
        served = byid[req["id"]]
        assert served["diag"]["steps"] == req["steps"] and not served["diag"]["domain_error"]
        assert np.array_equal(served["rho"], rho) and np.array_equal(served["u"], u), req
        assert served["diag"] == diag, req
    # two served requests (the smallest of each lattice) against the oracle
    for lat in (9, 27):
        req = min((r for r in trace if r["lattice"] == lat), key=lambda r: r["n"] ** (2 if lat == 9 else 3))
        rho0, u0 = workloads.request_fields(req)
        oracle.set_threads(16)
        r_ref, u_ref, bad = oracle.run(rho0, u0, req["tau"], req["steps"])
        er, eu = rel_err(byid[req["id"]]["rho"], r_ref), rel_err(byid[req["id"]]["u"], u_ref)
        print(f"[parity] served D{2 if lat == 9 else 3} {req['n']} {req['steps']} steps FP32 ({policy}): "
              f"rel err rho {er:.3e}  u {eu:.3e}", flush=True)
        assert bad == 0 and er < 1e-5 and eu < 1e-5
    s = serve.summarize(out)
    assert s["requests"] == len(trace) and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_serial_baseline_matches_served_diagnostics():
    from paper_2303_08163_amd import serve
    trace = _trace()[:5]
    base = {r["id"]: r for r in serve.serial_serve(trace)}
    for req in trace:
        _, _, diag = _alone(req)
        assert base[req["id"]]["diag"] == diag
