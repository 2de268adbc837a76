"""CPU tests of the serving scheduler (continuous batching) with a stand-in
backend and a virtual clock.  The stand-in lives here, in the tests: it models
a memory budget, a slot limit and a memory-bound step cost, so the scheduling
logic (arrival, admission by footprint, chunking, completion, release) can be
checked without a GPU.  No numerics run here."""
import math

import pytest

from paper_2303_08163_amd import serve, workloads


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def clock(self):
        return self.t

    def sleep(self, dt):
        self.t += max(0.0, dt)


class FakeBackend:
    def __init__(self, clock, budget, max_slots, bytes_per_s=5e12):
        self.clk = clock
        self.budget = budget
        self.max_slots = max_slots
        self.bps = bytes_per_s
        self.used = 0
        self.peak = 0
        self.slots = {}  # slot -> [req, remaining]
        self.finished = []
        self.reported = set()
        self.log = []
        # the device: runs execute one after another from the moment they are
        # enqueued or the previous one ends, whichever is later
        self.gpu_free = 0.0
        self.runs = 0
        self.run_end = {}
        self.done_at = {}
        self.spans = []  # (start, end) of every run on the device

    def footprint(self, req):
        q, nodes = (9, req["n"] ** 2) if req["lattice"] == 9 else (27, req["n"] ** 3)
        return 2 * q * 4 * nodes

    def step_bytes(self, req):
        return self.footprint(req)

    def try_admit(self, req, fields=None):
        fp = self.footprint(req)
        if len(self.slots) >= self.max_slots or self.used + fp > self.budget:
            return None
        slot = next(i for i in range(self.max_slots) if i not in self.slots)
        self.slots[slot] = [req, req["steps"]]
        self.used += fp
        self.peak = max(self.peak, self.used)
        self.log.append(("admit", req["id"], self.clk.t))
        return slot

    def step_seconds(self, slots):
        return sum(self.footprint(self.slots[s][0]) for s in slots) / self.bps

    def remaining(self, slot):
        return self.slots[slot][1]

    def run(self, k):
        """Enqueue: returns at once with the run's number; the device time of
        each step is the traffic of the slots still active at that step."""
        act = [s for s, (_, rem) in self.slots.items() if rem > 0]
        steps = sorted(set([min(k, self.slots[s][1]) for s in act]))
        t = max(self.clk.t, self.gpu_free)
        prev = 0
        for st in steps:
            live = [s for s in act if self.slots[s][1] > prev]
            t += (st - prev) * self.step_seconds(live)
            prev = st
        self.spans.append((max(self.clk.t, self.gpu_free), t))
        self.gpu_free = t
        self.runs += 1
        self.run_end[self.runs] = t
        for s in act:
            self.slots[s][1] -= min(k, self.slots[s][1])
            if self.slots[s][1] == 0:
                self.done_at[s] = t
        self.log.append(("run", k, self.clk.t))
        return self.runs

    def collect(self, after_run):
        """Wait for run after_run, then list finished slots whose work is done."""
        if after_run >= 1:
            self.clk.t = max(self.clk.t, self.run_end[after_run])
        out = [s for s, (_, rem) in self.slots.items()
               if rem == 0 and s not in self.reported and self.done_at.get(s, 0.0) <= self.clk.t]
        self.reported |= set(out)
        return out

    def result(self, slot):
        return {"steps": self.slots[slot][0]["steps"]}

    def release(self, slot):
        req, _ = self.slots.pop(slot)
        self.reported.discard(slot)
        self.done_at.pop(slot, None)
        self.used -= self.footprint(req)
        self.log.append(("release", req["id"], self.clk.t))


def _trace(n=60, rate=200.0, seed=8163, **kw):
    return workloads.serving_trace(n_requests=n, rate=rate, seed=seed, **kw)


def test_trace_distribution():
    tr = _trace(n=2000)
    assert all(0.5001 <= r["tau"] <= 0.6 and 0.01 <= r["u0"] <= 0.15 and 200 <= r["steps"] <= 5000 for r in tr)
    d2 = [r["n"] for r in tr if r["lattice"] == 9]
    d3 = [r["n"] for r in tr if r["lattice"] == 27]
    assert 0.45 < len(d3) / len(tr) < 0.55
    assert min(d2) >= 64 and max(d2) <= 1024 and min(d3) >= 32 and max(d3) <= 192
    gaps = [b["arrival"] - a["arrival"] for a, b in zip(tr, tr[1:])]
    assert abs(sum(gaps) / len(gaps) - 1 / 200.0) < 0.2 / 200.0  # Poisson, mean 1/rate


def test_all_requests_served_within_budget():
    clk = VirtualClock()
    be = FakeBackend(clk, budget=8 << 30, max_slots=16)
    srv = serve.Server(be, chunk_s=0.02, clock=clk.clock, sleep=clk.sleep)
    tr = _trace(n=80)
    out = srv.serve(tr)
    assert sorted(r["id"] for r in out) == [r["id"] for r in tr]
    assert be.peak <= 8 << 30 and len(be.slots) == 0
    for r in out:
        assert r["admitted"] >= r["arrival"] - 1e-12 and r["finished"] >= r["admitted"]
        assert r["latency"] == pytest.approx(r["finished"] - r["arrival"])


def test_work_overlaps_and_arrivals_join_running_batches():
    clk = VirtualClock()
    be = FakeBackend(clk, budget=64 << 30, max_slots=64)
    srv = serve.Server(be, chunk_s=0.01, clock=clk.clock, sleep=clk.sleep)
    out = srv.serve(_trace(n=40))
    byid = {r["id"]: r for r in out}
    # some request was admitted while an earlier-admitted one was still running
    overlap = any(a["admitted"] < b["finished"] and b["admitted"] < a["admitted"]
                  for a in out for b in out if a is not b)
    assert overlap
    # short requests admitted later can finish before long ones admitted earlier
    assert any(byid[i]["finished"] < byid[j]["finished"] and byid[i]["admitted"] > byid[j]["admitted"]
               for i in byid for j in byid)


def test_admission_waits_for_memory():
    clk = VirtualClock()
    big = dict(id=0, arrival=0.0, lattice=27, n=64, init="taylor_green", u0=0.05, tau=0.6, steps=100)
    reqs = [dict(big, id=i, arrival=0.001 * i) for i in range(4)]
    fp = FakeBackend(clk, 0, 1).footprint(big)
    be = FakeBackend(clk, budget=2 * fp + 1, max_slots=8)
    srv = serve.Server(be, chunk_s=1.0, clock=clk.clock, sleep=clk.sleep)
    out = srv.serve(reqs)
    assert be.peak <= 2 * fp + 1
    starts = sorted(r["admitted"] for r in out)
    # two at a time: the third starts only when memory from the first pair is released
    ends = sorted(r["finished"] for r in out)
    assert starts[2] >= ends[0] - 1e-12


def test_chunks_end_when_a_request_finishes():
    clk = VirtualClock()
    be = FakeBackend(clk, budget=64 << 30, max_slots=8)
    a = dict(id=0, arrival=0.0, lattice=9, n=256, init="shear_wave", u0=0.05, tau=0.6, steps=1000)
    b = dict(a, id=1, steps=10)
    srv = serve.Server(be, chunk_s=10.0, clock=clk.clock, sleep=clk.sleep)
    out = {r["id"]: r for r in srv.serve([a, b])}
    # b's result is available after 10 steps of both, not after a's 1000
    step_both = 2 * be.footprint(a) / be.bps
    assert out[1]["finished"] == pytest.approx(10 * step_both, rel=1e-9)


def test_oversized_request_is_reported():
    clk = VirtualClock()
    be = FakeBackend(clk, budget=1 << 20, max_slots=4)
    srv = serve.Server(be, clock=clk.clock, sleep=clk.sleep)
    req = dict(id=0, arrival=0.0, lattice=27, n=128, init="taylor_green", u0=0.05, tau=0.6, steps=10)
    with pytest.raises(RuntimeError):
        srv.serve([req])


def test_summarize():
    recs = [dict(latency=float(i), finished=float(i) + 1) for i in range(101)]
    s = serve.summarize(recs)
    assert s["p50_latency_s"] == 50.0 and s["p99_latency_s"] == pytest.approx(99.0)
    assert s["requests"] == 101 and s["solves_per_s"] == pytest.approx(101 / 101.0)
    assert math.isfinite(s["mean_latency_s"])


def test_shortest_work_first_cuts_median_latency_under_overload():
    """With requests arriving far faster than they can be served, ordering by
    estimated work (and not sharing the GPU with everything queued) lowers the
    median latency; every request is still served within the memory budget."""
    tr = _trace(n=80, rate=200.0)
    res = {}
    for policy in ("fifo", "swf"):
        clk = VirtualClock()
        be = FakeBackend(clk, budget=8 << 30, max_slots=32)
        srv = serve.Server(be, chunk_s=0.02, lookahead=len(tr), clock=clk.clock, sleep=clk.sleep, policy=policy)
        out = srv.serve(tr)
        assert sorted(r["id"] for r in out) == [r["id"] for r in tr] and be.peak <= 8 << 30
        res[policy] = serve.summarize(out)
    assert res["swf"]["p50_latency_s"] < 0.5 * res["fifo"]["p50_latency_s"]
    # same total work on a memory-bound device: the makespan does not grow
    assert res["swf"]["makespan_s"] <= res["fifo"]["makespan_s"] * 1.05


def test_swf_admission_stops_at_saturation():
    clk = VirtualClock()
    be = FakeBackend(clk, budget=64 << 30, max_slots=64)
    base = dict(arrival=0.0, lattice=9, n=512, init="shear_wave", u0=0.05, tau=0.6, steps=100)
    reqs = [dict(base, id=i) for i in range(10)]
    per = be.step_bytes(base)
    srv = serve.Server(be, chunk_s=1.0, lookahead=16, clock=clk.clock, sleep=clk.sleep, policy="swf",
                       saturate_bytes=3 * per)
    srv.serve(reqs)
    kinds = [kind for kind, _, _ in be.log]
    # three fill the saturation traffic of the first run; the next three are
    # admitted (still at t = 0) for the run enqueued behind it
    assert kinds[:4] == ["admit"] * 3 + ["run"]
    assert kinds[4:8] == ["admit"] * 3 + ["run"]


def test_policy_is_checked():
    clk = VirtualClock()
    with pytest.raises(ValueError):
        serve.Server(FakeBackend(clk, 1 << 30, 4), policy="lifo")


def test_thousand_request_trace():
    """The full-length serving trace (1000 Poisson arrivals at 200 req/s):
    every request served once within the budget under both policies, and
    shortest-work-first keeps the median well below FIFO batching."""
    tr = _trace(n=1000, rate=200.0)
    res = {}
    for policy in ("fifo", "swf"):
        clk = VirtualClock()
        be = FakeBackend(clk, budget=96 << 30, max_slots=512)
        out = serve.Server(be, clock=clk.clock, sleep=clk.sleep, policy=policy).serve(tr)
        assert sorted(r["id"] for r in out) == list(range(1000)) and be.peak <= 96 << 30
        res[policy] = serve.summarize(out)
    assert res["swf"]["p50_latency_s"] < 0.25 * res["fifo"]["p50_latency_s"]


def test_pipeline_keeps_the_device_busy():
    """The next run is enqueued before the server waits for the current one, so
    under load the device never idles between runs (with depth 1 it would, by
    the host's turn-around; here the virtual host takes no time, so a gap can
    only come from a run enqueued after its predecessor ended)."""
    clk = VirtualClock()
    be = FakeBackend(clk, budget=16 << 30, max_slots=32)
    tr = _trace(n=120, rate=2000.0)  # arrivals within 0.06 s: the queue never empties
    out = serve.Server(be, chunk_s=0.02, clock=clk.clock, sleep=clk.sleep).serve(tr)
    assert len(out) == len(tr)
    gaps = [b0 - a1 for (a0, a1), (b0, b1) in zip(be.spans, be.spans[1:])]
    assert max(gaps) < 1e-12
    busy = sum(b - a for a, b in be.spans)
    assert busy == pytest.approx(max(r["finished"] for r in out) - be.spans[0][0], rel=1e-9)
