"""Continuous-batching server for simulation requests on one GPU.

Requests (lattice, grid, initial field, u0, tau, step count) arrive over time.
The server keeps the populations of admitted requests resident in HBM as slots
of one pool, admits queued requests whenever a slot and a large enough block
of the arena are free (admission by memory footprint), advances every active
slot in chunks of K steps (one pool run: one kernel launch per step, or per
two steps, covering all active requests of a class), and returns a result as
soon as a request's steps are done.  Requests arriving while others run join
the next chunk, so their work overlaps on the device.

The loop is pipelined so that the GPU does not drain between chunks:
admissions are enqueued without a synchronisation, chunk n + 1 is enqueued
before the server waits for chunk n, and the results of the requests that
chunk n finished are read on a second stream while chunk n + 1 runs.

Latency is measured from a request's arrival to the moment its result
(diagnostics read back from the GPU) is available.

The scheduling logic takes a backend object (admit / run / collect / result /
release / cost estimate), so it can be exercised with a stand-in backend and a
virtual clock; the production backend is PoolBackend over the native pool.
"""
from __future__ import annotations

import math
import time
from collections import deque

import numpy as np


def init_fields_device(req: dict, device):
    """Initial (rho, u) of a request as float64 torch tensors on `device`,
    assembled on the device from 1-D profiles (the same formulas and the same
    numpy values as the workloads module).  The profiles go up through pinned
    host memory without blocking, so that a request can be prepared while
    earlier work is still running on the stream."""
    import torch
    n, u0 = req["n"], req["u0"]
    k = 2.0 * math.pi / n
    x = np.arange(n, dtype=np.float64)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).pin_memory().to(device, non_blocking=True)
    if req["lattice"] == 9:
        if req["init"] == "taylor_green":
            cx, sx, c2x = t(np.cos(k * x)), t(np.sin(k * x)), t(np.cos(2 * k * x))
            ux = -u0 * cx[None, :] * sx[:, None]
            uy = u0 * sx[None, :] * cx[:, None]
            rho = 1.0 * (1.0 - 0.75 * u0 * u0 * (c2x[None, :] + c2x[:, None]))
            return rho.contiguous(), torch.stack([ux, uy]).contiguous()
        s = t(u0 * np.sin(2.0 * math.pi * x / n))
        ux = s[:, None].expand(n, n)
        return torch.ones((n, n), dtype=torch.float64, device=device), \
            torch.stack([ux, torch.zeros_like(ux)]).contiguous()
    if req["init"] == "taylor_green":
        sx, cx, c2x = t(np.sin(k * x)), t(np.cos(k * x)), t(np.cos(2 * k * x))
        ux = u0 * sx[None, None, :] * cx[None, :, None] * cx[:, None, None]
        uy = -u0 * cx[None, None, :] * sx[None, :, None] * cx[:, None, None]
        rho = 1.0 + (3.0 * u0 * u0 / 16.0) * (c2x[None, None, :] + c2x[None, :, None]) * (c2x[:, None, None] + 2.0)
        return rho.contiguous(), torch.stack([ux, uy, torch.zeros_like(ux)]).contiguous()
    s = t(u0 * np.sin(2.0 * math.pi * x / n))
    ux = s[None, :, None].expand(n, n, n)
    z = torch.zeros((n, n, n), dtype=torch.float64, device=device)
    return torch.ones((n, n, n), dtype=torch.float64, device=device), torch.stack([ux, z, z]).contiguous()


class PoolBackend:
    """Backend over the native pool (one arena of `budget_bytes` of HBM).

    tuning None selects row fit (each slot's rows mapped to 64-, 128- or
    256-wide tiles): on the serving request mix (D2Q9 64^2..1024^2, D3Q27
    32^3..192^3) it served 2.5-4 % more requests per second than the pool's
    default 64 x 4 tiles; and two steps per launch for D2Q9 classes.

    Admissions are enqueued without a synchronisation (lbm_pool_admit_async)
    on the pool's stream, which is torch's current stream when the backend is
    made: the initial fields are built on that stream, so the allocator frees
    them in stream order behind the initialisation that reads them."""

    def __init__(self, budget_bytes: int, max_slots: int = 256, tuning=None, dtype: str = "fp32_dev",
                 device="cuda:0", bytes_per_s: float = 5.0e12):
        import torch
        from . import lbm
        self.lbm = lbm
        self.torch = torch
        if tuning is None:
            tuning = lbm.make_pool_tuning(64, 4, 0, row_fit=1, time_block=2)
        self.dtype = dtype
        self.pool = lbm.Pool(budget_bytes, max_slots=max_slots, tuning=tuning, device=device)
        self.device = self.pool.device
        self.bytes_per_s = bytes_per_s
        self.slot_req = {}
        self._events = []  # (start, end) CUDA events of every run, for the GPU-busy time

    def footprint(self, req) -> int:
        lbm = self.lbm
        n = req["n"]
        shape = (n, n) if req["lattice"] == 9 else (n, n, n)
        return lbm.lbm_pool_slot_bytes(lbm.make_config(req["lattice"], shape, req["tau"], self.dtype),
                                       self.pool.tuning)

    def try_admit(self, req, fields=None):
        lbm = self.lbm
        if self.footprint(req) > self.pool.stats()["largest_free_block"]:
            return None
        with self.torch.cuda.stream(self.pool.stream):
            rho, u = fields if fields is not None else init_fields_device(req, self.device)
        cfg = lbm.make_config(req["lattice"], tuple(rho.shape[::-1]), req["tau"], self.dtype)
        try:
            slot = lbm.lbm_pool_admit_async(self.pool.handle, cfg, rho.data_ptr(), u.data_ptr(), req["steps"])
        except lbm.LBMError as e:
            if e.status in (lbm.LBM_EBUSY, lbm.LBM_ENOMEM):
                return None
            raise
        self.pool.shapes[slot] = tuple(rho.shape)
        self.slot_req[slot] = req
        return slot

    @staticmethod
    def step_bytes(req) -> int:
        """HBM bytes of one step of a request (2 Q 4 bytes per node, FP32 storage)."""
        q, nodes = (9, req["n"] ** 2) if req["lattice"] == 9 else (27, req["n"] ** 3)
        return 2 * q * 4 * nodes

    def step_seconds(self, slots) -> float:
        """Estimated GPU time of one step of the given slots (memory-bound)."""
        return sum(self.step_bytes(self.slot_req[s]) for s in slots) / self.bytes_per_s

    def remaining(self, slot) -> int:
        return int(self.pool.slot_info(slot)["steps_remaining"])

    def run(self, k: int) -> int:
        """Enqueue k steps of every running slot; returns the run's number."""
        torch = self.torch
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(self.pool.stream)
        self.pool.run(k)
        ev1.record(self.pool.stream)
        self._events.append((ev0, ev1))
        return int(self.pool.stats()["runs"])

    def collect(self, after_run: int) -> list:
        """Wait for run `after_run`, then list the finished slots whose work is done."""
        return self.lbm.lbm_pool_collect(self.pool.handle, after_run, self.pool.max_slots)

    def result(self, slot, fields: bool = False) -> dict:
        if fields:
            rho, u, d = self.pool.moments(slot, fields=True, raise_on_domain=False)
            return dict(d, rho=rho, u=u)
        _, _, d = self.pool.moments(slot, fields=False, raise_on_domain=False)
        return d

    def release(self, slot) -> None:
        self.pool.release(slot)
        self.slot_req.pop(slot, None)

    def gpu_busy_seconds(self) -> float:
        """GPU time of all runs so far (synchronises)."""
        self.pool.stream.synchronize()
        return sum(a.elapsed_time(b) for a, b in self._events) / 1e3

    def close(self):
        self.pool.close()


class Server:
    """Continuous batching over a backend.

    chunk_s: target GPU time of one run (bounds how long a newly arrived
    request waits before it joins); lookahead: how many queued requests are
    tried per admission pass (first fit within the window); depth: runs kept
    in flight (2: the next chunk is enqueued before the server waits for the
    current one).
    policy:
      "fifo"  the window is taken in arrival order and every request that fits
              in memory is admitted (all admitted requests share the GPU);
      "swf"   (default) shortest work first: the queue is ordered by estimated work
              (bytes per step x steps), and admission stops once the running
              requests move `saturate_bytes` per step -- enough to keep the GPU
              busy -- so that short requests finish first instead of sharing
              the device with everything queued.  Admitted requests are never
              paused, so this approximates shortest-remaining-work order.
    keep_fields: also return each request's rho and u fields (numpy; for
    tests -- the copies to the host add to the loop's turn-around).
    """

    def __init__(self, backend, chunk_s: float = 0.02, lookahead: int = 64, max_chunk: int = 2000,
                 clock=time.perf_counter, sleep=time.sleep, policy: str = "swf",
                 saturate_bytes: float = 512e6, depth: int = 2, keep_fields: bool = False):
        if policy not in ("fifo", "swf"):
            raise ValueError("policy must be 'fifo' or 'swf'")
        if depth < 1:
            raise ValueError("depth must be >= 1")
        self.b = backend
        self.chunk_s = chunk_s
        self.lookahead = lookahead
        self.max_chunk = max_chunk
        self.clock = clock
        self.sleep = sleep
        self.policy = policy
        self.saturate_bytes = saturate_bytes
        self.depth = depth
        self.keep_fields = keep_fields

    def _work(self, req) -> float:
        return float(self.b.step_bytes(req)) * req["steps"]

    def serve(self, trace):
        """Serve a list of requests (dicts with 'arrival' seconds from start).
        Returns one record per request: id, arrival, admitted, finished,
        latency (finished - arrival), diagnostics."""
        b = self.b
        t0 = self.clock()
        now = lambda: self.clock() - t0
        queue = deque()
        active = {}  # slot -> (request, admitted time): admitted, result not yet read
        inflight = deque()  # runs enqueued and not yet waited for
        out = []
        i = 0
        trace = sorted(trace, key=lambda r: r["arrival"])

        def finish(slots):
            for slot in slots:
                req, adm = active.pop(slot)
                res = b.result(slot, fields=True) if self.keep_fields else b.result(slot)
                fin = now()
                rec = dict(id=req["id"], arrival=req["arrival"], admitted=adm, finished=fin,
                           latency=fin - req["arrival"], diag=res)
                if self.keep_fields:
                    rec["rho"], rec["u"] = res.pop("rho"), res.pop("u")
                out.append(rec)
                b.release(slot)

        while i < len(trace) or queue or active:
            t = now()
            while i < len(trace) and trace[i]["arrival"] <= t:
                queue.append(trace[i])
                i += 1
            running = [s for s in active if b.remaining(s) > 0]
            # admission: first fit within the look-ahead window, in arrival order
            # (fifo) or in order of estimated work up to the saturation traffic (swf)
            tried = 0
            if self.policy == "swf":
                order = sorted(queue, key=lambda r: (self._work(r), r["arrival"]))
                load = sum(b.step_bytes(active[s][0]) for s in running)
            else:
                order = list(queue)
                load = 0.0
            for req in order:
                if tried >= self.lookahead:
                    break
                if self.policy == "swf" and running and load >= self.saturate_bytes:
                    break
                tried += 1
                slot = b.try_admit(req)
                if slot is not None:
                    active[slot] = (req, now())
                    queue.remove(req)
                    load += b.step_bytes(req)
                    running.append(slot)
            running = [s for s in running if b.remaining(s) > 0]
            enqueued = False
            if running and len(inflight) < self.depth:
                # one chunk: long enough to amortise launches, short enough for admission,
                # and ending exactly when the next running request finishes
                step_s = max(b.step_seconds(running), 1e-7)
                k = int(max(1, min(self.max_chunk, self.chunk_s / step_s)))
                k = min(k, min(b.remaining(s) for s in running))
                inflight.append(b.run(max(1, k)))
                enqueued = True
            if inflight and (len(inflight) >= self.depth or not enqueued):
                # wait for the oldest run (the newer one keeps the GPU busy) and read
                # the results of the requests it finished
                finish(b.collect(inflight.popleft()))
                continue
            if not inflight and active and not running:
                finish(b.collect(0))  # finished slots whose work needs no run
                continue
            if not active:
                if i < len(trace):
                    wait = trace[i]["arrival"] - now()
                    if wait > 0:
                        self.sleep(wait)
                    continue
                if queue:
                    raise RuntimeError(f"request {queue[0]['id']} can never be admitted (larger than the pool)")
                break
        return out


def serial_serve(trace, dtype: str = "fp32_dev", device="cuda:0", clock=time.perf_counter, sleep=time.sleep):
    """The plain baseline: one request at a time, in arrival order, each a
    single domain stepped with one kernel launch per step."""
    import torch
    from . import lbm
    dev = torch.device(device)
    t0 = clock()
    out = []
    for req in sorted(trace, key=lambda r: r["arrival"]):
        wait = req["arrival"] - (clock() - t0)
        if wait > 0:
            sleep(wait)
        rho, u = init_fields_device(req, dev)
        start = clock() - t0
        d = lbm.Domain.from_device(rho, u, req["tau"], dtype=dtype)
        d.step(req["steps"])
        _, _, diag = d.moments(fields=False, raise_on_domain=False)
        d.close()
        fin = clock() - t0
        out.append(dict(id=req["id"], arrival=req["arrival"], admitted=start, finished=fin,
                        latency=fin - req["arrival"], diag=diag))
    return out


def summarize(records, wall_s: float | None = None) -> dict:
    lat = np.array([r["latency"] for r in records])
    fin = max(r["finished"] for r in records) if records else 0.0
    wall = wall_s if wall_s is not None else fin
    return {"requests": len(records), "solves_per_s": round(len(records) / wall, 3) if wall > 0 else None,
            "p50_latency_s": round(float(np.percentile(lat, 50)), 4) if len(lat) else None,
            "p99_latency_s": round(float(np.percentile(lat, 99)), 4) if len(lat) else None,
            "mean_latency_s": round(float(lat.mean()), 4) if len(lat) else None,
            "makespan_s": round(fin, 3)}
