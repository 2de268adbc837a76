"""Benchmark of the hot path: fused stream-and-collide steps of entropic-equilibrium
LBGK on one MI355X.

Headline workload: D3Q27, 256^3 periodic Taylor-Green vortex (u0 = 0.05,
tau = 0.5005), populations stored in FP32 as deviations f_i - w_i rho0, all
arithmetic in FP64, bulk correction off.  One "step" is one time step of the
whole domain (one kernel launch).  Inputs are resident in HBM before timing.

Prints ONE JSON line: MLUPS (= nodes * steps / s / 1e6), the roofline of the
stream-collide kernel (algorithmic bytes 2 * Q * 4 = 216 B per node update,
against the 8 TB/s HBM peak), and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS & % HBM roofline (D3Q27 256³ FP32); batched solves/s, p99 latency"
PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "stream_collide_d3q27_fp32dev_256.md")


def kernel_source_digest() -> str:
    """Digest of the sources that define the stream-collide kernels (node
    arithmetic and kernel bodies); counter-based traffic is reported only while
    they are unchanged since the counters were taken."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2303_08163_amd", "csrc")
    for fn in ("node.hpp", "kernels.hpp"):
        with open(os.path.join(csrc, fn), "rb") as f:
            h.update(fn.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None."""
    if not os.path.exists(PROFILE_SUMMARY):
        return None
    text = open(PROFILE_SUMMARY).read()
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    d = re.search(r"kernel_source_digest:\s*([0-9a-f]+)", text)
    if not m or not d or d.group(1) != kernel_source_digest():
        return None
    return float(m.group(1))


VALU_PEAK_GINST = 256 * 4 * 2.4 / 4  # G wavefront-instructions/s: 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles
VALU_PROFILE = os.path.join(ROOT, "profiles", "multistep_valu_d2q9_4096_d1q3_2e27_c4_512.md")


def multistep_source_digest() -> str:
    """Digest of the sources of the multi-step kernels (node arithmetic, one-step,
    two-step and pool kernels); their counted VALU instructions are used only
    while it matches the profile's."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2303_08163_amd", "csrc")
    for fn in ("node.hpp", "kernels.hpp", "kernels_t2.hpp", "pool_kernels.hpp", "tile_deps.hpp"):
        with open(os.path.join(csrc, fn), "rb") as f:
            h.update(fn.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def valu_counts() -> dict:
    """VALU wavefront-instructions per launch of the multi-step kernels, from the
    committed rocprofv3 summary, or {} when the kernels have changed since."""
    if not os.path.exists(VALU_PROFILE):
        return {}
    text = open(VALU_PROFILE).read()
    d = re.search(r"valu_kernel_source_digest:\s*([0-9a-f]+)", text)
    if not d or d.group(1) != multistep_source_digest():
        return {}
    return {m.group(1): float(m.group(2)) for m in re.finditer(r"valu_insts_per_launch\.(\S+):\s*([0-9.eE+]+)", text)}


def valu_roofline(key: str, launch_s: float):
    """Issue-rate roofline of a multi-step kernel: counted VALU instructions per
    launch over the launch time measured here, against 614.4 G/s."""
    n = valu_counts().get(key)
    if n is None:
        return None
    achieved = n / launch_s / 1e9
    return {"bound": "valu", "achieved": round(achieved, 1), "peak": VALU_PEAK_GINST,
            "unit": "G wavefront-instructions/s", "frac": round(achieved / VALU_PEAK_GINST, 4),
            "insts_per_launch": n}


def cpu_threads() -> int:
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(budget_s: float = 12.0) -> dict:
    """The CPU oracle (plain FP64 C, OpenMP over nodes) on a bounded sample of the
    same workload: D3Q27 Taylor-Green at 64^3, tau = 0.5005, steps chosen so the
    run takes about budget_s seconds."""
    import oracle
    from paper_2303_08163_amd import workloads
    threads = oracle.set_threads(cpu_threads())
    n = 64
    rho0, u0 = workloads.taylor_green_3d(n, u0=0.05)
    oracle.run(rho0, u0, 0.5005, 1)  # warm up threads and pages
    t0 = time.perf_counter()
    oracle.run(rho0, u0, 0.5005, 8)
    per_step = (time.perf_counter() - t0) / 8
    steps = int(max(8, min(20000, budget_s / max(per_step, 1e-6))))
    t0 = time.perf_counter()
    oracle.run(rho0, u0, 0.5005, steps)
    dt = time.perf_counter() - t0
    return {"value": round(n ** 3 * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"D3Q27 64^3 Taylor-Green, FP64, {steps} steps, {dt:.1f} s, {threads} OpenMP threads"}


def bench_batched(count: int, steps: int, dtypes=("fp32_dev", "fp64"), baseline: bool = True,
                  fixed_tuning: dict | None = None, other_forms: bool = True) -> dict:
    """Batched workload: `count` independent D2Q9 shear-wave domains (Nx, Ny
    uniform in 32..512, amplitude U[0.01, 0.2], nu log-uniform 1e-5..1e-1),
    `steps` steps each, all advanced together by one pool kernel launch per
    step (tile shape from the autotuner), against the plain path: one domain
    at a time, one kernel launch per step (count * steps launches)."""
    import torch

    from paper_2303_08163_amd import autotune, lbm, workloads
    specs = workloads.batch_domains(count=count, seed=2303)
    nodes = sum(sp["nx"] * sp["ny"] for sp in specs)
    fields = [workloads.shear_wave(sp["nx"], sp["ny"], sp["amp"]) for sp in specs]
    out = {"workload": f"{count} D2Q9 periodic shear-wave domains, Nx,Ny ~ U{{32..512}}, {steps} steps each",
           "nodes": nodes}
    for dtype in dtypes:
        doms = [(9, (sp["nx"], sp["ny"]), dtype) for sp in specs]
        if fixed_tuning is not None:
            tuning, rep = dict(fixed_tuning), {"cached": False, "fixed": True}
        else:
            tuning, rep = autotune.tune_pool(doms, steps=100)
        def timed_pool(tuning):
            tun = lbm.make_pool_tuning(**tuning)
            arena = lbm.lbm_pool_table_bytes(count) + sum(
                lbm.lbm_pool_slot_bytes(lbm.make_config(9, (sp["nx"], sp["ny"]), sp["tau"], dtype), tun)
                for sp in specs)
            with lbm.Pool(arena + (1 << 20), max_slots=count, tuning=tun) as pool:
                for sp, (r0, u0) in zip(specs, fields):
                    pool.admit(r0, u0, sp["tau"], steps, dtype=dtype)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                pool.run(steps)
                done = pool.poll()
                dt = time.perf_counter() - t0
                st = pool.stats()
            assert len(done) == count
            return dt, st

        dt, st = timed_pool(tuning)
        rec = {"solves_per_s": round(count / dt, 2), "seconds": round(dt, 4), "mlups": round(nodes * steps / dt / 1e6, 1),
               "tuning": tuning, "launches": st["launches"], "autotune_cached": rep.get("cached", False),
               "autotune_fastest": (rep.get("times") or [])[:4], "autotune_failed": rep.get("failed", [])}
        if tuning.get("time_block", 0) == 2 and other_forms:
            # the other launch forms of the same pool: one step per launch (what batching
            # alone gives), the same as one persistent launch per run with a grid barrier
            # between steps, and two steps per launch with the other persistent setting
            # (one launch per two steps, or one tile-ordered launch per run)
            one = dict(tuning, time_block=0, persistent=0)
            one.pop("time_rows", None)
            other = dict(tuning, persistent=0 if tuning.get("persistent") else 1)
            for key, tun in (("pool_one_step_per_launch", one), ("pool_one_step_grid_barrier", dict(one, persistent=1)),
                             ("pool_two_step_launches" if other["persistent"] == 0 else "pool_tile_ordered", other)):
                d1, st1 = timed_pool(tun)
                rec[key] = {"solves_per_s": round(count / d1, 2), "seconds": round(d1, 4),
                            "launches": st1["launches"], "tuning": tun}
        if baseline and dtype == dtypes[0]:
            doms_alone = [lbm.Domain(r0, u0, sp["tau"], dtype=dtype) for sp, (r0, u0) in zip(specs, fields)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for d in doms_alone:
                d.step(steps)
            torch.cuda.synchronize()
            tb = time.perf_counter() - t0
            for d in doms_alone:
                d.close()
            rec["one_domain_per_launch"] = {"solves_per_s": round(count / tb, 2), "seconds": round(tb, 3),
                                            "launches": count * steps, "mlups": round(nodes * steps / tb / 1e6, 1)}
            rec["speedup_vs_one_domain_per_launch"] = round(tb / dt, 2)
            if "pool_one_step_per_launch" in rec:
                rec["pool_one_step_per_launch"]["speedup_vs_one_domain_per_launch"] = round(
                    tb / rec["pool_one_step_per_launch"]["seconds"], 2)
        out[dtype] = rec
    return out


SERVE_TUNINGS = {"default": None, "64x4": dict(tile_x=64, tile_y=4, time_block=2),
                 "fit": dict(tile_x=64, tile_y=4, row_fit=1, time_block=2)}


def bench_serving(n_requests: int, rate: float, light_requests: int, policies=("swf",),
                  saturate_bytes: float = 512e6, tuning: str = "default") -> dict:
    """Serving: Poisson request stream (seed 8163) mixing D2Q9 64^2..1024^2 and
    D3Q27 32^3..192^3 (log-uniform sides), Taylor-Green or shear-wave starts,
    u0 ~ U[0.01, 0.15], tau ~ U[0.5001, 0.6], 200..5000 steps, FP32 storage;
    continuous batching on one pool (pipelined: the next chunk is enqueued
    before the server waits for the current one) against a serial
    one-request-at-a-time server on the same GPU.  The stated rate is far above
    one GPU's capacity, so latency there is queueing; a second, lighter stream
    at about half the measured capacity is reported as well.  gpu_busy_frac is
    the GPU time of the pool's runs over the makespan."""
    from paper_2303_08163_amd import serve, workloads
    res = {}
    trace = workloads.serving_trace(n_requests=n_requests, rate=rate, seed=8163)

    def pooled(tr, policy):
        from paper_2303_08163_amd import lbm
        tk = SERVE_TUNINGS[tuning]
        be = serve.PoolBackend(96 << 30, max_slots=512, tuning=None if tk is None else lbm.make_pool_tuning(**tk))
        try:
            kw = {"policy": "swf", "lookahead": 1 << 30, "saturate_bytes": saturate_bytes} if policy == "swf" \
                else {"policy": "fifo", "lookahead": 8}
            recs = serve.Server(be, **kw).serve(tr)
            out = serve.summarize(recs)
            busy = be.gpu_busy_seconds()
            out["gpu_busy_s"] = round(busy, 3)
            out["gpu_busy_frac"] = round(busy / out["makespan_s"], 4) if out["makespan_s"] else None
            out["launches"] = int(be.pool.stats()["launches"])
        finally:
            be.close()
        progress(f"serving {len(tr)} requests, continuous batching {policy}: {out}")
        return out

    def serial(tr):
        out = serve.summarize(serve.serial_serve(tr))
        progress(f"serving {len(tr)} requests, serial: {out}")
        return out

    names = {"swf": "continuous_batching_shortest_work_first", "fifo": "continuous_batching_fifo"}
    stated = {"rate_req_s": rate, "requests": n_requests}
    for pol in policies:
        stated[names[pol]] = pooled(trace, pol)
    stated["serial"] = serial(trace)
    first = stated[names[policies[0]]]
    stated["solves_per_s_vs_serial"] = round(first["solves_per_s"] / stated["serial"]["solves_per_s"], 3)
    res["stated_rate"] = stated
    cap = first["solves_per_s"] or 1.0
    light_rate = max(0.5, 0.5 * cap)
    trace_l = workloads.serving_trace(n_requests=light_requests, rate=light_rate, seed=8164)
    light = {"rate_req_s": round(light_rate, 2), "requests": light_requests}
    for pol in policies:
        light[names[pol]] = pooled(trace_l, pol)
    light["serial"] = serial(trace_l)
    res["half_capacity_rate"] = light
    return res


def bench_slab(steps: int = 200, nz: int = 32, n: int = 256) -> dict:
    """One GPU's share of the headline domain split along z over 8 GPUs: an
    n x n x nz FP32 slab of the n^3 Taylor-Green field with halo planes, its
    own neighbour on both sides (pack both faces, unpack both faces after
    every step; between GPUs the two packed buffers would travel over xGMI).
    HIP events on the slab's stream split each step into the stream-collide
    kernel and the two halo launches (pack both faces, unpack both);
    nothing is skipped.  Then the same slab with the exchange fused into the
    step kernel (lbm_step_halo: one launch per step, which reads the entering
    populations from the packed buffers and writes the leaving ones)."""
    import torch

    from paper_2303_08163_amd import lbm, workloads

    rho0, u0 = workloads.taylor_green_3d(n, u0=0.05, planes=(0, nz))
    with lbm.Domain(rho0, u0, 0.5005, dtype="fp32_dev", z_halo=True) as s:
        nb = s.halo_bytes()
        lo = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
        hi = torch.empty(nb, dtype=torch.uint8, device="cuda:0")

        def exchange():
            s.halo_pack(lo, hi)
            s.halo_unpack(hi, lo)

        exchange()
        for _ in range(20):
            s.step(1)
            exchange()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        s.stream.synchronize()
        t0 = time.perf_counter()
        for e in ev:
            e[0].record(s.stream)
            s.step(1)
            e[1].record(s.stream)
            exchange()
            e[2].record(s.stream)
        s.stream.synchronize()
        wall = time.perf_counter() - t0
        k_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / steps
        x_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / steps
        diag = s.moments(fields=False)[2]
        # the same slab with the exchange fused into the step (lbm_step_halo):
        # two sets of send buffers alternate, each step reads the other set
        bufs = [[torch.empty(nb, dtype=torch.uint8, device="cuda:0") for _ in range(2)] for _ in range(2)]
        s.halo_pack(bufs[1][0], bufs[1][1])
        for t in range(20):
            p = t % 2
            s.step_halo(bufs[1 - p][1], bufs[1 - p][0], bufs[p][0], bufs[p][1])
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.stream.synchronize()
        f0.record(s.stream)
        for t in range(steps):
            p = t % 2
            s.step_halo(bufs[1 - p][1], bufs[1 - p][0], bufs[p][0], bufs[p][1])
        f1.record(s.stream)
        s.stream.synchronize()
        fused_ms = f0.elapsed_time(f1) / steps
    nodes = n * n * nz
    return {"workload": f"D3Q27 {n}x{n}x{nz} z-slab of the {n}^3 Taylor-Green field (u0 = 0.05, tau = 0.5005), "
                        "FP32 deviations, halo planes exchanged with itself after every step",
            "steps": steps, "ms_per_step": round(k_ms + x_ms, 5), "stream_collide_ms": round(k_ms, 5),
            "halo_exchange_ms": round(x_ms, 5),
            "mlups": round(nodes / ((k_ms + x_ms) * 1e-3) / 1e6, 1),
            "stream_collide_gbs": round(nodes * 216 / (k_ms * 1e-3) / 1e9, 1),
            "stream_collide_frac_of_8tbs": round(nodes * 216 / (k_ms * 1e-3) / 8e12, 4),
            "halo_bytes_per_face": nb, "wall_s": round(wall, 4), "mass": diag["mass"],
            "fused_exchange": {"ms_per_step": round(fused_ms, 5), "mlups": round(nodes / (fused_ms * 1e-3) / 1e6, 1),
                               "frac_of_8tbs": round(nodes * 216 / (fused_ms * 1e-3) / 8e12, 4)}}


def bench_wave(steps: int = 2000) -> dict:
    """Isothermal pressure-wave sweep: effective viscosity vs U0 for the
    entropic and product-form equilibria, with and without the bulk correction
    (D1Q3, nx = 64, tau = 0.65, drho = 1e-3, FP64, energy every 10 steps, fit
    over t >= 200)."""
    import torch

    from paper_2303_08163_amd import wave

    U0s = [round(-0.3 + 0.05 * k, 2) for k in range(13)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rows = wave.sweep(U0s, nx=64, tau=0.65, drho=1e-3, steps=steps, every=10, t_min=200)
    wall = time.perf_counter() - t0
    table = {}
    for r in rows:
        key = f"{r['equilibrium']}_{'corrected' if r['bulk_correction'] else 'plain'}"
        table.setdefault(key, []).append(round(r["normalised"], 5))
    return {"workload": "D1Q3 pressure wave rho = 1 + 1e-3 sin(2 pi x / 64) at uniform U0, tau = 0.65, "
                        f"{steps} steps, nu_eff from the decay of the acoustic energy",
            "U0": sorted(set(U0s) | {0.0}), "nu_eff_over_nu_eff_at_rest": table,
            "nu_eff_over_nu_at_rest": round(next(r["ratio"] for r in rows if r["U0"] == 0.0), 5),
            "runs": len(rows), "wall_s": round(wall, 3)}


def progress(msg: str) -> None:
    """A progress line on stderr (the JSON result line goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_cpu() -> dict:
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(), "threads_used": cpu_threads()}


def bench_oracle_timing(budget_s: float = 6.0) -> dict:
    """The oracle on the host, one thread and all threads, on bounded samples of
    C1 (full), C2 (full grid, a few steps), C3 at 64^3 and four C4 domains."""
    import oracle
    from paper_2303_08163_amd import workloads

    cases = [("C1 D2Q9 64^2 Taylor-Green, tau 0.51", workloads.taylor_green_2d(64, u0=0.05), 0.51),
             ("C2 D2Q9 4096^2 double shear, tau 0.5001", workloads.double_shear_layer(4096), 0.5001),
             ("C3 D3Q27 64^3 Taylor-Green, tau 0.5005", workloads.taylor_green_3d(64, u0=0.05), 0.5005)]
    for sp in workloads.batch_domains(512, 2303)[:4]:
        cases.append((f"C4 D2Q9 {sp['nx']}x{sp['ny']} shear wave, tau {sp['tau']:.4f}",
                      workloads.shear_wave(sp["nx"], sp["ny"], sp["amp"]), sp["tau"]))
    out = {"host": host_cpu(), "runs": []}
    for threads in (1, cpu_threads()):
        oracle.set_threads(threads)
        for name, (r0, u0), tau in cases:
            for corr in ("off", "min"):
                n = r0.size
                t0 = time.perf_counter()
                oracle.run(r0, u0, tau, 1, corr=corr)
                one = max(time.perf_counter() - t0, 1e-6)
                steps = max(1, min(2000, int(budget_s / one)))
                t0 = time.perf_counter()
                oracle.run(r0, u0, tau, steps, corr=corr)
                dt = time.perf_counter() - t0
                out["runs"].append({"case": name, "correction": corr, "threads": threads, "steps": steps,
                                    "seconds": round(dt, 2), "mlups": round(n * steps / dt / 1e6, 2)})
    return out


def bench_variants(steps: int = 100, warmup: int = 10) -> dict:
    """Throughput of the other equilibria and of the correction on the headline
    grid (D3Q27 256^3 Taylor-Green, FP32 deviation storage, default vector
    kernel)."""
    import torch

    from paper_2303_08163_amd import lbm, workloads

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    out = {}

    def timed(dom, nodes, bytes_per_lup, steps=steps, warmup=warmup):
        dom.step(warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        dom.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3
        _, _, d = dom.moments(fields=False)
        mlups = nodes * steps / sec / 1e6
        return {"mlups": round(mlups, 1), "gbs": round(mlups * 1e6 * bytes_per_lup / 1e9, 1),
                "frac": round(mlups * 1e6 * bytes_per_lup / 1e9 / HBM_PEAK_GBS, 4), "domain_error": d["domain_error"]}

    rho0, u0 = workloads.taylor_green_3d(256, u0=0.05)
    rd = torch.from_numpy(rho0).to(dev)
    ud = torch.from_numpy(u0).to(dev)
    del rho0, u0
    for eq in ("entropic", "poly2", "product"):
        for corr in (False, True):
            dom = lbm.Domain(rd, ud, 0.5005, dtype="fp32_dev", bulk_correction=corr, equilibrium=eq, stream=stream)
            out[f"d3q27_256_fp32_{eq}{'_corrected' if corr else ''}"] = timed(dom, 256 ** 3, 216)
            dom.close()
    # full FP64 storage of the headline workload (432 B per node update)
    for corr in (False, True):
        dom = lbm.Domain(rd, ud, 0.5005, dtype="fp64", bulk_correction=corr, stream=stream)
        rec = timed(dom, 256 ** 3, 432)
        rec["kernel"] = dom.launch_info()
        out[f"d3q27_256_fp64_entropic{'_corrected' if corr else ''}"] = rec
        dom.close()
    del rd, ud
    return {"steps": steps, "results": out}


def bench_ceiling(n: int = 256, steps: int = 100, warmup: int = 10) -> dict:
    """The access pattern's own speed, measured in the library: a non-temporal
    float4 copy of 2 GiB (read + write bytes), and free streaming (the
    stream-collide kernel's launch, loads and stores without the collision) of
    the D3Q27 n^3 domain with FP32 deviation storage (216 B per node) and
    FP64 storage (432 B per node)."""
    import torch

    from paper_2303_08163_amd import lbm, workloads

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    nb = 2 << 30
    x = torch.empty(nb // 4, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    lbm.lbm_ceiling_copy(x.data_ptr(), y.data_ptr(), nb, stream.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = []
    for _ in range(3):
        e0.record(stream)
        for _ in range(10):
            lbm.lbm_ceiling_copy(x.data_ptr(), y.data_ptr(), nb, stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        reps.append(2 * nb * 10 / (e0.elapsed_time(e1) / 1e3) / 1e9)
    del x, y
    out = {"copy_nt_gbs": round(max(reps), 1), "copy_nt_gbs_reps": [round(v, 1) for v in reps],
           "copy_bytes": nb}
    rho0, u0 = workloads.taylor_green_3d(n, u0=0.05)
    rd = torch.from_numpy(rho0).to(dev)
    ud = torch.from_numpy(u0).to(dev)
    del rho0, u0
    for dt, b in (("fp32_dev", 216), ("fp64", 432)):
        dom = lbm.Domain(rd, ud, 0.5005, dtype=dt, stream=stream)
        lbm.lbm_ceiling_stream(dom.handle, warmup)
        torch.cuda.synchronize()
        reps = []
        for _ in range(3):
            e0.record(stream)
            lbm.lbm_ceiling_stream(dom.handle, steps)
            e1.record(stream)
            torch.cuda.synchronize()
            reps.append(b * n ** 3 * steps / (e0.elapsed_time(e1) / 1e3) / 1e9)
        kind = dom.launch_info()
        dom.close()
        out[f"free_streaming_d3q27_{dt}_gbs"] = round(max(reps), 1)
        out[f"free_streaming_d3q27_{dt}_gbs_reps"] = [round(v, 1) for v in reps]
        out[f"free_streaming_d3q27_{dt}_kernel"] = {k: kind[k] for k in ("kernel", "nodes_per_thread", "row_wave")}
    return out


def bench_d1q3(steps: int = 200, warmup: int = 64) -> dict:
    """A D1Q3 row of 2^27 nodes (a pressure wave, U = 0.1, tau 0.6, with the
    correction), FP32 deviations and FP64, with the default eight steps per
    launch and with one; more steps than elsewhere (one step takes ~0.6 ms,
    50 steps read up to 7 % low)."""
    import numpy as np
    import torch

    from paper_2303_08163_amd import lbm

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    out = {}

    def timed(dom, nodes, bytes_per_lup):
        k = dom.launch_info()["time_block"]
        dom.step(warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        dom.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3
        _, _, d = dom.moments(fields=False)
        mlups = nodes * steps / sec / 1e6
        own = bytes_per_lup * nodes / (k * sec / steps) / 1e9  # one read + one write per launch
        return {"mlups": round(mlups, 1), "us_per_step": round(sec / steps * 1e6, 2), "steps_per_launch": k,
                "gbs": round(own, 1), "frac": round(own / HBM_PEAK_GBS, 4),
                "gbs_2Qs_per_update": round(mlups * 1e6 * bytes_per_lup / 1e9, 1), "domain_error": d["domain_error"],
                "launch_s": k * sec / steps}

    n1 = 1 << 27
    x = np.arange(n1, dtype=np.float64)
    r1 = torch.from_numpy(1.0 + 1e-3 * np.sin(2 * math.pi * x / n1)).to(dev)
    u1 = torch.full((1, n1), 0.1, dtype=torch.float64, device=dev)
    del x
    # the default (eight steps per launch) and one step per launch; gbs / frac count
    # the bytes a launch moves (2 Q s per node), gbs_2Qs_per_update the equivalent
    # rate at 2 Q s per node update
    for dt, s in (("fp32_dev", 4), ("fp64", 8)):
        for name, tun in (("eight_steps_per_launch", None), ("one_step_per_launch", lbm.make_tuning(time_block=1))):
            dom = lbm.Domain(r1, u1, 0.6, dtype=dt, bulk_correction=True, stream=stream, tuning=tun)
            rec = timed(dom, n1, 2 * 3 * s)
            launch_s = rec.pop("launch_s")
            if rec["steps_per_launch"] > 1:
                rec["roofline_valu"] = valu_roofline(f"d1q3_2e27.{dt}_{name}", launch_s)
            out[f"{dt}_{name}"] = rec
            dom.close()
    return {"workload": "D1Q3 2^27 nodes, pressure wave rho = 1 + 1e-3 sin(2 pi x / N), U = 0.1, tau 0.6, "
                        "bulk correction on", "steps": steps, "results": out}


def bench_d2q9(steps: int = 100, warmup: int = 200) -> dict:
    """The D2Q9 4096^2 double shear layer (tau 0.5001), FP32 deviations and FP64,
    correction off and on, with the default two steps per launch and with one.
    gbs / frac count the bytes each launch moves by algorithm: one read and
    one write of every population per launch (2 Q s per node per launch, so
    Q s per node update with two steps per launch); gbs_2Qs_per_update is the
    rate at 2 Q s per node update, an equivalent figure for the two-step
    kernel, not bytes it moves."""
    import torch

    from paper_2303_08163_amd import lbm, workloads

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    r2, u2 = workloads.double_shear_layer(4096)
    out = {}
    for corr in (False, True):
        for dt, s in (("fp32_dev", 4), ("fp64", 8)):
            for name, tun in (("two_steps_per_launch", None), ("one_step_per_launch", lbm.make_tuning(time_block=1))):
                dom = lbm.Domain(r2, u2, 0.5001, dtype=dt, bulk_correction=corr, stream=stream, tuning=tun)
                info = dom.launch_info()
                dom.step(warmup)
                torch.cuda.synchronize()
                reps = []
                for _ in range(3):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    dom.step(steps)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    reps.append(e0.elapsed_time(e1) / 1e3 / steps)
                _, _, d = dom.moments(fields=False)
                dom.close()
                sec = min(reps)
                mlups = 4096 ** 2 / sec / 1e6
                k = info["time_block"]
                own = 2 * 9 * s * 4096 ** 2 / (k * sec) / 1e9  # bytes of one launch / its time
                key = f"{dt}_{name}{'_corrected' if corr else ''}"
                out[key] = {
                    "mlups": round(mlups, 1), "us_per_step": round(sec * 1e6, 1),
                    "us_per_step_reps": [round(v * 1e6, 1) for v in reps], "steps_per_launch": k,
                    "kernel": info["kernel"], "gbs": round(own, 1), "frac": round(own / HBM_PEAK_GBS, 4),
                    "gbs_2Qs_per_update": round(mlups * 1e6 * 2 * 9 * s / 1e9, 1), "domain_error": d["domain_error"]}
                if k > 1:
                    out[key]["roofline_valu"] = valu_roofline(f"d2q9_4096.{key}", k * sec)
    return {"workload": "D2Q9 4096^2 double shear layer, tau 0.5001", "steps": steps, "warmup_steps": warmup,
            "repetitions": 3, "statistic": "best of the repetitions", "results": out}


FP64_VECTOR_PEAK_TFLOPS = 78.6


def bench_stability(cpu_budget_s: float = 5.0, with_cpu: bool = True) -> dict:
    """Linear-stability domains of the three equilibria over the paper's 15
    viscosities and 19 directions (D2Q9, k grid 33 x 33 on [0, pi]^2, 24
    bisection steps), and the eigensolver kernel's FP64 rate."""
    import numpy as np
    import torch

    from paper_2303_08163_amd import vonneumann as vn

    thetas = [math.radians(5 * a) for a in range(19)]
    out = {"workload": "D2Q9 von Neumann stability domains: 15 nu x 19 theta x 3 equilibria, "
                       "k grid 33^2 on [0, pi]^2, 24 bisection steps run in lockstep for the three "
                       "equilibria (one host wait per step), FP64"}
    table = {}
    total_m = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for eq, (umax, st) in vn.stability_domains(vn.PAPER_NUS, thetas, ("entropic", "poly2", "product"), nk=33,
                                               iters=24).items():
        total_m += st["matrices"]
        table[eq] = {"u_max_theta0": [round(float(v), 5) for v in umax[:, 0]],
                     "u_max_theta45": [round(float(v), 5) for v in umax[:, 9]],
                     "unconverged": st["unconverged"]}
    wall = time.perf_counter() - t0
    out.update({"nu": vn.PAPER_NUS, "domains": table, "matrices": total_m, "wall_s": round(wall, 3),
                "matrices_per_s": round(total_m / wall, 1)})

    # kernel rate: one launch of the spectra kernel over 2^20 cases drawn like the sweep's
    rng = np.random.default_rng(5)
    n = 1 << 20
    nus = np.exp(rng.uniform(math.log(1e-6), math.log(1.2), n))
    sp, th = rng.uniform(0, 0.95, n), rng.uniform(0, math.pi / 2, n)
    cases = np.stack([0.5 + 3 * nus, sp * np.cos(th), sp * np.sin(th), rng.uniform(0, math.pi, n),
                      rng.uniform(0, math.pi, n)], axis=1)
    dev = torch.device("cuda:0")
    c = torch.from_numpy(cases).to(dev)
    radius = torch.empty(n, dtype=torch.float64, device=dev)
    info = torch.empty(n, dtype=torch.int32, device=dev)
    work = torch.empty(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    from paper_2303_08163_amd import lbm
    call = lambda: lbm.lbm_vn_spectra(lbm.LBM_D2Q9, "product", False, c.data_ptr(), n, radius.data_ptr(), None,
                                      info.data_ptr(), work.data_ptr(), stream.cuda_stream)
    call()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record(stream)
    for _ in range(reps):
        call()
    e1.record(stream)
    torch.cuda.synchronize()
    per_launch = e0.elapsed_time(e1) / 1e3 / reps
    steps = info.cpu().numpy().astype(np.int64)
    # FP64 operations of the solver as written, counted by the kernel per case:
    # its own active block at every QR step (a fused multiply-add counts 2)
    flops = int(work.sum().item())
    achieved = flops / per_launch / 1e12
    out["kernel"] = {"kernel": "k_vn_spectra<D2Q9, product form, no correction>", "cases": n,
                     "launch_avg_ms": round(per_launch * 1e3, 4), "matrices_per_s": round(n / per_launch, 1),
                     "qr_steps_mean": round(float(steps.mean()), 2), "unconverged": int((steps < 0).sum()),
                     "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                                  "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                                  "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 4), "traffic": None,
                                  "flops_per_launch": flops}}
    if with_cpu:
        from oracle import stability as ost
        ks = ost.k_grid(33)
        t0 = time.perf_counter()
        m = 0
        while time.perf_counter() - t0 < cpu_budget_s:
            ost.batch_spectral_radius(0.5 + 3 * 1e-3, [0.3, 0.2], ks, kind="product")
            m += len(ks)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(m / dt, 1), "unit": "matrices/s", "cores": 1, "kind": "oracle",
                               "sample": f"{m} D2Q9 amplification matrices (oracle Jacobian + LAPACK "
                                         f"eigenvalues), {dt:.1f} s"}
    return out


def env_info() -> dict:
    """ROCm version and the GPU's clocks as rocm-smi reports them, read in a
    child process before this process touches the GPU (rocm-smi reads the
    driver's sysfs files; a failure is recorded, not raised).  Under rocprofv3
    the clocks are not read: its preloaded library initialises the GPU in every
    process it starts, and rocm-smi re-executes itself through its interpreter."""
    import subprocess
    env = {}
    try:
        with open("/opt/rocm/.info/version") as f:
            env["rocm"] = f.read().strip()
    except OSError:
        env["rocm"] = None
    if any(k.startswith("ROCPROF_") for k in os.environ) or "rocprof" in os.environ.get("LD_PRELOAD", ""):
        env["rocm_smi_clocks_at_start"] = "not read under rocprofv3"
        return env
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True, timeout=30)
        data = json.loads(r.stdout) if r.returncode == 0 else None
        if isinstance(data, dict):
            env["rocm_smi_clocks_at_start"] = {card: {k: v for k, v in vals.items() if "clock" in k.lower()}
                                               for card, vals in data.items() if isinstance(vals, dict)}
        else:
            env["rocm_smi_clocks_at_start"] = f"unavailable (exit {r.returncode}): {(r.stderr or r.stdout)[-200:]}"
    except (OSError, ValueError, subprocess.SubprocessError) as err:
        env["rocm_smi_clocks_at_start"] = f"unavailable: {err}"
    return env


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="grid side (headline: 256)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sections", default="headline,ceiling,batched,serving,wave,stability,variants,slab,d2q9,d1q3",
                    help="comma list of headline, ceiling, batched, serving, wave, stability, variants, slab, d2q9, "
                         "d1q3, oracle_timing (not in the default run: several minutes of host time)")
    ap.add_argument("--d2q9-steps", type=int, default=100, help="timed steps per repetition of the d2q9 section")
    ap.add_argument("--d1q3-steps", type=int, default=200, help="timed steps of the d1q3 section")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--no-batch-baseline", action="store_true",
                    help="skip the one-domain-per-launch baseline of the batched section")
    ap.add_argument("--no-batch-forms", action="store_true",
                    help="batched: time the chosen tuning only, not the pool's other launch forms")
    ap.add_argument("--batch-tuning", default="",
                    help="TXxTY[,persistent][,flat][,fit][,t2]: fixed pool tile instead of the autotuner's "
                         "choice (t2: two steps per launch)")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-light-requests", type=int, default=40)
    ap.add_argument("--serve-policies", default="swf", help="comma list of swf, fifo (continuous batching policies)")
    ap.add_argument("--serve-saturate", type=float, default=512e6,
                    help="swf: per-step HBM bytes of the running requests at which admission pauses")
    ap.add_argument("--serve-tuning", default="default", choices=sorted(SERVE_TUNINGS),
                    help="pool tuning of the continuous-batching server (default: the backend's own)")
    args = ap.parse_args()
    sections = set(args.sections.split(","))
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: every workload runs on a single GPU (z-slabs "
              "with halo exchange model one GPU's share; the transfer between GPUs is not built).",
              file=sys.stderr)
        return 2

    env = env_info()  # before anything initialises the GPU

    import numpy as np
    import torch

    from paper_2303_08163_amd import lbm, workloads

    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(0)
    env.update(device=torch.cuda.get_device_name(0), arch=getattr(props, "gcnArchName", None),
               compute_units=props.multi_processor_count, hip=torch.version.hip, torch=torch.__version__)
    n, tau = args.n, 0.5005
    rho0, u0 = workloads.taylor_green_3d(n, u0=0.05)
    stream = torch.cuda.current_stream(dev)
    dom = lbm.Domain(rho0, u0, tau, dtype="fp32_dev", bulk_correction=False, stream=stream)
    launch = dom.launch_info()
    del rho0, u0
    nodes = n ** 3
    dom.step(args.warmup)
    torch.cuda.synchronize()

    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record(stream)
    dom.step(args.steps)
    stop.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = start.elapsed_time(stop)
    # four more repetitions of the same K steps (median of five reported beside)
    reps = [ms / args.steps]
    for _ in range(4):
        start.record(stream)
        dom.step(args.steps)
        stop.record(stream)
        torch.cuda.synchronize()
        reps.append(start.elapsed_time(stop) / args.steps)
    _, _, diag = dom.moments(fields=False)
    dom.close()

    sec = ms / 1e3
    mlups = nodes * args.steps / sec / 1e6
    bytes_per_lup = 2 * 27 * 4
    per_launch_s = sec / args.steps
    achieved = bytes_per_lup * nodes / per_launch_s / 1e9
    traffic = measured_traffic()

    ceiling = bench_ceiling(n) if "ceiling" in sections else None
    if ceiling:
        progress("ceiling done")

    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"D3Q27 entropic-equilibrium BGK, {n}^3 periodic Taylor-Green u0=0.05, tau=0.5005, "
                        "FP32 storage of f_i - w_i rho0 with FP64 arithmetic, bulk correction off",
            "lattice": "D3Q27", "grid": [n, n, n], "storage": "f32 deviations", "arithmetic": "f64",
            "bulk_correction": False, "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": f"k_stream_collide_vec<D3Q27, FP32 deviations/FP64 arithmetic, no correction, "
                      f"{launch['nodes_per_thread']} nodes per thread, row wave {launch['row_wave']}, "
                      f"row-interleaved layout>",
            "bytes_per_node_update": bytes_per_lup,
            "launch_avg_ms": round(per_launch_s * 1e3, 5),
        },
        "launch": launch,
        "wall_s_timed_region": round(t_wall, 4),
        "repetitions_ms_per_step": [round(v, 5) for v in reps],
        "median_of_5_mlups": round(nodes / (sorted(reps)[2] / 1e3) / 1e6, 1),
        "mass_drift": abs(diag["mass"] / (nodes * 1.0) - 1.0),
        "kernel_source_digest": kernel_source_digest(),
        "env": env,
    }
    if ceiling:
        out["ceiling"] = ceiling
        out["frac_of_free_streaming"] = round(achieved / ceiling["free_streaming_d3q27_fp32_dev_gbs"], 4)
        out["frac_of_copy_nt"] = round(achieved / ceiling["copy_nt_gbs"], 4)
    if "batched" in sections:
        fixed = None
        if args.batch_tuning:
            parts = args.batch_tuning.split(",")
            tx, ty = (int(v) for v in parts[0].lower().split("x"))
            fixed = {"tile_x": tx, "tile_y": ty, "persistent": int("persistent" in parts[1:])}
            if "flat" in parts[1:]:
                fixed["flat"] = 1
            if "fit" in parts[1:]:
                fixed["row_fit"] = 1
            if "t2" in parts[1:]:
                fixed["time_block"] = 2
        out["batched"] = bench_batched(args.batch_count, args.batch_steps, baseline=not args.no_batch_baseline,
                                       fixed_tuning=fixed, other_forms=not args.no_batch_forms)
        progress("batched done")
    if "serving" in sections:
        out["serving"] = bench_serving(args.serve_requests, args.serve_rate, args.serve_light_requests,
                                       tuple(args.serve_policies.split(",")), args.serve_saturate,
                                       args.serve_tuning)
    if "wave" in sections:
        out["wave"] = bench_wave()
        progress("wave done")
    if "oracle_timing" in sections:
        out["oracle_timing"] = bench_oracle_timing()
        progress("oracle_timing done")
    if "variants" in sections:
        out["variants"] = bench_variants()
        progress("variants done")
    if "slab" in sections:
        out["slab"] = bench_slab()
        progress("slab done")
    if "d2q9" in sections:
        out["d2q9"] = bench_d2q9(steps=args.d2q9_steps)
        progress("d2q9 done")
    if "d1q3" in sections:
        out["d1q3"] = bench_d1q3(steps=args.d1q3_steps)
        progress("d1q3 done")
    if "stability" in sections:
        out["stability"] = bench_stability(with_cpu=not args.no_cpu_baseline)
        progress("stability done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
