"""Autotuner for pool launch shapes.

For a set of domains (lattice, grid, storage), it times a short run of each
candidate pool tuning -- workgroup tile shape (one node per thread; rows of
tile_x nodes, rows fitted to each slot's width, or runs of consecutive nodes
across rows) and launch form (one launch per step or per two steps; two-step
classes also as one tile-ordered persistent launch per run; on request every
shape also as one grid-barrier persistent launch per run) -- on a scratch
pool holding domains
of exactly those sizes, and returns the fastest.  Results do not depend on
the tuning (the per-node arithmetic is the same in every kernel), so only
time is compared.  Choices are cached in a JSON file keyed by the candidate
set, device name, HIP runtime version and a coarse signature of the domain
sizes.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import time

import numpy as np

from . import lbm

TILES = [(64, 4), (64, 2), (64, 1), (32, 8), (32, 2), (128, 2), (128, 1), (256, 1), (16, 16), (16, 4)]
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "lbm_entropic", "autotune.json")


FLAT_TILES = [(64, 4), (64, 2), (64, 1)]  # flat mode: 256, 128 or 64 consecutive nodes per workgroup


def candidates(persistent: bool = False):
    """Tile shapes with one launch per step; with persistent, each also as one
    cooperative launch per run with a grid barrier between steps.  That form
    is left out by default: its grid barrier cost 200-260 us per step on
    MI355X (every workgroup polls one device-coherent counter and does an
    agent-scope release and acquire), against a few microseconds between
    back-to-back launches, and it was the slower form on every workload
    measured.  Two steps per launch come with three sweep lengths, and as one
    tile-ordered persistent launch per run (no grid barrier; the two-step
    classes only) with two."""
    forms = (0, 1) if persistent else (0,)
    rows = [dict(tile_x=tx, tile_y=ty, persistent=p) for (tx, ty) in TILES for p in forms]
    flat = [dict(tile_x=tx, tile_y=ty, persistent=p, flat=1) for (tx, ty) in FLAT_TILES for p in forms]
    fit = [dict(tile_x=64, tile_y=4, persistent=p, row_fit=1) for p in forms]
    # two steps per launch for large D2Q9 classes (the tile and row fit serve the
    # one-step launches of the other classes), with three sweep lengths
    two = [dict(tile_x=64, tile_y=4, persistent=0, row_fit=1, time_block=2, time_rows=r) for r in (0, 32, 64)]
    ordered = [dict(tile_x=64, tile_y=4, persistent=1, row_fit=1, time_block=2, time_rows=r) for r in (0, 32)]
    return rows + flat + fit + two + ordered


def signature(domains) -> str:
    """Coarse key of a domain set: lattice and storage mix plus a histogram of
    log2 extents (so that nearby size mixes share a tuning)."""
    hist = {}
    for lattice, shape, dtype in domains:
        key = (int(lattice), str(dtype)) + tuple(int(round(math.log2(max(1, s)) * 2)) for s in shape)
        hist[key] = hist.get(key, 0) + 1
    items = sorted((list(k), v) for k, v in hist.items())
    total = sum(hist.values())
    coarse = [[k, round(v / total, 2)] for k, v in items]
    return hashlib.sha256(json.dumps(coarse).encode()).hexdigest()[:16] + f"-n{int(round(math.log2(total)))}"


def _device_key() -> str:
    import torch
    name = torch.cuda.get_device_name(0)
    return f"{name}|hip {torch.version.hip}"


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(path, data):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def time_tuning(domains, tuning: dict, steps: int = 60, warmup: int = 10) -> float:
    """Seconds per step of one pool run over the domains (rest-state fields:
    the arithmetic per node is the same for any state).  Candidates a few per
    cent apart need runs of tens of launches to rank as they do over long
    runs: on the batched workload 10 steps ranked 32-row sweeps 1 % ahead of
    16, which 2000 steps put 2.6 % behind."""
    import torch
    t = lbm.make_pool_tuning(**tuning)
    need = lbm.lbm_pool_table_bytes(len(domains))
    for lattice, shape, dtype in domains:
        b = lbm.lbm_pool_slot_bytes(lbm.make_config(lattice, shape, 0.6, dtype), t)
        if b == 0:
            raise ValueError(f"tuning {tuning} rejected for {shape}")
        need += b
    with lbm.Pool(need + (1 << 20), max_slots=len(domains), tuning=t) as pool:
        for lattice, shape, dtype in domains:
            grid = tuple(shape[::-1])
            D = len(grid)
            pool.admit(np.ones(grid), np.zeros((D,) + grid), 0.6, warmup + steps, dtype=dtype)
        pool.run(warmup)
        pool.poll()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(pool.stream)
        pool.run(steps)
        e.record(pool.stream)
        pool.poll()
        return s.elapsed_time(e) / 1e3 / steps


def tune_pool(domains, steps: int = 60, cands=None, cache_path: str | None = DEFAULT_CACHE,
              use_cache: bool = True, verbose: bool = False):
    """domains: list of (lattice, (nx, ny[, nz]), dtype).  Returns (tuning dict,
    report) where report lists every candidate's time per step and, under
    "failed", each candidate that the library refused or that raised an error
    while it ran (for instance a persistent run whose grid barrier timed out),
    with the error text."""
    key = f"candidates-v9|{_device_key()}|{signature(domains)}" if cands is None else \
        f"custom-{hashlib.sha256(json.dumps(cands, sort_keys=True).encode()).hexdigest()[:12]}|{_device_key()}|" \
        f"{signature(domains)}"
    cache = _load_cache(cache_path) if cache_path else {}
    if use_cache and key in cache:
        return cache[key]["tuning"], {"cached": True, "key": key, "times": cache[key].get("times")}
    times, failed = [], []
    for c in (cands or candidates()):
        try:
            dt = time_tuning(domains, c, steps=steps)
        except (ValueError, lbm.LBMError) as err:
            failed.append([c, str(err)])
            if verbose:
                print(f"  autotune {c}: failed: {err}", flush=True)
            continue
        times.append((dt, c))
        if verbose:
            print(f"  autotune {c}: {dt * 1e3:.3f} ms/step", flush=True)
    if not times:
        raise RuntimeError("no tuning candidate ran")
    times.sort(key=lambda x: x[0])
    best = times[0][1]
    report = {"cached": False, "key": key, "times": [[round(t * 1e3, 4), c] for t, c in times], "failed": failed}
    if cache_path:
        cache[key] = {"tuning": best, "times": report["times"], "when": time.strftime("%Y-%m-%d %H:%M:%S")}
        _save_cache(cache_path, cache)
    return best, report
