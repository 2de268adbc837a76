"""Write the oracle's sampled results for the full-length parity cases.

Runs only the FP64 CPU oracle (oracle/) on the seeded inputs of
paper_2303_08163_amd.workloads and stores moments at seeded sample nodes:

  c2_double_shear_4096_1000.npz
      D2Q9 4096^2 double shear layer (width 80, u0 = 0.1, relative
      perturbation 0.05), tau = 0.5001, 1000 steps, bulk correction off and on
      (A = min over axes).  4096 nodes sampled uniformly (seed 4096).
  c4_subset_2000.npz
      The first 32 domains of the batched shear-wave workload (512 domains,
      seed 2303), 2000 steps each, correction off.  64 nodes per domain
      (seed 2000 + domain index).

Usage: python tests/golden/make_oracle_samples.py [c2] [c4] [--threads N]
(about 20 minutes for c2 and 3 minutes for c4 on 8 cores).
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2303_08163_amd import workloads  # noqa: E402

C2_FILE = os.path.join(HERE, "c2_double_shear_4096_1000.npz")
C4_FILE = os.path.join(HERE, "c4_subset_2000.npz")


def c2_points(n=4096, count=4096, seed=4096):
    rng = np.random.default_rng(seed)
    return rng.integers(0, n, size=count), rng.integers(0, n, size=count)  # x, y


def c4_points(nx, ny, k, count=64):
    rng = np.random.default_rng(2000 + k)
    return rng.integers(0, nx, size=count), rng.integers(0, ny, size=count)


def make_c2():
    n, tau, steps = 4096, 0.5001, 1000
    rho0, u0 = workloads.double_shear_layer(n)
    xs, ys = c2_points(n)
    out = dict(x=xs, y=ys, tau=tau, steps=steps)
    for corr in ("off", "min"):
        t = time.time()
        rho, u, bad = oracle.run(rho0, u0, tau, steps, corr=corr)
        print(f"c2 corr={corr}: {time.time() - t:.0f} s, out-of-domain {bad}", flush=True)
        out[f"rho_{corr}"] = rho[ys, xs]
        out[f"u_{corr}"] = u[:, ys, xs]
        out[f"bad_{corr}"] = bad
        del rho, u
    np.savez_compressed(C2_FILE, **out)


def make_c4(count=32, steps=2000):
    specs = workloads.batch_domains(count=512, seed=2303)[:count]
    out = dict(steps=steps, count=count)
    t = time.time()
    for k, sp in enumerate(specs):
        rho0, u0 = workloads.shear_wave(sp["nx"], sp["ny"], sp["amp"])
        rho, u, bad = oracle.run(rho0, u0, sp["tau"], steps)
        xs, ys = c4_points(sp["nx"], sp["ny"], k)
        out[f"x_{k}"], out[f"y_{k}"] = xs, ys
        out[f"rho_{k}"], out[f"u_{k}"] = rho[ys, xs], u[:, ys, xs]
        out[f"bad_{k}"] = bad
    print(f"c4: {time.time() - t:.0f} s", flush=True)
    np.savez_compressed(C4_FILE, **out)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="*", default=["c2", "c4"])
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    a = ap.parse_args()
    oracle.set_threads(a.threads)
    if "c4" in a.which:
        make_c4()
    if "c2" in a.which:
        make_c2()
