"""The eigensolver of the von Neumann kernels (csrc/vn.hpp), run on the CPU:
tests/c/vn_host.hip includes the same header and applies it to one matrix at a
time (the lockstep group is the thread itself; the reciprocal square root
estimate is the host stand-in).  Its eigenvalues must match LAPACK's on the
oracle's amplification matrix within the bound of the GPU test: a
backward-stable solver moves an eigenvalue by at most kappa(V) |dM| with
|dM| ~ c eps |M|, here 1e-13 kappa(V) |M|_2.  This checks the solver's steps
(Householder reduction, rotations, deflation, shifts, the loop per active block
size) without a GPU; the wavefront-uniform block size and the device's own
estimate are covered by tests/test_gpu_vonneumann.py."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import stability as ost

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
KINDS = ["entropic", "poly2", "product"]


@pytest.fixture(scope="module")
def vn_host(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("vn") / "vn_host")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17", "-ffp-contract=off",
                        "-I" + os.path.join(ROOT, "include"),
                        "-I" + os.path.join(ROOT, "paper_2303_08163_amd", "csrc"),
                        os.path.join(ROOT, "tests", "c", "vn_host.hip"), "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _cases(D, n, seed):
    rng = np.random.default_rng(seed)
    tau = 0.5 + 3 * np.exp(rng.uniform(np.log(1e-6), np.log(1.2), n))
    if D == 1:
        ux, uy = rng.uniform(-0.95, 0.95, n), np.zeros(n)
    else:
        sp, th = rng.uniform(0, 0.95, n), rng.uniform(0, np.pi / 2, n)
        ux, uy = sp * np.cos(th), sp * np.sin(th)
    kx, ky = rng.uniform(0, np.pi, n), rng.uniform(0, np.pi, n)
    # special cases: k = 0 (one eigenvalue 1 per conserved moment), k = pi,
    # a tiny k, and tau = 1 (omega = 1: rank-deficient, several zero eigenvalues)
    kx[:5], ky[:5] = [0, np.pi, 1e-4, 0, np.pi], [0, np.pi, 0, 1e-4, 0]
    tau[5] = 1.0
    tau[6] = 1.0
    kx[6] = ky[6] = 0.0
    return np.stack([tau, ux, uy, kx, ky], axis=1)


def _run(exe, D, eq, corr, cases, tmp_path):
    inp, outp = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(inp, "wb") as f:
        f.write(np.int64(len(cases)).tobytes())
        f.write(np.ascontiguousarray(cases, dtype=np.float64).tobytes())
    subprocess.run([exe, str(D), str(eq), str(int(corr)), inp, outp], check=True)
    N = 3 if D == 1 else 9
    raw = open(outp, "rb").read()
    n = len(cases)
    e = np.frombuffer(raw[:16 * N * n], dtype=np.float64).reshape(n, N, 2)
    steps = np.frombuffer(raw[16 * N * n:], dtype=np.int32)
    return e[..., 0] + 1j * e[..., 1], steps


@pytest.mark.parametrize("D", [1, 2])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("corr", [False, True])
def test_host_eigensolver_matches_lapack(vn_host, tmp_path, D, kind, corr):
    cases = _cases(D, 120, seed=50 + 10 * D + KINDS.index(kind) + (5 if corr else 0))
    eig, steps = _run(vn_host, D, KINDS.index(kind), corr, cases, tmp_path)
    assert np.all(steps >= 0), "iteration limit reached"
    for t, row in enumerate(cases):
        M = ost.amplification_matrix(row[0], row[1:1 + D], row[3:3 + D], corr="min" if corr else "off", kind=kind)
        ref, V = np.linalg.eig(M)
        bound = 1e-13 * np.linalg.cond(V) * np.linalg.norm(M, 2) + 1e-300
        rem = list(ref)
        for z in eig[t]:
            j = int(np.argmin([abs(z - r) for r in rem]))
            assert abs(z - rem[j]) <= bound, (t, row, z, rem[j])
            rem.pop(j)
