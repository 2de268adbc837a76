"""The library called from plain C: tests/c/abi_demo.c (built by
__graft_entry__.build()) creates, steps and reads a D3Q27 domain, runs a pool
of two D2Q9 domains, checks argument errors, and compares a z-slab that is its
own neighbour with the periodic domain bitwise, all through include/lbm.h."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BIN = os.path.join(ROOT, "tests", "c", "abi_demo")


def test_c_abi_demo_runs():
    if not os.path.exists(BIN):
        pytest.fail("tests/c/abi_demo is not built; run __graft_entry__.build()")
    print("[c abi] running tests/c/abi_demo", flush=True)
    r = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    print(r.stdout, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "abi_demo ok" in r.stdout
