"""lbm_step replays a captured HIP graph of 32 launches for long runs (the
launch rate bounds small domains).  The graph holds the same kernels with the
same arguments, so every replay must give the bits of plain one-step calls;
checked over several replays, from both starting buffers, with moments
(eager work and synchronisation) between the calls, on the default stream
and on a side stream -- also for graphs of multi-step launches (two steps
on D2Q9, eight on D1Q3), against one-step calls."""
import numpy as np
import pytest

from paper_2303_08163_amd import workloads

pytestmark = pytest.mark.gpu


def _lbm():
    from paper_2303_08163_amd import lbm
    return lbm


CASES = [  # (fields, dtype, correction, time_block)
    (lambda: workloads.taylor_green_2d(64), "fp64", False, 0),
    (lambda: workloads.random_field((33, 70), seed=5, umax=0.1), "fp32_dev", True, 0),
    (lambda: workloads.random_field((7, 9, 13), seed=6, umax=0.1), "fp32_dev", False, 0),
    (lambda: workloads.random_field((256,), seed=7, umax=0.1), "fp64", True, 0),
    # graphs of multi-step launches: 16 two-step D2Q9 launches, 4 eight-step D1Q3 launches
    (lambda: workloads.random_field((40, 128), seed=8, umax=0.1), "fp32_dev", True, 2),
    (lambda: workloads.random_field((2048,), seed=9, umax=0.1), "fp64", True, 8),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("side_stream", [False, True])
def test_graph_replay_equals_plain_launches_bitwise(case, side_stream):
    import torch
    lbm = _lbm()
    make, dtype, corr, tblock = CASES[case]
    rho0, u0 = make()
    stream = torch.cuda.Stream() if side_stream else None
    tun = lbm.make_tuning(time_block=tblock) if tblock else None
    with lbm.Domain(rho0, u0, 0.58, dtype=dtype, bulk_correction=corr, stream=stream, tuning=tun) as a, \
            lbm.Domain(rho0, u0, 0.58, dtype=dtype, bulk_correction=corr, stream=stream,
                       tuning=lbm.make_tuning(time_block=1)) as b:
        done = 0
        for n in (1, 100, 64, 3, 257):  # graph runs start from both buffers
            a.step(n)
            for _ in range(n):
                b.step(1)
            done += n
            ra, ua, da = a.moments(raise_on_domain=False)
            rb, ub, db = b.moments(raise_on_domain=False)
            assert da["steps"] == db["steps"] == done
            assert np.array_equal(ra, rb) and np.array_equal(ua, ub)
        assert np.array_equal(a.populations(), b.populations())
