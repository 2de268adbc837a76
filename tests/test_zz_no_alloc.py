"""GPU test of lbm_vn_max_radius_noalloc, the form of lbm_vn_max_radius that
allocates nothing and takes no scratch argument (its scratch is a static
device array of the library).  Called through the C ABI, it must give bitwise
the results of lbm_vn_max_radius on the same states (the maximum over the
wave-vector grid does not depend on the order of evaluation), on two calls in
a row, the second with fewer states (the static scratch keeps the first
call's contents and must be cleared for the second), and refuse more states
than its scratch holds."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _states(n, seed):
    rng = np.random.default_rng(seed)
    nu = np.exp(rng.uniform(np.log(1e-5), np.log(0.5), n))
    speed = rng.uniform(0.0, 0.6, n)
    theta = rng.uniform(0.0, np.pi / 2, n)
    return np.stack([0.5 + 3.0 * nu, speed * np.cos(theta), speed * np.sin(theta)], axis=1)


@pytest.mark.parametrize("lattice,eq,corr", [(9, 0, 0), (9, 2, 1), (3, 1, 0)])
def test_no_alloc_max_radius_equals_scratch_form(lattice, eq, corr):
    import torch
    from paper_2303_08163_amd import lbm
    lib = lbm.load_library()
    fn = lib.lbm_vn_max_radius_noalloc
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                   ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev).cuda_stream
    nk = 9
    for n, seed in ((3000, 1), (700, 2)):
        states = torch.from_numpy(_states(n, seed)).to(dev)
        ref = torch.empty(n, dtype=torch.float64, device=dev)
        scratch = torch.empty(n, dtype=torch.int64, device=dev)
        unc_ref = torch.zeros(1, dtype=torch.int32, device=dev)
        out = torch.full((n,), -1.0, dtype=torch.float64, device=dev)
        unc = torch.full((1,), -7, dtype=torch.int32, device=dev)
        lbm.lbm_vn_max_radius(lattice, eq, corr, states.data_ptr(), n, nk, ref.data_ptr(), scratch.data_ptr(),
                              unc_ref.data_ptr(), stream)
        st = fn(lattice, eq, corr, states.data_ptr(), n, nk, out.data_ptr(), unc.data_ptr(), stream)
        assert st == lbm.LBM_OK, lib.lbm_last_error().decode()
        torch.cuda.synchronize()
        r, o = ref.cpu().numpy(), out.cpu().numpy()
        assert np.all(np.isfinite(r)) and np.all(r > 0)
        assert np.array_equal(r, o), (n, np.max(np.abs(r - o)))
        assert int(unc.item()) == int(unc_ref.item())
    # more states than the static scratch holds: refused before any GPU work
    big = 65537
    st = fn(lattice, eq, corr, states.data_ptr(), big, nk, out.data_ptr(), unc.data_ptr(), stream)
    assert st == lbm.LBM_EINVAL and "65536" in lib.lbm_last_error().decode()
