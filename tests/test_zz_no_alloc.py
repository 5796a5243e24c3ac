"""lbm_step_static (the FP64 mass reduction's partial sums in the library's
static device scratch, no device allocation) against lbm_step, called through
the C ABI: two calls in a row, the second on a smaller lattice, so the second
call runs on a scratch array that still holds the first call's partials.  The
step kernels are the same, so states must agree bit for bit; the reduction is
the same with the same partial count and order, so the masses must too, and
they must equal a host sum of the populations to FP64 rounding."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2005_04642_amd import lbm, workloads as Wk

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def run_pair(lib, nx, ny, storage, steps):
    prm = Wk.base_params(Lambda=10.0, sigma=0.01)
    rn = Wk.static_drop(nx, ny, min(nx, ny) / 4.0)
    a = lbm.Simulation(nx, ny, prm, rn, storage=storage, device=DEV)
    b = lbm.Simulation(nx, ny, prm, rn, storage=storage, device=DEV)
    ma = torch.full((2,), float("nan"), dtype=torch.float64, device=DEV)
    mb = torch.full((2,), float("nan"), dtype=torch.float64, device=DEV)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.lbm_step(a.h, steps, ctypes.c_void_p(ma.data_ptr()), s) == lbm.LBM_OK
    assert lib.lbm_step_static(b.h, steps, ctypes.c_void_p(mb.data_ptr()), s) == lbm.LBM_OK, \
        lib.lbm_last_error()
    torch.cuda.synchronize()
    out = (ma.cpu().numpy(), mb.cpu().numpy(), a.live_pops().double().cpu().numpy(),
           b.live_pops().double().cpu().numpy())
    a.close()
    b.close()
    return out


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_step_static_matches_step_on_two_calls(storage):
    lib = lbm.load_library()
    for nx, ny, steps in [(300, 200, 6), (41, 37, 3)]:   # the second input is smaller
        print("lbm_step_static vs lbm_step: %s %dx%d, %d steps" % (storage, nx, ny, steps), flush=True)
        ma, mb, pa, pb = run_pair(lib, nx, ny, storage, steps)
        assert np.array_equal(pa, pb)
        assert np.array_equal(ma, mb), (ma, mb)
        host = np.array([pb[0].sum(), pb[1].sum()])
        assert np.all(np.abs(mb - host) <= 1e-12 * np.abs(host)), (mb, host)


def test_step_static_rejects_bad_arguments():
    lib = lbm.load_library()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.lbm_step_static(None, 1, None, s) == lbm.LBM_EINVAL
    prm = Wk.base_params(Lambda=10.0)
    a = lbm.Simulation(16, 16, prm, Wk.static_drop(16, 16, 4.0), storage="f32", device=DEV)
    assert lib.lbm_step_static(a.h, -1, None, s) == lbm.LBM_EINVAL
    assert lib.lbm_step_static(a.h, 2, None, s) == lbm.LBM_OK
    a.close()
