"""Allocation-free stepping: rlbm_step_static (tables in the library's static device array, no
handle, no device allocation) against rlbm_step on a handle, through the C ABI.  Three calls in a
row on one GPU: a lattice, a smaller one of another rule and storage (its tables replace the
first's in the array), and the first again; each bit-identical to rlbm_step (the same kernels
and tables), and the caller's flag left clear."""
import ctypes

import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

# (d, zeta, order, extent, bc, storage, tau, steps): the second is smaller than the first
CASES = [
    (2, 1.0, 3, (96, 70), ("periodic", "periodic"), "f64", 0.8, 5),
    (2, 2.5, 2, (33, 17), ("open", "periodic"), "f32dev", 1.3, 4),
    (2, 1.0, 3, (96, 70), ("periodic", "periodic"), "f64", 0.8, 3),
]


def test_static_step_matches_the_handle_step():
    from paper_1909_04502_amd import rlbm as R
    L = R.lib()
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    for k, (d, zeta, order, ext, bc, storage, tau, steps) in enumerate(CASES):
        print(f"[case] static step {k}: {ext} N={order} {storage} {steps} steps", flush=True)
        lat = R.Lattice(d=d, zeta=zeta, order=order, extent=ext, bc=bc, storage=storage, tau=tau)
        n, T, u = (torch.tensor(a) for a in W.taylor_green_2d(ext[0], ext[1], 0.05, density_sigma=1e-3, seed=k))
        f0 = lat.init(n, T, u)
        ref = lat.step(f0.clone(), lat.new_state(), steps)
        a, b = f0.clone(), lat.new_state()
        st = L.rlbm_step_static(ctypes.byref(lat.cfg), ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                steps, None, ctypes.c_void_p(flag.data_ptr()), R._stream())
        assert st == R.OK, R.lib().rlbm_last_error()
        lat.sync()
        got = b if steps % 2 == 1 else a
        assert torch.equal(got, ref), (k, (got.double() - ref.double()).abs().max().item())
        assert flag.item() == 0


def test_static_step_rejects_bad_arguments():
    from paper_1909_04502_amd import rlbm as R
    L = R.lib()
    lat = R.Lattice(d=2, zeta=1.0, order=3, extent=(16, 8), tau=0.8)
    a = lat.new_state()
    assert L.rlbm_step_static(None, None, None, 1, None, None, None) == R.ERR_INVALID_ARG
    assert L.rlbm_step_static(ctypes.byref(lat.cfg), ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(a.data_ptr()),
                              1, None, None, R._stream()) == R.ERR_INVALID_ARG          # f_a and f_b overlap
    bad = R.Config.from_buffer_copy(lat.cfg)
    bad.tau = -1.0
    b = lat.new_state()
    assert L.rlbm_step_static(ctypes.byref(bad), ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                              1, None, None, R._stream()) == R.ERR_INVALID_ARG


def test_static_step_sets_the_callers_flag_on_a_non_physical_state():
    """A state of all-zero populations has no timelike Landau eigenvector: the kernels set the
    caller's flag (and leave it clear for a physical state)."""
    from paper_1909_04502_amd import rlbm as R
    L = R.lib()
    lat = R.Lattice(d=2, zeta=1.0, order=3, extent=(16, 8), tau=0.8)
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    a, b = torch.zeros((lat.Q, 8, 16), dtype=torch.float64, device="cuda"), lat.new_state()
    st = L.rlbm_step_static(ctypes.byref(lat.cfg), ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), 1,
                            None, ctypes.c_void_p(flag.data_ptr()), R._stream())
    assert st == R.OK
    torch.cuda.synchronize()
    assert flag.item() == 1
    flag.zero_()
    n, T, u = (torch.tensor(x) for x in W.taylor_green_2d(16, 8, 0.05, seed=1))
    a = lat.init(n, T, u)
    st = L.rlbm_step_static(ctypes.byref(lat.cfg), ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), 2,
                            None, ctypes.c_void_p(flag.data_ptr()), R._stream())
    assert st == R.OK
    lat.sync()
    assert flag.item() == 0
