"""Host-side checks of the C-ABI library (no GPU): symbols, validation and quadratures."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import quadrature as qd

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "rlbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rlbm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(rlbm_lib):
    names = declared_functions()
    assert "rlbm_step" in names and "rlbm_init" in names and "rlbm_moments" in names
    for name in names:
        assert hasattr(rlbm_lib, name), name


@pytest.mark.parametrize("d,zeta,order,kind,ref", [
    (2, 0.0, 2, "ur_onlattice", lambda: qd.ur_onlattice_2d()),
    (2, 0.0, 3, "product", lambda: qd.product_2d(0.0, 3)),
    (2, 1.0, 3, "product", lambda: qd.product_2d(1.0, 3)),
    (2, 2.5, 2, "product", lambda: qd.product_2d(2.5, 2)),
    (2, 5.0, 3, "product", lambda: qd.product_2d(5.0, 3)),
    (3, 1.0, 3, "product", lambda: qd.product_3d(1.0, 3)),
    (3, 0.3, 2, "product", lambda: qd.product_3d(0.3, 2)),
])
def test_library_quadrature_matches_oracle(rlbm_lib, d, zeta, order, kind, ref):
    from paper_1909_04502_amd import rlbm as R
    p, w, disp = R.quadrature_build(d, zeta, order, kind)
    q = ref()
    assert p.shape[0] == q.Q
    assert np.abs(p.numpy() - q.p).max() < 1e-13 * max(1.0, np.abs(q.p).max())
    assert np.abs(w.numpy() - q.w).max() < 1e-14
    assert np.abs(disp.numpy() - q.disp).max() < 1e-14


def test_library_rejects_bad_models(rlbm_lib):
    from paper_1909_04502_amd import rlbm as R
    for args in [(2, 1.0, 2, "ur_onlattice"), (4, 1.0, 3, "product"), (2, -1.0, 3, "product"),
                 (2, 1.0, 5, "product")]:
        with pytest.raises(R.RLBMError) as e:
            R.quadrature_build(*args)
        assert e.value.status in (R.ERR_INVALID_ARG, R.ERR_UNSUPPORTED)


def test_create_validates_before_touching_the_device(rlbm_lib):
    from paper_1909_04502_amd import rlbm as R
    cfg = R.Config()
    cfg.model = R.Model(d=2, order=3, kind=1, pad_=0, zeta=1.0)
    cfg.extent[0], cfg.extent[1], cfg.extent[2] = 0, 8, 1
    cfg.tau = 0.8
    h = ctypes.c_void_p()
    assert rlbm_lib.rlbm_create(ctypes.byref(cfg), ctypes.byref(h)) == R.ERR_INVALID_ARG
    cfg.extent[0] = 8
    cfg.tau = -1.0
    assert rlbm_lib.rlbm_create(ctypes.byref(cfg), ctypes.byref(h)) == R.ERR_INVALID_ARG
    cfg.tau = 0.8
    cfg.storage = 7
    assert rlbm_lib.rlbm_create(ctypes.byref(cfg), ctypes.byref(h)) == R.ERR_INVALID_ARG
    assert rlbm_lib.rlbm_step(None, None, None, 1, None, None) == R.ERR_INVALID_ARG


def test_batch_create_validates_before_touching_the_device(rlbm_lib):
    """Mixed orders, storages, 3D or product/UR mixes and tau fields are refused up front."""
    from paper_1909_04502_amd import rlbm as R

    def cfg(d=2, order=3, kind=1, storage=0, tau_field=None):
        c = R.Config()
        c.model = R.Model(d=d, order=order, kind=kind, pad_=0, zeta=1.0)
        c.extent[0], c.extent[1], c.extent[2] = 8, 8, (8 if d == 3 else 1)
        c.storage = storage
        c.tau = 0.8
        c.tau_field = tau_field
        c.n_ref = 1.0
        return c

    h = ctypes.c_void_p()
    for pair in [(cfg(), cfg(order=2)), (cfg(), cfg(storage=1)), (cfg(d=3), cfg(d=3)),
                 (cfg(kind=0, order=2), cfg(kind=0, order=2)), (cfg(), cfg(tau_field=1024))]:
        arr = (R.Config * 2)(*pair)
        st = rlbm_lib.rlbm_batch_create(arr, 2, ctypes.byref(h))
        assert st == R.ERR_UNSUPPORTED
    assert rlbm_lib.rlbm_batch_create(None, 2, ctypes.byref(h)) == R.ERR_INVALID_ARG
    assert rlbm_lib.rlbm_batch_variant_count() == 12


@pytest.mark.parametrize("d,order,zetas", [(2, 3, (0.0, 0.01, 1.0, 5.0, 15.0)), (2, 2, (0.0, 30.0)),
                                          (3, 3, (0.0, 0.01, 0.3, 1.0, 5.0, 10.0)), (3, 2, (0.05, 30.0))])
def test_tables_build_over_the_zeta_range(rlbm_lib, d, order, zetas):
    """Host precompute (quadrature, projection checks, the d = 3 Chebyshev EOS fit) succeeds over the
    supported zeta range: without a device, rlbm_create then stops at the first device call."""
    import torch
    from paper_1909_04502_amd import rlbm as R
    if torch.cuda.is_available():
        pytest.skip("checks the host stage only where no device is present")
    for z in zetas:
        c = R.Config()
        c.model = R.Model(d=d, order=order, kind=1, pad_=0, zeta=z)
        c.extent[0], c.extent[1], c.extent[2] = 4, 4, (4 if d == 3 else 1)
        c.tau, c.n_ref = 0.8, 1.0
        h = ctypes.c_void_p()
        st = rlbm_lib.rlbm_create(ctypes.byref(c), ctypes.byref(h))
        assert st == R.ERR_DEVICE, (z, st, rlbm_lib.rlbm_last_error())
