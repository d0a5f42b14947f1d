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
    (2, 0.0, 3, "ur_onlattice", lambda: qd.ur_onlattice_2d(3)),
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
    cfg.storage = 0
    cfg.tau_T = 0.3                                     # the tau law is built for on-lattice rules
    assert rlbm_lib.rlbm_create(ctypes.byref(cfg), ctypes.byref(h)) == R.ERR_UNSUPPORTED
    cfg.tau_T = float("nan")
    assert rlbm_lib.rlbm_create(ctypes.byref(cfg), ctypes.byref(h)) == R.ERR_INVALID_ARG
    cfg.tau_T = 0.0
    assert rlbm_lib.rlbm_step(None, None, None, 1, None, None) == R.ERR_INVALID_ARG
    assert rlbm_lib.rlbm_step_static(None, None, None, 1, None, None, None) == R.ERR_INVALID_ARG
    assert rlbm_lib.rlbm_step_static(ctypes.byref(cfg), None, None, 1, None, None, None) == R.ERR_INVALID_ARG


def test_create_rejects_sizes_beyond_the_limits(rlbm_lib):
    """Extents above 2^20, 3D depths above 65,535 and population planes of 4 GiB or more (the
    kernels address a plane with 32-bit byte offsets) are refused before any allocation."""
    from paper_1909_04502_amd import rlbm as R
    cfg = R.Config()
    cfg.model = R.Model(d=2, order=3, kind=1, pad_=0, zeta=1.0)
    cfg.tau = 0.8
    h = ctypes.c_void_p()
    cfg.extent[0], cfg.extent[1], cfg.extent[2] = (1 << 20) + 1, 8, 1
    assert rlbm_lib.rlbm_create(ctypes.byref(cfg), ctypes.byref(h)) == R.ERR_INVALID_ARG
    cfg.extent[0], cfg.extent[1] = 1 << 16, 1 << 13           # 2^29 sites: an FP64 plane of 4 GiB
    assert rlbm_lib.rlbm_create(ctypes.byref(cfg), ctypes.byref(h)) == R.ERR_UNSUPPORTED
    cfg.extent[1] = 1 << 14                                   # float deviations: 2^30 sites x 4 B
    cfg.storage, cfg.n_ref = R.STORAGE["f32dev"], 1.0
    assert rlbm_lib.rlbm_create(ctypes.byref(cfg), ctypes.byref(h)) == R.ERR_UNSUPPORTED
    cfg.storage = 0
    cfg.model = R.Model(d=3, order=3, kind=1, pad_=0, zeta=1.0)
    cfg.extent[0], cfg.extent[1], cfg.extent[2] = 4, 4, 65536
    assert rlbm_lib.rlbm_create(ctypes.byref(cfg), ctypes.byref(h)) == R.ERR_UNSUPPORTED
    assert not h.value


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


def test_launch_and_store_mode_entry_points_reject_bad_arguments(rlbm_lib):
    """Null handles and out-of-range modes are argument errors, answered without a device."""
    from paper_1909_04502_amd import rlbm as R
    m, nt = ctypes.c_int32(-1), ctypes.c_int32(-1)
    assert rlbm_lib.rlbm_variant_count() == 13
    for mode in (0, 1, 2, 3, -1):
        assert rlbm_lib.rlbm_set_store_mode(None, mode) == R.ERR_INVALID_ARG
        assert rlbm_lib.rlbm_batch_set_store_mode(None, mode) == R.ERR_INVALID_ARG
    assert rlbm_lib.rlbm_get_store_mode(None, ctypes.byref(m), ctypes.byref(nt)) == R.ERR_INVALID_ARG
    assert rlbm_lib.rlbm_batch_get_store_mode(None, ctypes.byref(m), ctypes.byref(nt)) == R.ERR_INVALID_ARG
    assert rlbm_lib.rlbm_set_variant(None, 0) == R.ERR_INVALID_ARG
    assert m.value == -1 and nt.value == -1


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


@pytest.fixture(scope="module")
def massive_rules():
    return {(d, order): qd.massive_onlattice(d, 5.0, order) for d, order in ((2, 2), (2, 3), (3, 3))}


@pytest.mark.parametrize("d,order", [(2, 2), (2, 3), (3, 3)])
def test_library_massive_rule_matches_oracle(rlbm_lib, massive_rules, d, order):
    """The binary128 solver of the library against the oracle's mpmath solver (Sec. 5.3): the v0
    window, the rule at the oracle's v0 and the default (v0 = 0 -> middle of the window)."""
    from paper_1909_04502_amd import rlbm as R
    q = massive_rules[(d, order)]
    lo, hi = R.massive_window(5.0, order, d=d)
    qlo, qhi = q.window
    assert abs(lo - qlo) < 1e-15 and abs(hi - qhi) < 1e-15
    for v0 in (q.v0, 0.0):
        p, w, disp = R.quadrature_build(d, 5.0, order, "massive_onlattice", v0=v0)
        assert p.shape[0] == q.Q == {(2, 2): 29, (2, 3): 45, (3, 3): 143}[(d, order)]
        assert np.abs(p.numpy() - q.p).max() < 1e-14 * np.abs(q.p).max()
        assert np.abs(w.numpy() - q.w).max() < 1e-12 * q.w.max()
        assert np.all(disp.numpy() == q.disp)


def test_library_massive_rule_printed_example(rlbm_lib):
    """The worked example of Sec. 5.3 (m~ = 5, v0 = 0.2726): the printed group weights."""
    import json
    from paper_1909_04502_amd import rlbm as R
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "massive_2d_m5_order2.json")))
    p, w, disp = R.quadrature_build(2, g["m"], g["order"], "massive_onlattice", v0=g["v0"])
    w = w.numpy()
    per_group = [w[-1]] + [w[k] for k in (0, 4, 8, 16, 20)]       # rest, then each group's first member
    for got, want in zip(per_group, g["weights"]):
        assert abs(got - want) < 1e-10 * want


def test_library_massive_rule_rejections(rlbm_lib):
    from paper_1909_04502_amd import rlbm as R
    for args, kw in [((2, 0.0, 3, "massive_onlattice"), {}),            # massless
                     ((2, 5.0, 4, "massive_onlattice"), {}),            # order
                     ((3, 5.0, 2, "massive_onlattice"), {}),            # no 3D order-2 stencil
                     ((2, 5.0, 2, "massive_onlattice"), {"v0": 0.26}),  # outside the window
                     ((2, 5.0, 2, "massive_onlattice"), {"v0": 0.4})]:  # beyond 1/max|n|
        with pytest.raises(R.RLBMError) as e:
            R.quadrature_build(*args, **kw)
        assert e.value.status in (R.ERR_INVALID_ARG, R.ERR_UNSUPPORTED, R.ERR_QUADRATURE)


def test_create_validates_massive_lattices(rlbm_lib):
    """Checks that run before any device call: a periodic extent shorter than the longest integer
    displacement (the pull would wrap more than once) and a force on the 3D massive rule in double
    storage (its streaming kernel has no force term; the 2D massive rules take one)."""
    from paper_1909_04502_amd import rlbm as R
    cfg = R.Config()
    cfg.model = R.Model(d=2, order=3, kind=R.KIND["massive_onlattice"], pad_=0, zeta=5.0, v0=0.0)
    cfg.extent[0], cfg.extent[1], cfg.extent[2] = 3, 8, 1   # |n_x| reaches 4
    cfg.tau = 0.8
    h = ctypes.c_void_p()
    assert rlbm_lib.rlbm_create(ctypes.byref(cfg), ctypes.byref(h)) == R.ERR_INVALID_ARG
    cfg.model = R.Model(d=3, order=3, kind=R.KIND["massive_onlattice"], pad_=0, zeta=5.0, v0=0.0)
    cfg.extent[0], cfg.extent[1], cfg.extent[2] = 8, 8, 8
    cfg.force[0] = 1e-5
    assert rlbm_lib.rlbm_create(ctypes.byref(cfg), ctypes.byref(h)) == R.ERR_UNSUPPORTED
    cfg.force[0] = 0.0
    cfg.storage, cfg.n_ref = R.STORAGE["f32dev_f64"], 1.0   # double arithmetic on float storage: product rules
    assert rlbm_lib.rlbm_create(ctypes.byref(cfg), ctypes.byref(h)) == R.ERR_UNSUPPORTED
    ur = R.Config()
    ur.model = R.Model(d=2, order=2, kind=R.KIND["ur_onlattice"], pad_=0, zeta=0.0)
    ur.extent[0], ur.extent[1], ur.extent[2] = 16, 4, 1     # |n_y| reaches 5
    ur.tau = 0.8
    assert rlbm_lib.rlbm_create(ctypes.byref(ur), ctypes.byref(h)) == R.ERR_INVALID_ARG


def test_lds_loads_take_uniform_operands(rlbm_lib, tmp_path):
    """The LDS-staged step loads its windows with inline-assembly global-to-LDS loads: each sets m0
    (the LDS address) from a scalar register, waits one state, and loads with a scalar address pair
    and a vector offset.  A vector register in either scalar slot would be a build the hardware does
    not execute as written, so the built library's gfx950 code object (compiled from this repository's
    sources) is disassembled and every such load is checked."""
    import shutil
    import subprocess
    from paper_1909_04502_amd import build as b
    tools = {t: os.path.join("/opt/rocm/llvm/bin", t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-objdump")}
    if not all(os.path.exists(p) for p in tools.values()):
        pytest.skip("LLVM binary tools not installed")
    fat, co = str(tmp_path / "fatbin"), str(tmp_path / "gfx950.o")
    subprocess.run([tools["llvm-objcopy"], f"--dump-section=.hip_fatbin={fat}", b.LIB, str(tmp_path / "lib.so")],
                   check=True, capture_output=True)
    subprocess.run([tools["clang-offload-bundler"], "--type=o", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950",
                    f"--input={fat}", f"--output={co}", "--unbundle"], check=True, capture_output=True)
    dis = subprocess.run([tools["llvm-objdump"], "-d", co], check=True, capture_output=True, text=True).stdout
    lines = [l.split("//")[0].strip() for l in dis.splitlines()]
    lines = [l for l in lines if l and not l.endswith(">:")]
    loads = [i for i, l in enumerate(lines) if l.startswith("global_load_lds_dwordx4")]
    assert loads, "no global-to-LDS loads in the library"
    for i in loads:
        assert re.fullmatch(r"global_load_lds_dwordx4 v\d+, s\[\d+:\d+\]", lines[i]), lines[i]
        assert lines[i - 1] == "s_nop 0", lines[i - 2:i + 1]
        assert re.fullmatch(r"s_mov_b32 m0, s\d+", lines[i - 2]), lines[i - 2:i + 1]
    shutil.rmtree(tmp_path, ignore_errors=True)
