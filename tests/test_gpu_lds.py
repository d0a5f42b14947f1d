"""LDS-staged step of the 2D product rules (launch variant 12) against the register kernel.

The staged kernel reads the same upstream taps with the same weights and sums them in the same
order as the register kernel of the same tile shape (variant 1), so every state it produces must
equal that kernel's bit for bit: orders 2 and 3, the three storages, lattices narrower and shorter
than one window, ragged tiles in x and y, an open y axis, a per-site tau field, the fields of the
last step, and lattices of more tiles than fit on the chip at once.  One case is also checked
against the FP64 oracle.  Lattices the staged windows do not cover (x extent not a multiple of 4,
an open x axis, walls or a force) take the register kernel under that variant, with the same
results.  The staged kernel is the default above 384 MiB of state in every storage: the default
selection is checked, and a 2048 x 2048 float lattice's default run against the register kernel.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import lattice as OL
from oracle import quadrature as qd

pytestmark = pytest.mark.gpu

REG, LDS = 1, 12   # register kernel in 64 x 4 band tiles; the staged kernel

# name: (order, storage, extent, bc, tau field, force)
CASES = {
    "o3_f64": (3, "f64", (96, 70), ("periodic", "periodic"), False, None),
    "o3_f64_ragged_tau": (3, "f64", (132, 37), ("periodic", "periodic"), True, None),
    "o2_f64": (2, "f64", (64, 8), ("periodic", "periodic"), False, None),
    "o3_f64_narrow": (3, "f64", (8, 2), ("periodic", "periodic"), False, None),
    "o3_f64_one_row": (3, "f64", (12, 1), ("periodic", "periodic"), False, None),
    "o3_f64_open_y": (3, "f64", (68, 21), ("periodic", "open"), False, None),
    "o3_f32dev": (3, "f32dev", (96, 70), ("periodic", "periodic"), False, None),
    "o3_f32dev_narrow": (3, "f32dev", (4, 5), ("periodic", "periodic"), False, None),
    "o2_f32dev_open_y": (2, "f32dev", (200, 13), ("periodic", "open"), True, None),
    "o3_f32dev_f64": (3, "f32dev_f64", (96, 70), ("periodic", "periodic"), True, None),
    # more tiles than blocks fit on the chip at once
    "o3_f64_many_tiles": (3, "f64", (1024, 262), ("periodic", "periodic"), True, None),
    "o2_f64_many_tiles": (2, "f64", (768, 301), ("periodic", "open"), False, None),
    "o3_f32dev_many_tiles": (3, "f32dev", (1280, 300), ("periodic", "periodic"), False, None),
    "o3_f32dev_f64_many_tiles": (3, "f32dev_f64", (1024, 260), ("periodic", "periodic"), False, None),
    # not covered by the staged windows: the register kernel runs under every variant
    "fallback_x_not_multiple_of_4": (3, "f64", (70, 12), ("periodic", "periodic"), False, None),
    "fallback_open_x": (3, "f32dev", (64, 12), ("open", "periodic"), False, None),
    "fallback_walls_force": (3, "f64", (64, 12), ("wall", "periodic"), False, (0.0, 3e-4)),
}


def make(name):
    from paper_1909_04502_amd import rlbm as R
    order, storage, ext, bc, tau_field, force = CASES[name]
    nx, ny = ext
    kw = {"force": force} if force else {}
    if tau_field:
        g = np.random.default_rng(7)
        kw["tau_field"] = torch.tensor(0.8 + 0.2 * g.uniform(-1, 1, (ny, nx)))
    gl = R.Lattice(d=2, zeta=1.0, order=order, kind="product", extent=ext, bc=bc, storage=storage, tau=0.8, **kw)
    n, T, u = W.taylor_green_2d(nx, ny, 0.1, density_sigma=1e-3, seed=3)
    xi = W.population_noise(gl.Q, (ny, nx), seed=4)
    f0 = gl.init(torch.tensor(n), torch.tensor(T), torch.tensor(u), torch.tensor(xi), 1e-3)
    return gl, f0


def run(gl, f0, variant, nsteps):
    gl.variant = variant
    res, last = gl.step(f0.clone(), gl.new_state(), nsteps, want_last=True)
    gl.sync()
    return res.cpu(), {k: v.cpu() for k, v in last.items()}


@pytest.mark.parametrize("name", list(CASES))
def test_staged_step_equals_register_kernel(name):
    print(f"[case] lds {name} {CASES[name][2]}", flush=True)
    gl, f0 = make(name)
    for nsteps in (1, 5):   # one launch, and a cached graph of several
        ref, ref_last = run(gl, f0, REG, nsteps)
        assert torch.isfinite(ref).all()
        got, last = run(gl, f0, LDS, nsteps)
        assert torch.equal(got, ref), nsteps
        for k in ref_last:
            assert torch.equal(last[k], ref_last[k]), (nsteps, k)


def test_staged_step_against_oracle():
    """The staged kernel's 4 steps on the 96 x 70 FP64 case against the oracle's (1e-12)."""
    print("[case] lds oracle", flush=True)
    from paper_1909_04502_amd import rlbm as R
    nx, ny, tau = 96, 70, 0.8
    n, T, u = (torch.tensor(a) for a in W.taylor_green_2d(nx, ny, 0.1, density_sigma=1e-3, seed=3))
    gl = R.Lattice(d=2, zeta=1.0, order=3, kind="product", extent=(nx, ny), storage="f64", tau=tau)
    gl.variant = LDS
    res = gl.step(gl.init(n, T, u), gl.new_state(), 4)
    gl.sync()
    ol = OL.Lattice(qd.product_2d(1.0, 3), tau, (nx, ny))
    fs = ol.collide(ol.init(n, T, u))
    for _ in range(4):
        fs = ol.collide(ol.stream(fs))
    err = ((res.cpu() - fs).abs().max() / fs.abs().max()).item()
    print("staged vs oracle", err, flush=True)
    assert err < 1e-12


@pytest.mark.parametrize("storage,side,want", [("f64", 512, 5), ("f64", 1024, LDS), ("f32dev", 1024, 10),
                                               ("f32dev", 2048, LDS), ("f32dev_f64", 1024, 9),
                                               ("f32dev_f64", 2048, LDS), ("f64", 1026, 5)])
def test_default_variant_follows_the_state_size(storage, side, want):
    """The staged kernel is the default where the two state buffers exceed 384 MiB (and the x extent
    is a multiple of 4), in every storage; smaller lattices keep their register kernels."""
    from paper_1909_04502_amd import rlbm as R
    print(f"[case] default variant {storage} {side}", flush=True)
    gl = R.Lattice(d=2, zeta=1.0, order=3, kind="product", extent=(side, side), storage=storage, tau=0.8)
    assert gl.variant == want


def test_staged_default_at_2048_float_equals_register_kernel():
    """Float storage at 2048 x 2048 (two 512 MiB state buffers): two steps of the default launch (the
    staged kernel) against the register kernel, bit for bit."""
    from paper_1909_04502_amd import rlbm as R
    print("[case] lds default f32dev 2048", flush=True)
    L = 2048
    gl = R.Lattice(d=2, zeta=1.0, order=3, kind="product", extent=(L, L), storage="f32dev", tau=0.8)
    assert gl.variant == LDS
    n, T, u = (torch.tensor(a) for a in W.taylor_green_2d(L, L, 0.1, density_sigma=1e-3, seed=3))
    f0 = gl.init(n, T, u)
    got = gl.step(f0.clone(), gl.new_state(), 2)
    gl.sync()
    gl.variant = REG
    ref = gl.step(f0, gl.new_state(), 2)
    gl.sync()
    assert torch.equal(got, ref)
