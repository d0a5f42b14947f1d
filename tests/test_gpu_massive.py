"""Massive on-lattice rules (Sec. 5.3) on the GPU against the FP64 oracle.

The 29-vector order-2 stencil of the worked example and the 45-vector order-3
stencil of the GPU benchmark (Sec. 6.3), at m~ = 5, streamed exactly (integer
displacements up to 4 sites).  Bar as for the other rules: max-normalised error
1e-12 on populations and fields in double storage, 1e-5 on the fields in the
float-deviation storage.  The library runs at the v0 the oracle chose (the
same double), and by default picks the same v0 itself.
"""
import functools

import numpy as np
import pytest
import torch

import workloads as W
from oracle import lattice as OL
from oracle import quadrature as qd

pytestmark = pytest.mark.gpu

ZETA = 5.0


@functools.lru_cache(maxsize=None)
def oracle_rule(order):
    return qd.massive_onlattice_2d(ZETA, order)


def rel(a, b):
    a = a.detach().cpu().to(torch.float64)
    b = b.detach().cpu().to(torch.float64)
    return ((a - b).abs().max() / b.abs().max()).item()


# name: (order, extent, bc, tau, u0, density sigma, population-noise amp)
CASES = {
    "n2_periodic": (2, (37, 29), ("periodic", "periodic"), 0.8, 0.05, 1e-3, 1e-3),
    "n3_periodic": (3, (70, 33), ("periodic", "periodic"), 0.9, 0.1, 1e-3, 0.0),
    "n3_open": (3, (41, 12), ("open", "periodic"), 1.1, 0.08, 0.0, 1e-3),
    "n3_edge": (3, (4, 4), ("periodic", "periodic"), 0.7, 0.05, 1e-3, 1e-3),   # extent = max |n|
}


def setup_case(name, storage="f64"):
    from paper_1909_04502_amd import rlbm as R
    order, ext, bc, tau, u0, sig, amp = CASES[name]
    nx, ny = ext
    q = oracle_rule(order)
    n, T, u = W.taylor_green_2d(nx, ny, u0, density_sigma=sig, seed=3)
    gl = R.Lattice(d=2, zeta=ZETA, order=order, kind="massive_onlattice", extent=ext, bc=bc, storage=storage,
                   tau=tau, v0=q.v0)
    xi = W.population_noise(gl.Q, (ny, nx), seed=4) if amp else None
    ol = OL.Lattice(q, tau, ext, bc=bc)
    tens = [torch.tensor(a) for a in (n, T, u)] + [torch.tensor(xi) if xi is not None else None, amp]
    return gl, ol, tens


@pytest.mark.parametrize("name", list(CASES))
def test_massive_step_parity(name):
    print(f"[case] massive {name}", flush=True)
    gl, ol, (n, T, u, xi, amp) = setup_case(name)
    assert gl.Q == (29 if CASES[name][0] == 2 else 45) and gl.on_lattice
    nsteps = 5
    fa = gl.init(n, T, u, noise=xi, amp=amp)
    f0 = fa.clone()
    res = gl.step(fa, gl.new_state(), nsteps)
    mom = gl.moments(res)
    gl.sync()
    fs = ol.collide(ol.init(n, T, u, noise=xi, amp=amp))
    assert rel(f0, fs) < 1e-12
    for _ in range(nsteps):
        fs = ol.collide(ol.stream(fs))
    assert rel(res, fs) < 1e-12
    ref = ol.macro(ol.stream(fs))
    for k in ("n", "eps", "T"):
        assert rel(mom[k], ref[k]) < 1e-12, k
    assert rel(mom["U"], ref["U"]) < 1e-12


@pytest.mark.parametrize("name", ["n2_periodic", "n3_open"])
def test_massive_f32_deviation_storage(name):
    print(f"[case] massive f32dev {name}", flush=True)
    gl, ol, (n, T, u, xi, amp) = setup_case(name, storage="f32dev")
    nsteps = 12
    fa = gl.init(n, T, u, noise=xi, amp=amp)
    res = gl.step(fa, gl.new_state(), nsteps)
    mom = gl.moments(res)
    gl.sync()
    fs = ol.collide(ol.init(n, T, u, noise=xi, amp=amp))
    for _ in range(nsteps):
        fs = ol.collide(ol.stream(fs))
    ref = ol.macro(ol.stream(fs))
    for k in ("n", "eps", "T"):
        assert rel(mom[k], ref[k]) < 1e-5, k
    assert rel(mom["U"], ref["U"]) < 1e-5


def test_massive_tau_field():
    from paper_1909_04502_amd import rlbm as R
    print("[case] massive tau field", flush=True)
    q = oracle_rule(3)
    nx, ny = 24, 19
    n, T, u = W.taylor_green_2d(nx, ny, 0.1, density_sigma=1e-3, seed=6)
    tau = 0.8 + 0.3 * W.random_field((ny, nx), seed=7, lo=0.0, hi=1.0)
    gl = R.Lattice(d=2, zeta=ZETA, order=3, kind="massive_onlattice", extent=(nx, ny), tau=0.8,
                   tau_field=torch.tensor(tau), v0=q.v0)
    ol = OL.Lattice(q, torch.tensor(tau), (nx, ny))
    n, T, u = (torch.tensor(a) for a in (n, T, u))
    res = gl.step(gl.init(n, T, u), gl.new_state(), 3)
    gl.sync()
    fs = ol.collide(ol.init(n, T, u))
    for _ in range(3):
        fs = ol.collide(ol.stream(fs))
    assert rel(res, fs) < 1e-12


def test_massive_default_v0_is_the_window_middle():
    from paper_1909_04502_amd import rlbm as R
    print("[case] massive default v0", flush=True)
    for order in (2, 3):
        gl = R.Lattice(d=2, zeta=ZETA, order=order, kind="massive_onlattice", extent=(8, 8))
        assert gl.v0 == oracle_rule(order).v0


def test_massive_full_size_parity_and_conservation():
    """512^2, order 3, the benchmark's Taylor-Green start and launch shape: the whole grid against the
    oracle after two steps; over 20 more steps the totals of N^0 and T^0a (a = 1, 2) (conserved by streaming and by
    the Landau-frame collision) stay put."""
    from paper_1909_04502_amd import rlbm as R
    print("[case] massive 512^2", flush=True)
    q = oracle_rule(3)
    nx = ny = 512
    n, T, u = (torch.tensor(a) for a in W.taylor_green_2d(nx, ny, 0.1, density_sigma=1e-3, seed=8))
    gl = R.Lattice(d=2, zeta=ZETA, order=3, kind="massive_onlattice", extent=(nx, ny), tau=0.8, v0=q.v0)
    ol = OL.Lattice(q, 0.8, (nx, ny))
    fa = gl.init(n, T, u)
    fb = gl.new_state()
    res = gl.step(fa, fb, 2)
    gl.sync()
    fs = ol.collide(ol.init(n, T, u))
    for _ in range(2):
        fs = ol.collide(ol.stream(fs))
    assert rel(res, fs) < 1e-12
    p = torch.tensor(q.p, device="cuda")
    w0 = p[:, :1] * p                                   # p^0 p^a: N^0 (a = 0) and T^0a weights
    w0[:, 0] = p[:, 0]

    def totals(f):
        return torch.einsum("i...,ia->a", f, w0).cpu()
    t0 = totals(res)
    res = gl.step(res, fa if res.data_ptr() == fb.data_ptr() else fb, 18)
    gl.sync()
    t1 = totals(res)
    assert (t1 - t0).abs().max().item() < 1e-13 * t0.abs().max().item()


def test_massive_launch_variants_agree():
    from paper_1909_04502_amd import rlbm as R
    print("[case] massive variants", flush=True)
    q = oracle_rule(3)
    nx, ny = 130, 67
    n, T, u = (torch.tensor(a) for a in W.taylor_green_2d(nx, ny, 0.1, density_sigma=1e-3, seed=9))
    gl = R.Lattice(d=2, zeta=ZETA, order=3, kind="massive_onlattice", extent=(nx, ny), tau=0.9, v0=q.v0)
    f0 = gl.init(n, T, u)
    ref = None
    for v in range(R.lib().rlbm_variant_count()):
        gl.variant = v
        out = gl.step(f0.clone(), gl.new_state(), 3)
        gl.sync()
        if ref is None:
            ref = out.clone()
        else:
            assert rel(out, ref) < 1e-14, v


# ---------------------------------------------------------------- (3+1)-d, 143 vectors
# name: (extent, bc, tau, storage)
CASES3 = {
    "d3_periodic": ((9, 7, 6), ("periodic",) * 3, 0.8, "f64"),
    "d3_open": ((8, 5, 4), ("open", "periodic", "periodic"), 1.1, "f64"),
    "d3_edge": ((3, 3, 3), ("periodic",) * 3, 0.7, "f64"),          # extent = max |n|
    "d3_f32dev": ((9, 7, 6), ("periodic",) * 3, 0.9, "f32dev"),
}


@functools.lru_cache(maxsize=None)
def oracle_rule_3d():
    return qd.massive_onlattice(3, ZETA, 3)


def fields_3d(shape, seed):
    g = np.random.default_rng(seed)
    n = 1.0 + 0.02 * g.standard_normal(shape)
    T = 1.0 + 0.05 * g.uniform(-1, 1, shape)
    u = 0.05 * g.uniform(-1, 1, (3,) + shape)
    return n, T, u


@pytest.mark.parametrize("name", list(CASES3))
def test_massive_3d_parity(name):
    from paper_1909_04502_amd import rlbm as R
    print(f"[case] massive 3d {name}", flush=True)
    ext, bc, tau, storage = CASES3[name]
    q = oracle_rule_3d()
    n, T, u = (torch.tensor(a) for a in fields_3d(tuple(reversed(ext)), seed=11))
    gl = R.Lattice(d=3, zeta=ZETA, order=3, kind="massive_onlattice", extent=ext, bc=bc, storage=storage,
                   tau=tau, v0=q.v0)
    assert gl.Q == 143
    ol = OL.Lattice(q, tau, ext, bc=bc)
    nsteps = 4 if storage == "f64" else 10
    res = gl.step(gl.init(n, T, u), gl.new_state(), nsteps)
    mom = gl.moments(res)
    gl.sync()
    fs = ol.collide(ol.init(n, T, u))
    for _ in range(nsteps):
        fs = ol.collide(ol.stream(fs))
    ref = ol.macro(ol.stream(fs))
    tol = 1e-12 if storage == "f64" else 1e-5
    if storage == "f64":
        assert rel(res, fs) < tol
    for k in ("n", "eps", "T"):
        assert rel(mom[k], ref[k]) < tol, k
    assert rel(mom["U"], ref["U"]) < tol


def window_oracle(q, tau, fields, site, steps, R=3):
    """f* after `steps` steps at one site of a periodic lattice, from the oracle run on the periodic
    window of half-width steps * R around it (the update reaches R sites per step, so the window's
    own wrap-around never reaches the centre)."""
    h = steps * R
    n, T, u = fields
    idx = [np.arange(c - h, c + h + 1) % s for c, s in zip(site, n.shape)]
    ix = np.ix_(*idx)
    wn, wT = n[ix], T[ix]
    wu = np.stack([c[ix] for c in u])
    w = 2 * h + 1
    ol = OL.Lattice(q, tau, (w, w, w))
    fs = ol.collide(ol.init(torch.tensor(wn), torch.tensor(wT), torch.tensor(wu)))
    for _ in range(steps):
        fs = ol.collide(ol.stream(fs))
    return fs[(slice(None), h, h, h)]


@pytest.mark.parametrize("storage", ["f64", "f32dev"])
def test_massive_3d_full_size(storage):
    """192^3, the benchmark's lattice and launch shape: two steps compared with the oracle at sampled
    sites (windowed oracle, edges and interior), and over ten more steps the totals of N^0 and T^0a."""
    from paper_1909_04502_amd import rlbm as R
    print(f"[case] massive 3d 192^3 {storage}", flush=True)
    q = oracle_rule_3d()
    L = 192
    fields = W.taylor_green_3d(L, L, L, 0.1, density_sigma=1e-3, seed=12)
    gl = R.Lattice(d=3, zeta=ZETA, order=3, kind="massive_onlattice", extent=(L, L, L), tau=0.8, v0=q.v0,
                   storage=storage)
    fa = gl.init(*(torch.tensor(a) for a in fields))
    fb = gl.new_state()
    res = gl.step(fa, fb, 2)                 # even: the result is in fa
    gl.sync()
    g = np.random.default_rng(13)
    sites = [(0, 0, 0), (L - 1, L - 1, L - 1), (0, L // 2, L - 2)] + [tuple(g.integers(0, L, 3)) for _ in range(9)]
    fref = 0.0
    if storage == "f32dev":        # the buffer holds f - f^ref, f^ref the rest equilibrium at n = T = 1
        one = torch.ones((1, 1, 1), dtype=torch.float64)
        rest = torch.zeros((4, 1, 1, 1), dtype=torch.float64)
        rest[0] = 1.0
        fref = OL.Lattice(q, 0.8, (1, 1, 1)).equilibrium(one, one, rest)[:, 0, 0, 0]
    tol = 1e-12 if storage == "f64" else 1e-5
    for s in sites:
        ref = window_oracle(q, 0.8, fields, s, 2)
        got = res[(slice(None),) + tuple(int(c) for c in s)].cpu().to(torch.float64) + fref
        assert ((got - ref).abs().max() / ref.abs().max()).item() < tol, s
    if storage == "f64":
        p = torch.tensor(q.p, device="cuda")
        w0 = p[:, :1] * p
        w0[:, 0] = p[:, 0]

        def totals(f):
            return torch.einsum("i...,ia->a", f, w0).cpu()
        t0 = totals(res)
        res = gl.step(res, fb, 10)
        gl.sync()
        t1 = totals(res)
        assert (t1 - t0).abs().max().item() < 1e-13 * t0.abs().max().item()
