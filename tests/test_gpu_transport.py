"""Transport-coefficient calibrations (Secs. 7.2 and 7.3) on the GPU with the paper's on-lattice massive stencil
(the 45-vector (2+1)-d rule at m~ = 5, exact streaming), and parity of the walls at prescribed
temperatures that the thermal-conductivity set-up needs.

Thermal conductivity: a rod of 200 sites (four identical rows) between plates at T = 1.005 and 0.995
(walls at rest, own n), run to a steady state; lambda = -<q^x>/<dT/dx> over the interior with the
Eckart heat flux q^x = h (n U^x - N^x), h = (eps + P)/n, from the pre-collision moments.

Bulk viscosity: a periodic rod with u_x = u0 sin(2 pi x / L), n = T = 1 (u0 = 1e-5, as in the paper;
L = 1600 sites, four identical rows because the integer shifts reach 4 sites).  The dynamic pressure
is varpi = -(T^mu_mu - (eps - d P)) / d with T^mu_mu = m^2 sum_i f_i (every momentum is on the mass
shell) from the pre-collision populations, and mu = -varpi / div U by least squares over the sites and
the samples of half a sound period (div U by central differences; one site is v0 in units where c and
the time step are 1).  Pre-collision moments carry the kinetic tau: the measurement is compared with
the Chapman-Enskog mu = f_mu(zeta) P tau of App. C.
"""
import functools

import numpy as np
import pytest
import torch

from oracle import lattice as OL
from oracle import mj
from oracle import quadrature as qd

pytestmark = pytest.mark.gpu

ZETA = 5.0


@functools.lru_cache(maxsize=None)
def rule():
    return qd.massive_onlattice(2, ZETA, 3)


def streamed(lat, fs, disp):
    """The pre-collision populations f_i(x) = f*_i(x - n_i) of an integer-shift rule."""
    return torch.stack([torch.roll(fs[i], shifts=(int(disp[i, 1]), int(disp[i, 0])), dims=(0, 1))
                        for i in range(lat.Q)])


def bulk_viscosity(tau, L=1600, ny=4, u0=1e-5, nsteps=460, start=40, every=10):
    from paper_1909_04502_amd import rlbm as R
    q = rule()
    lat = R.Lattice(d=2, zeta=ZETA, order=3, kind="massive_onlattice", extent=(L, ny), tau=tau, v0=q.v0)
    x = np.arange(L)
    u = np.zeros((2, ny, L))
    u[0] = u0 * np.sin(2 * np.pi * x / L)[None, :]
    fa = lat.init(torch.ones((ny, L), dtype=torch.float64), torch.ones((ny, L), dtype=torch.float64),
                  torch.tensor(u))
    fb = lat.new_state()
    disp = q.disp
    num = den = 0.0
    Pm = []
    for s in range(every, nsteps + 1, every):
        lat.step(fa, fb, every)                # an even count: the state stays in fa
        if s < start:
            continue
        mac = lat.moments(fa)
        f = streamed(lat, fa, disp)
        P = mac["n"] * mac["T"]
        varpi = -(ZETA * ZETA * f.sum(0) - (mac["eps"] - 2 * P)) / 2
        Ux = mac["U"][1]
        div = (torch.roll(Ux, -1, dims=1) - torch.roll(Ux, 1, dims=1)) / (2 * q.v0)
        num += -(varpi * div).sum().item()
        den += (div * div).sum().item()
        Pm.append(P.mean().item())
    lat.sync()
    return num / den / np.mean(Pm)


@pytest.mark.parametrize("tau", [0.7, 1.0])
def test_bulk_viscosity_chapman_enskog(tau):
    print(f"[case] bulk viscosity tau={tau}", flush=True)
    mu = bulk_viscosity(tau)
    ce = mj.ce_bulk_ratio(ZETA, 2)
    print("mu / (P tau)", mu / tau, "Chapman-Enskog", ce, flush=True)
    assert abs(mu / tau / ce - 1.0) < 0.03


def rel(a, b):
    a = a.detach().cpu().to(torch.float64)
    b = b.detach().cpu().to(torch.float64)
    return ((a - b).abs().max() / b.abs().max()).item()


# name: (kind, zeta, order, extent, storage, wall_T of x)
WALLS = {
    "massive_f64": ("massive_onlattice", ZETA, 3, (23, 8), "f64", (1.005, 0.995)),
    "massive_own_T": ("massive_onlattice", ZETA, 3, (19, 6), "f64", (0.0, 1.02)),
    "massive_f32dev": ("massive_onlattice", ZETA, 3, (23, 8), "f32dev", (1.005, 0.995)),
    "product_f64": ("product", 1.0, 3, (21, 9), "f64", (1.1, 0.9)),
}


@pytest.mark.parametrize("name", list(WALLS))
def test_walls_at_prescribed_temperature_parity(name):
    from paper_1909_04502_amd import rlbm as R
    print(f"[case] walls {name}", flush=True)
    kind, zeta, order, ext, storage, wt = WALLS[name]
    nx, ny = ext
    g = np.random.default_rng(21)
    n = torch.tensor(1.0 + 0.01 * g.standard_normal((ny, nx)))
    T = torch.tensor(1.0 + 0.02 * g.uniform(-1, 1, (ny, nx)))
    u = torch.tensor(0.02 * g.uniform(-1, 1, (2, ny, nx)))
    kw = {"v0": rule().v0} if kind == "massive_onlattice" else {}
    gl = R.Lattice(d=2, zeta=zeta, order=order, kind=kind, extent=ext, bc=("wall", "periodic"), storage=storage,
                   tau=0.9, wall_T=(wt, (0.0, 0.0)), **kw)
    quad = rule() if kind == "massive_onlattice" else qd.product_2d(zeta, order)
    ol = OL.Lattice(quad, 0.9, ext, bc=("wall", "periodic"), wall_T=(wt, (0.0, 0.0)))
    nsteps = 5 if storage == "f64" else 16
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


def thermal_conductivity(tau, L=200, ny=4, chunk=1000, max_chunks=80):
    from paper_1909_04502_amd import rlbm as R
    q = rule()
    lat = R.Lattice(d=2, zeta=ZETA, order=3, kind="massive_onlattice", extent=(L, ny), tau=tau, v0=q.v0,
                    bc=("wall", "periodic"), wall_T=((1.005, 0.995), (0.0, 0.0)))
    ones = torch.ones((ny, L), dtype=torch.float64)
    fa = lat.init(ones, ones, torch.zeros((2, ny, L), dtype=torch.float64))
    fb = lat.new_state()
    p = torch.tensor(q.p, device="cuda")
    inner = slice(10, L - 10)
    prev = None
    for c in range(max_chunks):
        lat.step(fa, fb, chunk)               # an even count: the state stays in fa
        mac = lat.moments(fa)
        f = streamed(lat, fa, q.disp)
        Nx = torch.einsum("i,i...->...", p[:, 1], f)
        h = (mac["eps"] + mac["n"] * mac["T"]) / mac["n"]
        qx = h * (mac["n"] * mac["U"][1] - Nx)
        dT = (torch.roll(mac["T"], -1, 1) - torch.roll(mac["T"], 1, 1)) / (2 * q.v0)
        lam = -(qx[:, inner].mean() / dT[:, inner].mean()).item()
        if prev is not None and abs(lam - prev) < 1e-7 * abs(lam):
            break
        prev = lam
    lat.sync()
    spread = (qx[0, inner].std() / qx[0, inner].mean().abs()).item()
    return lam, mac["n"][:, inner].mean().item(), spread, (c + 1) * chunk


@pytest.mark.parametrize("tau", [0.8, 1.2])
def test_thermal_conductivity_chapman_enskog(tau):
    print(f"[case] thermal conductivity tau={tau}", flush=True)
    lam, n, spread, steps = thermal_conductivity(tau)
    ce = mj.ce_conductivity_ratio(ZETA, 2)
    print("lambda / (n tau)", lam / (n * tau), "Chapman-Enskog", ce, "flux spread", spread, "steps", steps,
          flush=True)
    assert spread < 2e-3
    assert abs(lam / (n * tau) / ce - 1.0) < 0.01
