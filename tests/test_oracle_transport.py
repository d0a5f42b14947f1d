"""The oracle's RLBM against the Chapman-Enskog transport coefficients of App. C (Secs. 7.2 and 7.3
calibrations), with the paper's on-lattice massive stencil (45 vectors, m~ = 5, exact streaming).

* Thermal conductivity: a rod between plates held at T = 1.005 and 0.995 (walls at rest, own n),
  run to a steady state; lambda = -<q^x> / <dT/dx> over the interior, with the Eckart heat flux
  q^x = h (n U^x - N^x) (h = (eps + P)/n) from the pre-collision moments.
* Bulk viscosity: a periodic sine wave u_x = u0 sin(2 pi x/L); mu = -varpi / div U by least squares
  with varpi = -(m^2 sum_i f_i - (eps - d P))/d from the pre-collision populations.
Pre-collision moments carry the kinetic tau, so both compare with f(zeta) x tau.  One site is v0 in
units where c and the time step are 1.
"""
import functools
import math

import numpy as np
import pytest
import torch

from oracle import lattice as OL
from oracle import mj
from oracle import quadrature as qd

ZETA = 5.0


@functools.lru_cache(maxsize=None)
def rule():
    return qd.massive_onlattice(2, ZETA, 3)


def test_thermal_conductivity_chapman_enskog():
    q = rule()
    L, ny, tau, steps = 60, 4, 0.9, 1800
    ol = OL.Lattice(q, tau, (L, ny), bc=("wall", "periodic"), wall_T=((1.005, 0.995), (0.0, 0.0)))
    ones = torch.ones((ny, L), dtype=torch.float64)
    fs = ol.collide(ol.init(ones, ones, torch.zeros((2, ny, L), dtype=torch.float64)))
    for _ in range(steps):
        fs = ol.collide(ol.stream(fs))
    f = ol.stream(fs)
    mac = ol.macro(f)
    p = torch.tensor(q.p)
    Nx = torch.einsum("i,i...->...", p[:, 1], f)
    h = (mac["eps"] + mac["n"] * mac["T"]) / mac["n"]
    qx = h * (mac["n"] * mac["U"][1] - Nx)
    dT = (torch.roll(mac["T"], -1, 1) - torch.roll(mac["T"], 1, 1)) / (2 * q.v0)
    inner = slice(8, L - 8)
    lam = -(qx[:, inner].mean() / dT[:, inner].mean()).item()
    n = mac["n"][:, inner].mean().item()
    assert qx[0, inner].std().item() < 1e-2 * abs(qx[0, inner].mean().item())      # steady
    assert abs(lam / (n * tau) / mj.ce_conductivity_ratio(ZETA, 2) - 1) < 0.01


def test_bulk_viscosity_chapman_enskog():
    q = rule()
    L, ny, tau, u0 = 800, 4, 0.8, 1e-5
    x = np.arange(L)
    u = np.zeros((2, ny, L))
    u[0] = u0 * np.sin(2 * np.pi * x / L)[None, :]
    ones = torch.ones((ny, L), dtype=torch.float64)
    ol = OL.Lattice(q, tau, (L, ny))
    fs = ol.collide(ol.init(ones, ones, torch.tensor(u)))
    num = den = 0.0
    for s in range(1, 231):
        f = ol.stream(fs)
        if s >= 20 and s % 5 == 0:
            mac = ol.macro(f)
            P = mac["n"] * mac["T"]
            varpi = -(ZETA * ZETA * f.sum(0) - (mac["eps"] - 2 * P)) / 2
            div = (torch.roll(mac["U"][1], -1, 1) - torch.roll(mac["U"][1], 1, 1)) / (2 * q.v0)
            num += -(varpi * div).sum().item() / P.mean().item()
            den += (div * div).sum().item()
        fs = ol.collide(f)
    mu = num / den
    assert abs(mu / tau / mj.ce_bulk_ratio(ZETA, 2) - 1) < 0.03


def test_lattice_shear_coefficient_of_isotropic_rules():
    """The rule's own xy-shear coefficient (Lattice.shear_coefficient) reduces to the App. C value
    f_CE(zeta) where the rule integrates the stress moment (nearly) exactly: the product rules
    (equally weighted directions) to 3e-4 in d = 2 and 1e-4 in d = 3, exactly for the massless 2D
    product rule (the stress moment is then a polynomial the rule integrates)."""
    for zeta in (0.0, 1.0, 5.0):
        c = OL.Lattice(qd.product_2d(zeta, 3), 1.0, (1, 1)).shear_coefficient()
        assert abs(c / mj.ce_shear_ratio(zeta, 2) - 1) < 3e-4, zeta
    c0 = OL.Lattice(qd.product_2d(0.0, 3), 1.0, (1, 1)).shear_coefficient()
    assert abs(c0 - 0.75) < 1e-12
    c3 = OL.Lattice(qd.product_3d(1.0, 3), 1.0, (1, 1, 1)).shear_coefficient()
    assert abs(c3 / mj.ce_shear_ratio(1.0, 3) - 1) < 1e-4


def _shear_wave_rate(quad, tau, L, u0=1e-4, nsteps=240, first=40):
    """Decay rate per step of a shear wave u_x = u0 sin(2 pi y / L) on a periodic 4 x L lattice."""
    lat = OL.Lattice(quad, tau, (4, L))
    y = np.arange(L)
    u = np.zeros((2, L, 4))
    u[0] = u0 * np.sin(2 * np.pi * y / L)[:, None]
    ones = torch.ones((L, 4), dtype=torch.float64)
    f = lat.collide(lat.init(ones, ones, torch.tensor(u)))
    mode = torch.tensor(np.sin(2 * np.pi * y / L))[:, None]
    ts, logs = [], []
    for t in range(1, nsteps + 1):
        f = lat.stream(f)
        if t >= first:
            mac = lat.macro(f)
            ux = mac["U"][1] / mac["U"][0]
            ts.append(t)
            logs.append(math.log(abs(float((ux * mode).sum()))))
        f = lat.collide(f)
    return -np.polyfit(ts, logs, 1)[0]


def test_shear_wave_decay_follows_the_lattice_coefficient():
    """On the 45-vector massive rule (m~ = 5, exact streaming) a decaying shear wave measures the xy
    viscosity directly: gamma = k^2 eta / (eps + P) with eta = c_eta P (tau - 1/2), eps + P = G_2 P,
    k = 2 pi / (L v0).  At L = 192 sites the rule's own c_eta (0.9928 f_CE) predicts the oracle's rate
    to 3e-4 (the remainder falls as 1/L^2: 4.9e-3, 1.2e-3, 3.0e-4, 7.6e-5 at L = 48, 96, 192, 384, the
    next order in k); the App. C value alone is 0.7 % off, outside the bound."""
    zeta, L = 5.0, 192
    q = qd.massive_onlattice_2d(zeta, 3)
    c = OL.Lattice(q, 1.0, (1, 1)).shear_coefficient()
    fce = mj.ce_shear_ratio(zeta, 2)
    assert abs(c / fce - 0.99281) < 5e-5
    k = 2 * math.pi / (L * q.v0)
    G = float(mj.G_d(zeta, 2))
    for tau in (0.8, 1.3):
        rate = _shear_wave_rate(q, tau, L)
        pred = k * k * c * (tau - 0.5) / G
        print("tau", tau, "rate", rate, "pred", pred, "with f_CE", k * k * fce * (tau - 0.5) / G)
        assert abs(rate / pred - 1) < 1e-3, (tau, rate, pred)
        assert abs(rate / (pred * fce / c) - 1) > 5e-3
