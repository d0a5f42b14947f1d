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
