"""Pins of the analytic ultra-relativistic Sod solution (App. D) against physics it must obey,
derived independently of the appendix's formulas: lab-frame jump conditions of the conserved
currents across the shock, the Riemann invariants and characteristic speed of the fan, and global
conservation of particle number, energy and momentum (momentum grows by the pressure difference)."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import sod

# the paper's inviscid set-up in lattice units: T_L = 1, T_R = 0.475, P_L / P_R = 5.43, n_L = 1
PL, nL = 1.0, 1.0
PR = 1.0 / 5.43
nR = PR / 0.475


def currents(d, n, P, b):
    """N^0, N^x, T^00, T^0x, T^xx of a perfect massless gas (eps = d P) moving at speed b."""
    g2 = 1.0 / (1.0 - b * b)
    h = (d + 1) * P                 # eps + P
    return {"N0": n * math.sqrt(g2), "Nx": n * math.sqrt(g2) * b, "T00": h * g2 - P, "T0x": h * g2 * b,
            "Txx": h * g2 * b * b + P}


@pytest.mark.parametrize("d", [2, 3])
def test_shock_jump_conditions(d):
    c = sod.waves(d, PL, nL, PR, nR)
    s = c["beta_s"]
    L = currents(d, c["n_II"], c["PC"], c["beta_C"])
    R = currents(d, nR, PR, 0.0)
    for q, F in (("N0", "Nx"), ("T00", "T0x"), ("T0x", "Txx")):
        assert abs((L[F] - s * L[q]) - (R[F] - s * R[q])) < 1e-13 * max(abs(L[F]), abs(R[q]), 1.0), q
    assert 0 < c["beta_C"] < s < 1 and c["n_II"] > nR and PR < c["PC"] < PL


@pytest.mark.parametrize("d", [2, 3])
def test_rarefaction_fan(d):
    c = sod.waves(d, PL, nL, PR, nR)
    t = 1.0
    x = np.linspace(c["w_H"] * t, c["w_T"] * t, 201)[1:-1]
    f = sod.solution(d, PL, nL, PR, nR, x, t)
    r = (1.0 + f["beta"]) / (1.0 - f["beta"])
    sd = math.sqrt(d)
    assert np.allclose(f["n"] * r ** (sd / 2), nL, rtol=1e-13)
    assert np.allclose(f["P"] * r ** ((d + 1) / (2 * sd)), PL, rtol=1e-13)
    # the fan is a left-moving characteristic family: x/t = (beta - c_s)/(1 - beta c_s), c_s = 1/sqrt(d)
    assert np.allclose(x / t, (f["beta"] - 1 / sd) / (1 - f["beta"] / sd), rtol=1e-12, atol=1e-14)
    # its tail joins the plateau (this checks the root P_C)
    tail = sod.solution(d, PL, nL, PR, nR, np.array([(c["w_T"] - 1e-12) * t]), t)     # just inside the fan
    assert abs(tail["P"][0] - c["PC"]) < 1e-10 and abs(tail["beta"][0] - c["beta_C"]) < 1e-10
    assert abs(tail["n"][0] - c["n_I"]) < 1e-10


@pytest.mark.parametrize("d", [2, 3])
def test_global_conservation(d):
    """Over [-X, X] (all waves inside) N^0 and T^00 keep their initial totals and the momentum grows
    by the pressure difference at the two ends, (P_L - P_R) t."""
    c = sod.waves(d, PL, nL, PR, nR)
    X = 2.0
    init = {"N0": (nL + nR) * X, "T00": d * (PL + PR) * X, "T0x": 0.0}
    for t in (0.5, 1.3):
        edges = [-X, c["w_H"] * t, c["w_T"] * t, c["w_C"] * t, c["w_S"] * t, X]
        tot = {"N0": 0.0, "T00": 0.0, "T0x": 0.0}
        for a, b in zip(edges[:-1], edges[1:]):
            for q in tot:
                def dens(x, q=q):
                    f = sod.solution(d, PL, nL, PR, nR, np.array([x]), t)
                    return currents(d, f["n"][0], f["P"][0], f["beta"][0])[q]
                val, err = integrate.quad(dens, a, b, epsabs=1e-14, epsrel=1e-13, limit=200)
                tot[q] += val
        assert abs(tot["N0"] - init["N0"]) < 1e-11 * init["N0"]
        assert abs(tot["T00"] - init["T00"]) < 1e-11 * init["T00"]
        assert abs(tot["T0x"] - (PL - PR) * t) < 1e-11


def test_oracle_lattice_reproduces_app_d():
    """The oracle's RLBM (printed order-3 massless rule, tau = 1/2 + tau_T/T for eta/s = 0.002) on the
    paper's inviscid Sod set-up against the analytic solution at t = 3.0 fm/c: mean absolute errors
    of a few 1e-3 (viscous layers at the shock and the contact) and the plateau speed to 1e-3."""
    import torch
    from oracle import lattice as OL
    from oracle import mj
    from oracle import quadrature as qd
    d, nx, ny, split, steps = 2, 6400, 5, 1600, 300
    k = np.arange(nx)
    left = np.where(k < nx // 2, k, nx - 1 - k) < split
    n = torch.tensor(np.where(left, nL, nR)[None, :] * np.ones((ny, 1)))
    T = torch.tensor(np.where(left, 1.0, 0.475)[None, :] * np.ones((ny, 1)))
    u = torch.zeros((2, ny, nx), dtype=torch.float64)
    tau_T = 0.002 * (d + 1) / mj.ce_shear_ratio(0.0, d) * (197.327 / 400.0) / 0.01
    ol = OL.Lattice(qd.ur_onlattice_2d(3), 0.5, (nx, ny), tau_T=tau_T)
    fs = ol.collide(ol.init(n, T, u))
    for _ in range(steps):
        fs = ol.collide(ol.stream(fs))
    mac = ol.macro(ol.stream(fs))
    x = np.arange(nx // 2) + 0.5 - split
    t = 5.0 * steps
    ref = sod.solution(d, PL, nL, PR, nR, x, t)
    nn = mac["n"][0, : nx // 2].numpy()
    TT = mac["T"][0, : nx // 2].numpy()
    beta = (mac["U"][1] / mac["U"][0])[0, : nx // 2].numpy()
    assert np.mean(np.abs(nn - ref["n"])) < 5e-3
    assert np.mean(np.abs(nn * TT - ref["P"])) < 4e-3
    assert np.mean(np.abs(beta - ref["beta"])) < 4e-3
    c = sod.waves(d, PL, nL, PR, nR)
    third = (c["w_C"] - c["w_T"]) * t / 3          # the plateau's middle third, away from the smoothed corners
    plateau = (x > c["w_T"] * t + third) & (x < c["w_C"] * t - third)
    assert np.max(np.abs(beta[plateau] - c["beta_C"])) < 1e-3 * c["beta_C"]


def test_oracle_3d_run_reproduces_app_d():
    """The oracle's (3+1)-d run of the same inviscid set-up (printed order-3 massless rule of App. H.1,
    288 populations, light crossing sqrt(41) sites per step, 234 steps = 3.0 fm/c; stored every 8th
    site by tests/golden/make_sod3d_profile.py) against the d = 3 solution of App. D: mean absolute
    errors of a few 1e-3, as in two dimensions (measured n 5.4e-3, P 3.0e-3, T 4.1e-3, beta 2.4e-3),
    and the plateau speed to 2.2e-4."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sod3d_eta002_234_profile.json")))
    x = np.array(g["sites"]) + 0.5 - g["split"]
    t = math.sqrt(41.0) * g["steps"]
    ref = sod.solution(3, PL, nL, PR, nR, x, t)
    n, T, b = (np.array(g[k]) for k in ("n", "T", "beta"))
    assert np.mean(np.abs(n - ref["n"])) < 7e-3
    assert np.mean(np.abs(n * T - ref["P"])) < 4e-3
    assert np.mean(np.abs(T - ref["T"])) < 5e-3
    assert np.mean(np.abs(b - ref["beta"])) < 3e-3
    c = sod.waves(3, PL, nL, PR, nR)
    third = (c["w_C"] - c["w_T"]) * t / 3
    plateau = (x > c["w_T"] * t + third) & (x < c["w_C"] * t - third)
    assert plateau.sum() > 20
    assert np.max(np.abs(b[plateau] - c["beta_C"])) < 1e-3 * c["beta_C"]
