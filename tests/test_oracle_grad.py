"""Pins of the oracle's reverse-mode gradient against central finite differences.

Finite differences of the plain forward oracle (no autograd involved) along
seeded directions; the gradient must match to the FD truncation error.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import grad as G
from oracle import lattice as OL
from oracle import quadrature as qd


def setup(nx=10, ny=8, zeta=1.0, order=3, seed=4):
    q = qd.product_2d(zeta, order)
    lat = OL.Lattice(q, 0.8, (nx, ny))
    n, T, u = W.taylor_green_2d(nx, ny, 0.1, density_sigma=1e-3, seed=2)
    g = np.random.default_rng(seed)
    tau = torch.tensor(0.8 + 0.2 * g.uniform(-1, 1, (ny, nx)))
    _, _, ut = W.taylor_green_2d(nx, ny, 0.08, phase=(0.3, -0.2))
    return lat, torch.tensor(n), torch.tensor(T), torch.tensor(u), tau, torch.tensor(ut)


def loss_plain(lat, n, T, u, tau, nsteps, ut):
    """Forward oracle only (eig, bisection): the finite-difference reference."""
    lat.tau = tau
    f = lat.collide(lat.init(n, T, u))
    for _ in range(nsteps):
        f = lat.collide(lat.stream(f))
    mac = lat.macro(lat.stream(f))
    return G.velocity_loss(mac, ut).item()


def test_differentiable_forward_matches_plain_forward():
    lat, n, T, u, tau, ut = setup()
    mac = G.run(lat, n, T, u, tau, 3)
    L1 = G.velocity_loss(mac, ut).item()
    L0 = loss_plain(lat, n, T, u, tau, 3, ut)
    assert abs(L1 - L0) / abs(L0) < 1e-13


@pytest.mark.parametrize("nsteps", [1, 4])
def test_gradient_matches_central_differences(nsteps):
    lat, n, T, u, tau, ut = setup()
    L, gtau, gu0 = G.gradient(lat, n, T, u, tau, nsteps, ut)
    g = np.random.default_rng(11)
    for _ in range(2):
        dtau = torch.tensor(g.normal(size=tau.shape))
        du = torch.tensor(g.normal(size=u.shape)) * 0.1
        h = 1e-5
        Lp = loss_plain(lat, n, T, u + h * du, tau + h * dtau, nsteps, ut)
        Lm = loss_plain(lat, n, T, u - h * du, tau - h * dtau, nsteps, ut)
        fd = (Lp - Lm) / (2 * h)
        an = (gtau * dtau).sum().item() + (gu0 * du).sum().item()
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-12, (fd, an)


def test_eigenpair_derivative_against_perturbation():
    """d eps / d T^ab = U_a U_b (lowered), a closed form of first-order perturbation theory."""
    lat, n, T, u, tau, ut = setup(nx=3, ny=2)
    f = lat.init(n, T, u)
    _, Tt = lat.moments(f)
    Tt = Tt.clone().requires_grad_(True)
    eps, U = G.landau_diff(lat, Tt)
    g = torch.autograd.grad(eps[0, 0], Tt)[0][:, :, 0, 0]
    Ul = (lat.eta @ U[:, 0, 0]).detach()
    assert torch.allclose(g, torch.outer(Ul, Ul), atol=1e-13)
