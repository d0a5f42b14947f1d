"""Reverse-mode gradient of a loss through the RLBM run (oracle; test infrastructure only).

torch autograd on the float64 CPU step of ``oracle.lattice``.  Two steps of
the algorithm are solved iteratively / by root finding in the forward pass;
they are made differentiable by one Newton step taken at the converged
solution, whose derivative is the implicit-function derivative:
* Landau frame (Sec. 6.2 step 2): the residual of M U = eps U with the
  normalisation U_a U^a = 1 (M = T eta);
* temperature (step 4): the residual of eps/n = T (G_d(m/T) - 1).
Everything else (moments, density, projected equilibrium, relaxation,
streaming, the initial equilibrium from u0) is plain torch arithmetic.
"""
from __future__ import annotations

import torch

from . import mj
from .lattice import Lattice, four_velocity


def landau_diff(lat: Lattice, T):
    """(eps, U) of T^ab U_b = eps U^a, differentiable in T (shape (D, D, ...))."""
    D = lat.d + 1
    grid = T.shape[2:]
    with torch.no_grad():
        eps0, U0 = lat.landau(T.detach())
    Tm = T.reshape(D, D, -1).permute(2, 0, 1)                  # (S, D, D)
    S = Tm.shape[0]
    eta = lat.eta
    M = Tm @ eta
    u0 = U0.reshape(D, -1).T                                     # (S, D)
    e0 = eps0.reshape(-1)
    eye = torch.eye(D, dtype=torch.float64)
    # residual F = [(M - eps I) U ; (U^T eta U - 1)/2] at the converged point
    F1 = torch.einsum("sab,sb->sa", M - e0[:, None, None] * eye, u0)
    F2 = 0.5 * (torch.einsum("sa,ab,sb->s", u0, eta, u0) - 1.0)
    J = torch.zeros(S, D + 1, D + 1, dtype=torch.float64)
    J[:, :D, :D] = M.detach() - e0[:, None, None] * eye
    J[:, :D, D] = -u0
    J[:, D, :D] = u0 @ eta
    delta = torch.linalg.solve(J, torch.cat([F1, F2[:, None]], dim=1))
    U = (u0 - delta[:, :D]).T.reshape((D,) + grid)
    eps = (e0 - delta[:, D]).reshape(grid)
    return eps, U


def temperature_diff(lat: Lattice, eps, n):
    """T from eps/n = T (G_d(m/T) - 1), differentiable in eps and n."""
    e = eps / n
    T0 = mj.temperature_from_energy(e.detach(), lat.m, lat.d)
    Tr = T0.clone().requires_grad_(True)
    with torch.enable_grad():
        eT = mj.energy_per_particle(Tr, lat.m, lat.d)
        slope = torch.autograd.grad(eT.sum(), Tr)[0]
    return T0 - (eT.detach() - e) / slope


def macro_diff(lat: Lattice, f):
    N, Tt = lat.moments(f)
    eps, U = landau_diff(lat, Tt)
    n = lat.density(N, U)
    T = temperature_diff(lat, eps, n)
    return {"n": n, "eps": eps, "T": T, "U": U}


def collide_diff(lat: Lattice, f, tau):
    mac = macro_diff(lat, f)
    feq = lat.equilibrium(mac["n"], mac["T"], mac["U"])
    Om = lat.omega(mac["U"], tau)
    return f + Om * (feq - f)


def run(lat: Lattice, n0, T0, u0, tau, nsteps: int, noise=None, amp: float = 0.0):
    """Macroscopic fields of F_{T+1} = S(B_T) with B_0 = C(f_0), B_t = C(S(B_{t-1}))."""
    U0 = four_velocity(u0)
    f0 = lat.equilibrium(n0, T0, U0)
    if noise is not None:
        f0 = f0 * (1.0 + amp * noise)
    B = collide_diff(lat, f0, tau)
    for _ in range(nsteps):
        B = collide_diff(lat, lat.stream(B), tau)
    return macro_diff(lat, lat.stream(B))


def velocity_loss(mac, target_u):
    """L = 1/2 sum_x |u(x) - u_target(x)|^2 with u = U^a / U^0 (three-velocity)."""
    U = mac["U"]
    u = U[1:] / U[0]
    return 0.5 * ((u - target_u) ** 2).sum()


def gradient(lat: Lattice, n0, T0, u0, tau, nsteps, target_u, noise=None, amp=0.0):
    """(loss, dL/dtau, dL/du0) by reverse-mode autograd in float64."""
    tau = tau.clone().to(torch.float64).requires_grad_(True)
    u0 = u0.clone().to(torch.float64).requires_grad_(True)
    mac = run(lat, n0.to(torch.float64), T0.to(torch.float64), u0, tau, nsteps, noise, amp)
    L = velocity_loss(mac, target_u)
    gtau, gu0 = torch.autograd.grad(L, [tau, u0])
    return L.detach(), gtau, gu0
