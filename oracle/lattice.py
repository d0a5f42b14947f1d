"""The RLBM time step of Sec. 6.2 on a grid, in plain torch float64 on the CPU.

Oracle module (test infrastructure only; see ``oracle/__init__``).

Layout: populations f have shape (Q, ny, nx) in 2D and (Q, nz, ny, nx) in
3D (x fastest); macroscopic fields have the grid shape, four-vectors a
leading (d+1) axis.  The quadrature order of populations is the one documented
in ``oracle.quadrature``.

One time step (Sec. 6.2, the eight numbered operations):
 1. N^a = sum_i f_i p_i^a,  T^ab = sum_i f_i p_i^a p_i^b
 2. eps U^a = T^ab U_b with eps the largest eigenvalue (Landau frame, Sec. 4)
 3. n = U_a N^a
 4. T from the equation of state eps/n = T (G_d(m/T) - 1)
 5. f^eq_i = w_i sum_k a^(k) J^(k)(p_i)
 6. optional external force (Sec. 5.4, scheme B): a constant acceleration g
    acting through the Minkowski force K = p^0 g, K^0 = g . p (so K.p = 0);
    with df^eq/dp^a = -(U_a/T) f^eq the force term of the kinetic equation is
    F^ext_i = -(m/T) (K^a U_a / p_i^0) f^eq_i, and the update subtracts it
    (the kinetic equation carries -F^ext; Sec. 6.2 prints "+ F^ext", read here
    as the same term with the equation's sign, which accelerates the fluid
    along g).
 7. tau: a constant or a per-site field, plus optionally tau_T / T(x), the law that
    keeps eta/s constant for a massless gas with s = (d + 1) n and the lattice shear
    viscosity eta = c_eta P (tau - 1/2) (Sec. 6.2 step 7 leaves the law open; reading:
    tau = 1/2 + (eta/s)(d + 1)/(c_eta T) in lattice units)
 8. f_i(x + v_i dt, t + dt) = (1 - Omega_i) f_i + Omega_i f^eq_i with
    Omega_i = dt p_i^mu U_mu / (p_i^0 tau), dt = 1.
Streaming moves f_i by its displacement delta_i.  For integer delta_i it is
a pure shift (Sec. 6.3: streaming is exact).  For off-lattice rules the
shifted value is read back on the grid by linear interpolation of the
post-collision field at x - delta_i (bilinear in 2D, trilinear in 3D); the
paper leaves interpolation schemes aside (Sec. 5.3), so this is a reading.
Boundaries: periodic, or "open" = zero-gradient: a read outside the grid
takes the value of the nearest boundary plane, or "wall": the open read plus
no-slip walls on the first and last plane of the axis, where the collision is
replaced by the local equilibrium at zero flow speed (n and T of the site,
U = (1, 0, ...)), as in the forcing validation of Sec. 8.1; a wall plane may
instead hold a prescribed temperature (the heated and cooled plates of the
thermal-conductivity measurement, Sec. 7.2), keeping the site's own n.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import torch

from . import mj
from .basis import Basis, equilibrium, gram_schmidt
from .quadrature import Quadrature


def eta_matrix(d: int) -> torch.Tensor:
    """Minkowski metric diag(1, -1, ..., -1) (Sec. 3)."""
    e = -torch.eye(d + 1, dtype=torch.float64)
    e[0, 0] = 1.0
    return e


def four_velocity(u: torch.Tensor) -> torch.Tensor:
    """U = gamma (1, u) from the three-velocity u of shape (d, ...), gamma = 1/sqrt(1 - |u|^2)."""
    gamma = 1.0 / torch.sqrt(1.0 - (u * u).sum(0))
    return torch.cat([gamma[None], gamma[None] * u], dim=0)


class Lattice:
    """A lattice with its quadrature, relaxation time and boundary conditions.

    ``extent`` = (nx, ny) or (nx, ny, nz); ``bc`` = per-axis "periodic" or
    "open" in the same order; ``tau`` a float or a tensor of grid shape.
    """

    def __init__(self, quad: Quadrature, tau, extent, bc=None, force=None, tau_T: float = 0.0, wall_T=None):
        self.quad = quad
        self.d = quad.d
        self.m = float(quad.m)
        self.basis: Basis = gram_schmidt(quad, quad.order)
        self.p = torch.as_tensor(quad.p, dtype=torch.float64)          # (Q, d+1)
        self.w = torch.as_tensor(quad.w, dtype=torch.float64)
        self.disp = np.asarray(quad.disp, dtype=np.float64)            # (Q, d)
        self.extent = tuple(int(e) for e in extent)
        self.grid_shape = tuple(reversed(self.extent))
        self.bc = tuple(bc) if bc is not None else ("periodic",) * self.d
        self.tau = tau
        self.eta = eta_matrix(self.d)
        self.force = None if force is None else torch.as_tensor(force, dtype=torch.float64)[: self.d]
        self.tau_T = float(tau_T)
        # per axis (T on the first plane, T on the last plane) of a "wall" axis; 0 = the site's own T
        self.wall_T = tuple(tuple(map(float, w)) for w in wall_T) if wall_T is not None else None

    # -- step 1 -------------------------------------------------------------
    def moments(self, f):
        """N^a = sum_i f_i p_i^a and T^ab = sum_i f_i p_i^a p_i^b (Sec. 6.2, step 1)."""
        N = torch.einsum("ia,i...->a...", self.p, f)
        T = torch.einsum("ia,ib,i...->ab...", self.p, self.p, f)
        return N, T

    # -- step 2 -------------------------------------------------------------
    def landau(self, T):
        """Largest eigenvalue eps and eigenvector U of T^ab U_b = eps U^a (Sec. 6.2, step 2).

        With lowered U_b = eta_bc U^c the problem is M U = eps U for the mixed
        tensor M = T eta.  U is normalised to U^a U_a = 1 with U^0 > 0.
        Returns eps (grid) and U (d+1, grid).
        """
        D = self.d + 1
        grid = T.shape[2:]
        Tm = T.reshape(D, D, -1).permute(2, 0, 1)                       # (S, D, D)
        M = Tm @ self.eta
        evals, evecs = torch.linalg.eig(M)
        k = torch.argmax(evals.real, dim=1)
        eps = evals.real.gather(1, k[:, None])[:, 0]
        v = evecs.gather(2, k[:, None, None].expand(-1, D, 1))[:, :, 0]  # (S, D)
        v = (v / v[:, :1]).real                                          # U^0 component set to 1
        norm = torch.sqrt(torch.einsum("sa,ab,sb->s", v, self.eta, v))
        U = (v / norm[:, None]).T.reshape((D,) + grid)
        return eps.reshape(grid), U

    # -- step 3 -------------------------------------------------------------
    def density(self, N, U):
        """n = U_a N^a (Sec. 6.2, step 3)."""
        return torch.einsum("a...,ab,b...->...", U, self.eta, N)

    # -- step 4 -------------------------------------------------------------
    def temperature(self, eps, n):
        """T from eps/n = T (G_d(m/T) - 1) (Sec. 6.2, step 4; Sec. 3 Eq. eos-ddim)."""
        return mj.temperature_from_energy(eps / n, self.m, self.d)

    # -- steps 1-4 together -------------------------------------------------
    def macro(self, f):
        """Macroscopic fields of the populations f: n, eps, P, T, U, N, T^ab."""
        N, Tt = self.moments(f)
        eps, U = self.landau(Tt)
        n = self.density(N, U)
        T = self.temperature(eps, n)
        return {"n": n, "eps": eps, "P": n * T, "T": T, "U": U, "N": N, "Tab": Tt}

    # -- step 5 -------------------------------------------------------------
    def equilibrium(self, n, T, U):
        """f^eq_i = w_i sum_k a^(k) J^(k)(p_i) (Sec. 6.2, step 5)."""
        return equilibrium(self.basis, n, T, U)

    def tau_at(self, like):
        if isinstance(self.tau, torch.Tensor):
            return self.tau.to(torch.float64)
        return torch.full(like.shape, float(self.tau), dtype=torch.float64)

    # -- steps 7-8 (collision) ------------------------------------------------
    def omega(self, U, tau):
        """Omega_i = dt p_i^mu U_mu / (p_i^0 tau) with dt = 1 (Sec. 6.2, step 8)."""
        pU = torch.einsum("ia,ab,b...->i...", self.p, self.eta, U)
        shape = (-1,) + (1,) * (pU.dim() - 1)
        return pU / (self.p[:, 0].reshape(shape) * tau)

    def forcing(self, T, U, feq):
        """F^ext_i = -(m/T) (K^a U_a / p_i^0) f^eq_i with K = (g . p_i, p_i^0 g) (Sec. 5.4, scheme B)."""
        g = self.force
        Kdot = torch.einsum("ia,a->i", self.p[:, 1:], g)                  # K^0 = g . p
        KU = Kdot.reshape((-1,) + (1,) * (U.dim() - 1)) * U[0] - \
            self.p[:, 0].reshape((-1,) + (1,) * (U.dim() - 1)) * torch.einsum("a,a...->...", g, U[1:])[None]
        return -(self.m / T)[None] * KU / self.p[:, 0].reshape((-1,) + (1,) * (U.dim() - 1)) * feq

    def wall_mask(self, grid_shape):
        """Sites on the first and last plane of every "wall" axis."""
        mask = torch.zeros(grid_shape, dtype=torch.bool)
        for ax in range(self.d):
            if self.bc[ax] == "wall":
                dim = len(grid_shape) - 1 - ax
                idx = [slice(None)] * len(grid_shape)
                idx[dim] = 0
                mask[tuple(idx)] = True
                idx[dim] = grid_shape[dim] - 1
                mask[tuple(idx)] = True
        return mask

    def collide(self, f, tau=None):
        """f*_i = f_i + Omega_i (f^eq_i - f_i) - F^ext_i at every site of ``f`` (shape (Q, ...));
        wall sites take the local equilibrium at rest."""
        mac = self.macro(f)
        feq = self.equilibrium(mac["n"], mac["T"], mac["U"])
        if tau is None:
            tau = self.tau_at(mac["n"])
            if self.tau_T != 0.0:                  # step 7: tau from the local temperature
                tau = tau + self.tau_T / mac["T"]
        Om = self.omega(mac["U"], tau)
        out = f + Om * (feq - f)
        if self.force is not None and self.m > 0.0:
            out = out - self.forcing(mac["T"], mac["U"], feq)
        if "wall" in self.bc:
            mask = self.wall_mask(f.shape[1:])
            if mask.any():
                rest = torch.zeros_like(mac["U"])
                rest[0] = 1.0
                Tw = mac["T"].clone()
                if self.wall_T is not None:
                    for ax in range(self.d):
                        if self.bc[ax] != "wall":
                            continue
                        dim = Tw.dim() - 1 - ax
                        for end, Tset in zip((0, Tw.shape[dim] - 1), self.wall_T[ax]):
                            if Tset > 0.0:
                                idx = [slice(None)] * Tw.dim()
                                idx[dim] = end
                                Tw[tuple(idx)] = Tset
                feq0 = self.equilibrium(mac["n"], Tw, rest)
                out = torch.where(mask[None], feq0, out)
        return out

    # -- streaming ----------------------------------------------------------
    def _gather(self, a, offset):
        """a(x + offset) on the grid (axes ordered x, y[, z]) with the lattice's boundary conditions."""
        out = a
        for ax, o in enumerate(offset):
            o = int(o)
            if o == 0:
                continue
            dim = a.dim() - 1 - ax
            nax = a.shape[dim]
            if self.bc[ax] == "periodic":
                out = torch.roll(out, shifts=-o, dims=dim)
            else:                                   # "open" and "wall" read the nearest plane
                idx = torch.clamp(torch.arange(nax) + o, 0, nax - 1)
                out = torch.index_select(out, dim, idx)
        return out

    def stream(self, fstar):
        """f_i(x, t+1) = f*_i(x - delta_i, t), read back by multilinear interpolation."""
        out = torch.empty_like(fstar)
        for i in range(fstar.shape[0]):
            s = -self.disp[i]
            base = np.floor(s)
            frac = s - base
            acc = torch.zeros_like(fstar[i])
            for corner in itertools.product((0, 1), repeat=self.d):
                wgt = 1.0
                for ax in range(self.d):
                    wgt *= frac[ax] if corner[ax] else 1.0 - frac[ax]
                if wgt == 0.0:
                    continue
                acc = acc + wgt * self._gather(fstar[i], base + np.array(corner))
            out[i] = acc
        return out

    # -- the lattice's own shear viscosity ----------------------------------
    def shear_coefficient(self) -> float:
        """c_eta with eta = c_eta P (tau - 1/2): the first-order (Chapman-Enskog) shear stress of this
        discrete update in the rest frame at n = T = 1.

        The relaxation of Sec. 6.2 (step 8) leaves, to first order in the gradients, the non-equilibrium
        part f1_i = -tau' p_i^a d_a f^eq_i / (p_i . U); for a shear flow u_x(y) it is
        -tau' (p_i^y / p_i^0) (d f^eq_i / d u_x) d_y u_x, and pi^xy = sum_i f1_i p_i^x p_i^y, so
            c_eta = sum_i (d f^eq_i / d u_x) p_i^x (p_i^y)^2 / p_i^0 / (n T),
        with tau' = tau - 1/2 on the lattice (the step's dt/2 shift).  The derivative is that of this
        rule's projected equilibrium (step 5), by autograd.  For the continuum Maxwell-Juettner
        distribution (d f / d u_x = f p^x / T at rest) the same sum is the App. C coefficient f_CE;
        a rule that cannot integrate the non-polynomial p^x^2 p^y^2 / p^0 moment of f^eq exactly has
        its own value.  This is the coefficient of the xy shear (a flow u_x(y), as in Poiseuille flow);
        a rule whose fourth-rank moments are not isotropic has another one for the normal-stress
        strain d_x u_x - d_y u_y of the Taylor-Green vortex.
        """
        ux = torch.zeros((), dtype=torch.float64, requires_grad=True)
        g = 1.0 / torch.sqrt(1.0 - ux * ux)
        U = torch.stack([g, g * ux] + [torch.zeros((), dtype=torch.float64)] * (self.d - 1))
        shape = (1,) * self.d
        one = torch.ones(shape, dtype=torch.float64)
        feq = self.equilibrium(one, one, U.reshape((-1,) + shape)).reshape(self.quad.Q)
        p = self.p
        weight = p[:, 1] * p[:, 2] ** 2 / p[:, 0]
        (dfeq,) = torch.autograd.grad((feq * weight).sum(), ux)
        return float(dfeq)

    # -- whole step ---------------------------------------------------------
    def step(self, f):
        """Collide, then stream (Sec. 6.2, step 8)."""
        return self.stream(self.collide(f))

    def run(self, f, nsteps: int):
        for _ in range(nsteps):
            f = self.step(f)
        return f

    # -- initial condition --------------------------------------------------
    def init(self, n, T, u, noise=None, amp: float = 0.0):
        """f_i(x, 0) = f^eq_i(n, T, U) (Sec. 6.2), times (1 + amp * noise_i) when noise is given."""
        U = four_velocity(u.to(torch.float64))
        f = self.equilibrium(n.to(torch.float64), T.to(torch.float64), U)
        if noise is not None:
            f = f * (1.0 + amp * noise.to(torch.float64))
        return f
