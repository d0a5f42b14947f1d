"""Maxwell-Juettner integrals, equation of state and transport coefficients.

Oracle module (test infrastructure only; see ``oracle/__init__``).

Natural lattice units throughout: c = k_B = 1 and the reference temperature
T0 = 1, so the reduced mass m~ = m c^2/(k_B T0) is simply ``m`` and the local
relativistic parameter is zeta = m/T (Sec. 3, definition of zeta in Sec. 2).

Sources in the paper:
* A_n coefficients and the tensor integrals Z^{a1..an}: App. B.1.
* Normalisation B(n,T) of the equilibrium: Sec. 3, Eq. (phys-normalization).
* G_d and the equation of state: Sec. 3, Eqs. (defG), (eos-ddim), and the
  limits (ultra-relativistic-eos) and eps_c = (d/2) P.
* Chapman-Enskog shear viscosity eta = P tau a_43, thermal conductivity
  lambda = n tau G (a_22 G - 1) and bulk viscosity mu: App. C (explicit d = 2
  and d = 3 forms), with Gamma(0, x) and the Bickley-Naylor function Ki_1
  as defined at the end of App. B.
"""
from __future__ import annotations

import math

import numpy as np
import torch
from scipy import integrate, special


# ---------------------------------------------------------------------------
# A_n ratios and G_d
# ---------------------------------------------------------------------------

def reverse_bessel_poly(n: int, z):
    """theta_n(z) = sum_k (n+k)! / ((n-k)! k! 2^k) z^(n-k).

    Textbook identity used for even d (App. E remarks that half-integer order
    Bessel functions reduce to reverse Bessel polynomials):
        z^(n+1/2) K_{n+1/2}(z) = sqrt(pi/2) e^{-z} theta_n(z).
    Works on python floats, numpy arrays and torch tensors.
    """
    out = 0.0
    for k in range(n + 1):
        c = math.factorial(n + k) / (math.factorial(n - k) * math.factorial(k) * 2 ** k)
        out = out + c * z ** (n - k)
    return out


def a_ratio(n: int, zeta, d: int):
    """A_n / A_1 with A_n = 2^{(d+1)/2} pi^{(d-1)/2} zeta^{n+(d-1)/2} K_{n+(d-1)/2}(zeta)  (App. B.1).

    The constant prefactor cancels, leaving zeta^{n-1} K_{n+(d-1)/2} / K_{(d+1)/2}.
    * d = 2: theta_n(zeta) / theta_1(zeta) (exact; differentiable in torch).
    * other d: scipy's exponentially scaled K_nu (float64, no autograd); at
      zeta = 0 the massless limit 2^{n-1} Gamma(n+(d-1)/2) / Gamma((d+1)/2).
    """
    if d == 2:
        return reverse_bessel_poly(n, zeta) / reverse_bessel_poly(1, zeta)
    was_torch = isinstance(zeta, torch.Tensor)
    z = zeta.detach().cpu().numpy() if was_torch else np.asarray(zeta, dtype=np.float64)
    nu_n = n + 0.5 * (d - 1)
    nu_1 = 1 + 0.5 * (d - 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = z ** (n - 1) * special.kve(nu_n, z) / special.kve(nu_1, z)
    lim = 2.0 ** (n - 1) * math.gamma(nu_n) / math.gamma(nu_1)
    r = np.where(z == 0.0, lim, r)
    if was_torch:
        return torch.as_tensor(r, dtype=torch.float64)
    return r if r.shape else float(r)


def G_d(zeta, d: int):
    """G_d = (eps + P)/P = zeta K_{(d+3)/2}(zeta) / K_{(d+1)/2}(zeta)  (Sec. 3, Eq. defG) = A_2/A_1."""
    return a_ratio(2, zeta, d)


# ---------------------------------------------------------------------------
# Equation of state
# ---------------------------------------------------------------------------

def energy_per_particle(T, m: float, d: int):
    """eps/n = T (G_d(m/T) - 1)   (Sec. 3, Eq. eos-ddim with P = n T)."""
    return T * (G_d(m / T, d) - 1.0)


def temperature_from_energy(e, m: float, d: int, iters: int = 200):
    """Invert eps/n = T (G_d(m/T) - 1) for T (step 4 of the algorithm, Sec. 6.2).

    Plain bisection on the definition (the map T -> eps/n is increasing, its
    slope being the heat capacity c_v > 0, Sec. 3).  The bracket uses
    d/2 <= G_d - 1 - zeta <= d, i.e. the classical and ultra-relativistic
    limits quoted in Sec. 3.  Massless particles: T = eps/(d n) exactly.
    ``e`` is a float64 torch tensor; the result is detached.
    """
    e = torch.as_tensor(e, dtype=torch.float64).detach()
    if m == 0.0:
        return e / d
    lo = 0.25 * (e - m) / d
    hi = 4.0 * (e - m) / d
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        below = energy_per_particle(mid, m, d) < e
        lo = torch.where(below, mid, lo)
        hi = torch.where(below, hi, mid)
    return 0.5 * (lo + hi)


# ---------------------------------------------------------------------------
# Maxwell-Juettner tensor moments (App. B.1)
# ---------------------------------------------------------------------------

def _pairings(positions, k):
    """All ways to pick k disjoint unordered pairs from ``positions``.

    Yields (pairs, rest).  Each distinct term of <U_{n-2k} eta_k> is produced
    exactly once (App. B.1: index permutations that give the same term are
    counted once).
    """
    if k == 0:
        yield [], list(positions)
        return
    if len(positions) < 2 * k:
        return
    first, rest = positions[0], positions[1:]
    # ``first`` stays unpaired
    for pairs, remaining in _pairings(rest, k):
        yield pairs, [first] + remaining
    # ``first`` is paired with one of the later positions
    for j in range(len(rest)):
        partner = rest[j]
        others = rest[:j] + rest[j + 1:]
        for pairs, remaining in _pairings(others, k - 1):
            yield [(first, partner)] + pairs, remaining


def minkowski(a: int, b: int) -> float:
    """eta^{ab} = diag(1, -1, ..., -1)  (Sec. 3 / App. A)."""
    if a != b:
        return 0.0
    return 1.0 if a == 0 else -1.0


def mj_tensor_moment(idx, n, T, U, m: float, d: int):
    """Integral of f^eq p^{idx_1} ... p^{idx_r} d^dp / p^0 for the equilibrium with (n, T, U).

    Combines Z^{a1..ar} of App. B.1,
        Z^{a1..ar} = T^{d+r-1} sum_k (-1)^k A_{r-k} <U_{r-2k} eta_k>,
    with B(n,T) = n / (T^d A_1) from Z^a = T^d A_1 U^a and B Z^a = n U^a
    (Sec. 3, Eq. phys-normalization).  Hence
        r >= 1:  n T^{r-1} sum_k (-1)^k (A_{r-k}/A_1) <U_{r-2k} eta_k>,
        r  = 0:  n (A_0/A_1) / T.
    ``idx`` is a tuple of space-time indices (0 = time).  ``U`` has shape
    (d+1, ...); n and T broadcast against U[0].
    """
    r = len(idx)
    zeta = m / T
    if r == 0:
        return n * a_ratio(0, zeta, d) / T
    total = 0.0
    for k in range(r // 2 + 1):
        term = 0.0
        for pairs, rest in _pairings(list(range(r)), k):
            eta_prod = 1.0
            for (a, b) in pairs:
                eta_prod *= minkowski(idx[a], idx[b])
            if eta_prod == 0.0:
                continue
            u_prod = 1.0
            for pos in rest:
                u_prod = u_prod * U[idx[pos]]
            term = term + eta_prod * u_prod
        total = total + (-1) ** k * a_ratio(r - k, zeta, d) * term
    return n * T ** (r - 1) * total


# ---------------------------------------------------------------------------
# Chapman-Enskog shear viscosity (App. C.1), used only by the physics pins
# ---------------------------------------------------------------------------

def bickley_ki1(x: float) -> float:
    """Ki_1(x) = int_0^inf exp(-x cosh t) / cosh t dt   (definition at the end of App. B)."""
    upper = math.acosh(max(2.0, 745.0 / x))      # beyond this the integrand underflows
    val, _ = integrate.quad(lambda t: math.exp(-x * math.cosh(t)) / math.cosh(t), 0.0, upper,
                            epsabs=0.0, epsrel=2e-13, limit=400)
    return val


def ce_shear_ratio(zeta: float, d: int) -> float:
    """f_CE(zeta) = eta / (P tau) from the Chapman-Enskog expansion (App. C.1, explicit forms).

    d = 2: (2 G - zeta^2 + e^zeta zeta^4 Gamma(0, zeta) / (zeta + 1)) / 8
    d = 3: (3 G - 5 zeta^2 + G zeta^2 - zeta^3 Ki_1 / K_2) / 15
    with G = G_d(zeta).  Both tend to (d+1)/(d+2) as zeta -> 0 (Sec. 4.1).
    """
    z = float(zeta)
    G = float(G_d(z, d))
    if d == 2:
        tail = 0.0 if z == 0.0 else math.exp(z) * z ** 4 * special.exp1(z) / (z + 1.0)
        return (2.0 * G - z * z + tail) / 8.0
    if d == 3:
        tail = 0.0 if z == 0.0 else z ** 3 * bickley_ki1(z) / special.kv(2, z)
        return (3.0 * G - 5.0 * z * z + G * z * z - tail) / 15.0
    raise ValueError("ce_shear_ratio: d must be 2 or 3")


def ce_conductivity_ratio(zeta: float, d: int) -> float:
    """lambda / (n tau) from the Chapman-Enskog expansion (App. C, thermal conductivity, explicit forms):
    d = 2: G (G/2 - 1 - G zeta^2 e^zeta Gamma(0, zeta) / (2 (zeta + 1)));
    d = 3: G (G (5 - G)/3 - 1 + G zeta Ki_1 / (3 K_2)).
    Both tend to (d + 1)/d as zeta -> 0."""
    z = float(zeta)
    G = float(G_d(z, d))
    if d == 2:
        tail = 0.0 if z == 0.0 else z * z * math.exp(z) * special.exp1(z) / (2.0 * (z + 1.0))
        return G * (G / 2.0 - 1.0 - G * tail)
    if d == 3:
        tail = 0.0 if z == 0.0 else z * bickley_ki1(z) / (3.0 * special.kv(2, z))
        return G * (G * (5.0 - G) / 3.0 - 1.0 + G * tail)
    raise ValueError("ce_conductivity_ratio: d must be 2 or 3")


def ce_bulk_ratio(zeta: float, d: int) -> float:
    """mu / (P tau) from the Chapman-Enskog expansion (App. C, bulk viscosity).

    General form: a_43 (1 + 2/d) - X / (X - 1) with X = zeta^2 - G^2 + (d + 2) G and
    a_43 = eta / (P tau) (the shear coefficient, ``ce_shear_ratio``).  d = 2 uses the explicit form
    (z^4 + 3 z^2 + 2 G^3 - 12 G^2 + 18 G - z^2 G^2 + 2 z^2 G) / (4 (-z^2 + G^2 - 4 G + 1))
    + e^z z^4 Gamma(0, z) / (4 (z + 1)), which equals the general one; the printed explicit d = 3
    form does not (it does not vanish as zeta -> 0), so d = 3 uses the general form.
    mu vanishes for massless particles."""
    z = float(zeta)
    if z == 0.0:
        return 0.0
    G = float(G_d(z, d))
    if d == 2:
        num = z ** 4 + 3 * z * z + 2 * G ** 3 - 12 * G * G + 18 * G - z * z * G * G + 2 * z * z * G
        return num / (4.0 * (-z * z + G * G - 4 * G + 1)) + math.exp(z) * z ** 4 * special.exp1(z) / (4.0 * (z + 1.0))
    if d == 3:
        X = z * z - G * G + (d + 2) * G
        return ce_shear_ratio(z, d) * (1.0 + 2.0 / d) - X / (X - 1.0)
    raise ValueError("ce_bulk_ratio: d must be 2 or 3")
