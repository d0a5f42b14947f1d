"""Pins of the oracle's special functions, equation of state and Maxwell-Juettner moments.

Each check compares ``oracle.mj`` with something it does not use itself:
scipy / mpmath Bessel functions, limits stated in the paper, or brute-force
numerical integration of the Maxwell-Juettner distribution.
"""
import itertools
import math

import mpmath
import numpy as np
import pytest
import torch
from scipy import integrate, special

from oracle import mj


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("zeta", [1e-3, 0.3, 1.0, 2.5, 5.0, 12.0])
def test_even_d_ratios_match_bessel(n, zeta):
    """d = 2: theta_n / theta_1 equals zeta^{n-1} K_{n+1/2} / K_{3/2} (App. B A_n, App. E remark)."""
    ref = zeta ** (n - 1) * special.kv(n + 0.5, zeta) / special.kv(1.5, zeta)
    got = mj.a_ratio(n, zeta, 2)
    assert got == pytest.approx(ref, rel=1e-13)


def test_massless_limits_of_ratios():
    # zeta -> 0: A_n/A_1 -> 2^{n-1} Gamma(n + (d-1)/2) / Gamma((d+1)/2)
    for n in range(5):
        lim2 = 2.0 ** (n - 1) * math.gamma(n + 0.5) / math.gamma(1.5)
        assert mj.a_ratio(n, 0.0, 2) == pytest.approx(lim2, rel=1e-14)
        assert float(mj.a_ratio(n, 0.0, 3)) == pytest.approx(2.0 ** (n - 1) * math.gamma(n + 1) / math.gamma(2), rel=1e-14)
        assert float(mj.a_ratio(n, 1e-7, 3)) == pytest.approx(2.0 ** (n - 1) * math.gamma(n + 1), rel=1e-5)


def test_bessel_recurrence_sign():
    """App. E prints K_{nu+1} = K_{nu-1} - (2 nu/x) K_nu; the identity holds with a plus sign."""
    for x in (0.4, 1.3, 3.0):
        for nu in (1, 2, 3):
            plus = special.kv(nu - 1, x) + 2 * nu / x * special.kv(nu, x)
            minus = special.kv(nu - 1, x) - 2 * nu / x * special.kv(nu, x)
            assert special.kv(nu + 1, x) == pytest.approx(plus, rel=1e-13)
            assert abs(special.kv(nu + 1, x) - minus) > 0.5 * special.kv(nu + 1, x)


def test_G_closed_forms_and_3d_identity():
    # d = 2: G_2 = (zeta^2 + 3 zeta + 3)/(zeta + 1); d = 3: eps = P (3 + zeta K1/K2) (Sec. 3 Eq. relativistic-eos-3D)
    for z in (0.1, 1.0, 4.0):
        assert mj.G_d(z, 2) == pytest.approx((z * z + 3 * z + 3) / (z + 1), rel=1e-15)
        G3 = float(mj.G_d(z, 3))
        assert G3 - 1 == pytest.approx(3 + z * special.kv(1, z) / special.kv(2, z), rel=1e-13)


@pytest.mark.parametrize("d", [2, 3])
def test_eos_limits(d):
    """zeta -> 0: eps = d P; zeta -> inf: (eps - n m)/P -> d/2 (Sec. 3)."""
    assert float(mj.G_d(0.0, d)) - 1 == pytest.approx(d, rel=1e-14)
    assert float(mj.G_d(1e-6, d)) - 1 == pytest.approx(d, rel=1e-5)
    z = 400.0
    kin = float(mj.G_d(z, d)) - 1 - z          # (eps - n m)/P with P = n T, m/T = zeta
    assert kin == pytest.approx(d / 2, rel=5e-3)


@pytest.mark.parametrize("d,m", [(2, 0.0), (2, 1.0), (2, 5.0), (3, 1.0), (3, 0.3)])
def test_temperature_inversion_roundtrip(d, m):
    T = torch.tensor([0.5, 0.9, 1.0, 1.37, 2.2], dtype=torch.float64)
    e = mj.energy_per_particle(T, m, d)
    T2 = mj.temperature_from_energy(e, m, d)
    assert torch.allclose(T2, T, rtol=2e-15, atol=0)


def test_temperature_2d_quadratic_formula():
    """In d = 2, e = eps/n solves 2T^2 + (2m - e) T + m^2 - e m = 0 (from G_2 above)."""
    m = 1.0
    e = torch.tensor([2.6, 3.0, 4.2], dtype=torch.float64)
    T = mj.temperature_from_energy(e, m, 2)
    closed = ((e - 2 * m) + torch.sqrt(e * e + 4 * e * m - 4 * m * m)) / 4
    assert torch.allclose(T, closed, rtol=1e-14)


# ---------------------------------------------------------------------------
# Maxwell-Juettner moments against brute-force integration
# ---------------------------------------------------------------------------

def _brute_2d(idx, T, U, m):
    """int exp(-U.p/T) p^{idx} d^2p/p^0 with d^2p/p^0 = dp^0 dphi (polar coordinates)."""
    phi = 2 * np.pi * np.arange(256) / 256

    def radial(p0):
        k = math.sqrt(max(p0 * p0 - m * m, 0.0))
        comps = [np.full_like(phi, p0), k * np.cos(phi), k * np.sin(phi)]
        Up = U[0] * p0 - U[1] * comps[1] - U[2] * comps[2]
        val = np.exp(-Up / T)
        for a in idx:
            val = val * comps[a]
        return val.mean() * 2 * np.pi

    out, _ = integrate.quad(radial, m, np.inf, epsabs=0, epsrel=2e-13, limit=500)
    return out


def _brute_3d(idx, T, U, m):
    """Same in d = 3: d^3p/p^0 = |p| dp^0 dOmega; trapezoid in phi, Gauss-Legendre in cos(theta)."""
    phi = 2 * np.pi * np.arange(96) / 96
    ct, wct = np.polynomial.legendre.leggauss(64)
    CT, PH = np.meshgrid(ct, phi, indexing="ij")
    ST = np.sqrt(1 - CT * CT)

    def radial(p0):
        k = math.sqrt(max(p0 * p0 - m * m, 0.0))
        comps = [np.full_like(CT, p0), k * ST * np.cos(PH), k * ST * np.sin(PH), k * CT]
        Up = U[0] * p0 - U[1] * comps[1] - U[2] * comps[2] - U[3] * comps[3]
        val = np.exp(-Up / T)
        for a in idx:
            val = val * comps[a]
        ang = (val.mean(axis=1) * 2 * np.pi * wct).sum()
        return k * ang

    out, _ = integrate.quad(radial, m, np.inf, epsabs=0, epsrel=1e-12, limit=500)
    return out


@pytest.mark.parametrize("d,m,T,u", [(2, 1.0, 1.3, (0.3, -0.2)), (2, 0.0, 0.8, (-0.25, 0.4)),
                                     (3, 1.0, 1.2, (0.2, -0.1, 0.3)), (3, 0.0, 0.9, (-0.3, 0.25, 0.1)),
                                     (3, 5.0, 1.0, (0.1, 0.35, -0.2))])
def test_mj_moments_brute_force(d, m, T, u):
    """App. B closed forms vs direct integration, all index tuples up to degree 3 (in d = 3 too: the
    degree-3 moments of a moving state are what the order-3 equilibrium of the (3+1)-d rules
    projects).

    The density normalisation is taken from the integral itself: n = U_a int f^eq p^a
    with f^eq = B exp(-U.p/T), so nothing of App. B enters the expectation.
    """
    u = np.array(u)
    g = 1 / math.sqrt(1 - u @ u)
    U = np.concatenate([[g], g * u])
    brute = _brute_2d if d == 2 else _brute_3d
    I1 = np.array([brute((a,), T, U, m) for a in range(d + 1)])
    Ulow = U * np.array([1.0] + [-1.0] * d)
    n_target = 0.7
    B = n_target / (Ulow @ I1)
    Ut = torch.tensor(U)
    Tt = torch.tensor(T, dtype=torch.float64)
    nt = torch.tensor(n_target, dtype=torch.float64)
    for deg in (0, 1, 2, 3):
        for idx in itertools.combinations_with_replacement(range(d + 1), deg):
            ref = B * brute(idx, T, U, m)
            got = float(mj.mj_tensor_moment(idx, nt, Tt, Ut, m, d))
            scale = max(1.0, abs(ref))
            assert abs(got - ref) / scale < 5e-10, (idx, got, ref)


def test_ce_shear_limits_and_table2():
    import json, os
    # ultra-relativistic limit (d+1)/(d+2) (Sec. 4.1)
    assert mj.ce_shear_ratio(0.0, 2) == pytest.approx(3 / 4, rel=1e-14)
    assert mj.ce_shear_ratio(0.0, 3) == pytest.approx(4 / 5, rel=1e-14)
    assert mj.ce_shear_ratio(1e-4, 2) == pytest.approx(3 / 4, rel=1e-3)
    # Table 2 of Sec. 7.1 (measured, d = 3) agrees with CE within the paper's 1-2 % systematic error
    path = os.path.join(os.path.dirname(__file__), "golden", "table2_shear_3d.json")
    tab = json.load(open(path))
    devs = []
    for j, z in enumerate(tab["zeta"]):
        ce = mj.ce_shear_ratio(z, 3)
        for row in tab["f"]:
            devs.append(abs(row[j] - ce) / ce)
            assert devs[-1] < 0.02, (z, row[j], ce)
    assert np.median(devs) < 0.005
    # the ultra-relativistic column is 4/5 to the printed digits
    assert all(abs(row[0] - 0.8) < 5e-4 for row in tab["f"])


def test_bickley_against_mpmath():
    for x in (0.5, 1.6, 4.0):
        ref = mpmath.quad(lambda t: mpmath.exp(-x * mpmath.cosh(t)) / mpmath.cosh(t), [0, 2, 4, 8])
        assert mj.bickley_ki1(x) == pytest.approx(float(ref), rel=1e-12)


@pytest.mark.parametrize("d", [2, 3])
def test_ce_conductivity_and_bulk_viscosity(d):
    """App. C: the explicit lambda forms equal the general lambda = n tau G (chi G - 1) with chi from
    a_43 = (G - zeta^2 chi)/(d + 2) = eta / (P tau) (the pinned shear coefficient); the explicit d = 2
    bulk form equals the general mu = P tau [a_43 (1 + 2/d) - X/(X - 1)], X = zeta^2 - G^2 + (d+2) G;
    the massless limits lambda -> (d + 1)/d n tau and mu -> 0; mu > 0 for massive particles."""
    for z in (0.3, 1.0, 2.5, 5.0):
        G = float(mj.G_d(z, d))
        a43 = mj.ce_shear_ratio(z, d)
        chi = (G - (d + 2) * a43) / (z * z)
        assert mj.ce_conductivity_ratio(z, d) == pytest.approx(G * (chi * G - 1.0), rel=1e-11)
        X = z * z - G * G + (d + 2) * G
        general = a43 * (1.0 + 2.0 / d) - X / (X - 1.0)
        assert mj.ce_bulk_ratio(z, d) == pytest.approx(general, rel=1e-9)
        assert mj.ce_bulk_ratio(z, d) > 0
    assert mj.ce_conductivity_ratio(0.0, d) == pytest.approx((d + 1) / d, rel=1e-14)
    assert mj.ce_conductivity_ratio(1e-4, d) == pytest.approx((d + 1) / d, rel=1e-3)
    assert mj.ce_bulk_ratio(1e-3, d) < 1e-5
