"""Pins of the oracle's quadratures, orthonormal basis and discrete equilibrium.

* Exactness of every rule against the Maxwell-Juettner rest-frame moments
  (degree <= 2N), which the paper requires (Sec. 5.3, Eq. mj-orthogonal-conditions).
* The paper's printed rules (golden fixtures): the massless (2+1)-d order-2
  table and the massive m~ = 5 second-order example.
* The numerically built basis / projection against the second-order (2+1)-d
  polynomials and projections printed in App. F and App. G.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import basis as bs
from oracle import mj
from oracle import quadrature as qd

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def max_moment_error(p, w, m, d, degree):
    worst = 0.0
    for idx in itertools.combinations_with_replacement(range(d + 1), degree):
        got = np.sum(w * np.prod([p[:, a] for a in idx], axis=0)) if idx else np.sum(w)
        ref = qd.rest_frame_moment(idx, m, d)
        worst = max(worst, abs(got - ref) / max(1.0, abs(ref)))
    return worst


def test_printed_ur_table_reading():
    """App. H.2 list vs the Sec. 5.3 main-text weights; only one group assignment sums to 1."""
    tab = json.load(open(os.path.join(GOLDEN, "ur_2d_order2_table.json")))
    wl = tab["weights_as_printed"]
    # reading: shell-major, (+-5,0) group first in each shell
    w50 = wl[0::2]
    w34 = wl[1::2]
    assert np.allclose(w50, tab["main_text"]["w_1j"], atol=1e-11)
    assert np.allclose(w34, tab["main_text"]["w_2j"], atol=1e-11)
    assert 4 * sum(w50) + 8 * sum(w34) == pytest.approx(1.0, abs=1e-14)
    # the literal caption order (all shells of the first group, then the second) does not normalise
    literal = 8 * sum(wl[0:3]) + 4 * sum(wl[3:6])
    assert abs(literal - 1.0) > 0.1
    # the shells are the 3-point Gauss-Laguerre nodes (weight e^{-p0}, d^2p/p0 = dp0 dphi)
    x, W = np.polynomial.laguerre.laggauss(3)
    assert np.allclose(tab["shells"], x, rtol=1e-15)
    assert np.allclose([8 * w34[j] + 4 * w50[j] for j in range(3)], W, rtol=1e-13)
    q = qd.ur_onlattice_2d()
    assert q.Q == 28
    expect = sorted([w34[j] for j in range(3) for _ in range(8)] + [w50[2]] * 4)
    assert np.array_equal(np.sort(q.w), np.array(expect))


def test_ur_rule_exact_to_degree_4_only():
    q = qd.ur_onlattice_2d()
    for deg in range(5):
        assert max_moment_error(q.p, q.w, 0.0, 2, deg) < 1e-13
    assert max_moment_error(q.p, q.w, 0.0, 2, 5) > 1e-2
    # on-lattice: every displacement is an integer vector of length 5 (speed of light, v0 = 1/5)
    assert np.all(q.disp == np.round(q.disp))
    assert np.allclose(np.hypot(q.disp[:, 0], q.disp[:, 1]), 5.0)
    # massless: p^0 = |p|
    assert np.allclose(q.p[:, 0], np.hypot(q.p[:, 1], q.p[:, 2]), rtol=1e-15)


def test_printed_massive_rule_m5():
    """Sec. 5.3 example: m~ = 5, v0 = 0.2726, six printed weights -> exact to degree 4 (order 2)."""
    g = json.load(open(os.path.join(GOLDEN, "massive_2d_m5_order2.json")))
    m, v0 = g["m"], g["v0"]
    p, w = [], []
    for grp, wk in zip(g["groups"], g["weights"]):
        a, b = grp
        vecs = set()
        for (x, y) in ((a, b), (b, a)):
            for sx in (1, -1):
                for sy in (1, -1):
                    vecs.add((sx * x, sy * y))
        for (x, y) in sorted(vecs):
            v = v0 * math.hypot(x, y)
            gam = 1 / math.sqrt(1 - v * v)
            p.append((m * gam, m * gam * v0 * x, m * gam * v0 * y))
            w.append(wk)
    p, w = np.array(p), np.array(w)
    assert len(w) == 29
    assert w.sum() == pytest.approx(1.0, abs=1e-13)
    for deg in range(5):
        assert max_moment_error(p, w, m, 2, deg) < 1e-12, deg
    assert max_moment_error(p, w, m, 2, 5) > 1e-6


@pytest.mark.parametrize("m", [0.0, 0.5, 1.0, 5.0])
def test_product_2d_exact_to_degree_7(m):
    q = qd.product_2d(m, 3)
    assert q.Q == 32 and q.w.sum() == pytest.approx(1.0, abs=1e-15)
    for deg in range(8):
        assert max_moment_error(q.p, q.w, m, 2, deg) < 1e-13, deg
    # mass shell and speeds
    assert np.allclose(q.p[:, 0] ** 2 - q.p[:, 1] ** 2 - q.p[:, 2] ** 2, m * m, atol=1e-11)
    speed = np.hypot(q.disp[:, 0], q.disp[:, 1])
    assert np.all(speed < 1.0 + 1e-15)
    # antipodal pairs are adjacent
    assert np.allclose(q.p[0::2, 1:], -q.p[1::2, 1:])


@pytest.mark.parametrize("m", [0.5, 1.0])
def test_product_3d_exact_to_degree_7(m):
    q = qd.product_3d(m, 3)
    assert q.Q == 104 and q.w.sum() == pytest.approx(1.0, abs=1e-14)
    for deg in range(8):
        assert max_moment_error(q.p, q.w, m, 3, deg) < 1e-12, deg
    assert np.allclose(q.p[0::2, 1:], -q.p[1::2, 1:])
    gw = qd.octahedral_group_weights()
    assert np.allclose(gw, [1 / 21, 4 / 105, 9 / 280], rtol=1e-13)


def test_shell_speeds_m1():
    q = qd.product_2d(1.0, 3)
    v = np.hypot(q.disp[::8, 0], q.disp[::8, 1])
    assert np.allclose(v, [0.654, 0.931, 0.984, 0.995], atol=1e-3)


# ---------------------------------------------------------------------------
# Basis and projection
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("rule", ["ur", "p2", "p3"])
def test_basis_orthonormal_and_dimension(rule):
    q = {"ur": qd.ur_onlattice_2d, "p2": lambda: qd.product_2d(1.0, 3), "p3": lambda: qd.product_3d(1.0, 3)}[rule]()
    b = bs.gram_schmidt(q, q.order)
    K = len(b.gens)
    N, d = q.order, q.d
    expect = (N + 1) ** 2 if d == 2 else (N + 1) * (N + 2) * (2 * N + 3) // 6
    assert K == expect
    G = (b.J * q.w) @ b.J.T
    assert np.abs(G - np.eye(K)).max() < 1e-12


def _appFG_2d_feq(p, w, m, n, T, U):
    """f^eq_i = w_i (n/T0) sum_k b^(k) J^(k)(p_i) with App. F / App. G (2+1)-d formulas (T0 = 1)."""
    Gt = m + 1.0                 # G~ = m~ + 1
    G = m / T + 1.0              # G  = zeta + 1
    p0, px, py = p[:, 0], p[:, 1], p[:, 2]
    U0, Ux, Uy = U
    s1 = math.sqrt((2 * m * (m + 3) + 3) / Gt)
    s2 = math.sqrt(3 * Gt + m * m)
    J = [np.ones_like(p0),
         p0 - Gt,
         px / math.sqrt(Gt),
         py / math.sqrt(Gt),
         p0 * (-m - 2) + 0.5 * m * (m + 4) + 0.5 * p0 ** 2 + 1,
         p0 * px * (m + 1) / (Gt * s1) + px * (-m * (m + 3) - 3) / (Gt * s1),
         -p0 ** 2 / (2 * s2) + px ** 2 / s2 + m * m / (2 * s2),
         p0 * py * (m + 1) / (Gt * s1) + py * (-m * (m + 3) - 3) / (Gt * s1),
         px * py / s2]
    b = [1 / (m + T),
         U0 - Gt / (m + T),
         Ux / math.sqrt(Gt),
         Uy / math.sqrt(Gt),
         0.5 * U0 ** 2 * T * (m * m / (G * T * T) + 3) + 0.5 * ((m * (m + 4) + 2) / (m + T) - T) + U0 * (-m - 2),
         U0 * Ux * (m + 1) * T * (m * m / T ** 2 + 3 * G) / (G * Gt * s1) - Ux * (m * (m + 3) + 3) / (Gt * s1),
         -U0 ** 2 * (3 * G * T * T + m * m) / (2 * G * T * s2) + Ux ** 2 * T * (m * m / T ** 2 + 3 * G) / (G * s2)
         + (3 * G * T * T + m * m) / (2 * G * T * s2),
         U0 * Uy * (m + 1) * T * (m * m / T ** 2 + 3 * G) / (G * Gt * s1) - Uy * (m * (m + 3) + 3) / (Gt * s1),
         Ux * Uy * T * (m * m / T ** 2 + 3 * G) / (G * s2)]
    return w * n * sum(bk * Jk for bk, Jk in zip(b, J)), J


@pytest.mark.parametrize("m", [0.5, 1.0, 3.0])
def test_projection_matches_appendix_F_G(m):
    q = qd.product_2d(m, 2)                      # 3 shells x 8 directions, exact to degree 5 >= 2N = 4
    # the printed polynomials are orthonormal under the rule (checks the transcription)
    _, J = _appFG_2d_feq(q.p, q.w, m, 1.0, 1.0, (1.0, 0.0, 0.0))
    Jm = np.array(J)
    assert np.abs((Jm * q.w) @ Jm.T - np.eye(9)).max() < 1e-12
    b = bs.gram_schmidt(q, 2)
    rng = np.random.default_rng(7)
    for _ in range(5):
        n = rng.uniform(0.5, 2.0)
        T = rng.uniform(0.6, 1.8)
        u = rng.uniform(-0.4, 0.4, size=2)
        g = 1 / math.sqrt(1 - u @ u)
        U = (g, g * u[0], g * u[1])
        ref, _ = _appFG_2d_feq(q.p, q.w, m, n, T, U)
        got = bs.equilibrium(b, torch.tensor(n, dtype=torch.float64), torch.tensor(T, dtype=torch.float64),
                             torch.tensor(U, dtype=torch.float64)).numpy()
        assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-13


def test_first_order_ur_limit_sec52():
    """Sec. 5.2, massless first-order polynomials and projections (ultra-relativistic limits):
    J0 = 1, J1_0 = p0/sqrt(d-1) - sqrt(d-1), J1_i = p^i/sqrt(d-1);
    a0 = n/((d-1)T), a1_0 = n (U^0 - 1/T)/sqrt(d-1), a1_i = n U^i/sqrt(d-1).

    Their sum, w_i sum_k a_k J_k, is what the oracle's order-1 projection must give.  The compact
    closed form printed right after them lacks the -p^0/T term that this sum contains; the
    reading kept here is the sum of the printed a_k J_k (checked at rest: it gives f = w n/(d-1)).
    """
    q = qd.ur_onlattice_2d()
    b = bs.gram_schmidt(q, 1)
    d = 2
    n, T = 1.3, 0.9
    U = np.array([0.0, 0.3, -0.2])
    U[0] = math.sqrt(1 + U[1] ** 2 + U[2] ** 2)
    feq = bs.equilibrium(b, torch.tensor(n, dtype=torch.float64), torch.tensor(T, dtype=torch.float64),
                         torch.tensor(U, dtype=torch.float64)).numpy()
    p0, pv = q.p[:, 0], q.p[:, 1:]
    s = math.sqrt(d - 1)
    J = [np.ones_like(p0), p0 / s - s, pv[:, 0] / s, pv[:, 1] / s]
    a = [n / ((d - 1) * T), n * (U[0] - 1 / T) / s, n * U[1] / s, n * U[2] / s]
    ref = q.w * sum(ak * Jk for ak, Jk in zip(a, J))
    assert np.abs(feq - ref).max() < 1e-14
    printed = q.w * n * (d / T + U[0] * p0 - (d - 1) * U[0] + pv @ U[1:]) / (d - 1)
    assert np.allclose(printed - ref, q.w * n * p0 / ((d - 1) * T), atol=1e-14)


def test_massive_solver_reproduces_printed_weights_and_window():
    """The line-search solver of Sec. 5.3 against the printed example: the group weights at
    v0 = 0.2726 and the two v0 where a weight reaches zero (pruning to 25 vectors)."""
    g = json.load(open(os.path.join(GOLDEN, "massive_2d_m5_order2.json")))
    w = qd.massive_group_weights(g["m"], g["order"], g["v0"])
    for got, want in zip(w, g["weights"]):
        assert abs(got - want) < 1e-10 * want, (got, want)
    lo, hi = qd.massive_feasible_window(g["m"], g["order"])
    assert abs(lo - g["pruning_v0"]["w2_zero"]) < 1e-10
    assert abs(hi - g["pruning_v0"]["w3_zero"]) < 1e-10
    wl = qd.massive_group_weights(g["m"], g["order"], lo)
    assert abs(wl[1]) < 1e-8 and min(wl) > -1e-8


def test_massive_third_order_rule():
    """The 45-vector stencil of the GPU table (Sec. 6.3) at m~ = 5: a non-empty window of
    non-negative weights; at its middle the rule is exact to degree 2N = 6 (every monomial, odd
    ones by symmetry) and not to degree 7; integer displacements; antipodal pairs adjacent with
    the rest vector last."""
    q = qd.massive_onlattice_2d(5.0, 3)
    assert q.Q == 45 and q.w.min() > 0 and q.w.sum() == pytest.approx(1.0, abs=1e-13)
    assert 0.2210 < q.v0 < 0.2212
    for deg in range(7):
        assert max_moment_error(q.p, q.w, 5.0, 2, deg) < 1e-11, deg
    assert max_moment_error(q.p, q.w, 5.0, 2, 7) > 1e-6
    assert np.all(q.disp == np.round(q.disp)) and np.abs(q.disp).max() == 4
    assert np.allclose(q.p[0:44:2, 1:], -q.p[1:44:2, 1:]) and np.all(q.disp[44] == 0)
    assert np.allclose(q.p[:, 0] ** 2 - q.p[:, 1] ** 2 - q.p[:, 2] ** 2, 25.0, rtol=1e-13)


@pytest.mark.parametrize("d", [2, 3])
def test_rest_frame_moment_closed_form(d):
    """The closed forms behind the massive weight systems against two other routes: the App. B
    moments (float64, through the A_n ratios), and, split into its factors, brute force: the angular
    average of n^e from the product rule's direction set (exact for angular degree <= 7) or, in 2D,
    an equispaced angle sum; the radial integral by numerical quadrature."""
    import mpmath
    m = 5.0
    mpmath.mp.dps = 30
    for a, e in [(0, (0,) * d), (1, (0,) * d), (0, (2,) + (0,) * (d - 1)), (1, (2, 2) + (0,) * (d - 2)),
                 (0, (4, 2) + (0,) * (d - 2)), (0, (2,) * d), (0, (6,) + (0,) * (d - 1))]:
        idx = (0,) * a + sum(((k + 1,) * c for k, c in enumerate(e)), ())
        got = qd.rest_frame_moment_mp(a, e, m, d)
        assert abs(float(got) / qd.rest_frame_moment(idx, m, d) - 1) < 1e-13, (a, e)
    # factors of the closed form, d = 3
    if d == 3:
        q = qd.product_3d(1.0, 3)
        dirs = q.p[:26, 1:] / np.linalg.norm(q.p[:26, 1:], axis=1)[:, None]
        wdir = q.w[:26] / q.w[:26].sum()
        for e in [(2, 0, 0), (4, 0, 0), (2, 2, 0), (6, 0, 0), (4, 2, 0), (2, 2, 2)]:
            ang = np.sum(wdir * np.prod(dirs ** np.array(e), axis=1))
            want = qd._dfact(e[0] - 1) * qd._dfact(e[1] - 1) * qd._dfact(e[2] - 1) / qd._dfact(sum(e) + 1)
            assert abs(ang - want) < 1e-14
        M = mpmath.mpf(m)
        norm = mpmath.quad(lambda p0: mpmath.e ** (-p0) * mpmath.sqrt(p0 * p0 - M * M), [M, M + 10, mpmath.inf])
        for a, k in [(0, 1), (1, 0), (1, 2), (0, 3)]:
            num = mpmath.quad(lambda p0: mpmath.e ** (-p0) * p0 ** a * (p0 * p0 - M * M) ** (k + mpmath.mpf(1) / 2),
                              [M, M + 10, mpmath.inf]) / norm
            e = (2 * k, 0, 0)
            ang = mpmath.mpf(qd._dfact(2 * k - 1)) / qd._dfact(2 * k + 1)
            assert abs(qd.rest_frame_moment_mp(a, e, m, 3) / ang / num - 1) < 1e-25
    else:
        M = mpmath.mpf(m)
        for a, ex, ey in [(0, 2, 2), (1, 4, 0), (0, 4, 2)]:
            ang = mpmath.fsum(mpmath.cos(2 * mpmath.pi * j / 64) ** ex * mpmath.sin(2 * mpmath.pi * j / 64) ** ey
                              for j in range(64)) / 64
            k = (ex + ey) // 2
            rad = mpmath.quad(lambda p0: mpmath.e ** (M - p0) * p0 ** a * (p0 * p0 - M * M) ** k, [M, M + 10, mpmath.inf])
            assert abs(qd.rest_frame_moment_mp(a, (ex, ey), m, 2) / (ang * rad) - 1) < 1e-25


@pytest.fixture(scope="module")
def massive3d():
    return qd.massive_onlattice(3, 5.0, 3)


def test_massive_3d_rule(massive3d):
    """The 143-vector (3+1)-d stencil of the GPU table (Sec. 6.3) at m~ = 5: a window of non-negative
    weights exists; at its middle the rule is exact to degree 2N = 6 for every monomial and not at
    degree 7; integer displacements up to 3; antipodal pairs adjacent, the rest vector last."""
    q = massive3d
    assert q.Q == 143 and q.w.min() > 0 and q.w.sum() == pytest.approx(1.0, abs=1e-13)
    lo, hi = q.window
    assert lo < q.v0 < hi and 0.2715 < q.v0 < 0.2720
    for deg in range(7):
        assert max_moment_error(q.p, q.w, 5.0, 3, deg) < 1e-11, deg
    assert max_moment_error(q.p, q.w, 5.0, 3, 7) > 1e-6
    assert np.all(q.disp == np.round(q.disp)) and np.abs(q.disp).max() == 3
    assert np.allclose(q.p[0:142:2, 1:], -q.p[1:142:2, 1:]) and np.all(q.disp[142] == 0)
    assert np.allclose(q.p[:, 0] ** 2 - (q.p[:, 1:] ** 2).sum(1), 25.0, rtol=1e-13)
    # at the window's ends one weight vanishes
    for v in (lo, hi):
        assert abs(min(qd.massive_group_weights(5.0, 3, v, d=3))) < 1e-9


def test_printed_ur_order3_rule():
    """App. H.2, (2+1)-d order 3: the shells are the 4-point Gauss-Laguerre nodes, the list read
    shell-major with the (+-5,0) group first normalises (the literal caption order does not), the
    per-shell sums are the Gauss-Laguerre weights, and the rule is exact to degree 2N = 6."""
    tab = json.load(open(os.path.join(GOLDEN, "ur_2d_order3_table.json")))
    wl = tab["weights_as_printed"]
    w50, w34 = wl[0::2], wl[1::2]
    assert 4 * sum(w50) + 8 * sum(w34) == pytest.approx(1.0, abs=1e-14)
    assert abs(8 * sum(wl[0:4]) + 4 * sum(wl[4:8]) - 1.0) > 0.1
    x, W = np.polynomial.laguerre.laggauss(4)
    assert np.allclose(tab["shells"], x, rtol=1e-15)
    assert np.allclose([8 * w34[j] + 4 * w50[j] for j in range(4)], W, rtol=1e-13)
    q = qd.ur_onlattice_2d(3)
    assert q.Q == 44 and q.order == 3
    for deg in range(7):       # the printed 16-digit weights limit the agreement (~7e-13 at degree 6)
        assert max_moment_error(q.p, q.w, 0.0, 2, deg) < 1e-11, deg
    assert max_moment_error(q.p, q.w, 0.0, 2, 7) > 1e-6
    assert np.all(np.abs(np.hypot(q.disp[:, 0], q.disp[:, 1]) - 5.0) == 0)
    assert np.allclose(q.p[0:44:2, 1:], -q.p[1:44:2, 1:])


def test_printed_ur_3d_order3_rule():
    """App. H.1, (3+1)-d order 3: the shells are the 4-point generalized Gauss-Laguerre nodes
    (alpha = 1, from d^3p/p^0 = |p| d|p| dOmega), the twelve printed weights read shell-major with the
    groups in the listed order normalise and integrate every rest-frame moment to degree 2N = 6 (the
    per-shell sums are the normalised Gauss weights); every other group order within a shell, and
    the group-major order, fails one of these; degree 7 is not exact."""
    from scipy.special import roots_genlaguerre
    tab = json.load(open(os.path.join(GOLDEN, "ur_3d_order3_table.json")))
    wl = tab["weights_as_printed"]
    x, W = roots_genlaguerre(4, 1)
    assert np.allclose(tab["shells"], x, rtol=1e-14)
    sizes = [len(qd.fs_group(g)) for g in tab["stencil_groups"]]
    assert sizes == [24, 24, 48]
    q = qd.ur_onlattice_3d(3)
    assert q.Q == 48 + 72 + 72 + 96 and q.order == 3
    assert q.w.sum() == pytest.approx(1.0, abs=1e-13)
    for j in range(4):
        shell = sum(sizes[g] * wl[3 * j + g] for g in range(3))
        assert shell == pytest.approx(W[j] / W.sum(), rel=1e-12)
    for deg in range(7):
        assert max_moment_error(q.p, q.w, 0.0, 3, deg) < 1e-11, deg
    assert max_moment_error(q.p, q.w, 0.0, 3, 7) > 1e-3
    # other readings of the list
    for perm in itertools.permutations(range(3)):
        if perm == (0, 1, 2):
            continue
        tot = sum(sizes[g] * wl[3 * j + slot] for j in range(4) for slot, g in enumerate(perm))
        if abs(tot - 1.0) < 1e-12:          # normalised but not exact
            ws = np.array([wl[3 * j + perm.index(g)] for j in range(4) for g in range(3)
                           if wl[3 * j + perm.index(g)] != 0 for _ in range(sizes[g])])
            pts = np.array([(tab["shells"][j],) + tuple(tab["shells"][j] * c / math.sqrt(41) for c in n)
                            for j in range(4) for g in range(3) if wl[3 * j + perm.index(g)] != 0
                            for n in qd.fs_group(tab["stencil_groups"][g])])
            assert max(max_moment_error(pts, ws, 0.0, 3, d) for d in range(7)) > 1e-3, perm
    group_major = sum(sizes[g] * wl[4 * g + j] for g in range(3) for j in range(4))
    assert abs(group_major - 1.0) > 0.1
    # on-lattice, massless, antipodes adjacent
    assert np.all(q.disp == np.round(q.disp))
    assert np.allclose((q.disp ** 2).sum(1), 41.0)
    assert np.allclose(q.p[:, 0], np.sqrt((q.p[:, 1:] ** 2).sum(1)), rtol=1e-15)
    assert np.allclose(q.p[0::2, 1:], -q.p[1::2, 1:])
