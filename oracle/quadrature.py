"""Quadrature rules for the RLBM (oracle; test infrastructure only).

A rule is the set of discrete momenta p_i = (p_i^0, p_i^1..p_i^d), weights w_i
and displacements delta_i (lattice sites travelled in one time step), see
Sec. 5.3, Eqs. (discrete-momentum-vectors), (ur-discrete-momentum-vectors),
and Sec. 6.1, Eq. (v0dt=dx).  The weights satisfy the orthonormality
conditions of Eq. (mj-orthogonal-conditions) for polynomials up to the
expansion order N, i.e. the rule integrates every polynomial of degree <= 2N
exactly against the weight omega(p^0) ~ exp(-p^0) with measure d^dp/p^0
(normalised so that sum_i w_i = 1, Eq. numerical-normalization-cond).

Population order (shared interface with the library, stated in its header):
shell-major, i = j * n_dirs + k, with the direction list below in which
antipodal directions are adjacent (k, k+1 for even k).  Zero-weight
populations of the printed ultra-relativistic rule are dropped.

Rules:
* ``ur_onlattice_2d``: the printed (2+1)-d massless rules of order 2
  (Sec. 5.3, worked example, and App. H.2 "Order 2") and order 3 (App. H.2
  "Order 3", four shells, used for the Sod tests), stencil
  (+-3,+-4)_FS U (+-5,0)_FS, three energy shells.  Displacements are the
  integer stencil vectors: speed c = 1 means |n_i| = 5 sites per step
  (v0 = 1/5).  Reading of the printed weight list: the main-text values
  w_{1j} = (0, 0, 1.7536e-3) belong to the (+-5,0) group and
  w_{2j} = (8.889e-2, 3.481e-2, 4.219e-4) to the (+-3,+-4) group, the only
  assignment with sum_i w_i = 1; the order-3 list is read the same way (again
  the only normalised assignment).
* ``ur_onlattice_3d``: the printed (3+1)-d massless rule of order 3 (App. H.1, the rule of the 3D
  Sod tube of Sec. 8.2): groups (+-4,+-4,+-3)_FS, (+-5,+-4,0)_FS, (+-6,+-2,+-1)_FS (|n_i|^2 = 41),
  four shells; the printed weights read shell-major with the groups in the listed order within a
  shell (the only normalised assignment that is exact to degree 6).
* ``product_2d`` / ``product_3d``: off-lattice product rules.  The paper names
  off-lattice schemes but does not build them (Sec. 5.3, last paragraphs;
  Sec. 7.3 closing remark); this is the reading used here.  In d = 2,
  d^2p/p^0 = dp^0 dphi, so with x = p^0 - m the radial weight is e^{-x}:
  Gauss-Laguerre nodes x_j (N+1 of them, exact to degree 2N+1) times eight
  equally weighted directions (exact for angular degree <= 7).  In d = 3,
  d^3p/p^0 = |p| dp^0 dOmega, radial weight sqrt(x^2 + 2 m x) e^{-x} (Gauss
  rule from its moments) times 26 directions (+-1,0,0)_FS, (+-1,+-1,0)_FS,
  (+-1,+-1,+-1)_FS with group weights fixed by exactness at degrees 0, 4, 6.
  Displacements: delta_i = v_i n_i / |n_i| with v_i = |p_i| / p_i^0 and
  c dt = dx (one lattice site per step at the speed of light).
* ``massive_onlattice`` (``massive_onlattice_2d``): on-lattice rules for massive particles (Sec. 5.3,
  Eqs. discrete-momentum-vectors, discrete-p0 and quadrature-problem):
  p_i = p_i^0 (1, v0 n_i), p_i^0 = m / sqrt(1 - v0^2 |n_i|^2), n_i integer, one
  weight per full-symmetric group of the stencil.  The weights solve the
  square system of the orthonormality conditions written as exact moments
  sum_i w_i (p^0)^a p^e = int omega (p^0)^a p^e for the invariants of degree
  <= 2N (a in {0, 1}; e even, up to exchange of components); a line search
  in v0 finds the window where all weights are non-negative.  Stencils: the
  second-order example of Sec. 5.3 (29 vectors) and the third-order 45-vector
  stencil and the (3+1)-d 143-vector stencil of the GPU table of Sec. 6.3.
  The right-hand side b is evaluated in closed form at mpmath precision
  (Bessel K in d = 3): the system's condition number (up to ~1e13) would
  amplify a double-rounded b into the weights.  Population order: the groups
  as listed, each group's vectors with first non-zero component positive in
  decreasing lexicographic order, each followed by its opposite; the rest
  vector last.
"""
from __future__ import annotations

import functools
import itertools
import math
from dataclasses import dataclass

import mpmath
import numpy as np

from . import mj

# Printed (2+1)-d ultra-relativistic order-2 rule (Sec. 5.3 worked example and App. H.2).
UR2D_SHELLS = (0.4157745567834790, 2.2942803602790417, 6.2899450829374791)
UR2D_W_34 = (0.0888866262411466, 0.0348147166961551, 0.0004218743543938)   # (+-3,+-4)_FS group
UR2D_W_50 = (0.0, 0.0, 0.0017535654166088)                                  # (+-5, 0)_FS group

# Printed (2+1)-d ultra-relativistic order-3 rule (App. H.2), same stencil, four shells; the printed
# weight list read shell-major with the (+-5,0) group first in each shell (as for order 2).
UR2D3_SHELLS = (0.3225476896193923, 1.7457611011583465, 4.5366202969211279, 9.3950709123011331)
UR2D3_W_50 = (0.0, 0.0410206173754781, 0.0044457884155769, 0.0000616926157132)
UR2D3_W_34 = (0.0753942630427042, 0.0241670278669858, 0.0026380943565871, 0.0000365655303385)

# Printed (3+1)-d ultra-relativistic order-3 rule (App. H.1): the full-symmetric groups of (4,4,3),
# (5,4,0) and (6,2,1), every vector of length sqrt(41) (v0 = 1/sqrt(41), Sec. 8.2), on four energy
# shells (the generalized Gauss-Laguerre nodes with alpha = 1: d^3p/p^0 = |p| d|p| dOmega); the
# printed list read shell-major with the groups in the listed order within each shell.
UR3D3_GROUPS = ((4, 4, 3), (5, 4, 0), (6, 2, 1))
UR3D3_SHELLS = (0.7432919279814314, 2.5716350076462784, 5.7311787516890996, 10.953894312683190)
UR3D3_W = ((0.0, 0.0, 0.0093098040253911),
           (0.0085195569675087, 0.0, 0.0056909667738262),
           (0.0013041770173120, 0.0, 0.0008932820065742),
           (0.0000029126213348, 0.0000338363537565, 0.0000090390475856))   # [shell][group]

DIRS_UR2D = [(3, 4), (-3, -4), (-3, 4), (3, -4), (4, 3), (-4, -3), (-4, 3), (4, -3),
             (5, 0), (-5, 0), (0, 5), (0, -5)]
DIRS_2D = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (-1, 1), (1, -1)]
DIRS_3D = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
           (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
           (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
           (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
           (1, 1, 1), (-1, -1, -1), (1, 1, -1), (-1, -1, 1),
           (1, -1, 1), (-1, 1, -1), (-1, 1, 1), (1, -1, -1)]


# Massive on-lattice stencils: full-symmetric groups, the rest vector first (as listed in Sec. 5.3
# and in the stencils of the GPU benchmark, Sec. 6.3), keyed by (d, order)
MASSIVE_GROUPS = {
    (2, 2): [(0, 0), (1, 0), (1, 1), (2, 1), (2, 2), (3, 1)],
    (2, 3): [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 2), (3, 3), (4, 0)],
    (3, 3): [(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 0, 0), (2, 1, 1), (2, 2, 0), (2, 2, 1), (2, 2, 2),
             (3, 0, 0), (3, 1, 1), (3, 2, 0)],
}
MASSIVE2D_GROUPS = {order: MASSIVE_GROUPS[(2, order)] for order in (2, 3)}


@dataclass
class Quadrature:
    d: int
    m: float            # reduced mass m~ (T0 = 1)
    order: int          # expansion order N the rule supports
    p: np.ndarray       # (Q, d+1) momenta, energy first
    w: np.ndarray       # (Q,) weights
    disp: np.ndarray    # (Q, d) displacement per step, in lattice sites
    on_lattice: bool

    @property
    def Q(self) -> int:
        return self.w.shape[0]


def ur_onlattice_2d(order: int = 2) -> Quadrature:
    """Printed massless (2+1)-d rules (Sec. 5.3 and App. H.2): order 2 (28 non-zero populations) and
    order 3 (44 non-zero populations)."""
    shells, w34, w50 = (UR2D_SHELLS, UR2D_W_34, UR2D_W_50) if order == 2 else \
        (UR2D3_SHELLS, UR2D3_W_34, UR2D3_W_50)
    p, w, disp = [], [], []
    for j, p0 in enumerate(shells):
        for (nx, ny) in DIRS_UR2D:
            wj = w50[j] if nx * ny == 0 else w34[j]
            if wj == 0.0:
                continue
            norm = math.hypot(nx, ny)          # = 5 for every vector of the stencil
            p.append((p0, p0 * nx / norm, p0 * ny / norm))
            w.append(wj)
            disp.append((float(nx), float(ny)))
    return Quadrature(2, 0.0, order, np.array(p), np.array(w), np.array(disp), True)


def ur_onlattice_3d(order: int = 3) -> Quadrature:
    """Printed massless (3+1)-d rule of order 3 (App. H.1): 288 non-zero populations, integer
    displacements n_i of length sqrt(41) (speed of light, v0 = 1/sqrt(41)), p_i = p^0_j (1, n_i/|n_i|).
    Population order: shell-major; within a shell the groups with non-zero weight in the listed order,
    each group in ``fs_group`` order (antipodes adjacent)."""
    if order != 3:
        raise ValueError("the (3+1)-d printed massless rule is built for order 3")
    p, w, disp = [], [], []
    for j, p0 in enumerate(UR3D3_SHELLS):
        for g, gen in enumerate(UR3D3_GROUPS):
            wj = UR3D3_W[j][g]
            if wj == 0.0:
                continue
            for n in fs_group(gen):
                norm = math.sqrt(sum(c * c for c in n))          # sqrt(41) for every vector
                p.append((p0,) + tuple(p0 * c / norm for c in n))
                w.append(wj)
                disp.append(tuple(float(c) for c in n))
    return Quadrature(3, 0.0, order, np.array(p), np.array(w), np.array(disp), True)


def product_2d(m: float, order: int) -> Quadrature:
    """Off-lattice (2+1)-d product rule: Gauss-Laguerre in x = p^0 - m times 8 directions."""
    x, W = np.polynomial.laguerre.laggauss(order + 1)
    p, w, disp = [], [], []
    for j in range(order + 1):
        p0 = m + x[j]
        pm = math.sqrt(x[j] * x[j] + 2.0 * m * x[j])
        v = pm / p0
        for (nx, ny) in DIRS_2D:
            norm = math.hypot(nx, ny)
            ux, uy = nx / norm, ny / norm
            p.append((p0, pm * ux, pm * uy))
            w.append(W[j] / len(DIRS_2D))
            disp.append((v * ux, v * uy))
    return Quadrature(2, float(m), order, np.array(p), np.array(w), np.array(disp), False)


def sphere_average(a: int, b: int, c: int) -> float:
    """Mean of x^a y^b z^c over the unit sphere: (a-1)!!(b-1)!!(c-1)!!/(a+b+c+1)!! for even a, b, c."""
    if a % 2 or b % 2 or c % 2:
        return 0.0

    def dfact(k):
        return 1 if k <= 0 else k * dfact(k - 2)
    return dfact(a - 1) * dfact(b - 1) * dfact(c - 1) / dfact(a + b + c + 1)


def octahedral_group_weights() -> np.ndarray:
    """Per-direction weights of the axis / edge / corner groups of DIRS_3D.

    Chosen so that the 26-point rule reproduces the sphere average of every
    monomial of degree <= 7 (odd ones vanish by symmetry); solved as a
    consistent least-squares system over all even monomials up to degree 6.
    """
    groups = [DIRS_3D[0:6], DIRS_3D[6:18], DIRS_3D[18:26]]
    rows, rhs = [], []
    for deg in (0, 2, 4, 6):
        for (a, b, c) in itertools.product(range(deg + 1), repeat=3):
            if a + b + c != deg:
                continue
            row = []
            for grp in groups:
                s = 0.0
                for n in grp:
                    u = np.array(n, dtype=float) / np.linalg.norm(n)
                    s += u[0] ** a * u[1] ** b * u[2] ** c
                row.append(s)
            rows.append(row)
            rhs.append(sphere_average(a, b, c))
    sol, *_ = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)
    return sol


def radial_gauss_3d(m: float, npts: int, dps: int = 50):
    """Gauss rule for int_0^inf g(x) sqrt(x^2 + 2 m x) e^{-x} dx with ``npts`` nodes.

    Plain construction at ``dps`` decimal digits: moments by mpmath.quad, the
    monic orthogonal polynomial from the Hankel system, its roots as nodes and
    the weights from the moment (Vandermonde) equations.
    """
    with mpmath.workdps(dps):
        mm = mpmath.mpf(m)
        wfun = lambda x: mpmath.sqrt(x * x + 2 * mm * x) * mpmath.exp(-x)
        mu = [mpmath.quad(lambda x, k=k: x ** k * wfun(x), [0, 1, 10, mpmath.inf])
              for k in range(2 * npts)]
        H = mpmath.matrix(npts, npts)
        rhs = mpmath.matrix(npts, 1)
        for i in range(npts):
            for j in range(npts):
                H[i, j] = mu[i + j]
            rhs[i] = -mu[i + npts]
        c = mpmath.lu_solve(H, rhs)                  # pi(x) = x^n + sum_j c_j x^j
        coeffs = [mpmath.mpf(1)] + [c[j] for j in reversed(range(npts))]
        nodes = sorted([mpmath.re(r) for r in mpmath.polyroots(coeffs, maxsteps=200, extraprec=200)])
        V = mpmath.matrix(npts, npts)
        b = mpmath.matrix(npts, 1)
        for k in range(npts):
            for j in range(npts):
                V[k, j] = nodes[j] ** k
            b[k] = mu[k]
        W = mpmath.lu_solve(V, b)
        return np.array([float(v) for v in nodes]), np.array([float(W[j]) for j in range(npts)])


def product_3d(m: float, order: int) -> Quadrature:
    """Off-lattice (3+1)-d product rule: radial Gauss rule times the 26-direction rule."""
    x, W = radial_gauss_3d(m, order + 1)
    W = W / W.sum()
    gw = octahedral_group_weights()
    dir_w = [gw[0]] * 6 + [gw[1]] * 12 + [gw[2]] * 8
    p, w, disp = [], [], []
    for j in range(order + 1):
        p0 = m + x[j]
        pm = math.sqrt(x[j] * x[j] + 2.0 * m * x[j])
        v = pm / p0
        for k, n in enumerate(DIRS_3D):
            u = np.array(n, dtype=float) / np.linalg.norm(n)
            p.append((p0, *(pm * u)))
            w.append(W[j] * dir_w[k])
            disp.append(tuple(v * u))
    return Quadrature(3, float(m), order, np.array(p), np.array(w), np.array(disp), False)


def rest_frame_moment(idx, m: float, d: int) -> float:
    """int omega(p^0) p^{idx} d^dp/p^0 for the weight omega = C exp(-p^0) normalised to 1.

    omega is the rest-frame Maxwell-Juettner at T = T0 = 1 (Sec. 5.2); its
    moments follow from ``mj.mj_tensor_moment`` with U = (1, 0, ..) and the
    density n = A_1/A_0 that makes the zeroth moment equal to one.
    """
    import torch
    U = torch.zeros(d + 1, dtype=torch.float64)
    U[0] = 1.0
    T = torch.tensor(1.0, dtype=torch.float64)
    z = torch.tensor(float(m), dtype=torch.float64)
    n = 1.0 / mj.a_ratio(0, z, d) if d == 2 else 1.0 / float(mj.a_ratio(0, float(m), d))
    return float(mj.mj_tensor_moment(tuple(idx), n, T, U, float(m), d))


# ---------------------------------------------------------------------------
# Massive on-lattice rules (Sec. 5.3)
# ---------------------------------------------------------------------------
def fs_group(gen):
    """The full-symmetric group of an integer vector, in the population order of the module header."""
    members = set()
    for perm in itertools.permutations(gen):
        for signs in itertools.product((1, -1), repeat=len(gen)):
            members.add(tuple(a * b for a, b in zip(perm, signs)))
    if members == {(0,) * len(gen)}:
        return [(0,) * len(gen)]
    pos = sorted((n for n in members if next(c for c in n if c != 0) > 0), key=lambda n: tuple(-c for c in n))
    out = []
    for n in pos:
        out.append(n)
        out.append(tuple(-c for c in n))
    return out


def _invariants(order: int, d: int = 2):
    """(a, e_1, .., e_d): the monomials (p^0)^a p^e with every e_k even and e_1 >= e_2 >= ..,
    of degree a + |e| <= 2N; for a rule symmetric under permutations and reflections of the axes
    these are the independent moment conditions."""
    rows = []
    for a in (0, 1):
        for deg in range(0, 2 * order + 1 - a, 2):
            parts = {tuple(sorted(q, reverse=True)) for q in itertools.product(range(0, deg + 1, 2), repeat=d)
                     if sum(q) == deg}
            for e in sorted(parts, reverse=True):
                rows.append((a,) + e)
    return rows


def _dfact(n: int) -> int:
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def rest_frame_moment_mp(a: int, e, m, d: int):
    """The moment of (p^0)^a p^e (e even) of omega = C exp(-p^0) (T0 = 1, normalised to 1) in closed
    form at mpmath precision.  The angular average of n^e over the unit sphere is
    prod (e_k - 1)!! / (|e| + d - 2)!!.  Radial part, k = |e|/2:
      d = 2 (d^2p/p^0 = dp^0 dphi, x = p^0 - m): int_0^inf e^{-x} (m + x)^a (x^2 + 2 m x)^k dx, a
            polynomial in m after binomial expansion;
      d = 3 (d^3p/p^0 = |p| dp^0 dOmega): I_k = int_m^inf e^{-p0} |p|^(2k+1) dp0
            = (2k+1)!!/2^(k+1) (2m)^(k+1) K_{k+1}(m), the a = 1 integral is I_{k+1}/(2k+3)
            (integration by parts), and the normalisation is I_0 = m K_1(m)."""
    m = mpmath.mpf(m)
    k = sum(e) // 2
    ang = mpmath.mpf(1)
    for c in e:
        ang *= _dfact(c - 1)
    ang /= _dfact(sum(e) + d - 2)
    if d == 2:
        rad = mpmath.mpf(0)
        for j in range(k + 1):
            c = mpmath.binomial(k, j) * (2 * m) ** (k - j)
            rad += c * (mpmath.factorial(k + j) if a == 0 else m * mpmath.factorial(k + j) + mpmath.factorial(k + j + 1))
        return ang * rad
    if d != 3:
        raise ValueError("d = 2 or 3")

    def I(kk):
        return mpmath.mpf(_dfact(2 * kk + 1)) / 2 ** (kk + 1) * (2 * m) ** (kk + 1) * mpmath.besselk(kk + 1, m)
    rad = I(k) if a == 0 else I(k + 1) / (2 * k + 3)
    return ang * rad / I(0)


def massive_group_weights(m: float, order: int, v0: float, dps: int = 40, d: int = 2):
    """Weights per group (the rest vector first) solving A(v0) w = b (Sec. 5.3), in mpmath at dps
    digits; b holds the exact rest-frame moments (the system is ill conditioned, so b is not rounded
    to double first)."""
    mpmath.mp.dps = dps
    rows, norms, sums = _group_sums(d, order)
    v = mpmath.mpf(v0)
    M = mpmath.mpf(m)
    A = mpmath.matrix(len(rows), len(norms))
    # every member n of group g has p^0_g = m / sqrt(1 - v0^2 |n|^2) and p = p^0_g v0 n, so
    # sum_{n in g} (p^0)^a p^e = (p^0_g)^a (p^0_g v0)^|e| sum_{n in g} n^e
    for g, nn in enumerate(norms):
        p0 = M / mpmath.sqrt(1 - v * v * nn)
        for r, row in enumerate(rows):
            A[r, g] = p0 ** row[0] * (p0 * v) ** sum(row[1:]) * sums[r][g]
    b = mpmath.matrix(_rest_moments(float(m), d, order, dps))
    return [float(x) for x in mpmath.lu_solve(A, b)]


@functools.lru_cache(maxsize=None)
def _rest_moments(m: float, d: int, order: int, dps: int):
    """The right-hand side b of the weight system (independent of v0), at dps digits."""
    mpmath.mp.dps = dps
    return [rest_frame_moment_mp(row[0], row[1:], m, d) for row in _invariants(order, d)]


@functools.lru_cache(maxsize=None)
def _group_sums(d: int, order: int):
    """Invariant rows, |n|^2 per group, and the integer sums sum_{n in g} n^e per (row, group)."""
    groups = [fs_group(g) for g in MASSIVE_GROUPS[(d, order)]]
    rows = _invariants(order, d)
    if len(rows) != len(groups):
        raise ValueError("the stencil must have as many groups as invariants")
    norms = [sum(c * c for c in mem[0]) for mem in groups]
    sums = [[sum(math.prod(c ** ex for c, ex in zip(n, row[1:])) for n in mem) for mem in groups] for row in rows]
    return rows, norms, sums


def massive_feasible_window(m: float, order: int, scan: int = 600, d: int = 2):
    """The v0 interval where every group weight is >= 0 (line search of Sec. 5.3): a scan of
    min_g w_g(v0) over (0, 1/max|n|), golden-section refinement of its maximum, then bisection on
    both sides of the best point."""
    nmax = max(math.sqrt(sum(c * c for c in g)) for g in MASSIVE_GROUPS[(d, order)])
    grid = np.linspace(1e-3, 1.0 / nmax - 1e-4, scan)

    def minw(v):
        return min(massive_group_weights(m, order, v, dps=30, d=d))
    vals = [minw(v) for v in grid]
    k = int(np.argmax(vals))
    lo, hi = grid[max(k - 1, 0)], grid[min(k + 1, scan - 1)]
    # golden-section search for the maximum of min_g w_g on [lo, hi]
    gr = (math.sqrt(5) - 1) / 2
    a, b = lo, hi
    c1, c2 = b - gr * (b - a), a + gr * (b - a)
    f1, f2 = minw(c1), minw(c2)
    for _ in range(60):
        if f1 > f2:
            b, c2, f2 = c2, c1, f1
            c1 = b - gr * (b - a)
            f1 = minw(c1)
        else:
            a, c1, f1 = c1, c2, f2
            c2 = a + gr * (b - a)
            f2 = minw(c2)
    vbest = (a + b) / 2
    if minw(vbest) < 0:
        raise ValueError("no v0 gives non-negative weights for this stencil and mass")

    def edge(inside, outside):
        for _ in range(80):
            mid = (inside + outside) / 2
            if minw(mid) >= 0:
                inside = mid
            else:
                outside = mid
        return inside
    return edge(vbest, lo), edge(vbest, hi)


def massive_onlattice(d: int, m: float, order: int, v0: float = None) -> Quadrature:
    """On-lattice massive (d+1)-dimensional rule (Sec. 5.3); v0 defaults to the middle of the
    feasible window."""
    window = None
    if v0 is None:
        window = massive_feasible_window(m, order, d=d)
        v0 = 0.5 * (window[0] + window[1])
    wg = massive_group_weights(m, order, v0, d=d)
    p, w, disp = [], [], []
    rest = None
    for gen, wgt in zip(MASSIVE_GROUPS[(d, order)], wg):
        for n in fs_group(gen):
            p0 = m / math.sqrt(1.0 - v0 * v0 * sum(c * c for c in n))
            row = ((p0,) + tuple(p0 * v0 * c for c in n), wgt, tuple(float(c) for c in n))
            if not any(n):
                rest = row
            else:
                p.append(row[0]), w.append(row[1]), disp.append(row[2])
    p.append(rest[0]), w.append(rest[1]), disp.append(rest[2])
    q = Quadrature(d, float(m), order, np.array(p), np.array(w), np.array(disp), True)
    q.v0 = float(v0)
    q.window = window
    return q


def massive_onlattice_2d(m: float, order: int, v0: float = None) -> Quadrature:
    return massive_onlattice(2, m, order, v0)
