// precompute.cpp -- host construction of quadratures, basis and tables.
//
// Quadratures (Sec. 5.3; App. H.2 for the printed massless rule):
//  * RLBM_QUAD_UR_ONLATTICE: the printed (2+1)-d rules of orders 2 and 3.
//    Shells and weights are the paper's numbers; the stencil vectors have
//    length 5, so a massless particle crosses 5 sites per step (v0 = 1/5,
//    Sec. 6.1).
//  * RLBM_QUAD_MASSIVE_ONLATTICE: massive on-lattice rules built in
//    massive.cpp (weights from the moment conditions, v0 by line search).
//  * RLBM_QUAD_PRODUCT: off-lattice product rule.  In d = 2 the measure
//    d^2p/p^0 = dp^0 dphi makes the radial weight e^{-(p^0 - m)}: Gauss-Laguerre
//    shells times 8 equally weighted directions.  In d = 3, d^3p/p^0 =
//    |p| dp^0 dOmega: a Gauss rule for sqrt(x^2 + 2 m x) e^{-x} times 26
//    directions with octahedral group weights 1/21, 4/105, 9/280 (exact for
//    spherical harmonics of degree <= 7).  Displacement per step
//    delta_i = p_i / p_i^0 in sites (c dt = dx).
// Gauss rules are computed with the Golub-Welsch method: the eigenvalues of
// the Jacobi matrix of the weight's orthogonal polynomials are the nodes.
#include "precompute.h"

#include <cmath>
#include <cstring>

#include "../../include/rlbm.h"

namespace rlbm {

typedef long double ld;

// ---------------------------------------------------------------------------
// small dense linear algebra (extended precision)
// ---------------------------------------------------------------------------

// Cyclic Jacobi eigenvalue method for a symmetric n x n matrix A (row major,
// destroyed).  Eigenvalues in ev, eigenvectors in the columns of V.
static void jacobi_eig(int n, std::vector<ld> &A, std::vector<ld> &ev, std::vector<ld> &V) {
  V.assign(n * n, 0.0L);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0L;
  for (int sweep = 0; sweep < 100; ++sweep) {
    ld off = 0.0L;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    if (off < 1e-60L) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        ld apq = A[p * n + q];
        if (fabsl(apq) < 1e-300L) continue;
        ld theta = (A[q * n + q] - A[p * n + p]) / (2.0L * apq);
        ld t = (theta >= 0 ? 1.0L : -1.0L) / (fabsl(theta) + sqrtl(theta * theta + 1.0L));
        ld c = 1.0L / sqrtl(t * t + 1.0L), s = t * c;
        for (int k = 0; k < n; ++k) {   // A <- A J
          ld akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {   // A <- J^T A
          ld apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          ld vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  ev.resize(n);
  for (int i = 0; i < n; ++i) ev[i] = A[i * n + i];
}

// Gauss rule from the recurrence coefficients (monic: x pi_k = pi_{k+1} + a_k pi_k + b_k pi_{k-1})
static void golub_welsch(int n, const std::vector<ld> &a, const std::vector<ld> &b, ld mu0,
                         std::vector<ld> &x, std::vector<ld> &w) {
  std::vector<ld> J(n * n, 0.0L), ev, V;
  for (int i = 0; i < n; ++i) {
    J[i * n + i] = a[i];
    if (i + 1 < n) J[i * n + i + 1] = J[(i + 1) * n + i] = sqrtl(b[i + 1]);
  }
  jacobi_eig(n, J, ev, V);
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (ev[order[j]] < ev[order[i]]) std::swap(order[i], order[j]);
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    x[i] = ev[order[i]];
    w[i] = mu0 * V[0 * n + order[i]] * V[0 * n + order[i]];
  }
}

// Gauss-Laguerre: weight x^alpha e^{-x}; a_k = 2k + alpha + 1, b_k = k (k + alpha).
static void gauss_laguerre(int n, ld alpha, std::vector<ld> &x, std::vector<ld> &w) {
  std::vector<ld> a(n), b(n + 1, 0.0L);
  for (int k = 0; k < n; ++k) a[k] = 2.0L * k + alpha + 1.0L;
  for (int k = 1; k <= n; ++k) b[k] = k * (k + alpha);
  golub_welsch(n, a, b, tgammal(alpha + 1.0L), x, w);
}

// Gauss rule for sqrt(x^2 + 2 m x) e^{-x} on [0, inf): Stieltjes procedure on
// a discretised measure.  With x = t^2 the integrand becomes the even,
// analytic function 2 t^2 sqrt(t^2 + 2m) e^{-t^2} g(t^2), for which the
// trapezoidal rule on the half line converges geometrically.
static void gauss_radial_3d(int n, ld m, std::vector<ld> &x, std::vector<ld> &w) {
  if (m == 0.0L) {       // weight x e^{-x}
    gauss_laguerre(n, 1.0L, x, w);
    return;
  }
  ld h = fminl(0.04L, sqrtl(2.0L * m) / 8.0L);
  int M = (int)(14.0L / h) + 1;
  std::vector<ld> xs(M), lam(M);
  for (int k = 1; k <= M; ++k) {
    ld t = k * h;
    xs[k - 1] = t * t;
    lam[k - 1] = h * 2.0L * t * t * sqrtl(t * t + 2.0L * m) * expl(-t * t);
  }
  std::vector<ld> a(n), b(n + 1, 0.0L), pim1(M, 0.0L), pi0(M, 1.0L), pi1(M);
  ld norm_prev = 1.0L, mu0 = 0.0L;
  for (int k = 0; k < n; ++k) {
    ld nrm = 0.0L, xn = 0.0L;
    for (int j = 0; j < M; ++j) {
      nrm += lam[j] * pi0[j] * pi0[j];
      xn += lam[j] * xs[j] * pi0[j] * pi0[j];
    }
    if (k == 0) mu0 = nrm;
    a[k] = xn / nrm;
    b[k] = (k == 0) ? nrm : nrm / norm_prev;
    for (int j = 0; j < M; ++j) pi1[j] = (xs[j] - a[k]) * pi0[j] - (k ? b[k] : 0.0L) * pim1[j];
    pim1.swap(pi0);
    pi0.swap(pi1);
    norm_prev = nrm;
  }
  golub_welsch(n, a, b, mu0, x, w);
}

// Printed massless order-2 rule (Sec. 5.3 example and App. H.2 table):
// shells p^0_j and weights of the (+-3,+-4) and (+-5,0) groups.
static const double kURShells[3] = {0.4157745567834790, 2.2942803602790417, 6.2899450829374791};
static const double kURW34[3] = {0.0888866262411466, 0.0348147166961551, 0.0004218743543938};
static const double kURW50[3] = {0.0, 0.0, 0.0017535654166088};
// Printed massless order-3 rule (App. H.2, (2+1) dimensions, Order 3), the list
// read as for order 2: shell-major, the (+-5,0) group first in each shell.
static const double kUR3Shells[4] = {0.3225476896193923, 1.7457611011583465, 4.5366202969211279,
                                     9.3950709123011331};
static const double kUR3W34[4] = {0.0753942630427042, 0.0241670278669858, 0.0026380943565871, 0.0000365655303385};
static const double kUR3W50[4] = {0.0, 0.0410206173754781, 0.0044457884155769, 0.0000616926157132};

// Printed (3+1)-d massless order-3 rule (App. H.1): generalized Gauss-Laguerre (alpha = 1) shells and
// the twelve printed weights, read shell-major with the groups (4,4,3), (5,4,0), (6,2,1) in that order
// within a shell.
static const double kUR3DShells[4] = {0.7432919279814314, 2.5716350076462784, 5.7311787516890996,
                                      10.953894312683190};
static const double kUR3DW[4][3] = {{0.0, 0.0, 0.0093098040253911},
                                    {0.0085195569675087, 0.0, 0.0056909667738262},
                                    {0.0013041770173120, 0.0, 0.0008932820065742},
                                    {0.0000029126213348, 0.0000338363537565, 0.0000090390475856}};

int build_quadrature(int d, double m, int order, int kind, double v0, QuadHost &q, std::string &err) {
  if (kind == RLBM_QUAD_MASSIVE_ONLATTICE) return build_massive(d, m, order, v0, q, err);
  q = QuadHost();
  q.d = d;
  q.m = m;
  q.order = order;
  q.kind = kind;
  if (kind == RLBM_QUAD_UR_ONLATTICE && d == 3) {
    if (order != 3 || m != 0.0) {
      err = "the printed (3+1)-d on-lattice rule is massless (zeta = 0) of order N = 3";
      return RLBM_ERR_UNSUPPORTED;
    }
    q.nshell = 4;
    q.ndir = kUR3DQ;
    q.Q = kUR3DQ;
    q.v0 = 1.0 / std::sqrt((double)kUR3DNorm2);
    for (int g = 0; g < kUR3DGroups; ++g) {
      const double p0 = kUR3DShells[kUR3DShellOf[g]], wg = kUR3DW[kUR3DShellOf[g]][kUR3DGenOf[g]];
      if (wg == 0.0) {
        err = "internal: zero-weight group in the printed rule";
        return RLBM_ERR_QUADRATURE;
      }
      q.gfirst.push_back(kUR3DDirs.first[g]);
      for (int i = kUR3DDirs.first[g]; i < kUR3DDirs.first[g] + kUR3DDirs.count[g]; ++i) {
        const int *n = kUR3DDirs.v[i];
        q.p.insert(q.p.end(), {p0, p0 * q.v0 * n[0], p0 * q.v0 * n[1], p0 * q.v0 * n[2]});
        q.w.push_back(wg);
        q.disp.insert(q.disp.end(), {(double)n[0], (double)n[1], (double)n[2]});
      }
    }
    return 0;
  }
  if (kind == RLBM_QUAD_UR_ONLATTICE) {
    if (d != 2 || (order != 2 && order != 3) || m != 0.0) {
      err = "the printed on-lattice rules are massless (zeta = 0): d = 2 with order N = 2 or 3, d = 3 with N = 3";
      return RLBM_ERR_UNSUPPORTED;
    }
    q.v0 = 0.2;
    q.nshell = order == 2 ? 3 : 4;
    q.ndir = 12;
    q.Q = order == 2 ? kUR2DQ : kUR3Q;
    for (int i = 0; i < q.Q; ++i) {
      const int j = order == 2 ? kURShell[i] : ur3_shell(i), k = order == 2 ? kURDir[i] : ur3_dir(i);
      double nx = kDirUR[k][0], ny = kDirUR[k][1];
      double len = std::sqrt(nx * nx + ny * ny);   // 5
      double wj = (nx * ny == 0.0) ? (order == 2 ? kURW50[j] : kUR3W50[j]) : (order == 2 ? kURW34[j] : kUR3W34[j]);
      double p0 = order == 2 ? kURShells[j] : kUR3Shells[j];
      if (wj == 0.0) {
        err = "internal: zero-weight population in the printed rule";
        return RLBM_ERR_QUADRATURE;
      }
      q.p.insert(q.p.end(), {p0, p0 * nx / len, p0 * ny / len});
      q.w.push_back(wj);
      q.disp.insert(q.disp.end(), {nx, ny});
    }
    // groups of equal energy and weight (the (+-3,+-4) and (+-5,0) directions of each shell)
    for (int i = 0; i < q.Q; ++i) {
      const int j = order == 2 ? kURShell[i] : ur3_shell(i), k = order == 2 ? kURDir[i] : ur3_dir(i);
      const int jp = i ? (order == 2 ? kURShell[i - 1] : ur3_shell(i - 1)) : -1;
      const int kp = i ? (order == 2 ? kURDir[i - 1] : ur3_dir(i - 1)) : -1;
      if (i == 0 || j != jp || (k >= 8) != (kp >= 8)) q.gfirst.push_back(i);
    }
    return 0;
  }
  if (kind != RLBM_QUAD_PRODUCT) {
    err = "unknown quadrature kind";
    return RLBM_ERR_INVALID_ARG;
  }
  if (!(m >= 0.0) || !std::isfinite(m)) {
    err = "zeta must be finite and >= 0";
    return RLBM_ERR_INVALID_ARG;
  }
  if (order < 2 || order > 3) {
    err = "product rules are provided for orders N = 2 and 3";
    return RLBM_ERR_UNSUPPORTED;
  }
  int nr = order + 1;
  std::vector<ld> x, W;
  if (d == 2) {
    gauss_laguerre(nr, 0.0L, x, W);
  } else if (d == 3) {
    gauss_radial_3d(nr, (ld)m, x, W);
  } else {
    err = "d must be 2 or 3";
    return RLBM_ERR_UNSUPPORTED;
  }
  ld Wsum = 0.0L;
  for (int j = 0; j < nr; ++j) Wsum += W[j];
  q.nshell = nr;
  q.ndir = d == 2 ? 8 : 26;
  for (int j = 0; j < nr; ++j) {
    ld p0 = (ld)m + x[j];
    ld pm = sqrtl(x[j] * x[j] + 2.0L * (ld)m * x[j]);
    ld v = pm / p0;
    for (int k = 0; k < q.ndir; ++k) {
      ld n[3] = {0, 0, 0}, len = 0.0L, dw;
      for (int a = 0; a < d; ++a) {
        n[a] = d == 2 ? kDir2D[k][a] : kDir3D[k][a];
        len += n[a] * n[a];
      }
      len = sqrtl(len);
      if (d == 2) {
        dw = 1.0L / 8.0L;
      } else {
        int nnz = (n[0] != 0) + (n[1] != 0) + (n[2] != 0);
        dw = nnz == 1 ? 1.0L / 21.0L : (nnz == 2 ? 4.0L / 105.0L : 9.0L / 280.0L);
      }
      q.p.push_back((double)p0);
      for (int a = 0; a < d; ++a) q.p.push_back((double)(pm * n[a] / len));
      q.w.push_back((double)(W[j] / Wsum * dw));
      for (int a = 0; a < d; ++a) q.disp.push_back((double)(v * n[a] / len));
    }
  }
  q.Q = nr * q.ndir;
  return 0;
}

// ---------------------------------------------------------------------------
// A_n ratios (App. B): r_n = A_n / A_1 at zeta.  d = 2 through the reverse
// Bessel polynomials theta_n; d = 3 through K_nu computed from
// K_nu(z) = int_0^inf exp(-z cosh t) cosh(nu t) dt (trapezoidal rule).
// ---------------------------------------------------------------------------
static ld bessel_k(ld nu, ld z) {
  // trapezoid rule on K_nu(z) = int_0^inf exp(-z cosh t) cosh(nu t) dt, the integrand being
  // analytic in a strip about the real axis: steps of 0.05 (errors far below long double rounding),
  // and no more than a quarter of the width 1/sqrt(z) of the integrand's peak at large z
  ld tmax = acoshl(fmaxl(2.0L, 11000.0L / z + 1.0L));
  const ld h = fminl(0.05L, 0.25L / sqrtl(z));
  ld s = 0.5L * expl(-z);
  for (int k = 1; k * h <= tmax; ++k) {
    ld t = k * h;
    s += expl(-z * coshl(t)) * coshl(nu * t);
  }
  return s * h;
}

static void a_ratios(int d, ld zeta, ld &r0, ld &r2, ld &r3) {
  if (d == 2) {
    ld t1 = zeta + 1.0L;
    r0 = 1.0L / t1;
    r2 = (zeta * zeta + 3.0L * zeta + 3.0L) / t1;
    r3 = (zeta * zeta * zeta + 6.0L * zeta * zeta + 15.0L * zeta + 15.0L) / t1;
    return;
  }
  // d = 3: A_n/A_1 = zeta^{n-1} K_{n+1}/K_2.  With r = K_1/K_2:
  // r0 = r/zeta, r2 = zeta r + 4 (K_3 = K_1 + 4 K_2/zeta), r3 = zeta^2 + 6 r2.
  if (zeta == 0.0L) {
    r0 = 0.5L;
    r2 = 4.0L;
    r3 = 24.0L;
    return;
  }
  ld r = bessel_k(1.0L, zeta) / bessel_k(2.0L, zeta);
  r0 = r / zeta;
  r2 = zeta * r + 4.0L;
  r3 = zeta * zeta + 6.0L * r2;
}

static inline ld eta(int a, int b) { return a != b ? 0.0L : (a == 0 ? 1.0L : -1.0L); }

// Maxwell-Juettner moment of the monomial with tensor index tuple idx (App. B):
// deg 0: n r0 / T; deg 1: n U^a; deg 2: n T (r2 U^a U^b - eta^ab);
// deg 3: n T^2 (r3 U^a U^b U^c - r2 (eta^ab U^c + eta^ac U^b + eta^bc U^a)).
static ld mj_moment(const signed char *idx, ld n, ld T, const ld *U, ld r0, ld r2, ld r3) {
  int deg = (idx[0] >= 0) + (idx[1] >= 0) + (idx[2] >= 0);
  if (deg == 0) return n * r0 / T;
  if (deg == 1) return n * U[idx[0]];
  int a = idx[0], b = idx[1];
  if (deg == 2) return n * T * (r2 * U[a] * U[b] - eta(a, b));
  int c = idx[2];
  return n * T * T * (r3 * U[a] * U[b] * U[c] - r2 * (eta(a, b) * U[c] + eta(a, c) * U[b] + eta(b, c) * U[a]));
}

template <int D, int N>
static void basis_moments_t(ld m, ld n, ld T, const ld *U, ld *M) {
  ld r0, r2, r3;
  a_ratios(D, m / T, r0, r2, r3);
  for (int k = 0; k < BasisDef<D, N>::NM; ++k) M[k] = mj_moment(BasisDef<D, N>::idx[k], n, T, U, r0, r2, r3);
}

static void basis_moments_ld(int d, int order, ld m, ld n, ld T, const ld *U, ld *M) {
  if (d == 2 && order == 2) basis_moments_t<2, 2>(m, n, T, U, M);
  else if (d == 2 && order == 3) basis_moments_t<2, 3>(m, n, T, U, M);
  else if (d == 3 && order == 2) basis_moments_t<3, 2>(m, n, T, U, M);
  else basis_moments_t<3, 3>(m, n, T, U, M);
}

void basis_moments_host(int d, int order, double m, double n, double T, const double *U, double *M) {
  ld Ul[4] = {0, 0, 0, 0}, Ml[kMaxNM];
  for (int a = 0; a <= d; ++a) Ul[a] = U[a];
  basis_moments_ld(d, order, m, n, T, Ul, Ml);
  for (int k = 0; k < basis_size(d, order); ++k) M[k] = (double)Ml[k];
}

static const signed char *basis_idx(int d, int order, int k) {
  if (d == 2 && order == 2) return BasisDef<2, 2>::idx[k];
  if (d == 2 && order == 3) return BasisDef<2, 3>::idx[k];
  if (d == 3 && order == 2) return BasisDef<3, 2>::idx[k];
  return BasisDef<3, 3>::idx[k];
}
static int basis_ne(int d, int order) {
  if (d == 2) return order == 2 ? BasisDef<2, 2>::NE : BasisDef<2, 3>::NE;
  return order == 2 ? BasisDef<3, 2>::NE : BasisDef<3, 3>::NE;
}

// Moments of the shifted monomials: M[(p^0 - m) p^e] = M[p^0 p^e] - m M[p^e].
static void shift_moments(int d, int order, ld m, ld *M) {
  const int NM = basis_size(d, order);
  for (int k = 0; k < NM; ++k) {
    const signed char *idx = basis_idx(d, order, k);
    int e[3] = {0, 0, 0}, a = 0;
    for (int s = 0; s < 3; ++s)
      if (idx[s] == 0) ++a;
      else if (idx[s] > 0) ++e[idx[s] - 1];
    if (!a) continue;
    for (int l = 0; l < NM; ++l) {
      const signed char *jdx = basis_idx(d, order, l);
      int f[3] = {0, 0, 0}, b = 0;
      for (int s = 0; s < 3; ++s)
        if (jdx[s] == 0) ++b;
        else if (jdx[s] > 0) ++f[jdx[s] - 1];
      if (b == 0 && f[0] == e[0] && f[1] == e[1] && f[2] == e[2]) M[k] -= m * M[l];
    }
  }
}

template <int D, int N>
static void pack_linv(Tables &t) {
  constexpr ClassTable<D, N> CL{};
  static_assert(CL.packed <= kMaxPacked, "packed Linv table too small");
  for (int c = 0; c < 8; ++c)
    for (int i = 0; i < CL.cnt[c]; ++i)
      for (int j = 0; j <= i; ++j) t.LinvP[CL.off[c] + i * (i + 1) / 2 + j] = t.Linv[CL.idx[c][i]][CL.idx[c][j]];
}

// Chebyshev coefficients of f on [-1, 1] (n terms, long double nodes).
template <class F>
static void cheb_fit(int n, F f, double *coef) {
  const ld pi = 3.141592653589793238462643383279502884L;
  ld fk[64];
  for (int k = 0; k < n; ++k) fk[k] = f(cosl(pi * (k + 0.5L) / n));
  for (int j = 0; j < n; ++j) {
    ld c = 0.0L;
    for (int k = 0; k < n; ++k) c += fk[k] * cosl(pi * j * (k + 0.5L) / n);
    c *= 2.0L / n;
    if (j == 0) c *= 0.5L;
    coef[j] = (double)c;
  }
}

static ld cheb_eval(const double *coef, int n, ld s) {
  ld b1 = 0.0L, b2 = 0.0L;
  for (int j = n - 1; j >= 1; --j) {
    ld b0 = 2.0L * s * b1 - b2 + (ld)coef[j];
    b2 = b1;
    b1 = b0;
  }
  return s * b1 - b2 + (ld)coef[0];
}

// The pieces split the variable u in [-1, 1] of the whole range into kEosPieces equal parts: the
// piece of u (u clamped to the range) and u as the local variable s in [-1, 1] of that piece, and
// back.  The kernels evaluate the same map.
static int cheb_piece(ld u, ld &s) {
  u = u < -1.0L ? -1.0L : (u > 1.0L ? 1.0L : u);
  const ld t = (u + 1.0L) * (0.5L * kEosPieces);
  int p = (int)t;
  p = p < 0 ? 0 : (p >= kEosPieces ? kEosPieces - 1 : p);
  s = 2.0L * (t - p) - 1.0L;
  return p;
}
static ld cheb_global(int p, ld s) { return ((s + 1.0L) * 0.5L + p) * (2.0L / kEosPieces) - 1.0L; }

static ld cheb_eval_pieces(const double (*coef)[48], int n, ld u) {
  ld s;
  const int p = cheb_piece(u, s);
  return cheb_eval(coef[p], n, s);
}

// e - m = m (r(m/T) - 1) + 3 T for d = 3 (e = eps/n = T (G_3 - 1), G_3 = z r + 4), with r from
// the long double Bessel functions; its derivative in T is 3 - z^2 r'(z), r' = r^2 + 3 r/z - 1
static ld kinetic_exact(ld m, ld T, ld &dk) {
  const ld z = m / T, r = bessel_k(1.0L, z) / bessel_k(2.0L, z);
  dk = 3.0L - z * z * (r * r + 3.0L * r / z - 1.0L);
  return m * (r - 1.0L) + 3.0L * T;
}

// r(z) = K1/K2 from the fitted series (what the kernels evaluate), and the kinetic energy from it
static ld r_fitted(const Tables &t, ld z) {
  const ld u = (2.0L * logl(z) - ((ld)t.cheb_lo + (ld)t.cheb_hi)) / ((ld)t.cheb_hi - (ld)t.cheb_lo);
  return cheb_eval_pieces(t.cheb, t.cheb_n, u) * z / (z + 2.0L);
}

// the temperature of kinetic energy d per particle.  kinetic(T) increases in T from 1.5 T (cold)
// to 3 T (hot), so the root lies in [d/3, d/1.5]: bisection on the kinetic energy of the fitted r
// (cheap, and good to about 1e-12 where the cold cancellation magnifies the fit's rounding), then
// safeguarded Newton steps on the exact kinetic energy
static ld temperature_exact(const Tables &t, ld m, ld d) {
  ld lo = d / 3.05L, hi = d / 1.45L;
  {
    ld a = fmaxl(lo, (ld)kEosTmin), b = fminl(hi, (ld)kEosTmax);
    for (int it = 0; it < 200 && b - a > 1e-18L * b; ++it) {
      const ld mid = 0.5L * (a + b);
      if (m * (r_fitted(t, m / mid) - 1.0L) + 3.0L * mid < d) a = mid;
      else b = mid;
    }
    lo = fmaxl(lo, 0.5L * (a + b) * (1.0L - 1e-6L));
    hi = fminl(hi, 0.5L * (a + b) * (1.0L + 1e-6L));
  }
  ld T = 0.5L * (lo + hi);
  for (int it = 0; it < 100; ++it) {
    ld dk;
    const ld f = kinetic_exact(m, T, dk) - d;
    if (f < 0.0L) lo = T;
    else hi = T;
    ld Tn = T - f / dk;
    if (!(Tn > lo && Tn < hi)) Tn = 0.5L * (lo + hi);
    const bool done = fabsl(Tn - T) <= 1e-20L * T;
    T = Tn;
    if (done) break;
  }
  return T;
}

int build_eos_fit(double m, Tables &t, std::string &err) {
  t.cheb_n = 0;
  t.chebT_n = 0;
  if (m == 0.0) return 0;
  const int n = kEosTerms;
  const ld tmin = kEosTmin, tmax = kEosTmax;
  // r(z) = K1(z)/K2(z) through h = r (z + 2)/z on log z in [log(m/tmax), log(m/tmin)], by pieces
  const ld lo = logl((ld)m / tmax), hi = logl((ld)m / tmin);
  auto hfun = [&](ld u) {
    const ld z = expl(0.5L * (hi + lo) + 0.5L * (hi - lo) * u);
    return bessel_k(1.0L, z) / bessel_k(2.0L, z) * (z + 2.0L) / z;
  };
  for (int p = 0; p < kEosPieces; ++p) cheb_fit(n, [&](ld s) { return hfun(cheb_global(p, s)); }, t.cheb[p]);
  t.cheb_n = n;
  t.cheb_lo = (double)lo;
  t.cheb_hi = (double)hi;
  for (int k = 0; k <= 64 * kEosPieces; ++k) {
    const ld u = -1.0L + 2.0L * k / (64.0L * kEosPieces), ref = hfun(u);
    if (fabsl(cheb_eval_pieces(t.cheb, n, u) - ref) > 5e-16L * fabsl(ref)) {
      err = "equation-of-state fit failed";
      return RLBM_ERR_QUADRATURE;
    }
  }
  // inverse: T = (e - m) u(x), x = log(e - m), over the same temperature range, fitted to the
  // exact equation of state (the kinetic energy m (r - 1) + 3 T cancels to 1.5 T from terms of
  // size m when cold, so it is taken from the long double Bessel functions, not the fitted r)
  ld dk;
  const ld xlo = logl(kinetic_exact(m, tmin, dk)), xhi = logl(kinetic_exact(m, tmax, dk));
  auto ufun = [&](ld u) {
    const ld d = expl(0.5L * (xhi + xlo) + 0.5L * (xhi - xlo) * u);
    return temperature_exact(t, m, d) / d;
  };
  for (int p = 0; p < kEosPieces; ++p) cheb_fit(n, [&](ld s) { return ufun(cheb_global(p, s)); }, t.chebT[p]);
  t.chebT_n = n;
  t.chebT_lo = (double)xlo;
  t.chebT_hi = (double)xhi;
  for (int k = 0; k <= 64 * kEosPieces; ++k) {
    const ld u = -1.0L + 2.0L * k / (64.0L * kEosPieces), ref = ufun(u);
    if (fabsl(cheb_eval_pieces(t.chebT, n, u) - ref) > 1e-15L * fabsl(ref)) {
      err = "inverse equation-of-state fit failed";
      return RLBM_ERR_QUADRATURE;
    }
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Tables
// ---------------------------------------------------------------------------
int build_tables(const QuadHost &q, double tau, double n_ref, int storage, const int64_t extent[3],
                 const int bc[3], Tables &t, std::string &err) {
  std::memset(&t, 0, sizeof(Tables));
  const int d = q.d, Q = q.Q, D1 = d + 1;
  const int NM = basis_size(d, q.order), NE = basis_ne(d, q.order), NO = NM - NE;
  // an odd population count means a rest population (p = (m, 0)) stored last
  const bool rest = (Q & 1) != 0;
  if (Q > kMaxQ || (rest && q.kind != RLBM_QUAD_MASSIVE_ONLATTICE)) {
    err = "internal: population count";
    return RLBM_ERR_UNSUPPORTED;
  }
  // on-lattice massive rules project over the shifted monomials (p^0 - m)^a p^e
  const bool shifted = q.kind == RLBM_QUAD_MASSIVE_ONLATTICE;
  const ld mshift = shifted ? (ld)q.m : 0.0L;
  t.nx = (int32_t)extent[0];
  t.ny = (int32_t)extent[1];
  t.nz = (int32_t)(d == 3 ? extent[2] : 1);
  for (int a = 0; a < 3; ++a) {
    t.open[a] = (a < d) ? (bc[a] == RLBM_OPEN || bc[a] == RLBM_WALL) : 0;
    t.wall[a] = (a < d) ? (bc[a] == RLBM_WALL) : 0;
  }
  t.storage = storage;
  t.sites = (int64_t)t.nx * t.ny * t.nz;
  t.m = q.m;
  t.tau = tau;
  t.inv_tau = 1.0 / tau;
  t.n_ref = n_ref;

  // Gram matrix of the basis under the discrete inner product, G = sum_i w_i phi phi^T
  std::vector<ld> Phi(Q * NM);
  for (int i = 0; i < Q; ++i)
    for (int k = 0; k < NM; ++k) {
      const signed char *idx = basis_idx(d, q.order, k);
      ld v = 1.0L;
      for (int s = 0; s < 3; ++s)
        if (idx[s] == 0) v *= (ld)q.p[i * D1] - mshift;
        else if (idx[s] > 0) v *= (ld)q.p[i * D1 + idx[s]];
      Phi[i * NM + k] = v;
    }
  std::vector<ld> G(NM * NM, 0.0L);
  for (int i = 0; i < Q; ++i)
    for (int a = 0; a < NM; ++a)
      for (int b = 0; b < NM; ++b) G[a * NM + b] += (ld)q.w[i] * Phi[i * NM + a] * Phi[i * NM + b];
  // Cholesky G = L L^T
  std::vector<ld> L(NM * NM, 0.0L);
  for (int j = 0; j < NM; ++j) {
    ld s = G[j * NM + j];
    for (int k = 0; k < j; ++k) s -= L[j * NM + k] * L[j * NM + k];
    if (!(s > 0.0L)) {
      err = "Gram matrix of the basis is not positive definite: the quadrature cannot carry order N";
      return RLBM_ERR_QUADRATURE;
    }
    L[j * NM + j] = sqrtl(s);
    for (int i = j + 1; i < NM; ++i) {
      ld r = G[i * NM + j];
      for (int k = 0; k < j; ++k) r -= L[i * NM + k] * L[j * NM + k];
      L[i * NM + j] = r / L[j * NM + j];
    }
  }
  // R[i][k] = w_i (G^{-1} phi(p_i))_k : f^eq_i = sum_k R[i][k] M_k reproduces every basis moment
  // (M over the shifted monomials when `shifted`).
  std::vector<ld> R(Q * NM);
  for (int i = 0; i < Q; ++i) {
    std::vector<ld> y(NM);
    for (int a = 0; a < NM; ++a) {
      ld s = Phi[i * NM + a];
      for (int k = 0; k < a; ++k) s -= L[a * NM + k] * y[k];
      y[a] = s / L[a * NM + a];
    }
    for (int a = NM - 1; a >= 0; --a) {
      ld s = y[a];
      for (int k = a + 1; k < NM; ++k) s -= L[k * NM + a] * R[i * NM + k];
      R[i * NM + a] = s / L[a * NM + a];
    }
    for (int a = 0; a < NM; ++a) R[i * NM + a] *= (ld)q.w[i];
  }
  // reproduction check: sum_i R[i][k] phi_l(p_i) = delta_kl
  ld worst = 0.0L;
  for (int k = 0; k < NM; ++k)
    for (int l = 0; l < NM; ++l) {
      ld s = 0.0L;
      for (int i = 0; i < Q; ++i) s += R[i * NM + k] * Phi[i * NM + l];
      worst = fmaxl(worst, fabsl(s - (k == l ? 1.0L : 0.0L)));
    }
  if (worst > 1e-9L) {
    err = "projection does not reproduce the basis moments";
    return RLBM_ERR_QUADRATURE;
  }
  if (rest) {   // the rest population: zero momentum, so its odd row vanishes
    const int i = Q - 1;
    for (int a = 1; a < D1; ++a)
      if (q.p[i * D1 + a] != 0.0) {
        err = "internal: the last population of an odd stencil must be at rest";
        return RLBM_ERR_QUADRATURE;
      }
    for (int k = 0; k < NE; ++k) {
      t.Rrest[k] = (double)R[i * NM + k];
      t.Rrestf[k] = (float)t.Rrest[k];
    }
  }
  // antipodal structure: R[2pr+1] = +-R[2pr] (even / odd basis part)
  for (int pr = 0; pr < Q / 2; ++pr) {
    int i = 2 * pr, j = i + 1;
    for (int a = 1; a < D1; ++a)
      if (std::fabs(q.p[i * D1 + a] + q.p[j * D1 + a]) > 1e-12 * (1.0 + std::fabs(q.p[i * D1 + a]))) {
        err = "internal: populations are not in antipodal pairs";
        return RLBM_ERR_QUADRATURE;
      }
    for (int k = 0; k < NM; ++k) {
      ld s = k < NE ? 1.0L : -1.0L;
      if (fabsl(R[j * NM + k] - s * R[i * NM + k]) > 1e-12L * (1.0L + fabsl(R[i * NM + k]))) {
        err = "internal: projection rows break antipodal symmetry";
        return RLBM_ERR_QUADRATURE;
      }
    }
    const double *p = &q.p[i * D1];
    for (int a = 0; a < d; ++a) {
      t.c[pr][a] = p[1 + a] / p[0];
      t.cf[pr][a] = (float)t.c[pr][a];
    }
    // even moments: N^0 <- p0, T^00 <- p0^2, T^ab <- p^a p^b (a <= b); odd: N^a <- p^a, T^0a <- p0 p^a
    int e = 0;
    t.mom_e[pr][e++] = p[0];
    t.mom_e[pr][e++] = p[0] * p[0];
    for (int a = 1; a <= d; ++a)
      for (int b = a; b <= d; ++b) t.mom_e[pr][e++] = p[a] * p[b];
    int o = 0;
    for (int a = 1; a <= d; ++a) t.mom_o[pr][o++] = p[a];
    for (int a = 1; a <= d; ++a) t.mom_o[pr][o++] = p[0] * p[a];
    for (int k = 0; k < e; ++k) t.mom_ef[pr][k] = (float)t.mom_e[pr][k];
    for (int k = 0; k < o; ++k) t.mom_of[pr][k] = (float)t.mom_o[pr][k];
    for (int k = 0; k < NE; ++k) {
      t.Re[pr][k] = (double)R[i * NM + k];
      t.Ref[pr][k] = (float)t.Re[pr][k];
    }
    for (int k = 0; k < NO; ++k) {
      t.Ro[pr][k] = (double)R[i * NM + NE + k];
      t.Rof[pr][k] = (float)t.Ro[pr][k];
    }
  }
  // interpolation weights: for each non-zero direction component (x, y, z
  // order) a tap bit; sign + : offsets {-1, 0} weights {|d|, 1-|d|};
  // sign - : offsets {0, +1} weights {1-|d|, |d|}.
  if (q.kind == RLBM_QUAD_PRODUCT) {
    for (int i = 0; i < Q; ++i) {
      int k = i % q.ndir;
      int sgn[3], nz = 0, axes[3];
      double mag[3];
      for (int a = 0; a < d; ++a) {
        sgn[a] = d == 2 ? kDir2D[k][a] : kDir3D[k][a];
        mag[a] = std::fabs(q.disp[i * d + a]);
        if (sgn[a] != 0) axes[nz++] = a;
        if (mag[a] > 1.0 + 1e-15) {
          err = "internal: displacement beyond one site";
          return RLBM_ERR_QUADRATURE;
        }
      }
      for (int tap = 0; tap < (1 << nz); ++tap) {
        double wgt = 1.0;
        for (int bI = 0; bI < nz; ++bI) {
          int a = axes[bI], c = (tap >> bI) & 1;
          double mg = std::fmin(mag[a], 1.0);
          if (sgn[a] > 0) wgt *= c ? 1.0 - mg : mg;
          else wgt *= c ? mg : 1.0 - mg;
        }
        t.tapw[i][tap] = wgt;
        t.tapwf[i][tap] = (float)wgt;
      }
    }
  }
  // The kernels evaluate the equilibrium as
  // f^eq_i = w_i psi(p_i)^T G'^{-1} M' over the shifted monomials
  // psi = (p^0 - m)^a p^e (M' the matching moments).  With the kinetic energy
  // p^0 - m instead of p^0 the Gram matrix stays well conditioned for large m
  // (1 and p^0 are nearly collinear over the shells when m >> 1).
  {
    std::vector<ld> Ps(Q * NM);
    for (int i = 0; i < Q; ++i)
      for (int k = 0; k < NM; ++k) {
        const signed char *idx = basis_idx(d, q.order, k);
        ld v = 1.0L;
        for (int s2 = 0; s2 < 3; ++s2)
          if (idx[s2] == 0) v *= (ld)q.p[i * D1] - (ld)q.m;
          else if (idx[s2] > 0) v *= (ld)q.p[i * D1 + idx[s2]];
        Ps[i * NM + k] = v;
      }
    std::vector<ld> Gs(NM * NM, 0.0L), Ls(NM * NM, 0.0L);
    for (int i = 0; i < Q; ++i)
      for (int a = 0; a < NM; ++a)
        for (int b = 0; b < NM; ++b) Gs[a * NM + b] += (ld)q.w[i] * Ps[i * NM + a] * Ps[i * NM + b];
    for (int j = 0; j < NM; ++j) {
      ld sd = Gs[j * NM + j];
      for (int k = 0; k < j; ++k) sd -= Ls[j * NM + k] * Ls[j * NM + k];
      if (!(sd > 0.0L)) {
        err = "shifted Gram matrix is not positive definite";
        return RLBM_ERR_QUADRATURE;
      }
      Ls[j * NM + j] = sqrtl(sd);
      for (int i = j + 1; i < NM; ++i) {
        ld r = Gs[i * NM + j];
        for (int k = 0; k < j; ++k) r -= Ls[i * NM + k] * Ls[j * NM + k];
        Ls[i * NM + j] = r / Ls[j * NM + j];
      }
    }
    // Linv = L^{-1} (lower triangular): the orthonormal polynomials of
    // Sec. 5.2 are J = Linv psi, their projection coefficients a = Linv M'
    for (int c = 0; c < NM; ++c) {
      std::vector<ld> y(NM, 0.0L);
      for (int a = c; a < NM; ++a) {
        ld sd = (a == c) ? 1.0L : 0.0L;
        for (int k = c; k < a; ++k) sd -= Ls[a * NM + k] * y[k];
        y[a] = sd / Ls[a * NM + a];
      }
      for (int a = 0; a < NM; ++a) t.Linv[a][c] = (double)y[a];
    }
    if (d == 2) {
      if (q.order == 2) pack_linv<2, 2>(t);
      else pack_linv<2, 3>(t);
    } else {
      if (q.order == 2) pack_linv<3, 2>(t);
      else pack_linv<3, 3>(t);
    }
  }
  if (!q.gfirst.empty()) {
    // group factors: p = (p0, v n) with v = v0 p0 for every member n of a group (v0 = 1/|n| = 1/5
    // for the printed massless rules)
    const double v0 = q.v0;
    if ((int)q.gfirst.size() > kMaxMassiveGroups) {
      err = "internal: too many groups";
      return RLBM_ERR_UNSUPPORTED;
    }
    for (size_t g = 0; g < q.gfirst.size(); ++g) {
      const int i = q.gfirst[g];
      const ld p0 = (ld)q.p[i * D1], v = (ld)v0 * p0, w = (ld)q.w[i], dl = p0 - (ld)q.m;
      ld f[13] = {p0, p0 * p0, v, p0 * v, v * v};
      ld vl = 1.0L;
      for (int l = 0; l < 4; ++l) {
        f[5 + l] = w * vl;
        f[9 + l] = w * dl * vl;
        vl *= v;
      }
      for (int k = 0; k < 13; ++k) {
        t.mgrp[g][k] = (double)f[k];
        t.mgrpf[g][k] = (float)f[k];
      }
    }
    t.wrest = rest ? q.w[Q - 1] : 0.0;
    t.wrestf = (float)t.wrest;
    t.v0 = v0;
    t.v0f = (float)v0;
  }
  if (q.kind == RLBM_QUAD_PRODUCT) {
    // shell factors: the radial weight W_j is w_i / (direction weight)
    for (int j = 0; j < q.nshell; ++j) {
      const int i = j * q.ndir;                    // direction 0 of shell j is an axis direction
      const double p0 = q.p[i * D1];
      double pm2 = 0.0;
      for (int a = 1; a <= d; ++a) pm2 += q.p[i * D1 + a] * q.p[i * D1 + a];
      const double pm = std::sqrt(pm2);
      const double dirw = d == 2 ? 1.0 / 8.0 : 1.0 / 21.0;
      const double Wj = q.w[i] / dirw;
      t.sv[j] = pm / p0;
      const double sm[5] = {p0, pm, p0 * p0, p0 * pm, pm * pm};
      for (int k = 0; k < 5; ++k) t.smom[j][k] = sm[k];
      for (int a = 0; a < 2; ++a) {
        double f = (d == 2 ? Wj / 8.0 : Wj) * (a ? p0 - q.m : 1.0);
        for (int l = 0; l < 4; ++l) {
          t.sfeq[j][a][l] = f;
          f *= pm;
        }
      }
      t.svf[j] = (float)t.sv[j];
      for (int k = 0; k < 5; ++k) t.smomf[j][k] = (float)t.smom[j][k];
      for (int a = 0; a < 2; ++a)
        for (int l = 0; l < 4; ++l) t.sfeqf[j][a][l] = (float)t.sfeq[j][a][l];
    }
  }
  // reference state f^ref = equilibrium at (n_ref, T = 1, U = 0) and its moments
  {
    ld U[4] = {1.0L, 0.0L, 0.0L, 0.0L}, M[kMaxNM];
    basis_moments_ld(d, q.order, (ld)q.m, (ld)n_ref, 1.0L, U, M);
    for (int k = 0; k < NM; ++k) t.Mref[k] = (double)M[k];   // plain monomials (kernels shift)
    if (shifted) shift_moments(d, q.order, mshift, M);
    ld Nr[4] = {0, 0, 0, 0}, Tr[4][4] = {{0}};
    for (int i = 0; i < Q; ++i) {
      ld f = 0.0L;
      for (int k = 0; k < NM; ++k) f += R[i * NM + k] * M[k];
      t.fref[i] = (double)f;
      t.freff[i] = (float)f;
      for (int a = 0; a < D1; ++a) {
        Nr[a] += f * (ld)q.p[i * D1 + a];
        for (int b = 0; b < D1; ++b) Tr[a][b] += f * (ld)q.p[i * D1 + a] * (ld)q.p[i * D1 + b];
      }
    }
    int s = 0;
    for (int a = 0; a < D1; ++a) {
      t.Nref[a] = (double)Nr[a];
      for (int b = a; b < D1; ++b) t.Tref[s++] = (double)Tr[a][b];
    }
  }
  return 0;
}

}  // namespace rlbm
