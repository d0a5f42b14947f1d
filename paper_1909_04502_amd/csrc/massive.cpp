// massive.cpp -- massive on-lattice (2+1)-d and (3+1)-d quadratures (Sec. 5.3).
//
// The stencil is a union of full-symmetric groups of integer vectors n; every
// member of a group carries the same weight, and the momenta lie on the mass
// shell with velocities proportional to n: p_i = p^0_i (1, v0 n_i),
// p^0_i = m / sqrt(1 - v0^2 |n_i|^2), so that one time step (1/v0 site
// spacings over c) moves population i by exactly n_i sites.  The weights are
// fixed by requiring that the rule reproduce the rest-frame moments of the
// weight omega(p^0) = C exp(-p^0) (T0 = 1, Sec. 5.2) for every monomial
// (p^0)^a p_x^ex p_y^ey of degree <= 2N: by the symmetry of the groups only
// a in {0, 1}, ex and ey even and ex >= ey remain, as many conditions as
// groups, a square linear system A(v0) w = b.  v0 is the one free parameter;
// the admissible rules are those with all weights >= 0, found by a line
// search over v0 (the paper's procedure).
//
// The system is badly conditioned (condition numbers up to ~1e13 for the
// 45-vector stencil), so it is assembled and solved in binary128
// (__float128, ~34 digits); the weights then carry full double precision.
//
// Rest-frame moments, k = |e|/2, with the angular average of n^e over the unit
// sphere prod (e_a - 1)!! / (|e| + d - 2)!!:
//  d = 2 (d^2p/p^0 = dp^0 dphi, C = e^m / (2 pi)): the radial integral
//    int_0^inf e^{-x} (m+x)^a (x^2 + 2 m x)^k dx (x = p^0 - m); expanding
//    (x^2 + 2 m x)^k binomially leaves int_0^inf x^q e^{-x} dx = q!, so b is a
//    polynomial in m;
//  d = 3 (d^3p/p^0 = |p| dp^0 dOmega): I_k = int_m^inf e^{-p0} |p|^(2k+1) dp0
//    = (2k+1)!!/2^(k+1) (2m)^(k+1) K_{k+1}(m); the a = 1 integral is
//    I_{k+1}/(2k+3) (by parts) and the normalisation I_0 = m K_1(m).  K_0 and
//    K_1 come from K_nu(z) = int_0^inf exp(-z cosh t) cosh(nu t) dt by the
//    trapezoidal rule (spectrally accurate for this analytic, even integrand),
//    higher orders from K_{nu+1} = K_{nu-1} + (2 nu / z) K_nu.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/rlbm.h"
#include "precompute.h"

namespace rlbm {

typedef __float128 qf;

static qf qsqrt(qf x) {   // Newton from the double estimate
  if (x <= 0) return 0;
  qf y = (qf)std::sqrt((double)x);
  for (int it = 0; it < 3; ++it) y = 0.5Q * (y + x / y);
  return y;
}

static qf qfact(int n) {
  qf r = 1;
  for (int k = 2; k <= n; ++k) r *= k;
  return r;
}

static qf qdfact(int n) {   // n!! with (-1)!! = 1
  qf r = 1;
  for (int k = n; k > 1; k -= 2) r *= k;
  return r;
}

static qf qbinom(int n, int k) { return qfact(n) / (qfact(k) * qfact(n - k)); }

// e^x in binary128: x = k ln2 + r, |r| <= ln2/2, Taylor series for e^r.
static qf qexp(qf x) {
  const qf ln2 = 0.6931471805599453094172321214581765680755Q;
  const double kd = std::nearbyint((double)(x / ln2));
  const qf r = x - (qf)kd * ln2;
  qf term = 1, sum = 1;
  for (int j = 1; j < 40; ++j) {
    term *= r / j;
    sum += term;
  }
  qf scale = 1, base = kd >= 0 ? (qf)2 : (qf)0.5Q;
  for (long k = (long)std::fabs(kd); k > 0; k >>= 1) {
    if (k & 1) scale *= base;
    base *= base;
  }
  return sum * scale;
}

// K_0(z) and K_1(z) for z > 0 (trapezoidal rule with step 1/32 until the terms vanish).
static void qbessel_k01(qf z, qf &k0, qf &k1) {
  const qf h = 0.03125Q;
  k0 = 0.5Q * qexp(-z);
  k1 = k0;
  for (int j = 1; j < 100000; ++j) {
    const qf t = h * j, et = qexp(t), ch = 0.5Q * (et + 1 / et);
    const qf f = qexp(-z * ch);
    k0 += f;
    k1 += f * ch;
    if (f < 1e-45Q * k0) break;
  }
  k0 *= h;
  k1 *= h;
}

// Rest-frame moment of p0^a p^e (e even) for omega = C exp(-p0), normalised to 1.
static qf rest_moment(int d, qf m, int a, const int *e) {
  int k = 0;
  qf ang = 1;
  for (int c = 0; c < d; ++c) {
    k += e[c];
    ang *= qdfact(e[c] - 1);
  }
  ang /= qdfact(k + d - 2);
  k /= 2;
  if (d == 2) {
    qf rad = 0;
    for (int j = 0; j <= k; ++j) {
      qf c = qbinom(k, j);
      for (int t = 0; t < k - j; ++t) c *= 2 * m;
      // x^(k+j) (m + x)^a
      rad += c * (a == 0 ? qfact(k + j) : m * qfact(k + j) + qfact(k + j + 1));
    }
    return ang * rad;
  }
  qf K[8];
  qbessel_k01(m, K[0], K[1]);
  for (int nu = 1; nu < 7; ++nu) K[nu + 1] = K[nu - 1] + (2 * nu) / m * K[nu];
  auto I = [&](int kk) {
    qf r = qdfact(2 * kk + 1) * K[kk + 1];
    for (int t = 0; t <= kk; ++t) r *= m;   // (2m)^(k+1) / 2^(k+1)
    return r;
  };
  const qf rad = a == 0 ? I(k) : I(k + 1) / (2 * k + 3);
  return ang * rad / I(0);
}

// The stencil of (d, order): members of each non-rest group in population order
// (shared with the kernels), their |n|^2, and the largest |n|.
struct MassiveSpec {
  int d = 0, ng = 0, n = 0;
  const int (*v)[3] = nullptr;
  const int *first = nullptr, *count = nullptr;
};

static bool massive_spec(int d, int order, MassiveSpec &sp) {
  sp.d = d;
  if (d == 2 && order == 2) {
    sp.ng = kMassiveDirs22.NG, sp.n = kMassiveDirs22.n, sp.v = kMassiveDirs22.v;
    sp.first = kMassiveDirs22.first, sp.count = kMassiveDirs22.count;
  } else if (d == 2 && order == 3) {
    sp.ng = kMassiveDirs23.NG, sp.n = kMassiveDirs23.n, sp.v = kMassiveDirs23.v;
    sp.first = kMassiveDirs23.first, sp.count = kMassiveDirs23.count;
  } else if (d == 3 && order == 3) {
    sp.ng = kMassiveDirs33.NG, sp.n = kMassiveDirs33.n, sp.v = kMassiveDirs33.v;
    sp.first = kMassiveDirs33.first, sp.count = kMassiveDirs33.count;
  } else {
    return false;
  }
  return true;
}

static int norm2(const MassiveSpec &sp, int i) {
  int r = 0;
  for (int a = 0; a < sp.d; ++a) r += sp.v[i][a] * sp.v[i][a];
  return r;
}

// Group weights (the rest group first, then the stencil's groups in order) at
// v0.  Every member n of group g has p^0_g = m / sqrt(1 - v0^2 |n|^2) and
// p = p^0_g v0 n, so its row entries are (p^0_g)^a (p^0_g v0)^|e| sum_n n^e.
// Returns false if the system is singular.
static bool massive_weights(int d, qf m, int order, qf v0, std::vector<qf> &w) {
  MassiveSpec sp;
  if (!massive_spec(d, order, sp)) return false;
  const int ng = sp.ng + 1;
  // invariant monomials (a, e): every e_c even, e_1 >= e_2 >= ..., degree a + |e| <= 2N
  std::vector<int> inv;
  for (int a = 0; a <= 1; ++a)
    for (int deg = 0; deg <= 2 * order - a; deg += 2)
      for (int e0 = deg; e0 >= 0; e0 -= 2)
        for (int e1 = std::min(e0, deg - e0); e1 >= 0; e1 -= 2) {
          const int e2 = deg - e0 - e1;
          if (d == 2 && e2 != 0) continue;
          if (e2 > e1) continue;
          inv.insert(inv.end(), {a, e0, e1, e2});
        }
  const int nr = (int)inv.size() / 4;
  if (nr != ng) return false;
  std::vector<qf> A(nr * (ng + 1), 0);   // augmented [A | b]
  for (int g = 0; g < ng; ++g) {
    qf p0 = m, sc = 0;
    int first = 0, cnt = 1;
    if (g > 0) {
      first = sp.first[g - 1], cnt = sp.count[g - 1];
      p0 = m / qsqrt(1 - v0 * v0 * (qf)norm2(sp, first));
      sc = p0 * v0;
    }
    for (int r = 0; r < nr; ++r) {
      const int *e = &inv[4 * r + 1];
      long s = 0;   // sum over the group of n^e (integers)
      for (int i = first; i < first + cnt; ++i) {
        long t = 1;
        for (int a = 0; a < d; ++a)
          for (int c = 0; c < e[a]; ++c) t *= (g > 0 ? sp.v[i][a] : 0);
        s += t;
      }
      qf v = inv[4 * r] ? p0 : (qf)1;
      for (int c = 0; c < e[0] + e[1] + e[2]; ++c) v *= sc;
      A[r * (ng + 1) + g] = v * (qf)s;
    }
  }
  for (int r = 0; r < nr; ++r) A[r * (ng + 1) + ng] = rest_moment(d, m, inv[4 * r], &inv[4 * r + 1]);
  // Gaussian elimination with partial pivoting
  const int W = ng + 1;
  for (int c = 0; c < ng; ++c) {
    int piv = c;
    for (int r = c + 1; r < nr; ++r) {
      qf a = A[r * W + c], b = A[piv * W + c];
      if ((a < 0 ? -a : a) > (b < 0 ? -b : b)) piv = r;
    }
    if (A[piv * W + c] == 0) return false;
    if (piv != c)
      for (int k = 0; k < W; ++k) std::swap(A[c * W + k], A[piv * W + k]);
    for (int r = c + 1; r < nr; ++r) {
      const qf f = A[r * W + c] / A[c * W + c];
      for (int k = c; k < W; ++k) A[r * W + k] -= f * A[c * W + k];
    }
  }
  w.assign(ng, 0);
  for (int c = ng - 1; c >= 0; --c) {
    qf s = A[c * W + ng];
    for (int k = c + 1; k < ng; ++k) s -= A[c * W + k] * w[k];
    w[c] = s / A[c * W + c];
  }
  return true;
}

static double min_weight(int d, double m, int order, double v0) {
  std::vector<qf> w;
  if (!massive_weights(d, (qf)m, order, (qf)v0, w)) return -1.0;
  qf lo = w[0];
  for (qf x : w) lo = x < lo ? x : lo;
  return (double)lo;
}

static double max_norm(int d, int order) {
  MassiveSpec sp;
  if (!massive_spec(d, order, sp)) return 1.0;
  int r = 0;
  for (int i = 0; i < sp.n; ++i) r = std::max(r, norm2(sp, i));
  return std::sqrt((double)r);
}

// The v0 window of non-negative weights: the largest min_g w_g over a scan of
// (0, 1/max|n|), refined by golden-section search, then bisection towards
// both ends.
int massive_window(int d, double m, int order, double &lo, double &hi, std::string &err) {
  const int scan = 600;
  const double a0 = 1e-3, a1 = 1.0 / max_norm(d, order) - 1e-4;
  int best = 0;
  double bestv = -1e300;
  for (int k = 0; k < scan; ++k) {
    const double v = a0 + (a1 - a0) * k / (scan - 1);
    const double mw = min_weight(d, m, order, v);
    if (mw > bestv) bestv = mw, best = k;
  }
  const double glo = a0 + (a1 - a0) * (best > 0 ? best - 1 : 0) / (scan - 1);
  const double ghi = a0 + (a1 - a0) * (best < scan - 1 ? best + 1 : scan - 1) / (scan - 1);
  const double gr = (std::sqrt(5.0) - 1.0) / 2.0;
  double a = glo, b = ghi, c1 = b - gr * (b - a), c2 = a + gr * (b - a);
  double f1 = min_weight(d, m, order, c1), f2 = min_weight(d, m, order, c2);
  for (int it = 0; it < 60; ++it) {
    if (f1 > f2) {
      b = c2, c2 = c1, f2 = f1;
      c1 = b - gr * (b - a);
      f1 = min_weight(d, m, order, c1);
    } else {
      a = c1, c1 = c2, f1 = f2;
      c2 = a + gr * (b - a);
      f2 = min_weight(d, m, order, c2);
    }
  }
  const double vbest = 0.5 * (a + b);
  if (min_weight(d, m, order, vbest) < 0.0) {
    err = "no v0 gives non-negative weights for this stencil and mass";
    return RLBM_ERR_QUADRATURE;
  }
  auto edge = [&](double inside, double outside) {
    for (int it = 0; it < 80; ++it) {
      const double mid = 0.5 * (inside + outside);
      if (min_weight(d, m, order, mid) >= 0.0) inside = mid;
      else outside = mid;
    }
    return inside;
  };
  lo = edge(vbest, glo);
  hi = edge(vbest, ghi);
  return 0;
}

int build_massive(int d, double m, int order, double v0, QuadHost &q, std::string &err) {
  if (!(m > 0.0) || !std::isfinite(m)) {
    err = "massive on-lattice rules need zeta > 0";
    return RLBM_ERR_INVALID_ARG;
  }
  MassiveSpec sp;
  if (!massive_spec(d, order, sp)) {
    err = "massive on-lattice rules are provided for d = 2 (N = 2, 3) and d = 3 (N = 3)";
    return RLBM_ERR_UNSUPPORTED;
  }
  if (v0 == 0.0) {
    double lo, hi;
    int rc = massive_window(d, m, order, lo, hi, err);
    if (rc) return rc;
    v0 = 0.5 * (lo + hi);
  }
  if (!(v0 > 0.0) || !(v0 * max_norm(d, order) < 1.0)) {
    err = "v0 must lie in (0, 1/max|n|)";
    return RLBM_ERR_INVALID_ARG;
  }
  std::vector<qf> wg;
  if (!massive_weights(d, (qf)m, order, (qf)v0, wg)) {
    err = "singular moment system for the massive stencil";
    return RLBM_ERR_QUADRATURE;
  }
  for (qf x : wg)
    if (x < 0) {
      err = "v0 lies outside the window of non-negative weights";
      return RLBM_ERR_QUADRATURE;
    }
  q = QuadHost();
  q.d = d;
  q.m = m;
  q.order = order;
  q.kind = RLBM_QUAD_MASSIVE_ONLATTICE;
  q.v0 = v0;
  q.nshell = 0;
  auto push = [&](const int *n, qf wgt) {
    const qf n2 = (qf)(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const qf p0 = (qf)m / qsqrt(1 - (qf)v0 * (qf)v0 * n2);
    q.p.push_back((double)p0);
    for (int a = 0; a < d; ++a) q.p.push_back((double)(p0 * (qf)v0 * n[a]));
    q.w.push_back((double)wgt);
    for (int a = 0; a < d; ++a) q.disp.push_back((double)n[a]);
  };
  for (int g = 0; g < sp.ng; ++g) {
    q.gfirst.push_back(sp.first[g]);
    for (int i = sp.first[g]; i < sp.first[g] + sp.count[g]; ++i) push(sp.v[i], wg[g + 1]);
  }
  const int zero[3] = {0, 0, 0};
  push(zero, wg[0]);
  q.Q = (int)q.w.size();
  q.ndir = q.Q;
  return 0;
}

}  // namespace rlbm
