// device_math.h -- per-site arithmetic of the RLBM update (HIP device code).
//
// Steps of Sec. 6.2 for one site, given its pre-collision populations:
//   moments N^a, T^ab (step 1); Landau eigenproblem T^ab U_b = eps U^a
//   (step 2); n = U_a N^a (step 3); T from the equation of state (step 4);
//   the projected equilibrium (step 5); Anderson-Witting relaxation (step 8).
#pragma once
#include <hip/hip_runtime.h>

#include "rlbm_defs.h"

namespace rlbm {

__device__ __forceinline__ constexpr double eta_c(int a, int b) { return a != b ? 0.0 : (a == 0 ? 1.0 : -1.0); }

// ---------------------------------------------------------------------------
// Landau frame (Sec. 4; Sec. 6.2 step 2).  With lowered U_b = eta_bc U^c the
// problem is M U = eps U for the mixed tensor M = T eta.  Rayleigh-quotient
// iteration: sigma = U_a T^ab U_b / (U_a U^a), then U <- adj(M - sigma I) U,
// normalised to U^a U_a = 1, U^0 > 0.  The adjugate needs no division, so the
// iteration stays finite when sigma reaches the eigenvalue exactly.  The
// start vector is U ~ (T^00 + P0, T^0i) with P0 = sum_i T^ii / d, exact for an
// equilibrium tensor at rest and first-order accurate in the velocity.
// Returns false for a state without a time-like eigenvector.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void adj_apply(const double (&A)[D + 1][D + 1], const double (&u)[D + 1],
                                          double (&y)[D + 1]);

template <>
__device__ __forceinline__ void adj_apply<2>(const double (&A)[3][3], const double (&u)[3], double (&y)[3]) {
  // adj(A) = cofactor matrix transposed
  const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  const double c10 = A[0][2] * A[2][1] - A[0][1] * A[2][2];
  const double c11 = A[0][0] * A[2][2] - A[0][2] * A[2][0];
  const double c12 = A[0][1] * A[2][0] - A[0][0] * A[2][1];
  const double c20 = A[0][1] * A[1][2] - A[0][2] * A[1][1];
  const double c21 = A[0][2] * A[1][0] - A[0][0] * A[1][2];
  const double c22 = A[0][0] * A[1][1] - A[0][1] * A[1][0];
  y[0] = c00 * u[0] + c10 * u[1] + c20 * u[2];
  y[1] = c01 * u[0] + c11 * u[1] + c21 * u[2];
  y[2] = c02 * u[0] + c12 * u[1] + c22 * u[2];
}

__device__ __forceinline__ double det3(double a, double b, double c, double d, double e, double f, double g,
                                       double h, double i) {
  return a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
}

template <>
__device__ __forceinline__ void adj_apply<3>(const double (&A)[4][4], const double (&u)[4], double (&y)[4]) {
  // y_j = sum_i adj(A)_{j i} u_i = sum_i C_{i j} u_i, C the cofactor matrix.
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int r0 = i == 0 ? 1 : 0, r1 = i <= 1 ? 2 : 1, r2 = i <= 2 ? 3 : 2;
      int q0 = j == 0 ? 1 : 0, q1 = j <= 1 ? 2 : 1, q2 = j <= 2 ? 3 : 2;
      double minor = det3(A[r0][q0], A[r0][q1], A[r0][q2], A[r1][q0], A[r1][q1], A[r1][q2], A[r2][q0], A[r2][q1],
                          A[r2][q2]);
      acc += (((i + j) & 1) ? -minor : minor) * u[i];
    }
    y[j] = acc;
  }
}

// y = adj(S) u for a symmetric 4 x 4 S, from the 2 x 2 minors of rows (0, 1) and (2, 3)
// (Laplace expansion); only the upper triangle of the adjugate is formed.
__device__ __forceinline__ void adj_apply_sym4(const double (&a)[4][4], const double (&u)[4], double (&y)[4]) {
  const double s0 = a[0][0] * a[1][1] - a[0][1] * a[0][1];
  const double s1 = a[0][0] * a[1][2] - a[0][1] * a[0][2];
  const double s2 = a[0][0] * a[1][3] - a[0][1] * a[0][3];
  const double s3 = a[0][1] * a[1][2] - a[1][1] * a[0][2];
  const double s4 = a[0][1] * a[1][3] - a[1][1] * a[0][3];
  const double s5 = a[0][2] * a[1][3] - a[1][2] * a[0][3];
  const double c5 = a[2][2] * a[3][3] - a[2][3] * a[2][3];
  const double c4 = a[1][2] * a[3][3] - a[1][3] * a[2][3];
  const double c3 = a[1][2] * a[2][3] - a[1][3] * a[2][2];
  const double c2 = a[0][2] * a[3][3] - a[0][3] * a[2][3];
  const double c1 = a[0][2] * a[2][3] - a[0][3] * a[2][2];
  const double b00 = a[1][1] * c5 - a[1][2] * c4 + a[1][3] * c3;
  const double b01 = -a[0][1] * c5 + a[0][2] * c4 - a[0][3] * c3;
  const double b02 = a[1][3] * s5 - a[2][3] * s4 + a[3][3] * s3;
  const double b03 = -a[1][2] * s5 + a[2][2] * s4 - a[2][3] * s3;
  const double b11 = a[0][0] * c5 - a[0][2] * c2 + a[0][3] * c1;
  const double b12 = -a[0][3] * s5 + a[2][3] * s2 - a[3][3] * s1;
  const double b13 = a[0][2] * s5 - a[2][2] * s2 + a[2][3] * s1;
  const double b22 = a[0][3] * s4 - a[1][3] * s2 + a[3][3] * s0;
  const double b23 = -a[0][2] * s4 + a[1][2] * s2 - a[2][3] * s0;
  const double b33 = a[0][2] * s3 - a[1][2] * s1 + a[2][2] * s0;
  y[0] = b00 * u[0] + b01 * u[1] + b02 * u[2] + b03 * u[3];
  y[1] = b01 * u[0] + b11 * u[1] + b12 * u[2] + b13 * u[3];
  y[2] = b02 * u[0] + b12 * u[1] + b22 * u[2] + b23 * u[3];
  y[3] = b03 * u[0] + b13 * u[1] + b23 * u[2] + b33 * u[3];
}

template <int D>
__device__ __forceinline__ double lorentz_dot(const double (&a)[D + 1], const double (&b)[D + 1]) {
  double s = a[0] * b[0];
#pragma unroll
  for (int k = 1; k <= D; ++k) s -= a[k] * b[k];
  return s;
}

// U_a T^ab U_b with T symmetric (contravariant) and U contravariant
template <int D>
__device__ __forceinline__ double rayleigh(const double (&T)[D + 1][D + 1], const double (&U)[D + 1]) {
  double s = 0.0;
#pragma unroll
  for (int a = 0; a <= D; ++a)
#pragma unroll
    for (int b = 0; b <= D; ++b) s += eta_c(a, a) * eta_c(b, b) * U[a] * T[a][b] * U[b];
  return s;
}

template <int D, int ITERS>
__device__ __forceinline__ bool landau_frame(const double (&T)[D + 1][D + 1], double &eps, double (&U)[D + 1]) {
  double P0 = 0.0;
#pragma unroll
  for (int k = 1; k <= D; ++k) P0 += T[k][k];
  P0 *= 1.0 / D;
  U[0] = T[0][0] + P0;
#pragma unroll
  for (int k = 1; k <= D; ++k) U[k] = T[0][k];
  bool ok = true;
#pragma unroll
  for (int it = 0; it <= ITERS; ++it) {
    double nn = lorentz_dot<D>(U, U);
    ok = nn > 0.0;
    double s = (U[0] >= 0.0 ? 1.0 : -1.0) * rsqrt(nn);
#pragma unroll
    for (int k = 0; k <= D; ++k) U[k] *= s;
    eps = rayleigh<D>(T, U);
    if (it == ITERS) break;
    double y[D + 1];
    if constexpr (D == 3) {
      // M - eps I = (T - eps eta) eta, so adj(M - eps I) U = -eta adj(S) U with S = T - eps eta
      // symmetric (the sign is fixed by the normalisation)
      double S[4][4];
#pragma unroll
      for (int a = 0; a <= 3; ++a)
#pragma unroll
        for (int b = 0; b <= 3; ++b) S[a][b] = T[a][b] - (a == b ? eps * eta_c(a, a) : 0.0);
      adj_apply_sym4(S, U, y);
      y[1] = -y[1];
      y[2] = -y[2];
      y[3] = -y[3];
    } else {
      double A[D + 1][D + 1];
#pragma unroll
      for (int a = 0; a <= D; ++a)
#pragma unroll
        for (int b = 0; b <= D; ++b) A[a][b] = T[a][b] * eta_c(b, b) - (a == b ? eps : 0.0);
      adj_apply<D>(A, U, y);
    }
#pragma unroll
    for (int k = 0; k <= D; ++k) U[k] = y[k];
  }
  return ok;
}

// ---------------------------------------------------------------------------
// Equation of state (Sec. 3, Eq. eos-ddim) and the A_n/A_1 ratios (App. B).
// d = 2: G_2 = (z^2 + 3z + 3)/(z + 1), so e = eps/n solves
//   2 T^2 + (2m - e) T + m^2 - e m = 0;
// the positive root is taken in the form that avoids cancellation.
// d = 3: G_3 = z r + 4 with r = K1/K2 from a Chebyshev fit in log z, so that
// e = eps/n = m r(m/T) + 3 T; its inverse T(e) is a second fit (built on the
// host from the first by Newton's method).
// ---------------------------------------------------------------------------
// Macroscopic state of a site (double).
template <int D>
struct Macro {
  double n, eps, T;
  double U[D + 1];
  bool ok;
};

struct Ratios {
  double r0, r2, r3;   // A_0/A_1, A_2/A_1 (= G_d), A_3/A_1
};

__device__ __forceinline__ bool temperature_2d(double e, double m, double &T) {
  if (m == 0.0) {
    T = 0.5 * e;
    return e > 0.0;
  }
  const double b = e - 2.0 * m;
  const double disc = e * e + 4.0 * e * m - 4.0 * m * m;
  const double sq = sqrt(disc);
  T = b >= 0.0 ? 0.25 * (b + sq) : 2.0 * m * (e - m) / (sq - b);
  return disc > 0.0 && e > m && T > 0.0;
}

__device__ __forceinline__ Ratios ratios_2d(double z) {
  const double inv = 1.0 / (z + 1.0);
  Ratios r;
  r.r0 = inv;
  r.r2 = ((z + 3.0) * z + 3.0) * inv;
  r.r3 = (((z + 6.0) * z + 15.0) * z + 15.0) * inv;
  return r;
}

__device__ __forceinline__ double cheb_eval(const double *__restrict__ c, double s) {
  double b1 = 0.0, b2 = 0.0;
#pragma unroll 4
  for (int k = kEosTerms - 1; k >= 1; --k) {
    double b0 = 2.0 * s * b1 - b2 + c[k];
    b2 = b1;
    b1 = b0;
  }
  return s * b1 - b2 + c[0];
}

// A piecewise series at u in [-1, 1] (the whole fitted range; clamped): the piece of u and the
// local variable s in [-1, 1] of that piece (the host's fit uses the same map).  When the wave's
// sites share a piece (the usual case: temperature varies smoothly) the series is read through
// uniform (scalar) loads of that piece; a wave that straddles a piece boundary evaluates every
// piece, each with uniform loads, and keeps its own.
__device__ __forceinline__ double cheb_eval_pieces(const double (*__restrict__ c)[48], double u) {
  u = fmin(1.0, fmax(-1.0, u));
  const double t = (u + 1.0) * (0.5 * kEosPieces);
  int p = (int)t;
  p = p < 0 ? 0 : (p >= kEosPieces ? kEosPieces - 1 : p);
  const double s = 2.0 * (t - p) - 1.0;
  const int q = __builtin_amdgcn_readfirstlane(p);
  if (__all(p == q)) return cheb_eval(c[q], s);
  double r = 0.0;
#pragma unroll 1
  for (int k = 0; k < kEosPieces; ++k) {
    const double v = cheb_eval(c[k], s);
    r = p == k ? v : r;
  }
  return r;
}

__device__ __forceinline__ double cheb_r(const Tables *__restrict__ tb, double z, bool &inrange) {
  // Clenshaw on the piece's s in [-1, 1], affine in log z; the series fits h = r (z + 2) / z, which
  // stays O(1) from z -> 0 (r ~ z/2) to z -> inf (r -> 1)
  const double u = (2.0 * log(z) - (tb->cheb_lo + tb->cheb_hi)) / (tb->cheb_hi - tb->cheb_lo);
  inrange = u >= -1.0 && u <= 1.0;
  return cheb_eval_pieces(tb->cheb, u) * (z / (z + 2.0));
}

// d = 3: T from e = eps/n through the fitted inverse T = (e - m) u(log(e - m)), then r = K1/K2 at
// z = m/T.  Both fits hold to ~1e-15 on T in [kEosTmin, kEosTmax] = [1/128, 128]; outside that range
// the site is flagged.
__device__ __forceinline__ bool temperature_3d(const Tables *__restrict__ tb, double e, double m, double &T,
                                               double &r_out) {
  if (m == 0.0) {
    T = e / 3.0;
    r_out = 0.0;
    return e > 0.0;
  }
  const double d = e - m;
  bool ok = d > 0.0;
  const double u = (2.0 * log(d) - (tb->chebT_lo + tb->chebT_hi)) / (tb->chebT_hi - tb->chebT_lo);
  ok = ok && u >= -1.0 && u <= 1.0;
  T = d * cheb_eval_pieces(tb->chebT, u);
  bool inr;
  r_out = cheb_r(tb, m / T, inr);
  return ok && inr && T > 0.0;
}

__device__ __forceinline__ Ratios ratios_3d(double z, double r) {
  Ratios q;
  if (z == 0.0) {
    q.r0 = 0.5;
    q.r2 = 4.0;
    q.r3 = 24.0;
  } else {
    q.r0 = r / z;
    q.r2 = z * r + 4.0;
    q.r3 = z * z + 6.0 * q.r2;
  }
  return q;
}

// ---------------------------------------------------------------------------
// Maxwell-Juettner moments of the basis monomials (App. B, Z tensors with the
// normalisation of Eq. phys-normalization):
//   deg 0: n r0 / T, deg 1: n U^a, deg 2: n T (r2 U^a U^b - eta^ab),
//   deg 3: n T^2 (r3 U^a U^b U^c - r2 (eta^ab U^c + eta^ac U^b + eta^bc U^a)).
// ---------------------------------------------------------------------------
// The same moment for one basis index k (k a compile-time constant after unrolling).
template <int D, int N>
__device__ __forceinline__ double basis_moment(int k, double n, double T, const double (&U)[D + 1], const Ratios &r) {
  using B = BasisDef<D, N>;
  const int a = B::idx[k][0], b = B::idx[k][1], c = B::idx[k][2];
  if (a < 0) return n * r.r0 / T;
  if (b < 0) return n * U[a];
  if (c < 0) return n * T * (r.r2 * U[a] * U[b] - eta_c(a, b));
  return n * T * T *
         (r.r3 * U[a] * U[b] * U[c] - r.r2 * (eta_c(a, b) * U[c] + eta_c(a, c) * U[b] + eta_c(b, c) * U[a]));
}

template <int D, int N>
__device__ __forceinline__ void basis_moments(double n, double T, const double (&U)[D + 1], const Ratios &r,
                                              double (&M)[BasisDef<D, N>::NM]) {
  using B = BasisDef<D, N>;
  const double nT = n * T, nT2 = nT * T;
#pragma unroll
  for (int k = 0; k < B::NM; ++k) {
    const int a = B::idx[k][0], b = B::idx[k][1], c = B::idx[k][2];
    if (a < 0) {
      M[k] = n * r.r0 / T;
    } else if (b < 0) {
      M[k] = n * U[a];
    } else if (c < 0) {
      M[k] = nT * (r.r2 * U[a] * U[b] - eta_c(a, b));
    } else {
      M[k] = nT2 * (r.r3 * U[a] * U[b] * U[c] -
                    r.r2 * (eta_c(a, b) * U[c] + eta_c(a, c) * U[b] + eta_c(b, c) * U[a]));
    }
  }
}

// One post-collision population: plane base (uniform) + 32-bit byte offset of the site.  NT marks
// the store non-temporal: the line is written towards memory without being kept in the L2 or the
// last-level cache, which pays when the two state buffers are larger than that cache (the next
// step reads the populations from memory either way) and costs when they would fit in it.
template <bool NT, typename S>
__device__ __forceinline__ void put_pop(S *__restrict__ fout, int64_t sites, uint32_t site_off, int i, S v) {
  S *p = (S *)((char *)(fout + (int64_t)i * sites) + site_off);
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

}  // namespace rlbm
