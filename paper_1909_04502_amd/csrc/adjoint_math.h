// adjoint_math.h -- reverse mode (vector-Jacobian products) of the product-rule
// collision and of the equilibrium evaluation (HIP device code).
//
// With F the pre-collision populations of a site and B = C(F; tau) the
// post-collision ones (Sec. 6.2, steps 1-8), collide_vjp maps the adjoint
// mu = dL/dB to dL/dF and dL/dtau.  Every stage of the forward collision is
// reversed in turn:
//   B_i = F_i + Omega_i (f^eq_i - F_i),  Omega_i = (U^0 - v_i . U)/tau
//   f^eq = w psi^T Linv^T Linv M'(n, T, U)          (projection, Sec. 5.2)
//   M'   = Maxwell-Juettner moments, shifted basis  (App. B)
//   T    = EOS^{-1}(eps / n)                        (Sec. 3)
//   n    = U_a N^a
//   (eps, U): T^ab U_b = eps U^a, U^a U_a = 1      (Landau frame, Sec. 4)
//   N^a, T^ab = sum_i F_i p_i^a (p_i^b)            (moments)
// The eigenvector is differentiated implicitly through the bordered system
// [[eta T - eps I, U_low], [U^T, 0]] [z; s] = [Ubar; 0], giving
// Tbar^ab = epsbar U_a U_b - z^a U_b (lowered U), the derivative of the
// exact eigenpair.
#pragma once
#include "prod_math.h"

namespace rlbm {

struct RatiosD {
  double r0, r2, r3, d0, d2, d3;   // A_n/A_1 and their zeta derivatives (d = 2)
};

__device__ __forceinline__ RatiosD ratios_2d_d(double z) {
  const double inv = 1.0 / (z + 1.0), inv2 = inv * inv;
  RatiosD r;
  r.r0 = inv;
  r.r2 = ((z + 3.0) * z + 3.0) * inv;
  r.r3 = (((z + 6.0) * z + 15.0) * z + 15.0) * inv;
  r.d0 = -inv2;
  r.d2 = (z + 2.0) * z * inv2;
  r.d3 = ((2.0 * z + 9.0) * z + 12.0) * z * inv2;
  return r;
}

// Reverse of basis_moments: accumulates dL/dn, dL/dT, dL/dU^a from dL/dM.
template <int D, int N>
__device__ __forceinline__ void basis_moments_vjp(double n, double T, const double (&U)[D + 1], double m,
                                                  const RatiosD &r, const double (&Mb)[BasisDef<D, N>::NM],
                                                  double &nb, double &Tb, double (&Ub)[D + 1]) {
  using B = BasisDef<D, N>;
  const double dzdT = -m / (T * T);
#pragma unroll
  for (int k = 0; k < B::NM; ++k) {
    const int a = B::idx[k][0], b = B::idx[k][1], c = B::idx[k][2];
    const double g = Mb[k];
    if (a < 0) {            // n r0 / T
      nb += g * r.r0 / T;
      Tb += g * n * (r.d0 * dzdT / T - r.r0 / (T * T));
    } else if (b < 0) {     // n U^a
      nb += g * U[a];
      Ub[a] += g * n;
    } else if (c < 0) {     // n T (r2 U^a U^b - eta^ab)
      const double P = r.r2 * U[a] * U[b] - eta_c(a, b);
      nb += g * T * P;
      Tb += g * n * (P + T * r.d2 * dzdT * U[a] * U[b]);
      Ub[a] += g * n * T * r.r2 * U[b];
      Ub[b] += g * n * T * r.r2 * U[a];
    } else {                // n T^2 (r3 U^a U^b U^c - r2 (eta^ab U^c + eta^ac U^b + eta^bc U^a))
      const double S3 = U[a] * U[b] * U[c];
      const double S1 = eta_c(a, b) * U[c] + eta_c(a, c) * U[b] + eta_c(b, c) * U[a];
      const double P = r.r3 * S3 - r.r2 * S1;
      const double nT2 = n * T * T;
      nb += g * T * T * P;
      Tb += g * n * (2.0 * T * P + T * T * dzdT * (r.d3 * S3 - r.d2 * S1));
      Ub[a] += g * nT2 * (r.r3 * U[b] * U[c] - r.r2 * eta_c(b, c));
      Ub[b] += g * nT2 * (r.r3 * U[a] * U[c] - r.r2 * eta_c(a, c));
      Ub[c] += g * nT2 * (r.r3 * U[a] * U[b] - r.r2 * eta_c(a, b));
    }
  }
}

// Reverse of the Landau eigenpair: Tbar (full (D+1)^2 matrix, added to).
template <int D>
__device__ __forceinline__ void landau_vjp(const double (&T)[D + 1][D + 1], double eps, const double (&U)[D + 1],
                                           double epsb, const double (&Ub)[D + 1], double (&Tb)[D + 1][D + 1]) {
  constexpr int K = D + 2;
  double Ul[D + 1];
#pragma unroll
  for (int a = 0; a <= D; ++a) Ul[a] = eta_c(a, a) * U[a];
  // K^T = [[eta T - eps I, U_low], [U^T, 0]], solve K^T [z; s] = [Ub; 0]
  double A[K][K + 1];
#pragma unroll
  for (int a = 0; a <= D; ++a) {
#pragma unroll
    for (int c = 0; c <= D; ++c) A[a][c] = eta_c(a, a) * T[a][c] - (a == c ? eps : 0.0);
    A[a][D + 1] = Ul[a];
    A[a][K] = Ub[a];
  }
#pragma unroll
  for (int c = 0; c <= D; ++c) A[D + 1][c] = U[c];
  A[D + 1][D + 1] = 0.0;
  A[D + 1][K] = 0.0;
  // Gaussian elimination with partial pivoting (K <= 5)
#pragma unroll
  for (int col = 0; col < K; ++col) {
    int piv = col;
    double best = fabs(A[col][col]);
#pragma unroll
    for (int r = col + 1; r < K; ++r)
      if (fabs(A[r][col]) > best) {
        best = fabs(A[r][col]);
        piv = r;
      }
#pragma unroll
    for (int r = col; r < K; ++r) {
      if (r == piv && r != col) {
#pragma unroll
        for (int c = 0; c <= K; ++c) {
          const double t = A[col][c];
          A[col][c] = A[r][c];
          A[r][c] = t;
        }
      }
    }
    const double inv = 1.0 / A[col][col];
#pragma unroll
    for (int r = col + 1; r < K; ++r) {
      const double f = A[r][col] * inv;
#pragma unroll
      for (int c = col; c <= K; ++c) A[r][c] -= f * A[col][c];
    }
  }
  double z[K];
#pragma unroll
  for (int r = K - 1; r >= 0; --r) {
    double s = A[r][K];
#pragma unroll
    for (int c = r + 1; c < K; ++c) s -= A[r][c] * z[c];
    z[r] = s / A[r][r];
  }
#pragma unroll
  for (int a = 0; a <= D; ++a)
#pragma unroll
    for (int b = 0; b <= D; ++b) Tb[a][b] += epsb * Ul[a] * Ul[b] - z[a] * Ul[b];
}

// de/dT of e(T) = T (G_2(m/T) - 1), used to reverse the d = 2 EOS inversion.
__device__ __forceinline__ double eos_slope_2d(double T, double m, const RatiosD &r) {
  const double z = m / T;
  return r.r2 - 1.0 - z * r.d2;
}

// Reverse of feq_coefficients (the deviation shift by M^ref has no derivative): given
// apb = dL/da', sets Mb = dL/dM (unshifted basis moments).
template <int D, int N>
__device__ __forceinline__ void coefficients_vjp(const Tables *__restrict__ tb, const double (&apb)[BasisDef<D, N>::NM],
                                                 double (&Mb)[BasisDef<D, N>::NM]) {
  using B = BasisDef<D, N>;
  constexpr AngTable<D, N> AT{};
  // a' = Linv^T a  ->  abar = Linv a'bar ;  a = Linv M'  ->  M'bar = Linv^T abar
  double ab[B::NM];
#pragma unroll
  for (int r = 0; r < B::NM; ++r) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c <= r; ++c)
      if (AT.cls[r] == AT.cls[c]) acc += tb->Linv[r][c] * apb[c];
    ab[r] = acc;
  }
#pragma unroll
  for (int c = 0; c < B::NM; ++c) {
    double acc = 0.0;
#pragma unroll
    for (int r = c; r < B::NM; ++r)
      if (AT.cls[r] == AT.cls[c]) acc += tb->Linv[r][c] * ab[r];
    Mb[c] = acc;
  }
  // M'_(1,e) = M_(1,e) - m M_(0,e)
  const double m = tb->m;
#pragma unroll
  for (int q = 0; q < AT.n; ++q)
    if (AT.m1[q] >= 0) Mb[AT.m0[q]] -= m * Mb[AT.m1[q]];
}

// Transposed product-rule equilibrium evaluation: given g_i = dL/df^eq_i,
// accumulate dL/dM (unshifted basis moments).
template <class ST, int N, typename A>
__device__ __forceinline__ void feq_vjp(const Tables *__restrict__ tb, const A (&g)[ST::Q],
                                        double (&Mb)[BasisDef<ST::D, N>::NM]) {
  constexpr int D = ST::D, ND = ST::NDIR, NPD = ND / 2, KR = ST::NSHELL;
  using B = BasisDef<D, N>;
  constexpr AngTable<D, N> AT{};
  double apb[B::NM];
#pragma unroll
  for (int k = 0; k < B::NM; ++k) apb[k] = 0.0;
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    double ceb[20];
#pragma unroll
    for (int q = 0; q < AT.n; ++q) ceb[q] = 0.0;
#pragma unroll
    for (int qp = 0; qp < NPD; ++qp) {
      const int k = 2 * qp;
      const double Eb = (double)g[j * ND + k] + (double)g[j * ND + k + 1];
      const double Ob = (double)g[j * ND + k] - (double)g[j * ND + k + 1];
#pragma unroll
      for (int q = 0; q < AT.n; ++q) {
        const double c = nhat_pow<ST>(k, AT.e[q][0], AT.e[q][1], AT.e[q][2]) * dir_weight<ST>(k);
        const bool odd = (AT.e[q][0] + AT.e[q][1] + AT.e[q][2]) & 1;
        if (c == 0.0) continue;
        ceb[q] += c * (odd ? Ob : Eb);
      }
    }
#pragma unroll
    for (int q = 0; q < AT.n; ++q) {
      const int l = AT.e[q][0] + AT.e[q][1] + AT.e[q][2];
      if (AT.m0[q] >= 0) apb[AT.m0[q]] += ceb[q] * tb->sfeq[j][0][l];
      if (AT.m1[q] >= 0) apb[AT.m1[q]] += ceb[q] * tb->sfeq[j][1][l];
    }
  }
  coefficients_vjp<D, N>(tb, apb, Mb);
}

// Coefficients a' = Linv^T Linv M' of the projected equilibrium over the shifted monomials
// (Sec. 5.2), from the basis moments Md (deviation form for DEV: Md becomes M - M^ref).
template <int D, int N, bool DEV>
__device__ __forceinline__ void feq_coefficients(const Tables *__restrict__ tb, double (&Md)[BasisDef<D, N>::NM],
                                                 double (&ap)[BasisDef<D, N>::NM]) {
  using B = BasisDef<D, N>;
  constexpr AngTable<D, N> AT{};
  if constexpr (DEV) {
#pragma unroll
    for (int k = 0; k < B::NM; ++k) Md[k] -= tb->Mref[k];
  }
  const double m = tb->m;
#pragma unroll
  for (int q = 0; q < AT.n; ++q)
    if (AT.m1[q] >= 0) Md[AT.m1[q]] -= m * Md[AT.m0[q]];
  double ak[B::NM];
#pragma unroll
  for (int r = 0; r < B::NM; ++r) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c <= r; ++c)
      if (AT.cls[r] == AT.cls[c]) acc += tb->Linv[r][c] * Md[c];
    ak[r] = acc;
  }
#pragma unroll
  for (int c = 0; c < B::NM; ++c) {
    double acc = 0.0;
#pragma unroll
    for (int r = c; r < B::NM; ++r)
      if (AT.cls[r] == AT.cls[c]) acc += tb->Linv[r][c] * ak[r];
    ap[c] = acc;
  }
}

// Angular coefficients of shell j: ce[q] multiplies the direction monomial n^e(q) in the
// equilibrium of that shell's populations.
template <int D, int N>
__device__ __forceinline__ void shell_coefficients(const Tables *__restrict__ tb, int j,
                                                   const double (&ap)[BasisDef<D, N>::NM], double (&ce)[20]) {
  constexpr AngTable<D, N> AT{};
#pragma unroll
  for (int q = 0; q < AT.n; ++q) {
    const int l = AT.e[q][0] + AT.e[q][1] + AT.e[q][2];
    double acc = 0.0;
    if (AT.m0[q] >= 0) acc += ap[AT.m0[q]] * tb->sfeq[j][0][l];
    if (AT.m1[q] >= 0) acc += ap[AT.m1[q]] * tb->sfeq[j][1][l];
    ce[q] = acc;
  }
}

// Forward equilibrium of the product rule from basis moments (deviation form
// for DEV): used by the initial condition.
template <class ST, int N, typename A, bool DEV>
__device__ __forceinline__ void feq_prod(const Tables *__restrict__ tb, double (&Md)[BasisDef<ST::D, N>::NM],
                                         A (&feq)[ST::Q]) {
  constexpr int D = ST::D, ND = ST::NDIR, NPD = ND / 2, KR = ST::NSHELL;
  using B = BasisDef<D, N>;
  constexpr AngTable<D, N> AT{};
  double ap[B::NM];
  feq_coefficients<D, N, DEV>(tb, Md, ap);
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    double ce[20];
    shell_coefficients<D, N>(tb, j, ap, ce);
#pragma unroll
    for (int qp = 0; qp < NPD; ++qp) {
      const int k = 2 * qp;
      double E = 0.0, O = 0.0;
#pragma unroll
      for (int q = 0; q < AT.n; ++q) {
        const double c = nhat_pow<ST>(k, AT.e[q][0], AT.e[q][1], AT.e[q][2]) * dir_weight<ST>(k);
        const bool odd = (AT.e[q][0] + AT.e[q][1] + AT.e[q][2]) & 1;
        if (c == 0.0) continue;
        if (odd) O += c * ce[q];
        else E += c * ce[q];
      }
      feq[j * ND + k] = (A)(E + O);
      feq[j * ND + k + 1] = (A)(E - O);
    }
  }
}

// Moment sums of a product rule, accumulated shell by shell.
template <int D>
struct MomAcc {
  double N0 = 0, T00 = 0, Na[D] = {}, T0a[D] = {}, Tab[D * (D + 1) / 2] = {};
};

// Adds shell j's populations f[base .. base + NDIR) to the moment sums.
template <class ST, typename S, int M>
__device__ __forceinline__ void moments_shell(const Tables *__restrict__ tb, int j, const S (&f)[M], int base,
                                              MomAcc<ST::D> &acc) {
  constexpr int D = ST::D, ND = ST::NDIR, NPD = ND / 2;
  double S0 = 0, Sa[D], Sab[D * (D + 1) / 2];
#pragma unroll
  for (int a = 0; a < D; ++a) Sa[a] = 0;
#pragma unroll
  for (int a = 0; a < D * (D + 1) / 2; ++a) Sab[a] = 0;
#pragma unroll
  for (int q = 0; q < NPD; ++q) {
    const int k = 2 * q;
    const double s = (double)f[base + k] + (double)f[base + k + 1];
    const double d = (double)f[base + k] - (double)f[base + k + 1];
    S0 += s;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double c = nhat<ST>(k, a);
      if (c != 0.0) Sa[a] += c * d;
    }
    int ab = 0;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = a; b < D; ++b) {
        const double c = nhat<ST>(k, a) * nhat<ST>(k, b);
        if (c != 0.0) Sab[ab] += c * s;
        ++ab;
      }
  }
  acc.N0 += tb->smom[j][0] * S0;
  acc.T00 += tb->smom[j][2] * S0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    acc.Na[a] += tb->smom[j][1] * Sa[a];
    acc.T0a[a] += tb->smom[j][3] * Sa[a];
  }
#pragma unroll
  for (int a = 0; a < D * (D + 1) / 2; ++a) acc.Tab[a] += tb->smom[j][4] * Sab[a];
}

// N^a and T^ab from the accumulated sums (plus the reference moments for DEV).
template <class ST, bool DEV>
__device__ __forceinline__ void moments_finish(const Tables *__restrict__ tb, const MomAcc<ST::D> &acc,
                                               double (&Nv)[ST::D + 1], double (&T)[ST::D + 1][ST::D + 1]) {
  constexpr int D = ST::D;
  Nv[0] = acc.N0;
  T[0][0] = acc.T00;
  int ab = 0;
#pragma unroll
  for (int a = 1; a <= D; ++a) {
    Nv[a] = acc.Na[a - 1];
    T[0][a] = T[a][0] = acc.T0a[a - 1];
#pragma unroll
    for (int b = a; b <= D; ++b) {
      T[a][b] = T[b][a] = acc.Tab[ab];
      ++ab;
    }
  }
  if constexpr (DEV) {
    int s = 0;
#pragma unroll
    for (int a = 0; a <= D; ++a) {
      Nv[a] += tb->Nref[a];
#pragma unroll
      for (int b = a; b <= D; ++b) {
        T[a][b] += tb->Tref[s];
        if (a != b) T[b][a] = T[a][b];
        ++s;
      }
    }
  }
}

// Moments of the populations (product structure), double.
template <class ST, typename S, bool DEV>
__device__ __forceinline__ void moments_prod(const Tables *__restrict__ tb, const S (&f)[ST::Q],
                                             double (&Nv)[ST::D + 1], double (&T)[ST::D + 1][ST::D + 1]) {
  MomAcc<ST::D> acc;
#pragma unroll
  for (int j = 0; j < ST::NSHELL; ++j) moments_shell<ST, S, ST::Q>(tb, j, f, j * ST::NDIR, acc);
  moments_finish<ST, DEV>(tb, acc, Nv, T);
}

// dL/dF_i of shell j's populations from dL/dN^a and the symmetric part Ts of dL/dT^ab:
// sum_a Nb_a p^a + sum_ab Ts_ab p^a p^b, added to out[base .. base + NDIR).
template <class ST, typename A, int M>
__device__ __forceinline__ void moments_vjp_shell(const Tables *__restrict__ tb, int j, const double (&Nb)[ST::D + 1],
                                                  const double (&Ts)[ST::D + 1][ST::D + 1], A (&out)[M], int base) {
  constexpr int D = ST::D, ND = ST::NDIR, NPD = ND / 2;
  const double p0 = tb->smom[j][0], pm = tb->smom[j][1];
#pragma unroll
  for (int qp = 0; qp < NPD; ++qp) {
    const int k = 2 * qp;
    double nN = 0.0, nT0 = 0.0, nTn = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double ca = nhat<ST>(k, a);
      if (ca == 0.0) continue;
      nN += ca * Nb[a + 1];
      nT0 += ca * Ts[0][a + 1];
#pragma unroll
      for (int b = 0; b < D; ++b) {
        const double cb = nhat<ST>(k, b);
        if (cb == 0.0) continue;
        nTn += ca * cb * Ts[a + 1][b + 1];
      }
    }
    const double even = Nb[0] * p0 + Ts[0][0] * p0 * p0 + pm * pm * nTn;
    const double odd = pm * nN + 2.0 * p0 * pm * nT0;
    out[base + k] = (A)((double)out[base + k] + even + odd);
    out[base + k + 1] = (A)((double)out[base + k + 1] + even - odd);
  }
}

// dL/dF_i from dL/dN^a and dL/dT^ab (full matrix): sum_a Nb_a p^a + sum_ab Tb_ab p^a p^b.
template <class ST, typename A>
__device__ __forceinline__ void moments_vjp_add(const Tables *__restrict__ tb, const double (&Nb)[ST::D + 1],
                                                const double (&Tb)[ST::D + 1][ST::D + 1], A (&out)[ST::Q]) {
  constexpr int D = ST::D;
  // symmetric parts of Tb
  double Ts[D + 1][D + 1];
#pragma unroll
  for (int a = 0; a <= D; ++a)
#pragma unroll
    for (int b = 0; b <= D; ++b) Ts[a][b] = 0.5 * (Tb[a][b] + Tb[b][a]);
#pragma unroll
  for (int j = 0; j < ST::NSHELL; ++j) moments_vjp_shell<ST, A, ST::Q>(tb, j, Nb, Ts, out, j * ST::NDIR);
}

// Reverse of the macroscopic map F -> (n, eps, T, U) given the forward values, up to the
// moments: dL/dN^a (Nb) and dL/dT^ab (Tbar, full matrix) from the incoming adjoints nb, epsb,
// Tb, Ub (Ub is updated in place).
template <int D>
__device__ __forceinline__ void macro_vjp_moments(const Tables *__restrict__ tb, const double (&Nv)[D + 1],
                                                  const double (&T)[D + 1][D + 1], const Macro<D> &mac, double nb,
                                                  double epsb, double Tb, double (&Ub)[D + 1], double (&Nb)[D + 1],
                                                  double (&Tbar)[D + 1][D + 1]) {
  const double m = tb->m;
  const RatiosD rd = ratios_2d_d(m / mac.T);
  // T = EOS^{-1}(e), e = eps / n
  const double eb = Tb / eos_slope_2d(mac.T, m, rd);
  epsb += eb / mac.n;
  nb -= eb * mac.eps / (mac.n * mac.n);
  // n = U_a N^a
#pragma unroll
  for (int a = 0; a <= D; ++a) {
    Nb[a] = nb * eta_c(a, a) * mac.U[a];
    Ub[a] += nb * eta_c(a, a) * Nv[a];
  }
#pragma unroll
  for (int a = 0; a <= D; ++a)
#pragma unroll
    for (int b = 0; b <= D; ++b) Tbar[a][b] = 0.0;
  landau_vjp<D>(T, mac.eps, mac.U, epsb, Ub, Tbar);
}

// Reverse of the macroscopic map F -> (n, eps, T, U) given the forward values:
// adds dL/dF to out.  nb, epsb, Tb, Ub are the incoming adjoints.
template <class ST, typename A>
__device__ __forceinline__ void macro_vjp(const Tables *__restrict__ tb, const double (&Nv)[ST::D + 1],
                                          const double (&T)[ST::D + 1][ST::D + 1], const Macro<ST::D> &mac,
                                          double nb, double epsb, double Tb, double (&Ub)[ST::D + 1],
                                          A (&out)[ST::Q]) {
  constexpr int D = ST::D;
  double Nb[D + 1], Tbar[D + 1][D + 1];
  macro_vjp_moments<D>(tb, Nv, T, mac, nb, epsb, Tb, Ub, Nb, Tbar);
  moments_vjp_add<ST, A>(tb, Nb, Tbar, out);
}

// Reverse of the collision.  In: f = pre-collision populations F (storage
// precision; deviations for DEV), mu = dL/dB.  Out: f <- dL/dF, taub = dL/dtau.
template <class ST, int N, typename S, bool DEV>
__device__ __forceinline__ bool collide_vjp(const Tables *__restrict__ tb, S (&f)[ST::Q], const S (&mu)[ST::Q],
                                            double tau, double &taub) {
  constexpr int D = ST::D, ND = ST::NDIR, NPD = ND / 2, KR = ST::NSHELL;
  using B = BasisDef<D, N>;
  constexpr AngTable<D, N> AT{};
  // ---- forward recomputation ----
  double Nv[D + 1], T[D + 1][D + 1];
  moments_prod<ST, S, DEV>(tb, f, Nv, T);
  Macro<D> mac;
  mac.ok = landau_frame<D, 3>(T, mac.eps, mac.U);
  mac.n = lorentz_dot<D>(mac.U, Nv);
  const double m = tb->m;
  mac.ok = temperature_2d(mac.eps / mac.n, m, mac.T) && mac.ok;
  mac.ok = mac.ok && mac.n > 0.0 && mac.eps > 0.0;
  const RatiosD rd = ratios_2d_d(m / mac.T);
  Ratios rr;
  rr.r0 = rd.r0;
  rr.r2 = rd.r2;
  rr.r3 = rd.r3;
  double Md[B::NM];
  basis_moments<D, N>(mac.n, mac.T, mac.U, rr, Md);
  S feq[ST::Q];
  feq_prod<ST, N, S, DEV>(tb, Md, feq);
  const double itau = 1.0 / tau;
  const double a0 = mac.U[0] * itau;
  double nU[NPD];
#pragma unroll
  for (int q = 0; q < NPD; ++q) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double c = nhat<ST>(2 * q, a);
      if (c != 0.0) acc += c * mac.U[a + 1];
    }
    nU[q] = acc * itau;
  }
  // ---- reverse of the relaxation ----
  double a0b = 0.0, nUb[NPD];
#pragma unroll
  for (int q = 0; q < NPD; ++q) nUb[q] = 0.0;
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    const double v = tb->sv[j];
#pragma unroll
    for (int qp = 0; qp < NPD; ++qp) {
      const int i = j * ND + 2 * qp;
      const double b = v * nU[qp];
      const double om0 = a0 - b, om1 = a0 + b;
      const double g0 = (double)mu[i] * ((double)feq[i] - (double)f[i]);
      const double g1 = (double)mu[i + 1] * ((double)feq[i + 1] - (double)f[i + 1]);
      a0b += g0 + g1;
      nUb[qp] += v * (g1 - g0);
      // dL/df^eq_i = mu_i Omega_i (kept in feq), direct term mu_i (1 - Omega_i) (kept in f)
      feq[i] = (S)((double)mu[i] * om0);
      feq[i + 1] = (S)((double)mu[i + 1] * om1);
      f[i] = (S)((double)mu[i] * (1.0 - om0));
      f[i + 1] = (S)((double)mu[i + 1] * (1.0 - om1));
    }
  }
  // Omega depends on tau through a0 = U^0 / tau and nU = (n . U) / tau
  double Ub[D + 1];
  Ub[0] = a0b * itau;
  taub = -a0b * a0;
#pragma unroll
  for (int a = 1; a <= D; ++a) Ub[a] = 0.0;
#pragma unroll
  for (int q = 0; q < NPD; ++q) {
    taub -= nUb[q] * nU[q];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double c = nhat<ST>(2 * q, a);
      if (c != 0.0) Ub[a + 1] += c * nUb[q] * itau;
    }
  }
  taub *= itau;
  // ---- reverse of the equilibrium ----
  double Mb[B::NM];
  feq_vjp<ST, N, S>(tb, feq, Mb);
  double nb = 0.0, Tb = 0.0;
  basis_moments_vjp<D, N>(mac.n, mac.T, mac.U, m, rd, Mb, nb, Tb, Ub);
  // ---- reverse of EOS, density, Landau frame and moments ----
  macro_vjp<ST, S>(tb, Nv, T, mac, nb, 0.0, Tb, Ub, f);
  return mac.ok;
}


// ---------------------------------------------------------------------------
// The reverse step streamed shell by shell (2D product rules, float storage).
// collide_vjp keeps the populations, the adjoint and the equilibrium of all Q
// directions in registers at once; the streamed kernel pulls what each pass
// over the shells needs again (from the cache: the same taps were read moments
// before), so that one shell's populations are live at a time.
// ---------------------------------------------------------------------------

// Pre-collision values of shell j's populations: the interpolated pull of pull_prod (2D) for the
// directions of that shell; TRANSPOSE mirrors the taps as there.
template <class ST, typename S, bool TRANSPOSE, typename A>
__device__ __forceinline__ void pull_shell(const Tables *__restrict__ tb, const S *fin, int64_t sites, const Offs &o,
                                           int j, A (&fs)[ST::NDIR]) {
  static_assert(ST::D == 2, "the streamed reverse step is built for the 2D product rules");
  constexpr int ND = ST::NDIR;
  typedef const __attribute__((address_space(1))) char gchar;
  gchar *base = (gchar *)fin;
  const A v = tab<A>(tb->sv[j], tb->svf[j]);
  A pw[3][3];
#pragma unroll
  for (int z = 1; z <= 2; ++z) {
    const A mag = v * (A)kInvNorm[z];
    const A cm = (A)1 - mag;
#pragma unroll
    for (int nf = 0; nf <= z; ++nf) {
      A r = 1;
#pragma unroll
      for (int t = 0; t < nf; ++t) r *= mag;
#pragma unroll
      for (int t = nf; t < z; ++t) r *= cm;
      pw[z][nf] = r;
    }
  }
#pragma unroll
  for (int k = 0; k < ND; ++k) {
    gchar *plane = base + (int64_t)(j * ND + k) * sites * (int64_t)sizeof(S);
    const int dx = ST::dir(k, 0), dy = ST::dir(k, 1);
    const int z = (dx != 0) + (dy != 0);
    A acc = 0;
#pragma unroll
    for (int tap = 0; tap < (1 << z); ++tap) {
      int bit = 0, ox = 0, oy = 0, nfar = 0;
      if (dx != 0) {
        const int c = (tap >> bit++) & 1;
        ox = dx > 0 ? (c ? 0 : -1) : (c ? 1 : 0);
        nfar += ox != 0;
      }
      if (dy != 0) {
        const int c = (tap >> bit++) & 1;
        oy = dy > 0 ? (c ? 0 : -1) : (c ? 1 : 0);
        nfar += oy != 0;
      }
      if (TRANSPOSE) {
        ox = -ox;
        oy = -oy;
      }
      const uint32_t off = o.x[ox + 1] + o.y[oy + 1];
      acc += pw[z][nfar] * (A) * (const __attribute__((address_space(1))) S *)(plane + off);
    }
    fs[k] = acc;
  }
}

// Shell j's part of the reverse of the relaxation and of the equilibrium evaluation.  With
// B_i = F_i + Omega_i (f^eq_i - F_i), Omega_i = (U^0 - v_j n_i . U)/tau = a0 -+ v_j nU:
// dL/dOmega_i = mu_i (f^eq_i - F_i) accumulates into a0b and nUb, and dL/df^eq_i = mu_i Omega_i,
// pushed through the shell's equilibrium evaluation, into apb = dL/da'.  f and mu are the shell's
// pre-collision populations and adjoint (deviations for DEV, as is the equilibrium from ap).
template <class ST, int N, typename A>
__device__ __forceinline__ void relax_vjp_shell(const Tables *__restrict__ tb, int j, const A (&f)[ST::NDIR],
                                                const A (&mu)[ST::NDIR],
                                                const double (&ap)[BasisDef<ST::D, N>::NM], double a0,
                                                const double (&nU)[ST::NDIR / 2], double &a0b,
                                                double (&nUb)[ST::NDIR / 2], double (&apb)[BasisDef<ST::D, N>::NM]) {
  constexpr int D = ST::D, ND = ST::NDIR, NPD = ND / 2;
  constexpr AngTable<D, N> AT{};
  const double v = tb->sv[j];
  double ce[20], ceb[20];
  shell_coefficients<D, N>(tb, j, ap, ce);
#pragma unroll
  for (int q = 0; q < AT.n; ++q) ceb[q] = 0.0;
#pragma unroll
  for (int qp = 0; qp < NPD; ++qp) {
    const int k = 2 * qp;
    double E = 0.0, O = 0.0;
#pragma unroll
    for (int q = 0; q < AT.n; ++q) {
      const double c = nhat_pow<ST>(k, AT.e[q][0], AT.e[q][1], AT.e[q][2]) * dir_weight<ST>(k);
      const bool odd = (AT.e[q][0] + AT.e[q][1] + AT.e[q][2]) & 1;
      if (c == 0.0) continue;
      if (odd) O += c * ce[q];
      else E += c * ce[q];
    }
    const double b = v * nU[qp];
    const double m0 = (double)mu[k], m1 = (double)mu[k + 1];
    const double g0 = m0 * ((E + O) - (double)f[k]);
    const double g1 = m1 * ((E - O) - (double)f[k + 1]);
    a0b += g0 + g1;
    nUb[qp] += v * (g1 - g0);
    const double e0 = m0 * (a0 - b), e1 = m1 * (a0 + b);
    const double Eb = e0 + e1, Ob = e0 - e1;
#pragma unroll
    for (int q = 0; q < AT.n; ++q) {
      const double c = nhat_pow<ST>(k, AT.e[q][0], AT.e[q][1], AT.e[q][2]) * dir_weight<ST>(k);
      const bool odd = (AT.e[q][0] + AT.e[q][1] + AT.e[q][2]) & 1;
      if (c == 0.0) continue;
      ceb[q] += c * (odd ? Ob : Eb);
    }
  }
#pragma unroll
  for (int q = 0; q < AT.n; ++q) {
    const int l = AT.e[q][0] + AT.e[q][1] + AT.e[q][2];
    if (AT.m0[q] >= 0) apb[AT.m0[q]] += ceb[q] * tb->sfeq[j][0][l];
    if (AT.m1[q] >= 0) apb[AT.m1[q]] += ceb[q] * tb->sfeq[j][1][l];
  }
}

}  // namespace rlbm
