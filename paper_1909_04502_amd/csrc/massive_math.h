// massive_math.h -- collide for the on-lattice rules (HIP device code).
//
// An on-lattice rule (Sec. 5.3) is a union of groups of integer vectors n whose
// members share the energy p0_g and the weight w_g, with p = (p0_g, v_g n):
// for the massive rules the full-symmetric groups of the stencil, v_g = v0 p0_g
// (plus a rest vector); for the printed massless rules each (energy shell,
// full-symmetric group) pair, v_g = p0_g / |n|.  The integer vectors are
// compile-time constants, so the update needs only a few scalars per group:
//  * moments: per group, S = sum f, D^a = sum n^a f, S^ab = sum n^a n^b f
//    (antipodal pairs give sums and differences; the integer factors are
//    literals), then N^0 = sum_g p0 S, N^a = sum_g v D^a, T^00 = sum_g p0^2 S,
//    T^0a = sum_g p0 v D^a, T^ab = sum_g v^2 S^ab; the rest population adds m
//    and m^2 to N^0 and T^00;
//  * equilibrium: the projection of Eq. mj-discrete-feq over the shifted
//    monomials psi = (p^0 - m)^a p^e, a' = Linv^T Linv M' (Linv the inverse
//    Cholesky factor of their Gram matrix under the rule, block diagonal over
//    the parity classes), and f^eq_i = w_g psi(p_i)^T a'
//    = sum_e n_i^e [w_g v_g^|e| (a'_(0,e) + (p0_g - m) a'_(1,e))]: per group
//    one coefficient per angular monomial e, per population integer powers
//    n_i^e; the rest population keeps only the constant monomial, w_r a'_(0,0);
//  * relaxation Omega_i = (U^0 - v0 n_i . U)/tau;
//  * external force (Sec. 5.4, scheme B, EXT builds): the update adds
//    (m/T) ((g . v_i) U^0 - g . U) f^eq_i with v_i = v0 n_i, so per population
//    one integer dot product g . n_i on top of the relaxation.
#pragma once
#include "prod_math.h"

namespace rlbm {

// n_i^e of stencil population i (an integer)
template <class ST>
RLBM_HD constexpr int ipow_dir(int i, int ex, int ey, int ez) {
  int r = 1;
  for (int k = 0; k < ex; ++k) r *= ST::dir(i, 0);
  for (int k = 0; k < ey; ++k) r *= ST::dir(i, 1);
  if (ST::D == 3)
    for (int k = 0; k < ez; ++k) r *= ST::dir(i, 2);
  return r;
}

// a' = Linv^T Linv M' (coefficients of f^eq / w over the shifted monomials)
// from the Maxwell-Juettner moments of (n, T, U), class by class.
template <int D, int N, bool DEV, typename A>
__device__ __forceinline__ void massive_coefficients(const Tables *__restrict__ tb, const Macro<D> &mac,
                                                     const Ratios &rr, A (&ap)[BasisDef<D, N>::NM]) {
  using B = BasisDef<D, N>;
  const double m = tb->m;
  if constexpr (D == 3) {
    constexpr ClassTable<D, N> CL{};
    // the packed blocks are read class by class; laundering the table pointer on the previous
    // block's result keeps the compiler from hoisting (and spilling) all their scalar loads
    typedef const __attribute__((address_space(4))) double cdouble;
    cdouble *lp = (cdouble *)tb->LinvP;
    A prev = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      constexpr int kMax = 8;
      double mc[kMax], ak[kMax];
      if (c > 0) asm volatile("" : "+s"(lp) : "v"(prev));
#pragma unroll
      for (int t = 0; t < CL.cnt[c]; ++t) {
        const int k = CL.idx[c][t];
        mc[t] = basis_moment<D, N>(k, mac.n, mac.T, mac.U, rr);
        if constexpr (DEV) mc[t] -= tb->Mref[k];
      }
#pragma unroll
      for (int t = 0; t < CL.cnt[c]; ++t) {
        const int pk = CL.partner[CL.idx[c][t]];
        if (pk >= 0) mc[t] -= m * mc[CL.pos[pk]];
      }
#pragma unroll
      for (int t = 0; t < CL.cnt[c]; ++t) {
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u <= t; ++u) acc += lp[CL.off[c] + t * (t + 1) / 2 + u] * mc[u];
        ak[t] = acc;
      }
      asm volatile("" : "+s"(lp) : "v"(ak[CL.cnt[c] - 1]));
#pragma unroll
      for (int u = 0; u < CL.cnt[c]; ++u) {
        double acc = 0.0;
#pragma unroll
        for (int t = u; t < CL.cnt[c]; ++t) acc += lp[CL.off[c] + t * (t + 1) / 2 + u] * ak[t];
        ap[CL.idx[c][u]] = (A)acc;
      }
      prev = ap[CL.idx[c][0]];
    }
  } else {
    constexpr AngTable<D, N> AT{};
    double Md[B::NM];
    basis_moments<D, N>(mac.n, mac.T, mac.U, rr, Md);
    if constexpr (DEV) {
#pragma unroll
      for (int k = 0; k < B::NM; ++k) Md[k] -= tb->Mref[k];
    }
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
      ap[c] = (A)acc;
    }
  }
}

// The update of one site with the populations reached through callbacks:
// fetch(i) returns the pre-collision f_i for the moments, refetch(i) returns it
// again for the relaxation, and put(i, v) takes the post-collision value.  The
// register-resident collide passes its array; the streaming kernel loads from
// memory twice and stores directly, so that no population stays live across
// the eigen-solve and the projection.
// EXT: no-slip wall planes (site_wall), in a separate instantiation: a wall
// site takes the equilibrium at rest of its own n and its own or the plane's
// prescribed temperature (Omega = 1).
// REVERSE relaxes the groups in the reverse of their loading order (the rest
// population first); every population's update is independent of the others,
// so only the instruction order changes (4 % faster for the register-resident
// 3D rule in float deviations, slower for the streaming kernel).
template <class ST, int N, typename S, bool DEV, bool RELAX, bool EXT, bool REVERSE, class Fetch, class Refetch,
          class Put>
__device__ __forceinline__ Macro<ST::D> massive_update(const Tables *__restrict__ tb, double tau, double wallT,
                                                       Fetch &&fetch, Refetch &&refetch, Put &&put) {
  constexpr int D = ST::D, Q = ST::Q, NG = ST::NG, NT = D * (D + 1) / 2;
  constexpr bool REST = (Q & 1) != 0;   // an odd count carries a rest population, the last one
  using B = BasisDef<D, N>;
  constexpr AngTable<D, N> AT{};
  typedef S A;
  // ---- step 1: moments ----
  A N0 = 0, T00 = 0, Na[D], T0a[D], Tab[NT];
#pragma unroll
  for (int a = 0; a < D; ++a) Na[a] = T0a[a] = 0;
#pragma unroll
  for (int a = 0; a < NT; ++a) Tab[a] = 0;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    A S0 = 0, Sa[D], Sab[NT];
#pragma unroll
    for (int a = 0; a < D; ++a) Sa[a] = 0;
#pragma unroll
    for (int a = 0; a < NT; ++a) Sab[a] = 0;
#pragma unroll
    for (int i = ST::gfirst(g); i < ST::gfirst(g) + ST::gcount(g); i += 2) {
      const A fi = fetch(i), fj = fetch(i + 1);
      const A s = fi + fj;
      const A d = fi - fj;
      S0 += s;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const int c = ST::dir(i, a);
        if (c == 1) Sa[a] += d;
        else if (c == -1) Sa[a] -= d;
        else if (c != 0) Sa[a] += (A)c * d;
      }
      int ab = 0;
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b) {
          const int c = ST::dir(i, a) * ST::dir(i, b);
          if (c == 1) Sab[ab] += s;
          else if (c == -1) Sab[ab] -= s;
          else if (c != 0) Sab[ab] += (A)c * s;
          ++ab;
        }
    }
    const A p0 = tab<A>(tb->mgrp[g][0], tb->mgrpf[g][0]);
    const A p00 = tab<A>(tb->mgrp[g][1], tb->mgrpf[g][1]);
    const A v = tab<A>(tb->mgrp[g][2], tb->mgrpf[g][2]);
    const A p0v = tab<A>(tb->mgrp[g][3], tb->mgrpf[g][3]);
    const A vv = tab<A>(tb->mgrp[g][4], tb->mgrpf[g][4]);
    N0 += p0 * S0;
    T00 += p00 * S0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      Na[a] += v * Sa[a];
      T0a[a] += p0v * Sa[a];
    }
#pragma unroll
    for (int a = 0; a < NT; ++a) Tab[a] += vv * Sab[a];
  }
  if constexpr (REST) {
    const double m = tb->m;
    const A fr = fetch(Q - 1);
    N0 += (A)m * fr;
    T00 += (A)(m * m) * fr;
  }
  double Nv[D + 1], T[D + 1][D + 1];
  Nv[0] = N0;
  T[0][0] = T00;
  {
    int ab = 0;
#pragma unroll
    for (int a = 1; a <= D; ++a) {
      Nv[a] = Na[a - 1];
      T[0][a] = T[a][0] = T0a[a - 1];
#pragma unroll
      for (int b = a; b <= D; ++b) {
        T[a][b] = T[b][a] = Tab[ab];
        ++ab;
      }
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
  // ---- steps 2-4 ----
  Macro<D> mac;
  mac.ok = landau_frame<D, 3>(T, mac.eps, mac.U);
  mac.n = lorentz_dot<D>(mac.U, Nv);
  const double m = tb->m;
  Ratios rr;
  if constexpr (D == 2) {
    mac.ok = temperature_2d(mac.eps / mac.n, m, mac.T) && mac.ok;
    rr = ratios_2d(m / mac.T);
  } else {
    double r;
    mac.ok = temperature_3d(tb, mac.eps / mac.n, m, mac.T, r) && mac.ok;
    rr = ratios_3d(m / mac.T, r);
  }
  mac.ok = mac.ok && mac.n > 0.0 && mac.eps > 0.0;
  if constexpr (!RELAX) return mac;
  // ---- step 5: a' over the shifted monomials ----
  A ap[B::NM];
  const bool wall = EXT && wallT >= 0.0;
  if (wall) {
    Macro<D> meq = mac;
    Ratios req;
    equilibrium_state<D>(tb, mac, rr, wallT, meq.T, req);
    meq.U[0] = 1.0;
#pragma unroll
    for (int a = 1; a <= D; ++a) meq.U[a] = 0.0;
    massive_coefficients<D, N, DEV, A>(tb, meq, req, ap);
  } else {
    massive_coefficients<D, N, DEV, A>(tb, mac, rr, ap);
  }
  // ---- step 7: the temperature-dependent part of tau ----
  if (tb->tau_T != 0.0) tau += tb->tau_T / mac.T;
  // ---- step 8: Omega_i = a0 - v0 (n_i . U)/tau (1 on a wall) ----
  const double itau = wall ? 0.0 : 1.0 / tau;
  const A a0 = wall ? (A)1 : (A)(mac.U[0] * itau);
  A ub[D];
#pragma unroll
  for (int a = 0; a < D; ++a) ub[a] = (A)(tb->v0 * mac.U[a + 1] * itau);
  // ---- step 6, external force (Sec. 5.4, scheme B): + (m/T) ((g . v_i) U^0 - g . U) f^eq_i ----
  const bool force = EXT && tb->has_force && !wall;
  A cF = 0, gU = 0, gv[D];
#pragma unroll
  for (int a = 0; a < D; ++a) gv[a] = 0;
  if (force) {
    cF = (A)(tb->m / mac.T);
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      acc += tb->g[a] * mac.U[a + 1];
      gv[a] = (A)(tb->v0 * tb->g[a] * mac.U[0]);   // (g . v_i) U^0 = sum_a n_i^a gv[a]
    }
    gU = (A)acc;
  }
  // full equilibrium of population i from its deviation part (float-deviation storage)
  auto feq_full = [&](int i, A e) { return DEV ? e + tab<A>(tb->fref[i], tb->freff[i]) : e; };
  auto relax_rest = [&]() {
    if constexpr (REST) {
      const A E = ap[0] * tab<A>(tb->wrest, tb->wrestf);   // the constant monomial is basis entry 0
      const A fr = refetch(Q - 1);
      A out = fr + a0 * (E - fr);
      if (force) out -= cF * gU * feq_full(Q - 1, E);
      put(Q - 1, out);
    }
  };
  if constexpr (REST && REVERSE) relax_rest();
  // each group's populations are fetched before any of it is relaxed: in the streaming kernel its
  // re-loads are then in flight together instead of one pair per memory round trip (a store between
  // two re-loads makes the wave wait for every access it has in flight)
  constexpr int GMAX = [] {
    int mx = 0;
    for (int g = 0; g < NG; ++g) mx = ST::gcount(g) > mx ? ST::gcount(g) : mx;
    return mx;
  }();
#pragma unroll
  for (int gg = 0; gg < NG; ++gg) {
    const int g = REVERSE ? NG - 1 - gg : gg;
    A fg[GMAX];
#pragma unroll
    for (int j = 0; j < ST::gcount(g); ++j) fg[j] = refetch(ST::gfirst(g) + j);
    A ce[20];
#pragma unroll
    for (int q = 0; q < AT.n; ++q) {
      const int l = AT.e[q][0] + AT.e[q][1] + AT.e[q][2];
      A acc = 0;
      if (AT.m0[q] >= 0) acc += ap[AT.m0[q]] * tab<A>(tb->mgrp[g][5 + l], tb->mgrpf[g][5 + l]);
      if (AT.m1[q] >= 0) acc += ap[AT.m1[q]] * tab<A>(tb->mgrp[g][9 + l], tb->mgrpf[g][9 + l]);
      ce[q] = acc;
    }
#pragma unroll
    for (int ii = 0; ii < ST::gcount(g); ii += 2) {
      const int i = REVERSE ? ST::gfirst(g) + ST::gcount(g) - 2 - ii : ST::gfirst(g) + ii;
      A E = 0, O = 0;
#pragma unroll
      for (int q = 0; q < AT.n; ++q) {
        const int c = ipow_dir<ST>(i, AT.e[q][0], AT.e[q][1], AT.e[q][2]);
        if (c == 0) continue;
        const bool odd = (AT.e[q][0] + AT.e[q][1] + AT.e[q][2]) & 1;
        const A t = c == 1 ? ce[q] : (c == -1 ? -ce[q] : (A)c * ce[q]);
        if (odd) O += t;
        else E += t;
      }
      A b = 0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const int c = ST::dir(i, a);
        if (c == 1) b += ub[a];
        else if (c == -1) b -= ub[a];
        else if (c != 0) b += (A)c * ub[a];
      }
      const A om0 = a0 - b, om1 = a0 + b;
      const A f0 = fg[i - ST::gfirst(g)], f1 = fg[i + 1 - ST::gfirst(g)];
      A out0 = f0 + om0 * ((E + O) - f0);
      A out1 = f1 + om1 * ((E - O) - f1);
      if (force) {
        A gn = 0;   // (g . v_i) U^0 of the pair's first member; the second has the opposite sign
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const int c = ST::dir(i, a);
          if (c == 1) gn += gv[a];
          else if (c == -1) gn -= gv[a];
          else if (c != 0) gn += (A)c * gv[a];
        }
        out0 += cF * (gn - gU) * feq_full(i, E + O);
        out1 += cF * (-gn - gU) * feq_full(i + 1, E - O);
      }
      put(i, out0);
      put(i + 1, out1);
    }
  }
  if constexpr (REST && !REVERSE) relax_rest();
  return mac;
}

template <class ST, int N, typename S, bool DEV, bool RELAX, bool EXT = false>
__device__ __forceinline__ Macro<ST::D> collide_massive(const Tables *__restrict__ tb, S (&f)[ST::Q], double tau,
                                                        double wallT = -1.0) {
  auto get = [&](int i) { return f[i]; };
  return massive_update<ST, N, S, DEV, RELAX, EXT, ST::D == 3>(tb, tau, wallT, get, get,
                                                                [&](int i, S v) { f[i] = v; });
}

}  // namespace rlbm
