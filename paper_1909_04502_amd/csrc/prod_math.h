// prod_math.h -- collide for the off-lattice product rules (HIP device code).
//
// The populations of a product rule are p_jk = (p0_j, |p|_j n_k): shells j
// times unit directions n_k.  The update is evaluated through that structure:
//  * moments: per shell, direction sums S0 = sum_k f, S^a = sum_k n^a f,
//    S^ab = sum_k n^a n^b f (antipodal pairs give sums / differences), then
//    N^0 = sum_j p0 S0, N^a = sum_j |p| S^a, T^00 = sum_j p0^2 S0,
//    T^0a = sum_j p0 |p| S^a, T^ab = sum_j |p|^2 S^ab;
//  * equilibrium: f^eq_i = w_i psi(p_i)^T G^{-1} M (M the Maxwell-Juettner
//    moments of the monomials psi = (p^0 - m)^a p^e, G their Gram matrix
//    under the quadrature; this is the projection of Eq. mj-discrete-feq).
//    G^{-1} = Linv^T Linv with Linv the inverse Cholesky factor, both block
//    diagonal over the parity classes of the monomials; a = Linv M are the
//    coefficients on the orthonormal polynomials J = Linv psi and with
//    a' = Linv^T a, per shell c_e = sum_a a'_(a,e) W_j (p0 - m)^a |p|^|e| and
//    f^eq_jk = omega_k sum_e c_e n_k^e, the direction powers n_k^e being
//    compile-time constants;
//  * relaxation Omega_jk = (U^0 - v_j n_k . U)/tau with per-site n_k . U.
// Only per-shell scalars and the used Linv entries are read from the tables.
#pragma once
#include "device_math.h"

namespace rlbm {

constexpr double kInvNorm[4] = {0.0, 1.0, 0.70710678118654752440, 0.57735026918962576451};

template <class ST>
RLBM_HD constexpr int nnz_dir(int k) {
  int c = 0;
  for (int a = 0; a < ST::D; ++a) c += ST::dir(k, a) != 0;
  return c;
}

// unit direction component n_k^a
template <class ST>
RLBM_HD constexpr double nhat(int k, int a) {
  return ST::dir(k, a) * kInvNorm[nnz_dir<ST>(k)];
}

// n_k^e = prod_a (n_k^a)^{e_a}
template <class ST>
RLBM_HD constexpr double nhat_pow(int k, int ex, int ey, int ez) {
  double r = 1.0;
  for (int i = 0; i < ex; ++i) r *= nhat<ST>(k, 0);
  for (int i = 0; i < ey; ++i) r *= nhat<ST>(k, 1);
  if (ST::D == 3)
    for (int i = 0; i < ez; ++i) r *= nhat<ST>(k, 2);
  return r;
}

// absolute direction weight in 3D (exact for spherical degree <= 7); folded in the shell factors in 2D
template <class ST>
RLBM_HD constexpr double dir_weight(int k) {
  if (ST::D == 2) return 1.0;
  const int z = nnz_dir<ST>(k);
  return z == 1 ? 1.0 / 21.0 : (z == 2 ? 4.0 / 105.0 : 9.0 / 280.0);
}

template <typename A>
__device__ __forceinline__ A tab(const double &d, const float &f) {
  if constexpr (sizeof(A) == 8) return d;
  else return f;
}

// Byte offsets of the upstream neighbours (-1, 0, +1) along each axis.
struct Offs {
  uint32_t x[3], y[3], z[3];
};

// Pre-collision populations of a product rule (pull + multilinear interpolation).
// Tap weights are mag^{n_far} (1 - mag)^{n_near}, mag = v_j / sqrt(number of
// non-zero direction components), n_far the number of taps one site upstream.
// With TRANSPOSE the taps are mirrored (offset -o, same weight): this applies
// the transpose of the streaming operator on a periodic grid (the adjoint
// gather dL/dB(y) = sum_taps w dL/dF(y - o)).
// 3D: the 26 directions of a shell fall into groups of at most 16 taps (the
// axes, the edges by fours, the corners by twos); the loads of group g depend
// (through an empty asm on the plane base) on every population of group g - 3,
// so at most three groups of taps are in flight per wave instead of all of
// them, and the registers their loads occupy stay bounded.
__device__ __forceinline__ constexpr bool group_start_3d(int k) {
  return k == 0 || k == 6 || k == 10 || k == 14 || k == 18 || k == 20 || k == 22 || k == 24;
}
__device__ __forceinline__ constexpr int group_first_3d(int k) { return k < 6 ? 0 : k < 18 ? 6 + 4 * ((k - 6) / 4) : k & ~1; }

// A is the arithmetic type of the interpolation and of the result (the storage type S, or double
// for float deviations updated in double).
template <class ST, typename S, bool TRANSPOSE = false, typename A = S>
__device__ __forceinline__ void pull_prod(const Tables *__restrict__ tb, const S *__restrict__ fin, int64_t sites,
                                          const Offs &o, A (&f)[ST::Q]) {
  constexpr int D = ST::D, ND = ST::NDIR, KR = ST::NSHELL;
  typedef const __attribute__((address_space(1))) char gchar;   // keeps the loads global after laundering
  gchar *base = (gchar *)fin;
  // population ranges [first, last] of the previous groups (index 0 most recent); the loads of a
  // group depend on every population of the group kDepth back
  constexpr int kDepth = 3;
  int gfirst[kDepth], glast[kDepth];
#pragma unroll
  for (int e = 0; e < kDepth; ++e) gfirst[e] = glast[e] = -1;
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    const A v = tab<A>(tb->sv[j], tb->svf[j]);
    A pw[4][4];
#pragma unroll
    for (int z = 1; z <= D; ++z) {
      const A mag = v * (A)kInvNorm[z];
      const A cm = (A)1 - mag;
      // pw[z][nf] = mag^nf (1-mag)^(z-nf)
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
      const int i = j * ND + k;
      if constexpr (D == 3) {
        if (group_start_3d(k) && glast[kDepth - 1] >= 0) {
#pragma unroll
          for (int q = gfirst[kDepth - 1]; q <= glast[kDepth - 1]; ++q) asm volatile("" : "+s"(base) : "v"(f[q]));
        }
      }
      gchar *plane = base + (int64_t)i * sites * (int64_t)sizeof(S);
      const int dx = ST::dir(k, 0), dy = ST::dir(k, 1), dz = D == 3 ? ST::dir(k, D - 1) : 0;
      const int z = (dx != 0) + (dy != 0) + (dz != 0);
      A acc = 0;
      {
#pragma unroll
      for (int tap = 0; tap < (1 << z); ++tap) {
        int bit = 0, ox = 0, oy = 0, oz = 0, nfar = 0;
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
        if (dz != 0) {
          const int c = (tap >> bit++) & 1;
          oz = dz > 0 ? (c ? 0 : -1) : (c ? 1 : 0);
          nfar += oz != 0;
        }
        if (TRANSPOSE) {
          ox = -ox;
          oy = -oy;
          oz = -oz;
        }
        const uint32_t off = o.x[ox + 1] + o.y[oy + 1] + o.z[oz + 1];
        acc += pw[z][nfar] * (A) * (const __attribute__((address_space(1))) S *)(plane + off);
      }
      f[i] = acc;
      }
      if constexpr (D == 3) {
        if (k == ND - 1 || group_start_3d(k + 1)) {
#pragma unroll
          for (int e = kDepth - 1; e > 0; --e) {
            gfirst[e] = gfirst[e - 1];
            glast[e] = glast[e - 1];
          }
          gfirst[0] = j * ND + group_first_3d(k);
          glast[0] = i;
        }
      }
    }
  }
}

// Wall temperature of a site: negative off the walls; on the first or last
// plane of a wall axis the prescribed temperature of that plane, or 0 for the
// site's own temperature.
__device__ __forceinline__ double site_wall(const Tables *__restrict__ tb, int x, int y, int z) {
  if (tb->wall[0] && (x == 0 || x == tb->nx - 1)) return tb->wallT[0][x == 0 ? 0 : 1];
  if (tb->wall[1] && (y == 0 || y == tb->ny - 1)) return tb->wallT[1][y == 0 ? 0 : 1];
  if (tb->wall[2] && (z == 0 || z == tb->nz - 1)) return tb->wallT[2][z == 0 ? 0 : 1];
  return -1.0;
}

// The temperature and moment ratios the equilibrium is built from: the
// site's own, or a wall plane's prescribed temperature.
template <int D>
__device__ __forceinline__ void equilibrium_state(const Tables *__restrict__ tb, const Macro<D> &mac,
                                                  const Ratios &rr, double wallT, double &Te, Ratios &re) {
  Te = mac.T;
  re = rr;
  if (wallT > 0.0) {
    Te = wallT;
    if constexpr (D == 2) {
      re = ratios_2d(tb->m / Te);
    } else {
      bool inr = true;
      const double r = tb->m == 0.0 ? 0.0 : cheb_r(tb, tb->m / Te, inr);
      re = ratios_3d(tb->m / Te, r);
    }
  }
}

// EXT: build the external-force term and the no-slip wall sites in (a separate
// instantiation, so that lattices without them keep the leaner kernel).
// wallT: see site_wall.
template <class ST, int N, typename S, bool DEV, bool RELAX, bool EXT = false>
__device__ __forceinline__ Macro<ST::D> collide_prod(const Tables *__restrict__ tb, S (&f)[ST::Q], double tau,
                                                     double wallT = -1.0) {
  const bool wall = EXT && wallT >= 0.0;
  constexpr int D = ST::D, ND = ST::NDIR, NPD = ND / 2, KR = ST::NSHELL;
  using B = BasisDef<D, N>;
  constexpr AngTable<D, N> AT{};
  typedef S A;
  // ---- step 1: moments ----
  A N0 = 0, T00 = 0, Na[D], T0a[D], Tab[D * (D + 1) / 2];
#pragma unroll
  for (int a = 0; a < D; ++a) Na[a] = T0a[a] = 0;
#pragma unroll
  for (int a = 0; a < D * (D + 1) / 2; ++a) Tab[a] = 0;
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    A S0 = 0, Sa[D], Sab[D * (D + 1) / 2];
#pragma unroll
    for (int a = 0; a < D; ++a) Sa[a] = 0;
#pragma unroll
    for (int a = 0; a < D * (D + 1) / 2; ++a) Sab[a] = 0;
#pragma unroll
    for (int q = 0; q < NPD; ++q) {
      const int k = 2 * q;
      const A s = f[j * ND + k] + f[j * ND + k + 1];
      const A d = f[j * ND + k] - f[j * ND + k + 1];
      S0 += s;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double c = nhat<ST>(k, a);
        if (c == 1.0) Sa[a] += d;
        else if (c == -1.0) Sa[a] -= d;
        else if (c != 0.0) Sa[a] += (A)c * d;
      }
      int ab = 0;
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b) {
          const double c = nhat<ST>(k, a) * nhat<ST>(k, b);
          if (c == 1.0) Sab[ab] += s;
          else if (c != 0.0) Sab[ab] += (A)c * s;
          ++ab;
        }
    }
    const A p0 = tab<A>(tb->smom[j][0], tb->smomf[j][0]);
    const A pm = tab<A>(tb->smom[j][1], tb->smomf[j][1]);
    const A p00 = tab<A>(tb->smom[j][2], tb->smomf[j][2]);
    const A p0m = tab<A>(tb->smom[j][3], tb->smomf[j][3]);
    const A pmm = tab<A>(tb->smom[j][4], tb->smomf[j][4]);
    N0 += p0 * S0;
    T00 += p00 * S0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      Na[a] += pm * Sa[a];
      T0a[a] += p0m * Sa[a];
    }
#pragma unroll
    for (int a = 0; a < D * (D + 1) / 2; ++a) Tab[a] += pmm * Sab[a];
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
  Macro<ST::D> mac;
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
  // a no-slip wall site relaxes fully (Omega = 1) to the equilibrium at rest of its own n and
  // its own or the wall's prescribed T
  double Ue[D + 1];
#pragma unroll
  for (int a = 0; a <= D; ++a) Ue[a] = wall ? (a == 0 ? 1.0 : 0.0) : mac.U[a];
  double Te = mac.T;
  Ratios re = rr;
  if (wall) equilibrium_state<D>(tb, mac, rr, wallT, Te, re);
  // ---- step 5: a' = G^{-1} M over parity blocks ----
  A ap[B::NM];
  if constexpr (D == 3) {
    // class by class (moments, shift, L^{-1}, L^{-T}), so that only one block's
    // temporaries are live next to the populations
    constexpr ClassTable<D, N> CL{};
    // the packed blocks are read class by class: laundering the table pointer on the previous
    // block's result keeps the compiler from hoisting (and spilling) all 91 scalar loads
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
        mc[t] = basis_moment<D, N>(k, mac.n, Te, Ue, re);
        if constexpr (DEV) mc[t] -= tb->Mref[k];
      }
      // moments of the shifted monomials (p^0 - m) p^e = p^0 p^e - m p^e
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
      // reload the block for the transposed pass rather than keep it in (spilled) scalar registers
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
    double Md[B::NM];
    basis_moments<D, N>(mac.n, Te, Ue, re, Md);
    if constexpr (DEV) {
#pragma unroll
      for (int k = 0; k < B::NM; ++k) Md[k] -= tb->Mref[k];
    }
    // moments of the shifted monomials (p^0 - m) p^e = p^0 p^e - m p^e
#pragma unroll
    for (int q = 0; q < AT.n; ++q)
      if (AT.m1[q] >= 0) Md[AT.m1[q]] -= m * Md[AT.m0[q]];
    // projection coefficients on the orthonormal polynomials J = Linv psi
    // (Eq. mj-projection-coefficients), then a' = Linv^T a so that
    // f^eq_i = w_i psi(p_i)^T a' = w_i sum_k a_k J_k(p_i)
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
  // ---- step 8 ingredients: Omega_jk = a0 - v_j (n_k . U)/tau ----
  const double itau = wall ? 0.0 : 1.0 / tau;
  const A a0 = wall ? (A)1 : (A)(mac.U[0] * itau);
  A nU[NPD];
#pragma unroll
  for (int q = 0; q < NPD; ++q) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double c = nhat<ST>(2 * q, a);
      if (c != 0.0) acc += c * mac.U[a + 1];
    }
    nU[q] = (A)(acc * itau);
  }
  // ---- step 6, external force (Sec. 5.4, scheme B): the update adds
  //      (m/T) (K^a U_a / p_i^0) f^eq_i = (m/T) ((g . v_i) U^0 - g . U) f^eq_i ----
  const bool force = EXT && tb->has_force && !wall;
  A cF = 0, cU0 = 0, gU = 0;
  if (force) {
    cF = (A)(tb->m / mac.T);
    cU0 = (A)mac.U[0];
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) acc += tb->g[a] * mac.U[a + 1];
    gU = (A)acc;
  }
  auto gdotn = [&](int q) {   // g . n_k of the pair's first member
    A acc = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double c = nhat<ST>(2 * q, a);
      if (c != 0.0) acc += (A)c * tab<A>(tb->g[a], tb->gf[a]);
    }
    return acc;
  };
  if constexpr (D == 3) {
    // Direction-major: f^eq_jk = sum_l (s0_jl P0_kl + s1_jl P1_kl) with the
    // shell-independent angular sums P_kl = sum_{|e| = l} a'_{m(e)} w_k n_k^e,
    // so only the 8 sums of one direction pair are live next to a'.
#pragma unroll
    for (int qp = 0; qp < NPD; ++qp) {
      const int k = 2 * qp;
      A P0[4] = {0, 0, 0, 0}, P1[4] = {0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < AT.n; ++q) {
        const double c = nhat_pow<ST>(k, AT.e[q][0], AT.e[q][1], AT.e[q][2]) * dir_weight<ST>(k);
        if (c == 0.0) continue;
        const int l = AT.e[q][0] + AT.e[q][1] + AT.e[q][2];
        if (AT.m0[q] >= 0) P0[l] += (A)c * ap[AT.m0[q]];
        if (AT.m1[q] >= 0) P1[l] += (A)c * ap[AT.m1[q]];
      }
#pragma unroll
      for (int j = 0; j < KR; ++j) {
        A E = 0, O = 0;
#pragma unroll
        for (int l = 0; l <= N; ++l) {
          const A t = tab<A>(tb->sfeq[j][0][l], tb->sfeqf[j][0][l]) * P0[l] +
                      tab<A>(tb->sfeq[j][1][l], tb->sfeqf[j][1][l]) * P1[l];
          if (l & 1) O += t;
          else E += t;
        }
        const A vj = tab<A>(tb->sv[j], tb->svf[j]);
        const A b = vj * nU[qp];
        const A om0 = a0 - b, om1 = a0 + b;
        const int i = j * ND + k;
        const A f0 = f[i], f1 = f[i + 1];
        f[i] = f0 + om0 * ((E + O) - f0);
        f[i + 1] = f1 + om1 * ((E - O) - f1);
        if (force) {
          const A gv = vj * gdotn(qp) * cU0;
          const A fe0 = (E + O) + (DEV ? tab<A>(tb->fref[i], tb->freff[i]) : (A)0);
          const A fe1 = (E - O) + (DEV ? tab<A>(tb->fref[i + 1], tb->freff[i + 1]) : (A)0);
          f[i] += cF * (gv - gU) * fe0;
          f[i + 1] += cF * (-gv - gU) * fe1;
        }
      }
    }
    return mac;
  }
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    A ce[20];
#pragma unroll
    for (int q = 0; q < AT.n; ++q) {
      const int l = AT.e[q][0] + AT.e[q][1] + AT.e[q][2];
      A acc = 0;
      if (AT.m0[q] >= 0) acc += ap[AT.m0[q]] * tab<A>(tb->sfeq[j][0][l], tb->sfeqf[j][0][l]);
      if (AT.m1[q] >= 0) acc += ap[AT.m1[q]] * tab<A>(tb->sfeq[j][1][l], tb->sfeqf[j][1][l]);
      ce[q] = acc;
    }
    const A v = tab<A>(tb->sv[j], tb->svf[j]);
#pragma unroll
    for (int qp = 0; qp < NPD; ++qp) {
      const int k = 2 * qp;
      A E = 0, O = 0;
#pragma unroll
      for (int q = 0; q < AT.n; ++q) {
        const double c = nhat_pow<ST>(k, AT.e[q][0], AT.e[q][1], AT.e[q][2]) * dir_weight<ST>(k);
        const bool odd = (AT.e[q][0] + AT.e[q][1] + AT.e[q][2]) & 1;
        if (c == 0.0) continue;
        if (odd) O += (A)c * ce[q];
        else E += (A)c * ce[q];
      }
      const A b = v * nU[qp];
      const A om0 = a0 - b, om1 = a0 + b;
      const int i = j * ND + k;
      const A f0 = f[i], f1 = f[i + 1];
      f[i] = f0 + om0 * ((E + O) - f0);
      f[i + 1] = f1 + om1 * ((E - O) - f1);
      if (force) {
        const A gv = v * gdotn(qp) * cU0;
        const A fe0 = (E + O) + (DEV ? tab<A>(tb->fref[i], tb->freff[i]) : (A)0);
        const A fe1 = (E - O) + (DEV ? tab<A>(tb->fref[i + 1], tb->freff[i + 1]) : (A)0);
        f[i] += cF * (gv - gU) * fe0;
        f[i + 1] += cF * (-gv - gU) * fe1;
      }
    }
  }
  return mac;
}

}  // namespace rlbm
