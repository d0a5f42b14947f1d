// rlbm_defs.h -- compile-time descriptions shared by the host precompute and
// the HIP kernels of the RLBM library: stencils (direction sets and
// population order), the polynomial basis used for the projected equilibrium,
// and the layout of the per-lattice constant tables in device memory.
#pragma once
#include <cstdint>

#ifndef RLBM_HD
#if defined(__HIPCC__)
#define RLBM_HD __host__ __device__
#else
#define RLBM_HD
#endif
#endif

namespace rlbm {

enum StencilId : int { ST_UR2D = 0, ST_PROD2D = 1, ST_PROD3D = 2, ST_MASSIVE2D = 3, ST_MASSIVE3D = 4, ST_UR3D = 5 };

// ---------------------------------------------------------------------------
// Direction sets.  Antipodal directions are adjacent (k, k+1 for even k).
// ---------------------------------------------------------------------------

// 2D product rule: unit vectors along these integer directions.
constexpr int kDir2D[8][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, -1}, {-1, 1}, {1, -1}};

// 3D product rule: 6 axis, 12 edge and 8 corner directions (octahedral symmetry).
constexpr int kDir3D[26][3] = {
    {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0}, {0, 0, 1},   {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1},
    {1, 0, -1}, {-1, 0, 1},  {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1},  {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, -1},
    {-1, 1, 1}, {1, -1, -1}};

// Printed massless (2+1)-d order-2 rule (Sec. 5.3 worked example, App. H.2):
// stencil (+-3,+-4)_FS U (+-5,0)_FS; populations in shell-major order with the
// zero-weight (+-5,0) members of shells 1 and 2 dropped.
constexpr int kDirUR[12][2] = {{3, 4},  {-3, -4}, {-3, 4}, {3, -4}, {4, 3},  {-4, -3},
                               {-4, 3}, {4, -3},  {5, 0},  {-5, 0}, {0, 5},  {0, -5}};
constexpr int kUR2DQ = 28;
// population -> (shell, direction) for the printed rule
constexpr int kURShell[kUR2DQ] = {0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 1,
                                  2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2};
constexpr int kURDir[kUR2DQ] = {0, 1, 2, 3, 4, 5, 6, 7, 0, 1, 2, 3, 4, 5, 6, 7,
                                0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11};

// Massive on-lattice rules (Sec. 5.3): generating vectors of the full-symmetric
// groups besides the rest vector.  2D order 2: the 29-vector stencil of the
// worked example; 2D order 3 and 3D order 3: the 45- and 143-vector stencils
// of the GPU benchmark (Sec. 6.3).
constexpr int kMassiveGroups2 = 5, kMassiveGroups3 = 9, kMassiveGroups3D = 10;
constexpr int kMassiveGen2[kMassiveGroups2][3] = {{1, 0, 0}, {1, 1, 0}, {2, 1, 0}, {2, 2, 0}, {3, 1, 0}};
constexpr int kMassiveGen3[kMassiveGroups3][3] = {{1, 0, 0}, {1, 1, 0}, {2, 0, 0}, {2, 1, 0}, {2, 2, 0},
                                                  {3, 0, 0}, {3, 2, 0}, {3, 3, 0}, {4, 0, 0}};
constexpr int kMassiveGen3D[kMassiveGroups3D][3] = {{1, 0, 0}, {1, 1, 1}, {2, 0, 0}, {2, 1, 1}, {2, 2, 0},
                                                    {2, 2, 1}, {2, 2, 2}, {3, 0, 0}, {3, 1, 1}, {3, 2, 0}};
constexpr int kMaxMassiveGroups = 10;

// Non-rest vectors of a massive stencil in population order: per group, the
// members with first non-zero component > 0 in decreasing lexicographic order,
// each followed by its opposite.  The rest vector is population Q - 1.
template <int D, int N>
struct MassiveDirs {
  static constexpr int NG = D == 3 ? kMassiveGroups3D : (N == 2 ? kMassiveGroups2 : kMassiveGroups3);
  int n = 0;                  // non-rest vectors
  int v[144][3] = {};
  int first[kMaxMassiveGroups] = {}, count[kMaxMassiveGroups] = {};
  int rmax = 0;               // largest |component|
  static constexpr int gen(int g, int a) {
    return D == 3 ? kMassiveGen3D[g][a] : (N == 2 ? kMassiveGen2[g][a] : kMassiveGen3[g][a]);
  }
  constexpr MassiveDirs() {
    constexpr int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    const int nperm = D == 3 ? 6 : 2;
    for (int g = 0; g < NG; ++g) {
      int pos[48][3] = {}, np = 0;
      for (int pi = 0; pi < nperm; ++pi)
        for (int sm = 0; sm < (1 << D); ++sm) {
          int c[3] = {0, 0, 0};
          for (int a = 0; a < D; ++a) {
            const int src = D == 3 ? perm[pi][a] : (pi == 0 ? a : 1 - a);
            c[a] = ((sm >> a) & 1) ? -gen(g, src) : gen(g, src);
          }
          int lead = 0;   // sign of the first non-zero component
          for (int a = D - 1; a >= 0; --a)
            if (c[a] != 0) lead = c[a];
          if (lead <= 0) continue;
          bool dup = false;
          for (int k = 0; k < np; ++k)
            if (pos[k][0] == c[0] && pos[k][1] == c[1] && pos[k][2] == c[2]) dup = true;
          if (dup) continue;
          pos[np][0] = c[0], pos[np][1] = c[1], pos[np][2] = c[2];
          ++np;
        }
      // decreasing lexicographic order
      for (int i = 0; i < np; ++i)
        for (int j = i + 1; j < np; ++j) {
          bool gt = false;
          for (int a = 0; a < 3; ++a)
            if (pos[j][a] != pos[i][a]) {
              gt = pos[j][a] > pos[i][a];
              break;
            }
          if (gt)
            for (int a = 0; a < 3; ++a) {
              const int t = pos[i][a];
              pos[i][a] = pos[j][a];
              pos[j][a] = t;
            }
        }
      first[g] = n;
      count[g] = 2 * np;
      for (int k = 0; k < np; ++k) {
        for (int a = 0; a < 3; ++a) {
          v[n][a] = pos[k][a];
          v[n + 1][a] = -pos[k][a];
          rmax = pos[k][a] > rmax ? pos[k][a] : (-pos[k][a] > rmax ? -pos[k][a] : rmax);
        }
        n += 2;
      }
    }
  }
};
constexpr MassiveDirs<2, 2> kMassiveDirs22{};
constexpr MassiveDirs<2, 3> kMassiveDirs23{};
constexpr MassiveDirs<3, 3> kMassiveDirs33{};
static_assert(kMassiveDirs22.n == 28 && kMassiveDirs23.n == 44 && kMassiveDirs33.n == 142, "massive stencil sizes");

template <int D, int N>
RLBM_HD constexpr const MassiveDirs<D, N> &massive_dirs() {
  if constexpr (D == 3) return kMassiveDirs33;
  else if constexpr (N == 2) return kMassiveDirs22;
  else return kMassiveDirs23;
}

// Printed massless (3+1)-d order-3 rule (App. H.1): the full-symmetric groups of (4,4,3), (5,4,0)
// and (6,2,1) (24, 24 and 48 vectors, all of length sqrt(41), so v0 = 1/sqrt(41)) on four energy
// shells.  The printed weights, read shell-major with the groups in the listed order, vanish for
// (4,4,3) on shell 0 and for (5,4,0) on shells 0-2; the populations are the non-zero (shell, group)
// pairs in that order (288 in all), each group's vectors in the massive-rule order (first non-zero
// component positive, decreasing lexicographic order, each followed by its opposite).
constexpr int kUR3DGroups = 8, kUR3DQ = 288, kUR3DNorm2 = 41;
constexpr int kUR3DGen[3][3] = {{4, 4, 3}, {5, 4, 0}, {6, 2, 1}};
constexpr int kUR3DShellOf[kUR3DGroups] = {0, 1, 1, 2, 2, 3, 3, 3};   // energy shell of group g
constexpr int kUR3DGenOf[kUR3DGroups] = {2, 0, 2, 0, 2, 0, 1, 2};     // generating vector of group g
struct UR3DDirs {
  int v[kUR3DQ][3] = {};
  int first[kUR3DGroups] = {}, count[kUR3DGroups] = {};
  constexpr UR3DDirs() {
    constexpr int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int n = 0;
    for (int g = 0; g < kUR3DGroups; ++g) {
      const int *gen = kUR3DGen[kUR3DGenOf[g]];
      int pos[48][3] = {}, np = 0;
      for (int pi = 0; pi < 6; ++pi)
        for (int sm = 0; sm < 8; ++sm) {
          int c[3] = {0, 0, 0};
          for (int a = 0; a < 3; ++a) c[a] = ((sm >> a) & 1) ? -gen[perm[pi][a]] : gen[perm[pi][a]];
          int lead = 0;   // the first non-zero component
          for (int a = 2; a >= 0; --a)
            if (c[a] != 0) lead = c[a];
          if (lead <= 0) continue;
          bool dup = false;
          for (int k = 0; k < np; ++k)
            if (pos[k][0] == c[0] && pos[k][1] == c[1] && pos[k][2] == c[2]) dup = true;
          if (dup) continue;
          for (int a = 0; a < 3; ++a) pos[np][a] = c[a];
          ++np;
        }
      for (int i = 0; i < np; ++i)   // decreasing lexicographic order
        for (int j = i + 1; j < np; ++j) {
          bool gt = false;
          for (int a = 0; a < 3; ++a)
            if (pos[j][a] != pos[i][a]) {
              gt = pos[j][a] > pos[i][a];
              break;
            }
          if (gt)
            for (int a = 0; a < 3; ++a) {
              const int t = pos[i][a];
              pos[i][a] = pos[j][a];
              pos[j][a] = t;
            }
        }
      first[g] = n;
      count[g] = 2 * np;
      for (int k = 0; k < np; ++k) {
        for (int a = 0; a < 3; ++a) {
          v[n][a] = pos[k][a];
          v[n + 1][a] = -pos[k][a];
        }
        n += 2;
      }
    }
  }
};
constexpr UR3DDirs kUR3DDirs{};
static_assert(kUR3DDirs.first[kUR3DGroups - 1] + kUR3DDirs.count[kUR3DGroups - 1] == kUR3DQ, "UR3D size");

template <int SID, int KR>
struct Stencil;

template <int KR>
struct Stencil<ST_PROD2D, KR> {
  static constexpr int D = 2, NDIR = 8, Q = KR * 8, NSHELL = KR;
  static constexpr bool ONLAT = false, SHIFT = false;
  RLBM_HD static constexpr int dir(int i, int a) { return kDir2D[i % 8][a]; }
};

template <int KR>
struct Stencil<ST_PROD3D, KR> {
  static constexpr int D = 3, NDIR = 26, Q = KR * 26, NSHELL = KR;
  static constexpr bool ONLAT = false, SHIFT = false;
  RLBM_HD static constexpr int dir(int i, int a) { return kDir3D[i % 26][a]; }
};

// Groups of equal energy and weight of the printed massless rules: the
// (+-3,+-4) directions (eight) and the (+-5,0) directions (four) of each shell.
constexpr int kURGroups2 = 4;
constexpr int kURFirst2[kURGroups2] = {0, 8, 16, 24};
constexpr int kURCount2[kURGroups2] = {8, 8, 8, 4};

template <>
struct Stencil<ST_UR2D, 3> {
  static constexpr int D = 2, NDIR = 12, Q = kUR2DQ, NSHELL = 3, RMAX = 5, NG = kURGroups2;
  static constexpr bool ONLAT = true, SHIFT = false;
  // integer displacement of population i (sites per step)
  RLBM_HD static constexpr int dir(int i, int a) { return kDirUR[kURDir[i]][a]; }
  RLBM_HD static constexpr int gfirst(int g) { return kURFirst2[g]; }
  RLBM_HD static constexpr int gcount(int g) { return kURCount2[g]; }
};

// Printed massless (2+1)-d order-3 rule (App. H.2): the same 12 directions on
// four shells; shell 0 carries no (+-5,0) population (zero weight), so the
// populations are shell 0's eight (+-3,+-4) directions, then all twelve
// directions of shells 1, 2, 3.
constexpr int kUR3Q = 44;
RLBM_HD constexpr int ur3_shell(int i) { return i < 8 ? 0 : 1 + (i - 8) / 12; }
RLBM_HD constexpr int ur3_dir(int i) { return i < 8 ? i : (i - 8) % 12; }

constexpr int kURGroups3 = 7;
constexpr int kURFirst3[kURGroups3] = {0, 8, 16, 20, 28, 32, 40};
constexpr int kURCount3[kURGroups3] = {8, 8, 4, 8, 4, 8, 4};

template <>
struct Stencil<ST_UR2D, 4> {
  static constexpr int D = 2, NDIR = 12, Q = kUR3Q, NSHELL = 4, RMAX = 5, NG = kURGroups3;
  static constexpr bool ONLAT = true, SHIFT = false;
  RLBM_HD static constexpr int dir(int i, int a) { return kDirUR[ur3_dir(i)][a]; }
  RLBM_HD static constexpr int gfirst(int g) { return kURFirst3[g]; }
  RLBM_HD static constexpr int gcount(int g) { return kURCount3[g]; }
};

template <>
struct Stencil<ST_UR3D, 4> {
  static constexpr int D = 3, NDIR = kUR3DQ, Q = kUR3DQ, NSHELL = 4, RMAX = 6, NG = kUR3DGroups;
  static constexpr bool ONLAT = true, SHIFT = false;
  RLBM_HD static constexpr int dir(int i, int a) { return kUR3DDirs.v[i][a]; }
  RLBM_HD static constexpr int gfirst(int g) { return kUR3DDirs.first[g]; }
  RLBM_HD static constexpr int gcount(int g) { return kUR3DDirs.count[g]; }
};

// Massive on-lattice rules (d = 2: Q = 29 for N = 2, 45 for N = 3; d = 3: Q =
// 143 for N = 3), the rest population last.  NG groups of equal weight and
// energy, group g holding populations [gfirst(g), gfirst(g) + gcount(g)).
template <int D_, int N>
struct MassiveStencil {
  static constexpr int D = D_, Q = massive_dirs<D_, N>().n + 1, NDIR = Q, NSHELL = 0;
  static constexpr int NG = MassiveDirs<D_, N>::NG, RMAX = massive_dirs<D_, N>().rmax;
  static constexpr bool ONLAT = true, SHIFT = true;
  RLBM_HD static constexpr int dir(int i, int a) { return i >= Q - 1 ? 0 : massive_dirs<D_, N>().v[i][a]; }
  RLBM_HD static constexpr int gfirst(int g) { return massive_dirs<D_, N>().first[g]; }
  RLBM_HD static constexpr int gcount(int g) { return massive_dirs<D_, N>().count[g]; }
};
template <int N>
struct Stencil<ST_MASSIVE2D, N> : MassiveStencil<2, N> {};
template <int N>
struct Stencil<ST_MASSIVE3D, N> : MassiveStencil<3, N> {};

// Number of interpolation taps of population i: 2^(number of non-zero direction components).
template <class ST>
RLBM_HD constexpr int n_taps(int i) {
  if (ST::ONLAT) return 1;
  int nz = 0;
  for (int a = 0; a < ST::D; ++a) nz += ST::dir(i, a) != 0;
  return 1 << nz;
}

// ---------------------------------------------------------------------------
// Polynomial basis on the mass shell: monomials p0^a p1^e1 p2^e2 p3^e3 with
// a in {0, 1} and total degree <= N (p0^2 = m^2 + |p|^2 removes the rest).
// Each entry is the tensor index tuple of the monomial (0 = time), unused
// slots -1.  Even spatial parity first (NE entries), then odd (NO entries):
// an antipodal pair p -> (p0, -p) keeps even monomials and flips odd ones.
// ---------------------------------------------------------------------------
template <int D, int N>
struct BasisDef;

template <>
struct BasisDef<2, 2> {
  static constexpr int NE = 5, NO = 4, NM = 9;
  static constexpr signed char idx[NM][3] = {
      {-1, -1, -1}, {0, -1, -1}, {1, 1, -1}, {1, 2, -1}, {2, 2, -1},   // even
      {1, -1, -1},  {2, -1, -1}, {0, 1, -1}, {0, 2, -1}};              // odd
};
template <>
struct BasisDef<2, 3> {
  static constexpr int NE = 8, NO = 8, NM = 16;
  static constexpr signed char idx[NM][3] = {
      {-1, -1, -1}, {0, -1, -1}, {1, 1, -1}, {1, 2, -1}, {2, 2, -1}, {0, 1, 1}, {0, 1, 2}, {0, 2, 2},
      {1, -1, -1},  {2, -1, -1}, {0, 1, -1}, {0, 2, -1}, {1, 1, 1},  {1, 1, 2}, {1, 2, 2}, {2, 2, 2}};
};
template <>
struct BasisDef<3, 2> {
  static constexpr int NE = 8, NO = 6, NM = 14;
  static constexpr signed char idx[NM][3] = {
      {-1, -1, -1}, {0, -1, -1}, {1, 1, -1}, {1, 2, -1}, {1, 3, -1}, {2, 2, -1}, {2, 3, -1}, {3, 3, -1},
      {1, -1, -1},  {2, -1, -1}, {3, -1, -1}, {0, 1, -1}, {0, 2, -1}, {0, 3, -1}};
};
template <>
struct BasisDef<3, 3> {
  static constexpr int NE = 14, NO = 16, NM = 30;
  static constexpr signed char idx[NM][3] = {
      // even: 1, p0, p_a p_b (6), p0 p_a p_b (6)
      {-1, -1, -1}, {0, -1, -1}, {1, 1, -1}, {1, 2, -1}, {1, 3, -1}, {2, 2, -1}, {2, 3, -1}, {3, 3, -1},
      {0, 1, 1}, {0, 1, 2}, {0, 1, 3}, {0, 2, 2}, {0, 2, 3}, {0, 3, 3},
      // odd: p_a (3), p0 p_a (3), p_a p_b p_c (10)
      {1, -1, -1}, {2, -1, -1}, {3, -1, -1}, {0, 1, -1}, {0, 2, -1}, {0, 3, -1},
      {1, 1, 1}, {1, 1, 2}, {1, 1, 3}, {1, 2, 2}, {1, 2, 3}, {1, 3, 3}, {2, 2, 2}, {2, 2, 3}, {2, 3, 3},
      {3, 3, 3}};
};

RLBM_HD constexpr int basis_size(int D, int N) {
  return D == 2 ? (N + 1) * (N + 1) : (N + 1) * (N + 2) * (2 * N + 3) / 6;
}

// ---------------------------------------------------------------------------
// Per-lattice constant tables (device memory).  Sized for the largest
// stencil; kernels index only what their stencil uses.
// ---------------------------------------------------------------------------
constexpr int kMaxQ = 288;
constexpr int kMaxPairs = kMaxQ / 2;
constexpr int kMaxNE = 14, kMaxNO = 16, kMaxNM = 30;
constexpr int kMaxShell = 4;
constexpr int kNMom3 = 14;   // 4 (N^a) + 10 (T^ab) in 3D; 2D uses 3 + 6

constexpr int kEosTerms = 44;
// the 3D equation-of-state fits cover T in [1/128, 128] in kEosPieces pieces of equal width in
// log T (an odd count: T = 1 lies mid-piece, so lattices near the reference temperature evaluate
// one piece per wave)
constexpr int kEosPieces = 5;
constexpr double kEosTmin = 1.0 / 128.0, kEosTmax = 128.0;
constexpr int kMaxPacked = 96;   // packed class blocks of Linv (91 entries for d = 3, N = 3)

struct Tables {
  // geometry and physics
  int32_t nx, ny, nz, pad0;
  int32_t open[3], storage;     // open[a]: reads clamp at the edges of axis a (open or wall)
  int32_t wall[3], has_force;   // wall[a]: no-slip equilibrium walls on the end planes of axis a
  double g[3];                  // external acceleration (Sec. 5.4, scheme B)
  float gf[3], pad2;
  int64_t sites;                // nx * ny * nz
  double m;                     // reduced mass zeta = m/T0
  double tau;                   // relaxation time (when no field)
  double inv_tau;
  double n_ref;
  // EOS helper for d = 3: Chebyshev series in log z of h(z) = r(z) (z + 2) / z, r = K1(z)/K2(z),
  // on [cheb_lo, cheb_hi] = [log z_lo, log z_hi], one series per piece of equal width
  double cheb_lo, cheb_hi;
  double cheb[kEosPieces][48];
  int32_t cheb_n, chebT_n;
  // and the inverse of the equation of state: T = (e - m) u(x), x = log(e - m), u a Chebyshev
  // series in x on [chebT_lo, chebT_hi] (e = eps/n; the same temperature range), also by pieces
  double chebT_lo, chebT_hi;
  double chebT[kEosPieces][48];
  // per pair of antipodal populations (even member 2pr):
  double c[kMaxPairs][3];       // velocity p^a / p^0
  double mom_e[kMaxPairs][8];   // even moment weights: p0, p0^2, p^a p^b (upper triangle)
  double mom_o[kMaxPairs][6];   // odd moment weights: p^a, p0 p^a
  double Re[kMaxPairs][kMaxNE]; // projection rows, even basis part
  double Ro[kMaxPairs][kMaxNO]; // projection rows, odd basis part
  double Rrest[kMaxNE];         // projection row of a rest population (p = (m, 0)), even part
  float Rrestf[kMaxNE];
  // on-lattice rules, per group g (p = (p0, v n), v = v0 p0, weight w, D = p0 - m):
  // p0, p0^2, v, p0 v, v^2, w v^l (l = 0..3), w D v^l (l = 0..3)
  double mgrp[kMaxMassiveGroups][13];
  float mgrpf[kMaxMassiveGroups][13];
  double wrest, v0;             // rest weight, lattice-speed parameter (1/5 for the printed massless rules)
  float wrestf, v0f;
  double tau_T;                 // on-lattice rules: tau(x) += tau_T / T(x) (0 = off)
  double wallT[3][2];           // prescribed temperature of the first / last plane of a wall axis (0 = own)
  float Ref[kMaxPairs][kMaxNE]; // float copies for the F32_DEV path
  float Rof[kMaxPairs][kMaxNO];
  float cf[kMaxPairs][3];
  float mom_ef[kMaxPairs][8];
  float mom_of[kMaxPairs][6];
  // per population
  double tapw[kMaxQ][8];        // interpolation weights in the stencil's tap order
  float tapwf[kMaxQ][8];
  double fref[kMaxQ];           // reference populations f^ref (F32_DEV)
  float freff[kMaxQ];
  // reference moments (F32_DEV): N^a, T^ab upper triangle, basis moments
  double Nref[4];
  double Tref[10];
  double Mref[kMaxNM];
  // product rules, per shell j: speed |p|/p^0, moment factors and
  // equilibrium factors W_j (p^0 - m)^a |p|^l (W_j the shell weight; in 2D
  // the direction weight 1/8 is folded in)
  double sv[kMaxShell];
  double smom[kMaxShell][5];       // p0, |p|, p0^2, p0 |p|, |p|^2
  double sfeq[kMaxShell][2][4];
  double Linv[kMaxNM][kMaxNM];     // product rules: inverse Cholesky factor of the Gram matrix of (p^0 - m)^a p^e
  double LinvP[kMaxPacked];        // its parity-class blocks, packed lower triangles (ClassTable order)
  float svf[kMaxShell];
  float smomf[kMaxShell][5];
  float sfeqf[kMaxShell][2][4];
};

// Angular structure of the basis for product rules: each basis monomial
// p0^a p^e is grouped by its angular multi-index e; m0[q] / m1[q] are the
// basis indices with a = 0 / a = 1 (-1 if absent) of angular monomial q.
template <int D, int N>
struct AngTable {
  int n = 0;
  int e[20][3] = {};
  int m0[20] = {};
  int m1[20] = {};
  int cls[kMaxNM] = {};   // parity class (e_x mod 2, e_y mod 2, e_z mod 2) of each basis monomial
  constexpr AngTable() {
    using B = BasisDef<D, N>;
    for (int m = 0; m < B::NM; ++m) {
      int a = 0, ee[3] = {0, 0, 0};
      for (int s = 0; s < 3; ++s) {
        int ix = B::idx[m][s];
        if (ix == 0) ++a;
        else if (ix > 0) ++ee[ix - 1];
      }
      cls[m] = (ee[0] & 1) | ((ee[1] & 1) << 1) | ((ee[2] & 1) << 2);
      int f = -1;
      for (int q = 0; q < n; ++q)
        if (e[q][0] == ee[0] && e[q][1] == ee[1] && e[q][2] == ee[2]) f = q;
      if (f < 0) {
        f = n++;
        e[f][0] = ee[0];
        e[f][1] = ee[1];
        e[f][2] = ee[2];
        m0[f] = -1;
        m1[f] = -1;
      }
      if (a == 0) m0[f] = m;
      else m1[f] = m;
    }
  }
};

// Basis indices grouped by parity class (ascending within a class), the position
// of each index inside its class, and for p0 p^e the index of p^e (else -1).
template <int D, int N>
struct ClassTable {
  int cnt[8] = {};
  int idx[8][kMaxNM] = {};
  int pos[kMaxNM] = {};
  int partner[kMaxNM] = {};
  int off[8] = {};   // start of class c's packed lower triangle
  int packed = 0;
  constexpr ClassTable() {
    constexpr AngTable<D, N> AT{};
    for (int m = 0; m < BasisDef<D, N>::NM; ++m) {
      const int c = AT.cls[m];
      pos[m] = cnt[c];
      idx[c][cnt[c]++] = m;
      partner[m] = -1;
    }
    for (int q = 0; q < AT.n; ++q)
      if (AT.m1[q] >= 0) partner[AT.m1[q]] = AT.m0[q];
    for (int c = 0; c < 8; ++c) {
      off[c] = packed;
      packed += cnt[c] * (cnt[c] + 1) / 2;
    }
  }
};

}  // namespace rlbm
