// kernels.hip -- HIP kernels of the RLBM update for gfx950 (MI355X).
//
// Design (memory-bound: 2 Q words of HBM traffic per site update):
//  * populations in SoA planes f[i][z][y][x]; one thread per site, 64-wide
//    wavefronts along x so every population plane is read and written with
//    fully coalesced 512 B (f64) / 256 B (f32) wavefront accesses;
//  * fused pull-stream + collide: the pre-collision value of population i at
//    x is read from the post-collision planes at the upstream taps (a pure
//    shift on-lattice; bilinear / trilinear interpolation off-lattice, taps
//    and their count fixed at compile time from the direction signs, weights
//    from the per-lattice table); neighbouring taps of a wavefront hit the
//    same cache lines, so the extra taps are served from L1/L2, not HBM;
//  * all constant tables are read through uniform (scalar) loads;
//  * antipodal populations are processed in pairs: sums and differences feed
//    the even / odd halves of the moments and of the projected equilibrium,
//    halving both the moment and the equilibrium arithmetic;
//  * the Landau eigenproblem, equation of state and equilibrium moments are
//    evaluated in double for every storage mode.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <type_traits>
#include <utility>

#include "device_math.h"
#include "kernels.h"
#include "massive_math.h"
#include "prod_math.h"

namespace rlbm {

__device__ __forceinline__ int wrap_or_clamp(int v, int n, int open) {
  if (open) return v < 0 ? 0 : (v >= n ? n - 1 : v);
  v = v < 0 ? v + n : v;
  return v >= n ? v - n : v;
}

// Moments of the shifted monomials (p^0 - m) p^e = p^0 p^e - m p^e, in place
// (stencils whose projection rows act on the shifted basis).
template <int D, int N>
__device__ __forceinline__ void shift_basis_moments(double m, double (&M)[BasisDef<D, N>::NM]) {
  constexpr ClassTable<D, N> CL{};
#pragma unroll
  for (int k = 0; k < BasisDef<D, N>::NM; ++k)
    if (CL.partner[k] >= 0) M[k] -= m * M[CL.partner[k]];
}

template <int D>
__device__ __forceinline__ void write_fields(const FieldPtrs &fp, int64_t site, int64_t sites, const Macro<D> &mac) {
  if (fp.n) fp.n[site] = mac.n;
  if (fp.eps) fp.eps[site] = mac.eps;
  if (fp.T) fp.T[site] = mac.T;
  if (fp.U) {
#pragma unroll
    for (int a = 0; a <= D; ++a) fp.U[a * sites + site] = mac.U[a];
  }
}

__device__ __forceinline__ void flag_error(int *err) {
  // all writers store the same value: a benign race, and a plain store (a volatile one would make
  // the wave wait for every load it has in flight)
  *err = 1;
}

template <typename S>
__device__ __forceinline__ double site_tau(const Tables *__restrict__ tb, const void *tau_field, int64_t site) {
  // the lattice's tau through a scalar load, chosen by value (a per-site load through a pointer
  // picked between the field and the table would be a vector load the wave waits for)
  const double tau = tb->tau;
  if (tau_field == nullptr) return tau;
  return (double)((const S *)tau_field)[site];
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
template <class ST, typename S>
__device__ __forceinline__ Offs make_offs(const Tables *__restrict__ tb, int x, int y, int z) {
  Offs o;
  const uint32_t nx = tb->nx, nxy = (uint32_t)tb->nx * tb->ny;
#pragma unroll
  for (int d = -1; d <= 1; ++d) {
    o.x[d + 1] = (uint32_t)wrap_or_clamp(x + d, tb->nx, tb->open[0]) * (uint32_t)sizeof(S);
    o.y[d + 1] = (uint32_t)wrap_or_clamp(y + d, tb->ny, tb->open[1]) * nx * (uint32_t)sizeof(S);
    o.z[d + 1] = ST::D == 3 ? (uint32_t)wrap_or_clamp(z + d, tb->nz, tb->open[2]) * nxy * (uint32_t)sizeof(S) : 0u;
  }
  return o;
}

// Integer streaming: population I at the site comes from x - n_I.  The byte
// offsets of the upstream rows are computed once per axis and distance (up to
// ST::RMAX sites), so each population costs one add and one load.
template <class ST>
RLBM_HD constexpr int dir_z(int i) {
  if constexpr (ST::D == 3) return ST::dir(i, 2);
  else return 0;
}

template <class ST, typename S, int R, int... I>
__device__ __forceinline__ void gather_onlat_impl(const S *__restrict__ fin, int64_t sites, const uint32_t (&ox)[2 * R + 1],
                                                  const uint32_t (&oy)[2 * R + 1], const uint32_t (&oz)[2 * R + 1],
                                                  S (&f)[ST::Q], std::integer_sequence<int, I...>) {
  ((f[I] = *(const S *)((const char *)(fin + (int64_t)I * sites) + ox[R - ST::dir(I, 0)] + oy[R - ST::dir(I, 1)] +
                        oz[R - dir_z<ST>(I)])),
   ...);
}

// byte offsets of the rows x + k - R, y + k - R, z + k - R (k = 0 .. 2R)
template <class ST, typename S>
__device__ __forceinline__ void onlat_offsets(const Tables *__restrict__ tb, int x, int y, int z,
                                              uint32_t (&ox)[2 * ST::RMAX + 1], uint32_t (&oy)[2 * ST::RMAX + 1],
                                              uint32_t (&oz)[2 * ST::RMAX + 1]) {
  constexpr int R = ST::RMAX;
  const uint32_t nx = tb->nx, nxy = (uint32_t)tb->nx * tb->ny;
#pragma unroll
  for (int k = 0; k <= 2 * R; ++k) {
    ox[k] = (uint32_t)wrap_or_clamp(x + k - R, tb->nx, tb->open[0]) * (uint32_t)sizeof(S);
    oy[k] = (uint32_t)wrap_or_clamp(y + k - R, tb->ny, tb->open[1]) * nx * (uint32_t)sizeof(S);
    oz[k] = ST::D == 3 ? (uint32_t)wrap_or_clamp(z + k - R, tb->nz, tb->open[2]) * nxy * (uint32_t)sizeof(S) : 0u;
  }
}

template <class ST, typename S>
__device__ __forceinline__ void gather_onlat(const Tables *__restrict__ tb, const S *__restrict__ fin, int64_t sites,
                                             int x, int y, int z, S (&f)[ST::Q]) {
  constexpr int R = ST::RMAX;
  uint32_t ox[2 * R + 1], oy[2 * R + 1], oz[2 * R + 1];
  onlat_offsets<ST, S>(tb, x, y, z, ox, oy, oz);
  gather_onlat_impl<ST, S, R>(fin, sites, ox, oy, oz, f, std::make_integer_sequence<int, ST::Q>{});
}

// pre-collision populations at the site, in the arithmetic type A (the storage type S, or double
// for float deviations updated in double: product rules)
template <class ST, typename S, typename A = S>
__device__ __forceinline__ void gather(const Tables *__restrict__ tb, const S *__restrict__ fin, int64_t sites, int x,
                                       int y, int z, A (&f)[ST::Q]) {
  if constexpr (ST::ONLAT) {
    static_assert(sizeof(A) == sizeof(S), "on-lattice rules compute in their storage type");
    gather_onlat<ST, S>(tb, fin, sites, x, y, z, f);
  } else {
    const Offs o = make_offs<ST, S>(tb, x, y, z);
    pull_prod<ST, S, false, A>(tb, fin, sites, o, f);
  }
}

// Collision of one site: f (pre-collision, storage precision; deviations in
// the F32_DEV mode) is replaced by f* in place; returns the macro state of the
// pre-collision populations.  wallT: see site_wall (negative off the walls).
template <class ST, int N, typename S, bool DEV, bool RELAX, bool EXT = false>
__device__ __forceinline__ Macro<ST::D> collide_site(const Tables *__restrict__ tb, S (&f)[ST::Q], double tau,
                                                     double wallT = -1.0) {
  if constexpr (ST::ONLAT)
    return collide_massive<ST, N, S, DEV, RELAX, EXT>(tb, f, tau, wallT);
  else
    return collide_prod<ST, N, S, DEV, RELAX, EXT>(tb, f, tau, wallT);
}

// post-collision populations of the site, rounded to the storage type
template <class ST, typename S, bool NT = false, typename A = S>
__device__ __forceinline__ void store_site(S *__restrict__ fout, int64_t sites, uint32_t site_off,
                                           const A (&f)[ST::Q]) {
#pragma unroll
  for (int i = 0; i < ST::Q; ++i) put_pop<NT>(fout, sites, site_off, i, (S)f[i]);
}

// Site of this thread.  Blocks form a 1D grid over tiles of tl.bx x tl.by x
// tl.bz sites.  The hardware deals consecutive blocks
// round-robin to the 8 XCDs, each with its own L2.  Tile orders:
//   xcd == 0: x fastest, then y, then z, as dealt;
//   xcd == 1: each XCD receives a contiguous range of that order (a band of
//             neighbouring rows whose halo rows stay in its L2);
//   xcd == 2: (3D) the rows are grouped in patches of kPatch x kPatch rows in
//             (y, z); XCD k takes patches k, k + 8, ... and walks each patch
//             with x fastest, so the blocks in flight on an XCD cover one
//             compact patch and read each other's y and z halo rows while
//             they are still in its L2.  The grid then has 8 * ceil(patches /
//             8) * tiles-per-patch blocks; those past the lattice return.
constexpr int kPatch = 8;

// The launch shape as kernel arguments (scalar registers): blockDim and gridDim would be read from
// the dispatch packet by vector loads that every wave waits for before its first tap load.
struct Tiling {
  int bx, by, bz;   // block shape
  int nb;           // blocks in the grid
  int order;        // tile order (0, 1, 2 as above)
};

__device__ __forceinline__ bool site_coords(const Tables *__restrict__ tb, const Tiling &tl, int &x, int &y, int &z) {
  const uint32_t bx = tl.bx, by = tl.by, bz = tl.bz;
  const uint32_t gx = (tb->nx + bx - 1) / bx;
  const uint32_t gy = (tb->ny + by - 1) / by;
  const uint32_t nb = tl.nb;
  const int xcd = tl.order;
  uint32_t t = blockIdx.x;
  uint32_t tx, ty, tz;
  if (xcd == 2) {
    const uint32_t py = max(1u, kPatch / by), pz = max(1u, kPatch / bz);   // tile rows per patch
    const uint32_t npy = (gy + py - 1) / py;
    const uint32_t per = gx * py * pz;                                     // tiles per patch
    const uint32_t k = t % 8, l = t / 8;
    const uint32_t p = (l / per) * 8 + k, w = l % per;
    tx = w % gx;
    ty = (p % npy) * py + (w / gx) % py;
    tz = (p / npy) * pz + w / (gx * py);
  } else {
    if (xcd) {
      const uint32_t q = nb / 8, r = nb % 8, k = t % 8, l = t / 8;
      t = k * q + (k < r ? k : r) + l;
    }
    tx = t % gx;
    ty = (t / gx) % gy;
    tz = t / (gx * gy);
  }
  x = tx * bx + threadIdx.x;
  y = ty * by + threadIdx.y;
  z = tz * bz + threadIdx.z;
  return x < tb->nx && y < tb->ny && z < tb->nz;
}

template <class ST, int N, typename S, bool DEV, int OCC, bool EXT, bool NT, typename A = S>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC > 0 ? OCC : 1, 8))) k_step(const Tables *__restrict__ tb, const S *__restrict__ fin,
                                              S *__restrict__ fout, const void *__restrict__ tau_field,
                                              FieldPtrs last, int *err, Tiling tl) {
  int x, y, z;
  if (!site_coords(tb, tl, x, y, z)) return;
  const int64_t sites = tb->sites;
  const int64_t site = ((int64_t)z * tb->ny + y) * tb->nx + x;
  A f[ST::Q];
  gather<ST, S, A>(tb, fin, sites, x, y, z, f);
  const double tau = site_tau<S>(tb, tau_field, site);
  const Macro<ST::D> mac = collide_site<ST, N, A, DEV, true, EXT>(tb, f, tau, EXT ? site_wall(tb, x, y, z) : -1.0);
  if (!mac.ok) flag_error(err);
  // a fresh copy of the plane size for the store addresses: otherwise the compiler keeps the
  // load phase's plane offsets alive (in spilled scalar registers) for reuse here
  int64_t sites_st = sites;
  if constexpr (ST::D == 3) asm volatile("" : "+s"(sites_st));
  store_site<ST, S, NT, A>(fout, sites_st, (uint32_t)site * (uint32_t)sizeof(S), f);
  if (last.any) write_fields<ST::D>(last, site, sites, mac);
}

// Massive rules whose populations do not fit in registers (the 143-vector 3D
// stencil in double storage): every population is loaded once for the
// moments; the first kStreamKeep of them stay in registers, the others are
// loaded again (from the caches or memory) for the relaxation; every result is
// stored at once.  Keeping about a third of them balances the re-read traffic
// against the registers the eigen-solve and the projection need.
template <class ST, int N, typename S, bool DEV, int OCC, bool NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC > 0 ? OCC : 1, 8)))
k_step_stream(const Tables *__restrict__ tb, const S *__restrict__ fin, S *__restrict__ fout,
              const void *__restrict__ tau_field, FieldPtrs last, int *err, Tiling tl) {
  int x, y, z;
  if (!site_coords(tb, tl, x, y, z)) return;
  const int64_t sites = tb->sites;
  const int64_t site = ((int64_t)z * tb->ny + y) * tb->nx + x;
  constexpr int R = ST::RMAX;
  uint32_t ox[2 * R + 1], oy[2 * R + 1], oz[2 * R + 1];
  onlat_offsets<ST, S>(tb, x, y, z, ox, oy, oz);
  // a second, opaque copy of the input pointer: the relaxation's loads are not merged with the
  // moment loads (which would keep every population live)
  const S *fin2 = fin;
  asm volatile("" : "+s"(fin2));
  const uint32_t site_off = (uint32_t)site * (uint32_t)sizeof(S);
  auto load = [&](const S *base, int i) {
    return *(const S *)((const char *)(base + (int64_t)i * sites) + ox[R - ST::dir(i, 0)] + oy[R - ST::dir(i, 1)] +
                        oz[R - dir_z<ST>(i)]);
  };
  const double tau = site_tau<S>(tb, tau_field, site);
  constexpr int kStreamKeep = 48;
  S keep[kStreamKeep];
  const Macro<ST::D> mac = massive_update<ST, N, S, DEV, true, false, false>(
      tb, tau, -1.0,
      [&](int i) {
        const S v = load(fin, i);
        if (i < kStreamKeep) keep[i < kStreamKeep ? i : 0] = v;
        return v;
      },
      [&](int i) { return i < kStreamKeep ? keep[i < kStreamKeep ? i : 0] : load(fin2, i); },
      [&](int i, S v) { put_pop<NT>(fout, sites, site_off, i, v); });
  if (!mac.ok) flag_error(err);
  if (last.any) write_fields<ST::D>(last, site, sites, mac);
}

// The moments and the initial state for stencils too large to hold in registers (the 288-vector
// (3+1)-d massless rule): the same arithmetic as k_moments and k_init, with every population loaded
// (or, at the initial state, evaluated from its projection row) when the update asks for it.
template <class ST, int N, typename S, bool DEV>
__global__ void __launch_bounds__(256) k_moments_stream(const Tables *__restrict__ tb, const S *__restrict__ fin,
                                                        FieldPtrs out, int *err, Tiling tl) {
  int x, y, z;
  if (!site_coords(tb, tl, x, y, z)) return;
  const int64_t sites = tb->sites;
  const int64_t site = ((int64_t)z * tb->ny + y) * tb->nx + x;
  constexpr int R = ST::RMAX;
  uint32_t ox[2 * R + 1], oy[2 * R + 1], oz[2 * R + 1];
  onlat_offsets<ST, S>(tb, x, y, z, ox, oy, oz);
  auto load = [&](int i) {
    return *(const S *)((const char *)(fin + (int64_t)i * sites) + ox[R - ST::dir(i, 0)] + oy[R - ST::dir(i, 1)] +
                        oz[R - dir_z<ST>(i)]);
  };
  const Macro<ST::D> mac = massive_update<ST, N, S, DEV, false, false, false>(
      tb, 1.0, -1.0, load, load, [&](int, S) {});
  if (!mac.ok) flag_error(err);
  write_fields<ST::D>(out, site, sites, mac);
}

template <class ST, int N, typename S, bool DEV>
__global__ void __launch_bounds__(256) k_init_stream(const Tables *__restrict__ tb, const double *__restrict__ n0,
                                                     const double *__restrict__ T0, const double *__restrict__ u0,
                                                     const double *__restrict__ noise, double amp,
                                                     S *__restrict__ fout, const void *__restrict__ tau_field,
                                                     FieldPtrs fields0, int *err, Tiling tl) {
  constexpr int D = ST::D, Q = ST::Q;
  static_assert(D == 3, "streaming init: the (3+1)-d rule");
  using B = BasisDef<D, N>;
  int x, y, z;
  if (!site_coords(tb, tl, x, y, z)) return;
  const int64_t sites = tb->sites;
  const int64_t site = ((int64_t)z * tb->ny + y) * tb->nx + x;
  double U[D + 1], uu = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    U[a + 1] = u0[a * sites + site];
    uu += U[a + 1] * U[a + 1];
  }
  const double g = 1.0 / sqrt(1.0 - uu);
  U[0] = g;
#pragma unroll
  for (int a = 1; a <= D; ++a) U[a] *= g;
  const double n = n0[site], T = T0[site];
  bool inr = true;
  const double r = tb->m == 0.0 ? 0.0 : cheb_r(tb, tb->m / T, inr);
  if (!inr || !(uu < 1.0) || !(n > 0.0) || !(T > 0.0)) flag_error(err);
  const Ratios rr = ratios_3d(tb->m / T, r);
  double M[B::NM];
  basis_moments<D, N>(n, T, U, rr, M);
  if constexpr (ST::SHIFT) shift_basis_moments<D, N>(tb->m, M);
  // f_i(x, 0) = f^eq_i (1 + amp xi_i) from the projection rows, in storage form
  auto feq = [&](int i) {
    const int pr = i >> 1;
    double E = 0.0, O = 0.0;
#pragma unroll
    for (int k = 0; k < B::NE; ++k) E += tb->Re[pr][k] * M[k];
#pragma unroll
    for (int k = 0; k < B::NO; ++k) O += tb->Ro[pr][k] * M[B::NE + k];
    double v = (i & 1) ? E - O : E + O;
    if (noise != nullptr) v *= 1.0 + amp * noise[(int64_t)i * sites + site];
    return DEV ? (S)(v - tb->fref[i]) : (S)v;
  };
  static_assert((Q & 1) == 0, "streaming init: stencils without a rest population");
  const double tau = site_tau<S>(tb, tau_field, site);
  const uint32_t site_off = (uint32_t)site * (uint32_t)sizeof(S);
  const Macro<D> mac = massive_update<ST, N, S, DEV, true, false, false>(
      tb, tau, -1.0, feq, feq, [&](int i, S v) { put_pop<false>(fout, sites, site_off, i, v); });
  if (!mac.ok) flag_error(err);
  if (fields0.any) write_fields<D>(fields0, site, sites, mac);
}

template <class ST, int N, typename S, bool DEV, typename A = S>
__global__ void __launch_bounds__(256) k_moments(const Tables *__restrict__ tb, const S *__restrict__ fin,
                                                 FieldPtrs out, int *err, Tiling tl) {
  int x, y, z;
  if (!site_coords(tb, tl, x, y, z)) return;
  const int64_t sites = tb->sites;
  const int64_t site = ((int64_t)z * tb->ny + y) * tb->nx + x;
  A f[ST::Q];
  gather<ST, S, A>(tb, fin, sites, x, y, z, f);
  const Macro<ST::D> mac = collide_site<ST, N, A, DEV, false>(tb, f, 1.0);
  if (!mac.ok) flag_error(err);
  write_fields<ST::D>(out, site, sites, mac);
}

// f(x, 0) = f^eq(n0, T0, U(u0)) (1 + amp xi), then collide; store f*(x, 0).
template <class ST, int N, typename S, bool DEV, typename A = S>
__global__ void __launch_bounds__(256) k_init(const Tables *__restrict__ tb, const double *__restrict__ n0,
                                              const double *__restrict__ T0, const double *__restrict__ u0,
                                              const double *__restrict__ noise, double amp, S *__restrict__ fout,
                                              const void *__restrict__ tau_field, FieldPtrs fields0, int *err,
                                              Tiling tl) {
  constexpr int D = ST::D, Q = ST::Q, NP = Q / 2;
  using B = BasisDef<D, N>;
  int x, y, z;
  if (!site_coords(tb, tl, x, y, z)) return;
  const int64_t sites = tb->sites;
  const int64_t site = ((int64_t)z * tb->ny + y) * tb->nx + x;
  double U[D + 1], uu = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    U[a + 1] = u0[a * sites + site];
    uu += U[a + 1] * U[a + 1];
  }
  const double g = 1.0 / sqrt(1.0 - uu);
  U[0] = g;
#pragma unroll
  for (int a = 1; a <= D; ++a) U[a] *= g;
  const double n = n0[site], T = T0[site];
  Ratios rr;
  if constexpr (D == 2) {
    rr = ratios_2d(tb->m / T);
  } else {
    bool inr = true;
    const double r = tb->m == 0.0 ? 0.0 : cheb_r(tb, tb->m / T, inr);
    if (!inr) flag_error(err);
    rr = ratios_3d(tb->m / T, r);
  }
  if (!(uu < 1.0) || !(n > 0.0) || !(T > 0.0)) flag_error(err);
  double M[B::NM];
  basis_moments<D, N>(n, T, U, rr, M);
  if constexpr (ST::SHIFT) shift_basis_moments<D, N>(tb->m, M);
  double fd[Q];
#pragma unroll
  for (int pr = 0; pr < NP; ++pr) {
    double E = 0.0, O = 0.0;
#pragma unroll
    for (int k = 0; k < B::NE; ++k) E += tb->Re[pr][k] * M[k];
#pragma unroll
    for (int k = 0; k < B::NO; ++k) O += tb->Ro[pr][k] * M[B::NE + k];
    fd[2 * pr] = E + O;
    fd[2 * pr + 1] = E - O;
  }
  if constexpr ((Q & 1) != 0) {
    double E = 0.0;
#pragma unroll
    for (int k = 0; k < B::NE; ++k) E += tb->Rrest[k] * M[k];
    fd[Q - 1] = E;
  }
  if (noise != nullptr) {
#pragma unroll
    for (int i = 0; i < Q; ++i) fd[i] *= 1.0 + amp * noise[(int64_t)i * sites + site];
  }
  // the update's form: f, or the deviations f - f^ref (in float, or in double when float deviations
  // are updated in double)
  A f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) f[i] = DEV ? (A)(fd[i] - tb->fref[i]) : (A)fd[i];
  const double tau = site_tau<S>(tb, tau_field, site);
  const Macro<D> mac = collide_site<ST, N, A, DEV, true, true>(tb, f, tau, site_wall(tb, x, y, z));
  if (!mac.ok) flag_error(err);
  store_site<ST, S, false, A>(fout, sites, (uint32_t)site * (uint32_t)sizeof(S), f);
  if (fields0.any) write_fields<D>(fields0, site, sites, mac);
}

// ---------------------------------------------------------------------------
// Dispatch
// ---------------------------------------------------------------------------
template <class ST, int N, typename S, bool DEV, typename A = S>
static hipError_t launch_t(const LaunchArgs &a) {
  const Variant vr = kVariants[(a.op == OP_STEP && a.variant >= 0 && a.variant < kNumVariants) ? a.variant : 0];
  const int by = ST::D == 2 ? vr.by * vr.bz : vr.by, bz = ST::D == 2 ? 1 : vr.bz;
  dim3 block(vr.bx, by, bz);
  const long gx = (a.nx + vr.bx - 1) / vr.bx, gy = (a.ny + by - 1) / by, gz = (a.nz + bz - 1) / bz;
  const int order = (ST::D == 2 && vr.xcd == 2) ? 1 : vr.xcd;
  long nb = gx * gy * gz;
  if (order == 2) {
    const long py = std::max(1, kPatch / by), pz = std::max(1, kPatch / bz);
    const long npatch = ((gy + py - 1) / py) * ((gz + pz - 1) / pz);
    nb = 8 * ((npatch + 7) / 8) * gx * py * pz;
  }
  dim3 grid((unsigned)nb, 1, 1);
  const Tiling tl{vr.bx, by, bz, (int)nb, order};
  // the 143 doubles of the 3D massive rule overflow the registers (scratch spills): stream them;
  // 143 floats fit, and there the single load is faster
  constexpr bool kStream = (ST::ONLAT && ST::SHIFT && ST::D == 3 && sizeof(S) == 8) || ST::Q > 144;
  // the 288 populations of the (3+1)-d massless rule do not fit in registers in either storage: its
  // moments and initial state take the streaming forms too
  constexpr bool kStreamAll = ST::Q > 144;
  switch (a.op) {
    case OP_STEP: {
      // one instantiation per (occupancy target 0, 2 or 4, force/walls, store kind)
      auto go = [&](auto occ, auto ext, auto nt) {
        constexpr int O = decltype(occ)::value;
        constexpr bool E = decltype(ext)::value, T = decltype(nt)::value;
        if constexpr (kStream) {
          hipLaunchKernelGGL((k_step_stream<ST, N, S, DEV, O, T>), grid, block, 0, a.stream, a.tb,
                             (const S *)a.fin, (S *)a.fout, a.tau_field, a.fields, a.err, tl);
        } else {
          hipLaunchKernelGGL((k_step<ST, N, S, DEV, O, E, T, A>), grid, block, 0, a.stream, a.tb, (const S *)a.fin,
                             (S *)a.fout, a.tau_field, a.fields, a.err, tl);
        }
      };
      using O0 = std::integral_constant<int, 0>;
      using O2 = std::integral_constant<int, 2>;
      using O4 = std::integral_constant<int, 4>;
      using F = std::false_type;
      using T = std::true_type;
      const bool ext = a.ext && !kStream;
      if constexpr (kStreamAll) {
        // one build (no occupancy target) for the 288-vector rule: every other build multiplies its
        // compile time and none is faster for a kernel that streams its populations
        if (a.nt) go(O0{}, F{}, T{});
        else go(O0{}, F{}, F{});
      } else if (ext) {
        if (a.nt) go(O0{}, T{}, T{});
        else go(O0{}, T{}, F{});
      } else if (vr.occ == 2) {
        if (a.nt) go(O2{}, F{}, T{});
        else go(O2{}, F{}, F{});
      } else if (vr.occ == 4) {
        if (a.nt) go(O4{}, F{}, T{});
        else go(O4{}, F{}, F{});
      } else {
        if (a.nt) go(O0{}, F{}, T{});
        else go(O0{}, F{}, F{});
      }
      break;
    }
    case OP_MOMENTS:
      if constexpr (kStreamAll)
        hipLaunchKernelGGL((k_moments_stream<ST, N, S, DEV>), grid, block, 0, a.stream, a.tb, (const S *)a.fin,
                           a.fields, a.err, tl);
      else
        hipLaunchKernelGGL((k_moments<ST, N, S, DEV, A>), grid, block, 0, a.stream, a.tb, (const S *)a.fin, a.fields,
                           a.err, tl);
      break;
    case OP_INIT:
      if constexpr (kStreamAll)
        hipLaunchKernelGGL((k_init_stream<ST, N, S, DEV>), grid, block, 0, a.stream, a.tb, a.n0, a.T0, a.u0,
                           a.noise, a.amp, (S *)a.fout, a.tau_field, a.fields, a.err, tl);
      else
        hipLaunchKernelGGL((k_init<ST, N, S, DEV, A>), grid, block, 0, a.stream, a.tb, a.n0, a.T0, a.u0, a.noise,
                           a.amp, (S *)a.fout, a.tau_field, a.fields, a.err, tl);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// storage 0: double; 1: float deviations updated in float; 2: float deviations updated in double
// (product rules)
template <class ST, int N>
static hipError_t launch_storage(const LaunchArgs &a) {
  if (a.storage == 0) return launch_t<ST, N, double, false>(a);
  if (a.storage == 1) return launch_t<ST, N, float, true>(a);
  if constexpr (!ST::ONLAT) return launch_t<ST, N, float, true, double>(a);
  return hipErrorInvalidValue;
}

hipError_t launch(const LaunchArgs &a) {
  if (a.stencil == ST_UR2D) {
    if (a.order == 2) return launch_storage<Stencil<ST_UR2D, 3>, 2>(a);
    return launch_storage<Stencil<ST_UR2D, 4>, 3>(a);
  }
  if (a.stencil == ST_MASSIVE2D) {
    if (a.order == 2) return launch_storage<Stencil<ST_MASSIVE2D, 2>, 2>(a);
    return launch_storage<Stencil<ST_MASSIVE2D, 3>, 3>(a);
  }
  if (a.stencil == ST_MASSIVE3D) return launch_storage<Stencil<ST_MASSIVE3D, 3>, 3>(a);
  if (a.stencil == ST_UR3D) return launch_storage<Stencil<ST_UR3D, 4>, 3>(a);
  if (a.stencil == ST_PROD2D) {
    if (a.order == 2) return launch_storage<Stencil<ST_PROD2D, 3>, 2>(a);
    return launch_storage<Stencil<ST_PROD2D, 4>, 3>(a);
  }
  if (a.stencil == ST_PROD3D) {
    if (a.order == 2) return launch_storage<Stencil<ST_PROD3D, 3>, 2>(a);
    return launch_storage<Stencil<ST_PROD3D, 4>, 3>(a);
  }
  return hipErrorInvalidValue;
}

}  // namespace rlbm
