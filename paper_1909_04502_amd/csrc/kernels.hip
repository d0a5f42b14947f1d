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

// LDS-staged pull of the 2D product rules (periodic x; every row a whole number of 16-byte chunks).
// A block of 64 x 4 sites stages, one shell at a time, the upstream windows of the shell's 8 planes
// in LDS: 5 rows (the tile's 4 and the row upstream of it in y) of 64 + 2E columns (E elements to
// either side), brought in by direct global-to-LDS loads of 16 bytes per lane, which hold no
// registers while in flight.  Two buffers alternate, so the loads of shell j + 1 are in flight
// while the taps of shell j are read from LDS and summed; the block's four waves share each window.
// The taps, weights and summation order are those of pull_prod, so the populations are the same
// values to the last bit.  Sites past the lattice's edge take part in the loads and barriers and
// skip the update.
template <class ST>
constexpr uint32_t lds_row_back() {
  uint32_t m = 0;
  for (int k = 0; k < ST::NDIR; ++k)
    if (ST::dir(k, 1) > 0) m |= 1u << k;
  return m;
}

template <class ST, typename S>
struct LdsWindow {
  static constexpr int E = 16 / (int)sizeof(S);   // elements per 16-byte chunk
  static constexpr int W = 64 + 2 * E;             // window columns, from x0 - E
  static constexpr int CR = W / E;                 // chunks per window row
  static constexpr int RW = 5;                     // window rows
  static constexpr int CP = RW * CR;               // chunks per plane
  static constexpr int NIP = (CP + 63) / 64;       // load instructions per plane (one plane each)
  static constexpr int PW = ST::NDIR / 4;          // planes per wave and shell
  static constexpr int NI = PW * NIP;              // load instructions per wave and shell
  static_assert(ST::NDIR % 4 == 0, "a shell's planes split evenly over the four waves");
  // directions whose window starts one row before the tile (upstream in y is y - 1)
  static constexpr uint32_t kRowBack = lds_row_back<ST>();
};

// s_waitcnt vmcnt(N) lgkmcnt(0) (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4 left at its
// maximum, lgkmcnt 11:8): all but the N most recent vector memory loads of this wave, to registers
// or to LDS, and every LDS read of this wave are done
template <int N>
__device__ __forceinline__ void wait_vm_lgkm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (0x7 << 4));
}
__device__ __forceinline__ void wait_lgkm() { __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (0x7 << 4)); }

// One direct global-to-LDS load: each active lane l reads the 16 bytes at base + voff and writes
// them to LDS at byte lds + 16 l (base and lds wave-uniform; m0 holds the LDS address, and one
// wait state separates its write from the load).  Written as asm so that the compiler does not
// track these loads: it would make every LDS read of the kernel wait for all of them.  The kernel
// waits for them itself (wait_vm_lgkm); they have no register results.
__device__ __forceinline__ void lds_load16(const void *base, uint32_t voff, uint32_t lds) {
  // both uniform operands pass through readfirstlane: the compiler may otherwise hold a uniform
  // value it cannot prove uniform in a vector register, which an "s" operand does not accept
  const uint64_t b = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)((uintptr_t)base >> 32)) << 32) |
                     (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)base);
  const uint32_t m = __builtin_amdgcn_readfirstlane(lds);
  asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, %0" : : "s"(b), "v"(voff), "s"(m)
               : "memory", "m0");
}

// Byte offsets within a plane of this lane's chunk in each load instruction of a plane, for windows
// starting at the tile's first row (back = 0) or one row before it (back = 1).  Wave w loads the
// planes w, w + 4, ... of every shell; a lane's chunk of instruction n is n * 64 + lane of the plane.
template <class ST, typename S>
__device__ __forceinline__ void lds_offsets(const Tables *__restrict__ tb, int x0, int y0,
                                            uint32_t (&off)[2][LdsWindow<ST, S>::NIP]) {
  using L = LdsWindow<ST, S>;
  const int nx = tb->nx, ny = tb->ny, openy = tb->open[1];
#pragma unroll
  for (int n = 0; n < L::NIP; ++n) {
    const int c = n * 64 + (int)threadIdx.x;
    const int r = c / L::CR, q = c - r * L::CR;
    // one wrap brings every row and column an update reads into the lattice; on lattices narrower
    // or shorter than the window the rest may still lie past the edge and are read from row or
    // column 0 instead (no site uses them); lanes past the window are masked off at the load
    int xs = x0 - L::E + q * L::E;
    xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
    xs = xs < nx ? xs : 0;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      int ys = wrap_or_clamp(y0 - b + r, ny, openy);
      ys = ys < ny ? ys : 0;
      off[b][n] = ((uint32_t)ys * (uint32_t)nx + (uint32_t)xs) * (uint32_t)sizeof(S);
    }
  }
}

template <class ST, typename S, int NIP>
__device__ __forceinline__ void lds_load_shell(const S *__restrict__ fin, int64_t sites, int shell, int w,
                                               const uint32_t (&off)[2][NIP], S *dst_) {
  using L = LdsWindow<ST, S>;
  // LDS byte address of the buffer (the low 32 bits of a local-address-space pointer)
  const uint32_t lds = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) S *)dst_;
#pragma unroll
  for (int e = 0; e < L::PW; ++e) {
    const int p = w + 4 * e;   // wave-uniform
    const int b = (L::kRowBack >> p) & 1u;
    const char *plane = (const char *)fin + (int64_t)(shell * ST::NDIR + p) * sites * (int64_t)sizeof(S);
#pragma unroll
    for (int n = 0; n < L::NIP; ++n) {
      if (L::CP % 64 == 0 || n * 64 + (int)threadIdx.x < L::CP)
        lds_load16(plane, b ? off[1][n] : off[0][n], lds + (uint32_t)((p * L::CP + n * 64) * 16));
    }
  }
}

// Taps of shell j from its staged windows: the values (read) and their weighted sums (interpolate)
// are separate steps, so that the next shell's loads can be issued between them.
template <class ST, typename S>
struct LdsTaps {
  static constexpr int count() {
    int c = 0;
    for (int k = 0; k < ST::NDIR; ++k) c += 1 << ((ST::dir(k, 0) != 0) + (ST::dir(k, 1) != 0));
    return c;
  }
  S v[count()];
};

// src: the buffer plus this thread's window offset (lds_lane_offset)
template <class ST, typename S>
__device__ __forceinline__ void lds_read_taps(const __attribute__((address_space(3))) S *src, LdsTaps<ST, S> &t) {
  using L = LdsWindow<ST, S>;
  int m = 0;
#pragma unroll
  for (int k = 0; k < ST::NDIR; ++k) {
    const int dx = ST::dir(k, 0), dy = ST::dir(k, 1);
    const int z = (dx != 0) + (dy != 0);
    const __attribute__((address_space(3))) S *pl = src + k * L::RW * L::W + (dy > 0 ? L::W : 0);
#pragma unroll
    for (int tap = 0; tap < (1 << z); ++tap) {
      int bit = 0, ox = 0, oy = 0;
      if (dx != 0) {
        const int c = (tap >> bit++) & 1;
        ox = dx > 0 ? (c ? 0 : -1) : (c ? 1 : 0);
      }
      if (dy != 0) {
        const int c = (tap >> bit++) & 1;
        oy = dy > 0 ? (c ? 0 : -1) : (c ? 1 : 0);
      }
      t.v[m++] = pl[oy * L::W + ox];
    }
  }
}

template <class ST, typename S, typename A>
__device__ __forceinline__ void lds_interpolate(const Tables *__restrict__ tb, int j, const LdsTaps<ST, S> &t,
                                                A (&f)[ST::Q]) {
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
      for (int q = 0; q < nf; ++q) r *= mag;
#pragma unroll
      for (int q = nf; q < z; ++q) r *= cm;
      pw[z][nf] = r;
    }
  }
  int m = 0;
#pragma unroll
  for (int k = 0; k < ST::NDIR; ++k) {
    const int dx = ST::dir(k, 0), dy = ST::dir(k, 1);
    const int z = (dx != 0) + (dy != 0);
    A acc = 0;
#pragma unroll
    for (int tap = 0; tap < (1 << z); ++tap) {
      int bit = 0, nfar = 0;
      if (dx != 0) nfar += dx > 0 ? !((tap >> bit++) & 1) : ((tap >> bit++) & 1);
      if (dy != 0) nfar += dy > 0 ? !((tap >> bit++) & 1) : ((tap >> bit++) & 1);
      acc += pw[z][nfar] * (A)t.v[m++];
    }
    f[j * ST::NDIR + k] = acc;
  }
}

// One 64 x 4 tile per block; tiles are dealt to the 8 XCDs in contiguous bands of the row-major tile
// order (block b runs on XCD b mod 8), as the register kernel's band order.
template <class ST, int N, typename S, bool DEV, bool NT, typename A = S>
__global__ void __launch_bounds__(256) k_step_lds(const Tables *__restrict__ tb, const S *__restrict__ fin,
                                                  S *__restrict__ fout, const void *__restrict__ tau_field,
                                                  FieldPtrs last, int *err, Tiling tl) {
  static_assert(ST::D == 2 && !ST::ONLAT && ST::NDIR == 8, "2D product rules");
  using L = LdsWindow<ST, S>;
  constexpr int KR = ST::NSHELL;
  static_assert(KR >= 2, "two shells in flight");
  constexpr int HALF = ST::NDIR * L::RW * L::W;   // elements of one buffer
  __shared__ __attribute__((aligned(16))) S buf[2 * HALF];
  typedef __attribute__((address_space(3))) S lds_t;
  const uint32_t gx = (tb->nx + 63) / 64;
  uint32_t t = blockIdx.x;
  {
    const uint32_t q = tl.nb / 8, r = tl.nb % 8, k = t % 8, l = t / 8;
    t = k * q + (k < r ? k : r) + l;
  }
  const int x0 = (int)(t % gx) * 64, y0 = (int)(t / gx) * 4;
  const int x = x0 + threadIdx.x, y = y0 + threadIdx.y;
  const int64_t sites = tb->sites;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.y);
  uint32_t off[2][L::NIP];
  lds_offsets<ST, S>(tb, x0, y0, off);
  lds_load_shell<ST, S>(fin, sites, 0, w, off, buf);
  lds_load_shell<ST, S>(fin, sites, 1, w, off, buf + HALF);
  const uint32_t lane_off = threadIdx.y * L::W + threadIdx.x + L::E;   // this thread's window offset
  A f[ST::Q];
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    // shell j has landed in this wave's part of its buffer once at most the loads of shell j + 1
    // are in flight (no other vector memory access is issued before the last shell); the barrier
    // extends that to the whole block
    if (j + 1 < KR) wait_vm_lgkm<L::NI>();
    else wait_vm_lgkm<0>();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    const lds_t *src = (const lds_t *)buf + (j & 1) * HALF + lane_off;
    LdsTaps<ST, S> taps;
    lds_read_taps<ST, S>(src, taps);
    if (j + 2 < KR) {
      // every wave has read shell j before its buffer is refilled with shell j + 2, whose loads
      // then overlap the interpolation and shell j + 1
      wait_lgkm();
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
      lds_load_shell<ST, S>(fin, sites, j + 2, w, off, buf + (j & 1) * HALF);
    }
    lds_interpolate<ST, S, A>(tb, j, taps, f);
    // the shell's sums are formed here, before the next barrier, so that its taps do not stay live
    // in registers across the later shells (the compiler would otherwise sink every sum to the end)
#pragma unroll
    for (int k = 0; k < ST::NDIR; ++k) asm volatile("" : "+v"(f[j * ST::NDIR + k]));
  }
  if (x >= tb->nx || y >= tb->ny) return;
  const int64_t site = (int64_t)y * tb->nx + x;
  const double tau = site_tau<S>(tb, tau_field, site);
  const Macro<ST::D> mac = collide_site<ST, N, A, DEV, true, false>(tb, f, tau, -1.0);
  if (!mac.ok) flag_error(err);
  store_site<ST, S, NT, A>(fout, sites, (uint32_t)site * (uint32_t)sizeof(S), f);
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
      if constexpr (ST::D == 2 && !ST::ONLAT) {
        if (vr.lds && a.lds_ok && !ext) {
          const long ntile = ((a.nx + 63) / 64) * (long)((a.ny + 3) / 4);
          const Tiling ltl{64, 4, 1, (int)ntile, 1};
          auto lds = [&](auto nt) {
            constexpr bool T = decltype(nt)::value;
            hipLaunchKernelGGL((k_step_lds<ST, N, S, DEV, T, A>), dim3((unsigned)ntile, 1, 1), dim3(64, 4, 1), 0,
                               a.stream, a.tb, (const S *)a.fin, (S *)a.fout, a.tau_field, a.fields, a.err, ltl);
          };
          if (a.nt) lds(T{});
          else lds(F{});
          break;
        }
      }
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
