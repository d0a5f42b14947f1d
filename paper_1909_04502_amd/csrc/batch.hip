// batch.hip -- many independent lattices in one persistent launch (HIP, gfx950).
//
// Every lattice keeps its own constant tables (zeta, tau, quadrature) and its
// own SoA population block inside one flat state buffer.  The work is a list
// of tiles (lattice, tile index: a 2D tile of sites, or a run of 256 consecutive
// sites); a fixed grid of workgroups walks it, each
// XCD taking a contiguous range of tiles so that neighbouring tiles of a
// lattice share that XCD's L2.  All lattices of a batch use the same stencil,
// order and storage (one kernel instantiation).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "prod_math.h"

namespace rlbm {

__device__ __forceinline__ int wrap_b(int v, int n, int open) {
  if (open) return v < 0 ? 0 : (v >= n ? n - 1 : v);
  v = v < 0 ? v + n : v;
  return v >= n ? v - n : v;
}

template <class ST, int N, typename S, bool DEV, int BX, int BY, bool EXT, bool NT, typename A = S>
__global__ void __launch_bounds__(BX * BY) k_step_batch(const Tables *__restrict__ tabs,
                                                        const int64_t *__restrict__ elem_off,
                                                        const int2 *__restrict__ tiles, int ntiles,
                                                        const S *__restrict__ fin, S *__restrict__ fout, int *err) {
  // a one-row block of 256 takes 256 consecutive sites (tile shape kBatchLinearTile)
  constexpr bool LINEAR = BX == 256 && BY == 1;
  // XCD k (blocks with blockIdx.x % 8 == k) walks tiles [k*chunk, (k+1)*chunk)
  const int per_xcd = gridDim.x / 8;
  const int k = blockIdx.x % 8, b = blockIdx.x / 8;
  const int chunk = (ntiles + 7) / 8;
  const int lo = k * chunk, hi = min(ntiles, lo + chunk);
  for (int t = lo + b; t < hi; t += per_xcd) {
    const int2 d = tiles[t];
    const Tables *__restrict__ tb = tabs + d.x;
    const int nx = tb->nx, ny = tb->ny;
    const int64_t sites = tb->sites;
    int x, y;
    int64_t site;
    if constexpr (LINEAR) {
      // 256 consecutive sites in row-major order
      site = (int64_t)d.y * BX + threadIdx.x;
      if (site >= sites) continue;
      y = (int)(site / nx);
      x = (int)(site - (int64_t)y * nx);
    } else {
      const int gx = (nx + BX - 1) / BX;
      x = (d.y % gx) * BX + threadIdx.x;
      y = (d.y / gx) * BY + threadIdx.y;
      if (x >= nx || y >= ny) continue;
      site = (int64_t)y * nx + x;
    }
    const S *fi = fin + elem_off[d.x];
    S *fo = fout + elem_off[d.x];
    Offs o;
#pragma unroll
    for (int dd = -1; dd <= 1; ++dd) {
      o.x[dd + 1] = (uint32_t)wrap_b(x + dd, nx, tb->open[0]) * (uint32_t)sizeof(S);
      o.y[dd + 1] = (uint32_t)wrap_b(y + dd, ny, tb->open[1]) * (uint32_t)nx * (uint32_t)sizeof(S);
      o.z[dd + 1] = 0u;
    }
    A f[ST::Q];
    pull_prod<ST, S, false, A>(tb, fi, sites, o, f);
    const Macro<ST::D> mac = collide_prod<ST, N, A, DEV, true, EXT>(tb, f, tb->tau, EXT ? site_wall(tb, x, y, 0) : -1.0);
    if (!mac.ok) *(volatile int *)err = 1;
    const uint32_t so = (uint32_t)site * (uint32_t)sizeof(S);
#pragma unroll
    for (int i = 0; i < ST::Q; ++i) put_pop<NT>(fo, sites, so, i, (S)f[i]);
  }
}

template <class ST, int N, typename S, bool DEV, bool EXT, bool NT, typename A = S>
static hipError_t launch_batch_t(const BatchArgs &a) {
  const int nb = a.blocks;
  switch (a.tile) {
    case 0:
      hipLaunchKernelGGL((k_step_batch<ST, N, S, DEV, 64, 4, EXT, NT, A>), dim3(nb), dim3(64, 4), 0, a.stream, a.tabs,
                         a.elem_off, a.tiles, a.ntiles, (const S *)a.fin, (S *)a.fout, a.err);
      break;
    case 1:
      hipLaunchKernelGGL((k_step_batch<ST, N, S, DEV, 64, 2, EXT, NT, A>), dim3(nb), dim3(64, 2), 0, a.stream, a.tabs,
                         a.elem_off, a.tiles, a.ntiles, (const S *)a.fin, (S *)a.fout, a.err);
      break;
    case 2:
      hipLaunchKernelGGL((k_step_batch<ST, N, S, DEV, 128, 2, EXT, NT, A>), dim3(nb), dim3(128, 2), 0, a.stream, a.tabs,
                         a.elem_off, a.tiles, a.ntiles, (const S *)a.fin, (S *)a.fout, a.err);
      break;
    default:
      hipLaunchKernelGGL((k_step_batch<ST, N, S, DEV, 256, 1, EXT, NT, A>), dim3(nb), dim3(256, 1), 0, a.stream, a.tabs,
                         a.elem_off, a.tiles, a.ntiles, (const S *)a.fin, (S *)a.fout, a.err);
      break;
  }
  return hipGetLastError();
}

// storage 0: double; 1: float deviations updated in float; 2: float deviations updated in double
template <class ST, int N, bool EXT, bool NT>
static hipError_t launch_batch_storage(const BatchArgs &a) {
  if (a.storage == 0) return launch_batch_t<ST, N, double, false, EXT, NT>(a);
  if (a.storage == 1) return launch_batch_t<ST, N, float, true, EXT, NT>(a);
  return launch_batch_t<ST, N, float, true, EXT, NT, double>(a);
}

template <bool NT>
static hipError_t launch_batch_ext(const BatchArgs &a) {
  if (a.ext) {
    if (a.order == 2) return launch_batch_storage<Stencil<ST_PROD2D, 3>, 2, true, NT>(a);
    return launch_batch_storage<Stencil<ST_PROD2D, 4>, 3, true, NT>(a);
  }
  if (a.order == 2) return launch_batch_storage<Stencil<ST_PROD2D, 3>, 2, false, NT>(a);
  return launch_batch_storage<Stencil<ST_PROD2D, 4>, 3, false, NT>(a);
}

hipError_t launch_batch(const BatchArgs &a) {
  // every XCD needs at least one workgroup of the persistent grid (blocks / 8 > 0)
  if (a.stencil != ST_PROD2D || a.blocks < 8 || a.blocks % 8 != 0 || a.tile < 0 || a.tile > 3)
    return hipErrorInvalidValue;
  if (a.ntiles == 0) return hipSuccess;
  return a.nt ? launch_batch_ext<true>(a) : launch_batch_ext<false>(a);
}

}  // namespace rlbm
