// adjoint.hip -- reverse-mode kernels of the RLBM step (HIP, gfx950).
//
// State sequence: B_0 = C(f_0), F_t = S(B_{t-1}), B_t = C(F_t) (S streaming,
// C collision).  Adjoints lam_t = dL/dF_t obey
//   lam_t = J_C(F_t)^T S^T lam_{t+1},   dL/dtau += (dC/dtau)^T S^T lam_{t+1},
// and the loss on the macroscopic fields of F_{T+1} = S(B_T) seeds
// lam_{T+1} = J_macro(F_{T+1})^T g.  Each kernel recomputes the forward
// values of its site from the stored state (no per-site tape is kept).
#include <hip/hip_runtime.h>

#include "adjoint_math.h"
#include "kernels.h"

namespace rlbm {

// Site of this thread: kAdjBX x kAdjBY tiles, dealt so that each XCD takes a contiguous band of
// them (the hardware deals consecutive blocks round-robin to the 8 XCDs) and the tap halos of
// neighbouring tiles stay in that XCD's L2 (4-5 % faster than the order as dealt).  The tile
// shape is a constant and the block count follows from the lattice (blockDim and gridDim would be
// vector loads from the dispatch packet that each wave waits for).
constexpr int kAdjBX = 64, kAdjBY = 4;

__device__ __forceinline__ bool site_xyz(const Tables *__restrict__ tb, int &x, int &y, int &z) {
  const uint32_t gx = (tb->nx + kAdjBX - 1) / kAdjBX, gy = (tb->ny + kAdjBY - 1) / kAdjBY;
  uint32_t t = blockIdx.x;
  {
    const uint32_t nb = gx * gy * (uint32_t)tb->nz, q = nb / 8, r = nb % 8, k = t % 8, l = t / 8;
    t = k * q + (k < r ? k : r) + l;
  }
  x = (t % gx) * kAdjBX + threadIdx.x;
  y = ((t / gx) % gy) * kAdjBY + threadIdx.y;
  z = t / (gx * gy);
  return x < tb->nx && y < tb->ny;
}

__device__ __forceinline__ int wrap_p(int v, int n) {
  v = v < 0 ? v + n : v;
  return v >= n ? v - n : v;
}

template <class ST, typename S>
__device__ __forceinline__ Offs offs_periodic(const Tables *__restrict__ tb, int x, int y, int z) {
  Offs o;
  const uint32_t nx = tb->nx, nxy = (uint32_t)tb->nx * tb->ny;
#pragma unroll
  for (int d = -1; d <= 1; ++d) {
    o.x[d + 1] = (uint32_t)wrap_p(x + d, tb->nx) * (uint32_t)sizeof(S);
    o.y[d + 1] = (uint32_t)wrap_p(y + d, tb->ny) * nx * (uint32_t)sizeof(S);
    o.z[d + 1] = ST::D == 3 ? (uint32_t)wrap_p(z + d, tb->nz) * nxy * (uint32_t)sizeof(S) : 0u;
  }
  return o;
}

template <typename S>
__device__ __forceinline__ double tau_at(const Tables *__restrict__ tb, const void *tau_field, int64_t site) {
  return tau_field == nullptr ? tb->tau : (double)((const S *)tau_field)[site];
}

// all writers store the same value: a plain store (a volatile one makes the wave wait for its loads)
__device__ __forceinline__ void set_err(int *err) { *err = 1; }

// lam_t(x) = J_C(F_t(x))^T (S^T lam_{t+1})(x), F_t = S(B_{t-1}); dtau(x) += dL/dtau(x)
template <class ST, int N, typename S, bool DEV, typename A = S>
__global__ void __launch_bounds__(256) k_adjoint(const Tables *__restrict__ tb, const S *__restrict__ Bprev,
                                                 const S *__restrict__ lam_next, S *__restrict__ lam,
                                                 const void *__restrict__ tau_field, double *__restrict__ dtau,
                                                 int *err) {
  int x, y, z;
  if (!site_xyz(tb, x, y, z)) return;
  const int64_t sites = tb->sites;
  const int64_t site = ((int64_t)z * tb->ny + y) * tb->nx + x;
  const Offs o = offs_periodic<ST, S>(tb, x, y, z);
  A f[ST::Q], mu[ST::Q];
  pull_prod<ST, S, false, A>(tb, Bprev, sites, o, f);
  pull_prod<ST, S, true, A>(tb, lam_next, sites, o, mu);
  double taub;
  if (!collide_vjp<ST, N, A, DEV>(tb, f, mu, tau_at<S>(tb, tau_field, site), taub)) set_err(err);
  const uint32_t so = (uint32_t)site * (uint32_t)sizeof(S);
#pragma unroll
  for (int i = 0; i < ST::Q; ++i) *(S *)((char *)(lam + (int64_t)i * sites) + so) = (S)f[i];
  if (dtau != nullptr) dtau[site] += taub;
}

// The same reverse step for float storage and arithmetic, in three passes over the shells that each
// pull what they need again (cache hits: the taps were read just before), so that one shell's
// populations are live at a time instead of all Q twice over: the moments of F_t; the reverse of the
// relaxation and of the equilibrium (F_t and S^T lam_{t+1}); and lam_t = mu (1 - Omega) + the terms
// through n, T and U, stored shell by shell.  That fits two waves per SIMD.
template <class ST, int N, typename S, bool DEV>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
k_adjoint_streamed(const Tables *__restrict__ tb, const S *__restrict__ Bprev, const S *__restrict__ lam_next,
                   S *__restrict__ lam, const void *__restrict__ tau_field, double *__restrict__ dtau, int *err) {
  constexpr int D = ST::D, ND = ST::NDIR, NPD = ND / 2, KR = ST::NSHELL;
  using B = BasisDef<D, N>;
  using A = S;
  int x, y, z;
  if (!site_xyz(tb, x, y, z)) return;
  const int64_t sites = tb->sites;
  const int64_t site = ((int64_t)z * tb->ny + y) * tb->nx + x;
  const Offs o = offs_periodic<ST, S>(tb, x, y, z);
  // ---- forward recomputation: moments, Landau frame, n, T, equilibrium coefficients ----
  MomAcc<D> acc;
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    A fs[ND];
    pull_shell<ST, S, false, A>(tb, Bprev, sites, o, j, fs);
    moments_shell<ST, A, ND>(tb, j, fs, 0, acc);
  }
  double Nv[D + 1], T[D + 1][D + 1];
  moments_finish<ST, DEV>(tb, acc, Nv, T);
  Macro<D> mac;
  mac.ok = landau_frame<D, 3>(T, mac.eps, mac.U);
  mac.n = lorentz_dot<D>(mac.U, Nv);
  const double m = tb->m;
  mac.ok = temperature_2d(mac.eps / mac.n, m, mac.T) && mac.ok;
  mac.ok = mac.ok && mac.n > 0.0 && mac.eps > 0.0;
  if (!mac.ok) set_err(err);
  const RatiosD rd = ratios_2d_d(m / mac.T);
  double ap[B::NM];
  {
    Ratios rr;
    rr.r0 = rd.r0;
    rr.r2 = rd.r2;
    rr.r3 = rd.r3;
    double Md[B::NM];
    basis_moments<D, N>(mac.n, mac.T, mac.U, rr, Md);
    feq_coefficients<D, N, DEV>(tb, Md, ap);
  }
  const double itau = 1.0 / tau_at<S>(tb, tau_field, site);
  const double a0 = mac.U[0] * itau;
  double nU[NPD];
#pragma unroll
  for (int q = 0; q < NPD; ++q) {
    double c0 = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double c = nhat<ST>(2 * q, a);
      if (c != 0.0) c0 += c * mac.U[a + 1];
    }
    nU[q] = c0 * itau;
  }
  // ---- reverse of the relaxation and of the equilibrium evaluation ----
  // (the base pointers pass through an empty asm on a forward result: the pulls are issued again
  // here rather than their values kept live from the pass above)
  const S *fb = Bprev, *lb = lam_next;
  asm volatile("" : "+s"(fb), "+s"(lb) : "v"(ap[0]));
  double a0b = 0.0, nUb[NPD], apb[B::NM];
#pragma unroll
  for (int q = 0; q < NPD; ++q) nUb[q] = 0.0;
#pragma unroll
  for (int k = 0; k < B::NM; ++k) apb[k] = 0.0;
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    A fs[ND], ms[ND];
    pull_shell<ST, S, false, A>(tb, fb, sites, o, j, fs);
    pull_shell<ST, S, true, A>(tb, lb, sites, o, j, ms);
    relax_vjp_shell<ST, N, A>(tb, j, fs, ms, ap, a0, nU, a0b, nUb, apb);
  }
  // Omega depends on tau through a0 = U^0 / tau and nU = (n . U) / tau
  double Ub[D + 1];
  Ub[0] = a0b * itau;
  double taub = -a0b * a0;
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
  // ---- reverse of the equilibrium coefficients, EOS, density and Landau frame ----
  double Mb[B::NM];
  coefficients_vjp<D, N>(tb, apb, Mb);
  double nb = 0.0, Tb = 0.0;
  basis_moments_vjp<D, N>(mac.n, mac.T, mac.U, m, rd, Mb, nb, Tb, Ub);
  double Nb[D + 1], Tbar[D + 1][D + 1], Ts[D + 1][D + 1];
  macro_vjp_moments<D>(tb, Nv, T, mac, nb, 0.0, Tb, Ub, Nb, Tbar);
#pragma unroll
  for (int a = 0; a <= D; ++a)
#pragma unroll
    for (int b = 0; b <= D; ++b) Ts[a][b] = 0.5 * (Tbar[a][b] + Tbar[b][a]);
  // ---- lam_t = mu (1 - Omega) + dL/dN^a p^a + dL/dT^ab p^a p^b, shell by shell ----
  const S *lb2 = lam_next;
  asm volatile("" : "+s"(lb2) : "v"(Nb[0]));
  const uint32_t so = (uint32_t)site * (uint32_t)sizeof(S);
#pragma unroll
  for (int j = 0; j < KR; ++j) {
    A ms[ND], out[ND];
    pull_shell<ST, S, true, A>(tb, lb2, sites, o, j, ms);
    const double v = tb->sv[j];
#pragma unroll
    for (int qp = 0; qp < NPD; ++qp) {
      const double b = v * nU[qp];
      out[2 * qp] = (A)((double)ms[2 * qp] * (1.0 - (a0 - b)));
      out[2 * qp + 1] = (A)((double)ms[2 * qp + 1] * (1.0 - (a0 + b)));
    }
    moments_vjp_shell<ST, A, ND>(tb, j, Nb, Ts, out, 0);
#pragma unroll
    for (int k = 0; k < ND; ++k) *(S *)((char *)(lam + (int64_t)(j * ND + k) * sites) + so) = (S)out[k];
  }
  if (dtau != nullptr) dtau[site] += taub;
}

// lam_{T+1}(x) = J_macro(F(x))^T g(x), F = S(B); g = (dL/dn, dL/deps, dL/dT, dL/dU)
template <class ST, int N, typename S, bool DEV, typename A = S>
__global__ void __launch_bounds__(256) k_moments_vjp(const Tables *__restrict__ tb, const S *__restrict__ B,
                                                     FieldPtrs g, S *__restrict__ lam, int *err) {
  constexpr int D = ST::D;
  int x, y, z;
  if (!site_xyz(tb, x, y, z)) return;
  const int64_t sites = tb->sites;
  const int64_t site = ((int64_t)z * tb->ny + y) * tb->nx + x;
  const Offs o = offs_periodic<ST, S>(tb, x, y, z);
  A f[ST::Q];
  pull_prod<ST, S, false, A>(tb, B, sites, o, f);
  double Nv[D + 1], T[D + 1][D + 1];
  moments_prod<ST, A, DEV>(tb, f, Nv, T);
  Macro<D> mac;
  mac.ok = landau_frame<D, 3>(T, mac.eps, mac.U);
  mac.n = lorentz_dot<D>(mac.U, Nv);
  mac.ok = temperature_2d(mac.eps / mac.n, tb->m, mac.T) && mac.ok && mac.n > 0.0 && mac.eps > 0.0;
  if (!mac.ok) set_err(err);
  double Ub[D + 1];
#pragma unroll
  for (int a = 0; a <= D; ++a) Ub[a] = g.U ? g.U[a * sites + site] : 0.0;
  const double nb = g.n ? g.n[site] : 0.0, eb = g.eps ? g.eps[site] : 0.0, Tb = g.T ? g.T[site] : 0.0;
  A out[ST::Q];
#pragma unroll
  for (int i = 0; i < ST::Q; ++i) out[i] = 0;
  macro_vjp<ST, A>(tb, Nv, T, mac, nb, eb, Tb, Ub, out);
  const uint32_t so = (uint32_t)site * (uint32_t)sizeof(S);
#pragma unroll
  for (int i = 0; i < ST::Q; ++i) *(S *)((char *)(lam + (int64_t)i * sites) + so) = (S)out[i];
}

// Reverse of the initial condition B_0 = C(f_0), f_0 = f^eq(n0, T0, U(u0)) (1 + amp xi):
// du0 (and dn0, dT0 when requested) from lam_1 = dL/dF_1; dtau(x) += dL/dtau(x).
template <class ST, int N, typename S, bool DEV, typename A = S>
__global__ void __launch_bounds__(256) k_init_vjp(const Tables *__restrict__ tb, const double *__restrict__ n0,
                                                  const double *__restrict__ T0, const double *__restrict__ u0,
                                                  const double *__restrict__ noise, double amp,
                                                  const S *__restrict__ lam1, const void *__restrict__ tau_field,
                                                  double *__restrict__ du0, double *__restrict__ dn0,
                                                  double *__restrict__ dT0, double *__restrict__ dtau, int *err) {
  constexpr int D = ST::D, Q = ST::Q;
  using B = BasisDef<D, N>;
  int x, y, z;
  if (!site_xyz(tb, x, y, z)) return;
  const int64_t sites = tb->sites;
  const int64_t site = ((int64_t)z * tb->ny + y) * tb->nx + x;
  double U[D + 1], u[D], uu = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    u[a] = u0[a * sites + site];
    uu += u[a] * u[a];
  }
  const double gam = 1.0 / sqrt(1.0 - uu);
  U[0] = gam;
#pragma unroll
  for (int a = 0; a < D; ++a) U[a + 1] = gam * u[a];
  const double n = n0[site], T = T0[site];
  const RatiosD rd = ratios_2d_d(tb->m / T);
  Ratios rr;
  rr.r0 = rd.r0;
  rr.r2 = rd.r2;
  rr.r3 = rd.r3;
  double M[B::NM];
  basis_moments<D, N>(n, T, U, rr, M);
  double fe[Q];
  feq_prod<ST, N, double, false>(tb, M, fe);
  A f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double sc = noise ? 1.0 + amp * noise[(int64_t)i * sites + site] : 1.0;
    const double fi = fe[i] * sc;
    f[i] = DEV ? (A)(fi - tb->fref[i]) : (A)fi;
  }
  const Offs o = offs_periodic<ST, S>(tb, x, y, z);
  A mu[Q];
  pull_prod<ST, S, true, A>(tb, lam1, sites, o, mu);
  double taub;
  if (!collide_vjp<ST, N, A, DEV>(tb, f, mu, tau_at<S>(tb, tau_field, site), taub)) set_err(err);
  if (dtau != nullptr) dtau[site] += taub;
  // f now holds dL/df_0; through the noise factor to dL/df^eq
  double g[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) g[i] = (double)f[i] * (noise ? 1.0 + amp * noise[(int64_t)i * sites + site] : 1.0);
  double Mb[B::NM];
  feq_vjp<ST, N, double>(tb, g, Mb);
  double nb = 0.0, Tb = 0.0, Ub[D + 1];
#pragma unroll
  for (int a = 0; a <= D; ++a) Ub[a] = 0.0;
  basis_moments_vjp<D, N>(n, T, U, tb->m, rd, Mb, nb, Tb, Ub);
  // U = gamma (1, u):  dL/du_b = gamma Ub^b + gamma^3 u_b (Ub^0 + sum_a Ub^a u_a)
  double s = Ub[0];
#pragma unroll
  for (int a = 0; a < D; ++a) s += Ub[a + 1] * u[a];
  if (du0 != nullptr) {
#pragma unroll
    for (int a = 0; a < D; ++a) du0[a * sites + site] = gam * Ub[a + 1] + gam * gam * gam * u[a] * s;
  }
  if (dn0 != nullptr) dn0[site] = nb;
  if (dT0 != nullptr) dT0[site] = Tb;
}

template <class ST, int N, typename S, bool DEV, typename A = S>
static hipError_t launch_adj_t(const AdjointArgs &a) {
  dim3 block(kAdjBX, kAdjBY, 1);
  const long nb = (long)((a.nx + kAdjBX - 1) / kAdjBX) * ((a.ny + kAdjBY - 1) / kAdjBY) * a.nz;
  dim3 grid((unsigned)nb, 1, 1);
  switch (a.op) {
    case ADJ_STEP:
      // float storage and arithmetic: the streamed kernel (two waves per SIMD); double storage or
      // arithmetic: the register-resident one (re-pulled doubles miss the L1 and the streamed form
      // is slower there)
      if constexpr (sizeof(S) == 4 && sizeof(A) == 4)
        hipLaunchKernelGGL((k_adjoint_streamed<ST, N, S, DEV>), grid, block, 0, a.stream, a.tb, (const S *)a.state,
                           (const S *)a.lam_in, (S *)a.lam_out, a.tau_field, a.dtau, a.err);
      else
        hipLaunchKernelGGL((k_adjoint<ST, N, S, DEV, A>), grid, block, 0, a.stream, a.tb, (const S *)a.state,
                           (const S *)a.lam_in, (S *)a.lam_out, a.tau_field, a.dtau, a.err);
      break;
    case ADJ_MOMENTS:
      hipLaunchKernelGGL((k_moments_vjp<ST, N, S, DEV, A>), grid, block, 0, a.stream, a.tb, (const S *)a.state,
                         a.grads, (S *)a.lam_out, a.err);
      break;
    case ADJ_INIT:
      hipLaunchKernelGGL((k_init_vjp<ST, N, S, DEV, A>), grid, block, 0, a.stream, a.tb, a.n0, a.T0, a.u0, a.noise,
                         a.amp, (const S *)a.lam_in, a.tau_field, a.du0, a.dn0, a.dT0, a.dtau, a.err);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// storage 0: double; 1: float deviations updated in float; 2: float deviations updated in double
template <class ST, int N>
static hipError_t launch_adj_storage(const AdjointArgs &a) {
  if (a.storage == 0) return launch_adj_t<ST, N, double, false>(a);
  if (a.storage == 1) return launch_adj_t<ST, N, float, true>(a);
  return launch_adj_t<ST, N, float, true, double>(a);
}

hipError_t launch_adjoint(const AdjointArgs &a) {
  if (a.stencil != ST_PROD2D) return hipErrorInvalidValue;
  if (a.order == 2) return launch_adj_storage<Stencil<ST_PROD2D, 3>, 2>(a);
  return launch_adj_storage<Stencil<ST_PROD2D, 4>, 3>(a);
}

}  // namespace rlbm
