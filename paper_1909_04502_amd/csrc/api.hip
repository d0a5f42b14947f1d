// api.hip -- the C ABI of include/rlbm.h: handles, validation and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/rlbm.h"
#include "kernels.h"
#include "precompute.h"

struct rlbm_lattice {
  rlbm_config cfg;
  rlbm::QuadHost quad;
  rlbm::Tables *d_tables = nullptr;
  int *d_err = nullptr;
  int stencil = 0;
  int variant = 1;
  int store_mode = RLBM_STORES_AUTO;
  int64_t sites = 0;
  std::string last_error;
  // launch graphs of recent multi-step rlbm_step calls (buffers, step count, variant), least
  // recently used replaced first
  struct StepGraph {
    hipGraphExec_t exec = nullptr;
    const void *fa = nullptr, *fb = nullptr;
    int n = -1, variant = -1, nt = -1;
    uint64_t used = 0;
  };
  static constexpr int kGraphs = 4;
  StepGraph graphs[kGraphs];
  uint64_t graph_clock = 0;
  hipStream_t cap_stream = nullptr;
};

constexpr int32_t kGraphMinSteps = 4;   // rlbm_step replays a cached graph from this many steps on
constexpr int32_t kGraphChunk = 256;    // and captures at most this many (even) steps in one graph

struct rlbm_batch {
  std::vector<rlbm_lattice *> lats;
  std::vector<int64_t> elem_off, site_off;
  int64_t total_elems = 0, total_sites = 0;
  rlbm::Tables *d_tabs = nullptr;
  int64_t *d_off = nullptr;
  int2 *d_tiles = nullptr;
  int ntiles = 0;
  int *d_err = nullptr;
  int stencil = 0, order = 0, storage = 0, elem = 8;
  int variant = 0;
  int store_mode = RLBM_STORES_AUTO;
  // cached launch graph of the last (f_a, f_b, nsteps, variant, store kind)
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  const void *g_fa = nullptr, *g_fb = nullptr;
  int g_n = -1, g_variant = -1, g_nt = -1;
};

namespace {

thread_local std::string g_last_error;

rlbm_status fail(rlbm_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

int stencil_of(const rlbm_model &m) {
  if (m.kind == RLBM_QUAD_UR_ONLATTICE) return m.d == 2 ? rlbm::ST_UR2D : rlbm::ST_UR3D;
  if (m.kind == RLBM_QUAD_MASSIVE_ONLATTICE) return m.d == 2 ? rlbm::ST_MASSIVE2D : rlbm::ST_MASSIVE3D;
  return m.d == 2 ? rlbm::ST_PROD2D : rlbm::ST_PROD3D;
}

rlbm::FieldPtrs field_ptrs(const rlbm_fields *f) {
  rlbm::FieldPtrs p = {nullptr, nullptr, nullptr, nullptr, 0};
  if (f) {
    p.n = f->n;
    p.eps = f->eps;
    p.T = f->T;
    p.U = f->U;
    p.any = (p.n || p.eps || p.T || p.U) ? 1 : 0;
  }
  return p;
}

// the lattice needs the force / wall build of the step kernel
int lattice_ext(const rlbm_lattice *h) {
  if (h->cfg.model.kind == RLBM_QUAD_UR_ONLATTICE) return 0;
  for (int a = 0; a < h->cfg.model.d; ++a) {
    if (h->cfg.bc[a] == RLBM_WALL) return 1;
    if (h->cfg.force[a] != 0.0 && h->cfg.model.zeta > 0.0) return 1;
  }
  return 0;
}

// Non-temporal population stores pay once the two state buffers are well beyond the 256 MiB
// last-level cache (just above it, much of the next step's input is still found there), and only
// when every row of sites starts on a 64-byte boundary: with ragged rows a wave's stores cover
// partial lines.  Measured on the step kernels: slower up to 281 MiB, 3-10 % faster from 405 MiB
// on with aligned rows, 3-14 % slower with ragged ones.
constexpr int64_t kNontemporalFootprint = 384ll << 20;
constexpr int64_t kNontemporalRowAlign = 64;

int uses_nontemporal(const rlbm_lattice *h) {
  if (h->store_mode != RLBM_STORES_AUTO) return h->store_mode == RLBM_STORES_NONTEMPORAL;
  const int64_t s = h->cfg.storage == RLBM_F64 ? 8 : 4;
  return 2 * s * h->quad.Q * h->sites > kNontemporalFootprint && (h->cfg.extent[0] * s) % kNontemporalRowAlign == 0;
}

rlbm::LaunchArgs base_args(const rlbm_lattice *h, hipStream_t stream) {
  rlbm::LaunchArgs a;
  a.stencil = h->stencil;
  a.order = h->cfg.model.order;
  a.storage = h->cfg.storage;
  a.nx = (int)h->cfg.extent[0];
  a.ny = (int)h->cfg.extent[1];
  a.nz = h->cfg.model.d == 3 ? (int)h->cfg.extent[2] : 1;
  a.tb = h->d_tables;
  a.tau_field = h->cfg.tau_field;
  a.err = h->d_err;
  a.stream = stream;
  a.variant = h->variant;
  a.ext = lattice_ext(h);
  a.nt = uses_nontemporal(h);
  // the staged windows are read in 16-byte chunks that wrap around x as a whole
  a.lds_ok = h->cfg.model.d == 2 && h->cfg.model.kind == RLBM_QUAD_PRODUCT && h->cfg.bc[0] == RLBM_PERIODIC &&
             h->cfg.extent[0] % 4 == 0;
  return a;
}

__global__ void k_fill(double *p, double v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Density 1 + amp (2 r - 1) with r in [0, 1) from a multiplicative hash of the site index: noise
// in every bit of every site's populations.
__global__ void k_noise_fill(double *n, double amp, int64_t sites) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= sites) return;
  const double r = (double)(((uint64_t)i * 0x9E3779B97F4A7C15ull) >> 11) * 0x1.0p-53;
  n[i] = 1.0 + amp * (2.0 * r - 1.0);
}

// Velocity field of a shear wave of amplitude amp: u_x(y), u_y(x) in 2D; u_x(y), u_y(z), u_z(x) in 3D,
// each amp sin(2 pi k / n_k) along its axis.  u holds d planes of `sites` doubles.
__global__ void k_shear_fill(double *u, int d, int nx, int ny, int nz, double amp, int64_t sites) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= sites) return;
  const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((int64_t)nx * ny));
  const double tp = 6.283185307179586;
  u[i] = amp * sin(tp * y / ny);
  if (d == 2) {
    u[sites + i] = amp * sin(tp * x / nx);
  } else {
    u[sites + i] = amp * sin(tp * z / nz);
    u[2 * sites + i] = amp * sin(tp * x / nx);
  }
}

}  // namespace

extern "C" {

const char *rlbm_status_string(rlbm_status s) {
  switch (s) {
    case RLBM_OK: return "ok";
    case RLBM_ERR_INVALID_ARG: return "invalid argument";
    case RLBM_ERR_UNSUPPORTED: return "unsupported";
    case RLBM_ERR_QUADRATURE: return "quadrature construction failed";
    case RLBM_ERR_DEVICE: return "HIP runtime error";
    case RLBM_ERR_NONPHYSICAL: return "non-physical state met by a kernel";
  }
  return "unknown status";
}

const char *rlbm_last_error(void) { return g_last_error.c_str(); }

rlbm_status rlbm_quadrature_build(const rlbm_model *model, int32_t *Q, double *p, double *w, double *disp) {
  if (!model || !Q) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  rlbm::QuadHost q;
  std::string err;
  int rc = rlbm::build_quadrature(model->d, model->zeta, model->order, model->kind, model->v0, q, err);
  if (rc) return fail((rlbm_status)rc, err);
  *Q = q.Q;
  if (p) std::memcpy(p, q.p.data(), q.p.size() * sizeof(double));
  if (w) std::memcpy(w, q.w.data(), q.w.size() * sizeof(double));
  if (disp) std::memcpy(disp, q.disp.data(), q.disp.size() * sizeof(double));
  return RLBM_OK;
}

rlbm_status rlbm_massive_window(const rlbm_model *model, double *lo, double *hi) {
  if (!model || !lo || !hi) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  if (model->kind != RLBM_QUAD_MASSIVE_ONLATTICE)
    return fail(RLBM_ERR_INVALID_ARG, "the window applies to massive on-lattice rules");
  if (!((model->d == 2 && (model->order == 2 || model->order == 3)) || (model->d == 3 && model->order == 3)))
    return fail(RLBM_ERR_UNSUPPORTED, "massive rules: d = 2 with N = 2, 3; d = 3 with N = 3");
  if (!(model->zeta > 0.0) || !std::isfinite(model->zeta)) return fail(RLBM_ERR_INVALID_ARG, "zeta must be > 0");
  std::string err;
  int rc = rlbm::massive_window(model->d, model->zeta, model->order, *lo, *hi, err);
  return rc ? fail((rlbm_status)rc, err) : RLBM_OK;
}

// Validates a configuration and fills the lattice description h and its host tables t (no
// device work; the caller owns both and frees them on failure).
static rlbm_status prepare_lattice(const rlbm_config *cfg, rlbm_lattice *h, rlbm::Tables *t) {
  const rlbm_model &m = cfg->model;
  if (m.d != 2 && m.d != 3) return fail(RLBM_ERR_UNSUPPORTED, "d must be 2 or 3");
  for (int a = 0; a < m.d; ++a) {
    if (cfg->extent[a] < 1 || cfg->extent[a] > (1 << 20)) return fail(RLBM_ERR_INVALID_ARG, "extent out of range");
    if (cfg->bc[a] != RLBM_PERIODIC && cfg->bc[a] != RLBM_OPEN && cfg->bc[a] != RLBM_WALL)
      return fail(RLBM_ERR_INVALID_ARG, "bad bc");
    if (cfg->bc[a] == RLBM_WALL && m.kind == RLBM_QUAD_UR_ONLATTICE)
      return fail(RLBM_ERR_UNSUPPORTED, "walls are built for the product and massive rules");
    if (cfg->bc[a] == RLBM_WALL && m.kind == RLBM_QUAD_MASSIVE_ONLATTICE && m.d == 3 && cfg->storage == RLBM_F64)
      return fail(RLBM_ERR_UNSUPPORTED, "walls: the streaming kernel of the 3D massive rule has none");
    for (int e = 0; e < 2; ++e) {
      if (!(cfg->wall_T[a][e] >= 0.0) || !std::isfinite(cfg->wall_T[a][e]))
        return fail(RLBM_ERR_INVALID_ARG, "wall temperatures must be finite and >= 0");
      if (cfg->wall_T[a][e] != 0.0 && cfg->bc[a] != RLBM_WALL)
        return fail(RLBM_ERR_INVALID_ARG, "a wall temperature needs a wall axis");
    }
    if (!std::isfinite(cfg->force[a])) return fail(RLBM_ERR_INVALID_ARG, "force must be finite");
  }
  if (!std::isfinite(cfg->tau_T)) return fail(RLBM_ERR_INVALID_ARG, "tau_T must be finite");
  if (cfg->tau_T != 0.0 && m.kind == RLBM_QUAD_PRODUCT)
    return fail(RLBM_ERR_UNSUPPORTED, "the temperature-dependent tau is built for the on-lattice rules");
  if (m.kind == RLBM_QUAD_MASSIVE_ONLATTICE && m.d == 3 && cfg->storage == RLBM_F64 &&
      (cfg->force[0] != 0.0 || cfg->force[1] != 0.0 || cfg->force[2] != 0.0))
    return fail(RLBM_ERR_UNSUPPORTED, "external force: the streaming kernel of the 3D massive rule has none");
  if (cfg->storage != RLBM_F64 && cfg->storage != RLBM_F32_DEV && cfg->storage != RLBM_F32_DEV_F64)
    return fail(RLBM_ERR_INVALID_ARG, "bad storage");
  if (cfg->storage == RLBM_F32_DEV_F64 && m.kind != RLBM_QUAD_PRODUCT)
    return fail(RLBM_ERR_UNSUPPORTED, "float storage with double arithmetic is built for the product rules");
  if (!(cfg->tau > 0.0) || !std::isfinite(cfg->tau)) return fail(RLBM_ERR_INVALID_ARG, "tau must be > 0");
  if (cfg->storage != RLBM_F64 && !(cfg->n_ref > 0.0)) return fail(RLBM_ERR_INVALID_ARG, "n_ref must be > 0");
  const int64_t nz = m.d == 3 ? cfg->extent[2] : 1;
  const int64_t sites = cfg->extent[0] * cfg->extent[1] * nz;
  if (m.d == 3 && nz > 65535) return fail(RLBM_ERR_UNSUPPORTED, "nz > 65535");
  // kernels address a population plane with 32-bit byte offsets
  if (sites * (cfg->storage == RLBM_F64 ? 8 : 4) >= (int64_t(1) << 32))
    return fail(RLBM_ERR_UNSUPPORTED, "a population plane must stay below 4 GiB");

  h->cfg = *cfg;
  h->stencil = stencil_of(m);
  // default launch shapes (from sweeps of every variant on MI355X):
  //  * 3D product rules: 64 x 4 tiles in (y, z) patches per XCD (half the re-reads from beyond
  //    the L2 of the untiled order: 1.19x the algorithmic bytes instead of 2.35x) with the
  //    unconstrained build, in float storage (4.39 ms at 256^3 in float arithmetic, 4.56 with
  //    the occupancy-2 build; 6.67 ms in double arithmetic, whose occupancy-2 build spills); in
  //    double storage the unconstrained build (468 registers, one wave per SIMD) in untiled
  //    64 x 4 tiles (10.5 ms, 10.7 in patches);
  //  * the 3D massive rule: 64 x 2 XCD-ordered tiles (double, streaming kernel) or 64 x 1 patches
  //    (float);
  //  * 2D product rules in double: rows of 64 sites; float storage with double arithmetic: 64 x 4
  //    band tiles of the occupancy-2 build (4 % faster than rows of 64); float storage and
  //    arithmetic: 64 x 4 band tiles of the occupancy-4 build (0.057 against 0.060 ms at 1024^2 for
  //    the unconstrained one); in every storage the LDS-staged kernel on lattices larger than the
  //    caches (below);
  //  * 2D on-lattice rules: 64 x 4 tiles of the occupancy-2 build, except the massive rules whose
  //    update fits in 128 registers (order 2, and order 3 in float deviations), which take the
  //    occupancy-4 build: four waves per SIMD instead of three, 7-27 % faster; and small lattices
  //    of the massless rules (at most 65,536 sites, such as 64 x 64), which take rows of 64 sites
  //    so that four times as many blocks spread over the CUs (about 9 % faster at 64 x 64)
  if (m.d == 3 && m.kind == RLBM_QUAD_MASSIVE_ONLATTICE) h->variant = cfg->storage == RLBM_F64 ? 4 : 8;
  else if (m.d == 3 && m.kind == RLBM_QUAD_UR_ONLATTICE) h->variant = 4;   // streaming kernel, as the 3D massive rule
  else if (m.d == 3) h->variant = cfg->storage == RLBM_F64 ? 0 : 11;
  else if (m.kind == RLBM_QUAD_PRODUCT && cfg->storage == RLBM_F64) h->variant = 5;
  else if (m.kind == RLBM_QUAD_PRODUCT && cfg->storage == RLBM_F32_DEV) h->variant = 10;
  else if (m.kind == RLBM_QUAD_PRODUCT && cfg->storage == RLBM_F32_DEV_F64) h->variant = 9;
  else if (m.kind == RLBM_QUAD_MASSIVE_ONLATTICE && (m.order == 2 || cfg->storage != RLBM_F64)) h->variant = 10;
  else if (m.kind == RLBM_QUAD_UR_ONLATTICE && sites <= 65536) h->variant = 5;
  else if (m.kind != RLBM_QUAD_PRODUCT) h->variant = 3;
  h->sites = sites;
  std::string err;
  int rc = rlbm::build_quadrature(m.d, m.zeta, m.order, m.kind, m.v0, h->quad, err);
  if (rc) return fail((rlbm_status)rc, err);
  // integer streaming reads x - n_i with one periodic wrap: a periodic axis must be at least as
  // long as the longest displacement along it
  for (int i = 0; i < h->quad.Q; ++i)
    for (int a = 0; a < m.d; ++a)
      if (cfg->bc[a] == RLBM_PERIODIC && std::fabs(h->quad.disp[i * m.d + a]) > (double)cfg->extent[a])
        return fail(RLBM_ERR_INVALID_ARG, "a periodic extent is shorter than the stencil's longest displacement");
  // 2D product rules whose state outgrows the caches (the non-temporal store threshold) take the
  // LDS-staged kernel where it applies, in every storage (double at 1024^2: 0.106 against 0.122 ms
  // per step for rows of 64 sites; at 2048^2 float storage 0.221 against 0.256 ms, float storage
  // with double arithmetic 0.255 against 0.266 ms); below that, where the halo re-reads hit the
  // Infinity Cache, the register kernels stay ahead (float storage at 1024^2: 0.057 against 0.059)
  const int64_t elem = cfg->storage == RLBM_F64 ? 8 : 4;
  if (m.d == 2 && m.kind == RLBM_QUAD_PRODUCT && cfg->bc[0] == RLBM_PERIODIC && cfg->extent[0] % 4 == 0 &&
      2 * elem * (int64_t)h->quad.Q * sites > kNontemporalFootprint)
    h->variant = 12;
  int bc[3] = {cfg->bc[0], cfg->bc[1], cfg->bc[2]};
  rc = rlbm::build_tables(h->quad, cfg->tau, cfg->storage != RLBM_F64 ? cfg->n_ref : 1.0, cfg->storage,
                          cfg->extent, bc, *t, err);
  if (!rc && m.d == 3) rc = rlbm::build_eos_fit(m.zeta, *t, err);
  if (!rc) {
    for (int a = 0; a < 3; ++a) {
      t->g[a] = a < m.d ? cfg->force[a] : 0.0;
      t->gf[a] = (float)t->g[a];
    }
    t->tau_T = cfg->tau_T;
    for (int a = 0; a < 3; ++a)
      for (int e = 0; e < 2; ++e) t->wallT[a][e] = a < m.d ? cfg->wall_T[a][e] : 0.0;
    // the force term carries the mass: nothing to add for zeta = 0
    t->has_force = (m.zeta > 0.0 && m.kind != RLBM_QUAD_UR_ONLATTICE &&
                    (t->g[0] != 0.0 || t->g[1] != 0.0 || t->g[2] != 0.0)) ? 1 : 0;
  }
  if (rc) return fail((rlbm_status)rc, err);
  return RLBM_OK;
}

rlbm_status rlbm_create(const rlbm_config *cfg, rlbm_lattice **out) {
  if (!cfg || !out) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  rlbm_lattice *h = new (std::nothrow) rlbm_lattice();
  rlbm::Tables *t = new (std::nothrow) rlbm::Tables;
  if (!h || !t) {
    delete h;
    delete t;
    return fail(RLBM_ERR_DEVICE, "out of host memory");
  }
  const rlbm_status st = prepare_lattice(cfg, h, t);
  if (st != RLBM_OK) {
    delete t;
    delete h;
    return st;
  }
  hipError_t he = hipMalloc(&h->d_tables, sizeof(rlbm::Tables));
  if (he == hipSuccess) he = hipMalloc(&h->d_err, sizeof(int));
  if (he == hipSuccess) he = hipMemcpy(h->d_tables, t, sizeof(rlbm::Tables), hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMemset(h->d_err, 0, sizeof(int));
  if (he == hipSuccess) he = hipDeviceSynchronize();
  delete t;
  if (he != hipSuccess) {
    rlbm_destroy(h);
    return fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
  }
  *out = h;
  return RLBM_OK;
}

rlbm_status rlbm_destroy(rlbm_lattice *h) {
  if (!h) return RLBM_OK;
  for (auto &g : h->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->d_tables) (void)hipFree(h->d_tables);
  if (h->d_err) (void)hipFree(h->d_err);
  delete h;
  return RLBM_OK;
}

rlbm_status rlbm_get_info(const rlbm_lattice *h, rlbm_info *info) {
  if (!h || !info) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  info->Q = h->quad.Q;
  info->n_basis = rlbm::basis_size(h->cfg.model.d, h->cfg.model.order);
  info->sites = h->sites;
  info->elem_bytes = h->cfg.storage == RLBM_F64 ? 8 : 4;
  info->state_bytes = (int64_t)info->elem_bytes * h->quad.Q * h->sites;
  info->on_lattice = h->cfg.model.kind != RLBM_QUAD_PRODUCT;
  info->v0 = h->quad.v0;
  return RLBM_OK;
}

rlbm_status rlbm_init(rlbm_lattice *h, const double *n0, const double *T0, const double *u0, const double *noise,
                      double noise_amp, void *f_out, const rlbm_fields *fields0, hipStream_t stream) {
  if (!h || !n0 || !T0 || !u0 || !f_out) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  if (!std::isfinite(noise_amp)) return fail(RLBM_ERR_INVALID_ARG, "noise_amp must be finite");
  rlbm::LaunchArgs a = base_args(h, stream);
  a.op = rlbm::OP_INIT;
  a.n0 = n0;
  a.T0 = T0;
  a.u0 = u0;
  a.noise = noise;
  a.amp = noise_amp;
  a.fout = f_out;
  a.fields = field_ptrs(fields0);
  hipError_t he = rlbm::launch(a);
  return he == hipSuccess ? RLBM_OK : fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
}

// nsteps step launches alternating between f_a and f_b (a: the lattice's launch arguments)
static hipError_t launch_steps(rlbm::LaunchArgs a, void *f_a, void *f_b, int32_t nsteps, const rlbm_fields *last) {
  a.op = rlbm::OP_STEP;
  for (int32_t s = 0; s < nsteps; ++s) {
    a.fin = (s & 1) ? f_b : f_a;
    a.fout = (s & 1) ? f_a : f_b;
    a.fields = field_ptrs(s == nsteps - 1 ? last : nullptr);
    const hipError_t he = rlbm::launch(a);
    if (he != hipSuccess) return he;
  }
  return hipSuccess;
}

static hipError_t step_launches(rlbm_lattice *h, void *f_a, void *f_b, int32_t nsteps, const rlbm_fields *last,
                                hipStream_t stream) {
  return launch_steps(base_args(h, stream), f_a, f_b, nsteps, last);
}

rlbm_status rlbm_step(rlbm_lattice *h, void *f_a, void *f_b, int32_t nsteps, const rlbm_fields *last,
                      hipStream_t stream) {
  if (!h || !f_a || !f_b || nsteps < 0) return fail(RLBM_ERR_INVALID_ARG, "bad argument");
  const int64_t bytes = (int64_t)(h->cfg.storage == RLBM_F64 ? 8 : 4) * h->quad.Q * h->sites;
  const char *pa = (const char *)f_a, *pb = (const char *)f_b;
  if (pa < pb + bytes && pb < pa + bytes) return fail(RLBM_ERR_INVALID_ARG, "f_a and f_b overlap");
  if (nsteps > kGraphChunk) {
    // long runs replay one cached graph of an even number of steps (the state returns to f_a after
    // each replay) instead of capturing every launch of the run into one graph; the last 1 ..
    // kGraphChunk steps (and the fields of the final one) follow as an ordinary call
    int32_t rest = nsteps;
    for (; rest > kGraphChunk; rest -= kGraphChunk) {
      const rlbm_status st = rlbm_step(h, f_a, f_b, kGraphChunk, nullptr, stream);
      if (st != RLBM_OK) return st;
    }
    return rlbm_step(h, f_a, f_b, rest, last, stream);
  }
  if (nsteps >= kGraphMinSteps && last == nullptr) {
    // many steps without field output: a cached HIP graph of the launches (no per-launch host cost)
    hipError_t he = hipSuccess;
    rlbm_lattice::StepGraph *sg = nullptr;
    for (auto &g : h->graphs)
      if (g.exec && g.fa == f_a && g.fb == f_b && g.n == nsteps && g.variant == h->variant &&
          g.nt == uses_nontemporal(h))
        sg = &g;
    if (!sg) {
      sg = &h->graphs[0];
      for (auto &g : h->graphs)
        if (g.used < sg->used) sg = &g;
      if (sg->exec) (void)hipGraphExecDestroy(sg->exec);
      *sg = rlbm_lattice::StepGraph{};
      if (!h->cap_stream) he = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
      hipGraph_t g = nullptr;
      if (he == hipSuccess) he = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
      if (he == hipSuccess) {
        const hipError_t he2 = step_launches(h, f_a, f_b, nsteps, nullptr, h->cap_stream);
        he = hipStreamEndCapture(h->cap_stream, &g);
        if (he == hipSuccess) he = he2;
      }
      if (he == hipSuccess) he = hipGraphInstantiate(&sg->exec, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (he == hipSuccess) {
        sg->fa = f_a;
        sg->fb = f_b;
        sg->n = nsteps;
        sg->variant = h->variant;
        sg->nt = uses_nontemporal(h);
      } else {
        sg->exec = nullptr;
      }
    }
    if (he == hipSuccess) {
      sg->used = ++h->graph_clock;
      he = hipGraphLaunch(sg->exec, stream);
    }
    return he == hipSuccess ? RLBM_OK : fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
  }
  const hipError_t he = step_launches(h, f_a, f_b, nsteps, last, stream);
  return he == hipSuccess ? RLBM_OK : fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
}

rlbm_status rlbm_moments(rlbm_lattice *h, const void *f, const rlbm_fields *out, hipStream_t stream) {
  if (!h || !f || !out) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  rlbm::LaunchArgs a = base_args(h, stream);
  a.op = rlbm::OP_MOMENTS;
  a.fin = f;
  a.fields = field_ptrs(out);
  hipError_t he = rlbm::launch(a);
  return he == hipSuccess ? RLBM_OK : fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
}

rlbm_status rlbm_sync(rlbm_lattice *h, hipStream_t stream) {
  if (!h) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  hipError_t he = hipStreamSynchronize(stream);
  if (he != hipSuccess) return fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
  int flag = 0;
  he = hipMemcpy(&flag, h->d_err, sizeof(int), hipMemcpyDeviceToHost);
  if (he != hipSuccess) return fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
  if (flag) {
    int zero = 0;
    (void)hipMemcpy(h->d_err, &zero, sizeof(int), hipMemcpyHostToDevice);
    return fail(RLBM_ERR_NONPHYSICAL, "a kernel met a non-physical state");
  }
  return RLBM_OK;
}

static rlbm_status adjoint_supported(const rlbm_lattice *h) {
  if (h->stencil != rlbm::ST_PROD2D)
    return fail(RLBM_ERR_UNSUPPORTED, "reverse mode is implemented for the 2D product rules");
  for (int a = 0; a < 2; ++a)
    if (h->cfg.bc[a] != RLBM_PERIODIC) return fail(RLBM_ERR_UNSUPPORTED, "reverse mode needs periodic boundaries");
  for (int a = 0; a < h->cfg.model.d; ++a)
    if (h->cfg.force[a] != 0.0 && h->cfg.model.zeta > 0.0)
      return fail(RLBM_ERR_UNSUPPORTED, "reverse mode has no force term");
  return RLBM_OK;
}

static rlbm::AdjointArgs adj_args(const rlbm_lattice *h, hipStream_t stream) {
  rlbm::AdjointArgs a;
  a.stencil = h->stencil;
  a.order = h->cfg.model.order;
  a.storage = h->cfg.storage;
  a.nx = (int)h->cfg.extent[0];
  a.ny = (int)h->cfg.extent[1];
  a.nz = 1;
  a.tb = h->d_tables;
  a.tau_field = h->cfg.tau_field;
  a.err = h->d_err;
  a.stream = stream;
  return a;
}

rlbm_status rlbm_adjoint_step(rlbm_lattice *h, const void *f_prev, const void *lam_next, void *lam,
                              double *dtau_accum, hipStream_t stream) {
  if (!h || !f_prev || !lam_next || !lam) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  if (lam == lam_next || lam == f_prev) return fail(RLBM_ERR_INVALID_ARG, "lam must not alias its inputs");
  rlbm_status st = adjoint_supported(h);
  if (st != RLBM_OK) return st;
  rlbm::AdjointArgs a = adj_args(h, stream);
  a.op = rlbm::ADJ_STEP;
  a.state = f_prev;
  a.lam_in = lam_next;
  a.lam_out = lam;
  a.dtau = dtau_accum;
  hipError_t he = rlbm::launch_adjoint(a);
  return he == hipSuccess ? RLBM_OK : fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
}

rlbm_status rlbm_moments_vjp(rlbm_lattice *h, const void *f, const rlbm_fields *grad, void *lam,
                             hipStream_t stream) {
  if (!h || !f || !grad || !lam) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  rlbm_status st = adjoint_supported(h);
  if (st != RLBM_OK) return st;
  rlbm::AdjointArgs a = adj_args(h, stream);
  a.op = rlbm::ADJ_MOMENTS;
  a.state = f;
  a.lam_out = lam;
  a.grads = field_ptrs(grad);
  hipError_t he = rlbm::launch_adjoint(a);
  return he == hipSuccess ? RLBM_OK : fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
}

rlbm_status rlbm_init_vjp(rlbm_lattice *h, const double *n0, const double *T0, const double *u0,
                          const double *noise, double noise_amp, const void *lam1, double *du0, double *dn0,
                          double *dT0, double *dtau_accum, hipStream_t stream) {
  if (!h || !n0 || !T0 || !u0 || !lam1) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  rlbm_status st = adjoint_supported(h);
  if (st != RLBM_OK) return st;
  rlbm::AdjointArgs a = adj_args(h, stream);
  a.op = rlbm::ADJ_INIT;
  a.n0 = n0;
  a.T0 = T0;
  a.u0 = u0;
  a.noise = noise;
  a.amp = noise_amp;
  a.lam_in = lam1;
  a.du0 = du0;
  a.dn0 = dn0;
  a.dT0 = dT0;
  a.dtau = dtau_accum;
  hipError_t he = rlbm::launch_adjoint(a);
  return he == hipSuccess ? RLBM_OK : fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
}

int32_t rlbm_variant_count(void) { return rlbm::kNumVariants; }

// ------------------------------------------------------------------ batches
static const int kBatchGrid[3] = {512, 1024, 2048};
static const int kNumBatchVariants = 12;   // 4 tile shapes x 3 grid sizes

static hipError_t batch_build_tiles(rlbm_batch *b) {
  const int tv = b->variant % 4;
  const int bx = rlbm::kBatchTiles[tv][0], by = rlbm::kBatchTiles[tv][1];
  std::vector<int2> tl;
  for (size_t l = 0; l < b->lats.size(); ++l) {
    const int64_t nx = b->lats[l]->cfg.extent[0], ny = b->lats[l]->cfg.extent[1];
    const int64_t n = tv == rlbm::kBatchLinearTile ? (nx * ny + bx - 1) / bx : ((nx + bx - 1) / bx) * ((ny + by - 1) / by);
    for (int64_t t = 0; t < n; ++t) tl.push_back(make_int2((int)l, (int)t));
  }
  // the cached graph's kernel arguments name the old tile list: drop it before that list is freed
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  b->gexec = nullptr;
  b->g_fa = b->g_fb = nullptr;
  b->g_n = b->g_variant = b->g_nt = -1;
  if (b->d_tiles) (void)hipFree(b->d_tiles);
  b->d_tiles = nullptr;
  b->ntiles = (int)tl.size();
  hipError_t he = hipMalloc(&b->d_tiles, sizeof(int2) * tl.size());
  if (he == hipSuccess) he = hipMemcpy(b->d_tiles, tl.data(), sizeof(int2) * tl.size(), hipMemcpyHostToDevice);
  return he;
}

rlbm_status rlbm_batch_destroy(rlbm_batch *b) {
  if (!b) return RLBM_OK;
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (auto *h : b->lats) rlbm_destroy(h);
  if (b->d_tabs) (void)hipFree(b->d_tabs);
  if (b->d_off) (void)hipFree(b->d_off);
  if (b->d_tiles) (void)hipFree(b->d_tiles);
  if (b->d_err) (void)hipFree(b->d_err);
  delete b;
  return RLBM_OK;
}

rlbm_status rlbm_batch_create(const rlbm_config *cfgs, int32_t nlat, rlbm_batch **out) {
  if (!cfgs || !out || nlat < 1) return fail(RLBM_ERR_INVALID_ARG, "bad argument");
  *out = nullptr;
  for (int l = 0; l < nlat; ++l) {
    const rlbm_config &c = cfgs[l];
    if (c.model.d != 2 || c.model.kind != RLBM_QUAD_PRODUCT || c.model.order != cfgs[0].model.order ||
        c.storage != cfgs[0].storage)
      return fail(RLBM_ERR_UNSUPPORTED, "a batch holds 2D product-rule lattices of one order and storage");
    if (c.tau_field != nullptr) return fail(RLBM_ERR_UNSUPPORTED, "batched lattices take a scalar tau");
  }
  rlbm_batch *b = new (std::nothrow) rlbm_batch();
  if (!b) return fail(RLBM_ERR_DEVICE, "out of host memory");
  b->stencil = rlbm::ST_PROD2D;
  b->order = cfgs[0].model.order;
  b->storage = cfgs[0].storage;
  b->elem = b->storage == RLBM_F64 ? 8 : 4;
  // default launch: runs of 256 consecutive sites (no lane idles past a row's end: 5-6 % faster
  // than 64 x 4 tiles on 256 lattices of sides 64..512), the 2048-block grid in double and the
  // 512-block grid in float
  b->variant = b->storage == RLBM_F64 ? 2 * 4 + rlbm::kBatchLinearTile : rlbm::kBatchLinearTile;
  for (int l = 0; l < nlat; ++l) {
    rlbm_lattice *h = nullptr;
    rlbm_status st = rlbm_create(&cfgs[l], &h);
    if (st != RLBM_OK) {
      rlbm_batch_destroy(b);
      return st;
    }
    b->lats.push_back(h);
    b->elem_off.push_back(b->total_elems);
    b->site_off.push_back(b->total_sites);
    b->total_elems += (int64_t)h->quad.Q * h->sites;
    b->total_sites += h->sites;
  }
  hipError_t he = hipMalloc(&b->d_tabs, sizeof(rlbm::Tables) * nlat);
  for (int l = 0; he == hipSuccess && l < nlat; ++l)
    he = hipMemcpy(b->d_tabs + l, b->lats[l]->d_tables, sizeof(rlbm::Tables), hipMemcpyDeviceToDevice);
  if (he == hipSuccess) he = hipMalloc(&b->d_off, sizeof(int64_t) * nlat);
  if (he == hipSuccess)
    he = hipMemcpy(b->d_off, b->elem_off.data(), sizeof(int64_t) * nlat, hipMemcpyHostToDevice);
  if (he == hipSuccess) he = hipMalloc(&b->d_err, sizeof(int));
  if (he == hipSuccess) he = hipMemset(b->d_err, 0, sizeof(int));
  if (he == hipSuccess) he = batch_build_tiles(b);
  if (he == hipSuccess) he = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
  if (he == hipSuccess) he = hipDeviceSynchronize();
  if (he != hipSuccess) {
    rlbm_batch_destroy(b);
    return fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
  }
  *out = b;
  return RLBM_OK;
}

rlbm_status rlbm_batch_layout(const rlbm_batch *b, int64_t *total_elems, int64_t *total_sites, int64_t *elem_off,
                              int64_t *site_off) {
  if (!b) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  if (total_elems) *total_elems = b->total_elems;
  if (total_sites) *total_sites = b->total_sites;
  for (size_t l = 0; l < b->lats.size(); ++l) {
    if (elem_off) elem_off[l] = b->elem_off[l];
    if (site_off) site_off[l] = b->site_off[l];
  }
  return RLBM_OK;
}

rlbm_status rlbm_batch_lattice(const rlbm_batch *b, int32_t l, rlbm_lattice **h) {
  if (!b || !h || l < 0 || l >= (int32_t)b->lats.size()) return fail(RLBM_ERR_INVALID_ARG, "bad argument");
  *h = b->lats[l];
  return RLBM_OK;
}

rlbm_status rlbm_batch_init(rlbm_batch *b, const double *n0, const double *T0, const double *u0, void *f_out,
                            hipStream_t stream) {
  if (!b || !n0 || !T0 || !u0 || !f_out) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  for (size_t l = 0; l < b->lats.size(); ++l) {
    const int64_t so = b->site_off[l];
    rlbm_status st = rlbm_init(b->lats[l], n0 + so, T0 + so, u0 + 2 * so, nullptr, 0.0,
                               (char *)f_out + b->elem_off[l] * b->elem, nullptr, stream);
    if (st != RLBM_OK) return st;
  }
  return RLBM_OK;
}

rlbm_status rlbm_batch_moments(rlbm_batch *b, const void *f, const rlbm_fields *out, hipStream_t stream) {
  if (!b || !f || !out) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  for (size_t l = 0; l < b->lats.size(); ++l) {
    const int64_t so = b->site_off[l];
    rlbm_fields o;
    o.n = out->n ? out->n + so : nullptr;
    o.eps = out->eps ? out->eps + so : nullptr;
    o.T = out->T ? out->T + so : nullptr;
    o.U = out->U ? out->U + 3 * so : nullptr;
    rlbm_status st = rlbm_moments(b->lats[l], (const char *)f + b->elem_off[l] * b->elem, &o, stream);
    if (st != RLBM_OK) return st;
  }
  return RLBM_OK;
}

static int batch_nontemporal(const rlbm_batch *b) {
  if (b->store_mode != RLBM_STORES_AUTO) return b->store_mode == RLBM_STORES_NONTEMPORAL;
  for (auto *h : b->lats)
    if ((h->cfg.extent[0] * b->elem) % kNontemporalRowAlign != 0) return 0;
  return 2 * b->total_elems * b->elem > kNontemporalFootprint;
}

static hipError_t batch_enqueue(rlbm_batch *b, void *f_a, void *f_b, int32_t nsteps, hipStream_t stream) {
  rlbm::BatchArgs a;
  a.stencil = b->stencil;
  a.order = b->order;
  a.storage = b->storage;
  a.tile = b->variant % 4;
  a.blocks = kBatchGrid[b->variant / 4];
  a.tabs = b->d_tabs;
  a.elem_off = b->d_off;
  a.tiles = b->d_tiles;
  a.ntiles = b->ntiles;
  a.err = b->d_err;
  a.stream = stream;
  a.ext = 0;
  for (auto *h : b->lats) a.ext |= lattice_ext(h);
  a.nt = batch_nontemporal(b);
  for (int32_t s = 0; s < nsteps; ++s) {
    a.fin = (s & 1) ? f_b : f_a;
    a.fout = (s & 1) ? f_a : f_b;
    hipError_t he = rlbm::launch_batch(a);
    if (he != hipSuccess) return he;
  }
  return hipSuccess;
}

rlbm_status rlbm_batch_step(rlbm_batch *b, void *f_a, void *f_b, int32_t nsteps, int32_t use_graph,
                            hipStream_t stream) {
  if (!b || !f_a || !f_b || nsteps < 0) return fail(RLBM_ERR_INVALID_ARG, "bad argument");
  const int64_t bytes = b->total_elems * b->elem;
  const char *pa = (const char *)f_a, *pb = (const char *)f_b;
  if (pa < pb + bytes && pb < pa + bytes) return fail(RLBM_ERR_INVALID_ARG, "f_a and f_b overlap");
  if (nsteps == 0) return RLBM_OK;
  if (use_graph && nsteps > kGraphChunk) {   // as rlbm_step: replays of one even-length graph
    int32_t rest = nsteps;
    for (; rest > kGraphChunk; rest -= kGraphChunk) {
      const rlbm_status st = rlbm_batch_step(b, f_a, f_b, kGraphChunk, 1, stream);
      if (st != RLBM_OK) return st;
    }
    // the batch caches one graph: the remainder runs eagerly rather than replace the chunk's graph
    return rlbm_batch_step(b, f_a, f_b, rest, rest == kGraphChunk ? 1 : 0, stream);
  }
  hipError_t he = hipSuccess;
  if (!use_graph) {
    he = batch_enqueue(b, f_a, f_b, nsteps, stream);
  } else {
    if (!(b->gexec && b->g_fa == f_a && b->g_fb == f_b && b->g_n == nsteps && b->g_variant == b->variant &&
          b->g_nt == batch_nontemporal(b))) {
      if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
      b->gexec = nullptr;
      hipGraph_t g = nullptr;
      he = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
      if (he == hipSuccess) {
        hipError_t he2 = batch_enqueue(b, f_a, f_b, nsteps, b->cap_stream);
        he = hipStreamEndCapture(b->cap_stream, &g);
        if (he == hipSuccess) he = he2;
      }
      if (he == hipSuccess) he = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (he == hipSuccess) {
        b->g_fa = f_a;
        b->g_fb = f_b;
        b->g_n = nsteps;
        b->g_variant = b->variant;
        b->g_nt = batch_nontemporal(b);
      }
    }
    if (he == hipSuccess) he = hipGraphLaunch(b->gexec, stream);
  }
  return he == hipSuccess ? RLBM_OK : fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
}

rlbm_status rlbm_batch_sync(rlbm_batch *b, hipStream_t stream) {
  if (!b) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  hipError_t he = hipStreamSynchronize(stream);
  if (he != hipSuccess) return fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
  int flag = 0;
  he = hipMemcpy(&flag, b->d_err, sizeof(int), hipMemcpyDeviceToHost);
  if (he != hipSuccess) return fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
  rlbm_status st = RLBM_OK;
  for (auto *h : b->lats) {
    rlbm_status s2 = rlbm_sync(h, stream);
    if (s2 != RLBM_OK) st = s2;
  }
  if (flag) {
    int zero = 0;
    (void)hipMemcpy(b->d_err, &zero, sizeof(int), hipMemcpyHostToDevice);
    return fail(RLBM_ERR_NONPHYSICAL, "a kernel met a non-physical state");
  }
  return st;
}

int32_t rlbm_batch_variant_count(void) { return kNumBatchVariants; }

rlbm_status rlbm_batch_set_variant(rlbm_batch *b, int32_t v) {
  if (!b || v < 0 || v >= kNumBatchVariants) return fail(RLBM_ERR_INVALID_ARG, "bad variant");
  const int old_tile = b->variant % 4;
  b->variant = v;
  if (v % 4 != old_tile) {
    hipError_t he = batch_build_tiles(b);
    if (he != hipSuccess) return fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
  }
  return RLBM_OK;
}

rlbm_status rlbm_batch_get_variant(const rlbm_batch *b, int32_t *v) {
  if (!b || !v) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  *v = b->variant;
  return RLBM_OK;
}

rlbm_status rlbm_batch_set_store_mode(rlbm_batch *b, int32_t mode) {
  if (!b || mode < RLBM_STORES_AUTO || mode > RLBM_STORES_NONTEMPORAL) return fail(RLBM_ERR_INVALID_ARG, "bad store mode");
  b->store_mode = mode;
  return RLBM_OK;
}

rlbm_status rlbm_batch_get_store_mode(const rlbm_batch *b, int32_t *mode, int32_t *nontemporal) {
  if (!b || !mode) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  *mode = b->store_mode;
  if (nontemporal) *nontemporal = batch_nontemporal(b);
  return RLBM_OK;
}

rlbm_status rlbm_batch_autotune(rlbm_batch *b, void *f_a, void *f_b, int32_t steps, float *ms_out,
                                hipStream_t stream) {
  // Times every variant on the caller's buffers: f_a must hold a valid state; f_a and f_b are
  // overwritten by an even number of steps per variant (the result stays in f_a).
  if (!b || !f_a || !f_b || steps < 1) return fail(RLBM_ERR_INVALID_ARG, "bad argument");
  const int ev = 2 * ((steps + 1) / 2);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  float best = 1e30f;
  int best_v = b->variant;
  for (int v = 0; he == hipSuccess && v < kNumBatchVariants; ++v) {
    if (rlbm_batch_set_variant(b, v) != RLBM_OK) {
      he = hipErrorUnknown;
      break;
    }
    he = batch_enqueue(b, f_a, f_b, 2, stream);
    if (he == hipSuccess) he = hipEventRecord(e0, stream);
    if (he == hipSuccess) he = batch_enqueue(b, f_a, f_b, ev, stream);
    if (he == hipSuccess) he = hipEventRecord(e1, stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    ms /= ev;
    if (ms_out) ms_out[v] = ms;
    if (he == hipSuccess && ms < best) {
      best = ms;
      best_v = v;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (he != hipSuccess) return fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
  rlbm_status st = rlbm_batch_set_variant(b, best_v);
  if (st != RLBM_OK) return st;
  return rlbm_batch_sync(b, stream);
}

rlbm_status rlbm_set_variant(rlbm_lattice *h, int32_t v) {
  if (!h || v < 0 || v >= rlbm::kNumVariants) return fail(RLBM_ERR_INVALID_ARG, "bad variant");
  h->variant = v;
  return RLBM_OK;
}

rlbm_status rlbm_get_variant(const rlbm_lattice *h, int32_t *v) {
  if (!h || !v) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  *v = h->variant;
  return RLBM_OK;
}

rlbm_status rlbm_set_store_mode(rlbm_lattice *h, int32_t mode) {
  if (!h || mode < RLBM_STORES_AUTO || mode > RLBM_STORES_NONTEMPORAL) return fail(RLBM_ERR_INVALID_ARG, "bad store mode");
  h->store_mode = mode;
  return RLBM_OK;
}

rlbm_status rlbm_get_store_mode(const rlbm_lattice *h, int32_t *mode, int32_t *nontemporal) {
  if (!h || !mode) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  *mode = h->store_mode;
  if (nontemporal) *nontemporal = uses_nontemporal(h);
  return RLBM_OK;
}

rlbm_status rlbm_autotune(rlbm_lattice *h, int32_t steps, float *ms_out, hipStream_t stream) {
  if (!h || steps < 1) return fail(RLBM_ERR_INVALID_ARG, "bad argument");
  const int d = h->cfg.model.d;
  const int64_t bytes = (int64_t)(h->cfg.storage == RLBM_F64 ? 8 : 4) * h->quad.Q * h->sites;
  void *fa = nullptr, *fb = nullptr;
  double *fields = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipMalloc(&fa, bytes);
  if (he == hipSuccess) he = hipMalloc(&fb, bytes);
  if (he == hipSuccess) he = hipMalloc(&fields, sizeof(double) * h->sites * (d + 2));
  if (he == hipSuccess) he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  rlbm_status st = RLBM_OK;
  if (he == hipSuccess) {
    // n = 1 with noise of 1e-3 from site to site, T = 1 and a shear wave of amplitude 0.05: a state
    // that differs in every bit from site to site, as a working lattice's does (a uniform state
    // steps 5-12 % faster at 1024^2, which would not be the timing of a working lattice)
    const int64_t nf = h->sites * 2;
    const int nz = d == 3 ? (int)h->cfg.extent[2] : 1;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, stream, fields, 1.0, nf);
    hipLaunchKernelGGL(k_noise_fill, dim3((unsigned)((h->sites + 255) / 256)), dim3(256), 0, stream, fields, 1e-3,
                       h->sites);
    hipLaunchKernelGGL(k_shear_fill, dim3((unsigned)((h->sites + 255) / 256)), dim3(256), 0, stream, fields + nf, d,
                       (int)h->cfg.extent[0], (int)h->cfg.extent[1], nz, 0.05, h->sites);
    he = hipGetLastError();
  }
  if (he == hipSuccess)
    st = rlbm_init(h, fields, fields + h->sites, fields + 2 * h->sites, nullptr, 0.0, fa, nullptr, stream);
  const int saved = h->variant;
  float best = 1e30f;
  int best_v = saved;
  for (int v = 0; he == hipSuccess && st == RLBM_OK && v < rlbm::kNumVariants; ++v) {
    h->variant = v;
    st = rlbm_step(h, fa, fb, 2, nullptr, stream);
    if (st == RLBM_OK) he = hipEventRecord(e0, stream);
    if (he == hipSuccess && st == RLBM_OK) st = rlbm_step(h, fa, fb, steps, nullptr, stream);
    if (he == hipSuccess && st == RLBM_OK) he = hipEventRecord(e1, stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    ms /= steps;
    if (ms_out) ms_out[v] = ms;
    if (he == hipSuccess && ms < best) {
      best = ms;
      best_v = v;
    }
  }
  h->variant = (he == hipSuccess && st == RLBM_OK) ? best_v : saved;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(stream);
  if (fa) (void)hipFree(fa);
  if (fb) (void)hipFree(fb);
  if (fields) (void)hipFree(fields);
  if (st != RLBM_OK) return st;
  if (he != hipSuccess) return fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
  return rlbm_sync(h, stream);
}

// ---------------------------------------------------------------------------
// Allocation-free step: the tables of the last configuration stepped on a GPU, and a spare error
// flag, live in a file-scope device array (one copy per GPU, kept until the process ends).
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

constexpr size_t kStaticTablesBytes = (sizeof(rlbm::Tables) + 255) & ~size_t(255);
constexpr size_t kStaticFlagOffset = kStaticTablesBytes;
static_assert(kStaticTablesBytes + 256 <= RLBM_STATIC_SCRATCH_BYTES,
              "the tables of one lattice and the error flag must fit the static scratch array");

// Host-side state per device: the device address of its scratch array and the configuration whose
// tables the array holds.
constexpr int kStaticMaxDevices = 64;
struct StaticSlot {
  void *scratch = nullptr;
  rlbm_lattice *lat = nullptr;   // description of the resident configuration (host)
};
StaticSlot g_static[kStaticMaxDevices];
std::mutex g_static_mu;

// Two configurations give the same tables and launch shape (the tau field pointer aside).
bool same_tables(const rlbm_config &a, const rlbm_config &b) {
  if (a.model.d != b.model.d || a.model.order != b.model.order || a.model.kind != b.model.kind ||
      a.model.zeta != b.model.zeta || a.model.v0 != b.model.v0 || a.storage != b.storage || a.tau != b.tau ||
      a.n_ref != b.n_ref || a.tau_T != b.tau_T)
    return false;
  for (int k = 0; k < 3; ++k) {
    if (a.extent[k] != b.extent[k] || a.bc[k] != b.bc[k] || a.force[k] != b.force[k]) return false;
    if (a.wall_T[k][0] != b.wall_T[k][0] || a.wall_T[k][1] != b.wall_T[k][1]) return false;
  }
  return true;
}

}  // namespace

static __device__ __align__(256) unsigned char scratch[RLBM_STATIC_SCRATCH_BYTES];

extern "C" {

rlbm_status rlbm_step_static(const rlbm_config *cfg, void *f_a, void *f_b, int32_t nsteps, const rlbm_fields *last,
                             int32_t *flag, hipStream_t stream) {
  if (!cfg || !f_a || !f_b || nsteps < 0) return fail(RLBM_ERR_INVALID_ARG, "bad argument");
  int dev = -1;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
  if (dev < 0 || dev >= kStaticMaxDevices) return fail(RLBM_ERR_UNSUPPORTED, "device index beyond the static slots");
  std::lock_guard<std::mutex> lock(g_static_mu);
  StaticSlot &slot = g_static[dev];
  if (!slot.scratch) {
    // once per device, with the device current: the array's address on this GPU
    void *ptr = nullptr;
    he = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (he != hipSuccess || !ptr) return fail(RLBM_ERR_DEVICE, he != hipSuccess ? hipGetErrorString(he) : "no scratch address");
    slot.scratch = ptr;
  }
  if (!slot.lat || !same_tables(slot.lat->cfg, *cfg)) {
    // a new configuration: build its tables on the host and copy them into the array (the copy is
    // ordered after earlier work on this stream, and waited for before the host copy is freed)
    rlbm_lattice *h = new (std::nothrow) rlbm_lattice();
    rlbm::Tables *t = new (std::nothrow) rlbm::Tables;
    rlbm_status st = (h && t) ? prepare_lattice(cfg, h, t) : fail(RLBM_ERR_DEVICE, "out of host memory");
    if (st == RLBM_OK) {
      he = hipMemcpyAsync(slot.scratch, t, sizeof(rlbm::Tables), hipMemcpyHostToDevice, stream);
      if (he == hipSuccess) he = hipStreamSynchronize(stream);
      if (he != hipSuccess) st = fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
    }
    delete t;
    if (st != RLBM_OK) {
      delete h;
      if (he != hipSuccess) {
        // the array's contents are unknown now
        delete slot.lat;
        slot.lat = nullptr;
      }
      return st;
    }
    delete slot.lat;
    slot.lat = h;
  }
  rlbm_lattice *h = slot.lat;
  h->cfg.tau_field = cfg->tau_field;
  const int64_t bytes = (int64_t)(h->cfg.storage == RLBM_F64 ? 8 : 4) * h->quad.Q * h->sites;
  const char *pa = (const char *)f_a, *pb = (const char *)f_b;
  if (pa < pb + bytes && pb < pa + bytes) return fail(RLBM_ERR_INVALID_ARG, "f_a and f_b overlap");
  rlbm::LaunchArgs a = base_args(h, stream);
  a.tb = (const rlbm::Tables *)slot.scratch;
  a.err = flag ? (int *)flag : (int *)((char *)slot.scratch + kStaticFlagOffset);
  he = launch_steps(a, f_a, f_b, nsteps, last);
  return he == hipSuccess ? RLBM_OK : fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
}

}  // extern "C"
