// api.hip -- the C ABI of include/rlbm.h: handles, validation and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>

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
  int64_t sites = 0;
  std::string last_error;
};

namespace {

thread_local std::string g_last_error;

rlbm_status fail(rlbm_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

int stencil_of(const rlbm_model &m) {
  if (m.kind == RLBM_QUAD_UR_ONLATTICE) return rlbm::ST_UR2D;
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
  return a;
}

__global__ void k_fill(double *p, double v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
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
  int rc = rlbm::build_quadrature(model->d, model->zeta, model->order, model->kind, q, err);
  if (rc) return fail((rlbm_status)rc, err);
  *Q = q.Q;
  if (p) std::memcpy(p, q.p.data(), q.p.size() * sizeof(double));
  if (w) std::memcpy(w, q.w.data(), q.w.size() * sizeof(double));
  if (disp) std::memcpy(disp, q.disp.data(), q.disp.size() * sizeof(double));
  return RLBM_OK;
}

rlbm_status rlbm_create(const rlbm_config *cfg, rlbm_lattice **out) {
  if (!cfg || !out) return fail(RLBM_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  const rlbm_model &m = cfg->model;
  if (m.d != 2 && m.d != 3) return fail(RLBM_ERR_UNSUPPORTED, "d must be 2 or 3");
  for (int a = 0; a < m.d; ++a) {
    if (cfg->extent[a] < 1 || cfg->extent[a] > (1 << 20)) return fail(RLBM_ERR_INVALID_ARG, "extent out of range");
    if (cfg->bc[a] != RLBM_PERIODIC && cfg->bc[a] != RLBM_OPEN) return fail(RLBM_ERR_INVALID_ARG, "bad bc");
  }
  if (m.d == 3 && m.kind == RLBM_QUAD_UR_ONLATTICE) return fail(RLBM_ERR_UNSUPPORTED, "on-lattice rule is 2D");
  if (cfg->storage != RLBM_F64 && cfg->storage != RLBM_F32_DEV) return fail(RLBM_ERR_INVALID_ARG, "bad storage");
  if (!(cfg->tau > 0.0) || !std::isfinite(cfg->tau)) return fail(RLBM_ERR_INVALID_ARG, "tau must be > 0");
  if (cfg->storage == RLBM_F32_DEV && !(cfg->n_ref > 0.0)) return fail(RLBM_ERR_INVALID_ARG, "n_ref must be > 0");
  const int64_t nz = m.d == 3 ? cfg->extent[2] : 1;
  const int64_t sites = cfg->extent[0] * cfg->extent[1] * nz;
  if (m.d == 3 && nz > 65535) return fail(RLBM_ERR_UNSUPPORTED, "nz > 65535");
  // kernels address a population plane with 32-bit byte offsets
  if (sites * (cfg->storage == RLBM_F64 ? 8 : 4) >= (int64_t(1) << 32))
    return fail(RLBM_ERR_UNSUPPORTED, "a population plane must stay below 4 GiB");

  rlbm_lattice *h = new (std::nothrow) rlbm_lattice();
  if (!h) return fail(RLBM_ERR_DEVICE, "out of host memory");
  h->cfg = *cfg;
  h->stencil = stencil_of(m);
  h->sites = sites;
  std::string err;
  int rc = rlbm::build_quadrature(m.d, m.zeta, m.order, m.kind, h->quad, err);
  if (rc) {
    delete h;
    return fail((rlbm_status)rc, err);
  }
  rlbm::Tables *t = new rlbm::Tables;
  int bc[3] = {cfg->bc[0], cfg->bc[1], cfg->bc[2]};
  rc = rlbm::build_tables(h->quad, cfg->tau, cfg->storage == RLBM_F32_DEV ? cfg->n_ref : 1.0, cfg->storage,
                          cfg->extent, bc, *t, err);
  if (!rc && m.d == 3) rc = rlbm::build_eos_fit(m.zeta, *t, err);
  if (rc) {
    delete t;
    delete h;
    return fail((rlbm_status)rc, err);
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
  info->on_lattice = h->cfg.model.kind == RLBM_QUAD_UR_ONLATTICE;
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

rlbm_status rlbm_step(rlbm_lattice *h, void *f_a, void *f_b, int32_t nsteps, const rlbm_fields *last,
                      hipStream_t stream) {
  if (!h || !f_a || !f_b || nsteps < 0) return fail(RLBM_ERR_INVALID_ARG, "bad argument");
  const int64_t bytes = (int64_t)(h->cfg.storage == RLBM_F64 ? 8 : 4) * h->quad.Q * h->sites;
  const char *pa = (const char *)f_a, *pb = (const char *)f_b;
  if (pa < pb + bytes && pb < pa + bytes) return fail(RLBM_ERR_INVALID_ARG, "f_a and f_b overlap");
  rlbm::LaunchArgs a = base_args(h, stream);
  a.op = rlbm::OP_STEP;
  for (int32_t s = 0; s < nsteps; ++s) {
    a.fin = (s & 1) ? f_b : f_a;
    a.fout = (s & 1) ? f_a : f_b;
    a.fields = field_ptrs(s == nsteps - 1 ? last : nullptr);
    hipError_t he = rlbm::launch(a);
    if (he != hipSuccess) return fail(RLBM_ERR_DEVICE, hipGetErrorString(he));
  }
  return RLBM_OK;
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
    // a rest state n = 1, T = 1, u = 0: the step executes the same instructions for any state
    const int64_t nf = h->sites * 2;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, stream, fields, 1.0, nf);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((h->sites * d + 255) / 256)), dim3(256), 0, stream,
                       fields + nf, 0.0, h->sites * d);
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

}  // extern "C"
