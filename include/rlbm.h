/*
 * rlbm.h -- C ABI of an MI355X (gfx950) library for the relativistic lattice
 * Boltzmann method (RLBM) of Gabbana, Simeoni, Succi, Tripiccione,
 * "Relativistic Lattice Boltzmann Methods: Theory and Applications",
 * arXiv:1909.04502.
 *
 * The library implements the per-site collide-and-stream update of Sec. 6.2:
 * moments N^a and T^ab (step 1), the Landau-frame eigenproblem
 * T^ab U_b = eps U^a (step 2), n = U_a N^a (step 3), the temperature from the
 * equation of state eps/n = T (G_d(m/T) - 1) (step 4, Sec. 3 Eqs. defG and
 * eos-ddim), the equilibrium projected on orthonormal polynomials up to order
 * N (step 5, Sec. 5.2 Eqs. mj-feq-expansion and mj-discrete-feq), and
 * Anderson-Witting relaxation Omega_i = p_i.U/(p_i^0 tau) followed by
 * streaming (step 8, Sec. 5.1 Eq. discrete-rbe).  Off-lattice velocities are
 * streamed by linear interpolation (bilinear in 2D, trilinear in 3D).
 *
 * Units: lattice units with c = k_B = 1 and reference temperature T0 = 1
 * (Sec. 6.1).  zeta = m c^2 / (k_B T0) is the reduced mass of Sec. 5.2.
 *
 * Memory and ownership
 *   All population, field and gradient buffers are allocated and owned by the
 *   caller, in device memory of the current HIP device, and are passed as
 *   plain pointers.  Every call enqueues its work on the given hipStream_t
 *   (0 = the null stream) and returns without synchronising.  A handle owns
 *   only small constant tables, an error flag and cached launch graphs; it is
 *   freed by the matching destroy call.  One handle must not be used from two
 *   streams at once.
 *
 * Population layout ("SoA")
 *   f[i * sites + s] with s = x + nx * (y + ny * z) (x fastest), i the
 *   population index.  Population order: shell-major, i = j * n_dirs + k,
 *   with directions (2D product rule)
 *     (1,0) (-1,0) (0,1) (0,-1) (1,1) (-1,-1) (-1,1) (1,-1)          [unit vectors]
 *   and (3D product rule) the 6 axis, 12 edge, 8 corner directions
 *     (+-1,0,0) (0,+-1,0) (0,0,+-1), (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0),
 *     (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1), (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1),
 *     (1,1,1) (-1,-1,-1) (1,1,-1) (-1,-1,1) (1,-1,1) (-1,1,-1) (-1,1,1) (1,-1,-1);
 *   for the printed on-lattice massless rules (Sec. 5.3 / App. H.2)
 *     (3,4) (-3,-4) (-3,4) (3,-4) (4,3) (-4,-3) (-4,3) (4,-3) (5,0) (-5,0) (0,5) (0,-5)
 *   on three (order 2) or four (order 3) shells, zero-weight populations
 *   dropped (28 / 44 populations);
 *   for the printed (3+1)-d massless rule (App. H.1) the groups (4,4,3)_FS,
 *   (5,4,0)_FS, (6,2,1)_FS on four shells, shell-major, within a shell the
 *   groups in that order with zero-weight groups dropped ((6,2,1) on shell 0;
 *   (4,4,3), (6,2,1) on shells 1 and 2; all three on shell 3: 288
 *   populations), each group's members ordered as for the massive rules;
 *   for the massive on-lattice rules the generating vectors of the groups
 *     order 2: (1,0) (1,1) (2,1) (2,2) (3,1)
 *     order 3: (1,0) (1,1) (2,0) (2,1) (2,2) (3,0) (3,2) (3,3) (4,0)
 *   in this order, each group's members with first non-zero component > 0 in
 *   decreasing (x, y) order, each followed by its opposite, and the rest
 *   vector (0,0) last (29 / 45 populations).
 *   Antipodal populations are always adjacent (i, i+1 for even i).
 *
 * State convention
 *   A state buffer holds the post-collision populations f*(x, t) (the values
 *   about to stream).  rlbm_init builds f*(x, 0) from the initial fields;
 *   rlbm_step advances t by streaming then colliding; the pre-collision
 *   populations of time t are f(x, t) = f*(x - delta_i, t - 1) (interpolated).
 *
 * Storage (rlbm_storage)
 *   RLBM_F64      populations stored as double.
 *   RLBM_F32_DEV  populations stored as float deviations g_i = f_i - f^ref_i
 *                 from the rest-frame equilibrium f^ref(n_ref, T = 1, U = 0);
 *                 moments accumulate the deviations in float, the
 *                 eigenproblem, equation of state and equilibrium
 *                 coefficients are computed in double.
 *   RLBM_F32_DEV_F64  the same float deviations in memory (same traffic),
 *                 but every step computes in double: the interpolated
 *                 pull, the moment sums and the relaxation; only the
 *                 store rounds to float.  Rounding in float arithmetic is
 *                 correlated from step to step and its error grows about
 *                 linearly with the number of steps; the rounding of the
 *                 stores alone does not build up.  Product rules only.
 *
 * Errors
 *   Functions return rlbm_status.  Invalid arguments are reported
 *   synchronously.  A non-physical state met by a kernel (n <= 0, eps <= 0,
 *   T <= 0, NaN, a space-like Landau eigenvector; in 3D with m > 0 also a
 *   temperature outside [1/128, 128], the range of the equation of state's
 *   fitted series) sets a device flag that rlbm_sync reports as
 *   RLBM_ERR_NONPHYSICAL.
 */
#ifndef RLBM_H
#define RLBM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RLBM_OK = 0,
  RLBM_ERR_INVALID_ARG = 1,   /* bad pointer, size, or parameter */
  RLBM_ERR_UNSUPPORTED = 2,   /* valid request outside what the library implements */
  RLBM_ERR_QUADRATURE = 3,    /* quadrature construction or verification failed */
  RLBM_ERR_DEVICE = 4,        /* a HIP runtime call failed */
  RLBM_ERR_NONPHYSICAL = 5    /* a kernel met a non-physical state (see above) */
} rlbm_status;

typedef enum { RLBM_F64 = 0, RLBM_F32_DEV = 1, RLBM_F32_DEV_F64 = 2 } rlbm_storage;
/* RLBM_WALL: reads clamp as RLBM_OPEN, and the first and last plane of the
 * axis are no-slip walls whose collision is replaced by the local equilibrium
 * at zero flow speed (the site's own n and T, or a prescribed T:
 * rlbm_config.wall_T; the walls of the forcing validation, Sec. 8.1, and the
 * plates of the thermal-conductivity measurement, Sec. 7.2).  Product and
 * massive rules (not the 3D massive rule in double storage). */
typedef enum { RLBM_PERIODIC = 0, RLBM_OPEN = 1, RLBM_WALL = 2 } rlbm_bc;
typedef enum {
  RLBM_QUAD_UR_ONLATTICE = 0, /* printed massless rules, integer streaming (zeta = 0): (2+1)-d of
                               * order 2 and 3 (App. H.2; 28 / 44 populations) and (3+1)-d of order
                               * 3 (App. H.1; 288 populations, the rule of the 3D Sod tube of
                               * Sec. 8.2) */
  RLBM_QUAD_PRODUCT = 1,      /* off-lattice product rule: shells x directions, interpolated streaming */
  RLBM_QUAD_MASSIVE_ONLATTICE = 2 /* massive (2+1)-d on-lattice rule (Sec. 5.3): integer vectors n_i in
                                   * full-symmetric groups, p_i = p^0_i (1, v0 n_i) with p^0_i =
                                   * zeta / sqrt(1 - v0^2 |n_i|^2), one weight per group solving the
                                   * moment conditions up to degree 2N; order 2: the 29-vector
                                   * stencil of the worked example, order 3: the 45-vector stencil of
                                   * the GPU benchmark (Sec. 6.3); zeta > 0, integer streaming */
} rlbm_quad_kind;

/* The paper's statement of the problem (Sec. 5.2-5.3): dimension d, reduced
 * mass zeta = m/T0, expansion order N and the quadrature. */
typedef struct {
  int32_t d;        /* spatial dimensions: 2 or 3 */
  int32_t order;    /* expansion order N: 2 or 3 */
  int32_t kind;     /* rlbm_quad_kind */
  int32_t pad_;
  double zeta;      /* reduced mass m c^2/(k_B T0), >= 0 */
  double v0;        /* RLBM_QUAD_MASSIVE_ONLATTICE: the lattice-speed parameter v0 of the stencil,
                     * inside the window where every group weight is >= 0; 0 = the middle of that
                     * window (found by the line search of Sec. 5.3).  Ignored by other kinds. */
} rlbm_model;

typedef struct {
  rlbm_model model;
  int64_t extent[3];   /* nx, ny, nz (nz = 1 for d = 2); each >= 1 */
  int32_t bc[3];       /* rlbm_bc per axis; RLBM_OPEN = zero-gradient (reads clamp to the edge) */
  int32_t storage;     /* rlbm_storage */
  double tau;          /* relaxation time, used where tau_field is NULL; > 0.5 recommended */
  const void *tau_field; /* device [sites] per-site tau, double (F64) or float (float storages), or NULL */
  double n_ref;        /* reference density of the float deviations (T_ref = 1, U = 0) */
  double force[3];     /* constant acceleration g (lattice units, first d used) of the external
                        * force of Sec. 5.4, scheme B: Minkowski force K = p^0 g, K^0 = g.p;
                        * the update subtracts F^ext_i = -(m/T) (K^a U_a / p_i^0) f^eq_i, the
                        * sign of the kinetic equation (the fluid accelerates along g).  Zero =
                        * no force; no effect for zeta = 0 (the term carries the mass). */
  double tau_T;        /* on-lattice rules: the relaxation time becomes tau(x) + tau_T / T(x),
                        * T the site's temperature of the step (Sec. 6.2 step 7, tau chosen so
                        * that eta/s stays constant: for a massless gas with s = (d + 1) n and
                        * the lattice shear viscosity eta = c_eta P (tau - 1/2), take tau = 1/2
                        * and tau_T = (eta/s)(d + 1)/c_eta in lattice units).  0 = off;
                        * RLBM_ERR_UNSUPPORTED for product rules. */
  double wall_T[3][2]; /* RLBM_WALL axes: the temperature imposed on the first [a][0] and last
                        * [a][1] plane (the heated and cooled plates of the thermal-conductivity
                        * measurement, Sec. 7.2); 0 = the site's own temperature.  The wall
                        * site keeps its own n.  >= 0; non-zero only on wall axes. */
} rlbm_config;

typedef struct {
  int32_t Q;           /* populations per site */
  int32_t n_basis;     /* dimension of the polynomial space (N+1)^2 (2D), (N+1)(N+2)(2N+3)/6 (3D) */
  int64_t sites;       /* nx * ny * nz */
  int64_t state_bytes; /* bytes of one population buffer */
  int32_t elem_bytes;  /* 8 (F64) or 4 (float storages) */
  int32_t on_lattice;  /* 1 if displacements are integers */
  double v0;           /* on-lattice rules: the lattice-speed parameter in use (massive rules: inside
                        * the window; the printed massless rules: 1/5 in 2D, 1/sqrt(41) in 3D);
                        * 0 for product rules */
} rlbm_info;

typedef struct rlbm_lattice rlbm_lattice;   /* opaque */

/* Macroscopic output fields (device, [sites] each; U is [d+1][sites]).
 * Any pointer may be NULL to skip that field. */
typedef struct {
  double *n;     /* particle density n = U_a N^a (Sec. 6.2 step 3) */
  double *eps;   /* energy density, largest eigenvalue of T^a_b (step 2) */
  double *T;     /* temperature from the equation of state (step 4) */
  double *U;     /* four-velocity, U^a U_a = 1, U^0 > 0 (step 2) */
} rlbm_fields;

/* ---------------------------------------------------------------- host only */

/* Build the quadrature of a model on the host (Sec. 5.3; App. H.2 for the
 * printed rule).  Call with p = w = disp = NULL to query *Q.  Otherwise p is
 * [Q][d+1] (energy first), w is [Q], disp is [Q][d] (sites per step), all host
 * memory of the caller.  No GPU is touched. */
rlbm_status rlbm_quadrature_build(const rlbm_model *model, int32_t *Q,
                                  double *p, double *w, double *disp);

/* The v0 window of a massive on-lattice model (model->kind ==
 * RLBM_QUAD_MASSIVE_ONLATTICE, d = 2, order 2 or 3, zeta > 0): the interval
 * [*lo, *hi] where every group weight is >= 0 (Sec. 5.3 line search: a scan
 * of min_g w_g(v0) over (0, 1/max|n|), golden-section refinement, bisection
 * to both ends).  model->v0 is ignored.  RLBM_ERR_QUADRATURE if no v0
 * qualifies.  Host only; takes tens of milliseconds. */
rlbm_status rlbm_massive_window(const rlbm_model *model, double *lo, double *hi);

const char *rlbm_status_string(rlbm_status s);

/* Message of the last failing call on this host thread (static storage, valid
 * until the next failing call on the same thread). */
const char *rlbm_last_error(void);

/* ---------------------------------------------------------------- lattices */

/* Create a lattice handle: builds and verifies the quadrature and the
 * projection matrix on the host, uploads them, and picks a launch shape.
 * Synchronous.  *out receives the handle. */
rlbm_status rlbm_create(const rlbm_config *cfg, rlbm_lattice **out);
rlbm_status rlbm_destroy(rlbm_lattice *h);
rlbm_status rlbm_get_info(const rlbm_lattice *h, rlbm_info *info);

/* Initial condition (Sec. 6.2: f(x, t0) = f^eq).  Inputs are device arrays of
 * [sites] doubles: density n0, temperature T0 and the d components of the
 * three-velocity u0 ([d][sites], |u0| < 1; U = gamma (1, u0)).  noise is NULL
 * or a device [Q][sites] double array xi; the pre-collision populations are
 * f^eq_i (1 + noise_amp xi_i).  Writes the post-collision state f*(x, 0) to
 * f_out (state layout above).  fields0 (may be NULL) receives the macroscopic
 * fields of the pre-collision state at t = 0. */
rlbm_status rlbm_init(rlbm_lattice *h, const double *n0, const double *T0, const double *u0,
                      const double *noise, double noise_amp, void *f_out,
                      const rlbm_fields *fields0, hipStream_t stream);

/* Advance nsteps >= 0 time steps, ping-ponging between f_a (input) and f_b.
 * The result is in f_b when nsteps is odd and in f_a when it is even.  f_a and
 * f_b must not overlap.  last (may be NULL) receives the macroscopic fields of
 * the pre-collision state of the final step's time level.  With nsteps >= 4 and
 * last == NULL the launches are captured once into a HIP graph (kept by the
 * handle for the same buffers, step count and launch variant) that is replayed
 * on `stream`; a handle serves one stream at a time.  A run of more than 256
 * steps replays the graph of 256 steps (an even count: the state is back in
 * f_a after each replay) and ends with the remaining 1 .. 256 steps. */
rlbm_status rlbm_step(rlbm_lattice *h, void *f_a, void *f_b, int32_t nsteps,
                      const rlbm_fields *last, hipStream_t stream);

/* Macroscopic fields of the populations obtained by streaming the state f
 * (i.e. the pre-collision state of the next time level). */
rlbm_status rlbm_moments(rlbm_lattice *h, const void *f, const rlbm_fields *out,
                         hipStream_t stream);

/* Drain the stream and report a deferred device error (clears the flag). */
rlbm_status rlbm_sync(rlbm_lattice *h, hipStream_t stream);

/* ------------------------------------------------ allocation-free stepping
 *
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): rlbm_step
 * without a handle.  The per-lattice tables that rlbm_create allocates (and a
 * spare error flag) live instead in a static device array of
 * RLBM_STATIC_SCRATCH_BYTES on each GPU the library runs on, held until the
 * process ends; every configuration's tables fit it (the size is checked when
 * the library is built).  No hipMalloc, hipFree or other allocating device
 * call is made.
 *
 * cfg is validated as by rlbm_create (same errors).  The first call on a GPU,
 * and each call whose configuration differs from the previous call's on that
 * GPU (tau_field aside), builds the tables on the host, copies them into the
 * array on `stream` and waits for that copy; later calls with the same
 * configuration only launch the steps.  The steps are those of rlbm_step
 * (same kernels, default launch shape and store kind, so the same results),
 * launched one by one on `stream` (no graph).  f_a, f_b, nsteps and last are
 * as for rlbm_step; the caller owns every buffer.
 *
 * flag (device int32, or NULL): set to 1 by a kernel that meets a
 * non-physical state; the caller clears and reads it.  NULL: the flag is
 * written to the array and not reported.
 *
 * All calls on one GPU share its array, which keeps the last call's tables:
 * calls that overlap on one GPU (several host threads, or several streams whose
 * work overlaps) with different configurations race.  Host threads are
 * serialised by a lock; the device work of calls on different streams is not. */
#define RLBM_STATIC_SCRATCH_BYTES (128 * 1024)
rlbm_status rlbm_step_static(const rlbm_config *cfg, void *f_a, void *f_b, int32_t nsteps,
                             const rlbm_fields *last, int32_t *flag, hipStream_t stream);

/* ------------------------------------------------------------ reverse mode
 *
 * Hand-written adjoint of the update (not part of the paper; it lets tau or
 * the initial fields be calibrated against a target flow).  With B_0 = C(f_0),
 * F_t = S(B_{t-1}), B_t = C(F_t) (S streaming, C collision, as above) and a
 * loss L on the macroscopic fields of F_{T+1} = S(B_T), the adjoint buffers
 * lam_t = dL/dF_t (same element type and layout as a state) obey
 *   lam_{T+1} = rlbm_moments_vjp(B_T, dL/dfields),
 *   lam_t     = rlbm_adjoint_step(B_{t-1}, lam_{t+1}),   t = T .. 1,
 * and rlbm_init_vjp(fields, lam_1) gives dL/du0 (and dL/dn0, dL/dT0).
 * dtau_accum (device [sites] doubles, or NULL) is incremented by each call's
 * contribution to dL/dtau(x) (per-site tau field or scalar tau alike).
 * Implemented for the 2D product rules with periodic boundaries; other
 * lattices return RLBM_ERR_UNSUPPORTED.  Every forward quantity of a site is
 * recomputed from the given state; the Landau eigenpair is differentiated
 * implicitly (exact derivative of the converged eigenpair). */
rlbm_status rlbm_adjoint_step(rlbm_lattice *h, const void *f_prev, const void *lam_next, void *lam,
                              double *dtau_accum, hipStream_t stream);
rlbm_status rlbm_moments_vjp(rlbm_lattice *h, const void *f, const rlbm_fields *grad, void *lam,
                             hipStream_t stream);
rlbm_status rlbm_init_vjp(rlbm_lattice *h, const double *n0, const double *T0, const double *u0,
                          const double *noise, double noise_amp, const void *lam1, double *du0,
                          double *dn0, double *dT0, double *dtau_accum, hipStream_t stream);

/* ----------------------------------------------------------------- batches
 *
 * Many independent 2D product-rule lattices (different extents, zeta and
 * scalar tau; one order and storage) advanced by one persistent launch per
 * step.  The state of a batch is one flat device buffer: lattice l owns the
 * elements [elem_off[l], elem_off[l] + Q * sites_l) in its own SoA layout.
 * Field arrays of a batch are concatenated per lattice: n0, T0, n, eps, T at
 * site_off[l]; u0 as [2][sites_l] at 2 site_off[l]; U as [3][sites_l] at
 * 3 site_off[l].  rlbm_batch_lattice exposes the member handles (their own
 * rlbm_step is the per-lattice reference path). */
typedef struct rlbm_batch rlbm_batch;   /* opaque */
rlbm_status rlbm_batch_create(const rlbm_config *cfgs, int32_t nlat, rlbm_batch **out);
rlbm_status rlbm_batch_destroy(rlbm_batch *b);
rlbm_status rlbm_batch_layout(const rlbm_batch *b, int64_t *total_elems, int64_t *total_sites,
                              int64_t *elem_off /* [nlat] or NULL */, int64_t *site_off /* [nlat] or NULL */);
rlbm_status rlbm_batch_lattice(const rlbm_batch *b, int32_t l, rlbm_lattice **h);
rlbm_status rlbm_batch_init(rlbm_batch *b, const double *n0, const double *T0, const double *u0, void *f_out,
                            hipStream_t stream);
/* nsteps steps of every lattice, ping-ponging as rlbm_step.  With use_graph != 0
 * the launches are captured once into a HIP graph (cached for the same
 * buffers, step count and variant) and the graph is replayed on `stream`;
 * more than 256 steps replay the graph of 256 steps, as rlbm_step does. */
rlbm_status rlbm_batch_step(rlbm_batch *b, void *f_a, void *f_b, int32_t nsteps, int32_t use_graph,
                            hipStream_t stream);
rlbm_status rlbm_batch_moments(rlbm_batch *b, const void *f, const rlbm_fields *out, hipStream_t stream);
rlbm_status rlbm_batch_sync(rlbm_batch *b, hipStream_t stream);
/* Batch launch variants: tile shape x persistent grid size.  rlbm_batch_autotune
 * times each on the caller's state (an even number of steps per variant, so the
 * evolved state ends in f_a) and keeps the fastest. */
int32_t rlbm_batch_variant_count(void);
rlbm_status rlbm_batch_set_variant(rlbm_batch *b, int32_t variant);
rlbm_status rlbm_batch_get_variant(const rlbm_batch *b, int32_t *variant);
rlbm_status rlbm_batch_autotune(rlbm_batch *b, void *f_a, void *f_b, int32_t steps, float *ms_out,
                                hipStream_t stream);

/* ------------------------------------------------------- launch variants */

/* The step kernel has rlbm_variant_count() launch variants (block shape,
 * register / occupancy target, XCD-aware tile order, and for the 2D product
 * rules on a periodic x axis whose extent is a multiple of 4, upstream windows
 * staged in LDS); results do not depend on the variant.  rlbm_autotune times every variant for `steps` steps on
 * scratch buffers of the lattice's size (allocated and freed inside the
 * call and holding a shear wave of amplitude 0.05 at T = 1 and a density
 * of 1 with site-to-site noise of 1e-3; the
 * caller's buffers are not touched), selects the fastest and
 * returns after synchronising the stream.  ms_out (host, may be NULL)
 * receives rlbm_variant_count() milliseconds per step. */
int32_t rlbm_variant_count(void);
rlbm_status rlbm_set_variant(rlbm_lattice *h, int32_t variant);
rlbm_status rlbm_get_variant(const rlbm_lattice *h, int32_t *variant);
rlbm_status rlbm_autotune(rlbm_lattice *h, int32_t steps, float *ms_out, hipStream_t stream);

/* How rlbm_step writes the post-collision populations (results do not depend
 * on it).  RLBM_STORES_AUTO (the default) uses non-temporal stores, which are
 * not kept in the L2 or the 256 MiB last-level cache, when the two state
 * buffers together (2 Q sites x element size) exceed 384 MiB, so that the
 * next step reads nearly all populations from memory anyway, and a row of
 * sites (extent[0] x element size) is a multiple of 64 bytes (with ragged
 * rows they were measured slower).  Otherwise ordinary stores are kept, and
 * smaller lattices find the populations in the cache on the next step.
 * RLBM_STORES_CACHED and RLBM_STORES_NONTEMPORAL force one kind.
 * rlbm_get_store_mode returns the mode and (nontemporal, may be NULL)
 * whether rlbm_step uses non-temporal stores for this lattice; an unknown
 * mode is RLBM_ERR_INVALID_ARG. */
typedef enum {
  RLBM_STORES_AUTO = 0,
  RLBM_STORES_CACHED = 1,
  RLBM_STORES_NONTEMPORAL = 2
} rlbm_store_mode;
rlbm_status rlbm_set_store_mode(rlbm_lattice *h, int32_t mode);
rlbm_status rlbm_get_store_mode(const rlbm_lattice *h, int32_t *mode, int32_t *nontemporal);
/* The same for the batched step: the footprint is that of the whole batch,
 * and every member's rows must be multiples of 64 bytes. */
rlbm_status rlbm_batch_set_store_mode(rlbm_batch *b, int32_t mode);
rlbm_status rlbm_batch_get_store_mode(const rlbm_batch *b, int32_t *mode, int32_t *nontemporal);

/* ---------------------------------------------------------- measurement
 *
 * The memory ceiling the step kernels are measured against (not part of the
 * method).  Copies `planes` population planes of `sites` elements of
 * elem_bytes (4 or 8) from src to dst, device buffers of the caller that must
 * not overlap.  mode 0 ("site"): one thread per site loads its element of
 * every plane, then stores them, the access pattern of the fused update
 * (planes 32 or 104, else RLBM_ERR_UNSUPPORTED); mode 1 ("flat"): the same
 * bytes as 16-byte vectors (16-byte aligned buffers and size).  nontemporal
 * = 1 writes with non-temporal stores as rlbm_set_store_mode does.
 * Asynchronous on `stream`. */
rlbm_status rlbm_copy_planes(const void *src, void *dst, int64_t sites, int32_t planes, int32_t elem_bytes,
                             int32_t mode, int32_t nontemporal, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* RLBM_H */
