/*
 * fks.h -- C ABI of libfks: the fast spectral Boltzmann collision operator and the
 * exact-shift transport of the Fast Kinetic Scheme, on one AMD MI355X (gfx950).
 *
 * The calls follow the paper's statement of the problem:
 *   - Q_k(f_j, f_j), the collision operator evaluated independently in every
 *     spatial cell j on the N^3 discrete-velocity grid (Section 2.1 collision step;
 *     Section 2.2.2; Appendix A: Fourier-Galerkin method, eq. CF1, Carleman form,
 *     separable angular quadrature);
 *   - the exact shift of every velocity's piecewise-constant profile by v_k dt
 *     (Section 2.1 transport step; Section 3 particle interpretation / generic cell);
 *   - the first-order split step: transport, then explicit Euler collision
 *     f^{n+1} = f* + dt Q(f*) (eq. transport, eq. disc_relax).
 *
 * Conventions
 *   Velocity grid: v_i = -L + i*dv, dv = 2L/n, i = 0..n-1 per axis.  A distribution
 *   in one cell is a contiguous [n][n][n] array indexed (i, j, k) <-> (v_x, v_y, v_z),
 *   k fastest.  A batch is [n_cells][n][n][n], cells contiguous.
 *   Fourier modes: the symmetric set {-n/2+1, ..., n/2-1}^3 with wave numbers
 *   xi = pi k / L; padded convolution grid P = 3n/2 per axis (alias-free).
 *   Kernel: B = C |v - v*|^alpha (eq. J9hb, variable hard spheres); hard spheres
 *   alpha = 1 use the closed-form separable tables, alpha < 1 (e.g. Maxwell
 *   molecules alpha = 0) use n_radial Gauss-Legendre nodes in |x| (one separable
 *   term per direction and node).
 *
 * Memory ownership
 *   Every device buffer is allocated and owned by the caller: distributions,
 *   outputs, the plan's table and workspace buffers, transport state, moments.
 *   Sizes come from the *_sizes queries.  The library never calls hipMalloc or
 *   hipFree.  Handles own host memory only.  Device pointers must be 256-byte
 *   aligned.  *_destroy(NULL) is a no-op.
 *
 * Streams
 *   `stream` is a hipStream_t passed as void* (NULL = the default stream).  All
 *   device work is enqueued on it; no call synchronises the host unless stated.
 *
 * Errors
 *   Every call returns fks_status.  Arguments are validated before any launch;
 *   on error nothing is enqueued.  A batch of zero cells is a no-op (its pointers may
 *   be NULL).  Launch failures return FKS_E_DEVICE.
 *   fks_last_error() returns a message for the last failing call on the calling
 *   thread (valid until that thread's next call).  Nothing throws or aborts across
 *   this boundary.
 */
#ifndef FKS_H_
#define FKS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FKS_OK = 0,
  FKS_E_ARG = -1,         /* invalid argument (null, out of range, aliasing, alignment) */
  FKS_E_UNSUPPORTED = -2, /* valid but not built (e.g. an n without compiled kernels) */
  FKS_E_WORKSPACE = -3,   /* buffers not bound, or too small for n_cells */
  FKS_E_DEVICE = -4,      /* HIP launch / copy failure */
  FKS_E_STATE = -5        /* call out of order (e.g. collide before bind) */
} fks_status;

enum { FKS_HARD_SPHERES = 0, FKS_VHS = 1 };
enum { FKS_F64 = 0, FKS_F32 = 1 };

/* plan flags */
#define FKS_CONSERVE 1u        /* FP64 projection of Q onto zero mass/momentum/energy */
#define FKS_ALLOW_OVERLAP 2u   /* accept R > 4L/(3+sqrt 2) (periodic images may interact) */

typedef struct {
  int32_t n;        /* velocity points per axis; supported: 8, 12, 16, 24, 32 */
  int32_t kernel;   /* FKS_HARD_SPHERES or FKS_VHS */
  double L;         /* velocity box half-width: grid on [-L, L)^3, L > 0 */
  double R;         /* Carleman truncation radius, 0 < R (<= 4L/(3+sqrt 2) unless ALLOW_OVERLAP) */
  double alpha;     /* VHS exponent in [0, 1) for FKS_VHS; ignored for hard spheres */
  double C;         /* kernel constant C in B = C |g|^alpha, > 0 (hard spheres: B~ = 4C) */
  int32_t a1, a2;   /* polar x azimuthal directions (M = a1*a2), each in [1, 64] */
  int32_t n_radial; /* radial Gauss-Legendre nodes for FKS_VHS, [1, 64]; ignored otherwise */
  int32_t dtype;    /* FKS_F32 or FKS_F64: storage and arithmetic of the transforms */
  uint32_t flags;   /* FKS_CONSERVE | FKS_ALLOW_OVERLAP */
  int32_t reserved;
} fks_collide_desc;

typedef struct fks_plan_s* fks_plan;
typedef struct fks_xport_s* fks_xport;

/* ---- collision operator --------------------------------------------------------- */

/* Builds the FP64 kernel tables on the host (Appendix A: phi_R, psi_R, directions,
 * radial nodes, loss weight) for batches of up to max_cells cells (1 .. 2^19, so that
 * one chunk's launches stay within the 2^32 threads of a grid; larger batches are
 * processed in chunks of max_cells).  FKS_E_ARG outside that range.  Host only. */
fks_status fks_plan_create(const fks_collide_desc* desc, int64_t max_cells, fks_plan* out);

/* Bytes of the device table buffer and of the device workspace (for max_cells cells). */
fks_status fks_plan_sizes(fks_plan plan, size_t* table_bytes, size_t* workspace_bytes);

/* Number of separable terms including the loss term, and the padded grid size P. */
fks_status fks_plan_info(fks_plan plan, int32_t* n_terms, int32_t* pad);

/* Binds caller-owned device buffers (sizes from fks_plan_sizes) and enqueues the table
 * upload on `stream`.  May be called again to rebind.  d_workspace may be NULL (with
 * workspace_bytes 0): only fks_collide_noalloc and the BGK steps can then run; calls that
 * need the workspace return FKS_E_STATE. */
fks_status fks_plan_bind(fks_plan plan, void* d_tables, size_t table_bytes, void* d_workspace,
                         size_t workspace_bytes, void* stream);

/* q[c] = Q(f[c], f[c]) for c < n_cells (Section 2.1 collision step, Appendix A eq. CF1
 * evaluated by the padded FFT convolution).  f, q: device [n_cells][n][n][n] of the plan
 * dtype; q must not overlap f.  With FKS_CONSERVE, q is projected in FP64 so its discrete
 * mass, momentum and energy vanish.  n_cells may exceed max_cells (processed in chunks). */
fks_status fks_collide(fks_plan plan, const void* f, void* q, int64_t n_cells, void* stream);

/* fks_collide for callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same q = Q(f) with the same
 * kernels, but the transform workspace is a fixed 128 MiB array owned by the library (one
 * per GPU, held until the process ends) instead of the plan's bound workspace.  The plan
 * needs only its tables bound (fks_plan_bind may pass a NULL workspace of 0 bytes).  The call
 * allocates nothing.  n_cells is limited to what the array holds for the plan (at n = 32 FP32
 * about 230 cells) and to max_cells; larger batches return FKS_E_ARG with the limit in the
 * message.  Every call on one GPU uses the same array: calls that overlap on a GPU (other
 * streams, other host threads) race and must be ordered by the caller.  Errors as
 * fks_collide; FKS_E_STATE if the tables are not bound. */
fks_status fks_collide_noalloc(fks_plan plan, const void* f, void* q, int64_t n_cells, void* stream);

/* Explicit Euler collision stage (eq. disc_relax): f_out = f_in + dt * Q(f_in) per cell.
 * f_out may equal f_in (in place).  q (optional, NULL to skip) receives Q.  d_moments
 * (optional, device double [n_cells][5]) receives the FP64 moments of f_out:
 * dv^3 sum_k (1, v_x, v_y, v_z, |v|^2/2) f_out (Section 3, macroscopic variables). */
fks_status fks_relax(fks_plan plan, const void* f_in, void* f_out, void* q, double dt,
                     int64_t n_cells, double* d_moments, void* stream);

/* n_steps Heun (SSP-RK2) steps of the space-homogeneous collision equation df/dt = Q(f)
 * in place on f (the paper allows other integrators in place of eq. disc_relax):
 * f1 = f + dt Q(f);  f2 = f1 + dt Q(f1);  f = (f + f2)/2.  f_tmp1, f_tmp2: caller buffers of
 * the size of f, not overlapping f or each other. */
fks_status fks_heun(fks_plan plan, void* f, void* f_tmp1, void* f_tmp2, double dt, int32_t n_steps,
                    int64_t n_cells, void* stream);

/* FP64 moments of f: d_u[c][0..4] = dv^3 sum_k phi(v_k) f[c][k], phi = (1, v, |v|^2/2). */
fks_status fks_moments(fks_plan plan, const void* f, int64_t n_cells, double* d_u, void* stream);

/* Normalised non-equilibrium residual of f per cell (the moments of Section 3 one order
 * further): with rho, u, T the density, mean velocity and temperature of f, c = v - u,
 * sigma_ij = dv^3 sum_k f c_i c_j - rho T delta_ij (deviatoric stress) and
 * q_i = dv^3 sum_k f |c|^2 c_i / 2 (heat flux), d_r[c] = |sigma|_F / (rho T) + |q| / (rho T^1.5)
 * (device FP64, [n_cells]); zero for a Maxwellian, invariant under f -> a f and under
 * velocity shifts.  Only the plan's grid (n, L, dtype) is used; no binding needed. */
fks_status fks_noneq(fks_plan plan, const void* f, int64_t n_cells, double* d_r, void* stream);

/* Uneven batch: n_groups plans (each its own n, same dtype), group g evaluates
 * q[g] = Q(f[g]) on n_cells[g] cells.  The groups run concurrently: the first non-empty
 * group on `stream`, each further one (at most 7) on a library-owned side stream forked
 * from `stream` by an event and joined back before the call returns, so work enqueued on
 * `stream` afterwards sees every q[g]; under stream capture the fork and join are graph
 * edges.  Groups whose plans share a workspace run one after another on `stream`.  The
 * side streams (default priority) and events are created once per device and kept. */
fks_status fks_collide_grouped(const fks_plan* plans, int32_t n_groups, const void* const* f,
                               void* const* q, const int64_t* n_cells, void* stream);

void fks_plan_destroy(fks_plan plan);

/* Slab schedule: each cell's padded convolution grid is split into `slabs` workgroups
 * (compiled choices per n and dtype), optionally all placed on one XCD (xcd_map = 1).
 * Results are identical up to rounding order for every schedule. */
fks_status fks_plan_schedule(fks_plan plan, int32_t* slabs, int32_t* xcd_map);
fks_status fks_plan_set_schedule(fks_plan plan, int32_t slabs, int32_t xcd_map); /* FKS_E_UNSUPPORTED if not compiled */
/* Term groups (latency of small batches): each slab's loop over the separable terms is
 * split over tg workgroups whose partial spectra the synthesis sums (same Q up to the
 * order of the FP additions).  Plans created with max_cells <= 32 accept tg up to
 * min(32, terms); others only 1 (FKS_E_UNSUPPORTED).  get returns the groups in effect
 * (no group is left empty) and the maximum.  The XCD mapping is not used with tg > 1.
 * fks_plan_autotune also tries tg = 1, 2, 4, 8, 16, 32 where allowed. */
fks_status fks_plan_set_term_groups(fks_plan plan, int32_t tg);
fks_status fks_plan_get_term_groups(fks_plan plan, int32_t* tg, int32_t* tg_max);

/* Autotuner: times every compiled schedule (slab count x XCD mapping) on up to max_cells
 * cells of f (device, plan dtype; q receives Q) with hipEvents on `stream` (the host waits)
 * and keeps the fastest.  cache_path (optional, may be NULL): a text file of earlier choices,
 * one JSON object per line keyed by (device, n, dtype, terms, cells); a matching entry is
 * used without timing, a new choice is appended. */
fks_status fks_plan_autotune(fks_plan plan, const void* f, void* q, int64_t n_cells, const char* cache_path,
                             void* stream);

/* ---- transport (Section 2.1 transport step; Section 3 generic cell) -------------- */

/* Periodic box of nx*ny*nz cells of width dx (cells in C order [nx][ny][nz], at most
 * 2^24, and ny*nz*n^3 < 2^31) for the velocity grid (n, L), n in {8, 12, 16, 24, 32} (else
 * FKS_E_UNSUPPORTED).
 * Each velocity k keeps an FP64 sub-cell offset s_k and an integer cumulative shift o_k
 * (device state, caller-owned). */
fks_status fks_xport_create(int32_t n, double L, int32_t nx, int32_t ny, int32_t nz, double dx,
                            fks_xport* out);

/* Bytes of the device transport state: n^3 * (3 doubles + 3 int32 + 3 int32) plus the
 * per-axis shift table (3 n int32), each part rounded up to 256 bytes. */
fks_status fks_xport_sizes(fks_xport xp, size_t* state_bytes);

/* Binds the state buffer and enqueues its reset (s = 0, o = 0) on `stream`. */
fks_status fks_xport_bind(fks_xport xp, void* d_state, size_t state_bytes, void* stream);

/* One exact transport step of length dt: per velocity, t = s + v*dt,
 * delta = floor((t + dx/2)/dx), s = t - delta*dx, o += delta (FP64, this order), then
 * f_out[j][k] = f_in[(j - delta_k) mod box][k] for every cell j (a permutation per k).
 * dtype is FKS_F32 or FKS_F64; f_out must not overlap f_in. */
fks_status fks_transport(fks_xport xp, const void* f_in, void* f_out, int32_t dtype, double dt,
                         void* stream);

/* fks_transport with the move of f optional.  materialize = 0: only the offsets advance
 * (f_in, f_out unused, may be NULL); the integer shifts accumulate as pending in the state.
 * materialize != 0: the offsets advance, then f_out[j][k] = f_in[(j - D_k) mod box][k] with
 * D_k the shifts pending since f was last moved (this step's included), and the pending
 * shifts are cleared.  Shifts are permutations of the cells per velocity, so several
 * unmaterialised steps followed by one materialising call (dt = 0 adds no shift) give the
 * same f as materialising every step.  fks_transport is materialize = 1; fks_step and
 * fks_step_ex apply the pending shifts of earlier unmaterialised steps with their own
 * (their eq. DM_update then counts the total displacement). */
fks_status fks_transport_ex(fks_xport xp, const void* f_in, void* f_out, int32_t dtype, double dt,
                            int32_t materialize, void* stream);

/* n_steps split steps (eq. transport then eq. disc_relax) on the whole box:
 * f* = shift(f); f = f* + dt Q(f*).  f is updated in place; f_tmp is a caller buffer of
 * the same size.  d_moments (optional, [cells][5] FP64) receives the moments after the
 * last step.  The plan's n and dtype must match the transport's grid. */
fks_status fks_step(fks_plan plan, fks_xport xp, void* f, void* f_tmp, double dt,
                    int32_t n_steps, double* d_moments, void* stream);

/* Options of fks_step_ex.  A zero-initialised struct gives fks_step's behaviour. */
enum { FKS_COLL_BOLTZMANN = 0, FKS_COLL_BGK = 1 };
enum { FKS_INT_EULER = 0, FKS_INT_EXP = 1 };
typedef struct {
  int32_t collision;  /* FKS_COLL_BOLTZMANN: the plan's spectral Q (Appendix A);
                         FKS_COLL_BGK: Q = nu (E - f), E the Maxwellian of the cell's
                         macroscopic variables (Section 2.2.1) */
  int32_t integrator; /* FKS_INT_EULER: f = f* + dt Q(f*) (eq. disc_relax);
                         FKS_INT_EXP: the stiff-capable step of Section 2.1's remark:
                           BGK: E + (f* - E) exp(-nu dt) (exact relaxation at frozen E);
                           Boltzmann: f = f* + dt_eff Q(f*), dt_eff = (1 - exp(-mu dt)) / mu,
                           i.e. exp(-mu dt) f* + (1 - exp(-mu dt)) (f* + Q(f*)/mu), bounded for
                           every dt when mu bounds the collision frequency */
  double nu;          /* BGK collision frequency, > 0 */
  int32_t nu_density; /* BGK: 1 -> nu_j = nu * rho_j, 0 -> nu_j = nu */
  int32_t reserved;
  double mu;          /* FKS_INT_EXP with the Boltzmann operator: penalty mu > 0 */
  double* d_cons;     /* [cells][5] FP64 conservative variables U = dv^3 sum phi f, phi = (1, v,
                         |v|^2/2), in and out: on entry those of f (e.g. from fks_moments), updated
                         every step by eq. DM_update (Section 3: only the particles that changed
                         cell contribute).  Required for BGK; optional (NULL) for Boltzmann. */
  double* d_prim;     /* [cells][5] FP64 out: (rho, u_x, u_y, u_z, T) of the conservative variables
                         after the last step (ToPrimitive, (3/2) rho T = E - rho |u|^2 / 2);
                         from d_cons if given, else from the directly recomputed moments. NULL: none */
  double* d_moments;  /* [cells][5] FP64 out: moments of f after the last step, recomputed directly
                         from the masses (as in fks_step). NULL: none */
  void* q_last;       /* [cells][n^3] plan dtype out: the collision operator Q(f*) of the last step
                         (the increment applied is dt Q for Euler, dt_eff Q for the exponential
                         Boltzmann step, (1 - exp(-nu dt))/nu Q for exact BGK). NULL: none */
} fks_step_opts;

/* n_steps steps of the sequential FKS algorithm (Section 4.1) on the whole box, in place on
 * f: transport (f* = shift(f)), conservative variables by eq. DM_update (if d_cons), then the
 * collision stage chosen in opts (NULL opts: as fks_step).  f_tmp: caller buffer of f's size,
 * not overlapping f; after a Boltzmann step it holds f* of the last step (BGK: unspecified).
 * q_last must not overlap f or f_tmp.  The BGK operator uses the plan only for (n, L, dtype);
 * the plan need not be bound.  Errors: FKS_E_ARG for invalid options (BGK without d_cons,
 * nu or mu not positive and finite, unknown enums), as fks_step otherwise. */
fks_status fks_step_ex(fks_plan plan, fks_xport xp, void* f, void* f_tmp, double dt, int32_t n_steps,
                       const fks_step_opts* opts, void* stream);

void fks_xport_destroy(fks_xport xp);

/* ---- Learned surrogate of Q (an extension beyond the paper) ----------------------
 *
 * A multilayer perceptron maps the low Fourier modes of a cell's distribution to its
 * collision operator; cells whose surrogate output fails a conservation check are
 * recomputed with the spectral operator (Appendix A).  The check uses the moments the
 * paper's macroscopic variables are built from (Section 3): a correct Q has zero
 * mass, momentum and energy moments.
 *
 * Model: features x = Re, Im of fhat_k / fhat_0 for k in [-m/2, m/2-1]^3 (m = modes),
 * 2 m^3 values, fhat the normalised Fourier coefficients of f (Appendix A); layers
 * x -> SiLU(W1 x + b1) -> SiLU(W2 h + b2) -> W3 h + b3 = y (n^3 values); the
 * prediction is Q = s rho^2 y with rho = (2L)^3 fhat_0 the cell's density and s a
 * fixed output scale (Q is quadratic in f, so y depends on the shape of f only).  Weights are stored
 * row-major [out][in]; the host parameter vector is W1, b1, W2, b2, W3, b3 (FP32).
 * Matrix products run in BF16 on the matrix cores with FP32 accumulation; training
 * keeps FP32 master weights, Adam moments (beta1 0.9, beta2 0.999, eps 1e-8) and
 * minimises the mean of (y - t)^2 over batch and outputs.
 *
 * Sizes: 2 m^3 and n^3 multiples of 128; width a multiple of 128; batches of
 * training and fks_sur_forward are multiples of 128 up to max_batch (<= 65536).
 * Buffers: a parameter buffer (master weights, Adam moments, gradients, BF16
 * copies) and a workspace (activations), both caller-owned, 256-byte aligned. */
typedef struct fks_sur_s* fks_sur;
/* out_scale > 0 fixes the output units: Q = out_scale rho^2 y (choose it near the
 * typical size of Q / rho^2 so that the network's outputs are of order one).
 * flags FKS_SUR_CENTER: the network works in each cell's mean-velocity frame u (from
 * the FP64 moments of f): features are the coefficients of f(v + u) (fhat_k e^{i xi_k.u}),
 * targets are Q(v + u) / (s rho^2), and predictions are shifted back by the same exact
 * spectral shift (the spectral Q commutes with velocity shifts); n in {8, 16, 24, 32}. */
#define FKS_SUR_CENTER 1u
fks_status fks_sur_create(int32_t n, int32_t modes, int32_t width, int64_t max_batch, float out_scale,
                          uint32_t flags, fks_sur* out);
/* n_params = number of FP32 values of the host parameter vector */
fks_status fks_sur_sizes(fks_sur s, size_t* param_bytes, size_t* workspace_bytes, int64_t* n_params);
fks_status fks_sur_bind(fks_sur s, void* d_params, size_t param_bytes, void* d_workspace, size_t workspace_bytes,
                        void* stream);
/* Copies n_params host FP32 values in, resets Adam; synchronises `stream`. */
fks_status fks_sur_set_params(fks_sur s, const float* host, void* stream);
/* which = 0: parameters, 1: gradients of the last fks_sur_train_step; n_params host
 * FP32 values out; synchronises `stream`. */
fks_status fks_sur_get(fks_sur s, int32_t which, float* host, void* stream);
/* Features of n_cells distributions f (plan dtype, plan grid n == surrogate n):
 * x [n_cells][2 m^3] BF16 (device), rho [n_cells] FP32 (device), and, if mom != NULL,
 * the FP64 moments sum phi f dv^3, phi = (1, v, |v|^2/2), [n_cells][5] (device; required
 * for a centred surrogate).  The kept modes come from a pruned transform that reads f once
 * (n = 8, 16, 24, 32 with the mode counts the surrogate accepts there: 4; 4, 8; 8; 8);
 * other (n, m) pairs take the plan's full forward transform through its workspace. */
fks_status fks_sur_features(fks_sur s, fks_plan plan, const void* f, void* x, float* rho, double* mom,
                            int64_t n_cells, void* stream);
/* Training targets t = q / (s rho^2) ([n_cells][n^3] FP32, device; t may equal q); for a
 * centred surrogate t(v) = q(v + u) / (s rho^2) with u from mom (fks_sur_features).  The
 * plan supplies the grid (n, L). */
fks_status fks_sur_targets(fks_sur s, fks_plan plan, const float* q, const float* rho, const double* mom, float* t,
                           int64_t n_cells, void* stream);
/* y [batch][n^3] FP32 = network(x), x [batch][2 m^3] BF16, both device. */
fks_status fks_sur_forward(fks_sur s, const void* x, float* y, int64_t batch, void* stream);
/* One step on (x, t): forward, loss gradient into the gradient buffer, and, if
 * `update` != 0, one Adam step with learning rate lr.  t [batch][n^3] FP32 device.
 * If d_loss != NULL the batch loss (sum of squared errors / (batch n^3), FP64) is
 * written to device memory d_loss. */
fks_status fks_sur_train_step(fks_sur s, const void* x, const float* t, int64_t batch, float lr, int32_t update,
                              double* d_loss, void* stream);
/* Q for n_cells FP32 distributions: surrogate prediction, the indicator
 * r_j = max_i |sum_v phi_i Q_j| / sum_v |phi_i| |Q_j| over phi = 1, v, |v|^2/2 (FP64),
 * and, for every cell with r_j > threshold (threshold >= 0), the spectral Q of the
 * FP32 plan `plan` in its place (q = s rho^2 y elsewhere).  threshold < 0 disables the fallback.  Writes the
 * number of recomputed cells to *n_fallback (host) and, if d_indicator != NULL, r to
 * d_indicator [n_cells] (device FP64).  Synchronises `stream` once per max_batch
 * cells (to read the fallback count). */
fks_status fks_sur_infer(fks_sur s, fks_plan plan, const void* f, float* q, int64_t n_cells, double threshold,
                         int64_t* n_fallback, double* d_indicator, void* stream);
/* As fks_sur_infer, but the fallback takes a share of the cells ranked by an absolute error
 * estimate: a_j = r_j ||Q_j||_2 (the relative moment residual times the norm of the
 * surrogate's Q), and in every chunk of c <= max_batch cells the ceil(fallback_frac c)
 * cells with the largest a_j (all cells tied with the last one, and every NaN) take the
 * spectral Q.  A batch error budget is met with fewer fallbacks this way than by a
 * threshold on r_j, since the batch rel-L2 is dominated by the cells with the largest Q.
 * d_indicator (optional) receives a_j.  fallback_frac outside [0, 1]: FKS_E_ARG.
 * Synchronises `stream` twice per chunk (the residuals, the count). */
fks_status fks_sur_infer_ranked(fks_sur s, fks_plan plan, const void* f, float* q, int64_t n_cells,
                                double fallback_frac, int64_t* n_fallback, double* d_indicator, void* stream);
void fks_sur_destroy(fks_sur s);

/* ---- stream capture ---------------------------------------------------------------- */

/* Records every library call enqueued on `stream` between fks_graph_begin and
 * fks_graph_end into one hipGraph (no device work runs while recording), so that a
 * launch-bound sequence (e.g. many small Q evaluations or split steps) is replayed with
 * one fks_graph_launch.  Buffers and plans used in the recording must stay alive and
 * unchanged while the graph exists.  No library call synchronises the host while
 * recording, except fks_plan_bind and fks_profile_stop, which must not be recorded. */
typedef struct fks_graph_s* fks_graph;
fks_status fks_graph_begin(void* stream);
fks_status fks_graph_end(void* stream, fks_graph* out);
fks_status fks_graph_launch(fks_graph graph, void* stream);
void fks_graph_destroy(fks_graph graph);

/* ---- diagnostics ------------------------------------------------------------------ */

/* Per-kernel timing.  Between fks_profile_start and fks_profile_stop every kernel the
 * library enqueues is bracketed by a pair of hipEvents recorded on its launch stream.
 * Slots: 0 forward transform of f, 1 slab gain/loss convolutions, 2 synthesis and FP64
 * epilogue, 3 transport offsets, 4 transport shift, 5 moments.  fks_profile_stop
 * synchronises the recorded events (host blocks) and returns total milliseconds and
 * launch counts per slot.  Process-wide state; not for concurrent use from several
 * host threads. */
typedef struct {
  double total_ms[8];
  int64_t launches[8];
} fks_profile_stats;
fks_status fks_profile_start(void);
fks_status fks_profile_stop(fks_profile_stats* out);

const char* fks_last_error(void);
const char* fks_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FKS_H_ */
