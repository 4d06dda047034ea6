/* les.h -- C ABI of the MI355X (gfx950) LES residual / Runge-Kutta library.
 *
 * Implements the hot path of the solver described in "Strong Scaling of
 * Numerical Solver for Supersonic Jet Flow Configurations" (arXiv 2003.08746):
 * the explicit five-stage Runge-Kutta update (Sec. 3 end, Sec. 4, Alg. 2) of
 * the conserved vector Q = [rho, rho u, rho v, rho w, e] (Eq. 13) on one
 * structured curvilinear block, whose residual (Eq. 12, 14, 15) combines
 * centred inviscid and viscous fluxes through the grid metrics, Turkel-Vatsa
 * artificial dissipation and a static-Smagorinsky eddy viscosity (Eq. 3-11).
 *
 * Memory: every pointer named "device" is HIP device memory owned by the
 * caller.  The library owns only what it allocates in les_create (metrics,
 * stage buffers, reduction scratch) and frees it in les_destroy.  Pointers
 * named "host" are ordinary host memory.
 *
 * Streams: every call enqueues its kernels on the stream given to
 * les_create and returns without waiting, except where a host output is
 * requested (dt_out, norms, J_out); then the call synchronises that stream.
 *
 * Errors: every call returns an les_status; it never aborts the process.  A
 * readable message is available from les_last_error (per context) or
 * les_last_create_error (for a failed les_create).  A non-finite value found
 * by a reduction is reported as LES_ERR_NONFINITE by the call that
 * synchronises (the state is left in place for inspection).
 *
 * Threads: a context is not thread-safe; distinct contexts are independent.
 *
 * Field layout ("library layout"): a state or metric array holds nf fields
 * of field_elems doubles each.  Within a field, node (i, j, k) -- interior
 * indices 0..n-1, ghost indices -2, -1, n, n+1 -- sits at element
 *     origin + i + j * stride_j + k * stride_k
 * with the values returned by les_layout (i is contiguous; two ghost layers
 * per side as in Sec. 4, Fig. 3; rows are padded for alignment; padding
 * elements are never read).  "Dense padded layout" means the plain array
 * [nf][nk+4][nj+4][ni+4] with node (i, j, k) at ((k+2)(nj+4) + j+2)(ni+4) + i+2.
 */
#ifndef LES_H
#define LES_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct les_ctx les_ctx;

typedef enum {
  LES_OK = 0,
  LES_ERR_ARG = -1,       /* invalid argument (null pointer, size, value) */
  LES_ERR_HIP = -2,       /* a HIP runtime call failed */
  LES_ERR_NOMEM = -3,     /* device allocation failed */
  LES_ERR_NONFINITE = -4, /* NaN/Inf (or non-positive density/pressure) met */
  LES_ERR_STATE = -5      /* call not valid in the context's state */
} les_status;

typedef enum { LES_FP64 = 0, LES_MIXED = 1 } les_precision;

typedef enum { LES_BC_PERIODIC = 0, LES_BC_DIRICHLET = 1, LES_BC_PERIODIC_SUPERPOSED = 2, LES_BC_AXIS = 3 } les_bc;

/* Treatment of one boundary face of a Dirichlet direction (les_set_face). */
typedef enum { LES_FACE_FROZEN = 0, LES_FACE_CHARACTERISTIC = 1, LES_FACE_EXIT = 2, LES_FACE_FARFIELD = 3 } les_face_type;

/* One structured block.  ni, nj, nk >= 5 interior points.
 * bc[d] for d = i, j, k:
 *   LES_BC_PERIODIC  -- period-wrap (Sec. 3: azimuthal periodicity); the
 *                       ghost coordinates must be the period-shifted images;
 *   LES_BC_DIRICHLET -- ghost nodes keep the values the caller stored in the
 *                       state's ghost layers (frozen far field), unless
 *                       les_set_face gives a face another treatment.
 *   LES_BC_PERIODIC_SUPERPOSED -- periodic with the first and last nodes at
 *                       the same place (Sec. 3: the azimuthal direction of
 *                       the O-grid): period n - 1, node n - 1 takes node 0's
 *                       metrics and the ghosts wrap with period n - 1; node
 *                       n - 1 is updated like every interior node, so it stays
 *                       equal to node 0 when it starts equal (it counts in the
 *                       norms; the statistics along k count it once, with
 *                       node 0).  A ghost takes the node
 *                       reached by wrapping its ghost coordinates only.
 *   LES_BC_AXIS      -- (j only) the O-grid's centerline (Sec. 3): node j = 0
 *                       lies on the polar axis, j-hi is a Dirichlet side; k
 *                       must be LES_BC_PERIODIC_SUPERPOSED with nk - 1 even.
 *                       Ghost (i, -m, k) is the node across the axis,
 *                       (i, m, k + (nk-1)/2) (frozen where i is a ghost of a
 *                       Dirichlet side).  The residual does not advance the
 *                       axis nodes (R = 0 there); before each residual
 *                       evaluation and after each stage every axis node takes
 *                       the mean over k' = 0..nk-2 of the ring (i, 1, k')
 *                       (zero-order extrapolation, then the azimuthal
 *                       average), written in place in the caller's state.
 *                       On the axis xi/J = eta/J = 0 and J is infinite: the
 *                       eta node flux and spectral radius take their limit 0,
 *                       and the fourth difference of the face between the
 *                       axis and j = 1 takes the cross-axis value by linear
 *                       extrapolation (no five-point stencil across the
 *                       axis).  The CFL bound skips the axis.  With sgs = 2
 *                       the axis nodes (zero volume) carry no strain products
 *                       and no contractions, the axis column takes the ring
 *                       j = 1's coefficients and ghost column (i, -m) ring
 *                       column (i, m).  The adjoint entry points
 *                       differentiate the centerline condition and the
 *                       cross-axis ghosts.
 * xyz: device, dense padded layout [3][nk+4][nj+4][ni+4], coordinates on every
 * node including ghosts and edges (read during les_create only). */
typedef struct {
  int ni, nj, nk;
  int bc[3];
  const double *xyz;
} les_grid;

/* Metrics and Jacobian given by the caller (Sec. 4: each process reads or
 * computes them for its block).  m: device, dense padded layout
 * [10][nk+4][nj+4][ni+4]: xi_x/J, xi_y/J, xi_z/J, eta_x/J, ..., zeta_z/J, J,
 * valid on all nodes with indices in [-1, n]; read during les_create only.
 * A NULL les_metrics pointer, or m = NULL, lets les_create compute them from
 * the grid coordinates. */
typedef struct {
  const double *m;
} les_metrics;

/* Flow and scheme parameters (nondimensional).  Sec. 3, Eq. 2-11:
 *   gamma, R_gas (p = rho R T), Pr (kappa = mu Cp/Pr), Pr_sgs
 *   (kappa_sgs = mu_sgs Cp/Pr_sgs), Sutherland mu = mu_ref (T/T_ref)^1.5
 *   (1+S)/(T/T_ref+S) with S = S1/T_ref (S_suth).
 *   sgs = 0: mu_sgs = 0 (the paper's runs); sgs = 1: static Smagorinsky
 *   mu_sgs = rho (Cs Delta)^2 sqrt(2 S_ij S_ij), Delta = (1/J)^(1/3);
 *   sgs = 2: dynamic closure (Germano's identity with a test filter of width
 *   2 Delta, weights 1/4, 1/2, 1/4 per index, in the Favre form of Moin,
 *   Squires, Cabot and Lee; Lilly's least squares summed over the distinct
 *   planes of the periodic k direction (nk - 1 along a superposed one),
 *   clipped at 0): mu_sgs = C rho Delta^2 |S| and kappa_sgs =
 *   Cp D_T rho Delta^2 |S| with one C, D_T per (i, j) column, re-evaluated
 *   with every residual (Pr_sgs and Cs are then unused).
 *   CI >= 0 (sgs >= 1): Yoshizawa's isotropic SGS stress (Eq. 11)
 *   sigma_kk = 2 CI rho Delta^2 |S|^2, added as sigma_kk/3 to the pressure of
 *   the momentum and energy fluxes (Eq. 1); CI = 0 leaves it out.
 *   The adjoint entry points need sgs <= 1 (LES_ERR_STATE); they differentiate
 *   the isotropic SGS stress with the rest of the residual.
 * Turkel-Vatsa dissipation constants k2, k4 and anisotropy exponent alpha:
 *   D = Lam_face (eps2 dQ - eps4 d3Q), eps2 = k2 max(nu_a, nu_b),
 *   eps4 = max(0, k4 - eps2), nu = |p+ - 2p + p-| / (p+ + 2p + p-),
 *   Lam_d = lam_d [1 + sum_{e != d} (lam_e / lam_d)^alpha],
 *   lam_d = |U~_d| + c |grad d / J|.
 * cfl: time step used when les_rk_step gets dt <= 0:
 *   dt = cfl * min_interior 1 / (sum_d (|U_d| + c |grad d|)
 *                               + 2 max(4/3, gamma/Pr) (mu/rho) sum_d |grad d|^2).
 * prec: LES_FP64, or LES_MIXED (stage states, fluxes and dissipation in FP32;
 *   Q^n, the RK accumulation, metrics and all reductions in FP64). */
typedef struct {
  double gamma, Pr, Pr_sgs;
  double mu_ref, T_ref, S_suth;
  double R_gas;
  int sgs;
  double Cs;
  double k2, k4, alpha;
  double cfl;
  int prec;
  double CI;
} les_flow_params;

/* Create a context for one block (Alg. 2: read mesh, compute Jacobian and
 * metrics, create ghost points).  Without caller metrics they are computed on
 * the device from grid->xyz by the conservative (Thomas-Lombard)
 * central-difference form, which preserves a uniform flow exactly up to
 * rounding; in a periodic direction the ghost-layer metrics are copies of the
 * wrapped interior ones.  With metrics->m given, those are copied and
 * grid->xyz is ignored (it may be NULL).  hip_stream: a hipStream_t (NULL =
 * default stream).
 * Returns LES_ERR_ARG for a null out/grid/params, no coordinates and no
 * metrics, n < 5, a padded k plane so large that seven of them reach 2^29
 * elements (the stage kernel's 32-bit offsets from its per-segment base;
 * about 7.7e7 nodes per plane), bad bc (LES_BC_AXIS elsewhere than j, or
 * without a superposed k of odd nk), gamma <= 1,
 * R_gas <= 0, Pr <= 0, negative k2/k4/mu_ref/CI, sgs outside 0..2, unknown
 * prec; LES_ERR_NOMEM when the block's arrays (20 FP64 fields of
 * field_elems doubles, 10 more FP32 ones when mixed) do not fit.  sgs = 2
 * allocates the dynamic closure's work arrays (27 fields) here too. */
int les_create(les_ctx **out, const les_grid *grid, const les_metrics *metrics,
               const les_flow_params *params, void *hip_stream);

void les_destroy(les_ctx *ctx);

/* Library layout of state arrays (see top of file).  strides[0] = 1,
 * strides[1] = stride_j, strides[2] = stride_k; *origin = element offset of
 * interior node (0, 0, 0) within a field; *field_elems = field pitch;
 * *ghost = ghost layers per side (2: the five-point stencils of the
 * fourth-difference dissipation, Sec. 4).  Any output may be NULL. */
int les_layout(const les_ctx *ctx, long long strides[3], long long *origin, long long *field_elems, int *ghost);

/* Same layout without a context (for allocating before les_create). */
int les_layout_for(int ni, int nj, int nk, long long strides[3], long long *origin, long long *field_elems,
                   int *ghost);

/* Copy the library's metrics (library layout) to a caller array
 * (device, dense padded layout [10][nk+4][nj+4][ni+4]); nodes outside
 * [-1, n]^3 are written as 0. */
int les_get_metrics(les_ctx *ctx, double *dense_out);

/* Residual R(Q) = J * sum_d [F_{d,+1/2} - F_{d,-1/2}] - f * [i == i_f]
 * (Eq. 12: dQ/dt = -R), F = (H_a + H_b)/2 - D with node fluxes
 * H = inviscid - viscous contravariant flux (Eq. 15).
 * Q: device, library layout [5][field_elems], FP64; its ghost layers are
 *    filled in place (periodic wrap; Dirichlet ghosts untouched); interior
 *    values are not modified.
 * R: device, library layout [5][field_elems]; interior nodes written (when
 *    R is 16-byte aligned the fused stage kernel computes it and the ghost
 *    layers of R are set to 0; otherwise the one-node-per-thread reference
 *    kernel computes it and leaves them as they were).
 * norms: host double[10] or NULL: RMS of R per variable (5) then max |R| (5)
 *    over the interior. */
int les_residual(les_ctx *ctx, double *Q, double *R, double *norms);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * residual of les_residual, computed by the fused stage kernel, with its
 * norms reduced through a static device scratch instead of the context's
 * buffers, and written to device memory.  The call allocates nothing,
 * frees nothing and never synchronises.
 * Q: device, library layout, FP64; its ghost layers are filled in place.
 * R: device, library layout, 16-byte aligned (LES_ERR_ARG otherwise);
 *    interior written, ghost layers set to 0.
 * norms_dev: device double[10] or NULL: RMS of R per variable (5) then
 *    max |R| (5); a non-finite residual shows as NaN there (no status).
 * Limit: the scratch holds LES_NOALLOC_BLOCKS per-block partials (320 KB
 *    per GPU, held until the process ends); a context whose stage kernel
 *    runs more blocks gets LES_ERR_ARG.  Every call on one GPU shares that
 *    GPU's scratch, so calls that overlap on one GPU (different streams or
 *    threads) race; calls in one stream's order do not. */
#define LES_NOALLOC_BLOCKS 4096
int les_residual_noalloc(les_ctx *ctx, double *Q, double *R, double *norms_dev);

/* Time step dt (CFL rule above) of the interior of Q; dt_out: host. */
int les_cfl_dt(les_ctx *ctx, const double *Q, double *dt_out);

/* Constant source f on the plane i = i_f (dQ/dt = -R + f); f: device, dense
 * [5][nk][nj]; the library keeps its own copy.  f = NULL removes it. */
int les_set_forcing(les_ctx *ctx, const double *f, int i_f);

/* One step of Jameson's five-stage scheme (Sec. 4, Alg. 2):
 *   Q^(0) = Q^n;  Q^(l) = Q^(0) - alpha_l dt R(Q^(l-1)),  l = 1..5,
 *   alpha = (1/4, 1/6, 3/8, 1/2, 1);  Q^{n+1} = Q^(5),
 * with the ghost layers refreshed before every residual evaluation.
 * Q: device, library layout, FP64, 16-byte aligned (LES_ERR_ARG otherwise),
 *    in/out (interior updated in place; its periodic ghosts hold the wrap of
 *    Q^n on return).
 * dt > 0: used as is; dt <= 0: the CFL time step of Q^n (computed on the
 *    device; no host round trip unless dt_out is given).
 * dt_out: host or NULL.  norms: host double[10] or NULL, norms of R(Q^n).
 * stage_ckpt: device or NULL; FP64 [5 stages][5 fields][field_elems]
 *    receives the stage inputs Q^(0..4) (ghosts filled) for les_adjoint_step. */
int les_rk_step(les_ctx *ctx, double *Q, double dt, double *dt_out, double *norms, double *stage_ckpt);

/* nsteps steps of the five-stage scheme, each at the CFL time step of its
 * own Q^n (Sec. 4, Alg. 2: the time loop; the same result as nsteps calls of
 * les_rk_step with dt <= 0).  The dt rule is pointwise in the state, so the
 * last stage of each step reduces the next step's dt while Q^{n+1} is in
 * registers (the first step's dt takes a pass of its own): no separate pass
 * over Q and the metrics per step.  In LES_MIXED the last stage of each step
 * but the final one also writes the FP32 copy of Q^{n+1} that the next step's
 * stencil reads (where the ghost layers are periodic or frozen) in place of
 * the FP64 Q^n; the result is still that of les_rk_step, bit for bit.
 * Q: device, library layout, FP64, 16-byte aligned (LES_ERR_ARG otherwise),
 *    in/out as for les_rk_step; the caller must not touch it until the call's
 *    work on the stream is done.
 * nsteps >= 1 (LES_ERR_ARG otherwise).
 * dt_out: host double[nsteps] or NULL: the time step of every step (then
 *    nsteps <= LES_ADVANCE_DT_MAX, else LES_ERR_ARG).
 * norms: host double[10] or NULL: norms of R(Q^n) of the last step (only
 *    the last step reduces them; a non-finite state of an earlier step shows
 *    in the next step's dt reduction).
 * A non-finite dt or norm found on the way is reported as LES_ERR_NONFINITE
 * when dt_out or norms is given (the call then synchronises). */
#define LES_ADVANCE_DT_MAX 4096
int les_advance(les_ctx *ctx, double *Q, int nsteps, double *dt_out, double *norms);

/* Reverse (adjoint) of one les_rk_step at fixed dt, from its stage inputs:
 *   qbar <- Qbar;  acc = 0;  for l = 5..1:  acc += qbar;
 *      fbar += alpha_l dt qbar[plane i_f];
 *      qbar = -alpha_l dt (dR/dQ |_{Q^(l-1)})^T qbar;
 *   Qbar <- acc + qbar.
 * dR/dQ includes the ghost fill: periodic ghost adjoints are folded onto the
 * interior, face ghosts (les_set_face) are pulled back to their boundary
 * node through the face rule, frozen Dirichlet ghosts carry no dependence.
 * Non-smooth points
 * take the derivative of the active branch: d|x|/dx = sign(x) (0 at 0),
 * max(a, b) follows a when a >= b.
 * stage_ckpt: device, as written by les_rk_step with the same dt.
 * Qbar: device, library layout, FP64, in: dJ/dQ^{n+1} (interior), out: dJ/dQ^n
 *    (interior; ghost layers are used as scratch).
 * fbar: device, dense [5][nk][nj], accumulated, or NULL.
 * The first adjoint call allocates the work arrays (84 fields of field_elems
 * doubles; LES_ERR_NOMEM if they do not fit).  LES_ERR_STATE for the
 * dynamic closure, and for a block of 2^30 padded nodes or more.  With
 * LES_BC_AXIS the centerline condition on every stage input and on the
 * result is part of the step (the axis entries of Qbar come out 0), and a
 * forcing plane's axis row (i_f, 0, k) receives no fbar: the centerline
 * condition overwrites it after each stage. */
int les_adjoint_step(les_ctx *ctx, const double *stage_ckpt, double dt, double *Qbar, double *fbar);

/* Adjoint (vector-Jacobian product) of the residual at Q:
 *   Qbar = (dR/dQ)^T Rbar on the interior,
 * the building block of les_adjoint_step.  dR/dQ includes the ghost fill
 * (periodic ghost adjoints are folded onto the interior; frozen Dirichlet
 * ghosts carry no dependence) and uses the same non-smooth rules as
 * les_adjoint_step (and d|S|/dS = 0 at |S| = 0 in the eddy viscosity).
 * Q: device, library layout, FP64; its ghost layers are filled in place.
 * Rbar: device, library layout; only interior values are read.
 * Qbar: device, library layout; interior written (must not alias Q or Rbar).
 * Allocates the adjoint work arrays on first use (84 fields of field_elems
 * doubles, kept by the context). */
int les_residual_adjoint(les_ctx *ctx, double *Q, const double *Rbar, double *Qbar);

/* Probe objective on the plane i = i_p (interior of Q):
 *   *J_accum += weight * sum_{j,k} (p - p_inf)^2          (J_accum: device)
 *   Qbar[i_p plane] += weight * 2 (p - p_inf) dp/dQ       (Qbar: device or NULL)
 * with p = (gamma - 1)(e - (m_1^2 + m_2^2 + m_3^2) / (2 rho)); k runs over the
 * distinct planes (0..nk-2 along a superposed k direction, whose last plane
 * repeats the first). */
int les_probe_objective(les_ctx *ctx, const double *Q, int i_p, double p_inf, double weight, double *J_accum,
                        double *Qbar);

/* Boundary face of a LES_BC_DIRICHLET direction (Sec. 3: entrance, far field
 * and exit of the jet domain).  face: 0 = i-lo, 1 = i-hi, 2 = j-lo, 3 = j-hi,
 * 4 = k-lo, 5 = k-hi.  The rule applies, at every ghost refresh, to the ghost
 * nodes that lie outside the interior along that direction only (periodic
 * indices wrapped); ghosts of two Dirichlet directions stay frozen.  Both
 * ghost layers take the state built from the boundary node r next to the
 * face (zero-order extrapolation):
 *   LES_FACE_FROZEN          -- the ghosts keep the caller's values (default);
 *   LES_FACE_CHARACTERISTIC  -- entrance (flat-hat profile through 1-D
 *      characteristic relations): locally one-dimensional characteristics
 *      along the outward unit normal n of the face at r.  Supersonic outflow
 *      keeps r's state, supersonic inflow takes the outside state; otherwise
 *      the outgoing Riemann invariant u.n + 2c/(gamma-1) comes from r, the
 *      incoming u.n - 2c/(gamma-1) from outside, and entropy p/rho^gamma and
 *      tangential velocity from the upwind side (r when u.n >= 0);
 *   LES_FACE_EXIT            -- subsonic exit: pressure p_exit imposed,
 *      velocity and internal energy per unit mass of r kept; density and
 *      total energy follow (Eq. 2);
 *   LES_FACE_FARFIELD        -- far field (Riemann invariants, normal
 *      velocity extrapolated at zero order, fixed flow angle, the remaining
 *      properties from the jet Mach number): u.n = r's u.n; tangential
 *      velocity = the outside state's; c from the outside state's incoming
 *      invariant, c = (gamma-1)(u.n - (u_o.n - 2c_o/(gamma-1)))/2; entropy
 *      from outside when u.n < 0, from r otherwise.  A state with
 *      c <= 0 (an inflow faster than about 5 c_o) gives NaN, reported by the
 *      next synchronising call as LES_ERR_NONFINITE.
 * Q_outside: device, library layout, FP64, or NULL; when given, its ghost
 *    values become the outside state of every characteristic and far-field
 *    face (copied now; required before the first such face).
 * p_exit: imposed pressure (> 0) of an exit face; ignored otherwise.
 * LES_ERR_ARG for a bad face, type or pressure, or a face that is not on a
 * Dirichlet side (face 3, j-hi, is one with LES_BC_AXIS).
 * With LES_BC_AXIS the i-side faces fill their ghosts for j >= 0 only (those
 * below the axis are edges of two boundary directions and stay frozen), and
 * on the axis node, where the metric row of xi vanishes, n is the normalised
 * azimuthal mean of the unit normals of the ring j = 1 at that face.
 * The adjoint entry points differentiate the face rules (the outside state
 * and p_exit are constants). */
int les_set_face(les_ctx *ctx, int face, int type, const double *Q_outside, double p_exit);

/* Running flow statistics for the time- and azimuth-averaged mean-flow and
 * RMS profiles of Sec. 6 (the periodic k direction is the averaged one):
 *   acc[s][j][i] += sum over k = 0..nk_s-1 of phi_s(i, j, k),
 *   phi = (rho, u, v, w, p, u u, v v, w w, u v, u w, v w, p p),
 * with the primitives of Eq. 2: u_a = (rho u_a) / rho and
 * p = (gamma - 1)(e - rho |u|^2 / 2); nk_s = nk, or nk - 1 when k is
 * LES_BC_PERIODIC_SUPERPOSED (node nk - 1 is node 0's place, counted once).
 * After N calls the Reynolds means are acc / (N nk_s); e.g.
 * u_rms = sqrt(<u u> - <u>^2).
 * Q: device, library layout, FP64 (interior read only).
 * acc: device, dense [LES_STATS_NF][nj][ni], FP64, caller-owned; zero it
 *    before the first call.  The sums over k are taken in a fixed order, so
 *    repeated runs give identical results. */
#define LES_STATS_NF 12
int les_stats_accumulate(les_ctx *ctx, const double *Q, double *acc);

/* Mean-flow and RMS profiles of Sec. 6 from the sums of les_stats_accumulate,
 * and the potential core (Sec. 6: where the mean axial velocity is at least
 * a fraction, 95 % in the paper, of the inlet jet velocity):
 *   <phi> = acc / samples (samples = calls times nk_s of
 *   les_stats_accumulate),
 *   prof = (<rho>, <u>, <v>, <w>, <p>, u_rms, v_rms, w_rms, p_rms, <u'v'>),
 *   a_rms = sqrt(max(0, <a a> - <a>^2)), <u'v'> = <u v> - <u><v>;
 *   core[j][i] = 1 where <u> >= core_frac * u_jet, else 0 (u is the
 *   i-direction velocity, the jet axis).
 * acc: device, dense [LES_STATS_NF][nj][ni] (read only).
 * prof: device, dense [LES_PROF_NF][nj][ni], written.
 * core: device, unsigned char [nj][ni], or NULL (u_jet, core_frac unused).
 * Returns LES_ERR_ARG for null acc/prof, samples <= 0, or (with core) u_jet
 * <= 0 or core_frac outside (0, 1]. */
#define LES_PROF_NF 10
int les_stats_profiles(les_ctx *ctx, const double *acc, double samples, double u_jet, double core_frac,
                       double *prof, unsigned char *core);

const char *les_last_error(const les_ctx *ctx);
const char *les_last_create_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LES_H */
