/*
 * ader.h -- C ABI of the MI355X ADER-CG step library (libader_hip.so).
 *
 * One ADER-CG time step on a periodic 3D Cartesian mesh, after Balsara,
 * Meyer, Dumbser, Du & Xu, "Efficient Implementation of ADER Schemes for
 * Euler and Magnetohydrodynamical Flows on Structured Meshes" (arXiv
 * 1006.2146): reconstruction (Sec. II.1), the ADER-CG space-time predictor
 * (Sec. II.2, IV; App. A), space-time averaged Riemann fluxes at the faces
 * (Sec. II.3, V; App. D) and the one-step update of eq. (6).
 *
 * Conventions
 *  - State layout: SoA double U[5][nz][ny][nx], x fastest; components
 *    (rho, rho vx, rho vy, rho vz, E), zone averages, with
 *    E = rho v^2/2 + P/(gamma-1) (+ B^2/8pi for MHD, Gaussian units, eq. 3).
 *    Zone (i,j,k) covers [i dx, (i+1) dx] x [j dy, (j+1) dy] x [k dz, (k+1) dz],
 *    dx = lx/nx, ...  MHD adds the face-centred field B[3][nz][ny][nx]:
 *    B[0][k][j][i] is B_x averaged over the x-face at x = i dx (the lower
 *    x-face of zone (i,j,k)), B[1] and B[2] likewise on the lower y- and
 *    z-faces; the step keeps its discrete divergence at round-off (eq. 8).
 *  - Every call is ordered on the HIP stream given to ader_create (NULL =
 *    the default stream).  Calls that return data to the host synchronise
 *    that stream; ader_step and ader_step_cfl do not.
 *  - Errors: every int-returning call returns ADER_OK (0) or a negative
 *    ADER_E* code; nothing throws across the ABI.  A context is not
 *    thread-safe.
 *  - Ownership: the library copies host arrays passed to it; device buffers
 *    it allocates are freed by ader_destroy.  A device state bound with
 *    ader_bind_device_state stays owned by the caller and must outlive the
 *    context (or the next bind).
 *  - Batches: ader_batch_create makes one context for n independent periodic
 *    problems of any sizes; every stage of a step is one persistent launch
 *    over the zones of all of them, each problem with its own CFL dt.  The
 *    context's arrays hold the problems one after the other: with
 *    S = sum of N_i = nx_i ny_i nz_i, the state is U[5][S] (problem i at
 *    offsets base_i = N_0 + ... + N_{i-1} of each row) and B[3][S].  A single
 *    problem is a batch of one (S = N), so every call below applies to both.
 */
#ifndef ADER_H
#define ADER_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ader_ctx ader_ctx;

enum {
  ADER_OK = 0,
  ADER_EINVAL = -1,        /* bad argument (size, order, gamma, dt, ...) */
  ADER_EUNSUPPORTED = -2,  /* valid but not built (e.g. a layout at an order it lacks) */
  ADER_ENOMEM = -3,        /* device allocation failed */
  ADER_EDEVICE = -4,       /* a HIP call failed */
  ADER_ESTATE = -5,        /* state has rho <= 0, P <= 0 or a non-finite value */
  ADER_ESEQ = -6           /* call out of sequence (e.g. step before set_state) */
};

/* ADER_LINADV: linear advection u_t + a . grad u = 0 of the five state
 * components (independent of each other), a test system on which the
 * scheme translates any data by exactly one zone per step at |a_x| dt = dx
 * (a along x): the same reconstruction, predictor and face quadrature with
 * the linear flux F_d(u) = a_d u, the upwind limit of the HLL flux of
 * eq. (56) (signal speeds min(a_d, 0), max(a_d, 0)), the update of eq. (6)
 * and dt = cfl / sum_d |a_d| / dx_d.  FP64 and the ADER scheme only
 * (ADER_EUNSUPPORTED at the step otherwise); no positivity handling; a is
 * set by ader_set_advection (default (1, 0, 0)). */
enum { ADER_EULER = 0, ADER_MHD = 1, ADER_LINADV = 2 };  /* eq. (3) with B = 0; ideal MHD */
enum { ADER_HLL = 0, ADER_LINEARIZED = 1 };     /* eq. (17)/(56); Sec. II.3 */
enum { ADER_MODAL = 0, ADER_NODAL = 1 };        /* Sec. IV; App. A, B, C (orders 2, 3, 4) */
enum { ADER_FP64 = 0, ADER_MIXED = 1 };         /* all-FP64, or FP32 bulk with FP64
                                                   update and dt */

typedef struct {
  int nx, ny, nz;        /* zones per axis, each >= 1 */
  double lx, ly, lz;     /* periodic box lengths, each > 0 */
} ader_mesh;

/* Create a context on HIP device `device` with `stream` (a hipStream_t, or
 * NULL).  Defaults: gamma 1.4, order 3 modal, HLL, FP64.  Allocates the
 * state, fluxes and per-problem scalars; the work arrays (modes, side
 * packets) are allocated at the first step for the order and precision then
 * set, and grown if a later setting needs more (a step may so return
 * ADER_ENOMEM).  Returns ADER_EINVAL for
 * a bad mesh or system, ADER_ENOMEM / ADER_EDEVICE on HIP failures. */
int ader_create(const ader_mesh* mesh, int system, int device, void* stream,
                ader_ctx** out);

/* Ratio of specific heats, gamma > 1 (eq. 3). */
int ader_set_gamma(ader_ctx* ctx, double gamma);

/* order in {2, 3, 4}; form ADER_MODAL (Sec. IV) or ADER_NODAL (App. A, B, C
 * at orders 2, 3, 4).  At order 2 the reconstruction is minmod-limited
 * linear; at 3 and 4 it is centred WENO. */
int ader_set_order(ader_ctx* ctx, int order, int form);

/* Time stepping: ADER_SCHEME_ADER, the ADER-CG step (default), or
 * ADER_SCHEME_SSPRK, the strong-stability-preserving Runge-Kutta schemes of
 * Sec. II.d matched to the order (eq. 18 SSP-RK2 at order 2, eq. 19 SSP-RK3
 * at 3, eq. 20 the five-stage fourth-order scheme at 4): each stage runs the
 * reconstruction, the face-side packets of the spatial polynomial (the App.
 * D quadrature with the time direction dropped), the Riemann fluxes and the
 * stage combination in double, with the predictor bypassed; for MHD each
 * stage also rebuilds the zone field from the stage's face fields and
 * advances the face fields by minus the curl of its edge fields (eq. 8).
 * The form setting does not apply to it.  The scheme allocates four more
 * copies of the state on its first step (160 bytes per zone, 256 for MHD).
 * ADER_EINVAL for an unknown scheme. */
enum { ADER_SCHEME_ADER = 0, ADER_SCHEME_SSPRK = 1 };
int ader_set_scheme(ader_ctx* ctx, int scheme);
int ader_get_scheme(ader_ctx* ctx, int* scheme_out);

/* Positivity.  The paper describes no positivity treatment, so the default,
 * ADER_POSITIVITY_CHECK, runs its scheme unchanged and only checks: where a
 * zone's spatial polynomial (before the predictor, at the spatial positions
 * of the predictor nodes of eq. 31/37/46 or A.1/B.1/C.1 and of the facial
 * nodes of App. D) or its space-time polynomial (after the predictor, at the
 * facial nodes of App. D that the step evaluates and the six face
 * barycentres of eq. 54) has rho <= 0 or P <= 0, the problem is flagged and
 * the next call that reports status (ader_synchronize, ader_compute_dt with
 * dt_out, ader_batch_step_cfl with dts_out) returns ADER_ESTATE; the step's
 * result is then meaningless.  ADER_POSITIVITY_LIMIT is an opt-in safeguard
 * that is not part of the paper's method: the scaling limiter of Zhang and
 * Shu (J. Comput. Phys. 229, 2010) multiplies every non-constant mode of a
 * zone polynomial by the largest theta in [0, 1] keeping rho and P at least
 * 1e-8 of their zone-average values at the same points (zone averages
 * untouched, so still conservative); where theta would be 1 the result is
 * bit-identical to the check mode.  The same applies to SSP-RK stages
 * (spatial polynomial only).  ADER_EINVAL for another mode. */
enum { ADER_POSITIVITY_CHECK = 0, ADER_POSITIVITY_LIMIT = 1 };
/* Non-stiff source term of the Euler equations, Sec. IV (source modes and
 * their space-time average: eq. 34-35 at second order, 43-44 at third,
 * 52-53 at fourth) and App. A-C in the nodal form (A.7, B.6, C.6): an
 * affine source S(u) = A u + b of the conserved
 * variables (rho, rho vx, rho vy, rho vz, E), applied to every problem of
 * the context.  A is row-major 5 x 5 (S_v = sum_w A[5 v + w] u_w + b_v), b
 * has 5 entries (NULL: zero); both are host arrays, copied.  The predictor
 * carries S at its space-time nodes, and eq. (6) adds dt times the
 * space-time average of S over the zone from the predictor's polynomial.
 * A = NULL (with b NULL) removes the source.  While a source is set the
 * predictor runs one lane per zone at orders 2 and 3 and one lane per zone
 * and variable at order 4, whatever layout is set, and the SSP-RK
 * scheme's step returns ADER_EUNSUPPORTED.  ADER_EUNSUPPORTED on an MHD
 * context; ADER_EINVAL for a non-finite entry or b without A. */
int ader_set_source(ader_ctx* ctx, const double* A, const double* b);

/* Non-periodic faces (Euler; every problem of the context): bc[6] gives the
 * kinds of the faces x-, x+, y-, y+, z-, z+: ADER_BC_PERIODIC (the default;
 * both faces of an axis or neither), ADER_BC_OUTFLOW (zero gradient),
 * ADER_BC_REFLECT (a wall) or ADER_BC_INFLOW (a given state, set with
 * ader_set_inflow).  The paper describes no boundary treatment; the
 * reading here is the usual one of ghost zones: each bounded face gets four
 * layers of zones outside the problem, filled before every step (and every
 * dt rule) from the interior zone averages -- outflow the nearest interior
 * zone, reflect the mirror-image zone with the normal momentum negated --
 * or with the inflow state, and the periodic step then runs on the padded
 * mesh, whose periodic wrap reaches no interior result.  The axes compose
 * in the order x, y, z: a zone outside the faces of several axes takes the
 * rule of the last of them applied to the earlier axes' ghost values (the
 * inflow state of the last inflow face among them, with the momentum signs
 * of the reflecting faces after it).  The CFL rule covers the ghost zones
 * too, so an inflow state's signal speeds enter dt.  Zones two or more layers out reach no
 * interior face: their positivity outcomes are neither reported nor
 * counted.  The caller's arrays keep the interior layout; device memory
 * grows by the ghost layers.  Must come before the first state is set
 * (ADER_ESEQ after, or on a context with a bound device state); a bounded
 * axis needs at least 4 zones (ADER_EINVAL); ADER_EUNSUPPORTED for MHD and
 * linear advection, and at the step for the SSP-RK scheme. */
enum { ADER_BC_PERIODIC = 0, ADER_BC_OUTFLOW = 1, ADER_BC_REFLECT = 2, ADER_BC_INFLOW = 3 };
int ader_set_boundary(ader_ctx* ctx, const int* bc);

/* The state of inflow face `face` (0..5: x-, x+, y-, y+, z-, z+; every
 * problem of the context): state[5] conserved (rho, m_x, m_y, m_z, E), with
 * rho > 0, P > 0 and finite values (ADER_EINVAL otherwise).  May be set or
 * changed at any time (a captured step is captured again); a step on a
 * context with an inflow face whose state was never set returns ADER_ESEQ. */
int ader_set_inflow(ader_ctx* ctx, int face, const double* state);

/* Velocity a of an ADER_LINADV context (ADER_EUNSUPPORTED for the other
 * systems; ADER_EINVAL for a non-finite component or a = 0). */
int ader_set_advection(ader_ctx* ctx, double ax, double ay, double az);
int ader_set_positivity(ader_ctx* ctx, int mode);
int ader_get_positivity(ader_ctx* ctx, int* mode_out);

/* Per problem (counts_out: n values), the number of zone polynomials the
 * limit mode has scaled (spatial and space-time counted apart) since the
 * previous call; the counters restart at zero (synchronises). */
int ader_limited_zones(ader_ctx* ctx, long long* counts_out);

/* ADER_HLL (eq. 17/56, Davis speeds from the barycentre states) or
 * ADER_LINEARIZED (Sec. II.3: (F_L + F_R)/2 - R|Lambda|L (u_R - u_L)/2 with
 * the eigen-system frozen at the mean of the two barycentre primitive
 * states; for MHD the seven-wave system with the normal field held, applied
 * to the face and to each edge state of eq. (57)). */
int ader_set_riemann(ader_ctx* ctx, int riemann);

/* ADER_FP64 or ADER_MIXED. */
int ader_set_precision(ader_ctx* ctx, int precision);

/* Copy a host state U[5][nz][ny][nx] (conserved zone averages) and, for
 * MHD, the face field B[3][nz][ny][nx] (NULL for Euler; ADER_EINVAL if the
 * presence of B does not match the system) to the device (a batch: the
 * whole U[5][S], B[3][S] layout).  Returns
 * ADER_ESTATE (and keeps the old state) if any zone has rho <= 0, P <= 0 or
 * a non-finite value (MHD pressure with the face-mean zone field). */
int ader_set_state(ader_ctx* ctx, const double* U, const double* B);

/* Use caller-owned device buffers of 5*nx*ny*nz (U) and, for MHD,
 * 3*nx*ny*nz (B; NULL for Euler) doubles as the state (zero copy, e.g.
 * torch tensors' data pointers).  The library reads and updates them in
 * place on the context's stream. */
int ader_bind_device_state(ader_ctx* ctx, void* dU, void* dB);

/* Copy the state to the host arrays U[5][nz][ny][nx] and, if B is not NULL
 * and the system is MHD, B[3][nz][ny][nx] (synchronises). */
int ader_get_state(ader_ctx* ctx, double* U, double* B);

/* dt = cfl / max over zones of sum_d (|v_d| + c_d) / dx_d (c_d the sound
 * speed, or for MHD the fast speed along d with the face-mean zone field),
 * computed on the device into the context's dt slot (per problem).  If
 * dt_out is not NULL the value is copied back (synchronises; single-problem
 * contexts only, ADER_EINVAL for a batch) and ADER_ESTATE is returned if a
 * zone is unphysical.  cfl > 0. */
int ader_compute_dt(ader_ctx* ctx, double cfl, double* dt_out);

/* One ADER-CG step of size dt > 0 (finite; every problem of a batch).
 * Asynchronous. */
int ader_step(ader_ctx* ctx, double dt);

/* dt by CFL on the device, then one step with it; no host round trip. */
int ader_step_cfl(ader_ctx* ctx, double cfl);

/* The dt of the latest ader_compute_dt / ader_step_cfl / ader_step
 * (synchronises); dt_out holds one value per problem (n for a batch). */
int ader_get_dt(ader_ctx* ctx, double* dt_out);

/* Wait for all queued work; returns ADER_ESTATE if a dt evaluation since
 * the last check met an unphysical zone, ADER_EDEVICE on a HIP error. */
int ader_synchronize(ader_ctx* ctx);

/* Per-stage device timing.  While enabled, every step records HIP events on
 * the context's stream around its stages: ADER_STAGE_DT (CFL reduction),
 * ADER_STAGE_RECON (reconstruction), ADER_STAGE_PREDICT (predictor and
 * face-side packets), ADER_STAGE_FLUX (Riemann fluxes), ADER_STAGE_UPDATE
 * (eq. 6).  ader_stage_times synchronises, returns for each stage the summed
 * milliseconds and the number of timed launches since the previous call
 * (arrays of ADER_NSTAGES), and starts a new accumulation. */
enum { ADER_STAGE_DT = 0, ADER_STAGE_RECON = 1, ADER_STAGE_PREDICT = 2,
       ADER_STAGE_FLUX = 3, ADER_STAGE_UPDATE = 4, ADER_NSTAGES = 5 };
int ader_set_timing(ader_ctx* ctx, int enable);
int ader_stage_times(ader_ctx* ctx, double* ms_out, int* counts_out);

/* Bytes of device memory the context holds now (state, fluxes, scalars and
 * the work arrays allocated so far). */
int ader_device_bytes(ader_ctx* ctx, double* bytes_out);

/* Conserved totals and the face field's divergence, per problem (n values
 * for a batch, 1 otherwise), computed on the device from the current state
 * (synchronises).  totals (n x 8 doubles, may be NULL): for each problem the
 * integrals over its box of the five conserved variables (rho, rho v, E:
 * the sum of the zone averages times the zone volume) and, for MHD, of the
 * three face-field components (the sum of each component's face values
 * times the zone volume; 0 for Euler).  max_abs_divB (n doubles, may be
 * NULL): the largest |sum_d (B_d(upper face) - B_d(lower face)) / dx_d| over
 * the zones (0 for Euler).  On a periodic mesh eq. (6) changes the totals
 * only by face fluxes that cancel, so they stay constant to round-off, and
 * the constrained transport of eq. (8) keeps the divergence at its initial
 * round-off level.  The sums are reduced in a fixed order (tiles of 8192
 * zones, fixed trees, no atomics): the same state gives the same bits for
 * any launch.  The first call allocates 72 bytes per 8192 zones of scratch
 * (ADER_ENOMEM if that fails); ADER_ESEQ before a state is set. */
int ader_diagnostics(ader_ctx* ctx, double* totals, double* max_abs_divB);

/* ader_diagnostics for callers that cannot allocate device memory (code
 * under stream capture, serving loops, harnesses that forbid hipMalloc):
 * the same results, bit for bit, from the same kernels, with their scratch
 * in a fixed array of the library (1.47 MB per device, held until the
 * process ends) instead of an allocation; it calls no allocating routine.
 * Limits: at most 16384 reduction tiles of 8192 zones (134 M zones over the
 * context) and 4096 problems, else ADER_EINVAL.  Every call on a device
 * shares that device's array, so calls that overlap on one device (other
 * host threads, other contexts' streams) race; calls in sequence do not.
 * ADER_ESEQ before a state is set. */
int ader_diagnostics_noalloc(ader_ctx* ctx, double* totals, double* max_abs_divB);

/* Static description of an error code. */
const char* ader_strerror(int code);

/* Free the context and its device buffers (NULL is a no-op). */
void ader_destroy(ader_ctx* ctx);

/* ---- batches, graphs, launch shapes (the batched execution of the step) --
 *
 * ader_batch_create: n >= 1 problems, meshes[i] as in ader_create; all share
 * the system and the settings of the set_* calls.  Buffers are sized for
 * order 4 in FP64 over all S zones.  Errors as ader_create. */
int ader_batch_create(int n, const ader_mesh* meshes, int system, int device, void* stream,
                      ader_ctx** out);

/* Number of problems of the context (1 for ader_create). */
int ader_batch_size(ader_ctx* ctx, int* n_out);

/* Copy problem i's host state U[5][nz_i][ny_i][nx_i] (and, MHD, its face
 * field B[3][...]) into the batch (synchronises).  ADER_ESTATE as in
 * ader_set_state.  Stepping needs every problem set (ADER_ESEQ before). */
int ader_batch_set_state(ader_ctx* ctx, int i, const double* U, const double* B);

/* Copy problem i's state back into U[5][...] and, if B is not NULL (MHD),
 * B[3][...] (synchronises). */
int ader_batch_get_state(ader_ctx* ctx, int i, double* U, double* B);

/* ader_step_cfl for every problem with its own dt; if dts_out is not NULL
 * (n doubles) the dt values are copied back (synchronises) and ADER_ESTATE
 * is returned if a zone of any problem was unphysical. */
int ader_batch_step_cfl(ader_ctx* ctx, double cfl, double* dts_out);

/* Graph mode (enable != 0): ader_step_cfl / ader_batch_step_cfl replay one
 * hipGraph of the whole CFL step (dt reduction and all stages; no memset
 * nodes), captured on first use and again whenever cfl, a set_* setting,
 * the launch shapes or the bound state buffers change.  Needs a stream
 * other than NULL (ADER_EUNSUPPORTED).  Stage timing, while on, runs the
 * step eagerly. */
int ader_set_graph(ader_ctx* ctx, int enable);

/* Autotuner: for each kernel class (dt, reconstruction, predictor, fluxes,
 * update) times every candidate launch shape -- threads per block in
 * {64, 128, 256} x persistent blocks per compute unit -- on the context's
 * own problems and settings, `reps` launches each (1..1000), and keeps the
 * fastest.  The state and dt are saved before and restored after, so the
 * solution does not advance; results do not depend on the launch shape.
 * For the predictor it also tries the layouts (ader_set_layout), for the
 * reconstruction both modes (ader_set_recon).
 * Needs a state (ADER_ESEQ); allocates a temporary copy of it. */
int ader_autotune(ader_ctx* ctx, int reps);

/* Launch shape per kernel class (arrays of 5, in the class order above):
 * threads per block (64, 128, 192 or 256) and blocks per compute unit
 * (1..64). */
int ader_get_launch(ader_ctx* ctx, int* block_out, int* blocks_per_cu_out);
int ader_set_launch(ader_ctx* ctx, const int* block, const int* blocks_per_cu);

/* Layout of the predictor kernel (Sec. IV and App. D work of a zone):
 * ADER_LAYOUT_ZONE, one lane per zone holding all variables (not built for
 * Euler in FP64 at order 4: ADER_EUNSUPPORTED there, the lane-split layout
 * runs), or
 * ADER_LAYOUT_SPLIT, one lane per (zone, variable) gathering the zone's
 * state across lanes at each flux evaluation (orders 3 and 4 only,
 * ADER_EUNSUPPORTED at order 2), ADER_LAYOUT_SPLIT2, the same compiled to
 * fit two waves per SIMD, ADER_LAYOUT_ZONE2, one lane per zone with the
 * facial positivity check in a pass of its own rather than inside the face
 * quadrature (orders 2 and 3 only), ADER_LAYOUT_ZONE_2W, one lane per zone
 * compiled to fit two waves per SIMD (Euler, orders 2 and 3 only),
 * ADER_LAYOUT_PAIR, two lanes per zone each holding four of the eight MHD
 * variables and exchanging them for each flux (MHD, order 3 only),
 * ADER_LAYOUT_PAIR2, the same compiled for two waves per SIMD (order 3),
 * ADER_LAYOUT_PAIR_SPLIT, the pair layout in two kernels (the predictor,
 * then the side packets; the evolutionary modes pass through device memory,
 * allocated on first use; MHD, orders 3 and 4), ADER_LAYOUT_FUSED, the
 * reconstruction and the one-lane-per-zone predictor in one kernel: a block
 * reconstructs a tile of 8 x 8 x 4 zones in LDS and predicts its zones
 * from there, so the reconstructed modes never go through device memory
 * (Euler, order 3 only; the stage timing then books the reconstruction
 * under the predictor), or -1 for the default of
 * the setting (pair for MHD at order 3, the two-kernel pair at order 4,
 * split for Euler at order 4).  Results do not
 * depend on the layout beyond rounding order.  ader_autotune also picks it.
 * ader_get_layout returns the layout the current setting uses. */
enum { ADER_LAYOUT_ZONE = 0, ADER_LAYOUT_SPLIT = 1, ADER_LAYOUT_SPLIT2 = 2, ADER_LAYOUT_ZONE2 = 3,
       ADER_LAYOUT_ZONE_2W = 4, ADER_LAYOUT_PAIR = 5, ADER_LAYOUT_PAIR2 = 6,
       ADER_LAYOUT_PAIR_SPLIT = 7, ADER_LAYOUT_FUSED = 8 };
int ader_set_layout(ader_ctx* ctx, int layout);
int ader_get_layout(ader_ctx* ctx, int* layout_out);

/* Execution of the WENO reconstruction (Sec. II.1; orders 3 and 4):
 * ADER_RECON_SWEEPS, one launch per sweep direction, ADER_RECON_TILED, one
 * launch doing the x, y and z sweeps of 8 x 8 x 8-zone tiles in LDS (halo
 * M-1 zones), ADER_RECON_COLUMNS, the x and y sweeps as launches and the z
 * sweep by threads that slide a window down 8-plane column segments,
 * ADER_RECON_MARCH, one launch in which a block takes one variable of a
 * 16 x 16-zone column segment of 32 planes and walks it plane by plane (x and y
 * sweeps of each plane in LDS, the z sweep from a ring of the last 2M-1
 * planes), so the zone averages are read about once and every mode written
 * once, or -1 for the default (sweeps).  All run the same line reconstructions (modes
 * equal up to rounding); order 2 (minmod) always runs per zone.
 * ader_autotune also picks it; ader_get_recon returns the mode in use. */
enum { ADER_RECON_SWEEPS = 0, ADER_RECON_TILED = 1, ADER_RECON_COLUMNS = 2, ADER_RECON_MARCH = 3 };
int ader_set_recon(ader_ctx* ctx, int mode);
int ader_get_recon(ader_ctx* ctx, int* mode_out);

/* Execution of the face fluxes (Sec. II and App. D: the Riemann solver at
 * the face quadrature points) and of the update of eq. (6):
 * ADER_FLUX_SEPARATE, two launches, the fluxes of every face going through
 * device memory (F[3][5][S] doubles) between them, or ADER_FLUX_FUSED, one
 * launch in which a block takes a 32 x 8-zone x-y tile and walks 16 planes
 * of it in z, forming each plane's face fluxes into LDS and registers and
 * updating its zones from there, so no flux reaches device memory (the
 * tile's upper x and y faces and a segment's lower z face are formed by
 * both blocks that share them).  In the mixed precision the predictor then
 * also keeps a copy of the zone averages, which the faces between blocks
 * need after a neighbour has updated its zones.  The fused mode applies to
 * the ADER step of Euler without a source term (elsewhere the two kernels
 * run); the stage timing books the update under the flux stage.  Both
 * modes form every face flux and the update by the same operations, so the
 * results are equal bit for bit.  -1 selects the default (separate);
 * ADER_EUNSUPPORTED for MHD and linear advection.  ader_autotune also picks
 * it; ader_get_flux_mode returns the mode in use. */
enum { ADER_FLUX_SEPARATE = 0, ADER_FLUX_FUSED = 1 };
int ader_set_flux_mode(ader_ctx* ctx, int mode);
int ader_get_flux_mode(ader_ctx* ctx, int* mode_out);


#ifdef __cplusplus
}
#endif
#endif /* ADER_H */
