/*
 * tlb.h -- C interface of the MI355X (gfx950) library that steps the vielbein lattice
 * Boltzmann binary-fluid model on a periodic torus (Ambrus, Busuioc, Wagner, Paillusson,
 * Kusumaatmaja, arXiv:1904.10070).
 *
 * State.  Sixteen velocity-space populations f_k(theta_q, phi_s) of the Q = 4 Hermite set
 * (section II C, eq. vmatrix) plus the Cahn-Hilliard order parameter phi(theta_q, phi_s)
 * (section II B, eq. CH) on the node grid theta_q = 2 pi q / n_theta, phi_s = 2 pi s / n_phi,
 * periodic in both angles (section II C, after eq. boltz_tor).  Population index
 * k = 4 i + j: i picks v^theta-hat = v_i, j picks v^phi-hat = v_j, with
 * v = (-sqrt(3+sqrt6), -sqrt(3-sqrt6), +sqrt(3-sqrt6), +sqrt(3+sqrt6)).
 *
 * Layout.  Every field lives in device memory as a dense structure of arrays of the
 * precision's element type T (float for precision 32, double for 64):
 *     f   : T[16][n_theta][n_phi]       (phi index fastest)
 *     phi, n, u_theta, u_phi, mu : T[n_theta][n_phi]
 * u_theta, u_phi are the orthonormal (vielbein) components of the fluid velocity.
 * Precision 32 stores each population as its deviation from the rest equilibrium of a
 * reference density, f_k - n_ref w_i w_j (w = (3 -/+ sqrt6)/12, the weights of the velocity
 * set; n_ref = the area-weighted mean density of the state loaded by tlb_set_state, rounded to
 * two significant digits): the stored values are a few per cent of f, so FP32 rounding loses
 * far less of the small per-step increments (it otherwise biases the mass by about 1e-2 over
 * 1e6 steps).  tlb_set_state and tlb_get_state convert; a caller reading an FP32 grid's f
 * buffers directly sees deviations.  Precision 64 stores f_k itself.
 * Precision 32 stores the order parameter as a base plane (owned by the library) plus the
 * phi buffers, which hold deviations from it: the per-step increments of phi in the bulk,
 * where phi sits near +-1, are far below half an ulp of 1 and would be rounded away on phi
 * itself (biasing the sum of phi), while on the small deviations they keep their precision.
 * After every 32nd time step counted from the last tlb_set_state (or tlb_restrict into the
 * grid; every learned step also ends with one) the deviation is moved into the base exactly
 * (error-free two-sum), so a state's bits do not depend on how its steps were split into
 * calls or checked runs.  tlb_set_state, tlb_get_state, tlb_get_moments and the diagnostics convert; a
 * caller reading an FP32 grid's phi buffers directly sees deviations.
 * Arithmetic in precision 32 differs from precision 64 in two places beyond the element type:
 * 1/n is the hardware reciprocal (1 ulp), and the Runge-Kutta combination of phi is taken on
 * the deviations as d^n + b (d_s - d^n + dt L) rather than (1 - b) phi^n + b (phi_s + dt L)
 * (the same value).  Grids whose three state copies exceed 1 GiB write their stage outputs
 * with streaming (nontemporal) stores.
 *
 * Ownership.  The caller allocates and owns every buffer passed in (state buffers, moment
 * buffers); they must outlive the grid handle.  The library owns its per-row geometry table,
 * small reduction workspaces, the step graphs, and (precision 32) the order parameter's base
 * plane and (TLB_CH4) three prepass planes, all freed by tlb_destroy.
 *
 * Streams.  All work is enqueued on the HIP stream given at creation (NULL = the default
 * stream), in call order, asynchronously with respect to the host.  The calls that return
 * host values wait for the stream (tlb_invariants, tlb_structure_length, tlb_autotune,
 * tlb_diagnostics with a host output, tlb_set_state in precision 32, tlb_step_n with
 * check_every > 0); the others do not.  A handle must not be used from two host threads at
 * once.
 *
 * Errors.  Every int32_t-returning function returns TLB_OK (0) or a negative TLB_E* code;
 * tlb_last_error() then returns a message for the calling thread.
 */
#ifndef TLB_H
#define TLB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TLB_OK 0
#define TLB_EINVAL (-1)     /* bad argument: parameters out of range, NULL where required   */
#define TLB_ENOMEM (-2)     /* the library's own small allocation failed                    */
#define TLB_EHIP (-3)       /* a HIP runtime call or kernel launch failed                    */
#define TLB_ENONFINITE (-4) /* NaN or Inf in the state (tlb_invariants, or a check of        *
                             * tlb_step_n under check_every)                               */
#define TLB_EUNSTABLE (-5)  /* dt exceeds the explicit stability bound of tlb_stable_dt     *
                             * (reported only for grids created with TLB_STRICT_DT)         */

/* flags */
#define TLB_FLAT 1u            /* flat limit: J = R and G = 0 (a doubly periodic plane with   *
                                * spacings R dphi and r dtheta)                              */
#define TLB_CH_NO_ADVECTION 2u /* drop -div(u phi) from the Cahn-Hilliard equation          */
#define TLB_NO_GRAPH 4u        /* tlb_step_n launches every kernel itself instead of replaying *
                                * prebuilt graphs of the step loop (same results, bit-exact)  */
#define TLB_WENO5 8u           /* advection face values by the nonlinear WENO-5 reconstruction *
                                * (Jiang-Shu weights, eps = 1e-6) instead of the linear UW5   *
                                * one; tiles of 8 rows only, not in batches                   */
#define TLB_STRICT_DT 16u      /* tlb_create_torus_grid refuses (TLB_EUNSTABLE) a dt above the *
                                * bound of tlb_stable_dt                                       */
#define TLB_CH4 32u            /* Cahn-Hilliard at fourth order: the surface Laplacian of mu   *
                                * and of M mu in conservative staggered form along theta and   *
                                * the five-point fourth-order difference along phi; fourth-    *
                                * order central flux differences for -div(u phi) and grad mu.  *
                                * mu and the advection fluxes come from a prepass per stage    *
                                * (the library allocates 3 planes for them); tiles of 8 rows   *
                                * only, not in batches, not with TLB_WENO5                     */

/* Physical and numerical parameters, in the paper's units (k_B T = m = 1, so the kinematic
 * viscosity is nu = tau, eq. nu).
 *   r, R        minor and major radius, 0 < r < R (a = r/R < 1 keeps R + r cos theta > 0)
 *   n_theta     nodes round the tube, n_phi nodes round the symmetry axis (each >= 1)
 *   A, kappa    Landau free-energy parameters (eq. Landau), kappa >= 0
 *   M           Cahn-Hilliard mobility (eq. CH), >= 0
 *   tau         BGK relaxation time (> 0)
 *   dt          time step of the three-stage SSP Runge-Kutta integrator (> 0)
 *   precision   32 or 64: element type T of every device buffer of this grid
 *   flags       TLB_FLAT | TLB_CH_NO_ADVECTION | TLB_NO_GRAPH | TLB_WENO5 | TLB_STRICT_DT |
 *               TLB_CH4
 *   check_every 0: tlb_step_n does not look at the state.  K > 0: tlb_step_n counts the
 *               non-finite values of the state (f and phi) after every K steps of a call and
 *               after its last step, waits for the stream at its end and returns
 *               TLB_ENONFINITE if any count was non-zero (the steps after a failed check still
 *               run; nothing is rolled back).  Each check reads the state once, about 1/8 of
 *               the memory traffic of a step.                                               */
typedef struct tlb_params {
  double r, R;
  int32_t n_theta, n_phi;
  double A, kappa, M, tau, dt;
  int32_t precision;
  uint32_t flags;
  int32_t check_every;
} tlb_params;

/* The three state copies the integrator cycles through (device pointers, each of the
 * layout above).  Copy 0 holds the current state between calls; copies 1 and 2 hold
 * Runge-Kutta stage values and are scratch to the caller.  All six must be distinct.
 * Rows are dense (the row pitch is n_phi elements): the halo copies of the stage kernel
 * handle rows of any length, so no padding is asked for.                                  */
typedef struct tlb_buffers {
  void* f[3];
  void* phi[3];
} tlb_buffers;

typedef struct tlb_grid tlb_grid;

/* Explicit stability bound of the time step for these parameters (host only, no GPU work):
 * the smallest of
 *   upwind advection at Courant number 1 along both angles over the smallest spacings,
 *     1 / (v_max (1/h_theta + 1/h_phi)),  v_max = sqrt(3 + sqrt 6) (eq. vmatrix),
 *     h_theta = r dtheta, h_phi = (R - r) dphi (the inner equator; R dphi if TLB_FLAT);
 *   BGK relaxation, 2.5 tau (the real-axis limit 2.51 of SSP-RK3 for the decay rate 1/tau);
 *   Cahn-Hilliard, 2.51 / (M kappa S^2 + 2 M |A| S), S = 4/h_theta^2 + 4/h_phi^2 the largest
 *     eigenvalue of the five-point surface Laplacian (eq. CH with eq. mu linearised about
 *     phi = 0).
 * The paper lowers its time step tenfold for the thick torus because of the small spacing at
 * its inner equator (section IV); the bound falls with that spacing in the same way.  Only
 * r, R, n_theta, n_phi, A, kappa, M, tau and flags are read.  Errors: TLB_EINVAL (the
 * parameters as for creation, dt aside).                                                   */
int32_t tlb_stable_dt(const tlb_params* params, double* dt_max);

/* Validate the parameters, build the per-row geometry of the torus (appendix A: metric
 * factors r and J = R + r cos theta at the nodes and half-nodes, connection coefficient
 * G = Gamma_{theta phi phi} = sin theta / J, eq. conn_torus) and the velocity-space
 * constants (eq. vmatrix, the weights w_k and the derivative kernel K^H of section II C),
 * and return a handle.  Errors: TLB_EINVAL (r <= 0, R <= r, a grid side < 1, dt, tau <= 0,
 * kappa or M < 0, precision not 32/64, check_every < 0, any NULL pointer or buffer),
 * TLB_EUNSTABLE (TLB_STRICT_DT set and dt > tlb_stable_dt), TLB_ENOMEM, TLB_EHIP.         */
int32_t tlb_create_torus_grid(const tlb_params* params, const tlb_buffers* buffers,
                              void* hip_stream, tlb_grid** out);

/* Load a state.  phi (required) is copied into state copy 0.  If f is non-NULL it is copied
 * as the populations; otherwise the populations are set to the discrete equilibrium
 * f_eq(n, u) of eq. feq from the moment fields n, u_theta, u_phi (then all three required).
 * Device pointers of element type T; stream-ordered for precision 64; precision 32 waits for
 * the stream (it measures the state's mean density to choose the reference density of its
 * storage, see Layout).  Errors: TLB_EINVAL, TLB_EHIP.                                      */
int32_t tlb_set_state(tlb_grid* grid, const void* f, const void* phi, const void* n,
                      const void* u_theta, const void* u_phi);

/* Advance n_steps >= 0 time steps.  One step is three right-hand-side evaluations of the
 * semi-discrete system -- moments; chemical potential mu = A phi (phi^2 - 1) - kappa
 * Delta_S phi (eq. mu); interface force n F = -phi grad mu (eq. pbin); BGK relaxation to
 * f_eq (eq. feq); finite-difference advection along the vielbein frame with the metric
 * factors r and J (eq. boltz_tor); velocity-space force and connection terms through K^H
 * (section II C); Cahn-Hilliard right-hand side -div(u phi) + M Delta_S mu (eq. CH) --
 * combined by the SSP Runge-Kutta stages.  Stream-ordered, asynchronous (unless check_every
 * > 0, see tlb_params).  The steps run in runs of at most 32 that end where the FP32 order
 * parameter is folded into its base (every 32nd step since tlb_set_state; FP64 grids: every
 * 32 steps of the call).  Unless TLB_NO_GRAPH, each run replays graphs of kernel nodes of
 * 32, 16, 8, 4, 2 and 1 steps (the binary digits of its length), all built together on the
 * first call that needs one and kept, so that no later call builds a graph; the graphs keep
 * the buffer pointers given at creation.
 * Errors: TLB_EINVAL, TLB_EHIP (launch or graph failure), TLB_ENONFINITE (check_every > 0
 * and a check of this call found NaN or Inf).                                             */
int32_t tlb_step_n(tlb_grid* grid, int64_t n_steps);

/* Moments of the current state into caller buffers (any may be NULL): density n = sum f,
 * velocity u = sum f v / n (section II C), the order parameter phi, and the chemical
 * potential mu (eq. mu).  Device pointers of element type T; stream-ordered.               */
int32_t tlb_get_moments(tlb_grid* grid, void* n, void* u_theta, void* u_phi, void* phi,
                        void* mu);

/* Copy the current state (checkpoint) into caller buffers (either may be NULL).
 * tlb_set_state(grid, f, phi, ...) with the same buffers restores it: exactly in precision
 * 64, to the rounding of the conversion from and to the stored deviations in precision 32.  */
int32_t tlb_get_state(tlb_grid* grid, void* f, void* phi);

/* Conservation diagnostics of the current state, reduced in FP64 in a fixed order (hence
 * bit-reproducible): out[0] = total mass sum_q,s r J_q dtheta dphi n, out[1] = the same
 * area-weighted sum of phi, out[2] = number of non-finite values in (f, phi).  out is a
 * host array of 3 doubles.  Waits for the stream.  Returns TLB_ENONFINITE if out[2] > 0.  */
int32_t tlb_invariants(tlb_grid* grid, double out[3]);

/* Coarsening and stripe diagnostics of the current state, in FP64 with a fixed reduction
 * order.  out (host, may be NULL; then nothing waits) receives out[0] = L_I, the interface
 * length of section IV (every node whose phi changes sign towards its phi neighbour adds
 * r dtheta, towards its theta neighbour (R + r cos theta_{q+1/2}) dphi, periodic), and
 * out[1] = A_total = sum r J dtheta dphi, so that L_d = A_total / L_I (eq. cart_scaling_L0).
 * phi_avg and p_avg (device arrays of n_theta doubles, may be NULL) receive the azimuthal
 * averages of phi (eq. phiavg) and of the pressure p = n + A(-phi^2/2 + 3 phi^4/4)
 * (eq. pbin; section III B measures the Laplace pressure with it).  Stream-ordered; waits
 * for the stream only when out is non-NULL.  Errors: TLB_EINVAL, TLB_EHIP.                 */
int32_t tlb_diagnostics(tlb_grid* grid, double out[2], double* phi_avg, double* p_avg);

/* Structure-factor coarsening length of phi, in the coordinate-space approximation of the
 * torus: S(m, m') = |DFT of phi over the node grid|^2 at mode numbers m (theta) and m' (phi),
 * wavenumbers k = (m / r, m' / R) with signed mode numbers (the Nyquist mode counts as -n/2),
 * the zero mode left out; out[0] = L_S = 2 pi sum S / sum |k| S, out[1] = sum S,
 * out[2] = sum |k| S (host array of 3 doubles).  A direct DFT in FP64 (rows, then columns),
 * fixed-order sums; the spinodal coarsening runs of section IV are the use.  The first call
 * allocates a workspace of about 16 n_theta n_phi bytes, kept until tlb_destroy.
 * n_phi <= 8192 and n_theta <= 4096.  Waits for the stream.  Errors: TLB_EINVAL,
 * TLB_ENOMEM, TLB_EHIP.                                                                    */
int32_t tlb_structure_length(tlb_grid* grid, double out[3]);

/* tlb_structure_length without any allocation, for callers that cannot allocate device
 * memory (serving loops, code that must not call hipMalloc): the same outputs (to rounding:
 * its twiddle factors are computed on the GPU and its final sums are taken in another fixed
 * order) from a workspace that is a static device array of 24 MiB per GPU, held from the
 * library's first use on that GPU until the process ends; nothing is allocated, on the device
 * or the host.  Grids need (n_theta n_phi + n_theta + n_phi) 16 + 16 n_phi + 24 bytes of it
 * (up to about 1.5 M nodes); larger grids get TLB_EINVAL.  Every call on one GPU uses the same
 * workspace, which keeps the last call's contents: calls that overlap on one GPU (on several
 * streams or host threads) race.  Waits for the grid's stream.  Errors: TLB_EINVAL, TLB_EHIP. */
int32_t tlb_structure_length_noalloc(tlb_grid* grid, double out[3]);

/* Release the handle and the library's own device memory (not the caller's buffers).      */
void tlb_destroy(tlb_grid* grid);

/* Tile height of the fused stage kernel: tiles of 64 (phi) x rows (theta) nodes, one block of
 * 64 rows threads each; rows = 4, 8 (default) or 16.  Results do not depend on it (every node
 * runs the same arithmetic); only speed does.  Errors: TLB_EINVAL.                          */
int32_t tlb_set_tile_rows(tlb_grid* grid, int32_t rows);

/* Autotuner: time the stage kernel for every tile height on this grid (stage-1 launches,
 * which leave the state unchanged) and keep the fastest; *rows (may be NULL) receives it.
 * Waits for the stream.  Errors: TLB_EINVAL, TLB_EHIP.                                     */
int32_t tlb_autotune(tlb_grid* grid, int32_t* rows);

/* Ensembles of tori (coarsening statistics over tori of different aspect ratios and grid
 * sizes, section IV): tlb_batch_step_n advances every grid of the batch by n_steps with one
 * fused launch per Runge-Kutta stage covering the tiles of all grids (each grid
 * keeps its own parameters, time step and buffers), replayed from graphs as tlb_step_n's.
 * Each grid ends exactly (bit for bit) where tlb_step_n on it alone would.  The batch
 * keeps pointers to the grids, which must outlive it and must not be stepped on their own
 * between batch calls on different streams.  All grids must have the same precision.
 * Ensembles whose state copies together exceed 1 GiB use streaming (nontemporal) stage
 * outputs and y^n loads, as large single grids do; the results are the same.
 * Errors: TLB_EINVAL (NULL, empty, mixed precision, duplicate), TLB_ENOMEM, TLB_EHIP.      */
typedef struct tlb_batch tlb_batch;
int32_t tlb_create_batch(tlb_grid* const* grids, int32_t n_grids, void* hip_stream,
                         tlb_batch** out);
int32_t tlb_batch_step_n(tlb_batch* batch, int64_t n_steps);
/* Autotuner of the batched launch (as tlb_autotune, over the whole ensemble).             */
int32_t tlb_batch_autotune(tlb_batch* batch, int32_t* rows);
void tlb_destroy_batch(tlb_batch* batch);

/* Message of the last error on the calling thread ("" if none).  Owned by the library.   */
const char* tlb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TLB_H */
