/*
 * lbm.h -- C ABI of the MI355X differentiable lattice Boltzmann library
 * (liblbm.so).
 *
 * The library computes the forward map of a BGK lattice Boltzmann solver
 * (D2Q9 or D3Q19, Section 2.1, Eq. 1-5 of Wang & Kumar, "An inverse analysis
 * of fluid flow through granular media using differentiable lattice
 * Boltzmann method") and the exact reverse-mode derivative of a final-time
 * velocity-mismatch loss (Section 2.2 and its loss listing; Eq. 7 and Eq. 15)
 * with respect to the inlet density (constant head or per-node profile,
 * Section 3.1), the outlet density and the relaxation time tau (viscosity,
 * Eq. 9; Section 3.4).
 *
 * Boundary conditions: halfway bounce-back on walls and solid nodes (grains,
 * spheres); density boundaries on the x faces (inlet x = 0, outlet x = nx-1)
 * by the Zou-He closure (bc_x = LBM_BC_PRESSURE) or by the paper's
 * anti-bounce-back rule (bc_x = LBM_BC_ABB, Section 2.1, Eq. 6); periodic or
 * wall y and z axes.
 *
 * Conventions
 *   - Populations are stored on the device as shifted values f_i - w_i in
 *     FP32 (structure of arrays over the fluid nodes only).  Where the ABI
 *     exchanges populations it uses the dense shifted layout
 *     [inst][i][nz][ny][nx], float (zero at solid nodes on output).
 *   - Velocity ordering:
 *       D2Q9 : (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1)
 *       D3Q19: rest, +x -x +y -y +z -z, (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0),
 *              (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1),
 *              (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1)
 *   - Densities cross the ABI as deviations drho = rho - 1 (FP64 parameters,
 *     FP32 fields); velocities as D = 2 (D2Q9) or D = 3 (D3Q19) components,
 *     node-major: u[inst][nz][ny][nx][D].
 *   - Per-node arrays of several instances are concatenated instance after
 *     instance.
 *
 * Ownership and streams
 *   - The caller owns all device memory.  lbm_workspace_bytes() sizes one
 *     workspace, which the caller allocates and passes to lbm_init(); the
 *     library never allocates device memory and the handle owns only host
 *     metadata.
 *   - All device work is ordered on the stream given to lbm_init().  Calls
 *     that return host values (loss, gradients, residuals) synchronise that
 *     stream; the others are asynchronous.  Internally the reverse sweep may
 *     run segment recomputes on a second stream of the handle's own, forked
 *     from and joined back into the caller's stream by events, and step
 *     loops are captured once into graphs (on a private capture stream) and
 *     replayed on the caller's stream; neither changes the ordering the
 *     caller sees.
 *   - Those streams, events and graphs are created on first use on the
 *     current device: call with the device that holds the workspace current.
 *   - A handle is not thread-safe: use one handle per stream.
 *
 * Errors: every call returns 0 (LBM_OK) or a negative LBM_E* code; nothing
 * aborts or throws across the ABI.  lbm_strerror() names a code and
 * lbm_last_error() gives the detail of the most recent failure on the
 * calling thread (including the HIP error string for LBM_EDEVICE).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_EINVAL (-1)    /* bad argument: dims, tau <= 0.5, NULL pointer, solid inlet in profile mode */
#define LBM_ENOMEM (-2)    /* workspace smaller than lbm_workspace_bytes() */
#define LBM_ESTATE (-3)    /* call out of order (adjoint without a taped forward, grad without adjoint) */
#define LBM_EUNSTABLE (-4) /* non-finite loss, residual or state */
#define LBM_ECORRUPT (-5)  /* a recomputed segment does not reproduce its checkpoint bit for bit */
#define LBM_EDEVICE (-6)   /* a HIP runtime call failed */

enum lbm_lattice { LBM_D2Q9 = 9, LBM_D3Q19 = 19 };
/* Axis boundary kinds.  PRESSURE and ABB apply to the x axis only; both
 * impose the densities 1 + drho_in at x = 0 and 1 + drho_out at x = nx-1:
 *   PRESSURE: Zou-He closure at the face nodes (density and zero tangential
 *             velocity at the node);
 *   ABB:      anti-bounce-back (Section 2.1, Eq. 6): an unknown population is
 *             the negated outgoing post-collision population plus twice the
 *             even part of the equilibrium at the imposed density and the
 *             face node's own velocity (density imposed half a link outside). */
/*   VELOCITY: Zou-He velocity inlet at x = 0 (normal velocity u_in taken from
 *             the drho_in parameters, zero tangential velocity; the node's
 *             density follows as K / (1 - u_in)) and a Zou-He density outlet
 *             at x = nx-1 (the free-stream inflow of Section 3.4's cylinder
 *             wake); lbm_grad's d_rho_in then holds dL/du_in. */
enum lbm_bc { LBM_BC_PRESSURE = 0, LBM_BC_PERIODIC = 1, LBM_BC_WALL = 2, LBM_BC_ABB = 3, LBM_BC_VELOCITY = 4 };
/* Collision operator: BGK (Eq. 4), or for D2Q9 the multiple-relaxation-time
 * operator of Section 3.4, f* = f - M^-1 S M (f - f_eq) with the moment basis
 * (rho, e, eps, jx, qx, jy, qy, pxx, pxy) and S = diag(mrt_rates), the two
 * stress rates being 1/tau. */
enum lbm_collision { LBM_COLL_BGK = 0, LBM_COLL_MRT = 1 };
enum lbm_loss_kind { LBM_LOSS_VEC = 0, LBM_LOSS_NORM = 1 };
enum lbm_loss_scale { LBM_SCALE_SUM = 0, LBM_SCALE_MEAN_FLUID = 1 };
enum lbm_inlet_mode { LBM_INLET_CONST = 0, LBM_INLET_PROFILE = 1 };
enum lbm_population_kind { LBM_POP_STATE = 0, LBM_POP_ADJOINT = 1 };

/* One lattice instance.  Host arrays are copied into the workspace by
 * lbm_init(); the caller may free them afterwards.  Size limits (LBM_EINVAL
 * beyond them): nx < 2^20; Q * nx * ny * nz < 2^31 - 2^20; and one state of
 * the instance, Q planes of its fluid nodes padded to a multiple of 64 at
 * 4 B each, below 4 GiB (D3Q19: at most 56 512 704 fluid nodes; D2Q9:
 * 119 304 640), since the kernels address it with 32-bit byte offsets.
 * Instances are independent lattices; the limit holds for each. */
typedef struct lbm_instance {
    int nx, ny, nz;          /* nz = 1 for D2Q9; nx >= 2 with density faces; nx < 2^20 */
    const uint8_t *solid;    /* [nz][ny][nx], nonzero = solid node; NULL = all fluid */
    const float *roi;        /* [nz][ny][nx] loss weights (Eq. 7 region of interest); NULL = 1 */
    const float *target_u;   /* [frames][nz][ny][nx][D] target velocity (frames = loss_frames, at
                                least 1); NULL = 0 */
} lbm_instance;

/* The problem: lattice, instances, boundary kinds, horizon and loss. */
typedef struct lbm_problem {
    int lattice;             /* LBM_D2Q9 or LBM_D3Q19 */
    int n_inst;              /* number of independent instances (>= 1) */
    const lbm_instance *inst;
    int bc_x, bc_y, bc_z;    /* lbm_bc per axis; PRESSURE, ABB and VELOCITY only on x */
    int steps;               /* T, number of time steps of lbm_forward() (>= 1) */
    int ckpt_interval;       /* K, checkpoint interval of the taped forward; 0 = ceil(sqrt(T)) */
    int tape;                /* nonzero: reserve checkpoints and a segment store for lbm_adjoint() */
    int loss_kind;           /* lbm_loss_kind: VEC |u - u_t|^2 or NORM (|u| - |u_t|)^2 */
    int loss_scale;          /* lbm_loss_scale: SUM, or MEAN_FLUID = 1 / (number of fluid nodes) (Eq. 15) */
    int inlet_mode;          /* lbm_inlet_mode: one inlet density per instance, or one per inlet node */
    int collision;           /* lbm_collision (0 = BGK; MRT needs LBM_D2Q9) */
    double mrt_rates[9];     /* MRT: rates of (rho, e, eps, jx, qx, jy, qy, pxx, pxy) in (0, 2);
                                the stress entries are ignored (1/tau) */
    int resident_segments;   /* tape: the taped forward keeps the states of its last R segments
                                (0 or 1 = the last one; clamped to the number of segments), and
                                lbm_adjoint() recomputes only the others.  Each costs K-1 states
                                of workspace; the gradient does not depend on R */
    int loss_frames;         /* time-windowed loss (Section 3.4 observes the periodic wake over
                                time): the loss is summed over the states after steps
                                T - (loss_frames - 1 - m) * loss_stride, m = 0 .. loss_frames - 1,
                                each against its own target frame.  0 or 1: the final state only */
    int loss_stride;         /* steps between loss frames (>= 1; (loss_frames - 1) * loss_stride < T) */
} lbm_problem;

/* Parameters of one forward evaluation (host arrays, read during the call). */
typedef struct lbm_params {
    const double *tau;       /* [n_inst] relaxation times, > 0.5 */
    const double *drho_in;   /* CONST: [n_inst]; PROFILE: per instance [nz][ny], concatenated */
    const double *drho_out;  /* [n_inst] outlet density deviations */
} lbm_params;

/* Elapsed device time per phase of the most recent calls (HIP events on the
 * library stream), filled when timing was enabled with lbm_set_timing(). */
typedef struct lbm_timing {
    double forward_ms;       /* lbm_forward step launches */
    long forward_launches;
    double recompute_ms;     /* segment recompute launches inside lbm_adjoint */
    long recompute_launches;
    double adjoint_ms;       /* adjoint step launches inside lbm_adjoint */
    long adjoint_launches;
} lbm_timing;

typedef struct lbm_handle lbm_handle;

/* Bytes of device workspace lbm_init() needs for problem p (pure query). */
int lbm_workspace_bytes(const lbm_problem *p, size_t *bytes);

/* Validates p, lays the workspace out, copies masks, weights and targets to
 * the device and sets the initial state to rest (rho = 1, u = 0).
 * d_workspace: device pointer of at least lbm_workspace_bytes() bytes, 256-B
 * aligned; hip_stream: hipStream_t (NULL = default stream). */
int lbm_init(lbm_handle **h, const lbm_problem *p, void *d_workspace, size_t bytes,
             void *hip_stream);

/* Releases the host metadata of h (the workspace stays the caller's). */
int lbm_destroy(lbm_handle *h);

/* Initial state f = f_eq(1 + drho, u) at fluid nodes (Eq. 5; the paper
 * starts from a uniform density of 1 at rest, Section 3.2, and the
 * network-based initial guess that Section 3.5 proposes passes a predicted
 * (drho, u)).  d_drho: device [nodes] float, d_u: device [nodes][D] float;
 * both NULL = rest.  The arrays are read by work enqueued on the handle's
 * stream: keep them valid until that work has run.  Invalidates a taped
 * forward. */
int lbm_set_initial(lbm_handle *h, const float *d_drho, const float *d_u);

/* Initial state from explicit populations: device dense shifted
 * [inst][i][nz][ny][nx] float (values at solid nodes are ignored). */
int lbm_set_populations(lbm_handle *h, const float *d_fbar);

/* Copies populations to device d_out in the dense shifted layout:
 * LBM_POP_STATE   -> the state after the last forward / run (post-collision);
 * LBM_POP_ADJOINT -> dL/d(initial state) after lbm_adjoint().
 * Solid nodes read as 0. */
int lbm_get_populations(lbm_handle *h, int which, float *d_out);

/* The forward map (Section 2.1): T steps from the initial state, each one
 * fused launch of streaming (Eq. 3, pull form), halfway bounce-back on walls
 * and solid nodes, the x-face closure (Zou-He, or anti-bounce-back, Eq. 6)
 * and the collision (BGK, Eq. 4, towards the equilibrium of Eq. 5 with the
 * moments of Eq. 1-2; or MRT, Eq. 16-18), then the velocity-mismatch loss of
 * Eq. 7 (weights = the region of interest; MEAN_FLUID = the normalised form
 * of Eq. 15) on the final state, or summed over the loss frames.
 * prm: host arrays read during the call (tau > 0.5 per instance; face
 * densities as deviations from 1, > -1).  With record_tape nonzero (requires
 * problem.tape) the checkpoints every K steps and the states of the last
 * resident_segments segments are kept for lbm_adjoint().  loss_out (host,
 * nullable): [n_inst] losses; passing it synchronises the stream.
 * Errors: LBM_EINVAL (parameters), LBM_ESTATE (record_tape without a tape),
 * LBM_EUNSTABLE (a non-finite loss), LBM_EDEVICE. */
int lbm_forward(lbm_handle *h, const lbm_params *prm, int record_tape, double *loss_out);

/* The reverse sweep (Section 2.2: the derivative the paper obtains by
 * replaying its recorded tape backwards), here the exact transpose of each
 * discrete step applied from T down to 1: the terminal seed dl/dg^T of the
 * loss (Eq. 7 / Eq. 15), then per step the closure, collision and streaming
 * transposes, accumulating dL/dtau and dL/d(face density) per face node in
 * FP64.  Segments of K steps that the taped forward did not keep are
 * recomputed from their checkpoints; each recomputed segment followed by a
 * checkpoint takes one more step that must reproduce that checkpoint bit for
 * bit (reported by lbm_grad as LBM_ECORRUPT).  d_seed_du NULL: the built-in
 * loss; otherwise a device array [nodes][D] float of dL/du(T) supplied by
 * the caller (any differentiable loss of the final velocity), copied on the
 * handle's stream.  Asynchronous.  Errors: LBM_ESTATE (no taped forward),
 * LBM_EINVAL (a caller seed with loss_frames > 1), LBM_EDEVICE. */
int lbm_adjoint(lbm_handle *h, const float *d_seed_du);

/* Gradients of the loss from the last lbm_adjoint() (Section 2.2; the
 * inverse problems of Section 3.1-3.4: the constant head or the inlet
 * pressure profile, the outlet density, and tau, i.e. the viscosity of
 * Eq. 9), as host arrays, each nullable:
 * d_rho_in  CONST: [n_inst]; PROFILE: per instance [nz][ny] (0 at solid nodes);
 *           a velocity inlet: dL/du_in;
 * d_tau     [n_inst];
 * d_rho_out [n_inst].
 * Synchronises the stream.  Errors: LBM_ESTATE (no adjoint), LBM_ECORRUPT (a
 * recomputed segment of that reverse sweep did not reproduce its checkpoint:
 * the outputs are not written), LBM_EUNSTABLE (a non-finite gradient),
 * LBM_EDEVICE. */
int lbm_grad(lbm_handle *h, double *d_rho_in, double *d_tau, double *d_rho_out);

/* Steady state of the forward map (Section 3.1.1 takes it from the plateau
 * of the kinetic energy): steps from the initial state until the velocity
 * residual of every instance is <= tol, testing every check_every steps
 * (even, >= 4), or until max_steps.  The residual at a check t is the mean
 * relative change per step of the two-step-mean velocity
 * ubar(t) = (u(t) + u(t-1)) / 2 over the last interval:
 *   r(t) = ||ubar(t) - ubar(t - check_every)|| / (check_every ||ubar(t)||)
 * over the fluid nodes (ubar(0) = u of the initial state).  For a smooth
 * transient it equals ||d ubar/dt|| / ||ubar||, the per-step rate; it
 * averages out the step-to-step rounding jitter of FP32 populations around
 * the steady state, and the two-step mean cancels the undamped period-2
 * mode of the scheme (an equilibrium momentum field alternating in sign
 * along x that streaming maps onto its negative).  steps_out / r_out (host,
 * nullable) receive the step count and the largest instance residual.
 * Synchronises the stream after every check.  Errors: LBM_EINVAL
 * (check_every, max_steps, parameters), LBM_EUNSTABLE (a non-finite
 * residual), LBM_EDEVICE. */
int lbm_run_to_residual(lbm_handle *h, const lbm_params *prm, double tol, int max_steps,
                        int check_every, int *steps_out, double *r_out);

/* Per-instance residuals (host [n_inst]) of the last check of the last
 * lbm_run_to_residual() call (NaN for an instance whose sums were not
 * finite).  Errors: LBM_EINVAL, LBM_ESTATE (no residual yet). */
int lbm_get_residuals(lbm_handle *h, double *r_out);

/* Macroscopic fields (Eq. 1-2: rho = sum f, u = sum f c / rho) of the
 * current state to device arrays: d_drho [nodes], d_u [nodes][D] (zeros at
 * solid nodes).  mean2 nonzero: the mean of the last two states (cancels the
 * undamped period-2 staggered mode; needs a state produced by at least two
 * steps, else LBM_ESTATE).  Asynchronous. */
int lbm_get_macro(lbm_handle *h, float *d_drho, float *d_u, int mean2);

/* Enables (default) or disables hipGraph replay of the step loops: each loop
 * (taped or plain forward, reverse sweep, residual chunk) is captured once on
 * a private stream and then launched as one graph on the handle's stream. */
int lbm_set_graphs(lbm_handle *h, int enable);

/* Device address (*d_state) and size (*bytes, nullable) of checkpoint c,
 * the state after c K steps kept by a taped forward, c = 1 .. n_seg - 1
 * (n_seg = ceil(T / K)), inside the caller's workspace: fluid-node SoA of
 * shifted FP32 populations.  For inspection and for fault-injection tests
 * of the checkpoint verification (overwriting it makes the next reverse
 * sweep that recomputes segment c - 1 report LBM_ECORRUPT).  Errors:
 * LBM_EINVAL, LBM_ESTATE (no tape planned). */
int lbm_checkpoint(lbm_handle *h, int c, void **d_state, size_t *bytes);

/* Enables (nonzero) or disables per-phase event timing; reset clears it.
 * Timed calls launch kernels one by one (no graphs) between HIP events. */
int lbm_set_timing(lbm_handle *h, int enable, int reset);
int lbm_get_timing(lbm_handle *h, lbm_timing *out);

/* Bandwidth calibration (measurement only, no part of the method): copies
 * `bytes` from device d_src to device d_dst with one 16-byte load and store
 * per lane, enqueued on hip_stream.  bytes and both pointers must be
 * multiples of 16 (LBM_EINVAL otherwise); the ranges must not overlap. */
int lbm_stream_copy(void *d_dst, const void *d_src, size_t bytes, void *hip_stream);

const char *lbm_strerror(int code);
const char *lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
