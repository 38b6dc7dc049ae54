/*
 * lbnlm — MI355X (gfx950) lattice-Boltzmann solver for channel flow of the
 * instantaneous nonlinear generalised Maxwell (inlM) fluid.
 *
 * C ABI. Plain pointers and sizes only; every call returns an lb_status
 * (0 = LB_OK, negative = error) and, on error, leaves a message readable with
 * lb_last_error(). A handle is bound to one HIP stream and is not thread
 * safe; calls on different handles may run concurrently.
 *
 * The method (Papenkort & Voigtmann, arXiv:1310.7450): a D2Q9 BGK scheme
 * whose forcing term carries the traceless non-Newtonian stress, the body
 * force and the flow-induced density change (Sec. II.A, Eqs. (lbupdate),
 * (rhoj), (bodyforce), (rhoplus)), with the stress taken each step from the
 * steady-state series of the nonlinear Maxwell model evaluated on the
 * instantaneous velocity gradient (Sec. III.A, Eqs. (sigtsum), (smalld),
 * (nlmaxwell) and the inlM paragraph), the gradient from three-point central
 * differences (Sec. II.C), in a channel with half-way bounce-back walls in y
 * and periodic x, driven by a body force that is switched off for cessation
 * (Sec. II.B, III.B, IV.B).
 *
 * Lattice units throughout: dx = dt = 1, reference density rho0 = 1,
 * c_s^2 = 1/3, two dimensions.
 */
#ifndef LBNLM_LB_H
#define LBNLM_LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb_handle lb_handle;

typedef enum {
  LB_OK = 0,
  LB_EINVAL = -1,     /* invalid argument (parameters, sizes, indices)       */
  LB_ENOMEM = -2,     /* workspace too small or host allocation failed       */
  LB_EHIP = -3,       /* a HIP runtime call failed                           */
  LB_EUNSTABLE = -4,  /* a convergence check saw NaN/Inf in a channel         */
  LB_ESTATE = -5      /* call not valid in the handle's current state        */
} lb_status;

typedef enum {
  LB_FP64 = 0,          /* populations stored and updated in FP64             */
  LB_FP32_SHIFTED = 1   /* populations stored in FP32 as n_i - a_i - E_i(U_y):*/
                        /* a_i the rest weights, E_i(u) = a_i (3 c_ix u +      */
                        /* (9/2 c_ix^2 - 3/2) u^2) the velocity part of the    */
                        /* equilibrium at density 1 and U_y a per-row          */
                        /* reference velocity, moved to the row's mean u_x at */
                        /* every block boundary (see lb_step) and at          */
                        /* lb_set_state; moments and updates in FP32          */
} lb_precision;

/*
 * One channel: nx periodic nodes along the flow (x), ny fluid rows between
 * half-way bounce-back walls at y = -1/2 and y = ny - 1/2 (half width
 * H = ny/2). Parameters follow the problem statement of Sec. III.B:
 *   force      body-force density g (= pressure drop per unit length with
 *              rho0 = 1) along +x, applied for steps t < t_startup and
 *              switched off afterwards (cessation, Sec. IV.B);
 *   tau_lb     BGK relaxation time of the solvent, tau_lb > 1/2: the
 *              high-shear (solvent) viscosity is eta_s = (tau_lb - 1/2)/3;
 *   G          plateau modulus G_inf of the Maxwell stress (>= 0; 0 gives a
 *              Newtonian fluid);
 *   tau0       quiescent Maxwell relaxation time tau in steps at eps = 0
 *              (> 0, may be +inf: the yield-stress limit);
 *   gamma_c    critical strain of Eq. (nlmaxwell) (> 0);
 *   eps        separation parameter: tau = tau0 * 10^(min(eps,0)/0.05),
 *              G_inf = G (1 + sqrt(max(eps,0))) (the paper has no eps; this
 *              closure is the library's definition);
 *   visc_split lambda in [0,1]: the collision carries eta_s + lambda G tau
 *              and the forcing Sigma^nN = sigma - lambda G tau D (lambda = 1
 *              is the split of Sec. IV; lambda > 0 needs a finite tau);
 *   t_startup  first step without the body force (and without the wall
 *              motion);
 *   wall_velocity  x velocity of the top wall for steps t < t_startup, 0
 *              afterwards: planar Couette flow driven by a wall that is
 *              switched on and off (Sec. IV.B); |u_w| < 0.3 (low Mach
 *              number). How the wall acts is set by top_wall.
 *   pressure_gradient  pressure drop per unit length G_p along +x (the
 *              problem statement's Delta p / L, equivalent to force = G_p)
 *              imposed by generalised periodic boundaries (Sec. II.B): the
 *              populations crossing the period take the equilibrium at the
 *              far end's pressure, p+- = c_s^2 +- (nx + 1) G_p / 2 on the
 *              virtual nodes beside the inlet (x = 0) and outlet
 *              (x = nx - 1) columns, plus the source's non-equilibrium part;
 *              acts for t < t_startup. Needs force = 0, wall_velocity = 0,
 *              nx >= 2, nn_pressure = 0 (the forcing keeps its first line
 *              only) and the half-way top wall. 0: plain periodic x.
 *   nn_pressure  1: the forcing of Eq. (bodyforce) keeps the flow-induced
 *              density terms of Eq. (rhoplus); 0: they are dropped
 *              (dt d(delta rho)/dt = 0), as Sec. II.B does with pressure
 *              boundaries. Per channel, so that one batch can run stiff
 *              channels without them (with them, the explicit stress
 *              amplifies round-off once G_inf tau exceeds about 0.3 at
 *              visc_split 0; without them and with visc_split 1/2 it stays
 *              well conditioned up to G_inf tau = 10).
 *   top_wall   LB_WALL_HALFWAY: half-way bounce-back at y = ny - 1/2 like the
 *              bottom wall; a moving wall reflects with the wall-momentum
 *              term -2 a_i (c_i . u_w) / c_s^2 (wall density rho0 = 1).
 *              LB_WALL_ZOU_HE: the moving wall of the paper's Couette runs,
 *              Zou and He's velocity boundary on the top node row y = ny - 1
 *              (Sec. II.B, last paragraph), so the channel spans
 *              L = ny - 1/2. After streaming, the three populations of that
 *              row entering from above (c_y = -1) follow from the other six:
 *              no flow through the wall, n_4 = n_2 (normal non-equilibrium
 *              bounce-back) and the diagonals such that the node's
 *              provisional velocity (m + f/2) / sum_i n_i is (u_w, 0); the
 *              node then collides like any other, and what it emits upwards
 *              leaves the lattice. Its velocity gradient uses the ghost
 *              mirrored through the wall node, u(ny) = 2 (u_w, 0) - u(ny-2).
 *              Needs ny >= 2, no pressure_gradient and no stress_force.
 */
typedef struct {
  int32_t nx;
  int32_t ny;
  double force;
  double tau_lb;
  double G;
  double tau0;
  double gamma_c;
  double eps;
  double visc_split;
  int64_t t_startup;
  double wall_velocity;
  double pressure_gradient;
  int32_t nn_pressure;
  int32_t top_wall;
} lb_channel;

/* Values of lb_channel.top_wall. */
enum { LB_WALL_HALFWAY = 0, LB_WALL_ZOU_HE = 1 };

/*
 * Options shared by all channels of a handle:
 *   precision    lb_precision;
 *   obs_every    K, the length of one block of steps (one captured graph);
 *                the convergence check and the FP32 reference move run at
 *                the block boundaries; even, >= 2 (default 1000 when 0);
 *   strip_rows   rows per wavefront strip of the sweep, also of the
 *                two-step sweep below (0: tuned default; the two-step
 *                default fills whole rounds of resident strips). While
 *                the active channels make fewer one-step strips than the
 *                GPU has SIMDs, their heights are divided alike (down to
 *                4 rows, or a narrow kernel's row group) to spread them
 *                over the GPU. The narrow widths' two-step strips take
 *                the smallest height among 1, 2, 4, the multiples of 8 up
 *                to 64 and the powers of two beyond (at most strip_rows
 *                when it is set) whose strips the GPU holds all at once.
 *                Results do not depend on strip heights;
 *                FP64 channels whose width is not a power of two up to 64
 *                (and whose nx * ny is at most 429,496,704) step on tiles of
 *                64 x 8 nodes instead and do not use it;
 *   steady_tol   if > 0, lb_step checks every K steps the residual
 *                R = max_y |ubar(t) - ubar(t-K)| / (K max_y |ubar(t)|) of the
 *                x-averaged velocity ubar and freezes each channel once
 *                R < steady_tol; 0 disables the checks;
 *   viscoelastic 0: the instantaneous model of Sec. III.A (the stress is the
 *                steady sum of Eq. (sigtsum) at the current velocity
 *                gradient); 1: the time-integrated nonlinear Maxwell model,
 *                Eq. (gkder) with d_t G = -G / tau_M(t) and tau_M of
 *                Eq. (nlmaxwell), stepped as
 *                sigma(t) = [sigma(t-1) + kappa sigma(t-1) + sigma(t-1) kappa^T
 *                            + G_inf D] / (1 + 1/tau_M)
 *                (upper-convected terms explicit, relaxation implicit; the
 *                fixed point is the instantaneous model's stress). The stress
 *                is then part of the state (three more fields per node, in
 *                the precision of the populations, zero at rest; see
 *                lb_get_stress), and the workspace grows accordingly;
 *   stress_force 0: the non-Newtonian stress enters through the second moment
 *                of the forcing of Eq. (bodyforce); 1: it enters as the force
 *                density div Sigma^nN in the body-force terms instead (the
 *                alternative Sec. II.C names), with Sigma^nN formed at every
 *                node first, central differences for the divergence and ghost
 *                rows extrapolated linearly through the walls; there is then
 *                no flow-induced density. Needs LB_FP64, the instantaneous
 *                model and channels with nn_pressure = 0, the half-way top
 *                wall, no pressure_gradient and at most 429,496,704 nodes.
 *                Runs as one fused pass per step (u~, Sigma^nN and the
 *                collide-and-stream of a tile of nodes in one workgroup);
 *   steps_per_sweep 0 (default) or 2: with either stress model, no
 *                stress_force and K a multiple of 4, the blocks of K steps
 *                advance the vector-class channels (width a multiple of 256
 *                in LB_FP32_SHIFTED, of 64 in LB_FP64, not a power of two up
 *                to 64) without pressure_gradient (any top wall) two
 *                steps per pass over the state (a
 *                strip's rows of step t are kept on chip for step t+1);
 *                without the viscoelastic option the narrow channels (width
 *                1, 2, 4, ..., 64) without pressure_gradient do too;
 *                other channels, other handles and steps outside whole
 *                blocks run one step per pass. Each node update is the
 *                arithmetic of the one-step pass; states agree with it to
 *                round-off; 1: one step per pass always.
 */
typedef struct {
  int32_t precision;
  int32_t obs_every;
  int32_t strip_rows;
  double steady_tol;
  int32_t viscoelastic;
  int32_t stress_force;
  int32_t steps_per_sweep;
} lb_options;

/* Observables for lb_observe. Profiles return ny doubles (x-averages per row,
 * row 0 next to the lower wall); scalars return one double. */
enum {
  LB_OBS_UX = 0,        /* u_x = j_x / rho_e                                 */
  LB_OBS_UY = 1,
  LB_OBS_SXX = 2,       /* Maxwell stress sigma (Eq. (sigtsum); with the    */
                        /* viscoelastic option the sigma(t) the next step   */
                        /* computes from the stored sigma(t-1))             */
  LB_OBS_SXY = 3,
  LB_OBS_SYY = 4,
  LB_OBS_N1 = 5,        /* sigma_xx - sigma_yy                              */
  LB_OBS_PRESSURE = 6,  /* c_s^2 rho_e                                      */
  LB_OBS_KXY = 7,       /* d_y u_x from the central difference              */
  LB_OBS_TRT = 8,       /* tr Sigma^nN                                      */
  LB_OBS_KXX = 9,       /* d_x u_x                                          */
  LB_OBS_MASS = 32,     /* sum_nodes (sum_i n_i - delta rho_prev)            */
  LB_OBS_MOMX = 33,     /* sum_nodes sum_i c_ix n_i                         */
  LB_OBS_FLUX = 34,     /* sum_nodes u_x                                    */
  LB_OBS_WALL_DRAG = 35,/* x momentum given to the walls in the last step;  */
                        /* at a Zou-He top wall: what the top row emitted  */
                        /* upwards minus what its completion supplied (not */
                        /* defined before the first step after            */
                        /* lb_set_state or lb_set_profile)                */
  LB_OBS_UMID = 36,     /* x-averaged u_x at the centre line                */
  LB_OBS_RESIDUAL = 37, /* last residual R (+inf before two checks)        */
  LB_OBS_STEP = 38,     /* steps the channel has taken                      */
  LB_OBS_ACTIVE = 39,   /* 1 while the channel advances, 0 once frozen      */
  LB_OBS_NAN = 40       /* 1 if the observation saw NaN/Inf                 */
};

/* Device workspace the caller must provide for these channels and options.
 * Returns LB_EINVAL for invalid channels or options. */
lb_status lb_workspace_bytes(const lb_channel *channels, int32_t n_channels,
                             const lb_options *opt, size_t *bytes);

/* Creates a handle for n_channels channels (array read, not kept).
 * dev_workspace: device memory of at least lb_workspace_bytes bytes, aligned
 * to 256 bytes, owned by the caller, which must keep it alive until
 * lb_destroy; the library never frees it. hip_stream: a hipStream_t (NULL:
 * the library creates and owns one). All channels start from rest
 * (n_i = a_i, previous stress trace 0) at step 0. */
lb_status lb_create(const lb_channel *channels, int32_t n_channels,
                    const lb_options *opt, void *dev_workspace, size_t ws_bytes,
                    void *hip_stream, lb_handle **out);

/* Releases the handle (graphs, host tables, an owned stream). Does not touch
 * the workspace. NULL is accepted. */
lb_status lb_destroy(lb_handle *h);

/* Advances every active channel by up to n_steps steps, asynchronously on the
 * handle's stream, except that with steady_tol > 0 it synchronises every K
 * steps to read the residuals; returns when all channels are frozen or
 * n_steps are done. LB_EUNSTABLE if a check saw NaN/Inf. Block boundaries
 * fall every K steps of a clock the handle keeps over all lb_step calls, so
 * that splitting n steps over several calls gives the same state, bit for
 * bit, as one call. */
lb_status lb_step(lb_handle *h, int64_t n_steps);

/* Reads one observable of channel ch at its current step into host_out
 * (n doubles available). Synchronises the stream. */
lb_status lb_observe(lb_handle *h, int32_t ch, int32_t what, double *host_out, size_t n);

/* lb_observe for callers that cannot allocate memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. Returns the
 * same values as lb_observe (arguments likewise), but the observation's
 * scratch (per-strip partials, per-row profiles, per-channel scalars and the
 * gathered result) lives in a 16 MiB device array that the library keeps on
 * each GPU for the life of the process, not in the handle's workspace, and
 * the call allocates nothing. Every call on one GPU shares that array and
 * finds the last call's contents in it: calls that overlap on one GPU (from
 * other host threads, or other handles on other streams) race and must be
 * serialised by the caller. LB_EINVAL when the handle's observation needs
 * more than 16 MiB (about 96 bytes per row of every channel and per row and
 * x strip, about 170,000 of them together), and for a stress-force handle
 * (whose observation needs scratch per node); lb_observe serves both. Does
 * not refresh what lb_observe caches. Synchronises the stream. */
lb_status lb_observe_noalloc(lb_handle *h, int32_t ch, int32_t what, double *host_out, size_t n);

/* Copies the state of channel ch to host memory: the post-streaming
 * populations n_i(x, y) of the current step as pops[9][ny][nx] (velocity
 * order (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1)) and the
 * previous stress trace P[ny][nx], in FP64. With a Zou-He top wall the three
 * populations of row ny - 1 entering from above are the ones the boundary
 * completes for the current step. Synchronises the stream. */
lb_status lb_get_state(lb_handle *h, int32_t ch, double *pops, double *P);

/* Overwrites the state of channel ch (same layout as lb_get_state) and sets
 * its step counter to t. With a Zou-He top wall the three populations of row
 * ny - 1 entering from above are not kept: the next step completes them.
 * Synchronises the stream. */
lb_status lb_set_state(lb_handle *h, int32_t ch, const double *pops, const double *P, int64_t t);

/* Time-integrated stress of channel ch (viscoelastic option only): the
 * stress sigma(t-1) the next step starts from, as sigma[3][ny][nx] (planes
 * xx, xy, yy), in FP64. lb_set_state and lb_set_profile leave it unchanged.
 * LB_EINVAL if the handle runs the instantaneous model. Synchronise the
 * stream. */
lb_status lb_get_stress(lb_handle *h, int32_t ch, double *sigma);
lb_status lb_set_stress(lb_handle *h, int32_t ch, const double *sigma);

/* Point sets of lb_set_profile. */
enum {
  LB_PROFILE_ROWS = 0,      /* n_pts == ny values at the lattice rows y = 0..ny-1 */
  LB_PROFILE_CHEBYSHEV = 1  /* values at d_k = cos(pi (2k+1) / (2 n_pts)), k < n_pts,
                               d = (y - y_c)/H across the channel; interpolated to
                               the rows with the barycentric formula */
};

/* Initialises channel ch from a predicted steady profile (a warm start):
 * u_x and N1 given at n_pts points of the set `points`. Populations are set
 * to the equilibrium at u = (u_x, 0) and rho_e = 1 - (3/2) N1 (rho_e = 1 for a
 * channel without the flow-induced density terms), so that the conserved
 * mass equals that of the rest state, and the previous trace to N1. The step
 * counter is kept. LB_EINVAL for an unknown point set or n_pts != ny with
 * LB_PROFILE_ROWS. */
lb_status lb_set_profile(lb_handle *h, int32_t ch, const double *ux, const double *n1, int32_t n_pts,
                         int32_t points);

/* Message of the last error on this handle (never NULL). */
const char *lb_last_error(const lb_handle *h);

/* Name of a status code. */
const char *lb_status_string(int32_t status);

#ifdef __cplusplus
}
#endif

#endif /* LBNLM_LB_H */
