/*
 * Plain FP64 CPU oracle of the modified D2Q9 lattice-Boltzmann scheme for a
 * fluid obeying the instantaneous nonlinear generalised Maxwell (inlM) model,
 * in a 2D channel: x periodic, bounce-back walls in y, driven by a body force.
 *
 * TEST INFRASTRUCTURE. This file is the independent reference the GPU path is
 * checked against. Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product library never does. It shares
 * no code, header or table with the GPU path.
 *
 * It is written to be read against the paper (Papenkort & Voigtmann,
 * arXiv:1310.7450), one step per passage, with no blocking, fusion or
 * reordering:
 *   - collide and stream, n_i(r + c_i, t + 1) = n_i + Delta_i + F_i:
 *     Sec. II.A, Eq. (lbupdate);
 *   - density and current from the half-way average of pre- and
 *     post-collision populations: Sec. II.A, Eq. (rhoj);
 *   - D2Q9 velocities, weights a = 4/9, 1/9, 1/36 and the second-order
 *     equilibrium: Sec. II.A (equilibrium distribution and the D2Q9 model);
 *   - BGK collision, Delta_i = -(n_i - n_i^eq)/tau: Sec. II.A;
 *   - forcing term F_i carrying the traceless non-Newtonian stress, the body
 *     force and the flow-induced density change: Sec. II.A, Eq. (bodyforce);
 *   - normal-stress advection, dt d(delta rho)/dt from the change of the stress
 *     trace between two steps: Sec. II.A, Eq. (rhoplus);
 *   - bounce-back walls: Sec. II.B;
 *   - velocity gradient kappa_ab = d_b u_a by three-point central differences:
 *     Sec. II.C;
 *   - steady-state stress as the series sigma = sum_{n>=1} G tau_M^n d^n with
 *     d^1 = D and d^{n+1} = kappa d^n + d^n kappa^T: Sec. III.A,
 *     Eqs. (sigtsum), (smalld);
 *   - shear-dependent relaxation 1/tau_M = 1/tau + sqrt(II_D)/gamma_c with
 *     II_D = tr(D^2)/2: Sec. III.A, Eq. (nlmaxwell);
 *   - the instantaneous model (kappa, tau_M taken at the current step):
 *     Sec. III.A, closing paragraph;
 *   - the viscosity split (tau_LB carrying part of G tau): Sec. IV, opening.
 *
 * Readings where the paper is silent or ambiguous (each is also listed in the
 * design notes):
 *   R1 the equilibrium density is rho_e = sum (n* + n)/2 (no -delta rho
 *      subtraction), so that sum_nodes (sum_i n_i - delta rho_prev) is
 *      conserved exactly;
 *   R2 kappa is taken from u~ = j / sum_i n_i (j = m + f/2), the equilibrium and
 *      the forcing use u = j / rho_e;
 *   R3 body force density f = rho0 g with rho0 = 1;
 *   R4 half-way bounce-back, walls at y = -1/2 and y = ny - 1/2;
 *   R5 at the wall rows the finite difference uses the ghost velocity
 *      u(-1) = -u(0), u(ny) = -u(ny-1) (no slip on the half link);
 *   R6 the stress series is summed until a term is below 1e-18 of the running
 *      sum; a node where it does not converge is counted and reported;
 *   R7 separation eps: tau = tau0 * 10^(min(eps,0)/0.05),
 *      G_inf = G (1 + sqrt(max(eps,0))); gamma_c fixed;
 *   R8 viscosity split lambda: the collision relaxes with
 *      tau_eff = 1/2 + 3 (eta_s + lambda G tau), eta_s = (tau_LB - 1/2)/3,
 *      and Sigma^nN = sigma - lambda G tau D.
 *   R9 planar Couette flow (Sec. IV.B): the top wall moves along x with u_w
 *      while t < t_startup; it stays on the half link and reflects with the
 *      wall-momentum term -2 a_i (c_i . u_w)/cs2 (rho_w = rho0 = 1), and the
 *      stencil ghost behind it is 2 u_w - u(ny-1). The paper's Couette runs
 *      used Zou and He's velocity boundary on a node row instead.
 *   R10 pressure drive by generalised periodic boundaries (Sec. II.B): the
 *      inlet pressure p+ = cs2 + dp/2 belongs to the virtual node x = -1
 *      before the inlet column, the outlet pressure p- = cs2 - dp/2 to the
 *      virtual node x = nx after the outlet column (mean density rho0 = 1),
 *      so dp spans nx + 1 spacings: a pressure gradient G_p is dp =
 *      (nx + 1) G_p, equivalent to a body force G_p. A population streaming from
 *      the outlet into the inlet becomes n^eq(p+/cs2 + rho - rho_bar_out, j)
 *      + (n* - n^eq(rho, j)), (rho, j) the moments of its source node and
 *      rho_bar_out the mean density of the outlet column; the reverse
 *      direction likewise with p- and the inlet column. With this drive the
 *      forcing keeps its first line only (no body force, no delta rho).
 *      The drop acts for t < t_startup; afterwards the same boundaries hold
 *      both ends at rho0 (cessation).
 *   R11 the time-integrated (viscoelastic) nonlinear Maxwell model: the
 *      differential form of Eq. (gkder) with d_t G = -G / tau_M(t), tau_M from
 *      Eq. (nlmaxwell) at the current kappa (the time-dependent generalisation
 *      Sec. III.A mentions and leaves aside):
 *        d sigma/dt - kappa sigma - sigma kappa^T = G D - sigma / tau_M.
 *      One step (dt = 1) takes the upper-convected terms and the source
 *      explicitly and the relaxation implicitly,
 *        sigma(t) = [sigma(t-1) + kappa sigma(t-1) + sigma(t-1) kappa^T + G D]
 *                   / (1 + 1/tau_M),
 *      with kappa, D and tau_M of step t. Its fixed point satisfies
 *      sigma = tau_M (kappa sigma + sigma kappa^T + G D), the relation whose
 *      solution is the series of Eq. (sigtsum), so the steady states of both
 *      models coincide. The stress of step t then enters the forcing as in
 *      the instantaneous model. The state carries sigma(t-1) (three more
 *      fields per node, zero at rest).
 *   R12 stress as a force (the alternative Sec. II.C names: the divergence of
 *      the stress taken as an external force density in Eq. (ns)): the
 *      non-Newtonian stress Sigma^nN = sigma - lambda G tau D of every node
 *      is formed first (kappa from u~ = (m + rho0 g/2)/s as in R2); the
 *      forcing then carries the total force f = rho0 g + div Sigma^nN in its
 *      body-force terms only, with no stress term in its second moment and
 *      no flow-induced density (the trace acts through the divergence, so
 *      r = 0). div Sigma^nN is taken by central differences, x periodic, with
 *      ghost rows extrapolated linearly through the walls,
 *      Sigma(-1) = 2 Sigma(0) - Sigma(1), Sigma(ny) = 2 Sigma(ny-1) -
 *      Sigma(ny-2) (one row: zero gradient), so that the summed force is
 *      the stress at the half-way walls. The equilibrium and forcing use
 *      u = (m + f/2)/s.
 *   R13 the moving wall of planar Couette flow as Zou and He's velocity
 *      boundary (Sec. II.B, last paragraph; Sec. IV.B): the top wall lies on
 *      the node row y = ny - 1, so the channel spans L = ny - 1/2 from the
 *      half-way wall at y = -1/2. After streaming, a node of that row lacks
 *      the three populations that would enter from above (c_y = -1). They
 *      follow from the six it has: no flow through the wall fixes the
 *      density, s = n0 + n1 + n3 + 2 (n2 + n5 + n6); the normal part of the
 *      non-equilibrium bounces back, n4 = n2; the two diagonals share what is
 *      left of the momentum such that the node's provisional velocity
 *      u~ = (m + f/2)/s is the wall's (u_w, 0). The node then collides like
 *      any other. Populations it emits upwards leave the lattice. Its
 *      velocity gradient uses the ghost mirrored through the wall node,
 *      u~(ny) = 2 (u_w, 0) - u~(ny-2). The state held after each step has
 *      the missing populations already completed for the next step.
 *
 * Lattice units: dx = dt = 1, rho0 = 1, c_s^2 = 1/3, d = 2.
 * Storage: populations n[i][y][x] (nine planes, x fastest), the previous
 * stress trace P[y][x] = tr Sigma^nN at the previous step. The state held here
 * is the post-streaming (pre-collision) population n_i(r, t).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D2Q9 velocities in the order (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),
 * (-1,-1),(1,-1) and their weights. */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const double CS2 = 1.0 / 3.0;

static int opposite(int i) {
  for (int k = 0; k < 9; ++k)
    if (CX[k] == -CX[i] && CY[k] == -CY[i]) return k;
  return -1;
}

typedef struct {
  double g;         /* body-force density along +x while t < t_startup       */
  double tau_eff;   /* BGK relaxation time of the collision                   */
  double G;         /* plateau modulus after the eps closure                  */
  double tau;       /* Maxwell relaxation time after the eps closure (or inf) */
  double gamma_c;   /* critical strain                                        */
  double lam;       /* viscosity split lambda in [0, 1]                       */
  long long t_startup;
  int nn_pressure;  /* 1: keep the delta-rho terms of the forcing            */
  double uw;        /* x velocity of the top wall while t < t_startup (R9)   */
  double dp;        /* pressure drop p+ - p- across the period (R10), 0: off */
  int ve;           /* 1: time-integrated stress (R11); 0: instantaneous     */
  int saf;          /* 1: stress as a force density (R12)                    */
  int zh;           /* 1: top wall is Zou-He's velocity boundary on the top  */
                    /*    node row (R13); 0: half-way bounce-back (R4, R9)   */
} orc_params;

/* Parameter resolution (readings R7, R8). Returns 0, or -1 for invalid input. */
int orc_resolve(double tau_lb, double G, double tau0, double gamma_c, double eps,
                double lam, double g, long long t_startup, int nn_pressure, double uw,
                double dp, int ve, int saf, int zh, orc_params *out) {
  if (!(tau_lb > 0.5) || !(G >= 0) || !(tau0 > 0) || !(gamma_c > 0) ||
      !(lam >= 0 && lam <= 1) || !isfinite(g) || !isfinite(eps) || !isfinite(uw) || !isfinite(dp))
    return -1;
  /* the pressure drive keeps the first line of Eq. (bodyforce) only */
  if (dp != 0 && (g != 0 || nn_pressure || uw != 0)) return -1;
  /* the stress force replaces the second-moment stress term and the
   * flow-induced density, and is defined for the instantaneous model */
  if (saf && (nn_pressure || ve || dp != 0)) return -1;
  /* the node wall closes the channel at the top; it is not combined with the
   * pressure drive or the stress force */
  if (zh && (dp != 0 || saf)) return -1;
  double eta_s = (tau_lb - 0.5) / 3.0;
  double tau = tau0 * pow(10.0, fmin(eps, 0.0) / 0.05);
  double Ginf = G * (1.0 + sqrt(fmax(eps, 0.0)));
  if (lam > 0 && isinf(tau)) return -1;
  out->g = g;
  out->tau_eff = 0.5 + 3.0 * (eta_s + (lam > 0 ? lam * Ginf * tau : 0.0));
  out->G = Ginf;
  out->tau = tau;
  out->gamma_c = gamma_c;
  out->lam = lam;
  out->t_startup = t_startup;
  out->nn_pressure = nn_pressure;
  out->uw = uw;
  out->dp = dp;
  out->ve = ve ? 1 : 0;
  out->saf = saf ? 1 : 0;
  out->zh = zh ? 1 : 0;
  return 0;
}

/* Reading R13: completes the populations of the top node row that enter from
 * outside the lattice (c_y = -1: 4, 7, 8) for step t, following Zou and He's
 * velocity boundary with the wall velocity (u_w, 0) of step t. n holds nine
 * planes of nx*ny post-streaming populations and is changed in place. */
void orc_zou_he_top(const orc_params *p, int nx, int ny, double *n, long long t) {
  const size_t N = (size_t)nx * ny;
  double uw = (t < p->t_startup) ? p->uw : 0.0;
  double fx = (t < p->t_startup) ? p->g : 0.0;
  for (int x = 0; x < nx; ++x) {
    size_t id = (size_t)(ny - 1) * nx + x;
    double v[9];
    for (int i = 0; i < 9; ++i) v[i] = n[i * N + id];
    /* no flow through the wall: sum_i c_iy n_i = 0 with the three unknowns
     * carrying c_y = -1, so s = (c_y = 0 populations) + 2 (c_y = +1 ones) */
    double s = v[0] + v[1] + v[3] + 2.0 * (v[2] + v[5] + v[6]);
    /* momentum the node must hold for u~ = (m + f/2)/s = (u_w, 0) */
    double mx = s * uw - 0.5 * fx;
    /* bounce-back of the non-equilibrium part normal to the wall; n4^eq and
     * n2^eq are equal when the wall has no normal velocity */
    double n4 = v[2];
    /* the diagonals: n7 + n8 = n5 + n6 (no normal flow, given n4 = n2), and
     * n8 - n7 supplies the x momentum the other six lack */
    double sum78 = v[5] + v[6];
    double diff87 = mx - ((v[1] - v[3]) + (v[5] - v[6]));
    double n8 = 0.5 * (sum78 + diff87);
    double n7 = 0.5 * (sum78 - diff87);
    n[4 * N + id] = n4;
    n[7 * N + id] = n7;
    n[8 * N + id] = n8;
  }
}

/* Second-order equilibrium n_i^eq(rho, u) = a_i rho [1 + c.u/cs2 +
 * (c_a c_b - cs2 delta_ab) u_a u_b / (2 cs2^2)]. */
void orc_equilibrium(double rho, double ux, double uy, double neq[9]) {
  for (int i = 0; i < 9; ++i) {
    double cu = CX[i] * ux + CY[i] * uy;
    double quad = 0.0;
    double c[2] = {CX[i], CY[i]}, u[2] = {ux, uy};
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        quad += (c[a] * c[b] - CS2 * (a == b)) * u[a] * u[b];
    neq[i] = W[i] * rho * (1.0 + cu / CS2 + quad / (2.0 * CS2 * CS2));
  }
}

/* Forcing term of Eq. (bodyforce). sbar = traceless non-Newtonian stress
 * (xx, xy, yy), r = dt d(delta rho)/dt, f = body-force density, u = velocity. */
void orc_forcing(double tau, const double sbar[3], double r, double fx, double fy,
                 double ux, double uy, double F[9]) {
  double S[2][2] = {{sbar[0], sbar[1]}, {sbar[1], sbar[2]}};
  double f[2] = {fx, fy}, u[2] = {ux, uy};
  for (int i = 0; i < 9; ++i) {
    double c[2] = {CX[i], CY[i]};
    double stress = 0.0, second = 0.0, cf = 0.0;
    for (int a = 0; a < 2; ++a) {
      cf += f[a] * c[a];
      for (int b = 0; b < 2; ++b) {
        double q = c[a] * c[b] - CS2 * (a == b);
        stress += S[a][b] * q;
        second += q * (-r * u[a] * u[b] + (u[b] * f[a] + u[a] * f[b]));
      }
    }
    F[i] = W[i] * (-stress / (2.0 * CS2 * CS2 * tau) +
                   (1.0 - 1.0 / (2.0 * tau)) *
                       (r + cf / CS2 + second / (2.0 * CS2 * CS2)));
  }
}

/* Steady-state stress of Eq. (sigtsum) for velocity gradient k[a][b] =
 * d_b u_a, relaxation time tau_M and modulus G: sigma = sum_{n>=1} G tau_M^n
 * d^n, summed term by term. Writes (xx, xy, yy). Returns the number of terms
 * used, or -1 if the series has not converged after 1000 terms. */
int orc_stress_series(const double k[2][2], double G, double tauM, double sig[3]) {
  double e[2][2]; /* e = tau_M^n d^n, starting from n = 1: tau_M D */
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) e[a][b] = tauM * (k[a][b] + k[b][a]);
  double s[2][2];
  memcpy(s, e, sizeof s);
  for (int n = 2; n <= 1000; ++n) {
    double nx[2][2];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        double v = 0.0;
        for (int c = 0; c < 2; ++c) v += k[a][c] * e[c][b] + e[a][c] * k[b][c];
        nx[a][b] = tauM * v;
      }
    double tmax = 0.0, smax = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        e[a][b] = nx[a][b];
        s[a][b] += e[a][b];
        if (fabs(e[a][b]) > tmax) tmax = fabs(e[a][b]);
        if (fabs(s[a][b]) > smax) smax = fabs(s[a][b]);
      }
    if (!isfinite(tmax)) break;
    if (tmax <= 1e-18 * smax || tmax == 0.0) {
      sig[0] = G * s[0][0];
      sig[1] = G * s[0][1];
      sig[2] = G * s[1][1];
      return n;
    }
  }
  sig[0] = sig[1] = sig[2] = NAN;
  return -1;
}

/* Shear-dependent Maxwell time of Eq. (nlmaxwell); +inf when both rates vanish. */
double orc_tau_M(const double k[2][2], double tau, double gamma_c) {
  double D[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) D[a][b] = k[a][b] + k[b][a];
  double trD2 = 0.0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) trD2 += D[a][b] * D[b][a];
  double II = 0.5 * trD2;
  double rate = 1.0 / tau + sqrt(II) / gamma_c;
  return 1.0 / rate;
}

/* One step of the time-integrated stress (reading R11): sigma_prev (xx, xy,
 * yy) at step t-1, velocity gradient k[a][b] = d_b u_a of step t, modulus G,
 * relaxation rate 1/tau_M = 1/tau + sqrt(II_D)/gamma_c (Eq. (nlmaxwell)).
 * Writes sigma of step t to sig. */
void orc_stress_ve_step(const double k[2][2], double G, double tau, double gamma_c,
                        const double sigma_prev[3], double sig[3]) {
  double s[2][2] = {{sigma_prev[0], sigma_prev[1]}, {sigma_prev[1], sigma_prev[2]}};
  double D[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) D[a][b] = k[a][b] + k[b][a];
  double trD2 = 0.0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) trD2 += D[a][b] * D[b][a];
  double rate = 1.0 / tau + sqrt(0.5 * trD2) / gamma_c;  /* 1 / tau_M */
  double out[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      /* (kappa sigma + sigma kappa^T)_ab = sum_c k_ac s_cb + s_ac k_bc */
      double conv = 0.0;
      for (int c = 0; c < 2; ++c) conv += k[a][c] * s[c][b] + s[a][c] * k[b][c];
      out[a][b] = (s[a][b] + conv + G * D[a][b]) / (1.0 + rate);
    }
  sig[0] = out[0][0];
  sig[1] = out[0][1];
  sig[2] = out[1][1];
}

/* Per-node observables written by orc_step / orc_observe, field-major
 * [field][y][x]. */
enum {
  OF_UTX, OF_UTY, OF_KXX, OF_KXY, OF_KYX, OF_KYY, OF_SXX, OF_SXY, OF_SYY,
  OF_TRT, OF_R, OF_RHOE, OF_UX, OF_UY, OF_S, OF_MX, OF_MY, OF_TAUM, OF_COUNT
};
int orc_num_fields(void) { return OF_COUNT; }

/* Threads an OpenMP loop of the oracle uses. */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Sets the threads later loops use (for timing at one thread and at all). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_step_saf(const orc_params *p, int nx, int ny, const double *n, const double *P,
                 long long t, double *n_out, double *P_out, double *fields);

/* One time step t -> t+1 of one channel. n: 9 planes of nx*ny post-streaming
 * populations at time t; P: stress trace of step t-1; S: with the
 * time-integrated model (R11), the stress (xx, xy, yy planes) of step t-1,
 * else unused (may be NULL). Writes the state at t+1 to n_out, P_out, S_out
 * (which must not alias n, P, S). If fields != NULL the per-node observables
 * of step t are stored there. If n_out == NULL nothing is advanced
 * (observation only). Returns the number of nodes at which the stress series
 * did not converge (0 on success). */
int orc_step(const orc_params *p, int nx, int ny, const double *n, const double *P,
             const double *S, long long t, double *n_out, double *P_out, double *S_out,
             double *fields) {
  if (p->saf) return orc_step_saf(p, nx, ny, n, P, t, n_out, P_out, fields);
  const size_t N = (size_t)nx * ny;
  double fx = (t < p->t_startup) ? p->g : 0.0, fy = 0.0;
  double uw = (t < p->t_startup) ? p->uw : 0.0;  /* top wall velocity at step t */
  double *utx = malloc(N * sizeof(double)), *uty = malloc(N * sizeof(double));
  int bad = 0;
  /* R13: the top node row's populations from outside, completed for step t */
  double *nz = NULL;
  if (p->zh) {
    nz = malloc(9 * N * sizeof(double));
    memcpy(nz, n, 9 * N * sizeof(double));
    orc_zou_he_top(p, nx, ny, nz, t);
    n = nz;
  }
  /* pressure drive: mean density of the inlet (x = 0) and outlet (x = nx-1)
   * columns; the collision keeps every node's density and momentum then */
  double rbar_in = 0, rbar_out = 0;
  if (p->dp != 0) {
    for (int y = 0; y < ny; ++y)
      for (int i = 0; i < 9; ++i) {
        rbar_in += n[i * N + (size_t)y * nx];
        rbar_out += n[i * N + (size_t)y * nx + nx - 1];
      }
    rbar_in /= ny;
    rbar_out /= ny;
  }

  /* Moments and the provisional velocity u~ = j / sum_i n_i of every node,
   * with j = m + f/2 (Eq. (rhoj), reading R2). */
#pragma omp parallel for
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t id = (size_t)y * nx + x;
      double s = 0, mx = 0, my = 0;
      for (int i = 0; i < 9; ++i) {
        double v = n[i * N + id];
        s += v;
        mx += CX[i] * v;
        my += CY[i] * v;
      }
      utx[id] = (mx + 0.5 * fx) / s;
      uty[id] = (my + 0.5 * fy) / s;
    }

#pragma omp parallel for reduction(+ : bad)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t id = (size_t)y * nx + x;
      double nn[9];
      double s = 0, mx = 0, my = 0;
      for (int i = 0; i < 9; ++i) {
        nn[i] = n[i * N + id];
        s += nn[i];
        mx += CX[i] * nn[i];
        my += CY[i] * nn[i];
      }
      double jx = mx + 0.5 * fx, jy = my + 0.5 * fy;

      /* kappa_ab = d_b u_a by central differences; x periodic, wall ghosts
       * u(-1) = -u(0), u(ny) = 2 u_w - u(ny-1) (readings R4, R5, R9), or
       * u(ny) = 2 u_w - u(ny-2) behind the node wall (R13). */
      int xm = (x - 1 + nx) % nx, xp = (x + 1) % nx;
      double uxm = utx[(size_t)y * nx + xm], uxp = utx[(size_t)y * nx + xp];
      double uym = uty[(size_t)y * nx + xm], uyp = uty[(size_t)y * nx + xp];
      double uxd, uyd, uxu, uyu;
      if (y > 0) { uxd = utx[id - nx]; uyd = uty[id - nx]; }
      else       { uxd = -utx[id];     uyd = -uty[id]; }
      if (y < ny - 1) { uxu = utx[id + nx]; uyu = uty[id + nx]; }
      else if (p->zh) { uxu = 2.0 * uw - utx[id - nx]; uyu = -uty[id - nx]; }
      else            { uxu = 2.0 * uw - utx[id]; uyu = -uty[id]; }
      double k[2][2];
      k[0][0] = 0.5 * (uxp - uxm);  /* d_x u_x */
      k[0][1] = 0.5 * (uxu - uxd);  /* d_y u_x */
      k[1][0] = 0.5 * (uyp - uym);  /* d_x u_y */
      k[1][1] = 0.5 * (uyu - uyd);  /* d_y u_y */

      /* inlM stress: Maxwell time of Eq. (nlmaxwell), then Eq. (sigtsum);
       * time-integrated model: one step of reading R11 from the stress of
       * the previous step. */
      double sig[3] = {0, 0, 0};
      double tauM = orc_tau_M(k, p->tau, p->gamma_c);
      if (p->ve) {
        const double sp[3] = {S[id], S[N + id], S[2 * N + id]};
        orc_stress_ve_step(k, p->G, p->tau, p->gamma_c, sp, sig);
      } else if (p->G > 0 && isfinite(tauM)) {
        if (orc_stress_series(k, p->G, tauM, sig) < 0) bad++;
      }
      /* inlM: tau_M infinite means tau = inf and D = 0, the series is zero. */

      /* Non-Newtonian stress carried by the forcing (viscosity split). */
      double D[2][2] = {{2 * k[0][0], k[0][1] + k[1][0]}, {k[0][1] + k[1][0], 2 * k[1][1]}};
      double lgt = (p->lam > 0) ? p->lam * p->G * p->tau : 0.0;
      double T[3] = {sig[0] - lgt * D[0][0], sig[1] - lgt * D[0][1], sig[2] - lgt * D[1][1]};
      double trT = T[0] + T[2];
      double sbar[3] = {T[0] - 0.5 * trT, T[1], T[2] - 0.5 * trT};

      /* Eq. (rhoplus): delta rho = -tr Sigma^nN / (cs2 d), and
       * r = dt d(delta rho)/dt is its change since the last step. */
      double r = 0.0;
      if (p->nn_pressure) {
        double drho_now = -trT / (CS2 * 2.0);
        double drho_prev = -P[id] / (CS2 * 2.0);
        r = drho_now - drho_prev;
      }

      /* Eq. (rhoj) with reading R1: rho_e = sum (n* + n)/2 = s + r/2. */
      double rho_e = s + 0.5 * r;
      double ux = jx / rho_e, uy = jy / rho_e;

      double neq[9], F[9];
      orc_equilibrium(rho_e, ux, uy, neq);
      orc_forcing(p->tau_eff, sbar, r, fx, fy, ux, uy, F);

      if (fields) {
        double vals[OF_COUNT] = {utx[id], uty[id], k[0][0], k[0][1], k[1][0], k[1][1],
                                 sig[0], sig[1], sig[2], trT, r, rho_e, ux, uy, s, mx, my,
                                 tauM};
        for (int q = 0; q < OF_COUNT; ++q) fields[q * N + id] = vals[q];
      }
      if (!n_out) continue;

      /* Collide (BGK + forcing) and stream; links leaving through a wall are
       * reflected back to the same node (half-way bounce-back); at the moving
       * top wall the reflected population gains the wall's momentum,
       * -2 a_i (c_i . u_w) / cs2 with the wall density rho0 = 1 (R9). Behind
       * the node wall of R13 there is no lattice: what leaves upwards is
       * gone. */
      for (int i = 0; i < 9; ++i) {
        double post = nn[i] - (nn[i] - neq[i]) / p->tau_eff + F[i];
        int xd = (x + CX[i] + nx) % nx, yd = y + CY[i];
        if (p->dp != 0 && yd >= 0 && yd < ny && (x + CX[i] < 0 || x + CX[i] >= nx)) {
          /* a link across the periodic boundary: equilibrium at the target
           * end's density, the source's non-equilibrium part (R10) */
          double dpn = (t < p->t_startup) ? p->dp : 0.0;  /* on for t < t_startup */
          double target = (x == nx - 1) ? 1.0 + 1.5 * dpn - rbar_out : 1.0 - 1.5 * dpn - rbar_in;
          double ea[9], eb[9];
          orc_equilibrium(s + target, mx / (s + target), my / (s + target), ea);
          orc_equilibrium(s, mx / s, my / s, eb);
          post += ea[i] - eb[i];
        }
        if (yd >= 0 && yd < ny)
          n_out[i * N + (size_t)yd * nx + xd] = post;
        else if (yd >= ny && p->zh)
          continue;
        else if (yd >= ny)
          n_out[opposite(i) * N + id] = post - 2.0 * W[i] * (CX[i] * uw) / CS2;
        else
          n_out[opposite(i) * N + id] = post;
      }
      P_out[id] = trT;
      if (p->ve) {
        S_out[id] = sig[0];
        S_out[N + id] = sig[1];
        S_out[2 * N + id] = sig[2];
      }
    }
  free(utx);
  free(uty);
  free(nz);
  /* R13: the state handed on is complete for the next step */
  if (p->zh && n_out) orc_zou_he_top(p, nx, ny, n_out, t + 1);
  return bad;
}

/* Non-Newtonian stress Sigma^nN (xx, xy, yy) of every node at step t, into
 * T[3][ny][nx] (reading R12, first pass); velocity gradient from
 * u~ = (m + rho0 g / 2)/s. Returns the count of non-converged series. */
static int saf_stress(const orc_params *p, int nx, int ny, const double *n, long long t, double *T) {
  const size_t N = (size_t)nx * ny;
  double fx = (t < p->t_startup) ? p->g : 0.0;
  double uw = (t < p->t_startup) ? p->uw : 0.0;
  double *utx = malloc(N * sizeof(double)), *uty = malloc(N * sizeof(double));
  int bad = 0;
#pragma omp parallel for
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t id = (size_t)y * nx + x;
      double s = 0, mx = 0, my = 0;
      for (int i = 0; i < 9; ++i) {
        double v = n[i * N + id];
        s += v;
        mx += CX[i] * v;
        my += CY[i] * v;
      }
      utx[id] = (mx + 0.5 * fx) / s;
      uty[id] = my / s;
    }
#pragma omp parallel for reduction(+ : bad)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t id = (size_t)y * nx + x;
      int xm = (x - 1 + nx) % nx, xp = (x + 1) % nx;
      double uxd, uyd, uxu, uyu;
      if (y > 0) { uxd = utx[id - nx]; uyd = uty[id - nx]; }
      else       { uxd = -utx[id];     uyd = -uty[id]; }
      if (y < ny - 1) { uxu = utx[id + nx]; uyu = uty[id + nx]; }
      else            { uxu = 2.0 * uw - utx[id]; uyu = -uty[id]; }
      double k[2][2];
      k[0][0] = 0.5 * (utx[(size_t)y * nx + xp] - utx[(size_t)y * nx + xm]);
      k[0][1] = 0.5 * (uxu - uxd);
      k[1][0] = 0.5 * (uty[(size_t)y * nx + xp] - uty[(size_t)y * nx + xm]);
      k[1][1] = 0.5 * (uyu - uyd);
      double sig[3] = {0, 0, 0};
      double tauM = orc_tau_M(k, p->tau, p->gamma_c);
      if (p->G > 0 && isfinite(tauM))
        if (orc_stress_series(k, p->G, tauM, sig) < 0) bad++;
      double lgt = (p->lam > 0) ? p->lam * p->G * p->tau : 0.0;
      T[id] = sig[0] - lgt * 2 * k[0][0];
      T[N + id] = sig[1] - lgt * (k[0][1] + k[1][0]);
      T[2 * N + id] = sig[2] - lgt * 2 * k[1][1];
    }
  free(utx);
  free(uty);
  return bad;
}

/* Reading R12: one step t -> t+1 with the stress as a force density. Same
 * arguments as orc_step (P is carried unchanged: there is no flow-induced
 * density). The fields of step t are stored if fields != NULL. */
int orc_step_saf(const orc_params *p, int nx, int ny, const double *n, const double *P,
                 long long t, double *n_out, double *P_out, double *fields) {
  const size_t N = (size_t)nx * ny;
  double g = (t < p->t_startup) ? p->g : 0.0;
  double uw = (t < p->t_startup) ? p->uw : 0.0;
  double *T = malloc(3 * N * sizeof(double));
  int bad = saf_stress(p, nx, ny, n, t, T);
  /* stress component c at (x, y), with the linearly extrapolated ghost rows */
#define TS(c, x, y) T[(size_t)(c) * N + (size_t)(y) * nx + (x)]
  double *utx = malloc(N * sizeof(double)), *uty = malloc(N * sizeof(double));
#pragma omp parallel for
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t id = (size_t)y * nx + x;
      double s = 0, mx = 0, my = 0;
      for (int i = 0; i < 9; ++i) {
        s += n[i * N + id];
        mx += CX[i] * n[i * N + id];
        my += CY[i] * n[i * N + id];
      }
      utx[id] = (mx + 0.5 * g) / s;
      uty[id] = my / s;
    }
#pragma omp parallel for
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t id = (size_t)y * nx + x;
      int xm = (x - 1 + nx) % nx, xp = (x + 1) % nx;
      double Tdn[3], Tup[3];
      for (int c = 0; c < 3; ++c) {
        if (ny == 1) {
          Tdn[c] = Tup[c] = TS(c, x, y);
        } else {
          Tdn[c] = (y > 0) ? TS(c, x, y - 1) : 2 * TS(c, x, 0) - TS(c, x, 1);
          Tup[c] = (y < ny - 1) ? TS(c, x, y + 1) : 2 * TS(c, x, ny - 1) - TS(c, x, ny - 2);
        }
      }
      /* (div Sigma)_a = d_x Sigma_xa + d_y Sigma_ya */
      double fsx = 0.5 * (TS(0, xp, y) - TS(0, xm, y)) + 0.5 * (Tup[1] - Tdn[1]);
      double fsy = 0.5 * (TS(1, xp, y) - TS(1, xm, y)) + 0.5 * (Tup[2] - Tdn[2]);
      double fx = g + fsx, fy = fsy;
      double nn[9], s = 0, mx = 0, my = 0;
      for (int i = 0; i < 9; ++i) {
        nn[i] = n[i * N + id];
        s += nn[i];
        mx += CX[i] * nn[i];
        my += CY[i] * nn[i];
      }
      double ux = (mx + 0.5 * fx) / s, uy = (my + 0.5 * fy) / s;
      double neq[9], F[9];
      const double zero[3] = {0, 0, 0};
      orc_equilibrium(s, ux, uy, neq);
      orc_forcing(p->tau_eff, zero, 0.0, fx, fy, ux, uy, F);
      if (fields) {
        double uxd = (y > 0) ? utx[id - nx] : -utx[id], uxu = (y < ny - 1) ? utx[id + nx] : 2.0 * uw - utx[id];
        double uyd = (y > 0) ? uty[id - nx] : -uty[id], uyu = (y < ny - 1) ? uty[id + nx] : -uty[id];
        double k[2][2] = {{0.5 * (utx[(size_t)y * nx + xp] - utx[(size_t)y * nx + xm]), 0.5 * (uxu - uxd)},
                          {0.5 * (uty[(size_t)y * nx + xp] - uty[(size_t)y * nx + xm]), 0.5 * (uyu - uyd)}};
        double tauM = orc_tau_M(k, p->tau, p->gamma_c);
        double lgt = (p->lam > 0) ? p->lam * p->G * p->tau : 0.0;
        /* sigma recovered from Sigma^nN by adding the split part back */
        double sxx = TS(0, x, y) + lgt * 2 * k[0][0], sxy = TS(1, x, y) + lgt * (k[0][1] + k[1][0]);
        double syy = TS(2, x, y) + lgt * 2 * k[1][1];
        double vals[OF_COUNT] = {utx[id], uty[id], k[0][0], k[0][1], k[1][0], k[1][1], sxx, sxy, syy,
                                 TS(0, x, y) + TS(2, x, y), 0.0, s, ux, uy, s, mx, my, tauM};
        for (int q = 0; q < OF_COUNT; ++q) fields[q * N + id] = vals[q];
      }
      if (!n_out) continue;
      for (int i = 0; i < 9; ++i) {
        double post = nn[i] - (nn[i] - neq[i]) / p->tau_eff + F[i];
        int xd = (x + CX[i] + nx) % nx, yd = y + CY[i];
        if (yd >= 0 && yd < ny)
          n_out[i * N + (size_t)yd * nx + xd] = post;
        else if (yd >= ny)
          n_out[opposite(i) * N + id] = post - 2.0 * W[i] * (CX[i] * uw) / CS2;
        else
          n_out[opposite(i) * N + id] = post;
      }
      P_out[id] = P[id];
    }
#undef TS
  free(T);
  free(utx);
  free(uty);
  return bad;
}

/* Rest state: n_i = a_i, P = 0, and (if S != NULL) zero stress. */
void orc_init_rest(int nx, int ny, double *n, double *P, double *S) {
  const size_t N = (size_t)nx * ny;
  for (int i = 0; i < 9; ++i)
    for (size_t id = 0; id < N; ++id) n[i * N + id] = W[i];
  for (size_t id = 0; id < N; ++id) P[id] = 0.0;
  if (S)
    for (size_t id = 0; id < 3 * N; ++id) S[id] = 0.0;
}

/* Advances (n, P, and S with the time-integrated model) in place from step t0
 * by nsteps. Returns the total count of non-converged stress evaluations, or
 * -1 on allocation failure. */
long long orc_run(const orc_params *p, int nx, int ny, double *n, double *P, double *S,
                  long long t0, long long nsteps) {
  const size_t N = (size_t)nx * ny;
  double *n2 = malloc(9 * N * sizeof(double)), *P2 = malloc(N * sizeof(double));
  double *S2 = p->ve ? malloc(3 * N * sizeof(double)) : NULL;
  if (!n2 || !P2 || (p->ve && !S2)) { free(n2); free(P2); free(S2); return -1; }
  long long bad = 0;
  for (long long s = 0; s < nsteps; ++s) {
    bad += orc_step(p, nx, ny, n, P, S, t0 + s, n2, P2, S2, NULL);
    memcpy(n, n2, 9 * N * sizeof(double));
    memcpy(P, P2, N * sizeof(double));
    if (p->ve) memcpy(S, S2, 3 * N * sizeof(double));
  }
  free(n2);
  free(P2);
  free(S2);
  return bad;
}

/* Momentum handed to the walls by the bounce-back links during the step that
 * produced the current state: the populations that were reflected are the
 * ones now travelling away from the wall in the wall rows. uw is the top
 * wall's velocity during that step: a reflected population n_i there left as
 * n_i + 2 a_i (c_i . u_w)/cs2 in the opposite direction. */
double orc_wall_drag(int nx, int ny, const double *n, double uw) {
  const size_t N = (size_t)nx * ny;
  double w = 0.0;
  for (int x = 0; x < nx; ++x) {
    size_t b = (size_t)x, t = (size_t)(ny - 1) * nx + x;
    for (int i = 0; i < 9; ++i) {
      /* bottom wall: populations now moving up (cy = +1) came from links
       * that pointed down, with x velocity -cx */
      if (CY[i] == 1) w += 2.0 * (-CX[i]) * n[i * N + b];
      if (CY[i] == -1) w += -CX[i] * (2.0 * n[i * N + t] + 2.0 * W[i] * (-CX[i] * uw) / CS2);
    }
  }
  return w;
}
