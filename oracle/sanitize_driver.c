/*
 * TEST INFRASTRUCTURE: drives every mode of the FP64 oracle (lb_oracle.c) for
 * a few steps on small lattices so that the oracle can be built and run under
 * AddressSanitizer and UndefinedBehaviorSanitizer on the host. Exit status 0
 * when every run completed with finite populations and (where the method
 * conserves it) the mass unchanged to round-off.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  double g, tau_eff, G, tau, gamma_c, lam;
  long long t_startup;
  int nn_pressure;
  double uw, dp;
  int ve, saf, zh;
} orc_params;

int orc_resolve(double tau_lb, double G, double tau0, double gamma_c, double eps, double lam, double g,
                long long t_startup, int nn_pressure, double uw, double dp, int ve, int saf, int zh, orc_params *out);
void orc_init_rest(int nx, int ny, double *n, double *P, double *S);
long long orc_run(const orc_params *p, int nx, int ny, double *n, double *P, double *S, long long t0,
                  long long nsteps);
int orc_step(const orc_params *p, int nx, int ny, const double *n, const double *P, const double *S, long long t,
             double *n_out, double *P_out, double *S_out, double *fields);
int orc_num_fields(void);
double orc_wall_drag(int nx, int ny, const double *n, double uw);
void orc_zou_he_top(const orc_params *p, int nx, int ny, double *n, long long t);

static int run_case(const char *name, int nx, int ny, double g, double lam, int nnp, double uw, double dp, int ve,
                    int saf, int zh, int check_mass) {
  orc_params p;
  if (orc_resolve(0.8, 2e-4, 500.0, 0.1, 0.01, lam, g, 7, nnp, uw, dp, ve, saf, zh, &p) != 0) {
    printf("%s: rejected\n", name);
    return 1;
  }
  const size_t N = (size_t)nx * ny;
  double *n = malloc(9 * N * sizeof(double)), *P = malloc(N * sizeof(double)), *S = malloc(3 * N * sizeof(double));
  double *f = malloc((size_t)orc_num_fields() * N * sizeof(double));
  orc_init_rest(nx, ny, n, P, S);
  if (zh) orc_zou_he_top(&p, nx, ny, n, 0);
  /* a small deterministic perturbation so that every term is exercised */
  for (size_t i = 0; i < 9 * N; ++i) n[i] *= 1.0 + 1e-4 * sin(0.7 * (double)i);
  double m0 = 0;
  for (size_t i = 0; i < 9 * N; ++i) m0 += n[i];
  long long bad = orc_run(&p, nx, ny, n, P, S, 0, 12);
  orc_step(&p, nx, ny, n, P, S, 12, NULL, NULL, NULL, f);
  (void)orc_wall_drag(nx, ny, n, uw);
  double m1 = 0;
  int finite = 1;
  for (size_t i = 0; i < 9 * N; ++i) {
    m1 += n[i];
    finite &= isfinite(n[i]);
  }
  int ok = finite && bad == 0 && (!check_mass || fabs(m1 - m0) < 1e-12 * (double)N);
  printf("%s: %s (mass change %.2e)\n", name, ok ? "ok" : "FAILED", m1 - m0);
  free(n);
  free(P);
  free(S);
  free(f);
  return ok ? 0 : 1;
}

int main(void) {
  int fails = 0;
  fails += run_case("plain", 5, 7, 1e-6, 0.3, 1, 0.0, 0.0, 0, 0, 0, 0);
  fails += run_case("no delta-rho", 4, 9, 1e-6, 0.0, 0, 0.0, 0.0, 0, 0, 0, 1);
  fails += run_case("one row", 3, 1, 1e-6, 0.0, 0, 0.0, 0.0, 0, 0, 0, 1);
  fails += run_case("half-link moving wall", 6, 5, 0.0, 0.5, 0, 0.02, 0.0, 0, 0, 0, 1);
  fails += run_case("zou-he wall", 6, 5, 1e-6, 0.5, 0, 0.02, 0.0, 0, 0, 1, 0);
  fails += run_case("zou-he two rows", 3, 2, 0.0, 0.0, 1, 0.01, 0.0, 1, 0, 1, 0);
  fails += run_case("viscoelastic", 5, 6, 1e-6, 0.3, 1, 0.0, 0.0, 1, 0, 0, 0);
  fails += run_case("pressure drive", 7, 5, 0.0, 0.0, 0, 0.0, 1e-5, 0, 0, 0, 0);
  fails += run_case("stress force", 5, 6, 1e-6, 0.3, 0, 0.0, 0.0, 0, 1, 0, 1);
  fails += run_case("stress force one row", 4, 1, 1e-6, 0.0, 0, 0.0, 0.0, 0, 1, 0, 1);
  return fails ? 1 : 0;
}
