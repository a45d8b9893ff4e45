/*
 * Driver for the sanitizer build of the oracle (tests/test_oracle_sanitizers.py).
 *
 * Built together with oracle/oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer (no OpenMP), it calls every entry point of
 * oracle.h on small grids -- both lattices, periodic and zero-gradient axes,
 * both anomaly differences, a general caloric law, degenerate 1-node axes --
 * so that an out-of-bounds access, a leak or undefined arithmetic anywhere in
 * the oracle stops the run.  It also checks that a periodic box keeps its
 * mass (Eq. (3)) and that invalid parameters are refused.  Exit status 0 on
 * success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

static int failures = 0;

#define CHECK(cond)                                                   \
  do {                                                                \
    if (!(cond)) {                                                    \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

static void fields(long N, int D, long nx, long ny, double* rho, double* u, double* T) {
  for (long n = 0; n < N; ++n) {
    double x = (double)(n % nx), y = (double)((n / nx) % ny), z = (double)(n / (nx * ny));
    rho[n] = 1.0 + 0.05 * sin(0.7 * x + 0.3 * y + 0.2 * z);
    T[n] = 0.15 + 0.02 * cos(0.4 * x - 0.5 * y + 0.1 * z);
    for (int a = 0; a < D; ++a) u[a * N + n] = 0.05 * sin(0.3 * (a + 1) * x + 0.6 * y - 0.2 * a * z + a);
  }
}

static void run_case(int D, long nx, long ny, long nz, int bcx, int bcy, int bcz, int deriv, const double* cv) {
  orc_params p = {0};
  p.D = D;
  p.n[0] = nx;
  p.n[1] = ny;
  p.n[2] = nz;
  p.bc[0] = bcx;
  p.bc[1] = bcy;
  p.bc[2] = bcz;
  p.gamma = 1.4;
  p.Pr = 0.71;
  p.mu0 = 0.02;
  p.visc_exp = 0.76;
  p.T_ref = 0.15;
  p.deriv = deriv;
  if (cv)
    for (int k = 0; k < 3; ++k) p.cv[k] = cv[k];
  orc_sim* s = orc_create(&p);
  CHECK(s != NULL);
  if (!s) return;
  const long N = nx * ny * nz;
  const int Q = orc_Q(D);
  double* rho = malloc(sizeof(double) * N);
  double* u = malloc(sizeof(double) * N * D);
  double* T = malloc(sizeof(double) * N);
  double* f = malloc(sizeof(double) * N * Q);
  double* g = malloc(sizeof(double) * N * Q);
  fields(N, D, nx, ny, rho, u, T);
  CHECK(orc_init(s, rho, u, T) == 0);
  double d0[ORC_NDIAG], d1[ORC_NDIAG];
  CHECK(orc_diagnostics(s, d0) == 0);
  CHECK(orc_step(s, 3) == 0);
  CHECK(orc_step_count(s) == 3);
  CHECK(orc_diagnostics(s, d1) == 0);
  if (bcx == ORC_PERIODIC && bcy == ORC_PERIODIC && bcz == ORC_PERIODIC)
    CHECK(fabs(d1[ORC_D_MASS] - d0[ORC_D_MASS]) <= 1e-12 * d0[ORC_D_MASS]);
  CHECK(d1[ORC_D_NONFINITE] == 0.0 && d1[ORC_D_NODES] == (double)N);
  CHECK(orc_moments(s, rho, u, T) == 0);
  long nodes[4] = {0, N - 1, N / 2, 0};
  signed char branch[12];
  for (int k = 0; k < 12; ++k) branch[k] = (signed char)(k % 3 - 1);
  double* fs = malloc(sizeof(double) * Q * 4);
  double* gs = malloc(sizeof(double) * Q * 4);
  CHECK(orc_step_sampled(s, nodes, 4, fs, gs) == 0);
  CHECK(orc_step_sampled_branch(s, nodes, 4, branch, fs, gs) == 0);
  long bad_node[1] = {N};
  CHECK(orc_step_sampled_branch(s, bad_node, 1, NULL, fs, gs) == -1);
  CHECK(orc_get_pops(s, f, g) == 0);
  CHECK(orc_set_pops(s, f, g, 7) == 0);
  double fr[27], gr[27], u0[3] = {0, 0, 0};
  orc_feq(D, 1.0, u0, 0.15, fr);
  orc_geq(D, 1.0, u0, 0.15, 2.5, gr);
  CHECK(orc_set_fp32_storage(s, fr, gr) == 0);
  CHECK(orc_step(s, 1) == 0);
  CHECK(orc_set_fp32_storage(s, NULL, NULL) == 0);
  double* out = malloc(sizeof(double) * N);
  double* Qt = malloc(sizeof(double) * N);
  for (long n = 0; n < N; ++n) Qt[n] = orc_anomaly(rho[n], u[n], T[n]);
  for (int a = 0; a < D; ++a) orc_derivative(s, a, Qt, u + a * N, out);
  free(out);
  free(Qt);
  free(fs);
  free(gs);
  free(rho);
  free(u);
  free(T);
  free(f);
  free(g);
  orc_destroy(s);
}

static void nodal(int D) {
  double u[3] = {0.1, -0.05, 0.02}, d[3] = {1e-3, -2e-3, 5e-4}, P[9] = {0};
  double f[27], g[27], fh[27], gh[27], fo[27], go[27], dq[3];
  orc_feq(D, 1.1, u, 0.15, f);
  orc_fex(D, 1.1, u, 0.15, 1.3, d, f);
  orc_geq(D, 1.1, u, 0.15, 2.5, g);
  orc_geq_u(D, 1.1, u, 0.15, 0.4, g);
  for (int a = 0; a < D; ++a) P[a * D + a] = 0.2;
  orc_dq(D, 1.1, u, 0.15, P, d, dq);
  orc_gstar(D, 1.1, u, 0.15, 2.5, P, d, g);
  double xi[3] = {0.1, 0.2, 0.3}, PP[3] = {0.3, 0.3, 0.3};
  orc_product_form(D, 1.0, xi, PP, f);
  orc_feq(D, 1.0, u, 0.15, fh);
  orc_geq(D, 1.0, u, 0.15, 2.5, gh);
  orc_params p = {0};
  p.D = D;
  p.n[0] = p.n[1] = p.n[2] = 1;
  p.gamma = 1.4;
  p.Pr = 0.7;
  p.mu0 = 0.01;
  p.T_ref = 0.15;
  orc_collide_node(&p, fh, gh, d, fo, go);
  double cv[3] = {1.5, 5.0, 20.0};
  double e = orc_internal_energy(cv, 0.2);
  CHECK(fabs(orc_temperature(cv, e) - 0.2) <= 1e-14);
  orc_caloric(&p, cv);
  CHECK(fabs(cv[0] - 2.5) <= 1e-12);
  CHECK(orc_omega(0.02, 1.0, 0.15) > 0.0 && orc_omega1(1.2, 0.7) > 0.0);
}

int main(void) {
  const double law[3] = {1.5, 5.0, 20.0};
  run_case(3, 5, 4, 3, ORC_PERIODIC, ORC_PERIODIC, ORC_PERIODIC, ORC_UPWIND, NULL);
  run_case(3, 4, 3, 5, ORC_ZERO_GRADIENT, ORC_PERIODIC, ORC_ZERO_GRADIENT, ORC_CENTRAL, NULL);
  run_case(3, 1, 1, 1, ORC_PERIODIC, ORC_PERIODIC, ORC_PERIODIC, ORC_UPWIND, NULL);
  run_case(3, 3, 1, 2, ORC_ZERO_GRADIENT, ORC_ZERO_GRADIENT, ORC_PERIODIC, ORC_UPWIND, law);
  run_case(2, 7, 5, 1, ORC_ZERO_GRADIENT, ORC_PERIODIC, ORC_PERIODIC, ORC_UPWIND, NULL);
  run_case(2, 1, 1, 1, ORC_PERIODIC, ORC_PERIODIC, ORC_PERIODIC, ORC_CENTRAL, law);
  nodal(2);
  nodal(3);
  orc_params bad = {0};
  bad.D = 3;
  bad.n[0] = bad.n[1] = bad.n[2] = 2;
  bad.gamma = 1.0; /* gamma must exceed 1 */
  bad.Pr = 0.7;
  bad.mu0 = 0.01;
  CHECK(orc_create(&bad) == NULL);
  bad.gamma = 1.4;
  bad.D = 4;
  CHECK(orc_create(&bad) == NULL);
  orc_destroy(NULL);
  if (failures) fprintf(stderr, "%d check(s) failed\n", failures);
  else printf("oracle sanitizer run: all checks passed\n");
  return failures ? 1 : 0;
}
