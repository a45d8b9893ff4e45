/*
 * CPU oracle of the two-population compressible lattice Boltzmann model of
 * Saadat, Hosseini, Dorschner and Karlin (arXiv:2102.09512).
 *
 * TEST INFRASTRUCTURE: the plain, slow FP64 reference the GPU library is
 * checked against.  Only tests, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares nothing with the GPU library.
 *
 * One time step is two whole-field passes, in the order the method needs:
 *   pass 1, every node: pull the post-collision populations along c_i
 *           (streaming, Eqs. (1)-(2)); moments rho, u, P, E, T (Eqs. (3)-(7),
 *           (47)); relaxation frequencies omega, omega_1 (Eqs. (92), (96));
 *           the diagonal anomaly Qt_a (Eq. (29)).
 *   pass 2, every node: the discrete derivative of Qt_a (Sec. III.A); the
 *           extended equilibrium f^ex (Eqs. (28), (30)); the energy
 *           equilibrium g^eq (Eq. (42)); the quasi-equilibrium g* (Eqs. (44),
 *           (46)); BGK relaxation of f and g (Eqs. (1), (2)).
 *
 * Readings of points the paper leaves open (each applies to the GPU library
 * as well):
 *   - the upwind side of d_a is chosen by u_a at the node where the derivative
 *     is taken; u_a == 0 takes the "otherwise" (forward) branch;
 *   - the anomaly and its derivative use the post-streaming moments of the
 *     same step;
 *   - P in Eq. (46) is the pressure tensor of the post-streaming populations
 *     and P^eq = rho T I + rho u u (Eqs. (23), (25));
 *   - omega follows the local rho T through Eq. (92) (mu is the dynamic
 *     viscosity), omega_1 follows from Eq. (96);
 *   - initial populations are f^eq and g^eq;
 *   - zero-gradient boundaries clamp the source index of streaming and the
 *     neighbour index of every difference to the domain;
 *   - D2Q9 uses the same formulas with the z factor dropped (the product form
 *     summed over c_z is the identity).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QMAX 27

struct orc_sim {
  orc_params p;
  long N;
  int Q;
  double cv[3]; /* caloric law in effect */
  long step;
  double* f;  /* [Q][N] post-collision populations */
  double* g;
  double* fh; /* [Q][N] post-streaming populations of the current step */
  double* gh;
  /* per-node moments of the post-streaming state (pass 1) */
  double* rho;
  double* u;     /* [D][N] */
  double* T;
  double* Qt;    /* [D][N] diagonal anomaly */
  double* d;     /* [N] scratch for one derivative */
  double* dd;    /* [D][N] derivatives */
  /* FP32 storage model (orc_set_fp32_storage): reference populations whose
     deviations are rounded to single precision after init and every step */
  int fp32_store;
  double fref[QMAX], gref[QMAX];
  /* upwind decisions with |u| <= band take the other side (orc_set_upwind_band) */
  double band;
};

static void round_storage(orc_sim* s);

int orc_Q(int D) { return D == 2 ? 9 : 27; }

void orc_velocity(int D, int i, int* c) {
  c[0] = i % 3 - 1;
  c[1] = (i / 3) % 3 - 1;
  c[2] = (D == 3) ? (i / 9) % 3 - 1 : 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the following parallel loops (n >= 1); the node arithmetic and
   every summation order are the same for any count. */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Product form, Sec. II.B                                                  */
/* ------------------------------------------------------------------------ */

/* The triplet Psi_0 = 1 - P, Psi_{+1} = (xi + P)/2, Psi_{-1} = (-xi + P)/2, Eqs. (9)-(11). */
static double psi(int c, double xi, double P) {
  if (c == 0) return 1.0 - P;
  if (c == 1) return 0.5 * (xi + P);
  return 0.5 * (-xi + P);
}

/* rho * Psi_{c_ix}(xi_x, P_xx) Psi_{c_iy}(xi_y, P_yy) [Psi_{c_iz}(xi_z, P_zz)], Eq. (12). */
void orc_product_form(int D, double rho, const double* xi, const double* P, double* out) {
  int Q = orc_Q(D);
  for (int i = 0; i < Q; ++i) {
    int c[3];
    orc_velocity(D, i, c);
    double v = rho;
    for (int a = 0; a < D; ++a) v *= psi(c[a], xi[a], P[a]);
    out[i] = v;
  }
}

/* f^eq: xi_a = u_a, P_aa = R T + u_a^2, Eqs. (18)-(20). */
void orc_feq(int D, double rho, const double* u, double T, double* f) {
  double P[3];
  for (int a = 0; a < D; ++a) P[a] = T + u[a] * u[a];
  orc_product_form(D, rho, u, P, f);
}

/* f^ex: P_aa^ex = P_aa^eq + delta_t (2 - omega)/(2 rho omega) d_a Qt_aaa, Eqs. (28), (30). */
void orc_fex(int D, double rho, const double* u, double T, double omega, const double* d, double* f) {
  double P[3];
  for (int a = 0; a < D; ++a) P[a] = T + u[a] * u[a] + (2.0 - omega) / (2.0 * rho * omega) * d[a];
  orc_product_form(D, rho, u, P, f);
}

/* Diagonal anomaly Qt_aaa = rho u_a (1 - 3 R T) - rho u_a^3, Eq. (29). */
double orc_anomaly(double rho, double u, double T) { return rho * u * (1.0 - 3.0 * T) - rho * u * u * u; }

/* ------------------------------------------------------------------------ */
/* Energy equilibrium by the operator product form, Sec. II.D               */
/* ------------------------------------------------------------------------ */

/* A polynomial in one velocity component u_a (T is a parameter, not a variable). */
#define PDEG 8
typedef struct {
  double c[PDEG + 1];
} poly;

/* O_a A = R T dA/du_a + u_a A, Eq. (33), on a function of u_a alone. */
static poly apply_O(const poly* A, double T) {
  poly r;
  memset(&r, 0, sizeof r);
  for (int k = 1; k <= PDEG; ++k) r.c[k - 1] += T * (double)k * A->c[k];
  for (int k = 0; k < PDEG; ++k) r.c[k + 1] += A->c[k];
  return r;
}

static double poly_eval(const poly* A, double u) {
  double v = 0.0;
  for (int k = PDEG; k >= 0; --k) v = v * u + A->c[k];
  return v;
}

/* Psi_c(O, O^2) A with xi = O and P = O^2 substituted into Eqs. (9)-(11), per
   Eqs. (40)-(41): Psi_0 = 1 - O^2, Psi_{+1} = (O + O^2)/2, Psi_{-1} = (-O + O^2)/2. */
static poly apply_psi_op(int c, const poly* A, double T) {
  poly o1 = apply_O(A, T);
  poly o2 = apply_O(&o1, T);
  poly r;
  for (int k = 0; k <= PDEG; ++k) {
    if (c == 0) r.c[k] = A->c[k] - o2.c[k];
    else if (c == 1) r.c[k] = 0.5 * (o1.c[k] + o2.c[k]);
    else r.c[k] = 0.5 * (-o1.c[k] + o2.c[k]);
  }
  return r;
}

/* g^eq_i = rho prod_a Psi_{c_ia}(O_a, O_a^2) E, Eq. (42), with the generating
   function E = U(T) + |u|^2 / 2 (Eqs. (6)-(7), T_ref = 0).
   E is a sum of terms that factor over the velocity components,
     E = U * 1 * 1 * 1 + sum_a (u_a^2 / 2) * prod_{b != a} 1,
   U does not depend on u, and O_a acts on the u_a factor only, so each term
   is transformed factor by factor with the one-variable operator above. */
void orc_geq_u(int D, double rho, const double* u, double T, double U, double* g) {
  int Q = orc_Q(D);
  poly one, sq;
  memset(&one, 0, sizeof one);
  memset(&sq, 0, sizeof sq);
  one.c[0] = 1.0;
  sq.c[2] = 1.0;
  /* t_one[a][c+1] = (Psi_c(O_a, O_a^2) 1)(u_a), t_sq[a][c+1] = (Psi_c(O_a, O_a^2) u_a^2)(u_a) */
  double t_one[3][3], t_sq[3][3];
  for (int a = 0; a < D; ++a)
    for (int c = -1; c <= 1; ++c) {
      poly p1 = apply_psi_op(c, &one, T);
      poly p2 = apply_psi_op(c, &sq, T);
      t_one[a][c + 1] = poly_eval(&p1, u[a]);
      t_sq[a][c + 1] = poly_eval(&p2, u[a]);
    }
  for (int i = 0; i < Q; ++i) {
    int c[3];
    orc_velocity(D, i, c);
    double s = U;
    for (int a = 0; a < D; ++a) s *= t_one[a][c[a] + 1];
    for (int a = 0; a < D; ++a) {
      double t = 0.5 * t_sq[a][c[a] + 1];
      for (int b = 0; b < D; ++b)
        if (b != a) t *= t_one[b][c[b] + 1];
      s += t;
    }
    g[i] = rho * s;
  }
}

/* Constant C_v: U = C_v T. */
void orc_geq(int D, double rho, const double* u, double T, double Cv, double* g) {
  orc_geq_u(D, rho, u, T, Cv * T, g);
}

/* ------------------------------------------------------------------------ */
/* Caloric law, Eq. (6): U(T) = integral of C_v from 0 to T                  */
/* ------------------------------------------------------------------------ */

void orc_caloric(const orc_params* p, double cv[3]) {
  if (p->cv[0] == 0.0 && p->cv[1] == 0.0 && p->cv[2] == 0.0) {
    cv[0] = 1.0 / (p->gamma - 1.0);
    cv[1] = cv[2] = 0.0;
  } else {
    for (int k = 0; k < 3; ++k) cv[k] = p->cv[k];
  }
}

double orc_internal_energy(const double* cv, double T) {
  return cv[0] * T + cv[1] * T * T / 2.0 + cv[2] * T * T * T / 3.0;
}

static double specific_heat(const double* cv, double T) { return cv[0] + cv[1] * T + cv[2] * T * T; }

/* Newton's method on U(T) = e, started from the constant-C_v guess e / cv[0];
   U is increasing (C_v > 0), and convex for cv[1], cv[2] >= 0, so the
   iterates approach the root monotonically after the first step. */
double orc_temperature(const double* cv, double e) {
  double T = e / cv[0];
  if (cv[1] == 0.0 && cv[2] == 0.0) return T;
  for (int it = 0; it < 100; ++it) {
    double dT = (orc_internal_energy(cv, T) - e) / specific_heat(cv, T);
    T -= dT;
    if (fabs(dT) <= 1e-16 * fabs(T)) break;
  }
  return T;
}

/* q* - q^eq = u . (P - P^eq + (delta_t/2) div Qt), Eq. (46).  Only the
   diagonal of div Qt is non-zero (Eq. (27)); its entries are the discrete
   derivatives d_a.  P^eq = rho T I + rho u u, Eqs. (23), (25). */
void orc_dq(int D, double rho, const double* u, double T, const double* P, const double* d, double* dq) {
  for (int a = 0; a < D; ++a) {
    double s = 0.0;
    for (int b = 0; b < D; ++b) {
      double Peq = rho * ((a == b ? T : 0.0) + u[b] * u[a]);
      double divQ = (a == b) ? 0.5 * d[a] : 0.0;
      s += u[b] * (P[b * D + a] - Peq + divQ);
    }
    dq[a] = s;
  }
}

/* g*_i = g^eq_i + c_i.(q* - q^eq)/2 where c_i^2 = 1, else g^eq_i, Eq. (44). */
static void quasi_equilibrium(int D, const double* geq, const double* dq, double* g) {
  int Q = orc_Q(D);
  for (int i = 0; i < Q; ++i) {
    int c[3];
    orc_velocity(D, i, c);
    int c2 = 0;
    double cdq = 0.0;
    for (int a = 0; a < D; ++a) {
      c2 += c[a] * c[a];
      cdq += c[a] * dq[a];
    }
    g[i] = (c2 == 1) ? geq[i] + 0.5 * cdq : geq[i];
  }
}

void orc_gstar(int D, double rho, const double* u, double T, double Cv, const double* P,
               const double* d, double* g) {
  double geq[QMAX], dq[3];
  orc_geq(D, rho, u, T, Cv, geq);
  orc_dq(D, rho, u, T, P, d, dq);
  quasi_equilibrium(D, geq, dq, g);
}

/* ------------------------------------------------------------------------ */
/* Transport, Sec. II.F                                                     */
/* ------------------------------------------------------------------------ */

/* mu = (1/omega - 1/2) P delta_t with P = rho R T, Eq. (92), solved for omega. */
double orc_omega(double mu, double rho, double T) { return 1.0 / (mu / (rho * T) + 0.5); }

/* Pr = omega_1 (2 - omega) / (omega (2 - omega_1)), Eq. (96), solved for omega_1. */
double orc_omega1(double omega, double Pr) { return 2.0 * Pr * omega / (2.0 - omega + Pr * omega); }

static double viscosity(const orc_params* p, double T) {
  if (p->visc_exp == 0.0) return p->mu0;
  return p->mu0 * pow(T / p->T_ref, p->visc_exp); /* Sec. III.D power law */
}

/* ------------------------------------------------------------------------ */
/* One node                                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
  double rho, u[3], T, P[9], omega, omega1;
} node_state;

/* rho = sum f, rho u = sum c f (Eqs. (3)-(4)), P = sum c c f (Eq. (47)),
   rho E = sum g (Eq. (5)), T from E = U(T) + u^2/2 (Eqs. (6)-(7)). */
static void node_moments(int D, const double* f, const double* g, const double* cv, node_state* m) {
  int Q = orc_Q(D);
  double rho = 0.0, j[3] = {0, 0, 0}, P[9] = {0}, rhoE = 0.0;
  for (int i = 0; i < Q; ++i) {
    int c[3];
    orc_velocity(D, i, c);
    rho += f[i];
    rhoE += g[i];
    for (int a = 0; a < D; ++a) {
      j[a] += c[a] * f[i];
      for (int b = 0; b < D; ++b) P[a * D + b] += c[a] * c[b] * f[i];
    }
  }
  m->rho = rho;
  double u2 = 0.0;
  for (int a = 0; a < 3; ++a) m->u[a] = 0.0;
  for (int a = 0; a < D; ++a) {
    m->u[a] = j[a] / rho;
    u2 += m->u[a] * m->u[a];
  }
  for (int k = 0; k < 9; ++k) m->P[k] = P[k];
  double E = rhoE / rho;
  m->T = orc_temperature(cv, E - 0.5 * u2);
}

static void node_relax_rates(const orc_params* p, node_state* m) {
  m->omega = orc_omega(viscosity(p, m->T), m->rho, m->T);
  m->omega1 = orc_omega1(m->omega, p->Pr);
}

/* f_i <- fh_i + omega (f^ex_i - fh_i), Eq. (1);
   g_i <- gh_i + omega_1 (g^eq_i - gh_i) + (omega - omega_1)(g^eq_i - g*_i), Eq. (2). */
static void node_collide(int D, const double* cv, const node_state* m, const double* fh, const double* gh,
                         const double* d, double* f_out, double* g_out) {
  int Q = orc_Q(D);
  double fex[QMAX], geq[QMAX], gst[QMAX], dq[3];
  orc_fex(D, m->rho, m->u, m->T, m->omega, d, fex);
  orc_geq_u(D, m->rho, m->u, m->T, orc_internal_energy(cv, m->T), geq);
  orc_dq(D, m->rho, m->u, m->T, m->P, d, dq);
  quasi_equilibrium(D, geq, dq, gst);
  for (int i = 0; i < Q; ++i) {
    f_out[i] = fh[i] + m->omega * (fex[i] - fh[i]);
    g_out[i] = gh[i] + m->omega1 * (geq[i] - gh[i]) + (m->omega - m->omega1) * (geq[i] - gst[i]);
  }
}

void orc_collide_node(const orc_params* p, const double* fh, const double* gh, const double* d,
                      double* f_out, double* g_out) {
  double cv[3];
  orc_caloric(p, cv);
  node_state m;
  node_moments(p->D, fh, gh, cv, &m);
  node_relax_rates(p, &m);
  node_collide(p->D, cv, &m, fh, gh, d, f_out, g_out);
}

/* ------------------------------------------------------------------------ */
/* Grid indexing                                                            */
/* ------------------------------------------------------------------------ */

/* Coordinate k + s along an axis of length n: wrapped when periodic, clamped
   to [0, n-1] when zero-gradient. */
static long shift_coord(long k, long s, long n, int bc) {
  long r = k + s;
  if (bc == ORC_PERIODIC) {
    r %= n;
    if (r < 0) r += n;
  } else {
    if (r < 0) r = 0;
    if (r > n - 1) r = n - 1;
  }
  return r;
}

static long node_shift(const orc_params* p, long node, const long* s /* 3 */) {
  long x = node % p->n[0];
  long y = (node / p->n[0]) % p->n[1];
  long z = node / (p->n[0] * p->n[1]);
  x = shift_coord(x, s[0], p->n[0], p->bc[0]);
  y = shift_coord(y, s[1], p->n[1], p->bc[1]);
  z = shift_coord(z, s[2], p->n[2], p->bc[2]);
  return x + p->n[0] * (y + p->n[1] * z);
}

static long neighbour(const orc_params* p, long node, int axis, long s) {
  long sh[3] = {0, 0, 0};
  sh[axis] = s;
  return node_shift(p, node, sh);
}

/* ------------------------------------------------------------------------ */
/* Whole field                                                              */
/* ------------------------------------------------------------------------ */

orc_sim* orc_create(const orc_params* p) {
  if (!p || (p->D != 2 && p->D != 3)) return NULL;
  if (p->n[0] < 1 || p->n[1] < 1 || p->n[2] < 1) return NULL;
  if (p->D == 2 && p->n[2] != 1) return NULL;
  if (!(p->gamma > 1.0) || !(p->Pr > 0.0) || !(p->mu0 > 0.0)) return NULL;
  if (p->visc_exp != 0.0 && !(p->T_ref > 0.0)) return NULL;
  for (int a = 0; a < 3; ++a)
    if (p->bc[a] != ORC_PERIODIC && p->bc[a] != ORC_ZERO_GRADIENT) return NULL;
  if (p->deriv != ORC_UPWIND && p->deriv != ORC_CENTRAL) return NULL;
  /* a caloric law, when given, needs C_v > 0 and U convex: c0 > 0, c1, c2 >= 0 */
  if ((p->cv[0] != 0.0 || p->cv[1] != 0.0 || p->cv[2] != 0.0) &&
      !(p->cv[0] > 0.0 && p->cv[1] >= 0.0 && p->cv[2] >= 0.0))
    return NULL;
  orc_sim* s = (orc_sim*)calloc(1, sizeof *s);
  if (!s) return NULL;
  s->p = *p;
  s->N = p->n[0] * p->n[1] * p->n[2];
  s->Q = orc_Q(p->D);
  orc_caloric(p, s->cv);
  size_t NQ = (size_t)s->N * (size_t)s->Q;
  size_t ND = (size_t)s->N * (size_t)p->D;
  s->f = (double*)malloc(NQ * sizeof(double));
  s->g = (double*)malloc(NQ * sizeof(double));
  s->fh = (double*)malloc(NQ * sizeof(double));
  s->gh = (double*)malloc(NQ * sizeof(double));
  s->rho = (double*)malloc((size_t)s->N * sizeof(double));
  s->u = (double*)malloc(ND * sizeof(double));
  s->T = (double*)malloc((size_t)s->N * sizeof(double));
  s->Qt = (double*)malloc(ND * sizeof(double));
  s->dd = (double*)malloc(ND * sizeof(double));
  s->d = NULL;
  if (!s->f || !s->g || !s->fh || !s->gh || !s->rho || !s->u || !s->T || !s->Qt || !s->dd) {
    orc_destroy(s);
    return NULL;
  }
  return s;
}

void orc_destroy(orc_sim* s) {
  if (!s) return;
  free(s->f);
  free(s->g);
  free(s->fh);
  free(s->gh);
  free(s->rho);
  free(s->u);
  free(s->T);
  free(s->Qt);
  free(s->dd);
  free(s);
}

long orc_step_count(const orc_sim* s) { return s->step; }

int orc_init(orc_sim* s, const double* rho, const double* u, const double* T) {
  int D = s->p.D;
  long N = s->N;
  for (long n = 0; n < N; ++n) {
    if (!isfinite(rho[n]) || !isfinite(T[n]) || !(rho[n] > 0.0) || !(T[n] > 0.0)) return -1;
    for (int a = 0; a < D; ++a)
      if (!isfinite(u[a * N + n])) return -1;
  }
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; ++n) {
    double un[3] = {0, 0, 0}, fe[QMAX], ge[QMAX];
    for (int a = 0; a < D; ++a) un[a] = u[a * N + n];
    orc_feq(D, rho[n], un, T[n], fe);
    orc_geq_u(D, rho[n], un, T[n], orc_internal_energy(s->cv, T[n]), ge);
    for (int i = 0; i < s->Q; ++i) {
      s->f[(size_t)i * N + n] = fe[i];
      s->g[(size_t)i * N + n] = ge[i];
    }
  }
  round_storage(s);
  s->step = 0;
  return 0;
}

/* Discrete derivative of a node field along an axis (Sec. III.A):
   d = Qt_{x+1/2} - Qt_{x-1/2} with the interface values reconstructed on the
   upwind side, Qt_{x+1/2} = Qt_x if u > 0 else Qt_{x+1}; the same sign of u
   (at the node x) picks Qt_{x-1/2} = Qt_{x-1} if u > 0 else Qt_x.
   Central variant (Sec. III.D.2): (Qt_{x+1} - Qt_{x-1}) / 2. */
void orc_derivative(const orc_sim* s, int axis, const double* Qt, const double* u, double* out) {
  const orc_params* p = &s->p;
#pragma omp parallel for schedule(static)
  for (long n = 0; n < s->N; ++n) {
    long np = neighbour(p, n, axis, +1), nm = neighbour(p, n, axis, -1);
    if (p->deriv == ORC_CENTRAL) {
      out[n] = 0.5 * (Qt[np] - Qt[nm]);
    } else {
      double q_plus, q_minus;
      int backward = u[n] > 0.0;
      if (s->band > 0.0 && fabs(u[n]) <= s->band) backward = !backward;
      if (backward) {
        q_plus = Qt[n];
        q_minus = Qt[nm];
      } else {
        q_plus = Qt[np];
        q_minus = Qt[n];
      }
      out[n] = q_plus - q_minus;
    }
  }
}

/* Pass 1 at one node: streaming by pull (Eqs. (1)-(2) read at x: the
   population arriving at x along c_i left x - c_i), then the moments. */
static void pass1_node(orc_sim* s, long n) {
  const orc_params* p = &s->p;
  int D = p->D, Q = s->Q;
  long N = s->N;
  double fl[QMAX], gl[QMAX];
  for (int i = 0; i < Q; ++i) {
    int c[3];
    orc_velocity(D, i, c);
    long sh[3] = {-c[0], -c[1], -c[2]};
    long src = node_shift(p, n, sh);
    fl[i] = s->f[(size_t)i * N + src];
    gl[i] = s->g[(size_t)i * N + src];
    s->fh[(size_t)i * N + n] = fl[i];
    s->gh[(size_t)i * N + n] = gl[i];
  }
  node_state m;
  node_moments(D, fl, gl, s->cv, &m);
  s->rho[n] = m.rho;
  s->T[n] = m.T;
  for (int a = 0; a < D; ++a) {
    s->u[(size_t)a * N + n] = m.u[a];
    s->Qt[(size_t)a * N + n] = orc_anomaly(m.rho, m.u[a], m.T);
  }
}

/* Pass 2 at one node: relaxation with the derivatives already in s->dd, or
   with d_in[0..D-1] when d_in is not NULL. */
static void pass2_node(const orc_sim* s, long n, const double* d_in, double* f_out, long f_stride, double* g_out,
                       long g_stride) {
  const orc_params* p = &s->p;
  int D = p->D, Q = s->Q;
  long N = s->N;
  double fl[QMAX] = {0}, gl[QMAX] = {0}, fo[QMAX], go[QMAX], d[3] = {0, 0, 0};
  for (int i = 0; i < Q; ++i) {
    fl[i] = s->fh[(size_t)i * N + n];
    gl[i] = s->gh[(size_t)i * N + n];
  }
  node_state m;
  node_moments(D, fl, gl, s->cv, &m);
  node_relax_rates(p, &m);
  for (int a = 0; a < D; ++a) d[a] = d_in ? d_in[a] : s->dd[(size_t)a * N + n];
  node_collide(D, s->cv, &m, fl, gl, d, fo, go);
  for (int i = 0; i < Q; ++i) {
    f_out[(size_t)i * f_stride] = fo[i];
    g_out[(size_t)i * g_stride] = go[i];
  }
}

static void pass1(orc_sim* s) {
#pragma omp parallel for schedule(static)
  for (long n = 0; n < s->N; ++n) pass1_node(s, n);
  for (int a = 0; a < s->p.D; ++a)
    orc_derivative(s, a, s->Qt + (size_t)a * s->N, s->u + (size_t)a * s->N, s->dd + (size_t)a * s->N);
}

/* The FP32 storage model: every stored population becomes its reference
   value plus its deviation from it rounded to single precision. */
static void round_storage(orc_sim* s) {
  if (!s->fp32_store) return;
  long N = s->N;
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; ++n)
    for (int i = 0; i < s->Q; ++i) {
      double* f = s->f + (size_t)i * N + n;
      double* g = s->g + (size_t)i * N + n;
      *f = s->fref[i] + (double)(float)(*f - s->fref[i]);
      *g = s->gref[i] + (double)(float)(*g - s->gref[i]);
    }
}

int orc_set_upwind_band(orc_sim* s, double band) {
  if (!(band >= 0.0) || !isfinite(band)) return -1;
  s->band = band;
  return 0;
}

int orc_set_fp32_storage(orc_sim* s, const double* f_ref, const double* g_ref) {
  if (!f_ref || !g_ref) {
    s->fp32_store = 0;
    return 0;
  }
  for (int i = 0; i < s->Q; ++i) {
    if (!isfinite(f_ref[i]) || !isfinite(g_ref[i])) return -1;
    s->fref[i] = f_ref[i];
    s->gref[i] = g_ref[i];
  }
  s->fp32_store = 1;
  return 0;
}

int orc_step(orc_sim* s, long nsteps) {
  if (nsteps < 0) return -1;
  long N = s->N;
  for (long k = 0; k < nsteps; ++k) {
    pass1(s);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) pass2_node(s, n, NULL, s->f + n, N, s->g + n, N);
    round_storage(s);
    s->step += 1;
  }
  return 0;
}

/* Upwind difference of Qt along an axis at node n on a given side:
   0 = the backward difference Qt(x) - Qt(x - e), the side Sec. III.A takes
   when u > 0; 1 = the forward difference Qt(x + e) - Qt(x). */
static double upwind_side(const orc_sim* s, const double* Qt, long n, int axis, int side) {
  long np = neighbour(&s->p, n, axis, +1), nm = neighbour(&s->p, n, axis, -1);
  return side == 0 ? Qt[n] - Qt[nm] : Qt[np] - Qt[n];
}

int orc_step_sampled_branch(const orc_sim* s_in, const long* nodes, long count, const signed char* branch,
                            double* f_out, double* g_out) {
  /* Run pass 1 on a private copy of the per-node scratch, then pass 2 at the
     requested nodes only.  The stored populations are not modified. */
  int D = s_in->p.D;
  for (long k = 0; k < count; ++k) {
    if (nodes[k] < 0 || nodes[k] >= s_in->N) return -1;
    if (branch)
      for (int a = 0; a < D; ++a)
        if (branch[k * D + a] < -1 || branch[k * D + a] > 1) return -1;
  }
  orc_sim tmp = *s_in;
  size_t NQ = (size_t)s_in->N * s_in->Q, ND = (size_t)s_in->N * D;
  tmp.fh = (double*)malloc(NQ * sizeof(double));
  tmp.gh = (double*)malloc(NQ * sizeof(double));
  tmp.rho = (double*)malloc((size_t)s_in->N * sizeof(double));
  tmp.u = (double*)malloc(ND * sizeof(double));
  tmp.T = (double*)malloc((size_t)s_in->N * sizeof(double));
  tmp.Qt = (double*)malloc(ND * sizeof(double));
  tmp.dd = (double*)malloc(ND * sizeof(double));
  int ok = tmp.fh && tmp.gh && tmp.rho && tmp.u && tmp.T && tmp.Qt && tmp.dd;
  if (ok) {
    pass1(&tmp);
    for (long k = 0; k < count; ++k) {
      const long node = nodes[k];
      double d[3] = {0, 0, 0};
      for (int a = 0; a < D; ++a) {
        d[a] = tmp.dd[(size_t)a * tmp.N + node];
        if (branch && branch[k * D + a] >= 0 && tmp.p.deriv == ORC_UPWIND)
          d[a] = upwind_side(&tmp, tmp.Qt + (size_t)a * tmp.N, node, a, branch[k * D + a]);
      }
      pass2_node(&tmp, node, d, f_out + k, count, g_out + k, count);
    }
  }
  free(tmp.fh);
  free(tmp.gh);
  free(tmp.rho);
  free(tmp.u);
  free(tmp.T);
  free(tmp.Qt);
  free(tmp.dd);
  return ok ? 0 : -1;
}

int orc_step_sampled(const orc_sim* s, const long* nodes, long count, double* f_out, double* g_out) {
  return orc_step_sampled_branch(s, nodes, count, NULL, f_out, g_out);
}

int orc_moments(const orc_sim* s, double* rho, double* u, double* T) {
  int D = s->p.D, Q = s->Q;
  long N = s->N;
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; ++n) {
    double fl[QMAX], gl[QMAX];
    for (int i = 0; i < Q; ++i) {
      fl[i] = s->f[(size_t)i * N + n];
      gl[i] = s->g[(size_t)i * N + n];
    }
    node_state m;
    node_moments(D, fl, gl, s->cv, &m);
    if (rho) rho[n] = m.rho;
    if (T) T[n] = m.T;
    if (u)
      for (int a = 0; a < D; ++a) u[(size_t)a * N + n] = m.u[a];
  }
  return 0;
}

/* Pairwise (recursive halving) sum in a fixed order. */
static double pairwise_sum(const double* x, long n) {
  if (n <= 8) {
    double s = 0.0;
    for (long k = 0; k < n; ++k) s += x[k];
    return s;
  }
  long h = n / 2;
  return pairwise_sum(x, h) + pairwise_sum(x + h, n - h);
}

/* Central difference of a node field along an axis, with the wrap/clamp rule. */
static double central(const orc_sim* s, const double* F, long n, int axis) {
  return 0.5 * (F[neighbour(&s->p, n, axis, +1)] - F[neighbour(&s->p, n, axis, -1)]);
}

int orc_diagnostics(const orc_sim* s, double* out) {
  const orc_params* p = &s->p;
  int D = p->D;
  long N = s->N;
  double* rho = (double*)malloc((size_t)N * sizeof(double));
  double* u = (double*)calloc((size_t)N * 3, sizeof(double));
  double* T = (double*)malloc((size_t)N * sizeof(double));
  double* w = (double*)malloc((size_t)N * ORC_NDIAG * sizeof(double));
  if (!rho || !u || !T || !w) {
    free(rho);
    free(u);
    free(T);
    free(w);
    return -1;
  }
  orc_moments(s, rho, u, T);
#pragma omp parallel for schedule(static)
  for (long n = 0; n < N; ++n) {
    double* c = w + (size_t)n;  /* column n of a [ORC_NDIAG][N] table */
    double ux = u[n], uy = u[N + n], uz = u[2 * N + n];
    double uu = ux * ux + uy * uy + uz * uz;
    double rhoE = 0.0; /* rho E = sum_i g_i, Eq. (5) */
    for (int i = 0; i < s->Q; ++i) rhoE += s->g[(size_t)i * N + n];
    double div = 0.0, du[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) {
      du[a] = central(s, u + (size_t)a * N, n, a);
      div += du[a];
    }
    /* curl u by central differences; components along missing axes vanish */
    double gx = 0, gy = 0, gz = 0;
    if (D == 3) {
      gx = central(s, u + 2 * (size_t)N, n, 1) - central(s, u + (size_t)N, n, 2);
      gy = central(s, u, n, 2) - central(s, u + 2 * (size_t)N, n, 0);
    }
    gz = central(s, u + (size_t)N, n, 0) - central(s, u, n, 1);
    double vort2 = gx * gx + gy * gy + gz * gz;
    int finite = isfinite(rho[n]) && isfinite(T[n]) && isfinite(ux) && isfinite(uy) && isfinite(uz);
    c[(size_t)ORC_D_MASS * N] = rho[n];
    c[(size_t)ORC_D_MOMX * N] = rho[n] * ux;
    c[(size_t)ORC_D_MOMY * N] = rho[n] * uy;
    c[(size_t)ORC_D_MOMZ * N] = rho[n] * uz;
    c[(size_t)ORC_D_ENERGY * N] = rhoE;
    c[(size_t)ORC_D_KINETIC * N] = 0.5 * rho[n] * uu;
    c[(size_t)ORC_D_DIL2 * N] = div * div;
    c[(size_t)ORC_D_U2 * N] = uu;
    /* sound speed sqrt(gamma(T) T), gamma = C_p / C_v = (C_v + 1) / C_v, Eq. (97) */
    double gam = p->gamma;
    if (s->cv[1] != 0.0 || s->cv[2] != 0.0) {
      double cvT = specific_heat(s->cv, T[n]);
      gam = (cvT + 1.0) / cvT;
    }
    c[(size_t)ORC_D_CS * N] = sqrt(gam * T[n]);
    c[(size_t)ORC_D_RHO2 * N] = rho[n] * rho[n];
    c[(size_t)ORC_D_VORT2 * N] = vort2;
    c[(size_t)ORC_D_DISS * N] = viscosity(p, T[n]) * vort2;
    c[(size_t)ORC_D_UX2 * N] = ux * ux;
    c[(size_t)ORC_D_UY2 * N] = uy * uy;
    c[(size_t)ORC_D_UZ2 * N] = uz * uz;
    c[(size_t)ORC_D_DUX2 * N] = du[0] * du[0];
    c[(size_t)ORC_D_DUY2 * N] = du[1] * du[1];
    c[(size_t)ORC_D_DUZ2 * N] = du[2] * du[2];
    c[(size_t)ORC_D_NONFINITE * N] = finite ? 0.0 : 1.0;
    c[(size_t)ORC_D_NONPOSITIVE * N] = (rho[n] <= 0.0 || T[n] <= 0.0) ? 1.0 : 0.0;
    c[(size_t)ORC_D_NODES * N] = 1.0;
  }
  for (int k = 0; k < ORC_NDIAG; ++k) out[k] = pairwise_sum(w + (size_t)k * N, N);
  free(rho);
  free(u);
  free(T);
  free(w);
  return 0;
}

int orc_get_pops(const orc_sim* s, double* f, double* g) {
  size_t NQ = (size_t)s->N * s->Q;
  if (f) memcpy(f, s->f, NQ * sizeof(double));
  if (g) memcpy(g, s->g, NQ * sizeof(double));
  return 0;
}

int orc_set_pops(orc_sim* s, const double* f, const double* g, long step) {
  size_t NQ = (size_t)s->N * s->Q;
  memcpy(s->f, f, NQ * sizeof(double));
  memcpy(s->g, g, NQ * sizeof(double));
  s->step = step;
  return 0;
}
