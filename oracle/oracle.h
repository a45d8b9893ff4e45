/*
 * CPU oracle of the two-population compressible lattice Boltzmann model of
 * Saadat, Hosseini, Dorschner and Karlin, "Extended lattice Boltzmann model
 * for gas dynamics" (arXiv:2102.09512).
 *
 * TEST INFRASTRUCTURE.  This is the plain, slow, FP64 reference against which
 * the GPU library is checked.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no source, header
 * or generated table with the GPU library, and the GPU library never calls it.
 *
 * Lattice units throughout: delta_t = delta_x = 1 and R = 1 (Sec. III.A).
 * Caloric law (Sec. II.A, Eq. (6)): C_v(T) = cv[0] + cv[1] T + cv[2] T^2, so
 * U(T) = cv[0] T + cv[1] T^2/2 + cv[2] T^3/3 and C_p = C_v + 1 (Mayer);
 * cv all zero selects the constant C_v = 1/(gamma-1) of the paper's runs.
 *
 * Velocity numbering (the paper fixes none): c_i = (i%3-1, (i/3)%3-1, (i/9)%3-1)
 * with Q = 3^D; for D = 2 the z component is dropped (Q = 9).
 * Population storage of this oracle: f[i*N + node], node = x + nx*(y + ny*z).
 *
 * Field arrays (rho, u, T) are node-major FP64: rho[node], u[a*N + node], T[node].
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_PERIODIC = 0, ORC_ZERO_GRADIENT = 1 };
enum { ORC_UPWIND = 0, ORC_CENTRAL = 1 };

typedef struct {
  int D;            /* 2 or 3 */
  long n[3];        /* nx, ny, nz; nz == 1 when D == 2 */
  int bc[3];        /* per axis, both ends: ORC_PERIODIC or ORC_ZERO_GRADIENT */
  double gamma;     /* adiabatic exponent, Eq. (97) */
  double Pr;        /* Prandtl number, Eq. (96) */
  double mu0;       /* dynamic viscosity at T_ref */
  double visc_exp;  /* mu = mu0 (T/T_ref)^visc_exp  (Sec. III.D); 0 = constant mu */
  double T_ref;     /* reference temperature of the power law */
  int deriv;        /* ORC_UPWIND (Sec. III.A) or ORC_CENTRAL (Sec. III.D.2) */
  double cv[3];     /* C_v(T) coefficients (see above); all zero = 1/(gamma-1) */
} orc_params;

/* Diagnostic slots written by orc_diagnostics (all FP64 sums over nodes). */
enum {
  ORC_D_MASS = 0,     /* sum rho */
  ORC_D_MOMX, ORC_D_MOMY, ORC_D_MOMZ, /* sum rho u_a */
  ORC_D_ENERGY,       /* sum rho E */
  ORC_D_KINETIC,      /* sum rho |u|^2 / 2 */
  ORC_D_DIL2,         /* sum (div u)^2, central differences */
  ORC_D_U2,           /* sum |u|^2 */
  ORC_D_CS,           /* sum sqrt(gamma T) */
  ORC_D_RHO2,         /* sum rho^2 */
  ORC_D_VORT2,        /* sum |curl u|^2, central differences */
  ORC_D_DISS,         /* sum mu(T) |curl u|^2 */
  ORC_D_UX2, ORC_D_UY2, ORC_D_UZ2,    /* sum u_a^2 */
  ORC_D_DUX2, ORC_D_DUY2, ORC_D_DUZ2, /* sum (d_a u_a)^2 */
  ORC_D_NONFINITE,    /* nodes with a non-finite rho, u or T */
  ORC_D_NONPOSITIVE,  /* nodes with rho <= 0 or T <= 0 */
  ORC_D_NODES,        /* node count */
  ORC_NDIAG
};

/* Caloric law: the coefficients in effect for p (cv, or 1/(gamma-1) when cv
   is all zero); U(T) (Eq. (6)); T from U by Newton's method on U(T) = e. */
void orc_caloric(const orc_params* p, double cv[3]);
double orc_internal_energy(const double* cv, double T);
double orc_temperature(const double* cv, double e);

typedef struct orc_sim orc_sim;

/* Whole-field simulation (returns NULL on invalid parameters). */
orc_sim* orc_create(const orc_params* p);
void orc_destroy(orc_sim* s);
/* f = f^eq(rho,u,T), g = g^eq(rho,u,T), step = 0.  Returns 0, or -1 when a
   value is non-finite or rho <= 0 or T <= 0. */
int orc_init(orc_sim* s, const double* rho, const double* u, const double* T);
int orc_step(orc_sim* s, long nsteps);
/* Same as one orc_step but only for the listed nodes: writes their
   post-collision populations to f_out[i*count + k], g_out[i*count + k] and
   leaves the state unchanged. */
int orc_step_sampled(const orc_sim* s, const long* nodes, long count, double* f_out, double* g_out);
/* orc_step_sampled with the upwind side of the anomaly difference (Sec. III.A)
   at sampled node k forced on the axes where branch[k*D + a] is 0 (backward
   difference Qt(x) - Qt(x - e_a), the side taken when u_a > 0) or 1 (forward
   difference Qt(x + e_a) - Qt(x)); -1 leaves the choice to the sign of u_a.
   branch may be NULL.  Ignored for the central variant.  Returns -1 on a node
   index outside the field or a branch value outside -1..1. */
int orc_step_sampled_branch(const orc_sim* s, const long* nodes, long count, const signed char* branch,
                            double* f_out, double* g_out);
/* FP32 storage model: from now on, after orc_init and after every step, each
   population becomes ref_i + (double)(float)(value - ref_i), the value that a
   single-precision store of its deviation from the reference populations
   f_ref[Q], g_ref[Q] keeps (the arithmetic stays FP64).  This measures what
   FP32 deviation storage alone costs a flow.  NULL pointers switch it off.
   Returns -1 on a non-finite reference value. */
int orc_set_fp32_storage(orc_sim* s, const double* f_ref, const double* g_ref);
/* Upwind-side ambiguity model: from now on every upwind decision of
   Sec. III.A whose |u_a| <= band takes the other side than the sign test
   (where a perturbation of u of that size could change the side, both are
   valid readings).  band = 0 (default) is the plain scheme, u_a = 0
   included.  Returns -1 on a
   negative or non-finite band. */
int orc_set_upwind_band(orc_sim* s, double band);
long orc_step_count(const orc_sim* s);
/* Moments of the stored populations (no streaming). */
int orc_moments(const orc_sim* s, double* rho, double* u, double* T);
int orc_diagnostics(const orc_sim* s, double* out /* ORC_NDIAG */);
int orc_get_pops(const orc_sim* s, double* f, double* g);
int orc_set_pops(orc_sim* s, const double* f, const double* g, long step);
int orc_num_threads(void);
void orc_set_num_threads(int n);

/* ---- nodal building blocks (the functions the step itself uses) ---- */
int orc_Q(int D);
void orc_velocity(int D, int i, int* c /* 3 */);
/* rho * prod_a Psi_{c_ia}(xi_a, P_a): the product form, Eqs. (9)-(12). */
void orc_product_form(int D, double rho, const double* xi, const double* P, double* out);
/* f^eq, Eq. (20). */
void orc_feq(int D, double rho, const double* u, double T, double* f);
/* f^ex with a given discrete derivative d_a of the anomaly, Eqs. (28), (30). */
void orc_fex(int D, double rho, const double* u, double T, double omega, const double* d, double* f);
/* g^eq by operator product form, Eq. (42), with E of Eq. (7) at constant C_v. */
void orc_geq(int D, double rho, const double* u, double T, double Cv, double* g);
/* The same with the internal energy U = U(T) of any caloric law given. */
void orc_geq_u(int D, double rho, const double* u, double T, double U, double* g);
/* q* - q^eq, Eq. (46); P is the D x D pressure tensor of the populations (row-major). */
void orc_dq(int D, double rho, const double* u, double T, const double* P, const double* d, double* dq);
/* g*, Eq. (44). */
void orc_gstar(int D, double rho, const double* u, double T, double Cv, const double* P,
               const double* d, double* g);
double orc_anomaly(double rho, double u, double T);           /* Eq. (29) */
double orc_omega(double mu, double rho, double T);              /* Eq. (92) */
double orc_omega1(double omega, double Pr);                     /* Eq. (96) */
/* One node: moments of (fh, gh), relaxation of both populations, Eqs. (1), (2). */
void orc_collide_node(const orc_params* p, const double* fh, const double* gh, const double* d,
                      double* f_out, double* g_out);
/* Discrete derivative along axis of a field Qt[node] whose upwind side is
   chosen by u[node] (Sec. III.A); out[node]. */
void orc_derivative(const orc_sim* s, int axis, const double* Qt, const double* u, double* out);

#ifdef __cplusplus
}
#endif
#endif
