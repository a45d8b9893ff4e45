// Per-node arithmetic of the two-population compressible LBM on the GPU.
//
// The equilibria are evaluated in tensor-product form: every population
// is a sum of products of one-dimensional factors, one per axis, so the
// per-axis factors are formed once per node and combined over (c_y, c_z)
// pairs before the loop over c_x.
//
//   f^ex_i = rho prod_a Psi_{c_ia}(u_a, P_a)                    Eqs. (12), (28)-(30)
//     Psi_0 = 1 - P, Psi_{+-1} = (+-u + P)/2                    Eqs. (9)-(11)
//     P_a  = T + u_a^2 + (2 - omega)/(2 rho omega) d_a          Eq. (28)
//   g^eq_i = rho [C_v T prod_a a_a + sum_a b_a prod_{b!=a} a_b]  Eq. (42)
//     with a_a = Psi_{c}(O_a, O_a^2) 1 and b_a = Psi_c(O_a, O_a^2) u_a^2 / 2,
//     O_a = T d/du_a + u_a (Eq. (33)) applied to the separable terms of
//     E = C_v T + |u|^2/2 (Eqs. (6)-(7)):
//       a(0) = 1 - T - u^2,        a(+-1) = (+-u + T + u^2)/2
//       b(0) = u^2/2 - B2,         b(+-1) = (+-B1 + B2)/2
//       B1 = u (u^2 + 2T)/2,       B2 = (u^4 + 5 u^2 T + 2 T^2)/2
//   g*_i - g^eq_i = c_i.dq / 2 on the directions with c_i^2 = 1    Eq. (44)
//     dq = u.(P - P^eq) + u_a d_a / 2 (diagonal)                 Eq. (46)
//
// Deviation storage (DEV): populations are stored minus the rest state
// w = (f, g)^eq(rho0, 0, T0).  Every equilibrium is then formed as
// (value - rest) directly, by telescoping the products
//   prod_a X_a - prod_a X0_a = dX_x X_y X_z + X0_x dX_y X_z + X0_x X0_y dX_z,
// with per-axis differences dX that are computed without cancellation from
// (rho - rho0), (T - T0) and u.  All rounding is then relative to the
// deviation, not to the full population.  With rho0 = T0 = 0 (FP64 storage)
// the same code reduces to the plain equilibria.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm.h"

namespace lbm {

__host__ __device__ constexpr int lat_q(int D) { return D == 2 ? 9 : 27; }
__host__ __device__ constexpr int vx(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int vy(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int vz(int i) { return (i / 9) % 3 - 1; }

// Moments of one node after streaming, in compute precision R.
template <typename R>
struct NodeMoments {
  R rho;     // density
  R drho;    // rho - rho0
  R T;       // temperature
  R dT;      // T - T0
  R u[3];
  R du[3];   // u - u0
  R pn[6];   // P - P^eq: xx, yy, zz, xy, xz, yz
  R irho;    // 1 / rho
  R omega, omega1;
  R corr;    // (2 - omega) / (2 rho omega), the factor of d_a in P^ex (Eq. (30))
};

// Constants of a step.  The reference state (rho0, u0, T0) of the FP32
// deviation storage is zero for FP64 storage.  Per axis a, with
// P0_a = T0 + u0_a^2, the reference factors of the product form are
// psi0_a(c) = Psi_c(u0_a, P0_a) (also the a-factors of g^eq) and b0_a(c), the
// b-factors of g^eq at (u0_a, T0); index c + 1.
struct NodeConsts {
  double rho0, T0;
  double inv_Cv, Cv, Pr;
  double cv1, cv2, U0;  // caloric law (see caloric_*)
  int caloric;
  double mu0, visc_exp, inv_Tref;
  double u0[3], P0[3], psi0[3][3], b0[3][3];
  float u0f[3], P0f[3], psi0f[3][3], b0f[3][3];
};

// The reference constants in compute precision.
__device__ inline double ref(double d, float) { return d; }
__device__ inline float ref(float, float f) { return f; }
template <typename R>
__device__ inline R ref_u0(const NodeConsts& k, int a) { return ref(R(k.u0[a]), k.u0f[a]); }
template <typename R>
__device__ inline R ref_P0(const NodeConsts& k, int a) { return ref(R(k.P0[a]), k.P0f[a]); }
template <typename R>
__device__ inline R ref_psi0(const NodeConsts& k, int a, int c) { return ref(R(k.psi0[a][c]), k.psi0f[a][c]); }
template <typename R>
__device__ inline R ref_b0(const NodeConsts& k, int a, int c) { return ref(R(k.b0[a][c]), k.b0f[a][c]); }

// Caloric law (Eq. (6)), with caloric_cv and caloric_u: U(T0 + dT) - U(T0)
// is formed from dT directly, so a small step loses nothing to cancellation.
template <typename R>
__device__ inline R caloric_du(R c0, R c1, R c2, R T0, R dT) {
  return dT * (c0 + c1 * (T0 + (R)0.5 * dT) + c2 * (T0 * T0 + T0 * dT + dT * dT * (R)(1.0 / 3.0)));
}
// dT with U(T0 + dT) - U(T0) = dU: Newton's method from the step of the
// constant C_v(T0), until the correction is below 1e-15 of T (U is increasing
// and convex for c0 > 0, c1, c2 >= 0, so the iterates converge monotonically
// after the first step); at most 40 steps.
__device__ inline double caloric_step(double c0, double c1, double c2, double T0, double dU) {
  double dT = dU / caloric_cv(c0, c1, c2, T0);
  for (int it = 0; it < 40; ++it) {
    const double h = (caloric_du<double>(c0, c1, c2, T0, dT) - dU) / caloric_cv(c0, c1, c2, T0 + dT);
    dT -= h;
    if (fabs(h) <= 1e-15 * fabs(T0 + dT)) break;
  }
  return dT;
}

// Reciprocal: the hardware approximation (about 1 ulp) in FP32, IEEE
// division in FP64.
__device__ inline float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double recip(double x) { return 1.0 / x; }

// mu = mu0 (T / T_ref)^n; FP32 through the hardware log2 / exp2.
__device__ inline double viscosity(const NodeConsts& k, double T) {
  if (k.visc_exp == 0.0) return k.mu0;
  return k.mu0 * pow(T * k.inv_Tref, k.visc_exp);
}
__device__ inline float viscosity(const NodeConsts& k, float T) {
  if (k.visc_exp == 0.0) return (float)k.mu0;
  return (float)k.mu0 * __builtin_amdgcn_exp2f((float)k.visc_exp * __builtin_amdgcn_logf(T * (float)k.inv_Tref));
}

// P - P^eq with P = sum c c f (Eq. (47)) and P^eq = rho T I + rho u u
// (Eqs. (23), (25)).  p holds the sums over the stored values, i.e. P minus
// the reference rho0 (T0 I + u0 u0); so what is subtracted is
// rho T - rho0 T0 = drho T0 + rho dT on the diagonal and
// rho u_a u_b - rho0 u0_a u0_b = drho u_a u_b + rho0 (du_a u_b + u0_a du_b).
template <int D, typename R>
__device__ inline void nonequilibrium_pressure(NodeMoments<R>& m, const R* p, const NodeConsts& k) {
  const R iso = m.drho * (R)k.T0 + m.rho * m.dT;
  const R rho0 = (R)k.rho0;
  auto uu = [&](int a, int b) {
    return m.drho * m.u[a] * m.u[b] + rho0 * (m.du[a] * m.u[b] + ref_u0<R>(k, a) * m.du[b]);
  };
  m.pn[0] = p[0] - uu(0, 0) - iso;
  m.pn[1] = p[1] - uu(1, 1) - iso;
  m.pn[2] = (D == 3) ? p[2] - uu(2, 2) - iso : (R)0;
  m.pn[3] = p[3] - uu(0, 1);
  m.pn[4] = (D == 3) ? p[4] - uu(0, 2) : (R)0;
  m.pn[5] = (D == 3) ? p[5] - uu(1, 2) : (R)0;
}

// u, u - u0 and T - T0 from the sums of the stored values (s0 = sum f,
// j = sum c f, se = sum g), all in deviation form: u - u0 = (j - drho u0) / rho
// and rho (U(T) - U(T0)) = se - (1/2) sum_a [rho0 du_a (u_a + u0_a) + drho u_a^2]
// - drho U(T0), which follow from rho u = rho0 u0 + j and
// rho E = rho0 (U(T0) + |u0|^2 / 2) + se; then T - T0 = that / C_v for a
// constant C_v, or by caloric_step for a general law.
// The sums and this recovery are done in FP64 for every storage precision.
template <int D, typename R>
__device__ inline void velocity_temperature(NodeMoments<R>& m, double s0, const double* j, double se,
                                            const NodeConsts& k) {
  const double rho = k.rho0 + s0, irho = 1.0 / rho;
  double ke = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a < D) {
      const double u0 = k.u0[a];
      const double du = (j[a] - s0 * u0) * irho;
      const double u = u0 + du;
      ke += k.rho0 * du * (u + u0) + s0 * u * u;
      m.du[a] = (R)du;
      m.u[a] = (R)u;
    } else {
      m.du[a] = m.u[a] = (R)0;
    }
  }
  const double dU = (se - 0.5 * ke - s0 * k.U0) * irho;  // U(T) - U(T0)
  const double dT = k.caloric ? caloric_step(k.Cv, k.cv1, k.cv2, k.T0, dU) : dU * k.inv_Cv;
  m.drho = (R)s0;
  m.rho = (R)rho;
  m.irho = (R)irho;
  m.dT = (R)dT;
  m.T = (R)(k.T0 + dT);
}

// FP64 sums of the conserved moments of the stored values: s0 = sum f,
// j = sum c f, se = sum g, row by row as in moment_sums.
template <int D, typename R>
__device__ inline void conserved_sums(const R* f, const R* g, double& s0, double* j, double& se) {
  constexpr int NR = (D == 3) ? 9 : 3;
  double r0[NR], rx[NR], rg[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const double a = (double)f[3 * r], b = (double)f[3 * r + 1], c = (double)f[3 * r + 2];
    rx[r] = c - a;
    r0[r] = (c + a) + b;
    rg[r] = ((double)g[3 * r + 2] + (double)g[3 * r]) + (double)g[3 * r + 1];
  }
  if (D == 3) {
    double l0[3], lx[3], lg[3];
#pragma unroll
    for (int z = 0; z < 3; ++z) {
      l0[z] = (r0[3 * z] + r0[3 * z + 2]) + r0[3 * z + 1];
      lx[z] = (rx[3 * z] + rx[3 * z + 2]) + rx[3 * z + 1];
      lg[z] = (rg[3 * z] + rg[3 * z + 2]) + rg[3 * z + 1];
    }
    s0 = (l0[0] + l0[2]) + l0[1];
    se = (lg[0] + lg[2]) + lg[1];
    j[0] = (lx[0] + lx[2]) + lx[1];
    j[1] = ((r0[2] - r0[0]) + (r0[8] - r0[6])) + (r0[5] - r0[3]);
    j[2] = l0[2] - l0[0];
  } else {
    s0 = (r0[0] + r0[2]) + r0[1];
    se = (rg[0] + rg[2]) + rg[1];
    j[0] = (rx[0] + rx[2]) + rx[1];
    j[1] = r0[2] - r0[0];
    j[2] = 0.0;
  }
}

// omega from mu = (1/omega - 1/2) rho T (Eq. (92)): 1/omega = nu + 1/2 with
// nu = mu / (rho T).  Eq. (96) then reduces to 1/omega_1 = nu / Pr + 1/2, and
// the factor (2 - omega) / (2 rho omega) of Eq. (30) to nu / rho.
template <typename R>
__device__ inline void relaxation_rates(NodeMoments<R>& m, const NodeConsts& k) {
  const R mu = viscosity(k, m.T);
  const R nu = mu * recip(m.rho * m.T);
  m.omega = recip(nu + (R)0.5);
  m.omega1 = recip(nu * (R)(1.0 / k.Pr) + (R)0.5);
  m.corr = nu * m.irho;
}

// Zeroth, first and second moments of one population set (Eqs. (3), (4),
// (47)), summed row by row: for each (c_y, c_z) the three x-neighbours are
// combined first, then the rows.  s[0] = sum f, j[a] = sum c_a f,
// p = (xx, yy, zz, xy, xz, yz) of sum c c f.
template <int D, typename R>
__device__ inline void moment_sums(const R* f, R& s, R* j, R* p) {
  if constexpr (sizeof(R) == 8) {
    // FP64: one pass in population order (fewer live registers)
    constexpr int Q = lat_q(D);
    s = 0;
    j[0] = j[1] = j[2] = 0;
    p[0] = p[1] = p[2] = p[3] = p[4] = p[5] = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int cx = vx(i), cy = vy(i), cz = (D == 3) ? vz(i) : 0;
      const R w = f[i];
      s += w;
      if (cx) j[0] += cx > 0 ? w : -w;
      if (cy) j[1] += cy > 0 ? w : -w;
      if (cz) j[2] += cz > 0 ? w : -w;
      if (cx) p[0] += w;
      if (cy) p[1] += w;
      if (cz) p[2] += w;
      if (cx && cy) p[3] += (cx == cy) ? w : -w;
      if (cx && cz) p[4] += (cx == cz) ? w : -w;
      if (cy && cz) p[5] += (cy == cz) ? w : -w;
    }
    return;
  }
  constexpr int NR = (D == 3) ? 9 : 3;  // rows: index jy + 3 jz, jy = c_y + 1, jz = c_z + 1
  R r0[NR], rx[NR], rxx[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    rxx[r] = f[3 * r + 2] + f[3 * r];
    rx[r] = f[3 * r + 2] - f[3 * r];
    r0[r] = rxx[r] + f[3 * r + 1];
  }
  if (D == 3) {
    R l0[3], lx[3], lxx[3];  // per z layer
#pragma unroll
    for (int z = 0; z < 3; ++z) {
      l0[z] = (r0[3 * z] + r0[3 * z + 2]) + r0[3 * z + 1];
      lx[z] = (rx[3 * z] + rx[3 * z + 2]) + rx[3 * z + 1];
      lxx[z] = (rxx[3 * z] + rxx[3 * z + 2]) + rxx[3 * z + 1];
    }
    s = (l0[0] + l0[2]) + l0[1];
    j[0] = (lx[0] + lx[2]) + lx[1];
    p[0] = (lxx[0] + lxx[2]) + lxx[1];
    j[1] = ((r0[2] - r0[0]) + (r0[8] - r0[6])) + (r0[5] - r0[3]);
    p[1] = ((r0[2] + r0[0]) + (r0[8] + r0[6])) + (r0[5] + r0[3]);
    j[2] = l0[2] - l0[0];
    p[2] = l0[2] + l0[0];
    p[3] = ((rx[2] - rx[0]) + (rx[8] - rx[6])) + (rx[5] - rx[3]);
    p[4] = lx[2] - lx[0];
    p[5] = (r0[8] + r0[0]) - (r0[6] + r0[2]);
  } else {
    s = (r0[0] + r0[2]) + r0[1];
    j[0] = (rx[0] + rx[2]) + rx[1];
    p[0] = (rxx[0] + rxx[2]) + rxx[1];
    j[1] = r0[2] - r0[0];
    p[1] = r0[2] + r0[0];
    p[3] = rx[2] - rx[0];
    j[2] = p[2] = p[4] = p[5] = (R)0;
  }
}

// Plain sum of Q values, three at a time then rows.
template <int D, typename R>
__device__ inline R total(const R* g) {
  constexpr int NR = (D == 3) ? 9 : 3;
  R r[NR];
#pragma unroll
  for (int i = 0; i < NR; ++i) r[i] = (g[3 * i] + g[3 * i + 2]) + g[3 * i + 1];
  if (D == 3) {
    const R l0 = (r[0] + r[2]) + r[1], l1 = (r[3] + r[5]) + r[4], l2 = (r[6] + r[8]) + r[7];
    return (l0 + l2) + l1;
  }
  return (r[0] + r[2]) + r[1];
}

// Moments of the post-streaming populations f, g (Eqs. (3)-(7), (47)): the
// stored values are deviations from the reference state (rho0, u0, T0) for
// FP32 storage and full populations for FP64 storage (reference zero).
// rho, u and T come from FP64 sums in deviation form (velocity_temperature);
// P - P^eq is summed in the compute precision.
template <int D, typename R>
__device__ inline NodeMoments<R> node_moments(const R* f, const R* g, const NodeConsts& k) {
  R s0r, jr[3], p[6];
  moment_sums<D, R>(f, s0r, jr, p);  // only p is used: the conserved sums are FP64
  double s0, j[3], se;
  conserved_sums<D, R>(f, g, s0, j, se);
  NodeMoments<R> m;
  velocity_temperature<D, R>(m, s0, j, se, k);
  nonequilibrium_pressure<D, R>(m, p, k);
  relaxation_rates<R>(m, k);
  return m;
}

// Density, velocity and temperature only (no P - P^eq, no rates): where
// nothing but the anomaly is needed (the halo ring and the plane before a
// march chunk) in the FP32 kernels.
template <int D>
__device__ inline NodeMoments<float> node_moments_light(const float* f, const float* g, const NodeConsts& k) {
  double s0, j[3], se;
  conserved_sums<D, float>(f, g, s0, j, se);
  NodeMoments<float> m;
  velocity_temperature<D, float>(m, s0, j, se, k);
  return m;
}

// Diagonal anomaly Qt_a = rho u_a (1 - 3T - u_a^2), Eq. (29), less its value
// at the reference state (a constant that no difference sees; zero for FP64
// storage), formed from deviations: with w = 1 - 3T - u_a^2,
// Qt_a - Qt0_a = (rho u_a - rho0 u0_a) w + rho0 u0_a (w - w0).
template <typename R>
__device__ inline R anomaly(const NodeMoments<R>& m, int a, const NodeConsts& k) {
  const R u0 = ref_u0<R>(k, a), rho0 = (R)k.rho0;
  const R w = (R)1 - (R)3 * m.T - m.u[a] * m.u[a];
  const R dw = -(R)3 * m.dT - m.du[a] * (m.u[a] + u0);
  const R dj = m.drho * m.u[a] + rho0 * m.du[a];
  return dj * w + rho0 * u0 * dw;
}

// Upwind (Sec. III.A) or central (Sec. III.D.2) difference from the anomaly
// at x - e, x, x + e; the upwind side follows the sign of u at x.
template <typename R>
__device__ inline R anomaly_derivative(int scheme, R u, R qm, R q0, R qp) {
  if (scheme == LBM_DERIV_CENTRAL) return (R)0.5 * (qp - qm);
  return (u > (R)0) ? (q0 - qm) : (qp - q0);
}

// Per-axis factors of f^ex - w (w: the reference populations, zero for
// FP64 storage): Psi(c) = Psi_c(u, P) and dPsi(c) = Psi(c) - psi0(c), so that
// with h(c) = drho Psi(c) + rho0 dPsi(c) and kf(c) = rho0 psi0_x(c),
// f^ex_i - w_i = h_x(cx) PY(cy,cz) + kf_x(cx) DY(cy,cz), PY = Psi_y Psi_z,
// DY = Psi_y Psi_z - psi0_y psi0_z.
template <typename R>
struct AxisF {
  R psi[3], dpsi[3];
};

// u, du = u - u0, dP = P - P0 (P = T + u^2 + corr d, the diagonal of Eq. (30)).
template <typename R, bool DEV>
__device__ inline AxisF<R> axis_f(R u, R du, R dP, R P0) {
  AxisF<R> a;
  a.psi[1] = ((R)1 - P0) - dP;
  a.psi[2] = (R)0.5 * (u + P0 + dP);
  a.psi[0] = (R)0.5 * (-u + P0 + dP);
  if (DEV) {
    a.dpsi[1] = -dP;
    a.dpsi[2] = (R)0.5 * (du + dP);
    a.dpsi[0] = (R)0.5 * (-du + dP);
  } else {
    a.dpsi[0] = a.dpsi[1] = a.dpsi[2] = (R)0;
  }
  return a;
}

// Per-axis factors of g^eq (Eq. (42) in closed form): a(c) = Psi_c(u, T + u^2),
// b(0) = u^2/2 - B2, b(+-1) = (+-B1 + B2)/2 with B1 = u (u^2 + 2T)/2,
// B2 = (u^4 + 5 u^2 T + 2 T^2)/2, and their departures da, db from the
// reference (u0, T0), formed from du and dT so that no large terms cancel.
template <typename R>
struct AxisG {
  R a[3], b[3], da[3], db[3];
};

template <typename R, bool DEV>
__device__ inline AxisG<R> axis_g(R u, R du, R u0, R T, R dT, R T0) {
  AxisG<R> x;
  const R u2 = u * u;
  const R B1 = (R)0.5 * u * (u2 + (R)2 * T);
  const R B2 = (R)0.5 * (u2 * u2 + (R)5 * u2 * T) + T * T;
  x.a[1] = (R)1 - T - u2;
  x.a[2] = (R)0.5 * (u + T + u2);
  x.a[0] = (R)0.5 * (-u + T + u2);
  x.b[1] = (R)0.5 * u2 - B2;
  x.b[2] = (R)0.5 * (B1 + B2);
  x.b[0] = (R)0.5 * (-B1 + B2);
  if (DEV) {
    const R su = u + u0;
    const R du2 = du * su;                                    // u^2 - u0^2
    const R u02 = u0 * u0;
    const R dB1 = (R)0.5 * du * (u2 + u * u0 + u02) + du * T + u0 * dT;
    const R dB2 = (R)0.5 * du2 * (u2 + u02) + (R)2.5 * (du2 * T + u02 * dT) + dT * (T + T0);
    x.da[1] = -(dT + du2);
    x.da[2] = (R)0.5 * (du + dT + du2);
    x.da[0] = (R)0.5 * (-du + dT + du2);
    x.db[1] = (R)0.5 * du2 - dB2;
    x.db[2] = (R)0.5 * (dB1 + dB2);
    x.db[0] = (R)0.5 * (-dB1 + dB2);
  } else {
    x.da[0] = x.da[1] = x.da[2] = (R)0;
    x.db[0] = x.db[1] = x.db[2] = (R)0;
  }
  return x;
}

// Builds (f^ex - w) and (g^eq - w) (the equilibria with the corrections d_a;
// d = 0 gives f^eq) row by row, a row being the three populations
// jx + 3p, jx = c_x + 1, of one (c_y, c_z) pair p: the per-axis factors are
// formed once and each row costs a few products, so a caller can relax a
// row as soon as it is built.
template <int D, typename R, bool DEV>
struct EqBuilder {
  AxisF<R> F[3];
  AxisG<R> G[3];
  R hx[3], kx[3], G1[3], G2[3], G3[3], G4[3];
  R p0y[3], b0y[3];  // y-axis reference factors (a0 = psi0)
  R eps, deps, eps0;

  __device__ inline EqBuilder(const NodeMoments<R>& m, const R* d, const NodeConsts& k) {
    const R T0 = (R)k.T0, rho0 = (R)k.rho0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const R u0 = ref_u0<R>(k, a);
      const R dP = m.dT + m.du[a] * (m.u[a] + u0) + m.corr * d[a];  // P - P0
      F[a] = axis_f<R, DEV>(m.u[a], m.du[a], dP, ref_P0<R>(k, a));
      G[a] = axis_g<R, DEV>(m.u[a], m.du[a], u0, m.T, m.dT, T0);
    }
    if (k.caloric) {  // U(T) = U(T0) + (U(T) - U(T0))
      deps = caloric_du<R>((R)k.Cv, (R)k.cv1, (R)k.cv2, T0, m.dT);
      eps0 = (R)k.U0;
      eps = eps0 + deps;
    } else {
      eps = (R)k.Cv * m.T;
      deps = (R)k.Cv * m.dT;
      eps0 = (R)k.Cv * T0;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      hx[c] = m.drho * F[0].psi[c] + (DEV ? rho0 * F[0].dpsi[c] : (R)0);
      kx[c] = DEV ? rho0 * ref_psi0<R>(k, 0, c) : (R)0;
      G1[c] = m.drho * G[0].a[c] + (DEV ? rho0 * G[0].da[c] : (R)0);
      G2[c] = m.drho * G[0].b[c] + (DEV ? rho0 * G[0].db[c] : (R)0);
      G3[c] = DEV ? rho0 * ref_psi0<R>(k, 0, c) : (R)0;
      G4[c] = DEV ? rho0 * ref_b0<R>(k, 0, c) : (R)0;
      p0y[c] = ref_psi0<R>(k, 1, c);
      b0y[c] = ref_b0<R>(k, 1, c);
    }
  }

  __device__ inline void row(int p, R* fe, R* ge) const {
    const int jy = p % 3, jz = p / 3;  // index = c + 1
    R PY, DY, A, Bs, dA, dBs;
    if (D == 3) {
      PY = F[1].psi[jy] * F[2].psi[jz];
      DY = F[1].dpsi[jy] * F[2].psi[jz] + p0y[jy] * F[2].dpsi[jz];
      A = G[1].a[jy] * G[2].a[jz];
      Bs = G[1].b[jy] * G[2].a[jz] + G[1].a[jy] * G[2].b[jz];
      dA = G[1].da[jy] * G[2].a[jz] + p0y[jy] * G[2].da[jz];
      dBs = G[1].db[jy] * G[2].a[jz] + b0y[jy] * G[2].da[jz] + G[1].da[jy] * G[2].b[jz] + p0y[jy] * G[2].db[jz];
    } else {
      PY = F[1].psi[jy];
      DY = F[1].dpsi[jy];
      A = G[1].a[jy];
      Bs = G[1].b[jy];
      dA = G[1].da[jy];
      dBs = G[1].db[jy];
    }
    const R V1 = eps * A + Bs;
    const R V2 = deps * A + eps0 * dA + dBs;
#pragma unroll
    for (int jx = 0; jx < 3; ++jx) {
      R fv = hx[jx] * PY;
      R gv = G1[jx] * V1 + G2[jx] * A;
      if (DEV) {
        fv += kx[jx] * DY;
        gv += G3[jx] * V2 + G4[jx] * dA;
      }
      fe[jx] = fv;
      ge[jx] = gv;
    }
  }
};

// All Q populations: f^ex - w into fe, g^eq - w into ge.
template <int D, typename R, bool DEV>
__device__ inline void equilibria(const NodeMoments<R>& m, const R* d, const NodeConsts& k, R* fe, R* ge) {
  const EqBuilder<D, R, DEV> E(m, d, k);
  constexpr int NR = (D == 3) ? 9 : 3;
#pragma unroll
  for (int p = 0; p < NR; ++p) E.row(p, fe + 3 * p, ge + 3 * p);
}

// BGK relaxation of both populations in place (Eqs. (1), (2)): f, g hold the
// post-streaming values (deviations when DEV) on entry and the
// post-collision values on exit.
template <int D, typename R, bool DEV>
__device__ inline void collide(R* f, R* g, const NodeMoments<R>& m, const R* d, const NodeConsts& k) {
  constexpr int Q = lat_q(D);
  const EqBuilder<D, R, DEV> E(m, d, k);
  // q* - q^eq, Eq. (46)
  R dq[3];
  dq[0] = m.u[0] * m.pn[0] + m.u[1] * m.pn[3] + (D == 3 ? m.u[2] * m.pn[4] : (R)0) + (R)0.5 * m.u[0] * d[0];
  dq[1] = m.u[0] * m.pn[3] + m.u[1] * m.pn[1] + (D == 3 ? m.u[2] * m.pn[5] : (R)0) + (R)0.5 * m.u[1] * d[1];
  dq[2] = (D == 3) ? m.u[0] * m.pn[4] + m.u[1] * m.pn[5] + m.u[2] * m.pn[2] + (R)0.5 * m.u[2] * d[2] : (R)0;
  const R half_dw = (R)0.5 * (m.omega - m.omega1);
  // Row sums of the collision increments (DEV only), rows as in moment_sums.
  constexpr int NR = (D == 3) ? 9 : 3;
  R r0[NR], rx[NR], rg[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    R fe[3], ge[3], df[3], dg[3];
    E.row(r, fe, ge);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int i = 3 * r + c;
      const int cx = vx(i), cy = vy(i), cz = (D == 3) ? vz(i) : 0;
      df[c] = m.omega * (fe[c] - f[i]);
      dg[c] = m.omega1 * (ge[c] - g[i]);
      const int c2 = cx * cx + cy * cy + cz * cz;
      if (c2 == 1) {
        const R cdq = cx ? (cx > 0 ? dq[0] : -dq[0]) : cy ? (cy > 0 ? dq[1] : -dq[1]) : (cz > 0 ? dq[2] : -dq[2]);
        dg[c] -= half_dw * cdq;
      }
      f[i] += df[c];
      g[i] += dg[c];
    }
    if (DEV) {
      rx[r] = df[2] - df[0];
      r0[r] = (df[2] + df[0]) + df[1];
      rg[r] = (dg[2] + dg[0]) + dg[1];
    }
  }
  R sf = 0, sx = 0, sy = 0, sz = 0, sg = 0;
  if (DEV) {
    if (D == 3) {
      R l0[3], lx[3], lg[3];
#pragma unroll
      for (int z = 0; z < 3; ++z) {
        l0[z] = (r0[3 * z] + r0[3 * z + 2]) + r0[3 * z + 1];
        lx[z] = (rx[3 * z] + rx[3 * z + 2]) + rx[3 * z + 1];
        lg[z] = (rg[3 * z] + rg[3 * z + 2]) + rg[3 * z + 1];
      }
      sf = (l0[0] + l0[2]) + l0[1];
      sx = (lx[0] + lx[2]) + lx[1];
      sg = (lg[0] + lg[2]) + lg[1];
      sy = ((r0[2] - r0[0]) + (r0[8] - r0[6])) + (r0[5] - r0[3]);
      sz = l0[2] - l0[0];
    } else {
      sf = (r0[0] + r0[2]) + r0[1];
      sx = (rx[0] + rx[2]) + rx[1];
      sg = (rg[0] + rg[2]) + rg[1];
      sy = r0[2] - r0[0];
    }
  }
  if (DEV) {
    // The collision conserves rho, rho u and rho E exactly (Eqs. (3)-(5)), so
    // the increments sum to zero in exact arithmetic.  In FP32 the equilibria
    // are evaluated with rounding errors that keep their sign from node to
    // node and step to step, and the totals would drift.  The increments are
    // small, so their FP32 sums are accurate: take the momentum residual off
    // the +-e_a pair and the mass and energy residuals off the rest
    // populations.
    constexpr int rest = (Q - 1) / 2;
    constexpr int px = rest + 1, mx = rest - 1, py = rest + 3, my = rest - 3, pz = rest + 9, mz = rest - 9;
    const R hx = (R)0.5 * sx, hy = (R)0.5 * sy;
    f[px] -= hx;
    f[mx] += hx;
    f[py] -= hy;
    f[my] += hy;
    if (D == 3) {
      const R hz = (R)0.5 * sz;
      f[pz] -= hz;
      f[mz] += hz;
    }
    f[rest] -= sf;
    g[rest] -= sg;
  }
}

}  // namespace lbm
