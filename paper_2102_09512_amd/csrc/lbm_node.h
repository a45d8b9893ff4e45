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
  R pn[6];   // P - P^eq: xx, yy, zz, xy, xz, yz
  R omega, omega1;
};

struct NodeConsts {
  double rho0, T0;
  double inv_Cv, Cv, Pr;
  double mu0, visc_exp, inv_Tref;
};

template <typename R>
__device__ inline R viscosity(const NodeConsts& k, R T) {
  if (k.visc_exp == 0.0) return (R)k.mu0;
  return (R)k.mu0 * pow(T * (R)k.inv_Tref, (R)k.visc_exp);
}

// P - P^eq with P = sum c c f (Eq. (47)) and P^eq = rho T I + rho u u
// (Eqs. (23), (25)); the isotropic part rho T - rho0 T0 = drho T0 + rho dT.
template <int D, typename R>
__device__ inline void nonequilibrium_pressure(NodeMoments<R>& m, const R* p, const NodeConsts& k) {
  const R iso = m.drho * (R)k.T0 + m.rho * m.dT;
  m.pn[0] = p[0] - m.rho * m.u[0] * m.u[0] - iso;
  m.pn[1] = p[1] - m.rho * m.u[1] * m.u[1] - iso;
  m.pn[2] = (D == 3) ? p[2] - m.rho * m.u[2] * m.u[2] - iso : (R)0;
  m.pn[3] = p[3] - m.rho * m.u[0] * m.u[1];
  m.pn[4] = (D == 3) ? p[4] - m.rho * m.u[0] * m.u[2] : (R)0;
  m.pn[5] = (D == 3) ? p[5] - m.rho * m.u[1] * m.u[2] : (R)0;
}

// omega from mu = (1/omega - 1/2) rho T (Eq. (92)); omega_1 from Eq. (96).
template <typename R>
__device__ inline void relaxation_rates(NodeMoments<R>& m, const NodeConsts& k) {
  const R mu = viscosity<R>(k, m.T);
  m.omega = (R)1 / (mu / (m.rho * m.T) + (R)0.5);
  m.omega1 = (R)2 * (R)k.Pr * m.omega / ((R)2 - m.omega + (R)k.Pr * m.omega);
}

// Moments of the post-streaming populations f, g (Eqs. (3)-(7)); deviations
// from the rest state (rho0, 0, T0) when the storage is FP32.  FP64 storage
// (rho0 = 0, rhoE0 = 0) sums the full populations.  The FP32 path keeps
// every quantity a deviation: rho Cv (T - T0) = sum g - rho |u|^2 / 2 -
// (rho - rho0) Cv T0, so no large terms cancel.
template <int D, typename R>
__device__ inline NodeMoments<R> node_moments(const R* f, const R* g, const NodeConsts& k) {
  constexpr int Q = lat_q(D);
  R s0 = 0, jx = 0, jy = 0, jz = 0, se = 0;
  R p[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = vx(i), cy = vy(i), cz = (D == 3) ? vz(i) : 0;
    const R w = f[i];
    s0 += w;
    se += g[i];
    if (cx) jx += cx > 0 ? w : -w;
    if (cy) jy += cy > 0 ? w : -w;
    if (cz) jz += cz > 0 ? w : -w;
    if (cx) p[0] += w;
    if (cy) p[1] += w;
    if (cz) p[2] += w;
    if (cx && cy) p[3] += (cx == cy) ? w : -w;
    if (cx && cz) p[4] += (cx == cz) ? w : -w;
    if (cy && cz) p[5] += (cy == cz) ? w : -w;
  }
  NodeMoments<R> m;
  m.drho = s0;
  m.rho = (R)k.rho0 + s0;
  const R inv = (R)1 / m.rho;
  m.u[0] = jx * inv;
  m.u[1] = jy * inv;
  m.u[2] = (D == 3) ? jz * inv : (R)0;
  const R ke = (R)0.5 * m.rho * (m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2]);
  m.dT = (se - ke - m.drho * (R)(k.Cv * k.T0)) * inv * (R)k.inv_Cv;
  m.T = (R)k.T0 + m.dT;
  nonequilibrium_pressure<D, R>(m, p, k);
  relaxation_rates<R>(m, k);
  return m;
}

// Density, velocity and temperature only (no P - P^eq, no rates): where
// nothing but the anomaly is needed (the halo ring and the plane before a
// march chunk) in the FP32 kernels.
template <int D>
__device__ inline NodeMoments<float> node_moments_light(const float* f, const float* g, const NodeConsts& k) {
  constexpr int Q = lat_q(D);
  float s0 = 0.f, jx = 0.f, jy = 0.f, jz = 0.f, se = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = vx(i), cy = vy(i), cz = (D == 3) ? vz(i) : 0;
    const float v = f[i];
    s0 += v;
    se += g[i];
    if (cx) jx += cx > 0 ? v : -v;
    if (cy) jy += cy > 0 ? v : -v;
    if (cz) jz += cz > 0 ? v : -v;
  }
  NodeMoments<float> m;
  m.drho = s0;
  m.rho = (float)k.rho0 + s0;
  const float inv = 1.f / m.rho;
  m.u[0] = jx * inv;
  m.u[1] = jy * inv;
  m.u[2] = (D == 3) ? jz * inv : 0.f;
  const float ke = 0.5f * m.rho * (m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2]);
  m.dT = (se - ke - s0 * (float)(k.Cv * k.T0)) * inv * (float)k.inv_Cv;
  m.T = (float)k.T0 + m.dT;
  return m;
}

// Diagonal anomaly Qt_a = rho u_a (1 - 3T) - rho u_a^3, Eq. (29).
template <typename R>
__device__ inline R anomaly(const NodeMoments<R>& m, int a) {
  const R u = m.u[a];
  return m.rho * u * ((R)1 - (R)3 * m.T) - m.rho * u * u * u;
}

// Upwind (Sec. III.A) or central (Sec. III.D.2) difference from the anomaly
// at x - e, x, x + e; the upwind side follows the sign of u at x.
template <typename R>
__device__ inline R anomaly_derivative(int scheme, R u, R qm, R q0, R qp) {
  if (scheme == LBM_DERIV_CENTRAL) return (R)0.5 * (qp - qm);
  return (u > (R)0) ? (q0 - qm) : (qp - q0);
}

// Per-axis factors of f^ex - w:  Psi(c), and h(c) = drho Psi(c) + rho0 dPsi(c),
// k(c) = rho0 Psi0(c), so that f^ex_i - w_i = h_x(cx) PY(cy,cz) + k_x(cx) DY(cy,cz)
// with PY = Psi_y Psi_z and DY = Psi_y Psi_z - Psi0_y Psi0_z.
template <typename R>
struct AxisF {
  R psi[3], dpsi[3];
};

template <typename R, bool DEV>
__device__ inline AxisF<R> axis_f(R u, R dP, R T0) {
  // dP = P - T0, the departure of the diagonal second moment from the rest value
  AxisF<R> a;
  a.dpsi[1] = -dP;
  a.dpsi[2] = (R)0.5 * (u + dP);
  a.dpsi[0] = (R)0.5 * (-u + dP);
  a.psi[1] = ((R)1 - T0) - dP;
  a.psi[2] = (R)0.5 * (u + T0 + dP);
  a.psi[0] = (R)0.5 * (-u + T0 + dP);
  if (!DEV) {
    a.dpsi[0] = a.dpsi[1] = a.dpsi[2] = (R)0;
  }
  return a;
}

// Per-axis factors of g^eq - w (see the header comment).
template <typename R>
struct AxisG {
  R a[3], b[3], da[3], db[3];
};

template <typename R, bool DEV>
__device__ inline AxisG<R> axis_g(R u, R T, R dT, R T0) {
  AxisG<R> x;
  const R u2 = u * u;
  const R B1 = (R)0.5 * u * (u2 + (R)2 * T);
  const R B2v = (R)0.5 * (u2 * u2 + (R)5 * u2 * T);  // B2 without the T^2 term
  x.a[1] = (R)1 - T - u2;
  x.a[2] = (R)0.5 * (u + T + u2);
  x.a[0] = (R)0.5 * (-u + T + u2);
  const R B2 = B2v + T * T;
  x.b[1] = (R)0.5 * u2 - B2;
  x.b[2] = (R)0.5 * (B1 + B2);
  x.b[0] = (R)0.5 * (-B1 + B2);
  if (DEV) {
    const R dT2 = dT * (T + T0);  // T^2 - T0^2
    x.da[1] = -(dT + u2);
    x.da[2] = (R)0.5 * (u + dT + u2);
    x.da[0] = (R)0.5 * (-u + dT + u2);
    x.db[1] = (R)0.5 * u2 - B2v - dT2;
    x.db[2] = (R)0.5 * (B1 + B2v + dT2);
    x.db[0] = (R)0.5 * (-B1 + B2v + dT2);
  } else {
    x.da[0] = x.da[1] = x.da[2] = (R)0;
    x.db[0] = x.db[1] = x.db[2] = (R)0;
  }
  return x;
}

// Rest-state per-axis factors at temperature T0 (u = 0).
template <typename R>
struct Rest {
  R psi0[3], a0[3], b0[3];
};

template <typename R>
__device__ inline Rest<R> rest_factors(R T0) {
  Rest<R> r;
  r.psi0[1] = (R)1 - T0;
  r.psi0[0] = r.psi0[2] = (R)0.5 * T0;
  r.a0[1] = (R)1 - T0;
  r.a0[0] = r.a0[2] = (R)0.5 * T0;
  r.b0[1] = -T0 * T0;
  r.b0[0] = r.b0[2] = (R)0.5 * T0 * T0;
  return r;
}

// Writes (f^ex - w) and (g^eq - w) for all Q populations (the equilibria with
// the corrections d_a; d = 0 gives f^eq).  Population i of the f set goes to
// fe[i], of the g set to ge[i].
template <int D, typename R, bool DEV>
__device__ inline void equilibria(const NodeMoments<R>& m, const R* d, const NodeConsts& k, R* fe, R* ge) {
  const R T0 = (R)k.T0, rho0 = (R)k.rho0;
  const Rest<R> rs = rest_factors<R>(T0);
  const R corr = ((R)2 - m.omega) / ((R)2 * m.rho * m.omega);

  AxisF<R> F[3];
  AxisG<R> G[3];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const R dP = m.dT + m.u[a] * m.u[a] + corr * d[a];
    F[a] = axis_f<R, DEV>(m.u[a], dP, T0);
    G[a] = axis_g<R, DEV>(m.u[a], m.T, m.dT, T0);
  }
  const R eps = (R)k.Cv * m.T;
  const R deps = (R)k.Cv * m.dT;
  const R eps0 = (R)k.Cv * T0;

  // x-axis coefficients
  R hx[3], kx[3], G1[3], G2[3], G3[3], G4[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    hx[c] = m.drho * F[0].psi[c] + (DEV ? rho0 * F[0].dpsi[c] : (R)0);
    kx[c] = DEV ? rho0 * rs.psi0[c] : (R)0;
    G1[c] = m.drho * G[0].a[c] + (DEV ? rho0 * G[0].da[c] : (R)0);
    G2[c] = m.drho * G[0].b[c] + (DEV ? rho0 * G[0].db[c] : (R)0);
    G3[c] = DEV ? rho0 * rs.a0[c] : (R)0;
    G4[c] = DEV ? rho0 * rs.b0[c] : (R)0;
  }

  constexpr int NP = (D == 3) ? 9 : 3;  // (cy, cz) pairs
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int jy = p % 3, jz = p / 3;   // index = c + 1
    R PY, DY, A, Bs, dA, dBs;
    if (D == 3) {
      PY = F[1].psi[jy] * F[2].psi[jz];
      DY = F[1].dpsi[jy] * F[2].psi[jz] + rs.psi0[jy] * F[2].dpsi[jz];
      A = G[1].a[jy] * G[2].a[jz];
      Bs = G[1].b[jy] * G[2].a[jz] + G[1].a[jy] * G[2].b[jz];
      dA = G[1].da[jy] * G[2].a[jz] + rs.a0[jy] * G[2].da[jz];
      dBs = G[1].db[jy] * G[2].a[jz] + rs.b0[jy] * G[2].da[jz] + G[1].da[jy] * G[2].b[jz] +
            rs.a0[jy] * G[2].db[jz];
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
      const int i = jx + 3 * p;
      R fv = hx[jx] * PY;
      R gv = G1[jx] * V1 + G2[jx] * A;
      if (DEV) {
        fv += kx[jx] * DY;
        gv += G3[jx] * V2 + G4[jx] * dA;
      }
      fe[i] = fv;
      ge[i] = gv;
    }
  }
}

// BGK relaxation of both populations in place (Eqs. (1), (2)): f, g hold the
// post-streaming values (deviations when DEV) on entry and the
// post-collision values on exit.
template <int D, typename R, bool DEV>
__device__ inline void collide(R* f, R* g, const NodeMoments<R>& m, const R* d, const NodeConsts& k) {
  constexpr int Q = lat_q(D);
  R fe[Q], ge[Q];
  equilibria<D, R, DEV>(m, d, k, fe, ge);
  // q* - q^eq, Eq. (46)
  R dq[3];
  dq[0] = m.u[0] * m.pn[0] + m.u[1] * m.pn[3] + (D == 3 ? m.u[2] * m.pn[4] : (R)0) + (R)0.5 * m.u[0] * d[0];
  dq[1] = m.u[0] * m.pn[3] + m.u[1] * m.pn[1] + (D == 3 ? m.u[2] * m.pn[5] : (R)0) + (R)0.5 * m.u[1] * d[1];
  dq[2] = (D == 3) ? m.u[0] * m.pn[4] + m.u[1] * m.pn[5] + m.u[2] * m.pn[2] + (R)0.5 * m.u[2] * d[2] : (R)0;
  const R half_dw = (R)0.5 * (m.omega - m.omega1);
  // Sums of the collision increments (DEV only): mass, momentum, energy.
  R sf = 0, sx = 0, sy = 0, sz = 0, sg = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cx = vx(i), cy = vy(i), cz = (D == 3) ? vz(i) : 0;
    const R df = m.omega * (fe[i] - f[i]);
    R dg = m.omega1 * (ge[i] - g[i]);
    const int c2 = cx * cx + cy * cy + cz * cz;
    if (c2 == 1) {
      const R cdq = cx ? (cx > 0 ? dq[0] : -dq[0]) : cy ? (cy > 0 ? dq[1] : -dq[1]) : (cz > 0 ? dq[2] : -dq[2]);
      dg -= half_dw * cdq;
    }
    f[i] += df;
    g[i] += dg;
    if (DEV) {
      sf += df;
      sg += dg;
      if (cx) sx += cx > 0 ? df : -df;
      if (cy) sy += cy > 0 ? df : -df;
      if (cz) sz += cz > 0 ? df : -df;
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
