"""What FP32 deviation storage alone costs a flow, measured by the oracle.

The library's FP32 storage keeps f_i - f^eq_i(rho_0, u_0, T_0) and the same
for g in single precision.  Two oracle runs measure what that costs a flow:

* the FP32 storage model (orc_set_fp32_storage) rounds exactly those
  deviations after init and after every step and keeps FP64 arithmetic;
* the upwind band run (orc_set_upwind_band) takes the other upwind side of
  Sec. III.A at every decision whose |u_a| is within the FP32 resolution of
  the velocity, where FP32 cannot decide the sign.

Their departures from the plain FP64 oracle run are floors of the case:
where the flow amplifies perturbations (a shock) or a velocity component
crosses zero (a switch of the upwind side changes the anomaly difference by
its second difference, far above FP32 rounding) an FP32 path lands somewhere
among such outcomes.  Nothing here comes from the GPU library.
"""
import numpy as np

import oracle


def fp32_reference(D, rho_ref=1.0, u_ref=None, T_ref=0.15, gamma=1.4, cv=None):
    """Reference populations of FP32 deviation storage at the reference
    state rounded to FP32 (the library rounds rho_ref, u_ref and T_ref)."""
    r = float(np.float32(rho_ref))
    T = float(np.float32(T_ref))
    u = [0.0, 0.0, 0.0]
    for a, v in enumerate(list(u_ref or [])[:D]):
        u[a] = float(np.float32(v))
    f = oracle.feq(D, r, u, T)
    law = oracle.caloric(cv, gamma)
    g = oracle.geq_u(D, r, u, T, oracle.internal_energy(law, T))
    return f, g


def storage_run(D, dims, fields, steps, rho_ref=1.0, u_ref=None, T_ref=0.15, **sim_kw):
    """Oracle run of `steps` steps with the FP32 storage model; sim_kw as for
    oracle.Sim (mu, Pr, gamma, visc_exp, T_ref of the power law, bc, deriv, cv)."""
    gamma = sim_kw.get("gamma", 1.4)
    s = oracle.Sim(D, dims, T_ref=T_ref, **sim_kw)
    s.set_fp32_storage(*fp32_reference(D, rho_ref, u_ref, T_ref, gamma, sim_kw.get("cv")))
    s.init(*fields)
    s.step(steps)
    return s


def velocity_resolution(u):
    """One unit in the last place of FP32 at the largest initial velocity
    component: below this size the sign of a velocity component that passed
    through FP32 storage and arithmetic is not determined."""
    return float(2.0 ** -24 * np.abs(np.asarray(u)).max())


def band_run(D, dims, fields, steps, band, T_ref=0.15, **sim_kw):
    """Oracle run (FP64) in which every upwind decision with |u_a| <= band
    takes the other side (orc_set_upwind_band): the other valid reading of
    the sign test wherever FP32 cannot resolve it."""
    s = oracle.Sim(D, dims, T_ref=T_ref, **sim_kw)
    s.set_upwind_band(band)
    s.init(*fields)
    s.step(steps)
    return s


def rel(a, b):
    """max |a - b| / max |b| over the grid (per field; for u, the max of |u|)."""
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def field_errors(out, ref):
    return {k: rel(a, b) for k, a, b in zip(("rho", "u", "T"), out, ref)}
