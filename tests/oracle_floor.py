"""What FP32 deviation storage alone costs a flow, measured by the oracle.

The library's FP32 storage keeps f_i - f^eq_i(rho_0, u_0, T_0) and the same
for g in single precision.  An oracle run with its FP32 storage model
(orc_set_fp32_storage) rounds exactly those deviations after init and after
every step and keeps FP64 arithmetic otherwise; its departure from the plain
FP64 oracle run is the floor of FP32 storage for the case: where the flow
amplifies perturbations (a shock, the sign of a velocity component that
decides the upwind side of Sec. III.A) no FP32 path can do better than this
by more than a small factor.  Nothing here comes from the GPU library.
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


def rel(a, b):
    """max |a - b| / max |b| over the grid (per field; for u, the max of |u|)."""
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def field_errors(out, ref):
    return {k: rel(a, b) for k, a, b in zip(("rho", "u", "T"), out, ref)}
