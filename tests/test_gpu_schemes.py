"""The derivative scheme of the anomaly in subsonic turbulence (Sec. III.D.2):
with first-order upwind or second-order central differences of the anomaly,
decaying turbulence at Ma_t = 0.3, Re_lambda = 72 has the same statistics
(the paper reports the enstrophy history as insensitive to the scheme and the
other statistics as behaving alike).  The paper's figure is not available, so
the bound is this build's: histories of K, Ma_t, theta_rms, rho_rms and the
enstrophy over five large-eddy turnovers agree within 2% (the largest
difference is printed)."""
import math

import numpy as np
import pytest

from paper_2102_09512_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _stats_history(lbm, n, fields, mu, deriv, steps, every):
    h = lbm.lbm_create(3, (n, n, n), 1.4, 0.7, mu, precision=lbm.LBM_FP32_DEV, visc_exponent=0.76, T_ref=0.15,
                       deriv_scheme=deriv)
    rows = []
    try:
        lbm.lbm_set_stream(h, torch.cuda.current_stream())
        lbm.lbm_init_fields(h, *(torch.from_numpy(a).cuda() for a in fields))
        for k in range(steps // every):
            lbm.lbm_step(h, every)
            d = lbm.lbm_diagnostics(h)
            N = d["nodes"]
            assert d["nonfinite"] == 0
            rows.append([d["kinetic_energy"] / N, math.sqrt(d["u2_sum"] / N) / (d["cs_sum"] / N),
                         math.sqrt(d["dilatation_sq_sum"] / N),
                         math.sqrt(max(d["rho2_sum"] / N - (d["mass"] / N) ** 2, 0.0)),
                         0.5 * d["vorticity_sq_sum"] / N])
    finally:
        lbm.lbm_destroy(h)
    return np.array(rows)


def test_central_and_upwind_give_the_same_subsonic_statistics():
    from paper_2102_09512_amd import lbm

    n = 256
    fields = I.turbulence(3, n, seed=0, k0_index=4, Ma_t=0.3, T0=0.15)
    mu = I.turbulence_viscosity(n, k0_index=4, Ma_t=0.3, T0=0.15, Re_lambda=72.0)
    u_rms = math.sqrt(np.mean(np.sum(fields[1] ** 2, axis=0)) / 3.0)
    tau = math.sqrt(2.0 * math.pi) / (4 * 2 * math.pi / n) / u_rms  # L_I / u_rms, in steps
    every = 100
    steps = every * int(math.ceil(5.0 * tau / every))
    print(f"[gpu case] 256^3 Ma_t 0.3: upwind vs central over {steps} steps (tau = {tau:.0f} steps)", flush=True)
    up = _stats_history(lbm, n, fields, mu, lbm.LBM_DERIV_UPWIND, steps, every)
    ce = _stats_history(lbm, n, fields, mu, lbm.LBM_DERIV_CENTRAL, steps, every)
    names = ("K", "Ma_t", "theta_rms", "rho_rms", "enstrophy")
    rel = np.abs(up - ce) / np.abs(ce)
    for j, name in enumerate(names):
        k = int(np.argmax(rel[:, j]))
        print(f"  {name}: max relative difference {rel[k, j]:.2e} at step {(k + 1) * every} "
              f"(upwind {up[k, j]:.5e}, central {ce[k, j]:.5e})", flush=True)
    # the enstrophy peaks and decays; theta_rms rises from 0 and decays (Sec. III.D)
    assert np.argmax(up[:, 4]) not in (0, len(up) - 1)
    assert rel.max() < 0.02
