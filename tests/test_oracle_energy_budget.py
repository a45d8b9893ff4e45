"""Long-time dynamics of the oracle pinned by the kinetic-energy budget of
decaying turbulence (Sec. III.D's setting, at low Mach number).

For a periodic flow with constant dynamic viscosity mu, the Navier-Stokes
equations that the method recovers (Eqs. (92)-(97)) give

    d/dt sum 1/2 rho |u|^2 = - mu sum |curl u|^2 - (4/3 mu + zeta) sum (div u)^2
                              + sum p div u,

and at turbulent Mach 0.1 the last two terms are a fraction of a percent of the
first.  So between two times the kinetic energy the oracle loses must equal the
time integral of mu sum |curl u|^2.  The vorticity is taken spectrally from the
oracle's own velocity field (exact for a periodic grid field), so the check
does not depend on the diagnostics' difference formula.  The first 50 steps are
left out: the solenoidal start with uniform pressure sheds sound that takes
kinetic energy in that time.

Measured: the energy lost between steps 50 and 300 is 1.031 times the integral
(first-order upwind anomaly difference; 1.023 with central differences): the
lattice's own dissipation at this resolution.  The bar is 5 %.  Planted in a
copy of the oracle, the g rate in place of the f rate gives 1.72, and a
relaxation rate built from mu / rho instead of mu / p gives 0.16."""
import numpy as np
import pytest

import oracle
from paper_2102_09512_amd import inputs as I


def _enstrophy_sum(u, n):
    """sum over nodes of |curl u|^2 from the discrete Fourier transform of
    u (components x, y, z over (z, y, x) arrays)."""
    k = np.fft.fftfreq(n, d=1.0 / n) * 2.0 * np.pi / n
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    ux, uy, uz = (np.fft.fftn(u[a]) for a in range(3))
    wx = 1j * (ky * uz - kz * uy)
    wy = 1j * (kz * ux - kx * uz)
    wz = 1j * (kx * uy - ky * ux)
    return float((np.abs(wx) ** 2 + np.abs(wy) ** 2 + np.abs(wz) ** 2).sum() / n ** 3)


@pytest.mark.parametrize("deriv", [oracle.UPWIND, oracle.CENTRAL])
def test_kinetic_energy_budget_of_decaying_turbulence(deriv):
    n, mu, every, t0, t1 = 48, 0.02, 5, 50, 300
    fields = I.turbulence(3, n, seed=2, k0_index=2, Ma_t=0.1, T0=0.15)
    s = oracle.Sim(3, (n, n, n), gamma=1.4, Pr=0.7, mu=mu, visc_exp=0.0, T_ref=0.15, deriv=deriv)
    s.init(*fields)
    times, kin, diss = [], [], []
    for step in range(t1 + 1):
        if step >= t0 and step % every == 0:
            rho, u, _ = s.moments()
            times.append(step)
            kin.append(0.5 * float((rho * (u ** 2).sum(0)).sum()))
            diss.append(mu * _enstrophy_sum(u, n))
        if step < t1:
            s.step(1)
    lost = kin[0] - kin[-1]
    dissipated = float(np.trapezoid(diss, dx=every))
    ratio = lost / dissipated
    print(f"kinetic energy {kin[0]:.3f} -> {kin[-1]:.3f}; lost {lost:.4f}, dissipated {dissipated:.4f}, "
          f"ratio {ratio:.4f}")
    assert kin[-1] < 0.8 * kin[0]  # a decay long enough to measure
    assert abs(ratio - 1.0) <= 0.05, ratio
