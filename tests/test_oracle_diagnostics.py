"""Pins of the oracle's whole-field diagnostics against closed forms.

The diagnostics are sums over the stored state of the totals of Eqs. (3)-(5)
(mass, momentum, energy) and of the turbulence statistics of Sec. III.D
(kinetic energy K, dilatation, vorticity / enstrophy, dissipation mu |curl u|^2,
per-axis velocity and gradient variances).  Each case below initialises the
oracle with an analytic field (the stored populations are then the equilibria
of that field, whose moments return it to rounding) and compares every slot
with the value the field gives in closed form:

* a single Fourier mode sin(2 pi m x / n) sums to 0 over a period and its
  square to n/2 (n >= 3), and its central difference (f(x+1) - f(x-1))/2 is
  sin(2 pi m / n) cos(2 pi m x / n);
* a linear profile a x on a zero-gradient axis has central difference a
  inside and a/2 at both clamped ends.

The cases are chosen so that a dropped factor (the 1/2 of K or of the central
difference), a sign or axis mistake in the curl, or a wrong viscosity in the
dissipation changes some slot by far more than rounding.
"""
import math

import numpy as np
import pytest

import oracle

CV = 2.5  # 1 / (gamma - 1) at gamma = 1.4
GAMMA = 1.4
TOL = 1e-12


def _diag(D, dims, rho, u, T, bc=(0, 0, 0), mu=0.02, visc_exp=0.0, T_ref=0.15):
    s = oracle.Sim(D, dims, gamma=GAMMA, Pr=0.7, mu=mu, visc_exp=visc_exp, T_ref=T_ref, bc=bc)
    s.init(rho, u, T)
    return s.diagnostics()


def _close(got, want, scale):
    assert abs(got - want) <= TOL * scale, (got, want)


def _mode(n, m=1):
    return 2.0 * math.pi * m / n


def test_compressive_mode_dilatation_kinetic_energy_and_density_moments():
    """u_x = a sin(k x) on a periodic box whose density varies along z:
    Sum (div u)^2 = a^2 sin^2(k) N/2, K = Sum rho u^2/2 = a^2 N/4 (the density
    mode averages out against the x-mode), no vorticity."""
    nx, ny, nz = 16, 6, 10
    N = nx * ny * nz
    a, eps, T0 = 0.05, 0.1, 0.15
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    k = _mode(nx)
    rho = 1.0 + eps * np.sin(_mode(nz) * z)
    u = np.zeros((3, nz, ny, nx))
    u[0] = a * np.sin(k * x)
    T = np.full((nz, ny, nx), T0)
    d = _diag(3, (nx, ny, nz), rho, u, T)
    s2 = math.sin(k) ** 2
    _close(d["mass"], N, N)
    for m in ("mom_x", "mom_y", "mom_z"):
        _close(d[m], 0.0, a * N)
    _close(d["kinetic"], a * a * N / 4, a * a * N)
    _close(d["energy"], CV * T0 * N + a * a * N / 4, N)
    _close(d["u2"], a * a * N / 2, a * a * N)
    _close(d["ux2"], a * a * N / 2, a * a * N)
    _close(d["uy2"], 0.0, a * a * N)
    _close(d["uz2"], 0.0, a * a * N)
    _close(d["dil2"], a * a * s2 * N / 2, a * a * N)
    _close(d["dux2"], a * a * s2 * N / 2, a * a * N)
    _close(d["duy2"], 0.0, a * a * N)
    _close(d["duz2"], 0.0, a * a * N)
    _close(d["vort2"], 0.0, a * a * N)
    _close(d["diss"], 0.0, a * a * N)
    _close(d["rho2"], N * (1 + eps * eps / 2), N)
    _close(d["cs"], N * math.sqrt(GAMMA * T0), N)
    assert d["nodes"] == N and d["nonfinite"] == 0 and d["nonpositive"] == 0


@pytest.mark.parametrize("plane", [(0, 1), (1, 2), (2, 0)])
def test_diagonal_shear_mode_vorticity_and_dilatation(plane):
    """u_p = a sin(theta), u_q = b sin(theta), theta = k (x_p + x_q), on a
    periodic cube: div u = (a + b) sin(k) cos(theta) and the curl has the one
    component normal to the (p, q) plane, +-(b - a) sin(k) cos(theta).  With
    a != b both terms of that component matter, so a sign or axis mistake in
    the curl gives (a + b)^2 instead of (b - a)^2."""
    n = 9
    N = n ** 3
    a, b, T0 = 0.02, 0.07, 0.15
    p, q = plane
    X = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")[::-1]  # x, y, z coordinates
    k = _mode(n)
    th = k * (X[p] + X[q])
    u = np.zeros((3, n, n, n))
    u[p] = a * np.sin(th)
    u[q] = b * np.sin(th)
    rho = np.ones((n, n, n))
    T = np.full((n, n, n), T0)
    d = _diag(3, (n, n, n), rho, u, T)
    s2 = math.sin(k) ** 2
    sc = (a * a + b * b) * N
    _close(d["dil2"], (a + b) ** 2 * s2 * N / 2, sc)
    _close(d["vort2"], (b - a) ** 2 * s2 * N / 2, sc)
    _close(d["diss"], 0.02 * (b - a) ** 2 * s2 * N / 2, sc)
    amp = [0.0, 0.0, 0.0]
    amp[p], amp[q] = a, b
    for ax, name in enumerate(("x", "y", "z")):
        _close(d[f"u{name}2"], amp[ax] ** 2 * N / 2, sc)
        _close(d[f"du{name}2"], amp[ax] ** 2 * s2 * N / 2, sc)
    _close(d["kinetic"], (a * a + b * b) * N / 4, sc)


def test_shear_mode_in_two_dimensions():
    """D2Q9: u_x = a sin(theta), u_y = b sin(theta), theta = k (x + y)."""
    n = 12
    N = n * n
    a, b = 0.03, -0.05
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    k = _mode(n, 2)
    th = k * (x + y)
    u = np.zeros((2, 1, n, n))
    u[0, 0] = a * np.sin(th)
    u[1, 0] = b * np.sin(th)
    rho = np.ones((1, n, n))
    T = np.full((1, n, n), 0.2)
    d = _diag(2, (n, n), rho, u, T)
    s2 = math.sin(k) ** 2
    sc = (a * a + b * b) * N
    _close(d["dil2"], (a + b) ** 2 * s2 * N / 2, sc)
    _close(d["vort2"], (b - a) ** 2 * s2 * N / 2, sc)
    _close(d["dux2"], a * a * s2 * N / 2, sc)
    _close(d["duy2"], b * b * s2 * N / 2, sc)
    _close(d["uz2"], 0.0, sc)
    _close(d["mom_z"], 0.0, sc)


def test_dissipation_follows_the_power_law_viscosity():
    """A shear u_x = a sin(k y) over a temperature that varies along z:
    Sum mu(T) |curl u|^2 = (Sum_z mu(T(z))) * n_x a^2 sin^2(k) n_y/2, with
    mu = mu0 (T/T_ref)^0.76 (Sec. III.D); the sound-speed sum likewise."""
    nx, ny, nz = 5, 8, 7
    N = nx * ny * nz
    a, mu0, Tr = 0.04, 0.03, 0.15
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    k = _mode(ny)
    Tz = Tr * (1.0 + 0.3 * np.cos(_mode(nz) * np.arange(nz)))
    T = Tz[:, None, None] * np.ones((nz, ny, nx))
    u = np.zeros((3, nz, ny, nx))
    u[0] = a * np.sin(k * y)
    rho = np.ones((nz, ny, nx))
    d = _diag(3, (nx, ny, nz), rho, u, T, mu=mu0, visc_exp=0.76, T_ref=Tr)
    plane_vort = nx * a * a * math.sin(k) ** 2 * ny / 2
    mu_z = mu0 * (Tz / Tr) ** 0.76
    _close(d["vort2"], nz * plane_vort, a * a * N)
    _close(d["diss"], mu_z.sum() * plane_vort, mu0 * a * a * N)
    _close(d["cs"], nx * ny * np.sqrt(GAMMA * Tz).sum(), N)
    _close(d["energy"], CV * nx * ny * Tz.sum() + a * a * N / 4, N)


def test_clamped_central_differences_on_zero_gradient_axes():
    """u_x = a x, u_y = b x with x zero-gradient (y, z periodic): the central
    difference is a (or b) inside and a/2 (b/2) at the two clamped ends, so
    Sum (d_x u_x)^2 = n_y n_z a^2 (n_x - 3/2) and Sum |curl u|^2 =
    n_y n_z b^2 (n_x - 3/2)."""
    nx, ny, nz = 11, 4, 3
    a, b = 0.01, 0.007
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    u = np.zeros((3, nz, ny, nx))
    u[0] = a * x
    u[1] = b * x
    rho = np.ones((nz, ny, nx))
    T = np.full((nz, ny, nx), 0.15)
    d = _diag(3, (nx, ny, nz), rho, u, T, bc=(1, 0, 0))
    w = ny * nz * (nx - 1.5)
    _close(d["dux2"], a * a * w, a * a * w)
    _close(d["dil2"], a * a * w, a * a * w)
    _close(d["vort2"], b * b * w, b * b * w)
    _close(d["duy2"], 0.0, b * b * w)
    xs = np.arange(nx)
    _close(d["u2"], ny * nz * (a * a + b * b) * (xs ** 2).sum(), 1.0)


def test_nonfinite_and_nonpositive_counts():
    dims = (6, 5, 4)
    s = oracle.Sim(3, dims, gamma=GAMMA, Pr=0.7, mu=0.02)
    rho = np.ones((4, 5, 6))
    u = np.zeros((3, 4, 5, 6))
    T = np.full((4, 5, 6), 0.15)
    s.init(rho, u, T)
    f, g = s.get_pops()
    f[7, 1, 2, 3] = float("nan")
    f[:, 3, 4, 5] *= -1.0  # rho < 0 at one node (with rho E < 0 too, so T > 0 there)
    g[:, 3, 4, 5] *= -1.0
    g[:, 0, 0, 0] *= -1.0  # E < 0, so T < 0, at another
    s.set_pops(f, g)
    d = s.diagnostics()
    assert d["nonfinite"] == 1
    assert d["nonpositive"] == 2
    assert d["nodes"] == 120
