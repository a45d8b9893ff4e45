"""Pins of the seeded initial-condition generators (Sec. III.C, III.D)."""
import math

import numpy as np
import pytest

from paper_2102_09512_amd import inputs as I


def _spectral(u, D):
    """FFT over the spatial axes of a (D, z, y, x) or (D, 1, y, x) field; wave
    numbers per array axis."""
    if D == 2:
        u = u[:, 0]
    n = u.shape[-1]
    uh = np.fft.fftn(u, axes=tuple(range(1, D + 1))) / n ** D
    k = np.fft.fftfreq(n, d=1.0 / n)
    K = np.meshgrid(*([k] * D), indexing="ij")
    # array axes are (z, y, x) / (y, x): component a (x, y, z) varies along array axis D-1-a
    Ka = [K[D - 1 - a] for a in range(D)]
    return uh, Ka


@pytest.mark.parametrize("D,n", [(3, 32), (2, 64)])
def test_turbulence_is_real_solenoidal_and_scaled(D, n):
    Ma_t, T0, gamma = 0.5, 0.15, 1.4
    rho, u, T = I.turbulence(D, n, seed=0, Ma_t=Ma_t, T0=T0, gamma=gamma)
    assert np.all(rho == 1.0) and np.all(T == T0)
    assert abs(math.sqrt((u ** 2).sum(0).mean()) / (Ma_t * math.sqrt(gamma * T0)) - 1) < 1e-12
    uh, Ka = _spectral(u, D)
    div = sum(Ka[a] * uh[a] for a in range(D))
    assert np.abs(div).max() <= 1e-12 * np.abs(uh).max()
    # deterministic in the seed, different across seeds
    assert np.array_equal(I.turbulence(D, n, seed=0)[1], I.turbulence(D, n, seed=0)[1])
    assert not np.allclose(I.turbulence(D, n, seed=1)[1], u)


def test_turbulence_shell_spectrum_and_length_scales():
    """E(k) ~ k^4 exp(-2 (k/k0)^2) shell by shell; Taylor microscale
    lambda = sqrt(<u_x^2>/<(d_x u_x)^2>) = 2/k0 and integral scale
    L_I = 3 pi int(E/k) / (4 int E) = sqrt(2 pi)/k0 (Sec. III.D) within the
    discreteness of integer shells."""
    n, k0i = 64, 4
    rho, u, T = I.turbulence(3, n, seed=3, k0_index=k0i)
    uh, Ka = _spectral(u, 3)
    kmag = np.sqrt(sum(k * k for k in Ka))
    shell = np.rint(kmag).astype(int)
    E = np.bincount(shell.ravel(), weights=0.5 * (np.abs(uh) ** 2).sum(0).ravel())
    kk = np.arange(E.size)
    target = kk ** 4 * np.exp(-2.0 * (kk / k0i) ** 2)
    sel = (kk >= 1) & (kk <= 12)
    ratio = E[sel] / target[sel]
    assert np.max(np.abs(ratio / ratio.mean() - 1)) < 1e-10
    k0 = k0i * 2 * math.pi / n
    dudx = np.fft.ifftn(1j * Ka[0] * 2 * math.pi / n * uh[0] * n ** 3).real
    lam = math.sqrt((u[0] ** 2).mean() / (dudx ** 2).mean())
    assert abs(lam / (2.0 / k0) - 1) < 0.03
    kw = kk[1:] * 2 * math.pi / n
    LI = 3 * math.pi * np.sum(E[1:] / kw) / (4 * np.sum(E[1:]))
    assert abs(LI / (math.sqrt(2 * math.pi) / k0) - 1) < 0.03


def test_turbulence_viscosity_from_taylor_reynolds():
    """Re_lambda = <rho> u_rms lambda / mu_0 with lambda = 2/k0: the 256^3 case
    gives mu_0 = 0.03743 (Ma_t 0.5, T0 0.15, Re_lambda 72)."""
    mu0 = I.turbulence_viscosity(256, Ma_t=0.5, T0=0.15, Re_lambda=72.0)
    u_rms = 0.5 * math.sqrt(1.4 * 0.15) / math.sqrt(3)
    assert abs(mu0 - u_rms * (2 / (4 * 2 * math.pi / 256)) / 72.0) < 1e-15
    assert abs(mu0 - 0.03743) < 5e-5


def test_shock_vortex_states():
    """Sec. III.C: upstream (1, 0.05, Ma_a sqrt(gamma T_l), 0), Rankine-Hugoniot
    downstream; the vortex is isentropic (p / rho^gamma of the base state)."""
    g = 1.4
    rho, u, T, rh = I.shock_vortex(256, 128, r_v=16.0, x_s=128)
    assert abs(rh["u1"] - 1.2 * math.sqrt(g * 0.05)) < 1e-15
    # RH: mass, momentum, energy flux continuity
    m1, m2 = rh["rho1"] * rh["u1"], rh["rho2"] * rh["u2"]
    assert abs(m1 - m2) < 1e-14
    assert abs(m1 * rh["u1"] + rh["p1"] - (m2 * rh["u2"] + rh["p2"])) < 1e-14
    h = lambda p, r, v: g / (g - 1) * p / r + 0.5 * v * v
    assert abs(h(rh["p1"], rh["rho1"], rh["u1"]) - h(rh["p2"], rh["rho2"], rh["u2"])) < 1e-14
    p = rho * T
    up = np.zeros_like(rho, dtype=bool)
    up[..., :128] = True
    assert np.allclose((p / rho ** g)[up], rh["p1"] / rh["rho1"] ** g, rtol=1e-12)
    assert np.allclose((p / rho ** g)[~up], rh["p2"] / rh["rho2"] ** g, rtol=1e-12)
    # far from the vortex the base state is recovered
    assert abs(rho[0, 0, 5] - rh["rho1"]) < 1e-6 and abs(rho[0, 0, 250] - rh["rho2"]) < 1e-6


@pytest.mark.parametrize("nx,ny", [(64, 96), (160, 64), (128, 128)])
def test_box2d_turbulence_is_real_solenoidal_and_scaled(nx, ny):
    rho, u, T = I.turbulence_box2d(nx, ny, seed=3, Ma_t=0.4, T0=0.15)
    assert u.shape == (2, 1, ny, nx) and rho.shape == (1, ny, nx)
    ux, uy = u[0, 0], u[1, 0]
    # spectral divergence of the real field (physical wave numbers per axis)
    kx = 2 * np.pi * np.fft.fftfreq(nx)
    ky = 2 * np.pi * np.fft.fftfreq(ny)
    div = np.fft.ifft2(1j * kx[None, :] * np.fft.fft2(ux) + 1j * ky[:, None] * np.fft.fft2(uy)).real
    assert np.abs(div).max() < 1e-12 * np.abs(u).max()
    assert np.sqrt((u ** 2).sum(0).mean()) == pytest.approx(0.4 * np.sqrt(1.4 * 0.15), rel=1e-12)
    # the energy peaks at the shell k0 = 4 (units of 2 pi / min(nx, ny))
    L = min(nx, ny)
    KX, KY = np.meshgrid(np.fft.fftfreq(nx, 1 / nx) / nx, np.fft.fftfreq(ny, 1 / ny) / ny, indexing="xy")
    shell = np.rint(np.sqrt(KX ** 2 + KY ** 2) * L).astype(int)
    e = np.bincount(shell.ravel(), (np.abs(np.fft.fft2(ux)) ** 2 + np.abs(np.fft.fft2(uy)) ** 2).ravel())
    assert 3 <= int(np.argmax(e)) <= 4  # continuous maximum of k^4 exp(-2 k^2/16) is at k = 4


def test_taylor_viscosity_matches_closed_form_on_a_cube():
    """On the 3-D cube generator the measured microscale gives the closed-form
    mu_0 of turbulence_viscosity (lambda = 2/k0) to within the discreteness of
    the shells."""
    n = 64
    rho, u, T = I.turbulence(3, n, seed=1, Ma_t=0.5, T0=0.15)
    mu_meas = I.taylor_viscosity(u, Re_lambda=72.0)
    mu_closed = I.turbulence_viscosity(n, Ma_t=0.5, T0=0.15, Re_lambda=72.0)
    assert mu_meas == pytest.approx(mu_closed, rel=0.02)


def test_ensemble_2d_sizes_and_parameters():
    boxes = I.ensemble_2d(count=8)
    assert [b["seed"] for b in boxes] == list(range(8))
    for b in boxes:
        nx, ny = b["dims"]
        assert nx in range(64, 513, 32) and ny in range(64, 513, 32)
        assert 0.1 <= b["Ma_t"] <= 0.6 and b["mu"] > 0
        assert b["fields"][1].shape == (2, 1, ny, nx)
    again = I.ensemble_2d(count=2)
    assert np.array_equal(again[1]["fields"][1], boxes[1]["fields"][1])
