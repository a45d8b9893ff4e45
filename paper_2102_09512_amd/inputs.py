"""Seeded synthetic initial fields (rho, u, T) for the compressible LBM.

This module holds only input generators.  It contains none of the lattice
Boltzmann arithmetic: it builds macroscopic fields from the set-ups of the
paper's benchmarks (Sec. III) and from textbook gas dynamics, and hands the same
arrays to the GPU library and to the CPU oracle.

All fields are FP64 numpy arrays in lattice units (R = 1, delta_x = delta_t = 1):
rho and T of shape (nz, ny, nx), u of shape (D, nz, ny, nx); node x sits at
coordinate x (integer), node = x + nx*(y + ny*z).
"""
from __future__ import annotations

import math

import numpy as np


def _shape(D, dims):
    nx, ny = int(dims[0]), int(dims[1])
    nz = int(dims[2]) if D == 3 else 1
    return (nz, ny, nx)


# ---------------------------------------------------------------------------
# Sod shock tube (Sec. III.B)
# ---------------------------------------------------------------------------

def sod(nx=800, ny=4, T_left=0.0256, rho_left=1.0, rho_right=0.125, p_ratio=0.1):
    """Sod's Riemann problem: (rho, u, p) = (1, 0, T_l) for x < nx/2 and
    (0.125, 0, 0.1 T_l) otherwise (the paper's left/right pressure ratio 10 and
    density ratio 8, left pressure = left temperature T_l in lattice units)."""
    shape = (1, ny, nx)
    x = np.arange(nx)
    left = (x < nx // 2)[None, None, :]
    rho = np.where(left, rho_left, rho_right) * np.ones(shape)
    p = np.where(left, rho_left * T_left, p_ratio * rho_left * T_left) * np.ones(shape)
    T = p / rho
    u = np.zeros((2,) + shape)
    return rho, u, T


# ---------------------------------------------------------------------------
# Normal shock and isentropic vortex (Sec. III.C)
# ---------------------------------------------------------------------------

def rankine_hugoniot(M1, rho1, T1, gamma):
    """Downstream state of a stationary normal shock with upstream Mach M1
    (textbook normal-shock relations; p = rho T)."""
    u1 = M1 * math.sqrt(gamma * T1)
    p1 = rho1 * T1
    r = (gamma + 1.0) * M1 * M1 / ((gamma - 1.0) * M1 * M1 + 2.0)
    p2 = p1 * (1.0 + 2.0 * gamma / (gamma + 1.0) * (M1 * M1 - 1.0))
    rho2 = rho1 * r
    u2 = u1 / r
    return dict(rho1=rho1, u1=u1, T1=T1, p1=p1, rho2=rho2, u2=u2, p2=p2, T2=p2 / rho2)


def shock_vortex(nx=1024, ny=1024, Ma_a=1.2, Ma_v=0.25, r_v=32.0, x_s=None, x_v=None, y_v=None,
                 T_l=0.05, rho_l=1.0, gamma=1.4, vortex=True):
    """Standing normal shock at x_s with an isentropic vortex of radius r_v at
    (x_v, y_v).  Upstream (x < x_s) state (rho, T, u_x, u_y) = (rho_l, T_l,
    Ma_a sqrt(gamma T_l), 0), Rankine-Hugoniot downstream.  The vortex formula
    of Sec. III.C perturbs the local base state (rho_inf, P_inf, u_inf)."""
    if x_s is None:
        x_s = nx // 2
    if x_v is None:
        x_v = x_s - 2.0 * r_v
    if y_v is None:
        y_v = ny / 2.0
    rh = rankine_hugoniot(Ma_a, rho_l, T_l, gamma)
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    up = x < x_s
    rho_inf = np.where(up, rh["rho1"], rh["rho2"]) * np.ones((ny, nx))
    p_inf = np.where(up, rh["p1"], rh["p2"]) * np.ones((ny, nx))
    ux_inf = np.where(up, rh["u1"], rh["u2"]) * np.ones((ny, nx))
    rho, p, ux, uy = rho_inf, p_inf, ux_inf, np.zeros((ny, nx))
    if vortex:
        r2 = ((x - x_v) ** 2 + (y - y_v) ** 2) / (r_v * r_v)
        b = 1.0 - 0.5 * (gamma - 1.0) * Ma_v * Ma_v * np.exp(1.0 - r2)
        rho = rho_inf * b ** (1.0 / (gamma - 1.0))
        p = p_inf * b ** (gamma / (gamma - 1.0))
        a = math.sqrt(gamma * T_l) * Ma_v * np.exp(0.5 * (1.0 - r2)) / r_v
        ux = ux_inf + a * (y - y_v)
        uy = -a * (x - x_v)
    T = p / rho
    u = np.stack([ux, uy])[:, None, :, :]
    return rho[None], u, T[None], rh


def shock_vortex_viscosity(Re=800.0, r_v=32.0, T_l=0.05, rho_l=1.0, gamma=1.4):
    """mu from Re = rho_l c_{s,l} r_v / mu (Sec. III.C)."""
    return rho_l * math.sqrt(gamma * T_l) * r_v / Re


# ---------------------------------------------------------------------------
# Decaying isotropic turbulence (Sec. III.D)
# ---------------------------------------------------------------------------

def turbulence(D, n, seed, k0_index=4, Ma_t=0.5, T0=0.15, rho0=1.0, gamma=1.4):
    """Divergence-free random velocity with shell spectrum
    E(k) = A k^4 exp(-2 (k/k0)^2), k0 = k0_index * 2 pi / n, scaled so that
    sqrt(<u.u>) = Ma_t <c_s> with c_s = sqrt(gamma T0); rho = rho0, T = T0.

    Random-phase Fourier synthesis (the paper names kinematic simulation but
    does not describe it): every integer wave vector gets a random direction
    orthogonal to k (solenoidal) and a random phase, with an amplitude that
    makes each integer shell carry exactly the target spectrum; the spectrum is
    made Hermitian so the field is real.  Fields of different n are cubes
    (D = 3) or squares (D = 2)."""
    rng = np.random.default_rng(seed)
    shape = (n,) * D
    freqs = np.fft.fftfreq(n, d=1.0 / n)  # integer wave numbers
    K = np.stack(np.meshgrid(*([freqs] * D), indexing="ij"))  # K[a] = k_a over axes (a0, a1, ...)
    kmag = np.sqrt((K ** 2).sum(0))
    shell = np.rint(kmag).astype(np.int64)
    # random complex vectors, projected orthogonal to k, normalised to unit length
    a = rng.standard_normal((D,) + shape) + 1j * rng.standard_normal((D,) + shape)
    with np.errstate(invalid="ignore", divide="ignore"):
        kdota = (K * a).sum(0) / np.where(kmag > 0, kmag ** 2, 1.0)
    a = a - K * kdota
    norm = np.sqrt((np.abs(a) ** 2).sum(0))
    a = a / np.where(norm > 0, norm, 1.0)
    # shell amplitude: sum over a shell of |u_hat|^2 / 2 = E(shell) (up to a global factor)
    kk = np.arange(shell.max() + 1, dtype=np.float64)
    E = kk ** 4 * np.exp(-2.0 * (kk / k0_index) ** 2)
    count = np.bincount(shell.ravel(), minlength=kk.size).astype(np.float64)
    amp2 = np.where(count > 0, 2.0 * E / np.maximum(count, 1.0), 0.0)
    amp = np.sqrt(amp2[shell])
    nyq = np.zeros(shape, dtype=bool)
    for ax in range(D):
        nyq |= np.abs(K[ax]) == n // 2 if n % 2 == 0 else np.zeros(shape, dtype=bool)
    amp = np.where(nyq | (kmag == 0), 0.0, amp)
    uh = a * amp
    # Hermitian: keep a canonical half-space, mirror the rest as conj(u_hat(-k))
    idx = np.indices(shape)
    minus = tuple((-idx[ax]) % n for ax in range(D))
    canon = np.zeros(shape, dtype=bool)
    decided = np.zeros(shape, dtype=bool)
    for ax in range(D - 1, -1, -1):  # last axis first, then lexicographic tie-break
        pos = (K[ax] > 0) & ~decided
        negm = (K[ax] < 0) & ~decided
        canon |= pos
        decided |= pos | negm
    uh = np.where(canon[None], uh, np.conj(uh[(slice(None),) + minus]))
    u = np.fft.ifftn(uh, axes=tuple(range(1, D + 1))).real
    # array axes are (a0, a1, a2) = (x, y, z) in meshgrid 'ij' order; store as (z, y, x)
    u = np.stack([u[c] for c in range(D)])
    u = np.transpose(u, (0,) + tuple(range(D, 0, -1)))
    cs = math.sqrt(gamma * T0)
    scale = Ma_t * cs / math.sqrt((u ** 2).sum(0).mean())
    u = u * scale
    if D == 2:
        u = u[:, None, :, :]
    sh = u.shape[1:]
    rho = np.full(sh, rho0)
    T = np.full(sh, T0)
    return rho, np.ascontiguousarray(u), T


def turbulence_fine(n, seed, n_gen=64, k0_index=4, Ma_t=0.5, T0=0.15, rho0=1.0, gamma=1.4):
    """The field of turbulence(3, n_gen, seed, ...) sampled on an n^3 grid of
    the same box (n >= n_gen, n a multiple of 2): its Fourier modes are copied
    into an n^3 spectrum padded with zeros, so the fine field is the same
    band-limited function (modes |k_a| < n_gen / 2) on a finer grid, with the
    same u_rms.  The initial spectrum of turbulence() decays as exp(-2 (k/k0)^2),
    so nothing above n_gen / 2 is lost for k0 = 4, n_gen = 64.  Much faster
    than turbulence(3, n, ...) at n = 256, and one draw serves every grid."""
    from scipy import fft as sfft

    rho_g, u_g, T_g = turbulence(3, n_gen, seed, k0_index=k0_index, Ma_t=Ma_t, T0=T0, rho0=rho0, gamma=gamma)
    h = n_gen // 2
    u = np.empty((3, n, n, n))
    for a in range(3):
        uh = sfft.rfftn(u_g[a], workers=-1)  # (z, y, x//2+1) modes of the n_gen grid
        big = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
        big[:h, :h, :h] = uh[:h, :h, :h]
        big[:h, -h + 1:, :h] = uh[:h, -h + 1:, :h]
        big[-h + 1:, :h, :h] = uh[-h + 1:, :h, :h]
        big[-h + 1:, -h + 1:, :h] = uh[-h + 1:, -h + 1:, :h]
        u[a] = sfft.irfftn(big, s=(n, n, n), workers=-1) * (n / n_gen) ** 3
    return np.full((n, n, n), rho0), u, np.full((n, n, n), T0)


def turbulence_viscosity(n, k0_index=4, Ma_t=0.5, T0=0.15, rho0=1.0, gamma=1.4, Re_lambda=72.0, D=3):
    """mu_0 from Re_lambda = <rho> u_rms lambda / mu_0 (Sec. III.D) with
    u_rms = sqrt(<u.u>/D) and the Taylor microscale of the initial spectrum,
    lambda = sqrt(<u_x^2>/<(d_x u_x)^2>) = 2/k0 (the closed form for
    E ~ k^4 exp(-2 k^2/k0^2) in 3D)."""
    k0 = k0_index * 2.0 * math.pi / n
    u_rms = Ma_t * math.sqrt(gamma * T0) / math.sqrt(D)
    lam = 2.0 / k0
    return rho0 * u_rms * lam / Re_lambda


def turbulence_box2d(nx, ny, seed, k0_index=4, Ma_t=0.5, T0=0.15, rho0=1.0, gamma=1.4):
    """2-D solenoidal random velocity on a periodic nx x ny box with the shell
    spectrum E(k) = A k^4 exp(-2 (k/k0)^2) in physical wave number
    k = 2 pi (i/nx, j/ny): shells of width 2 pi / L and k0 = k0_index 2 pi / L
    with L = min(nx, ny) (the box fits k0_index wavelengths of the peak in
    both directions).  Same synthesis as turbulence(): random solenoidal
    directions and phases, exact per-shell energy, Hermitian, scaled so that
    sqrt(<u.u>) = Ma_t sqrt(gamma T0).  Returns rho, u, T with shapes
    (1, ny, nx) and (2, 1, ny, nx)."""
    rng = np.random.default_rng(seed)
    L = min(nx, ny)
    ix = np.fft.fftfreq(nx, d=1.0 / nx)
    iy = np.fft.fftfreq(ny, d=1.0 / ny)
    IX, IY = np.meshgrid(ix, iy, indexing="xy")  # arrays (ny, nx)
    KX, KY = IX / nx, IY / ny                      # wave number / (2 pi)
    kmag = np.sqrt(KX ** 2 + KY ** 2)
    shell = np.rint(kmag * L).astype(np.int64)      # in units of 2 pi / L
    a = rng.standard_normal((2, ny, nx)) + 1j * rng.standard_normal((2, ny, nx))
    with np.errstate(invalid="ignore", divide="ignore"):
        kdota = (KX * a[0] + KY * a[1]) / np.where(kmag > 0, kmag ** 2, 1.0)
    a = a - np.stack([KX, KY]) * kdota
    norm = np.sqrt((np.abs(a) ** 2).sum(0))
    a = a / np.where(norm > 0, norm, 1.0)
    kk = np.arange(shell.max() + 1, dtype=np.float64)
    E = kk ** 4 * np.exp(-2.0 * (kk / k0_index) ** 2)
    count = np.bincount(shell.ravel(), minlength=kk.size).astype(np.float64)
    amp = np.sqrt(np.where(count > 0, 2.0 * E / np.maximum(count, 1.0), 0.0)[shell])
    nyq = np.zeros((ny, nx), dtype=bool)
    if nx % 2 == 0:
        nyq |= np.abs(IX) == nx // 2
    if ny % 2 == 0:
        nyq |= np.abs(IY) == ny // 2
    amp = np.where(nyq | (kmag == 0), 0.0, amp)
    uh = a * amp
    # Hermitian: canonical half (j > 0, or j == 0 and i > 0), the rest mirrored
    jj, ii = np.indices((ny, nx))
    canon = (IY > 0) | ((IY == 0) & (IX > 0))
    mirror = uh[:, (-jj) % ny, (-ii) % nx]
    uh = np.where(canon[None], uh, np.conj(mirror))
    u = np.fft.ifft2(uh, axes=(1, 2)).real
    scale = Ma_t * math.sqrt(gamma * T0) / math.sqrt((u ** 2).sum(0).mean())
    u = (u * scale)[:, None, :, :]
    rho = np.full((1, ny, nx), rho0)
    T = np.full((1, ny, nx), T0)
    return rho, np.ascontiguousarray(u), T


def taylor_viscosity(u, rho0=1.0, Re_lambda=72.0):
    """mu_0 = <rho> u_rms lambda / Re_lambda with lambda measured on the field:
    lambda = sqrt(<u_x^2> / <(d_x u_x)^2>) (spectral x-derivative) and
    u_rms = sqrt(<u.u> / D).  u has shape (D, ..., nx) with x the last axis."""
    D = u.shape[0]
    nx = u.shape[-1]
    kx = 2.0 * math.pi * np.fft.fftfreq(nx, d=1.0)
    dudx = np.fft.ifft(1j * kx * np.fft.fft(u[0], axis=-1), axis=-1).real
    lam = math.sqrt((u[0] ** 2).mean() / (dudx ** 2).mean())
    u_rms = math.sqrt((u ** 2).sum(0).mean() / D)
    return rho0 * u_rms * lam / Re_lambda


def ensemble_2d(count=64, sizes=tuple(range(64, 513, 32)), Ma_range=(0.1, 0.6), T0=0.15, Re_lambda=72.0):
    """The batched workload: count independent periodic D2Q9 boxes; box s
    draws n_x, n_y (independently, uniformly from sizes) and Ma_t (uniformly
    in Ma_range) from seed s and carries turbulence_box2d(seed = s) with mu_0
    from its own measured Taylor microscale."""
    boxes = []
    for s in range(count):
        r = np.random.default_rng(s)
        nx, ny = int(r.choice(sizes)), int(r.choice(sizes))
        ma = float(r.uniform(*Ma_range))
        rho, u, T = turbulence_box2d(nx, ny, seed=s, Ma_t=ma, T0=T0)
        boxes.append(dict(seed=s, dims=(nx, ny), Ma_t=ma, fields=(rho, u, T),
                          mu=taylor_viscosity(u[:, 0], Re_lambda=Re_lambda)))
    return boxes


# ---------------------------------------------------------------------------
# Small test fields
# ---------------------------------------------------------------------------

def smooth_random(D, dims, seed, rho_amp=0.05, u_amp=0.05, T0=0.15, T_amp=0.02, modes=3):
    """Smooth periodic random fields built from a few low Fourier modes."""
    rng = np.random.default_rng(seed)
    shape = _shape(D, dims)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")

    def field(amp):
        f = np.zeros(shape)
        for _ in range(modes):
            kx, ky = rng.integers(0, 3, size=2)
            kz = rng.integers(0, 3) if D == 3 else 0
            ph = rng.uniform(0, 2 * math.pi)
            f += np.cos(2 * math.pi * (kx * x / nx + ky * y / ny + kz * z / nz) + ph)
        return amp * f / modes

    rho = 1.0 + field(rho_amp)
    T = T0 + field(T_amp)
    u = np.stack([field(u_amp) for _ in range(D)])
    return rho, u, T


def uniform(D, dims, rho=1.0, u=(0.0, 0.0, 0.0), T=0.15):
    shape = _shape(D, dims)
    return (np.full(shape, float(rho)), np.stack([np.full(shape, float(u[a])) for a in range(D)]),
            np.full(shape, float(T)))


def linear_wave(D, n, kind, eps=1e-4, rho0=1.0, T0=0.15, U=0.0, gamma=1.4, mode=1):
    """One-dimensional linear perturbations along x on a D-dimensional box of
    n x 1 (x 1) nodes: kind = 'acoustic' (isentropic pressure pulse,
    u = 0), 'shear' (u_y = eps sin(kx)) or 'entropy' (T' = eps cos(kx) at
    uniform p).  U adds a uniform background velocity along x."""
    dims = (n, 1, 1)
    rho, u, T = uniform(D, dims, rho0, (U, 0.0, 0.0), T0)
    x = np.arange(n, dtype=np.float64)
    k = 2.0 * math.pi * mode / n
    c = np.cos(k * x)[None, None, :]
    if kind == "acoustic":
        p0 = rho0 * T0
        dp = eps * p0 * c
        drho = dp / (gamma * T0)          # isentropic: drho = dp / c_s^2
        rho = rho + drho
        T = (p0 + dp) / rho
    elif kind == "shear":
        u[1] = u[1] + eps * np.sin(k * x)[None, None, :]
    elif kind == "entropy":
        p0 = rho0 * T0
        T = T0 * (1.0 + eps * c) * np.ones_like(T)
        rho = p0 / T
    else:
        raise ValueError(kind)
    return rho, u, T


class PopulationPerturbation:
    """Seeded smooth periodic perturbations of raw population arrays, one
    row (a population) at a time: row i is
        amp * cos(k_x x + a) cos(k_y y + b) cos(k_z z + c)
    with wave numbers of 1 to 3 periods per axis and phases drawn from
    (seed, i).  Added to the stored populations of an initial state it gives a
    generic non-equilibrium state for one-step parity checks; it is plain
    random input, independent of the method's arithmetic."""

    def __init__(self, dims, seed, amp):
        self.dims = tuple(int(d) for d in dims) + (1,) * (3 - len(dims))
        self.seed = int(seed)
        self.amp = float(amp)

    def row(self, i) -> np.ndarray:
        """Row i as a flat FP64 array in node order (x fastest)."""
        r = np.random.default_rng((self.seed, int(i)))
        nx, ny, nz = self.dims
        fac = []
        for n in (nx, ny, nz):
            k = 2.0 * math.pi * int(r.integers(1, 4)) / n
            fac.append(np.cos(k * np.arange(n) + r.uniform(0.0, 2.0 * math.pi)))
        out = self.amp * fac[2][:, None, None] * fac[1][None, :, None] * fac[0][None, None, :]
        return out.reshape(-1)
