"""Learned coarse-grid corrector for decaying compressible turbulence on D3Q27.

A coarse run of the method (n_c^3) is corrected every few steps by a small
3x3x3 convolutional network toward what a fine run of the same method
(n_f^3, n_f = 4 n_c) gives after a conservative box filter to the coarse grid.
The network reads rho, u and T and corrects u: trained on all five fields,
the density and temperature corrections lower the pointwise error of those
fields but damp the small-scale velocity, so the kinetic-energy spectrum gets
worse; the velocity-only corrector improves both.  Each correction is clipped
to two standard deviations of the training corrections: near the method's
stability limit (early acoustic transients at Ma_t ~ 0.5 on the coarse grid)
a rare large correction can otherwise tip a run over.
The corrector is not part of the paper; its training data come from the
method's own fine runs, and the fine run remains the reference for its error.

Time and viscosity follow the acoustic scaling of the lattice units: one
coarse step spans n_f / n_c fine steps, and the dynamic viscosity of a grid
of n nodes per side is set from the same Taylor-microscale Reynolds number,
so it grows in proportion to n (turbulence_viscosity).

Data (teacher forcing).  For each training seed the fine and the coarse run
advance together; every `every` coarse steps the coarse fields x and the
filtered fine fields t form one pair, and then the coarse moments are set to
t by re-equilibration (lbm_fields_set), which keeps the coarse populations'
non-equilibrium parts, exactly as a correction does when the network is used.

Evaluation.  The kinetic-energy spectrum E(k) of the velocity on the coarse grid
against that of the filtered fine run, as the RMS over shells 1..n_c/2 of
log(E / E_ref).  Plain runs on finer grids n_p are timed too; their fields are
taken to the coarse grid by the same box filter of width L / n_c
(overlap-weighted means of the conserved densities, which for an integer
ratio is the library's filter) before the spectrum is taken, and the plain
run at equal wall time is the most accurate one whose time does not exceed
the corrected run's.

Every operation on the fields runs in liblbm.so: stepping, moments, the box
filter, re-equilibration, the network's forward and backward passes and the
Adam step.  This module sequences those calls and owns device memory through
torch; the spectrum and the overlap remap between grids of different sizes
are host-side (numpy) diagnostics.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import inputs as I
from . import lbm

FIELDS = 5  # rho, u_x, u_y, u_z, T


@dataclass
class Workload:
    n_fine: int = 256
    n_coarse: int = 64
    k0_index: int = 4
    T0: float = 0.15
    gamma: float = 1.4
    Pr: float = 0.7
    visc_exp: float = 0.76
    Re_lambda: float = 72.0
    every: int = 4  # coarse steps between corrections
    windows: int = 32  # corrections per run
    channels: tuple = (5, 32, 32, 32, 3)  # reads rho, u, T; corrects u
    out_offset: int = 1  # output c corrects field out_offset + c
    limit: float = 2.0  # corrections clipped to 2 standard deviations of the training corrections

    @property
    def factor(self) -> int:
        return self.n_fine // self.n_coarse

    @property
    def coarse_steps(self) -> int:
        return self.every * self.windows

    @property
    def Cv(self) -> float:
        return 1.0 / (self.gamma - 1.0)


def training_seeds(count=32, Ma_range=(0.3, 0.6), first=0):
    """Seeds first..first+count-1 with turbulent Mach numbers drawn uniformly
    from Ma_range (one seeded draw per seed)."""
    seeds = list(range(first, first + count))
    return seeds, [float(np.random.default_rng(10_000 + s).uniform(*Ma_range)) for s in seeds]


def evaluation_seeds(count=4, Ma_range=(0.3, 0.6)):
    """Held-out seeds 1000.. with Ma_t spread evenly over the open range."""
    lo, hi = Ma_range
    return list(range(1000, 1000 + count)), [lo + (hi - lo) * (i + 0.5) / count for i in range(count)]


# ---- host diagnostics -------------------------------------------------------

def spectrum(u):
    """E(k) of a velocity field u[3][n][n][n]: shells k = rint(|k|) of
    sum |u_hat|^2 / 2 with u_hat the FFT divided by the node count."""
    n = u.shape[-1]
    uh = np.fft.fftn(u, axes=(1, 2, 3)) / n ** 3
    k = np.fft.fftfreq(n, d=1.0 / n)
    kk = np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2)
    shells = np.rint(kk).astype(np.int64).ravel()
    return np.bincount(shells, (0.5 * (np.abs(uh) ** 2).sum(0)).ravel())


def spectrum_error(E, E_ref, kmax):
    """RMS over shells 1..kmax of log(E / E_ref)."""
    r = np.log(E[1: kmax + 1] / E_ref[1: kmax + 1])
    return float(np.sqrt(np.mean(r * r)))


def overlap_matrix(n_out, n_in):
    """R[c][f] = |cell c of n_out cells  intersect  cell f of n_in cells| of a
    unit period, divided by the width of cell c (rows sum to 1)."""
    eo = np.arange(n_out + 1) / n_out
    ei = np.arange(n_in + 1) / n_in
    lo = np.maximum(eo[:-1, None], ei[None, :-1])
    hi = np.minimum(eo[1:, None], ei[None, 1:])
    return np.clip(hi - lo, 0.0, None) * n_out


def remap(rho, u, T, n_out, Cv):
    """Box filter of width 1/n_out of the piecewise-constant fields on a cubic
    grid: overlap-weighted means of rho, rho u and rho E (E = Cv T + |u|^2/2),
    then u and T from the means, so mass, momentum and energy are kept."""
    n_in = rho.shape[-1]
    if n_out == n_in:
        return rho.copy(), u.copy(), T.copy()
    R = overlap_matrix(n_out, n_in)

    def down(a):
        a = np.tensordot(a, R, axes=([2], [1]))  # x
        a = np.tensordot(a, R, axes=([1], [1])).transpose(0, 2, 1)  # y
        return np.tensordot(R, a, axes=([1], [0]))  # z

    E = Cv * T + 0.5 * (u * u).sum(0)
    r = down(rho)
    uc = np.stack([down(rho * u[a]) / r for a in range(3)])
    Ec = down(rho * E) / r
    return r, uc, (Ec - 0.5 * (uc * uc).sum(0)) / Cv


# ---- runs -------------------------------------------------------------------

def _torch():
    import torch

    return torch


def make_handle(w: Workload, n: int, Ma_t: float):
    mu = I.turbulence_viscosity(n, k0_index=w.k0_index, Ma_t=Ma_t, T0=w.T0, gamma=w.gamma, Re_lambda=w.Re_lambda)
    return lbm.lbm_create(lbm.LBM_D3Q27, (n, n, n), w.gamma, w.Pr, mu, precision=lbm.LBM_FP32_DEV,
                          visc_exponent=w.visc_exp, T_ref=w.T0)


def _device_fields(n):
    torch = _torch()
    return (torch.empty((n, n, n), dtype=torch.float64, device="cuda"),
            torch.empty((3, n, n, n), dtype=torch.float64, device="cuda"),
            torch.empty((n, n, n), dtype=torch.float64, device="cuda"))


def _healthy(h) -> bool:
    d = lbm.lbm_diagnostics(h)
    return d["nonfinite"] == 0 and d["nonpositive"] == 0


def generate_pairs(w: Workload, seeds, Ma_ts, log=print):
    """Training pairs (coarse fields x, filtered fine fields t), FP32 planes on
    the device: a tensor [pairs][2][5][n_c^3].  Seeds whose runs develop a bad
    node are skipped (and logged)."""
    torch = _torch()
    nc = w.n_coarse
    V = nc ** 3
    pairs = torch.empty((len(seeds) * w.windows, 2, FIELDS, V), dtype=torch.float32, device="cuda")
    fr, fu, fT = _device_fields(nc)
    cr, cu, cT = _device_fields(nc)
    used = 0
    for seed, Ma in zip(seeds, Ma_ts):
        t0 = time.perf_counter()
        rho, u, T = I.turbulence_fine(w.n_fine, seed, n_gen=nc, k0_index=w.k0_index, Ma_t=Ma, T0=w.T0,
                                      gamma=w.gamma)
        fine = make_handle(w, w.n_fine, Ma)
        coarse = make_handle(w, nc, Ma)
        ok = True
        try:
            lbm.lbm_init_fields(fine, rho, u, T)
            del rho, u, T
            lbm.lbm_filter_moments(fine, w.factor, fr, fu, fT)
            lbm.lbm_init_fields(coarse, fr, fu, fT)
            for k in range(w.windows):
                lbm.lbm_step(fine, w.every * w.factor)
                lbm.lbm_step(coarse, w.every)
                lbm.lbm_filter_moments(fine, w.factor, fr, fu, fT)
                lbm.lbm_moments(coarse, cr, cu, cT)
                lbm.lbm_nn_fields_to_planes(3, cr, cu, cT, pairs[used + k, 0])
                lbm.lbm_nn_fields_to_planes(3, fr, fu, fT, pairs[used + k, 1])
                lbm.lbm_fields_set(coarse, fr, fu, fT)  # refuses a bad filtered field
            ok = _healthy(fine) and _healthy(coarse)
        except lbm.LbmError:  # the fine run left the method's stable range
            ok = False
        finally:
            lbm.lbm_destroy(fine)
            lbm.lbm_destroy(coarse)
        torch.cuda.synchronize()
        log(f"[data] seed {seed} Ma_t {Ma:.3f}: {'ok' if ok else 'bad node, skipped'} "
            f"({time.perf_counter() - t0:.1f} s)")
        if ok:
            used += w.windows
    return pairs[:used]


def scaling_from(pairs, out_fields, sample=64, seed=0):
    """Per-field mean and std of the inputs and std of the corrections t - x of
    the corrected fields (a slice), from a host copy of up to `sample` pairs."""
    idx = np.random.default_rng(seed).choice(pairs.shape[0], min(sample, pairs.shape[0]), replace=False)
    h = pairs[np.sort(idx)].cpu().numpy().astype(np.float64)
    x, t = h[:, 0], h[:, 1]
    mean = x.mean(axis=(0, 2))
    std = np.maximum(x.std(axis=(0, 2)), 1e-12)
    out = np.maximum((t - x)[:, out_fields].std(axis=(0, 2)), 1e-12)
    return mean, std, out


def out_fields(w: Workload):
    return slice(w.out_offset, w.out_offset + w.channels[-1])


def no_correction_loss(w: Workload, pairs, out_std):
    """The library loss of a network that outputs zero: mean of ((x - t) / s)^2
    over the corrected fields."""
    h = pairs.cpu().numpy().astype(np.float64)
    d = (h[:, 0] - h[:, 1])[:, out_fields(w)] / out_std[None, :, None]
    return float(np.mean(d * d))


def initial_params(channels, seed=0, last_gain=0.1):
    """He-normal weights (the last layer scaled by last_gain, so the first
    corrections are small), zero biases; the library's parameter layout."""
    r = np.random.default_rng(seed)
    out = []
    L = len(channels) - 1
    for l in range(L):
        ci, co = channels[l], channels[l + 1]
        g = last_gain if l == L - 1 else 1.0
        out.append(r.normal(0.0, g * math.sqrt(2.0 / (27 * ci)), 27 * ci * co))
        out.append(np.zeros(co))
    return np.concatenate(out).astype(np.float32)


@dataclass
class TrainResult:
    net: int
    scaling: tuple
    history: list = field(default_factory=list)  # mean loss per epoch
    seconds: float = 0.0


def train(w: Workload, pairs, epochs=20, lr=1e-3, batch=4, seed=0, log=print) -> TrainResult:
    """Adam on the library's loss (mean squared error of the corrected field in
    units of the correction std), cosine learning-rate decay to lr / 20."""
    torch = _torch()
    nc = w.n_coarse
    net = lbm.lbm_nn_create(list(w.channels), (nc, nc, nc))
    try:
        lbm.lbm_nn_set_params(net, initial_params(w.channels, seed))
        mean, std, out = scaling_from(pairs, out_fields(w), seed=seed)
        lbm.lbm_nn_set_scaling(net, mean, std, out)
        lbm.lbm_nn_set_output_offset(net, w.out_offset)
        lbm.lbm_nn_set_correction_limit(net, w.limit)
        rng = np.random.default_rng(seed)
        P = pairs.shape[0]
        steps_per_epoch = (P + batch - 1) // batch
        total = epochs * steps_per_epoch
        step = 0
        hist = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lbm.lbm_nn_take_loss(net)  # start the device-side loss sum from zero
        for ep in range(epochs):
            perm = rng.permutation(P)
            for b in range(0, P, batch):
                mb = perm[b: b + batch]
                lbm.lbm_nn_zero_grad(net)
                for i in mb:  # asynchronous: the host does not wait for the GPU within an epoch
                    lbm.lbm_nn_loss_backward(net, pairs[i, 0], pairs[i, 1], sync=False)
                step += 1
                rate = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * (step - 1) / max(total - 1, 1))))
                lbm.lbm_nn_adam_step(net, rate, 0.9, 0.999, 1e-8, 1.0 / len(mb), step)
            s, count = lbm.lbm_nn_take_loss(net)
            assert count == P
            hist.append(s / P)
            log(f"[train] epoch {ep + 1}/{epochs}: loss {hist[-1]:.4f} ({time.perf_counter() - t0:.1f} s)")
        torch.cuda.synchronize()
        return TrainResult(net, (mean, std, out), hist, time.perf_counter() - t0)
    except Exception:
        lbm.lbm_nn_destroy(net)
        raise


def validation_loss(net, pairs):
    """Mean library loss over pairs, and the loss of no correction at all
    (the network replaced by zero), which the trained loss should undercut."""
    s = 0.0
    for i in range(pairs.shape[0]):
        lbm.lbm_nn_zero_grad(net)
        s += lbm.lbm_nn_loss_backward(net, pairs[i, 0], pairs[i, 1])
    return s / pairs.shape[0]


def run(w: Workload, h, steps, net=None, every=None):
    """Advances h by `steps` steps; with a network, applies the correction
    after every `every` steps.  Returns the device time in seconds (host clock
    around synchronised work, launch overheads included)."""
    torch = _torch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if net is None:
        lbm.lbm_step(h, steps)
    else:
        done = 0
        while done < steps:
            k = min(every, steps - done)
            lbm.lbm_step(h, k)
            done += k
            if k == every:
                lbm.lbm_nn_correct(net, h)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def _host_fields(h, n):
    rho, u, T = np.zeros((n, n, n)), np.zeros((3, n, n, n)), np.zeros((n, n, n))
    lbm.lbm_moments(h, rho, u, T)
    return rho, u, T


def _timed_final(w, n, Ma, init, steps, net=None, every=None, reps=3):
    """Fields after `steps` steps from init on an n^3 grid, and the best of
    `reps` timed runs (the first run also warms the library's buffers)."""
    best, fields, ok = float("inf"), None, True
    h = make_handle(w, n, Ma)
    try:
        for _ in range(reps):
            lbm.lbm_init_fields(h, *init)
            best = min(best, run(w, h, steps, net, every))
        ok = _healthy(h)
        fields = _host_fields(h, n)
    except lbm.LbmError:  # a correction met a bad node: the run left the stable range
        ok = False
        fields = tuple(np.full(s, np.nan) for s in ((n,) * 3, (3,) + (n,) * 3, (n,) * 3))
    finally:
        lbm.lbm_destroy(h)
    return fields, best, ok


def _error(u, E_ref, kmax, ok):
    return spectrum_error(spectrum(u), E_ref, kmax) if ok else float("inf")


def evaluate(w: Workload, net, seeds, Ma_ts, grids=None, log=print):
    """Per held-out seed: spectrum errors of the plain coarse run, the
    corrected coarse run and the plain runs on finer grids, each against the
    filtered fine run at the same physical time, with their wall times; the
    equal-time plain run is the most accurate of the plain runs whose time
    does not exceed the corrected run's."""
    nc, kmax = w.n_coarse, w.n_coarse // 2
    if grids is None:
        grids = list(range(nc, 2 * nc + 1, 8))
    rows = []
    for seed, Ma in zip(seeds, Ma_ts):
        t0 = time.perf_counter()
        rho, u, T = I.turbulence_fine(w.n_fine, seed, n_gen=nc, k0_index=w.k0_index, Ma_t=Ma, T0=w.T0,
                                      gamma=w.gamma)
        fine = make_handle(w, w.n_fine, Ma)
        try:
            lbm.lbm_init_fields(fine, rho, u, T)
            init_c = (np.zeros((nc,) * 3), np.zeros((3,) + (nc,) * 3), np.zeros((nc,) * 3))
            lbm.lbm_filter_moments(fine, w.factor, *init_c)
            lbm.lbm_step(fine, w.coarse_steps * w.factor)
            ref = (np.zeros((nc,) * 3), np.zeros((3,) + (nc,) * 3), np.zeros((nc,) * 3))
            lbm.lbm_filter_moments(fine, w.factor, *ref)
            fine_ok = _healthy(fine)
        finally:
            lbm.lbm_destroy(fine)
        if not fine_ok:
            log(f"[eval] seed {seed} Ma_t {Ma:.3f}: the fine run left the stable range; seed skipped")
            continue
        E_ref = spectrum(ref[1])
        row = {"seed": seed, "Ma_t": Ma, "fine_ok": fine_ok}
        (_, u_l, _), t_l, ok_l = _timed_final(w, nc, Ma, init_c, w.coarse_steps, net, w.every)
        row["learned"] = {"error": _error(u_l, E_ref, kmax, ok_l), "seconds": t_l, "ok": ok_l}
        plain = []
        for n in grids:
            steps = w.coarse_steps * n // nc
            init = init_c if n == nc else remap(rho, u, T, n, w.Cv)
            (r_p, u_p, T_p), t_p, ok_p = _timed_final(w, n, Ma, init, steps)
            if n != nc and ok_p:
                r_p, u_p, T_p = remap(r_p, u_p, T_p, nc, w.Cv)
            plain.append({"n": n, "steps": steps, "error": _error(u_p, E_ref, kmax, ok_p), "seconds": t_p,
                          "ok": ok_p})
        row["plain"] = plain
        fit = [p for p in plain if p["seconds"] <= t_l]
        row["plain_coarse"] = plain[0]
        # the best plain run the corrected run's wall time allows (the coarse
        # grid itself when nothing finer fits)
        row["plain_equal_time"] = min(fit, key=lambda p: p["error"]) if fit else plain[0]
        rows.append(row)
        log(f"[eval] seed {seed} Ma_t {Ma:.3f}: learned {row['learned']['error']:.4f} in "
            f"{1e3 * t_l:.1f} ms; plain {nc}^3 {plain[0]['error']:.4f} in {1e3 * plain[0]['seconds']:.1f} ms; "
            f"plain at equal time n={row['plain_equal_time']['n']} {row['plain_equal_time']['error']:.4f} in "
            f"{1e3 * row['plain_equal_time']['seconds']:.1f} ms ({time.perf_counter() - t0:.1f} s)")
        del rho, u, T
    return rows


def summarize(rows):
    """Means over seeds of the three errors, and how many seeds the corrected
    run beat the equal-time plain run on.  Seeds on which the plain coarse run
    itself leaves the stable range (nothing to compare with) are counted
    apart; a corrected run that fails where the plain one does not counts
    with an infinite error."""
    kept = [r for r in rows if math.isfinite(r["plain_coarse"]["error"])]
    m = lambda key: float(np.mean([r[key]["error"] for r in kept])) if kept else float("nan")
    return {
        "learned": m("learned"),
        "plain_coarse": m("plain_coarse"),
        "plain_equal_time": m("plain_equal_time"),
        "equal_time_grids": [r["plain_equal_time"]["n"] for r in kept],
        "wins_equal_time": int(sum(r["learned"]["error"] < r["plain_equal_time"]["error"] for r in kept)),
        "seeds": len(kept),
        "seeds_plain_coarse_unstable": len(rows) - len(kept),
    }
