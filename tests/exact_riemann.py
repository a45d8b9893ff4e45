"""Exact solution of the Riemann problem for the 1-D Euler equations of an
ideal gas (the textbook method: star pressure from the shock/rarefaction wave
curves by Newton iteration, then self-similar sampling in x/t).

Independent of the lattice Boltzmann code; used to pin the oracle on Sod's
shock tube (Sec. III.B).  Pressure p = rho T (R = 1).
"""
from __future__ import annotations

import math

import numpy as np


def _wave_curve(p, rho_k, p_k, c_k, gamma):
    """Velocity jump f_K(p) across the left/right wave and its derivative."""
    if p > p_k:  # shock
        A = 2.0 / ((gamma + 1.0) * rho_k)
        B = (gamma - 1.0) / (gamma + 1.0) * p_k
        sq = math.sqrt(A / (p + B))
        f = (p - p_k) * sq
        df = sq * (1.0 - 0.5 * (p - p_k) / (B + p))
    else:  # rarefaction
        e = (gamma - 1.0) / (2.0 * gamma)
        f = 2.0 * c_k / (gamma - 1.0) * ((p / p_k) ** e - 1.0)
        df = 1.0 / (rho_k * c_k) * (p / p_k) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(rho_l, u_l, p_l, rho_r, u_r, p_r, gamma):
    c_l = math.sqrt(gamma * p_l / rho_l)
    c_r = math.sqrt(gamma * p_r / rho_r)
    p = 0.5 * (p_l + p_r)
    for _ in range(100):
        fl, dfl = _wave_curve(p, rho_l, p_l, c_l, gamma)
        fr, dfr = _wave_curve(p, rho_r, p_r, c_r, gamma)
        dp = (fl + fr + (u_r - u_l)) / (dfl + dfr)
        p_new = max(p - dp, 1e-14 * p)
        if abs(p_new - p) <= 1e-15 * (p_new + p):
            p = p_new
            break
        p = p_new
    fl, _ = _wave_curve(p, rho_l, p_l, c_l, gamma)
    fr, _ = _wave_curve(p, rho_r, p_r, c_r, gamma)
    u = 0.5 * (u_l + u_r) + 0.5 * (fr - fl)

    def star_rho(rho_k, p_k):
        if p > p_k:
            g = (gamma - 1.0) / (gamma + 1.0)
            return rho_k * (p / p_k + g) / (g * p / p_k + 1.0)
        return rho_k * (p / p_k) ** (1.0 / gamma)

    return dict(p=p, u=u, rho_l=star_rho(rho_l, p_l), rho_r=star_rho(rho_r, p_r), c_l=c_l, c_r=c_r)


def sample(xi, rho_l, u_l, p_l, rho_r, u_r, p_r, gamma):
    """(rho, u, p) at similarity coordinate xi = (x - x0)/t (array)."""
    s = star_state(rho_l, u_l, p_l, rho_r, u_r, p_r, gamma)
    ps, us = s["p"], s["u"]
    c_l, c_r = s["c_l"], s["c_r"]
    g1 = (gamma - 1.0) / (gamma + 1.0)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for k, x in np.ndenumerate(xi):
        if x <= us:  # left of the contact
            if ps > p_l:  # left shock
                S = u_l - c_l * math.sqrt((gamma + 1) / (2 * gamma) * ps / p_l + (gamma - 1) / (2 * gamma))
                st = (rho_l, u_l, p_l) if x <= S else (s["rho_l"], us, ps)
            else:  # left rarefaction
                c_star = c_l * (ps / p_l) ** ((gamma - 1) / (2 * gamma))
                head, tail = u_l - c_l, us - c_star
                if x <= head:
                    st = (rho_l, u_l, p_l)
                elif x >= tail:
                    st = (s["rho_l"], us, ps)
                else:
                    fac = 2.0 / (gamma + 1) + g1 / c_l * (u_l - x)
                    st = (rho_l * fac ** (2 / (gamma - 1)), 2 / (gamma + 1) * (c_l + (gamma - 1) / 2 * u_l + x),
                          p_l * fac ** (2 * gamma / (gamma - 1)))
        else:
            if ps > p_r:  # right shock
                S = u_r + c_r * math.sqrt((gamma + 1) / (2 * gamma) * ps / p_r + (gamma - 1) / (2 * gamma))
                st = (rho_r, u_r, p_r) if x >= S else (s["rho_r"], us, ps)
            else:
                c_star = c_r * (ps / p_r) ** ((gamma - 1) / (2 * gamma))
                head, tail = u_r + c_r, us + c_star
                if x >= head:
                    st = (rho_r, u_r, p_r)
                elif x <= tail:
                    st = (s["rho_r"], us, ps)
                else:
                    fac = 2.0 / (gamma + 1) - g1 / c_r * (u_r - x)
                    st = (rho_r * fac ** (2 / (gamma - 1)), 2 / (gamma + 1) * (-c_r + (gamma - 1) / 2 * u_r + x),
                          p_r * fac ** (2 * gamma / (gamma - 1)))
        rho[k], u[k], p[k] = st
    return rho, u, p


def wave_speeds(rho_l, u_l, p_l, rho_r, u_r, p_r, gamma):
    """Left rarefaction head/tail, contact and right shock speeds (Sod-type problems)."""
    s = star_state(rho_l, u_l, p_l, rho_r, u_r, p_r, gamma)
    ps, us, c_l, c_r = s["p"], s["u"], s["c_l"], s["c_r"]
    c_star = c_l * (ps / p_l) ** ((gamma - 1) / (2 * gamma))
    S_r = u_r + c_r * math.sqrt((gamma + 1) / (2 * gamma) * ps / p_r + (gamma - 1) / (2 * gamma))
    return dict(head=u_l - c_l, tail=us - c_star, contact=us, shock=S_r, star=s)
