"""Pins of the oracle's nodal functions against what the paper fixes
independently of the oracle's own code: Maxwell-Boltzmann moments (by
Gauss-Hermite quadrature of the Maxwellian), the operator definition of the
energy moments (by symbolic differentiation), the printed closed forms of the
fluxes and of the anomaly, conservation, and the transport-coefficient maps.
"""
import itertools
import math

import numpy as np
import pytest
import sympy as sp

RNG = np.random.default_rng(20210218)


def _states(D, k=4):
    out = []
    for _ in range(k):
        rho = RNG.uniform(0.3, 2.0)
        u = RNG.uniform(-0.4, 0.4, size=D)
        T = RNG.uniform(0.05, 0.5)
        out.append((rho, u, T))
    return out


def _moment(c, w, l):
    """sum_i prod_a c_ia^l_a w_i."""
    return float(np.sum(np.prod(c[:, : len(l)] ** np.array(l), axis=1) * w))


def _maxwell_moment(D, rho, u, T, l, energy=False):
    """rho (2 pi T)^{-D/2} int c^l exp(-(c-u)^2 / 2T) [c^2/2] dc by tensor-product
    Gauss-Hermite quadrature (exact for these polynomial degrees); Eq. (22)
    and Eq. (32)."""
    x, w = np.polynomial.hermite_e.hermegauss(12)
    w = w / math.sqrt(2.0 * math.pi)
    grids = np.meshgrid(*([x] * D), indexing="ij")
    wt = np.ones_like(grids[0])
    for a in range(D):
        wt = wt * np.meshgrid(*([w] * D), indexing="ij")[a]
    cs = [u[a] + math.sqrt(T) * grids[a] for a in range(D)]
    integrand = np.ones_like(grids[0])
    for a in range(D):
        integrand = integrand * cs[a] ** l[a]
    if energy:
        integrand = integrand * 0.5 * sum(ca * ca for ca in cs)
    return rho * float(np.sum(wt * integrand))


def test_velocity_numbering(oracle_mod):
    for D in (2, 3):
        c = oracle_mod.velocities(D)
        Q = oracle_mod.Q(D)
        assert c.shape == (Q, 3)
        assert len({tuple(v) for v in c}) == Q
        # opposite of i is Q-1-i, rest population (Q-1)/2
        assert np.array_equal(c[::-1], -c)
        assert np.all(c[(Q - 1) // 2] == 0)


@pytest.mark.parametrize("D", [2, 3])
def test_feq_moments_are_maxwell_boltzmann(oracle_mod, D):
    """Eq. (21): all moments with exponents in {0,1,2} equal the MB ones."""
    c = oracle_mod.velocities(D)
    for rho, u, T in _states(D):
        f = oracle_mod.feq(D, rho, u, T)
        for l in itertools.product(range(3), repeat=D):
            ref = _maxwell_moment(D, rho, u, T, l)
            assert abs(_moment(c, f, l) - ref) <= 1e-13 * max(1.0, abs(ref)), (l, ref)


@pytest.mark.parametrize("D", [2, 3])
def test_feq_third_moment_anomaly(oracle_mod, D):
    """Eqs. (24), (27), (29): only the diagonal third moments deviate from MB,
    by rho u_a (1 - 3T) - rho u_a^3; the mixed ones (e.g. xxy) are MB."""
    c = oracle_mod.velocities(D)
    for rho, u, T in _states(D):
        f = oracle_mod.feq(D, rho, u, T)
        for a in range(D):
            l = [0] * D
            l[a] = 3
            dev = _moment(c, f, l) - _maxwell_moment(D, rho, u, T, l)
            assert abs(dev - oracle_mod.anomaly(rho, u[a], T)) <= 1e-13
            # and the printed closed form itself
            assert abs(dev - (rho * u[a] * (1 - 3 * T) - rho * u[a] ** 3)) <= 1e-13
        l = [2, 1] + [0] * (D - 2)
        assert abs(_moment(c, f, l) - _maxwell_moment(D, rho, u, T, l)) <= 1e-13


@pytest.mark.parametrize("D", [2, 3])
def test_fex_pressure_tensor(oracle_mod, D):
    """Eq. (31): P^ex = P^eq + (2 - omega)/(2 omega) div Qt, diagonal only;
    density and momentum as f^eq (Eqs. (3)-(4))."""
    c = oracle_mod.velocities(D)
    for rho, u, T in _states(D):
        om = RNG.uniform(0.6, 1.9)
        d = RNG.uniform(-0.05, 0.05, size=D)
        f = oracle_mod.fex(D, rho, u, T, om, d)
        assert abs(f.sum() - rho) <= 1e-14 * rho
        for a in range(D):
            e = [0] * D
            e[a] = 1
            assert abs(_moment(c, f, e) - rho * u[a]) <= 1e-14
            e[a] = 2
            ref = rho * (T + u[a] ** 2) + (2 - om) / (2 * om) * d[a]
            assert abs(_moment(c, f, e) - ref) <= 1e-14
            for b in range(a + 1, D):
                e = [0] * D
                e[a] = e[b] = 1
                assert abs(_moment(c, f, e) - rho * u[a] * u[b]) <= 1e-14


def _operator_moments_symbolic(D):
    """rho O_x^l O_y^m O_z^n E with O_a A = T dA/du_a + u_a A (Eq. (33)) and
    E = C_v T + |u|^2/2, by symbolic differentiation."""
    us = sp.symbols("ux uy uz")[:D]
    T, Cv = sp.symbols("T Cv", positive=True)
    E = Cv * T + sum(x * x for x in us) / 2

    def O(a, A):
        return sp.expand(T * sp.diff(A, us[a]) + us[a] * A)

    table = {}
    for l in itertools.product(range(3), repeat=D):
        A = E
        for a in range(D):
            for _ in range(l[a]):
                A = O(a, A)
        table[l] = sp.lambdify((us, T, Cv), A, "math")
    return table


@pytest.mark.parametrize("D", [2, 3])
def test_geq_moments_by_operator_definition(oracle_mod, D):
    """Eq. (43): sum c^l c^m c^n g^eq = rho O^l O^m O^n E for exponents <= 2."""
    c = oracle_mod.velocities(D)
    table = _operator_moments_symbolic(D)
    for rho, u, T in _states(D):
        Cv = RNG.uniform(1.2, 3.5)
        g = oracle_mod.geq(D, rho, u, T, Cv)
        for l, fn in table.items():
            ref = rho * fn(list(u), T, Cv)
            assert abs(_moment(c, g, l) - ref) <= 1e-13 * max(1.0, abs(ref)), l


@pytest.mark.parametrize("D", [2, 3])
def test_geq_monatomic_is_maxwell_energy_moment(oracle_mod, D):
    """Eqs. (32), (34)-(35): for the monatomic gas (C_v = D/2) the energy
    moments are those of c^2/2 under the Maxwellian."""
    c = oracle_mod.velocities(D)
    for rho, u, T in _states(D):
        g = oracle_mod.geq(D, rho, u, T, D / 2.0)
        for l in itertools.product(range(3), repeat=D):
            ref = _maxwell_moment(D, rho, u, T, l, energy=True)
            assert abs(_moment(c, g, l) - ref) <= 1e-13 * max(1.0, abs(ref)), l


@pytest.mark.parametrize("D", [2, 3])
def test_geq_energy_flux_closed_forms(oracle_mod, D):
    """Eqs. (5), (37), (38): sum g^eq = rho E, q^eq = (H + u^2/2) rho u and
    R^eq = (H + u^2/2) P^eq + P u u with H = C_p T, P = rho T."""
    c = oracle_mod.velocities(D)
    for rho, u, T in _states(D):
        gamma = RNG.uniform(1.1, 1.7)
        Cv = 1.0 / (gamma - 1.0)
        Cp = gamma * Cv
        g = oracle_mod.geq(D, rho, u, T, Cv)
        u2 = float(u @ u)
        assert abs(g.sum() - rho * (Cv * T + u2 / 2)) <= 1e-14 * max(1, rho)
        h = Cp * T + u2 / 2
        for a in range(D):
            e = [0] * D
            e[a] = 1
            assert abs(_moment(c, g, e) - h * rho * u[a]) <= 1e-13
            for b in range(D):
                e = [0] * D
                e[a] += 1
                e[b] += 1
                Peq = rho * T * (a == b) + rho * u[a] * u[b]
                ref = h * Peq + rho * T * u[a] * u[b]
                assert abs(_moment(c, g, e) - ref) <= 1e-13


@pytest.mark.parametrize("D", [2, 3])
def test_gstar_moments(oracle_mod, D):
    """Eqs. (44)-(45): g* carries q* = q^eq + dq as first moment and the
    g^eq moments otherwise."""
    c = oracle_mod.velocities(D)
    for rho, u, T in _states(D):
        Cv = 2.5
        S = RNG.uniform(-0.02, 0.02, size=(D, D))
        Peq = rho * (T * np.eye(D) + np.outer(u, u))
        P = Peq + S + S.T
        d = RNG.uniform(-0.03, 0.03, size=D)
        gs = oracle_mod.gstar(D, rho, u, T, Cv, P, d)
        ge = oracle_mod.geq(D, rho, u, T, Cv)
        dq = oracle_mod.dq(D, rho, u, T, P, d)
        for l in itertools.product(range(3), repeat=D):
            ref = _moment(c, ge, l)
            if sum(l) == 1:
                ref += dq[list(l).index(1)]
            assert abs(_moment(c, gs, l) - ref) <= 1e-14, l


def test_dq_special_cases(oracle_mod):
    """Eq. (46): q* - q^eq vanishes at rest and at P = P^eq, d = 0; a hand
    example: u = (1/2, 0), P - P^eq = [[a, b], [b, e]], d = (d_x, d_y) gives
    (a/2 + d_x/4, b/2)."""
    rho, T = 1.2, 0.3
    u = np.array([0.5, 0.0])
    Peq = rho * (T * np.eye(2) + np.outer(u, u))
    assert np.allclose(oracle_mod.dq(2, rho, u, T, Peq, [0, 0]), 0, atol=1e-16)
    assert np.allclose(oracle_mod.dq(2, rho, [0, 0], T, Peq + 0.1, [0.3, 0.2]), 0, atol=1e-16)
    a, b, e, dx, dy = 0.04, -0.02, 0.01, 0.08, -0.06
    P = Peq + np.array([[a, b], [b, e]])
    got = oracle_mod.dq(2, rho, u, T, P, [dx, dy])
    assert np.allclose(got, [a / 2 + dx / 4, b / 2], atol=1e-15)


@pytest.mark.parametrize("D", [2, 3])
def test_collision_conserves_mass_momentum_energy(oracle_mod, D):
    """Eqs. (3)-(5): relaxation conserves rho, rho u and rho E at a node."""
    c = oracle_mod.velocities(D)
    for rho, u, T in _states(D, 6):
        p = oracle_mod.make_params(D, (4, 4, 4 if D == 3 else 1), gamma=1.4, Pr=RNG.uniform(0.5, 1.5),
                                   mu=RNG.uniform(0.001, 0.05), visc_exp=0.76, T_ref=0.15)
        fh = oracle_mod.feq(D, rho, u, T) * (1 + RNG.uniform(-0.05, 0.05, size=oracle_mod.Q(D)))
        gh = oracle_mod.geq(D, rho, u, T, 2.5) * (1 + RNG.uniform(-0.05, 0.05, size=oracle_mod.Q(D)))
        d = RNG.uniform(-0.02, 0.02, size=D)
        fo, go = oracle_mod.collide_node(p, fh, gh, d)
        assert abs(fo.sum() - fh.sum()) <= 2e-15 * abs(fh.sum())
        assert abs(go.sum() - gh.sum()) <= 2e-15 * abs(gh.sum())
        for a in range(D):
            e = [0] * D
            e[a] = 1
            assert abs(_moment(c, fo, e) - _moment(c, fh, e)) <= 2e-15 * abs(fh.sum())


def test_collision_is_bgk_with_published_rates(oracle_mod):
    """Eqs. (1), (2), (92), (96): with fh = f^eq, gh = g^eq and d = 0 the
    populations are a fixed point; the non-equilibrium parts relax with
    1 - omega (f) and, on populations with c_i^2 != 1, 1 - omega_1 (g)."""
    D = 2
    rho, u, T = 1.1, np.array([0.1, -0.05]), 0.2
    mu, Pr = 0.02, 0.7
    p = oracle_mod.make_params(D, (4, 4), gamma=1.4, Pr=Pr, mu=mu)
    Cv = 2.5
    fe = oracle_mod.feq(D, rho, u, T)
    ge = oracle_mod.geq(D, rho, u, T, Cv)
    fo, go = oracle_mod.collide_node(p, fe, ge, [0, 0])
    assert np.allclose(fo, fe, atol=1e-15) and np.allclose(go, ge, atol=1e-15)
    # perturb g on the rest and diagonal populations only: rho, u, T, P unchanged
    # requires a perturbation with zero mass and energy moments; use two diagonals
    dg = np.zeros(9)
    dg[0] = 1e-3   # (-1,-1)
    dg[8] = 1e-3   # (+1,+1)
    dg[4] = -2e-3  # rest
    om = 1.0 / (mu / (rho * T) + 0.5)
    om1 = 1.0 / ((1.0 / om - 0.5) / Pr + 0.5)
    _, go = oracle_mod.collide_node(p, fe, ge + dg, [0, 0])
    # the momentum-like first moment of dg changes T? sum c_x dg != 0 only touches g, not f:
    # rho E changes by sum dg = 0, so T is unchanged and g^eq is unchanged.
    assert np.allclose(go - ge, (1 - om1) * dg, atol=1e-15)


def test_omega_inverts_viscosity(oracle_mod):
    """Eq. (92): mu = (1/omega - 1/2) rho T."""
    for mu, rho, T in [(0.01, 1.0, 0.15), (0.0374, 0.8, 0.2), (1e-4, 2.0, 0.05)]:
        om = oracle_mod.omega(mu, rho, T)
        assert abs((1 / om - 0.5) * rho * T - mu) <= 1e-15 * max(mu, 1e-3)


def test_omega1_prandtl_round_trip(oracle_mod):
    """Eq. (96): Pr = omega_1 (2 - omega) / (omega (2 - omega_1)), and the
    conductivity/viscosity form (1/omega_1 - 1/2) = (1/omega - 1/2)/Pr."""
    for om in (0.3, 1.0, 1.5, 1.99):
        for Pr in (0.5, 0.7, 0.71, 1.0, 2.0):
            om1 = oracle_mod.omega1(om, Pr)
            # (2 - omega) and (2 - omega_1) cancel near omega = 2: allow their conditioning
            assert abs(om1 * (2 - om) / (om * (2 - om1)) - Pr) <= 1e-15 * Pr * 2 / (2 - om1) * 4
            assert abs((1 / om1 - 0.5) - (1 / om - 0.5) / Pr) <= 1e-13


def _field_sim(oracle_mod, n, bc, deriv):
    return oracle_mod.Sim(3, (n, 3, 2), bc=(bc, 0, 0), deriv=deriv)


@pytest.mark.parametrize("bc", [0, 1])
def test_upwind_derivative_linear_and_branches(oracle_mod, bc):
    """Sec. III.A: the upwind difference of a linear field is its slope on
    either branch; for a quadratic field the branch is backward where u > 0
    and forward where u <= 0 (u == 0 takes the 'otherwise' branch)."""
    n = 12
    s = _field_sim(oracle_mod, n, bc, oracle_mod.UPWIND)
    x = np.arange(n, dtype=float)
    lin = np.broadcast_to(0.3 * x - 1.0, (2, 3, n)).copy()
    u = np.broadcast_to(np.where(x < 6, 0.2, -0.1), (2, 3, n)).copy()
    d = s.derivative(0, lin, u)
    interior = slice(1, n - 1)
    assert np.allclose(d[..., interior], 0.3, atol=1e-14)
    quad = np.broadcast_to(x * x, (2, 3, n)).copy()
    u2 = np.broadcast_to(np.array([0.1 if k % 3 == 0 else (-0.1 if k % 3 == 1 else 0.0) for k in range(n)]),
                         (2, 3, n)).copy()
    d = s.derivative(0, quad, u2)
    for k in range(1, n - 1):
        want = (k * k - (k - 1) ** 2) if u2[0, 0, k] > 0 else ((k + 1) ** 2 - k * k)
        assert d[0, 0, k] == want
    # ends: periodic wraps, zero-gradient clamps (the ghost equals the boundary node)
    k0 = quad[0, 0, 0]
    if bc == 0:
        assert d[0, 0, 0] == k0 - quad[0, 0, n - 1]          # u > 0 at x = 0
    else:
        assert d[0, 0, 0] == 0.0
        assert d[0, 0, n - 1] == quad[0, 0, n - 1] - quad[0, 0, n - 1]  # u <= 0: forward into the clamp


def test_central_derivative(oracle_mod):
    """Sec. III.D.2: second-order central difference (Q_{x+1} - Q_{x-1}) / 2."""
    n = 10
    s = _field_sim(oracle_mod, n, 0, oracle_mod.CENTRAL)
    x = np.arange(n, dtype=float)
    quad = np.broadcast_to(x * x, (2, 3, n)).copy()
    d = s.derivative(0, quad, np.zeros_like(quad))
    assert np.allclose(d[..., 1:-1], 2 * x[1:-1])
