"""The patch reduction used at grid sizes the whole-field oracle cannot hold
(tests/oracle_patch.py): the centre of a 9^3 periodic patch stepped twice has
the moments of the whole periodic grid at that node, for nodes next to the
grid's own periodic edges too, with the plain FP64 oracle and with its FP32
storage model.  A patch of radius 2 is too small, which shows the check can
fail."""
import numpy as np
import pytest

import oracle
from paper_2102_09512_amd import inputs as I
import oracle_patch as P
import oracle_floor

KW = dict(gamma=1.4, Pr=0.7, visc_exp=0.76, T_ref=0.15)


def _fields(n):
    rho, u, T = I.turbulence(3, n, seed=4, k0_index=2, Ma_t=0.5, T0=0.15)
    rho = rho + 0.02 * np.cos(2 * np.pi * np.arange(n) / n)[None, None, :]  # density varies too
    return rho, u, T


@pytest.mark.parametrize("fp32", [False, True])
def test_patch_centre_equals_whole_grid(fp32):
    n = 16
    fields = _fields(n)
    mu = I.turbulence_viscosity(n, k0_index=2, Ma_t=0.5, T0=0.15, Re_lambda=72.0)
    kw = dict(KW, mu=mu)
    rest = oracle_floor.fp32_reference(3) if fp32 else None
    s = oracle.Sim(3, (n, n, n), **kw)
    if rest is not None:
        s.set_fp32_storage(*rest)
    s.init(*fields)
    s.step(2)
    rho, u, T = s.moments()
    rng = np.random.default_rng(1)
    nodes = np.concatenate([[0, n - 1, n * n - 1, n ** 3 - 1, n * n * (n // 2) + n // 2], rng.integers(0, n ** 3, 20)])
    for node in nodes:
        (r, v, t), _, _ = P.two_step_moments(fields, node, n, kw, rest)
        flat = int(node)
        assert abs(r - rho.reshape(-1)[flat]) <= 1e-14
        assert np.abs(v - u.reshape(3, -1)[:, flat]).max() <= 1e-14
        assert abs(t - T.reshape(-1)[flat]) <= 1e-14


def test_too_small_patch_differs():
    n = 16
    fields = _fields(n)
    mu = I.turbulence_viscosity(n, k0_index=2, Ma_t=0.5, T0=0.15, Re_lambda=72.0)
    kw = dict(KW, mu=mu)
    s = oracle.Sim(3, (n, n, n), **kw)
    s.init(*fields)
    s.step(2)
    rho, u, T = s.moments()
    worst = 0.0
    for node in [5, 300, 2000]:
        (_, v, _), _, _ = P.two_step_moments(fields, node, n, kw, r=2)
        worst = max(worst, float(np.abs(v - u.reshape(3, -1)[:, node]).max()))
    assert worst > 1e-8
