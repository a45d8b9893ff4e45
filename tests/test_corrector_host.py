"""Host-side parts of the learned-corrector workflow (no GPU): the spectrum,
the overlap remap between grids and the seed tables, against the oracle's
independent definitions and closed forms."""
import numpy as np
import pytest

from oracle import convnet as N
from paper_2102_09512_amd import corrector as Cr
from paper_2102_09512_amd import inputs as I


def _fields(n, seed):
    r = np.random.default_rng(seed)
    rho = 1.0 + 0.05 * r.random((n, n, n))
    u = 0.1 * r.normal(size=(3, n, n, n))
    T = 0.15 + 0.01 * r.random((n, n, n))
    return rho, u, T


def test_spectrum_matches_the_oracle():
    u = np.random.default_rng(1).normal(size=(3, 12, 12, 12))
    a, b = Cr.spectrum(u), N.kinetic_energy_spectrum(u)
    assert a.shape == b.shape and np.allclose(a, b, rtol=1e-12, atol=0)


def test_spectrum_error_is_zero_for_equal_and_log_ratio_for_scaled():
    E = np.array([0.0, 1.0, 2.0, 3.0, 4.0])
    assert Cr.spectrum_error(E, E, 4) == 0.0
    assert Cr.spectrum_error(2.0 * E, E, 4) == pytest.approx(np.log(2.0), rel=1e-14)


@pytest.mark.parametrize("factor", [2, 4])
def test_remap_with_an_integer_ratio_is_the_box_filter(factor):
    rho, u, T = _fields(8, 2)
    got = Cr.remap(rho, u, T, 8 // factor, 2.5)
    ref = N.box_filter(rho, u, T, factor, 2.5)
    for a, b in zip(got, ref):
        assert np.allclose(a, b, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("n_out", [5, 7, 11])
def test_remap_keeps_mass_momentum_energy(n_out):
    rho, u, T = _fields(9, 3)
    r, uc, Tc = Cr.remap(rho, u, T, n_out, 2.5)
    w = (9 / n_out) ** 3  # fine cells per coarse cell
    E, Ec = 2.5 * T + 0.5 * (u ** 2).sum(0), 2.5 * Tc + 0.5 * (uc ** 2).sum(0)
    assert (r.sum() * w) == pytest.approx(rho.sum(), rel=1e-13)
    for a in range(3):
        assert (r * uc[a]).sum() * w == pytest.approx((rho * u[a]).sum(), rel=1e-11, abs=1e-12)
    assert (r * Ec).sum() * w == pytest.approx((rho * E).sum(), rel=1e-13)
    one = Cr.remap(np.ones((9,) * 3), np.full((3,) + (9,) * 3, 0.1), np.full((9,) * 3, 0.15), n_out, 2.5)
    assert np.allclose(one[0], 1.0) and np.allclose(one[1], 0.1) and np.allclose(one[2], 0.15)


def test_overlap_matrix_rows_and_columns():
    R = Cr.overlap_matrix(5, 7)
    assert np.allclose(R.sum(1), 1.0)  # each coarse cell is fully covered
    assert np.allclose(R.sum(0), 5 / 7)  # each fine cell is spread in full
    assert np.array_equal(Cr.overlap_matrix(4, 4), np.eye(4))


def test_fine_turbulence_is_the_coarse_field_sampled_finer():
    rho, u, T = I.turbulence_fine(32, 5, n_gen=16, Ma_t=0.4)
    r2, u2, T2 = I.turbulence(3, 16, 5, Ma_t=0.4)
    assert np.abs(u[:, ::2, ::2, ::2] - u2).max() < 1e-14
    assert np.sqrt((u ** 2).sum(0).mean()) == pytest.approx(np.sqrt((u2 ** 2).sum(0).mean()), rel=1e-12)
    k = np.fft.fftfreq(32, d=1.0 / 32)
    uh = np.fft.fftn(u, axes=(1, 2, 3))
    kd = uh[0] * k[None, None, :] + uh[1] * k[None, :, None] + uh[2] * k[:, None, None]
    assert np.abs(kd).max() < 1e-9 * np.abs(uh).max()  # still solenoidal


def test_seed_tables():
    s, m = Cr.training_seeds(32)
    assert s == list(range(32)) and all(0.3 <= x <= 0.6 for x in m) and len(set(m)) == 32
    e, me = Cr.evaluation_seeds(4)
    assert not set(e) & set(s) and me == pytest.approx([0.3375, 0.4125, 0.4875, 0.5625])


def test_summary_sets_apart_seeds_where_the_plain_run_fails():
    inf = float("inf")
    row = lambda l, p, q, n=64: {"learned": {"error": l}, "plain_coarse": {"error": p, "n": 64},
                                "plain_equal_time": {"error": q, "n": n}}
    s = Cr.summarize([row(0.1, 0.7, 0.6, 80), row(inf, 0.8, 0.8), row(inf, inf, inf)])
    assert s["seeds"] == 2 and s["seeds_plain_coarse_unstable"] == 1
    assert s["wins_equal_time"] == 1 and s["learned"] == inf  # a corrected run that fails alone counts
    assert s["plain_coarse"] == pytest.approx(0.75) and s["equal_time_grids"] == [80, 64]
