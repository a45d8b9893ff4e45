"""Pins of the FP64 reference network, box filter and spectrum (oracle/convnet.py)
against definitions that do not go through its own code paths: impulse
responses, translation equivariance, finite differences, the first Adam step,
conservation of the filter and Parseval's identity."""
import numpy as np
import pytest

from oracle import convnet as N


def _rand_params(channels, seed, scale=0.2):
    r = np.random.default_rng(seed)
    return r.normal(0.0, scale, N.param_count(channels))


def test_impulse_response_fixes_the_tap_convention():
    """One layer, no ReLU: a unit impulse in channel i at node u gives, at the
    node u - s_t, W[t][i][:] + b (y(v) = sum_t x(v + s_t) W[t])."""
    ch = [2, 3]
    p = _rand_params(ch, 1)
    (W, b), = N.unpack(p, ch)
    shape = (5, 6, 7)  # z, y, x
    x = np.zeros((2,) + shape)
    uz, uy, ux = 2, 3, 4
    x[1, uz, uy, ux] = 1.0
    y, _ = N.forward(p, ch, x)
    for t, (dx, dy, dz) in enumerate(N.TAPS):
        v = ((uz - dz) % 5, (uy - dy) % 6, (ux - dx) % 7)
        assert np.allclose(y[(slice(None),) + v], W[t, 1] + b, atol=1e-15)


def test_translation_equivariance():
    ch = [3, 32, 3]
    p = _rand_params(ch, 2)
    x = np.random.default_rng(3).normal(size=(3, 4, 5, 6))
    y, _ = N.forward(p, ch, x)
    ys, _ = N.forward(p, ch, np.roll(x, (1, -2, 3), axis=(1, 2, 3)))
    assert np.allclose(ys, np.roll(y, (1, -2, 3), axis=(1, 2, 3)), atol=1e-13)


@pytest.mark.parametrize("ch,offset", [([3, 32, 32, 3], 0), ([3, 32, 32, 2], 1)])
def test_gradients_match_finite_differences(ch, offset):
    p = _rand_params(ch, 4, scale=0.15)
    r = np.random.default_rng(5)
    x = 1.0 + 0.1 * r.normal(size=(3, 4, 4, 5))
    t = x + 0.05 * r.normal(size=x.shape)
    mean, std = np.array([1.0, 0.9, 1.1]), np.array([0.1, 0.2, 0.15])
    loss, g = N.loss_and_grad(p, ch, x, t, mean, std, out_offset=offset)
    assert loss > 0
    idx = r.choice(p.size, 60, replace=False)
    eps = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += eps
        pm[k] -= eps
        fd = (N.loss_and_grad(pp, ch, x, t, mean, std, out_offset=offset)[0]
              - N.loss_and_grad(pm, ch, x, t, mean, std, out_offset=offset)[0]) / (2 * eps)
        assert fd == pytest.approx(g[k], rel=1e-5, abs=1e-9 * max(1.0, abs(loss)))


def test_first_adam_step_closed_form():
    """With zero moments the first bias-corrected step moves every parameter
    by lr * g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p = np.zeros(4)
    m, v = np.zeros(4), np.zeros(4)
    N.adam_step(p, g, m, v, lr=0.1, b1=0.9, b2=0.999, eps=1e-8, t=1)
    assert np.allclose(p, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


@pytest.mark.parametrize("D", [2, 3])
def test_box_filter_conserves_mass_momentum_energy(D):
    r = np.random.default_rng(6)
    shape = (8, 8, 12) if D == 3 else (1, 8, 12)
    rho = 1.0 + 0.1 * r.random(shape)
    u = 0.1 * r.normal(size=(D,) + shape)
    T = 0.15 + 0.02 * r.random(shape)
    Cv = 2.5
    rc, uc, Tc = N.box_filter(rho, u, T, 4, Cv)
    cells = 4 ** D
    E = Cv * T + 0.5 * (u ** 2).sum(0)
    Ec = Cv * Tc + 0.5 * (uc ** 2).sum(0)
    assert (rc * cells).sum() == pytest.approx(rho.sum(), rel=1e-14)
    for a in range(D):
        assert (rc * uc[a] * cells).sum() == pytest.approx((rho * u[a]).sum(), rel=1e-12, abs=1e-14)
    assert (rc * Ec * cells).sum() == pytest.approx((rho * E).sum(), rel=1e-14)
    # a uniform state is unchanged
    one = N.box_filter(np.ones(shape), np.full((D,) + shape, 0.1), np.full(shape, 0.15), 2, Cv)
    assert np.allclose(one[0], 1.0) and np.allclose(one[1], 0.1) and np.allclose(one[2], 0.15)


def test_spectrum_parseval_and_single_mode():
    r = np.random.default_rng(7)
    u = r.normal(size=(3, 8, 8, 8))
    E = N.kinetic_energy_spectrum(u)
    assert E.sum() == pytest.approx(0.5 * (u ** 2).sum(0).mean(), rel=1e-12)
    z, y, x = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
    w = np.zeros((3, 8, 8, 8))
    w[1] = np.cos(2 * np.pi * 3 * x / 8)  # one mode at |k| = 3
    E = N.kinetic_energy_spectrum(w)
    assert E[3] == pytest.approx(0.25, rel=1e-12) and E.sum() == pytest.approx(0.25, rel=1e-12)


def test_bf16_rounding_follows_the_format():
    """bfloat16 keeps 8 significant bits: representable values pass unchanged,
    halfway cases go to the even neighbour, and the relative error of any
    normal value is at most 2^-8 (half a unit in the 8th significant bit)."""
    for v in (0.0, 1.0, 1.5, -2.0, 2.0 ** -100, 3.0 * 2.0 ** 60, 1.0 + 2.0 ** -7):
        assert N.bf16(v) == v
    assert N.bf16(1.0 + 2.0 ** -8) == 1.0  # tie, 1.0 is even
    assert N.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # tie, 1 + 2^-7 is odd
    assert N.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7  # above the tie
    assert N.bf16(-(1.0 + 2.0 ** -8 + 2.0 ** -20)) == -(1.0 + 2.0 ** -7)
    x = np.random.default_rng(8).normal(size=10000) * 10.0 ** np.random.default_rng(9).integers(-20, 20, 10000)
    r = N.bf16(x)
    assert np.all(np.abs(r - x) <= (2.0 ** -8 + 2.0 ** -24) * np.abs(x))  # FP32 first, then bf16
    assert np.all(N.bf16(r) == r)


def test_bf16_storage_changes_the_network_by_its_rounding_only():
    """With bf16 storage the loss stays within a few roundings of FP64 and the
    gradients keep their direction; with representable operands and a single
    linear layer (no stored activations) nothing changes at all."""
    ch = [3, 32, 32, 3]
    p = _rand_params(ch, 10, scale=0.15)
    r = np.random.default_rng(11)
    x = 1.0 + 0.1 * r.normal(size=(3, 4, 4, 8))
    t = x + 0.05 * r.normal(size=x.shape)
    mean, std = np.array([1.0, 1.0, 1.0]), np.array([0.1, 0.1, 0.1])
    l64, g64 = N.loss_and_grad(p, ch, x, t, mean, std)
    l16, g16 = N.loss_and_grad(p, ch, x, t, mean, std, store=N.bf16)
    assert l16 == pytest.approx(l64, rel=2e-2) and l16 != l64
    assert g16 @ g64 / (np.linalg.norm(g16) * np.linalg.norm(g64)) > 0.99
    one = [2, 3]
    q = N.bf16(_rand_params(one, 12))
    xi = N.bf16(r.normal(size=(2, 3, 4, 5)))
    assert np.array_equal(N.forward(q, one, xi, store=N.bf16)[0], N.forward(q, one, xi)[0])


def test_output_offset_compares_the_named_fields():
    """With offset 1 the outputs are compared with fields 1 and 2: changing the
    target of field 0 changes nothing, changing field 1's does."""
    ch = [3, 32, 2]
    p = _rand_params(ch, 13)
    r = np.random.default_rng(14)
    x = 1.0 + 0.1 * r.normal(size=(3, 4, 4, 4))
    t = x + 0.05 * r.normal(size=x.shape)
    mean, std = np.ones(3), np.full(3, 0.1)
    l0 = N.loss_and_grad(p, ch, x, t, mean, std, out_offset=1)[0]
    t2 = t.copy()
    t2[0] += 1.0
    assert N.loss_and_grad(p, ch, x, t2, mean, std, out_offset=1)[0] == l0
    t2[1] += 0.01
    assert N.loss_and_grad(p, ch, x, t2, mean, std, out_offset=1)[0] != l0
