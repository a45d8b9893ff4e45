"""Pins of the oracle's sampled step, its upwind-side override and its FP32
storage model.

* orc_step_sampled computes, at listed nodes only, what one orc_step writes
  there: bit for bit, on unsorted node lists with repeats.
* orc_step_sampled_branch forces the side of the upwind difference of
  Sec. III.A per node and axis.  The pin is independent of the oracle's own
  step: the streamed populations at the node are formed here by shifting
  whole arrays (pull streaming, Eqs. (1)-(2)), the anomaly Qt_a of Eq. (29) of
  the node and its two neighbours from their moments (Eqs. (3)-(7)), and the
  named side's difference is fed to the oracle's one-node collision.
* orc_set_fp32_storage keeps every stored population at its reference value
  plus an FP32 deviation (up to the FP64 rounding of the sum), within half an
  FP32 ulp of the deviation from the unrounded value.
"""
import numpy as np
import pytest

import oracle
from paper_2102_09512_amd import inputs as I

CV = 2.5


def _sim(D, dims, deriv=0, bc=(0, 0, 0), steps=3, seed=4):
    f = I.smooth_random(D, dims, seed=seed, u_amp=0.08, T_amp=0.03)
    s = oracle.Sim(D, dims, gamma=1.4, Pr=0.7, mu=0.02, visc_exp=0.76, T_ref=0.15, bc=bc, deriv=deriv)
    s.init(*f)
    s.step(steps)
    return s


def _copy(s, D, dims, deriv=0, bc=(0, 0, 0)):
    t = oracle.Sim(D, dims, gamma=1.4, Pr=0.7, mu=0.02, visc_exp=0.76, T_ref=0.15, bc=bc, deriv=deriv)
    f, g = s.get_pops()
    t.set_pops(f, g, s.step_count)
    return t


@pytest.mark.parametrize("D,dims,deriv,bc", [
    (3, (9, 8, 7), 0, (0, 0, 0)),
    (3, (7, 6, 9), 1, (0, 1, 0)),
    (2, (17, 13), 0, (1, 0, 0)),
])
def test_sampled_step_equals_the_full_step_bit_for_bit(D, dims, deriv, bc):
    s = _sim(D, dims, deriv, bc)
    N = int(np.prod(dims))
    rng = np.random.default_rng(1)
    nodes = np.concatenate([rng.permutation(N)[: N // 3], [0, N - 1, 0]]).astype(np.int64)
    fs, gs = s.step_sampled(nodes)
    t = _copy(s, D, dims, deriv, bc)
    t.step(1)
    f, g = t.get_pops()
    Q = oracle.Q(D)
    assert np.array_equal(fs, f.reshape(Q, N)[:, nodes])
    assert np.array_equal(gs, g.reshape(Q, N)[:, nodes])
    # the state itself is untouched by the sampled step
    f0, g0 = s.get_pops()
    f1, _ = _copy(s, D, dims, deriv, bc).get_pops()
    assert np.array_equal(f0, f1)


def _streamed_moments(s, D):
    """Pull-streamed populations and their rho, u, T, by whole-array shifts
    (periodic box): fh_i(x) = f_i(x - c_i)."""
    f, g = s.get_pops()
    c = oracle.velocities(D)
    fh, gh = np.empty_like(f), np.empty_like(g)
    for i in range(oracle.Q(D)):
        sh = (c[i, 2], c[i, 1], c[i, 0])
        fh[i] = np.roll(f[i], sh, axis=(0, 1, 2))
        gh[i] = np.roll(g[i], sh, axis=(0, 1, 2))
    rho = fh.sum(0)
    u = np.stack([np.tensordot(c[:, a], fh, axes=(0, 0)) / rho for a in range(D)])
    T = (gh.sum(0) / rho - 0.5 * (u ** 2).sum(0)) / CV
    return fh, gh, rho, u, T


def test_branch_override_takes_the_named_side():
    D, dims = 3, (8, 7, 6)
    s = _sim(D, dims, steps=4, seed=9)
    fh, gh, rho, u, T = _streamed_moments(s, D)
    Q, N = oracle.Q(D), int(np.prod(dims))
    rng = np.random.default_rng(2)
    nodes = rng.permutation(N)[:12].astype(np.int64)
    choices = rng.integers(0, 2, size=(nodes.size, D)).astype(np.int8)
    f_o, g_o = s.step_sampled_branch(nodes, choices)
    f_nat, _ = s.step_sampled(nodes)
    nshape = (dims[2], dims[1], dims[0])
    differs = 0
    for k, node in enumerate(nodes):
        z, y, x = np.unravel_index(node, nshape)
        d = np.zeros(3)
        natural = True
        for a in range(D):
            def qt(shift):
                p = [z, y, x]
                p[2 - a] = (p[2 - a] + shift) % nshape[2 - a]
                return oracle.anomaly(rho[tuple(p)], u[a][tuple(p)], T[tuple(p)])
            side = choices[k, a]
            d[a] = qt(0) - qt(-1) if side == 0 else qt(1) - qt(0)
            natural &= (side == 0) == (u[a][z, y, x] > 0)
        fo, go = oracle.collide_node(s.params, fh[:, z, y, x], gh[:, z, y, x], d)
        scale = np.abs(fo).max()
        assert np.abs(f_o[:, k] - fo).max() <= 1e-13 * scale
        assert np.abs(g_o[:, k] - go).max() <= 1e-13 * np.abs(go).max()
        if not natural:
            differs += 1
            assert np.abs(f_o[:, k] - f_nat[:, k]).max() > 1e-9 * scale
    assert differs >= 3


def test_branch_override_minus_one_and_the_natural_side_change_nothing():
    D, dims = 3, (7, 6, 5)
    s = _sim(D, dims, steps=2, seed=5)
    _, _, _, u, _ = _streamed_moments(s, D)
    N = int(np.prod(dims))
    nodes = np.arange(N, dtype=np.int64)
    f_nat, g_nat = s.step_sampled(nodes)
    f_m, g_m = s.step_sampled_branch(nodes, -np.ones((N, D), dtype=np.int8))
    natural = np.stack([np.where(u[a].ravel() > 0, 0, 1) for a in range(D)], axis=1).astype(np.int8)
    f_n, g_n = s.step_sampled_branch(nodes, natural)
    assert np.array_equal(f_nat, f_m) and np.array_equal(g_nat, g_m)
    assert np.array_equal(f_nat, f_n) and np.array_equal(g_nat, g_n)
    with pytest.raises(ValueError):
        s.step_sampled_branch(nodes[:2], np.full((2, D), 2, dtype=np.int8))
    with pytest.raises(ValueError):
        s.step_sampled_branch(np.array([N], dtype=np.int64), np.zeros((1, D), dtype=np.int8))


def test_fp32_storage_model_rounds_only_the_deviation():
    D, dims = 3, (6, 5, 4)
    f_in = I.smooth_random(D, dims, seed=3, u_amp=0.1, T_amp=0.03)
    ref = (1.0, [0.0, 0.0, 0.0], 0.15)
    f_ref = oracle.feq(D, ref[0], ref[1], ref[2])
    g_ref = oracle.geq(D, ref[0], ref[1], ref[2], CV)
    exact = oracle.Sim(D, dims, gamma=1.4, Pr=0.7, mu=0.02)
    exact.init(*f_in)
    rounded = oracle.Sim(D, dims, gamma=1.4, Pr=0.7, mu=0.02)
    rounded.set_fp32_storage(f_ref, g_ref)
    rounded.init(*f_in)
    for sim_pair_step in range(2):
        fe, ge = exact.get_pops()
        fr, gr = rounded.get_pops()
        for e, r, w in ((fe, fr, f_ref), (ge, gr, g_ref)):
            dev = r - w[:, None, None, None]
            # an FP32 value, up to the FP64 rounding of reference + deviation
            assert (np.abs(dev - dev.astype(np.float32)) <= 2.0 ** -52 * np.abs(r)).all()
            de = e - w[:, None, None, None]
            assert (np.abs(r - e) <= 2.0 ** -24 * np.abs(de) + 1e-17).all()
            assert np.abs(r - e).max() > 0  # something was rounded
        # one step each, from the same (rounded) state: the model rounds the result again
        exact.set_pops(fr, gr)
        exact.step(1)
        rounded.step(1)
    rounded.set_fp32_storage(None)
    fr, gr = rounded.get_pops()
    exact.set_pops(fr, gr)
    exact.step(1)
    rounded.step(1)
    assert np.array_equal(exact.get_pops()[0], rounded.get_pops()[0])


def test_upwind_band_reverses_only_the_decisions_within_the_band():
    """orc_set_upwind_band: every upwind decision of Sec. III.A with
    |u_a| <= band takes the other side; the others, and every decision with
    band 0 (u_a = 0 included: the 'otherwise' side), are the plain scheme's."""
    dims = (12, 3, 2)
    s = oracle.Sim(3, dims, gamma=1.4, Pr=0.7, mu=0.02)
    x = np.arange(12, dtype=float)
    Qt = np.broadcast_to(x ** 2 + 0.5 * x ** 3, (2, 3, 12)).copy()
    uv = np.array([0.3, 1e-9, -1e-9, 0.0, -0.2, 5e-9, 2e-8, -2e-8, 1e-8, -1e-8, 0.1, -0.1])
    u = np.broadcast_to(uv, (2, 3, 12)).copy()
    q = Qt[0, 0]

    def expected(band):
        out = np.zeros(12)
        for k in range(12):
            backward = uv[k] > 0
            if band > 0 and abs(uv[k]) <= band:
                backward = not backward
            out[k] = q[k] - q[k - 1] if backward else q[(k + 1) % 12] - q[k]
        return out

    for band in (0.0, 1e-8, 3e-9):
        s.set_upwind_band(band)
        d = s.derivative(0, Qt, u)
        assert np.array_equal(d[0, 0], expected(band)), band
    assert not np.array_equal(expected(1e-8), expected(0.0))
    with pytest.raises(ValueError):
        s.set_upwind_band(-1.0)
