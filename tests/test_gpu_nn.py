"""The learned corrector's kernels against the FP64 reference network
(oracle/convnet.py): forward, loss and gradients on bf16 matrix cores (FP32
accumulation), the Adam step, training on a toy problem; and the coupling to
the lattice Boltzmann library: field increments by re-equilibration and the
conservative box filter against the oracle."""
import numpy as np
import pytest

import oracle
from oracle import convnet as N
from paper_2102_09512_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CH = [5, 32, 32, 32, 5]


def _lbm():
    from paper_2102_09512_amd import lbm

    return lbm


def _params(seed, channels=CH, gain=1.0):
    """He-scaled random weights, small biases."""
    r = np.random.default_rng(seed)
    out = []
    for l in range(len(channels) - 1):
        ci, co = channels[l], channels[l + 1]
        out.append(r.normal(0.0, gain * np.sqrt(2.0 / (27 * ci)), 27 * ci * co))
        out.append(r.normal(0.0, 0.01, co))
    return np.concatenate(out)


def _fields(shape, seed):
    r = np.random.default_rng(seed)
    x = np.empty((5,) + shape)
    x[0] = 1.0 + 0.05 * r.normal(size=shape)
    x[1:4] = 0.1 * r.normal(size=(3,) + shape)
    x[4] = 0.15 + 0.01 * r.normal(size=shape)
    return x


MEAN = np.array([1.0, 0.0, 0.0, 0.0, 0.15])
STD = np.array([0.05, 0.1, 0.1, 0.1, 0.01])
OUT = np.array([0.002, 0.004, 0.003, 0.005, 0.0005])  # output scale of a corrector


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_forward_matches_reference():
    lbm = _lbm()
    shape = (8, 8, 64)  # z, y, x: two tiles along x, two along y and z
    p = _params(1)
    x = _fields(shape, 2)
    n = lbm.lbm_nn_create(CH, shape[::-1])
    try:
        lbm.lbm_nn_set_params(n, p.astype(np.float32))
        lbm.lbm_nn_set_scaling(n, MEAN, STD)
        xd = torch.from_numpy(x.astype(np.float32)).cuda()
        yd = torch.zeros((5,) + shape, dtype=torch.float32, device="cuda")
        lbm.lbm_nn_forward(n, xd, yd)
        torch.cuda.synchronize()
        y = yd.cpu().numpy()
    finally:
        lbm.lbm_nn_destroy(n)
    xn = (x - MEAN[:, None, None, None]) / STD[:, None, None, None]
    ref16, _ = N.forward(p, CH, xn, store=N.bf16)
    ref, _ = N.forward(p, CH, xn)
    e16, e = _rel(y, ref16), _rel(y, ref)
    print(f"  forward: max error {e16:.2e} against bf16 storage, {e:.2e} against FP64, "
          f"max |y| {np.abs(ref).max():.3f}", flush=True)
    assert e16 < 5e-3  # FP32 accumulation order, rare flips of a bf16 rounding
    assert e < 3e-2  # bf16 operands (8 significant bits) through four layers


def test_forward_at_the_benchmark_size():
    """The forward in the configuration the benchmark times (64^3, channels
    5-32-32-32-3, He-normal weights, unit scaling, standard-normal input):
    every output against the bf16-storage reference."""
    from paper_2102_09512_amd import corrector as Cr

    lbm = _lbm()
    w = Cr.Workload()
    ch, n = list(w.channels), w.n_coarse
    p = Cr.initial_params(ch, seed=0, last_gain=1.0)
    x = np.random.default_rng(5).standard_normal((5, n, n, n)).astype(np.float32)
    print(f"[gpu case] network forward {n}^3, channels {ch}", flush=True)
    net = lbm.lbm_nn_create(ch, (n, n, n))
    try:
        lbm.lbm_nn_set_params(net, p)
        lbm.lbm_nn_set_scaling(net, np.zeros(5), np.ones(5), np.ones(ch[-1]))
        yd = torch.zeros((ch[-1], n, n, n), dtype=torch.float32, device="cuda")
        lbm.lbm_nn_forward(net, torch.from_numpy(x).cuda(), yd)
        torch.cuda.synchronize()
        y = yd.cpu().numpy()
    finally:
        lbm.lbm_nn_destroy(net)
    ref16, _ = N.forward(p.astype(np.float64), ch, x.astype(np.float64), store=N.bf16)
    e16 = _rel(y, ref16)
    print(f"  forward {n}^3: max error {e16:.2e} against bf16 storage, max |y| {np.abs(ref16).max():.3f}", flush=True)
    assert e16 < 5e-3


def test_loss_and_gradients_match_reference():
    lbm = _lbm()
    shape = (8, 4, 64)
    p = _params(3)
    x = _fields(shape, 4)
    t = x + 0.3 * OUT[:, None, None, None] * np.random.default_rng(5).normal(size=x.shape)
    x, t = (a.astype(np.float32).astype(np.float64) for a in (x, t))  # what the library receives
    n = lbm.lbm_nn_create(CH, shape[::-1])
    try:
        lbm.lbm_nn_set_params(n, p.astype(np.float32))
        lbm.lbm_nn_set_scaling(n, MEAN, STD, OUT)
        lbm.lbm_nn_zero_grad(n)
        loss = lbm.lbm_nn_loss_backward(n, torch.from_numpy(x.astype(np.float32)).cuda(),
                                        torch.from_numpy(t.astype(np.float32)).cuda())
        g = lbm.lbm_nn_get_grads(n).astype(np.float64)
    finally:
        lbm.lbm_nn_destroy(n)
    l16, g16 = N.loss_and_grad(p, CH, x, t, MEAN, STD, store=N.bf16, out_std=OUT)
    l64, g64 = N.loss_and_grad(p, CH, x, t, MEAN, STD, out_std=OUT)
    print(f"  loss {loss:.6e}, bf16-storage reference {l16:.6e}, FP64 reference {l64:.6e}", flush=True)
    assert loss == pytest.approx(l16, rel=1e-4)
    assert loss == pytest.approx(l64, rel=2e-2)
    cos = lambda a, b: float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
    off = 0
    for l in range(len(CH) - 1):
        for size, name in ((27 * CH[l] * CH[l + 1], "W"), (CH[l + 1], "b")):
            sl = slice(off, off + size)
            off += size
            a = g[sl]
            print(f"  layer {l} {name}: against bf16 storage max error {_rel(a, g16[sl]):.2e} cosine "
                  f"{cos(a, g16[sl]):.7f}; against FP64 max error {_rel(a, g64[sl]):.2e} cosine "
                  f"{cos(a, g64[sl]):.6f}", flush=True)
            # same roundings: only the accumulation order differs
            assert cos(a, g16[sl]) > 0.99999 and _rel(a, g16[sl]) < 1e-2
            # the format itself: the input layer's gradient is a sum of
            # products of uncorrelated fields and loses most to the bf16
            # gradients passed down three layers
            assert cos(a, g64[sl]) > 0.995


def test_adam_step_matches_reference():
    lbm = _lbm()
    shape = (4, 4, 32)
    p = _params(6)
    x = _fields(shape, 7)
    t = x * 1.01
    n = lbm.lbm_nn_create(CH, shape[::-1])
    try:
        lbm.lbm_nn_set_params(n, p.astype(np.float32))
        lbm.lbm_nn_set_scaling(n, MEAN, STD)
        lbm.lbm_nn_zero_grad(n)
        lbm.lbm_nn_loss_backward(n, torch.from_numpy(x.astype(np.float32)).cuda(),
                                 torch.from_numpy(t.astype(np.float32)).cuda())
        g = lbm.lbm_nn_get_grads(n).astype(np.float64)
        lbm.lbm_nn_adam_step(n, 1e-3, 0.9, 0.999, 1e-8, 0.5, 1)
        lbm.lbm_nn_adam_step(n, 1e-3, 0.9, 0.999, 1e-8, 0.5, 2)
        q = lbm.lbm_nn_get_params(n).astype(np.float64)
    finally:
        lbm.lbm_nn_destroy(n)
    ref = p.astype(np.float32).astype(np.float64)
    m, v = np.zeros_like(ref), np.zeros_like(ref)
    for step in (1, 2):
        N.adam_step(ref, 0.5 * g, m, v, 1e-3, 0.9, 0.999, 1e-8, step)
    assert np.abs(q - ref).max() < 1e-6


def test_training_reduces_the_loss():
    """A target that is a fixed smooth function of the input: the network
    learns it (the loss falls tenfold in 150 Adam steps on one sample set; the
    FP64 reference network trained the same way falls from 6.5e-3 to 1.5e-4)."""
    lbm = _lbm()
    shape = (8, 8, 32)
    xs, ts = [], []
    for s in range(4):
        rho, u, T = I.smooth_random(3, shape[::-1], seed=30 + s, u_amp=0.1)
        x = np.concatenate([rho[None], u, T[None]])
        t = x.copy()
        t[4] += 0.3 * STD[4] * np.tanh((x[0] - 1.0) / STD[0])  # T nudged by the local density
        t[1] += 0.3 * STD[1] * (np.roll(x[2], 1, axis=2) - x[2]) / STD[2]
        xs.append(torch.from_numpy(x.astype(np.float32)).cuda())
        ts.append(torch.from_numpy(t.astype(np.float32)).cuda())
    n = lbm.lbm_nn_create(CH, shape[::-1])
    try:
        lbm.lbm_nn_set_params(n, _params(8, gain=0.5).astype(np.float32))
        lbm.lbm_nn_set_scaling(n, MEAN, STD)
        losses = []
        for it in range(1, 151):
            lbm.lbm_nn_zero_grad(n)
            losses.append(sum(lbm.lbm_nn_loss_backward(n, x, t) for x, t in zip(xs, ts)) / len(xs))
            lbm.lbm_nn_adam_step(n, 2e-3, 0.9, 0.999, 1e-8, 1.0 / len(xs), it)
        print(f"  loss {losses[0]:.3e} -> {losses[-1]:.3e}", flush=True)
        assert losses[-1] < 0.1 * losses[0]
        # asynchronous losses: the device-side sum equals the synchronous ones
        lbm.lbm_nn_zero_grad(n)
        sync = [lbm.lbm_nn_loss_backward(n, x, t) for x, t in zip(xs, ts)]
        g_sync = lbm.lbm_nn_get_grads(n)
        lbm.lbm_nn_zero_grad(n)
        assert all(lbm.lbm_nn_loss_backward(n, x, t, sync=False) is None for x, t in zip(xs, ts))
        total, count = lbm.lbm_nn_take_loss(n)
        assert count == len(xs)
        assert total == pytest.approx(sum(sync), rel=1e-13)
        assert np.array_equal(lbm.lbm_nn_get_grads(n), g_sync)  # same gradients either way
        assert lbm.lbm_nn_take_loss(n) == (0.0, 0)
    finally:
        lbm.lbm_nn_destroy(n)


@pytest.mark.parametrize("fp32", [False, True])
def test_fields_add_matches_reference(fp32):
    """The state changes by f^eq(new) - f^eq(old) (and g likewise) node by
    node, computed here by the oracle's nodal equilibria from the moments of
    the oracle's own run of the same 5 steps; the new moments are the old
    ones plus the increments."""
    lbm = _lbm()
    dims = (6, 5, 4)
    rho, u, T = I.smooth_random(3, dims, seed=9, u_amp=0.05)
    h = lbm.lbm_create(3, dims, 1.4, 0.7, 0.02, precision=lbm.LBM_FP32_DEV if fp32 else lbm.LBM_FP64,
                       visc_exponent=0.76, T_ref=0.15)
    r = np.random.default_rng(10)
    drho = 0.01 * r.normal(size=rho.shape)
    du = 0.01 * r.normal(size=u.shape)
    dT = 0.002 * r.normal(size=T.shape)
    try:
        lbm.lbm_init_fields(h, rho, u, T)
        lbm.lbm_step(h, 5)  # some non-equilibrium content
        nb = lbm.lbm_state_bytes(h)
        before = np.zeros(nb // (4 if fp32 else 8), dtype=np.float32 if fp32 else np.float64)
        lbm.lbm_get_state(h, before)
        m0 = [np.zeros(a.shape) for a in (rho, u, T)]
        lbm.lbm_moments(h, *m0)
        lbm.lbm_fields_add(h, drho, du, dT)
        after = np.zeros_like(before)
        lbm.lbm_get_state(h, after)
        m1 = [np.zeros(a.shape) for a in (rho, u, T)]
        lbm.lbm_moments(h, *m1)
    finally:
        lbm.lbm_destroy(h)
    Q, Nn, Cv = 27, rho.size, 2.5
    so = oracle.Sim(3, dims, gamma=1.4, Pr=0.7, mu=0.02, visc_exp=0.76, T_ref=0.15)
    so.init(rho, u, T)
    so.step(5)
    mo = so.moments()
    r0, u0, T0 = mo[0].reshape(-1), mo[1].reshape(3, -1), mo[2].reshape(-1)
    rn, un, Tn = r0 + drho.reshape(-1), u0 + du.reshape(3, -1), T0 + dT.reshape(-1)
    ref = np.zeros((2 * Q, Nn))
    for k in range(Nn):
        ref[:Q, k] = oracle.feq(3, rn[k], un[:, k], Tn[k]) - oracle.feq(3, r0[k], u0[:, k], T0[k])
        ref[Q:, k] = oracle.geq(3, rn[k], un[:, k], Tn[k], Cv) - oracle.geq(3, r0[k], u0[:, k], T0[k], Cv)
    got = after.astype(np.float64).reshape(2 * Q, Nn) - before.astype(np.float64).reshape(2 * Q, Nn)
    if fp32:  # one rounding of each stored float
        tol = 1e-6 * np.abs(ref).max() + 2.0 ** -23 * np.abs(after).max()
    else:
        tol = 1e-12 * np.abs(ref).max()
    e = float(np.abs(got - ref).max())
    print(f"  state increment error {e:.2e} (bound {tol:.2e})", flush=True)
    assert e <= tol
    mt = 2e-6 if fp32 else 1e-13
    assert np.abs(m1[0] - (m0[0] + drho)).max() < mt
    assert np.abs(m1[1] - (m0[1] + du)).max() < mt
    assert np.abs(m1[2] - (m0[2] + dT)).max() < mt


@pytest.mark.parametrize("D", [2, 3])
def test_filter_moments_matches_reference(D):
    lbm = _lbm()
    dims = (16, 12, 8) if D == 3 else (16, 12)
    rho, u, T = I.smooth_random(D, dims, seed=11, u_amp=0.05)
    h = lbm.lbm_create(D, dims, 1.4, 0.7, 0.02)
    try:
        lbm.lbm_init_fields(h, rho, u, T)
        lbm.lbm_step(h, 3)
        mom = [np.zeros(a.shape) for a in (rho, u, T)]
        lbm.lbm_moments(h, *mom)
        f = 4
        cshape = (dims[2] // f if D == 3 else 1, dims[1] // f, dims[0] // f)
        out = (np.zeros(cshape), np.zeros((D,) + cshape), np.zeros(cshape))
        lbm.lbm_filter_moments(h, f, *out)
    finally:
        lbm.lbm_destroy(h)
    so = oracle.Sim(D, dims, gamma=1.4, Pr=0.7, mu=0.02)
    so.init(rho, u, T)
    so.step(3)
    ref = N.box_filter(*so.moments(), 4, 2.5)  # the oracle's filter of the oracle's own run
    for a, b in zip(out, ref):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_correct_adds_the_network_output():
    """lbm_nn_correct = moments -> network -> increments out_std * y -> fields_add."""
    lbm = _lbm()
    dims = (32, 8, 4)
    rho, u, T = I.smooth_random(3, dims, seed=12, u_amp=0.05)
    h = lbm.lbm_create(3, dims, 1.4, 0.7, 0.02, precision=lbm.LBM_FP32_DEV, visc_exponent=0.76, T_ref=0.15)
    n = lbm.lbm_nn_create(CH, dims)
    try:
        lbm.lbm_nn_set_params(n, (0.3 * _params(13)).astype(np.float32))
        lbm.lbm_nn_set_scaling(n, MEAN, STD, OUT)
        lbm.lbm_init_fields(h, rho, u, T)
        lbm.lbm_step(h, 2)
        before = [np.zeros(a.shape) for a in (rho, u, T)]
        lbm.lbm_moments(h, *before)
        x = np.concatenate([before[0][None], before[1], before[2][None]]).astype(np.float32)
        yd = torch.zeros(x.shape, dtype=torch.float32, device="cuda")
        lbm.lbm_nn_forward(n, torch.from_numpy(x).cuda(), yd)
        torch.cuda.synchronize()
        y = yd.cpu().numpy().astype(np.float64)
        lbm.lbm_nn_correct(n, h)
        after = [np.zeros(a.shape) for a in (rho, u, T)]
        lbm.lbm_moments(h, *after)
    finally:
        lbm.lbm_nn_destroy(n)
        lbm.lbm_destroy(h)
    assert np.abs(after[0] - (before[0] + OUT[0] * y[0])).max() < 1e-6
    assert np.abs(after[1] - (before[1] + OUT[1:4, None, None, None] * y[1:4])).max() < 1e-6
    assert np.abs(after[2] - (before[2] + OUT[4] * y[4])).max() < 1e-7
    assert np.abs(y).max() > 1e-3 and np.abs(OUT[4] * y[4]).max() > 1e-6  # not trivially zero


def test_velocity_only_network_loss_gradients_and_correction():
    """A 5 -> 3 network with output offset 1 (it corrects u only): loss and
    gradients against the bf16-storage reference, and lbm_nn_correct leaves
    rho and T unchanged."""
    lbm = _lbm()
    ch = [5, 32, 32, 3]
    shape = (4, 8, 32)
    p = _params(15, channels=ch)
    x = _fields(shape, 16)
    t = x + 0.3 * OUT[:, None, None, None] * np.random.default_rng(17).normal(size=x.shape)
    x, t = (a.astype(np.float32).astype(np.float64) for a in (x, t))
    n = lbm.lbm_nn_create(ch, shape[::-1])
    try:
        lbm.lbm_nn_set_params(n, p.astype(np.float32))
        lbm.lbm_nn_set_scaling(n, MEAN, STD, OUT[1:4])
        lbm.lbm_nn_set_output_offset(n, 1)
        lbm.lbm_nn_zero_grad(n)
        loss = lbm.lbm_nn_loss_backward(n, torch.from_numpy(x.astype(np.float32)).cuda(),
                                        torch.from_numpy(t.astype(np.float32)).cuda())
        g = lbm.lbm_nn_get_grads(n).astype(np.float64)
        l16, g16 = N.loss_and_grad(p, ch, x, t, MEAN, STD, store=N.bf16, out_std=OUT[1:4], out_offset=1)
        print(f"  loss {loss:.6e} reference {l16:.6e}", flush=True)
        assert loss == pytest.approx(l16, rel=1e-4)
        assert float(g @ g16 / (np.linalg.norm(g) * np.linalg.norm(g16))) > 0.99999
        with pytest.raises(lbm.LbmError):
            lbm.lbm_nn_set_output_offset(n, 3)  # 3 + 3 outputs > 5 fields
        dims = shape[::-1]
        rho, u, T = I.smooth_random(3, dims, seed=18, u_amp=0.05)
        h = lbm.lbm_create(3, dims, 1.4, 0.7, 0.02, precision=lbm.LBM_FP32_DEV, visc_exponent=0.76, T_ref=0.15)
        try:
            lbm.lbm_init_fields(h, rho, u, T)
            lbm.lbm_step(h, 2)
            before = [np.zeros(a.shape) for a in (rho, u, T)]
            lbm.lbm_moments(h, *before)
            lbm.lbm_nn_correct(n, h)
            after = [np.zeros(a.shape) for a in (rho, u, T)]
            lbm.lbm_moments(h, *after)
        finally:
            lbm.lbm_destroy(h)
    finally:
        lbm.lbm_nn_destroy(n)
    assert np.abs(after[0] - before[0]).max() < 1e-6
    assert np.abs(after[2] - before[2]).max() < 1e-7
    assert np.abs(after[1] - before[1]).max() > 1e-5


def test_fields_set_replaces_the_moments_and_keeps_the_rest():
    """lbm_fields_set: the moments become the given fields and the state moves
    by f^eq(new) - f^eq(old) (g likewise), so the non-equilibrium part stays."""
    lbm = _lbm()
    dims = (6, 5, 4)
    rho, u, T = I.smooth_random(3, dims, seed=19, u_amp=0.05)
    r2, u2, T2 = I.smooth_random(3, dims, seed=20, u_amp=0.05)
    h = lbm.lbm_create(3, dims, 1.4, 0.7, 0.02)
    try:
        lbm.lbm_init_fields(h, rho, u, T)
        lbm.lbm_step(h, 5)
        before = np.zeros(lbm.lbm_state_bytes(h) // 8)
        lbm.lbm_get_state(h, before)
        m0 = [np.zeros(a.shape) for a in (rho, u, T)]
        lbm.lbm_moments(h, *m0)
        lbm.lbm_fields_set(h, r2, u2, T2)
        after = np.zeros_like(before)
        lbm.lbm_get_state(h, after)
        m1 = [np.zeros(a.shape) for a in (rho, u, T)]
        lbm.lbm_moments(h, *m1)
        with pytest.raises(lbm.LbmError):  # a non-positive temperature is refused, nothing changes
            lbm.lbm_fields_set(h, r2, u2, -T2)
        again = np.zeros_like(before)
        lbm.lbm_get_state(h, again)
    finally:
        lbm.lbm_destroy(h)
    for a, b in zip(m1, (r2, u2, T2)):
        assert np.abs(a - b).max() <= 1e-13
    Q, Nn = 27, rho.size
    so = oracle.Sim(3, dims, gamma=1.4, Pr=0.7, mu=0.02)
    so.init(rho, u, T)
    so.step(5)
    mo = so.moments()  # the old moments, from the oracle's own run
    ref = np.zeros((2 * Q, Nn))
    o0, o1 = mo[1].reshape(3, -1), u2.reshape(3, -1)
    for k in range(Nn):
        ro, rn = mo[0].reshape(-1)[k], r2.reshape(-1)[k]
        to, tn = mo[2].reshape(-1)[k], T2.reshape(-1)[k]
        ref[:Q, k] = oracle.feq(3, rn, o1[:, k], tn) - oracle.feq(3, ro, o0[:, k], to)
        ref[Q:, k] = oracle.geq(3, rn, o1[:, k], tn, 2.5) - oracle.geq(3, ro, o0[:, k], to, 2.5)
    got = (after - before).reshape(2 * Q, Nn)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.array_equal(again, after)


def test_fields_to_planes_and_correction_limit():
    """FP64 fields -> FP32 planes is a plain conversion; with a limit of 0.5
    no correction exceeds 0.5 out_std, without one the same network moves a
    field further."""
    lbm = _lbm()
    dims = (32, 4, 4)
    rho, u, T = I.smooth_random(3, dims, seed=21, u_amp=0.05)
    d = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (rho, u, T)]
    x = torch.empty((5, rho.size), dtype=torch.float32, device="cuda")
    lbm.lbm_nn_fields_to_planes(3, *d, x)
    torch.cuda.synchronize()
    ref = np.concatenate([rho.reshape(1, -1), u.reshape(3, -1), T.reshape(1, -1)]).astype(np.float32)
    assert np.array_equal(x.cpu().numpy(), ref)
    ch = [5, 32, 3]
    n = lbm.lbm_nn_create(ch, dims)
    deltas = []
    try:
        lbm.lbm_nn_set_params(n, (3.0 * _params(22, channels=ch)).astype(np.float32))  # large outputs
        lbm.lbm_nn_set_scaling(n, MEAN, STD, OUT[1:4])
        lbm.lbm_nn_set_output_offset(n, 1)
        for limit in (0.5, 0.0):
            lbm.lbm_nn_set_correction_limit(n, limit)
            h = lbm.lbm_create(3, dims, 1.4, 0.7, 0.02, precision=lbm.LBM_FP32_DEV, T_ref=0.15)
            try:
                lbm.lbm_init_fields(h, rho, u, T)
                lbm.lbm_nn_correct(n, h)
                m = [np.zeros(a.shape) for a in (rho, u, T)]
                lbm.lbm_moments(h, *m)
            finally:
                lbm.lbm_destroy(h)
            deltas.append(np.abs(m[1] - u).reshape(3, -1).max(axis=1))
        with pytest.raises(lbm.LbmError):
            lbm.lbm_nn_set_correction_limit(n, -1.0)
    finally:
        lbm.lbm_nn_destroy(n)
    assert np.all(deltas[0] <= 0.5 * OUT[1:4] * (1 + 1e-4) + 1e-7)
    assert np.any(deltas[1] > 0.5 * OUT[1:4] * 1.01)
