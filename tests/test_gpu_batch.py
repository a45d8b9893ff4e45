"""Batches of independent boxes stepped by one launch per step: every box must
end exactly where lbm_step takes it (same kernel body and parameters), with
and without HIP-graph replay, across replays interleaved with the program's
own work, after the autotuner, and when boxes are also stepped on their own."""
import numpy as np
import pytest

from paper_2102_09512_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lbm():
    from paper_2102_09512_amd import lbm

    return lbm


def _boxes_2d(count, seed0=0):
    """Uneven, resolved boxes (the spectral peak has at least 16 nodes per
    wavelength) at subsonic turbulent Mach numbers."""
    sizes = tuple(range(64, 161, 32))
    boxes = []
    for s in range(count):
        r = np.random.default_rng(seed0 + s)
        nx, ny = int(r.choice(sizes)), int(r.choice(sizes))
        ma = float(r.uniform(0.1, 0.4))
        rho, u, T = I.turbulence_box2d(nx, ny, seed=seed0 + s, Ma_t=ma, T0=0.15)
        boxes.append(dict(dims=(nx, ny), fields=(rho, u, T), mu=I.taylor_viscosity(u[:, 0])))
    return boxes


def _make(lbm, boxes, precision, D=2):
    hs = []
    for b in boxes:
        dims = b["dims"] if D == 2 else b["dims"]
        h = lbm.lbm_create(D, dims, 1.4, 0.7, b["mu"], precision=precision, visc_exponent=0.76, T_ref=0.15)
        lbm.lbm_set_stream(h, torch.cuda.current_stream())
        lbm.lbm_init_fields(h, *(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in b["fields"]))
        hs.append(h)
    return hs


def _states(lbm, hs, fp32):
    out = []
    for h in hs:
        nb = lbm.lbm_state_bytes(h)
        t = torch.empty(nb // (4 if fp32 else 8), dtype=torch.float32 if fp32 else torch.float64, device="cuda")
        lbm.lbm_get_state(h, t)
        torch.cuda.synchronize()
        out.append(t.cpu().numpy())
    return out


def _same(a, b):
    for x, y in zip(a, b):
        assert np.isfinite(x).all() and np.isfinite(y).all(), "a box blew up"
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("fp32", [True, False])
def test_batch_equals_individual_steps(fp32):
    lbm = _lbm()
    prec = lbm.LBM_FP32_DEV if fp32 else lbm.LBM_FP64
    boxes = _boxes_2d(7)
    print(f"[gpu case] batch of {len(boxes)} D2Q9 boxes {[b['dims'] for b in boxes]} fp32={fp32}", flush=True)
    ref, bat = _make(lbm, boxes, prec), _make(lbm, boxes, prec)
    b = lbm.lbm_batch_create(bat)
    try:
        for h in ref:
            lbm.lbm_step(h, 37)
        lbm.lbm_batch_step(b, 37)
        assert all(lbm.lbm_step_count(h) == 37 for h in bat)
        assert _same(_states(lbm, ref, fp32), _states(lbm, bat, fp32))
    finally:
        lbm.lbm_batch_destroy(b)
        for h in ref + bat:
            lbm.lbm_destroy(h)


@pytest.mark.parametrize("fp32", [True, False])
def test_persistent_launch_equals_individual_steps(fp32):
    """The fixed-grid launch form, on a batch of more tiles than the device
    holds at once (64 x 1 tiles with 4-row chunks over three ragged boxes of
    up to a million nodes: 10,976 tiles), so that work-groups loop over
    several tiles each: every box ends bit for bit where lbm_step takes it
    with the same tile, also across graph replays."""
    lbm = _lbm()
    prec = lbm.LBM_FP32_DEV if fp32 else lbm.LBM_FP64
    dims = [(1024, 1024), (960, 1088), (1000, 700)]
    boxes = []
    for k, (nx, ny) in enumerate(dims):
        rho, u, T = I.turbulence_box2d(nx, ny, seed=80 + k, Ma_t=0.3, T0=0.15)
        boxes.append(dict(dims=(nx, ny), fields=(rho, u, T), mu=I.taylor_viscosity(u[:, 0])))
    tile = (64, 1, 4)
    print(f"[gpu case] persistent batch {dims} tile {tile} fp32={fp32}", flush=True)
    hs = []
    for lst_tile in (tile, None):
        for b in boxes:
            h = lbm.lbm_create(2, b["dims"], 1.4, 0.7, b["mu"], precision=prec, visc_exponent=0.76, T_ref=0.15,
                               tile=lst_tile)
            lbm.lbm_set_stream(h, torch.cuda.current_stream())
            lbm.lbm_init_fields(h, *(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in b["fields"]))
            hs.append(h)
    ref, bat = hs[:3], hs[3:]
    b = lbm.lbm_batch_create(bat)
    try:
        lbm.lbm_batch_set_tile(b, tile)
        lbm.lbm_batch_set_persistent(b, True)
        assert lbm.lbm_batch_get_persistent(b) and lbm.lbm_batch_get_tile(b) == tile
        lbm.lbm_batch_step(b, 5)
        lbm.lbm_batch_step(b, 12, 4)
        for h in ref:
            lbm.lbm_step(h, 17)
        assert _same(_states(lbm, ref, fp32), _states(lbm, bat, fp32))
    finally:
        lbm.lbm_batch_destroy(b)
        for h in hs:
            lbm.lbm_destroy(h)


def test_batch_graph_replays_interleaved_with_other_work():
    """Graph replays (even and odd captured lengths, remainders launched
    directly), with diagnostics, a single-box step and host synchronisation
    in between; every stage equals the individually stepped boxes."""
    lbm = _lbm()
    boxes = _boxes_2d(5, seed0=20)
    ref, bat = _make(lbm, boxes, lbm.LBM_FP32_DEV), _make(lbm, boxes, lbm.LBM_FP32_DEV)
    b = lbm.lbm_batch_create(bat)
    try:
        total = 0
        for n, g in [(10, 4), (9, 3), (12, 4), (7, 3), (5, 0)]:
            print(f"[gpu case] batch graph: {n} steps, graph of {g}", flush=True)
            lbm.lbm_batch_step(b, n, g)
            for h in ref:
                lbm.lbm_step(h, n)
            total += n
            lbm.lbm_diagnostics(bat[0])
            torch.cuda.synchronize()
            assert _same(_states(lbm, ref, True), _states(lbm, bat, True)), (n, g)
            # one box stepped on its own between batched steps
            lbm.lbm_step(bat[1], 1)
            lbm.lbm_step(ref[1], 1)
        assert lbm.lbm_step_count(bat[0]) == total and lbm.lbm_step_count(bat[1]) == total + 5
    finally:
        lbm.lbm_batch_destroy(b)
        for h in ref + bat:
            lbm.lbm_destroy(h)


@pytest.mark.parametrize("fp32", [True, False])
def test_autotuner_keeps_states_and_tuned_steps_match(fp32):
    lbm = _lbm()
    prec = lbm.LBM_FP32_DEV if fp32 else lbm.LBM_FP64
    boxes = _boxes_2d(6, seed0=40)
    ref, bat = _make(lbm, boxes, prec), _make(lbm, boxes, prec)
    b = lbm.lbm_batch_create(bat)
    try:
        lbm.lbm_batch_step(b, 3)
        for h in ref:
            lbm.lbm_step(h, 3)
        before = _states(lbm, bat, fp32)
        ms = lbm.lbm_batch_tune(b, 3)
        tile = lbm.lbm_batch_get_tile(b)
        print(f"[gpu case] tuned tile {tile}, {ms:.4f} ms per step", flush=True)
        assert tile[0] in (64, 128, 256) and tile[1] == 1 and tile[2] in (4, 8, 16, 32, 64)
        assert _same(before, _states(lbm, bat, fp32))  # tuning leaves the states alone
        lbm.lbm_batch_step(b, 20, 5)
        for h in ref:
            lbm.lbm_step(h, 20)
        for x, y in zip(_states(lbm, ref, fp32), _states(lbm, bat, fp32)):
            # another tile only changes which thread does what (rounding-level at most)
            assert np.abs(x - y).max() <= (1e-6 if fp32 else 1e-13) * np.abs(x).max()
    finally:
        lbm.lbm_batch_destroy(b)
        for h in ref + bat:
            lbm.lbm_destroy(h)


def test_batch_d3q27_uneven_boxes():
    lbm = _lbm()
    dims = [(24, 20, 18), (40, 12, 30), (13, 33, 9)]
    hs_ref, hs_bat = [], []
    for k, d in enumerate(dims):
        f = I.smooth_random(3, d, seed=60 + k, u_amp=0.05)
        for lst in (hs_ref, hs_bat):
            h = lbm.lbm_create(3, d, 1.4, 0.7, 0.02, precision=lbm.LBM_FP32_DEV, visc_exponent=0.76, T_ref=0.15)
            lbm.lbm_init_fields(h, *f)
            lst.append(h)
    b = lbm.lbm_batch_create(hs_bat)
    try:
        print("[gpu case] D3Q27 batch", dims, flush=True)
        lbm.lbm_batch_step(b, 11, 4)
        for h in hs_ref:
            lbm.lbm_step(h, 11)
        assert _same(_states(lbm, hs_ref, True), _states(lbm, hs_bat, True))
        print("[gpu case] D3Q27 batch, launch form switches", flush=True)
        lbm.lbm_batch_set_tile(b, (64, 8, 0))
        with pytest.raises(lbm.LbmError) as e:  # the fixed grid needs <= 256 work-items per tile
            lbm.lbm_batch_set_persistent(b, True)
        assert e.value.code == lbm.LBM_EINVAL
        lbm.lbm_batch_set_tile(b, (32, 8, 0))
        lbm.lbm_batch_set_persistent(b, True)
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_batch_set_tile(b, (64, 8, 0))
        assert e.value.code == lbm.LBM_EINVAL
        assert lbm.lbm_batch_get_tile(b)[:2] == (32, 8) and lbm.lbm_batch_get_persistent(b)
    finally:
        lbm.lbm_batch_destroy(b)
        for h in hs_ref + hs_bat:
            lbm.lbm_destroy(h)


@pytest.mark.parametrize("fp32,tile", [(True, (32, 8, 2)), (False, (64, 4, 2))])
def test_persistent_launch_d3q27(fp32, tile):
    """The fixed-grid form of the D3Q27 batch on about a thousand tiles (the
    device holds a few hundred 256-work-item work-groups of this kernel at
    once): bit for bit where lbm_step takes each box with the same tile."""
    lbm = _lbm()
    prec = lbm.LBM_FP32_DEV if fp32 else lbm.LBM_FP64
    dims = [(64, 64, 40), (48, 72, 36), (40, 40, 64)]
    print(f"[gpu case] D3Q27 persistent batch {dims} tile {tile} fp32={fp32}", flush=True)
    hs = []
    for t in (tile, tile):
        for k, d in enumerate(dims):
            f = I.smooth_random(3, d, seed=90 + k, u_amp=0.05)
            h = lbm.lbm_create(3, d, 1.4, 0.7, 0.02, precision=prec, visc_exponent=0.76, T_ref=0.15, tile=t)
            lbm.lbm_set_stream(h, torch.cuda.current_stream())
            lbm.lbm_init_fields(h, *f)
            hs.append(h)
    ref, bat = hs[:3], hs[3:]
    b = lbm.lbm_batch_create(bat)
    try:
        lbm.lbm_batch_set_tile(b, tile)
        lbm.lbm_batch_set_persistent(b, True)
        lbm.lbm_batch_step(b, 3)
        lbm.lbm_batch_step(b, 6, 3)
        for h in ref:
            lbm.lbm_step(h, 9)
        assert _same(_states(lbm, ref, fp32), _states(lbm, bat, fp32))
    finally:
        lbm.lbm_batch_destroy(b)
        for h in hs:
            lbm.lbm_destroy(h)


def test_batch_argument_errors():
    lbm = _lbm()
    h1 = lbm.lbm_create(2, (32, 32), 1.4, 0.7, 0.02, precision=lbm.LBM_FP32_DEV)
    h2 = lbm.lbm_create(2, (32, 32), 1.4, 0.7, 0.02, precision=lbm.LBM_FP64)
    try:
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_batch_create([h1, h2])
        assert e.value.code == lbm.LBM_EINVAL
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_batch_create([h1, h1])
        assert e.value.code == lbm.LBM_EINVAL
        b = lbm.lbm_batch_create([h1])
        try:
            with pytest.raises(lbm.LbmError) as e:
                lbm.lbm_batch_step(b, 1)
            assert e.value.code == lbm.LBM_ESTATE  # no lbm_init_fields yet
            with pytest.raises(lbm.LbmError) as e:
                lbm.lbm_batch_set_tile(b, (48, 1, 8))
            assert e.value.code == lbm.LBM_EINVAL
            assert lbm.raw().lbm_batch_set_persistent(b, 2) == lbm.LBM_EINVAL
        finally:
            lbm.lbm_batch_destroy(b)
    finally:
        lbm.lbm_destroy(h1)
        lbm.lbm_destroy(h2)


def test_full_ensemble_in_the_benchmark_configuration():
    """The benchmark's ensemble (64 D2Q9 boxes of 64^2 .. 512^2, seeds 0..63,
    FP32, autotuned tile, 50-step graphs, 1000 steps): every box ends bit for
    bit where lbm_step takes it alone with the same launch tile (another tile
    changes the rounding, which 1000 steps of turbulence amplify).  Then the
    largest and the smallest of the boxes that stay finite get a state that
    both sides build on their own (the equilibria of the box's initial
    fields, deviations rounded to FP32 as stored, plus a seeded smooth
    perturbation of every population); one more batched launch steps all 64
    boxes, and those two boxes are compared with the oracle's step at every
    node (where a velocity component is within rounding of zero, both upwind
    sides are computed by the oracle and the GPU must match one)."""
    import oracle

    lbm = _lbm()
    boxes = I.ensemble_2d(64)
    print(f"[gpu case] full ensemble: {len(boxes)} boxes, "
          f"{sum(b['dims'][0] * b['dims'][1] for b in boxes)} nodes, 1000 steps", flush=True)
    prec = lbm.LBM_FP32_DEV

    def make(tile=None):
        hs = []
        for b in boxes:
            h = lbm.lbm_create(2, b["dims"], 1.4, 0.7, b["mu"], precision=prec, visc_exponent=0.76, T_ref=0.15,
                               tile=tile)
            lbm.lbm_set_stream(h, torch.cuda.current_stream())
            lbm.lbm_init_fields(h, *(torch.from_numpy(a).cuda() for a in b["fields"]))
            hs.append(h)
        return hs

    bat = make()
    batch = lbm.lbm_batch_create(bat)
    ref = []
    try:
        lbm.lbm_batch_tune(batch, 5)
        tile = lbm.lbm_batch_get_tile(batch)
        print(f"  tuned tile {tile}", flush=True)
        ref = make(tile)  # chunk 0: each box's default chunk for the shape, as in the batch
        lbm.lbm_batch_step(batch, 1000, 50)
        for h in ref:
            lbm.lbm_step(h, 1000)
        torch.cuda.synchronize()
        finite = []
        for i, (a, b) in enumerate(zip(ref, bat)):
            nb = lbm.lbm_state_bytes(a) // 4
            sa = torch.empty(nb, dtype=torch.float32, device="cuda")
            sb = torch.empty(nb, dtype=torch.float32, device="cuda")
            lbm.lbm_get_state(a, sa)
            lbm.lbm_get_state(b, sb)
            torch.cuda.synchronize()
            # bit patterns: boxes that left the stable range hold NaNs, which must match too
            assert torch.equal(sa.view(torch.int32), sb.view(torch.int32)), f"box {i} {boxes[i]['dims']}"
            finite.append(bool(torch.isfinite(sa).all()))
        print(f"  {finite.count(False)} of {len(boxes)} boxes left the stable range (the method's limit at this "
              f"resolution and Mach number, also in the oracle)", flush=True)
        areas = [b["dims"][0] * b["dims"][1] if ok else 0 for b, ok in zip(boxes, finite)]
        small = [a if a else 1 << 40 for a in areas]
        picks = [int(np.argmax(areas)), int(np.argmin(small))]
        rho0, T0 = float(np.float32(1.0)), float(np.float32(0.15))
        rest = np.concatenate([np.asarray(oracle.feq(2, rho0, [0.0, 0.0, 0.0], T0)),
                               np.asarray(oracle.geq(2, rho0, [0.0, 0.0, 0.0], T0, 2.5))])
        sims = {}
        for i in picks:
            (nx, ny), N = boxes[i]["dims"], boxes[i]["dims"][0] * boxes[i]["dims"][1]
            pert = I.PopulationPerturbation((nx, ny), seed=100 + i, amp=2e-3)
            # GPU: the box's own init, then the perturbation added in FP32
            h = bat[i]
            lbm.lbm_init_fields(h, *(torch.from_numpy(a).cuda() for a in boxes[i]["fields"]))
            dev = torch.empty(lbm.lbm_state_bytes(h) // 4, dtype=torch.float32, device="cuda")
            lbm.lbm_get_state(h, dev)
            st = dev.view(18, N)
            for q in range(18):
                st[q] += torch.from_numpy(pert.row(q).astype(np.float32)).cuda()
            lbm.lbm_set_state(h, dev, step=1000)
            # oracle: its own init, deviations rounded to FP32, the same FP32 addition
            s = oracle.Sim(2, (nx, ny), gamma=1.4, Pr=0.7, mu=boxes[i]["mu"], visc_exp=0.76, T_ref=0.15)
            s.init(*boxes[i]["fields"])
            f, g = s.get_pops()
            full = np.concatenate([f.reshape(9, N), g.reshape(9, N)])
            for q in range(18):
                d32 = (full[q] - rest[q]).astype(np.float32)
                d32 += pert.row(q).astype(np.float32)
                full[q] = rest[q] + d32.astype(np.float64)
            s.set_pops(full[:9], full[9:], 1000)
            sims[i] = (s, N)
        lbm.lbm_batch_step(batch, 1)  # one launch over all 64 boxes
        torch.cuda.synchronize()
        for i in picks:
            s, N = sims[i]
            h = bat[i]
            dev = torch.empty(lbm.lbm_state_bytes(h) // 4, dtype=torch.float32, device="cuda")
            lbm.lbm_get_state(h, dev)
            torch.cuda.synchronize()
            after = dev.cpu().numpy().reshape(18, N).astype(np.float64)
            nodes = np.arange(N, dtype=np.int64)
            f_ref, g_ref = s.step_sampled(nodes)
            ref_pops = np.concatenate([f_ref, g_ref]) - rest[:, None]
            c = oracle.velocities(2)
            u = (c.T[:2] @ f_ref) / f_ref.sum(axis=0)
            amb = np.nonzero((np.abs(u) <= 1e-7).any(axis=0))[0]
            scale = np.abs(ref_pops).max(axis=1, keepdims=True)
            err = (np.abs(after - ref_pops) / scale).max(axis=0)
            for k in amb:  # either upwind side at these nodes
                axes = np.nonzero(np.abs(u[:, k]) <= 1e-7)[0]
                best = err[k]
                for combo in range(1 << axes.size):
                    br = -np.ones((1, 2), dtype=np.int8)
                    for j, a in enumerate(axes):
                        br[0, a] = (combo >> j) & 1
                    fa, ga = s.step_sampled_branch(nodes[k:k + 1], br)
                    alt = np.concatenate([fa[:, 0], ga[:, 0]]) - rest
                    best = min(best, float((np.abs(after[:, k] - alt) / scale[:, 0]).max()))
                err[k] = best
            print(f"  box {i} {boxes[i]['dims']}: one batched step from an independently built state, max error "
                  f"{err.max():.2e} over all {N} nodes ({amb.size} with a velocity component within rounding of "
                  f"zero)", flush=True)
            assert err.max() <= 1e-5
    finally:
        lbm.lbm_batch_destroy(batch)
        for h in ref + bat:
            lbm.lbm_destroy(h)
