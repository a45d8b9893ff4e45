"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on
the same seeded inputs.  FP64 storage must agree to 1e-12 relative
(per field, max-norm error over max-norm value) after 100 steps; FP32
deviation storage to 1e-5."""
import math

import numpy as np
import pytest

import oracle
import oracle_floor
from paper_2102_09512_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lbm():
    from paper_2102_09512_amd import lbm

    return lbm


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def run_gpu(D, dims, fields, steps, mu, Pr=0.71, gamma=1.4, fp32=False, bc=(0, 0, 0), visc_exp=0.0, T_ref=0.15,
            deriv=0, device_io=True, tile=None, want_state=True, want_diag=False, u_ref=None, cv=None):
    lbm = _lbm()
    print(f"[gpu case] D={D} dims={dims} steps={steps} fp32={fp32} bc={bc} deriv={deriv} tile={tile} "
          f"io={'device' if device_io else 'host'}", flush=True)
    rho, u, T = fields
    h = lbm.lbm_create(D, dims, gamma, Pr, mu, precision=lbm.LBM_FP32_DEV if fp32 else lbm.LBM_FP64, bc=bc,
                       visc_exponent=visc_exp, T_ref=T_ref, rho_ref=1.0, deriv_scheme=deriv, tile=tile, u_ref=u_ref,
                       cv_poly=cv)
    try:
        lbm.lbm_set_stream(h, torch.cuda.current_stream())
        if device_io:
            lbm.lbm_init_fields(h, *(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (rho, u, T)))
        else:
            lbm.lbm_init_fields(h, rho, u, T)
        lbm.lbm_step(h, steps)
        if device_io:
            out = [torch.zeros(a.shape, dtype=torch.float64, device="cuda") for a in (rho, u, T)]
            lbm.lbm_moments(h, *out)
            torch.cuda.synchronize()
            out = [o.cpu().numpy() for o in out]
        else:
            out = [np.zeros_like(a) for a in (rho, u, T)]
            lbm.lbm_moments(h, *out)
        state = None
        if want_state:
            state = np.zeros(lbm.lbm_state_bytes(h) // (4 if fp32 else 8), dtype=np.float32 if fp32 else np.float64)
            lbm.lbm_get_state(h, state)
        diag = lbm.lbm_diagnostics(h) if want_diag else None
        assert lbm.lbm_step_count(h) == steps
    finally:
        lbm.lbm_destroy(h)
    return out, state, diag


def run_oracle(D, dims, fields, steps, mu, Pr=0.71, gamma=1.4, bc=(0, 0, 0), visc_exp=0.0, T_ref=0.15, deriv=0,
               cv=None):
    s = oracle.Sim(D, dims, gamma=gamma, Pr=Pr, mu=mu, visc_exp=visc_exp, T_ref=T_ref, bc=bc, deriv=deriv, cv=cv)
    s.init(*fields)
    s.step(steps)
    return s


def check_fields(out, s, tol):
    ref = s.moments()
    errs = {n: rel(a, b) for n, a, b in zip(("rho", "u", "T"), out, ref)}
    print("  field errors", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for n, e in errs.items():
        assert e <= tol, (n, e)
    return errs


def check_fp32_with_floor(D, dims, fields, steps, out, s, u_ref=None, T_ref=0.15, **kw):
    """FP32 fields within 1e-5 of the oracle, or within twice the case's FP32
    floor where that is larger: the larger departure from the plain oracle of
    the oracle's FP32 storage model and (upwind scheme) of its run with every
    upwind decision within the FP32 resolution of the velocity reversed
    (tests/oracle_floor.py).  Near a shock, or where the sign of a velocity
    component picks the upwind side, a flow can carry FP32-level differences
    beyond 1e-5 within 100 steps."""
    okw = {k: v for k, v in kw.items() if k in ("mu", "Pr", "gamma", "bc", "visc_exp", "deriv", "cv")}
    ref = s.moments()
    fs = oracle_floor.storage_run(D, dims, fields, steps, rho_ref=1.0, u_ref=u_ref, T_ref=T_ref, **okw)
    floor = oracle_floor.field_errors(fs.moments(), ref)
    if kw.get("deriv", 0) == 0:
        band = oracle_floor.velocity_resolution(fields[1])
        fb = oracle_floor.band_run(D, dims, fields, steps, band, T_ref=T_ref, **okw)
        fl_b = oracle_floor.field_errors(fb.moments(), ref)
        floor = {k: max(floor[k], fl_b[k]) for k in floor}
    errs = oracle_floor.field_errors(out, ref)
    vs_model = oracle_floor.field_errors(out, fs.moments())
    print("  FP32 field errors", {k: f"{v:.2e}" for k, v in errs.items()},
          "floor", {k: f"{v:.2e}" for k, v in floor.items()},
          "vs FP32-storage oracle", {k: f"{v:.2e}" for k, v in vs_model.items()}, flush=True)
    for n in errs:
        assert errs[n] <= max(1e-5, 2.0 * floor[n]), (n, errs[n], floor[n])


def check_pops(state, s, tol):
    f, g = s.get_pops()
    ref = np.concatenate([f.ravel(), g.ravel()])
    e = float(np.abs(state - ref).max() / np.abs(ref).max())
    print(f"  population error {e:.2e}", flush=True)
    assert e <= tol
    return e


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("D,dims", [(2, (37, 29)), (3, (13, 11, 9))])
def test_init_equals_oracle_equilibria(D, dims):
    f = I.smooth_random(D, dims, seed=11, u_amp=0.1)
    out, state, _ = run_gpu(D, dims, f, 0, mu=0.02)
    s = run_oracle(D, dims, f, 0, mu=0.02)
    check_pops(state, s, 2e-16 * 8)
    check_fields(out, s, 1e-15)


@pytest.mark.parametrize("D,dims,tile", [
    (2, (70, 45), None),            # ragged x tile, 2 y-chunks
    (2, (300, 33), (256, 1, 7)),    # ragged march chunks
    (3, (24, 20, 18), None),        # ragged in x, y and z
    (3, (70, 9, 5), (32, 8, 2)),    # ragged y tiles (8 + 1 rows), three x tiles
    (3, (13, 40, 33), (32, 8, 32)),
])
def test_fp64_periodic_turbulence_100_steps(D, dims, tile):
    n = max(dims)
    rho, u, T = I.turbulence(D, n, seed=5, Ma_t=0.4)
    if D == 3:
        f = (rho[: dims[2], : dims[1], : dims[0]], u[:, : dims[2], : dims[1], : dims[0]],
             T[: dims[2], : dims[1], : dims[0]])
    else:
        f = (rho[:, : dims[1], : dims[0]], u[:, :, : dims[1], : dims[0]], T[:, : dims[1], : dims[0]])
    f = tuple(np.ascontiguousarray(a) for a in f)
    kw = dict(mu=0.02, Pr=0.7, visc_exp=0.76, T_ref=0.15)
    out, state, _ = run_gpu(D, dims, f, 100, tile=tile, **kw)
    s = run_oracle(D, dims, f, 100, **kw)
    check_fields(out, s, 1e-12)
    check_pops(state, s, 1e-12)


def test_fp64_mixed_boundaries_3d():
    dims = (20, 16, 22)
    f = I.smooth_random(3, dims, seed=2, u_amp=0.08)
    kw = dict(mu=0.015, Pr=0.75, bc=(1, 0, 1))
    out, state, _ = run_gpu(3, dims, f, 100, device_io=False, **kw)
    s = run_oracle(3, dims, f, 100, **kw)
    check_fields(out, s, 1e-12)
    check_pops(state, s, 1e-12)


@pytest.mark.parametrize("D", [2, 3])
def test_fp64_central_difference_variant(D):
    dims = (30, 20) if D == 2 else (16, 14, 12)
    f = I.smooth_random(D, dims, seed=4, u_amp=0.1)
    kw = dict(mu=0.02, Pr=0.71, deriv=1)
    out, state, _ = run_gpu(D, dims, f, 100, **kw)
    s = run_oracle(D, dims, f, 100, **kw)
    check_fields(out, s, 1e-12)
    check_pops(state, s, 1e-12)


def test_fp64_sod_shock_tube():
    """Sod shock tube in the lattice scaling of Sec. III.B: 800 x 4, x zero-gradient, y periodic."""
    f = I.sod(800, 4, T_left=0.15)
    kw = dict(mu=0.015, Pr=0.71, bc=(1, 0, 0))
    for steps, tol in ((100, 1e-12), (1000, 1e-10)):
        out, state, _ = run_gpu(2, (800, 4), f, steps, **kw)
        s = run_oracle(2, (800, 4), f, steps, **kw)
        check_fields(out, s, tol)
        check_pops(state, s, tol)


def test_fp64_shock_vortex_crop():
    rho, u, T, rh = I.shock_vortex(256, 128, r_v=16.0, x_s=128)
    f = (rho, u, T)
    kw = dict(mu=0.0198, Pr=0.75, bc=(1, 0, 0))
    out, state, _ = run_gpu(2, (256, 128), f, 100, **kw)
    s = run_oracle(2, (256, 128), f, 100, **kw)
    check_fields(out, s, 1e-12)
    check_pops(state, s, 1e-12)


def test_fp32_deviation_turbulence_3d_central():
    """FP32 deviation storage vs the FP64 oracle, 100 steps of Ma_t = 0.5
    turbulence (32^3 periodic, a violent case: the large-eddy turnover is 24
    steps), central anomaly differences (no branch)."""
    n = 32
    f = I.turbulence(3, n, seed=0, Ma_t=0.5, T0=0.15)
    mu = I.turbulence_viscosity(n, Ma_t=0.5, T0=0.15)
    kw = dict(mu=mu, Pr=0.7, visc_exp=0.76, T_ref=0.15, deriv=1)
    out, _, _ = run_gpu(3, (n, n, n), f, 100, fp32=True, want_state=False, **kw)
    s = run_oracle(3, (n, n, n), f, 100, **kw)
    check_fields(out, s, 1e-5)


@pytest.mark.parametrize("u_ref", [None, (0.1, 0.1, 0.1)])
def test_fp32_deviation_upwind_without_sign_changes(u_ref):
    """FP32 deviation storage vs the FP64 oracle with the upwind anomaly
    difference, on a flow whose velocity components stay away from zero
    (mean flow 0.1 + perturbations of at most 0.05), so both runs take the
    same upwind branches (see test_fp32_upwind_sign_ambiguity); deviations
    from the rest state and from the mean-flow state."""
    dims = (40, 36, 32)
    rho, u, T = I.smooth_random(3, dims, seed=6, rho_amp=0.05, u_amp=0.05, T_amp=0.02)
    u = u + 0.1
    kw = dict(mu=0.01, Pr=0.7, visc_exp=0.76, T_ref=0.15)
    out, _, _ = run_gpu(3, dims, (rho, u, T), 100, fp32=True, want_state=False, u_ref=u_ref, **kw)
    s = run_oracle(3, dims, (rho, u, T), 100, **kw)
    assert np.abs(s.moments()[1]).min() > 1e-3
    check_fields(out, s, 1e-5)


def test_fp32_upwind_sign_ambiguity():
    """Without a mean flow some node eventually has |u_a| at the FP32 rounding
    level, where the FP32 and FP64 runs may take different upwind branches
    (both valid readings of the sign test of Sec. III.A).  The two branches
    differ by the second difference of the anomaly, so one switch leaves a
    local difference far above 1e-5; the bar is therefore 1e-5 or twice the
    FP32 storage floor the oracle measures (its own run with FP32-rounded
    stored deviations meets the same kind of events), and the totals must
    agree to 1e-9."""
    n = 32
    f = I.turbulence(3, n, seed=0, Ma_t=0.3, T0=0.15)
    mu = I.turbulence_viscosity(n, Ma_t=0.3, T0=0.15)
    kw = dict(mu=mu, Pr=0.7, visc_exp=0.76, T_ref=0.15)
    out, _, d = run_gpu(3, (n, n, n), f, 100, fp32=True, want_state=False, want_diag=True, **kw)
    s = run_oracle(3, (n, n, n), f, 100, **kw)
    check_fp32_with_floor(3, (n, n, n), f, 100, out, s, **kw)
    r = s.diagnostics()
    assert abs(d["mass"] - r["mass"]) <= 1e-9 * r["mass"]
    assert abs(d["energy"] - r["energy"]) <= 1e-9 * r["energy"]
    assert abs(d["kinetic_energy"] - r["kinetic"]) <= 1e-5 * r["kinetic"]


@pytest.mark.parametrize("u_ref", [None, "upstream"])
def test_fp32_deviation_shock_vortex_crop(u_ref):
    rho, u, T, rh = I.shock_vortex(256, 128, r_v=16.0, x_s=128)
    kw = dict(mu=0.0198, Pr=0.75, bc=(1, 0, 0), T_ref=0.05)
    ur = (float(u[0, 0, 0, 0]), 0.0) if u_ref else None  # the free stream ahead of the shock
    out, _, _ = run_gpu(2, (256, 128), (rho, u, T), 100, fp32=True, want_state=False, u_ref=ur, **kw)
    s = run_oracle(2, (256, 128), (rho, u, T), 100, **kw)
    check_fp32_with_floor(2, (256, 128), (rho, u, T), 100, out, s, u_ref=ur, **kw)


def test_fp32_deviation_sod():
    """The deviation reference is taken at the low-density (right) state: a
    population is then never stored as a deviation larger than itself.  The
    temperature of the power law is not used (constant mu)."""
    f = I.sod(800, 4, T_left=0.15)
    kw = dict(mu=0.015, Pr=0.71, bc=(1, 0, 0))
    lbm = _lbm()
    print("[gpu case] Sod FP32, reference (0.125, 0.12)", flush=True)
    h = lbm.lbm_create(2, (800, 4), 1.4, 0.71, 0.015, precision=lbm.LBM_FP32_DEV, bc=(1, 0, 0), T_ref=0.12,
                       rho_ref=0.125)
    try:
        lbm.lbm_init_fields(h, *f)
        lbm.lbm_step(h, 100)
        out = [np.zeros(a.shape) for a in f]
        lbm.lbm_moments(h, *out)
    finally:
        lbm.lbm_destroy(h)
    s = run_oracle(2, (800, 4), f, 100, **kw)
    check_fields(out, s, 1e-5)


@pytest.mark.parametrize("fp32", [False, True])
def test_diagnostics_match_oracle(fp32):
    dims = (24, 18, 20)
    f = I.smooth_random(3, dims, seed=9, u_amp=0.1)
    kw = dict(mu=0.02, Pr=0.7, visc_exp=0.76, T_ref=0.15, bc=(0, 1, 0))
    _, _, d = run_gpu(3, dims, f, 20, fp32=fp32, want_state=False, want_diag=True, **kw)
    s = run_oracle(3, dims, f, 20, **kw)
    r = s.diagnostics()
    tol = 1e-5 if fp32 else 1e-12
    pairs = [("mass", d["mass"], r["mass"]), ("energy", d["energy"], r["energy"]),
             ("kinetic", d["kinetic_energy"], r["kinetic"]), ("dil2", d["dilatation_sq_sum"], r["dil2"]),
             ("u2", d["u2_sum"], r["u2"]), ("cs", d["cs_sum"], r["cs"]), ("rho2", d["rho2_sum"], r["rho2"]),
             ("vort2", d["vorticity_sq_sum"], r["vort2"]), ("diss", d["dissipation_sum"], r["diss"])]
    pairs += [(f"u{a}2", d["u_axis_sq_sum"][a], r[k]) for a, k in enumerate(("ux2", "uy2", "uz2"))]
    pairs += [(f"du{a}2", d["du_axis_sq_sum"][a], r[k]) for a, k in enumerate(("dux2", "duy2", "duz2"))]
    for name, a, b in pairs:
        assert abs(a - b) <= tol * abs(b), (name, a, b)
    scale = r["mass"] * math.sqrt(r["u2"] / r["nodes"])
    for a, k in enumerate(("mom_x", "mom_y", "mom_z")):
        assert abs(d["momentum"][a] - r[k]) <= tol * scale, (k, d["momentum"][a], r[k])
    assert d["nodes"] == r["nodes"] == np.prod(dims)
    assert d["nonfinite"] == 0 and d["nonpositive"] == 0


@pytest.mark.parametrize("fp32", [False, True])
def test_checkpoint_resume_is_bit_exact(fp32):
    lbm = _lbm()
    dims = (20, 12, 10)
    f = I.smooth_random(3, dims, seed=1, u_amp=0.1)
    prec = lbm.LBM_FP32_DEV if fp32 else lbm.LBM_FP64
    dt = np.float32 if fp32 else np.float64

    def new():
        h = lbm.lbm_create(3, dims, 1.4, 0.7, 0.02, precision=prec, T_ref=0.15)
        lbm.lbm_set_stream(h, torch.cuda.current_stream())
        return h

    print(f"[gpu case] checkpoint fp32={fp32}", flush=True)
    a, b = new(), new()
    try:
        lbm.lbm_init_fields(a, *f)
        lbm.lbm_step(a, 40)
        full = np.zeros(lbm.lbm_state_bytes(a) // np.dtype(dt).itemsize, dtype=dt)
        lbm.lbm_get_state(a, full)
        lbm.lbm_init_fields(b, *f)
        lbm.lbm_step(b, 20)
        ck = torch.zeros(lbm.lbm_state_bytes(b) // np.dtype(dt).itemsize,
                         dtype=torch.float32 if fp32 else torch.float64, device="cuda")
        lbm.lbm_get_state(b, ck)
        lbm.lbm_init_fields(b, *I.uniform(3, dims))  # overwrite, then restore
        lbm.lbm_set_state(b, ck, step=20)
        lbm.lbm_step(b, 20)
        assert lbm.lbm_step_count(b) == 40
        res = np.zeros_like(full)
        lbm.lbm_get_state(b, res)
        assert np.array_equal(res, full)
    finally:
        lbm.lbm_destroy(a)
        lbm.lbm_destroy(b)


def test_error_paths_and_instability_flag():
    lbm = _lbm()
    dims = (16, 8, 1)
    print("[gpu case] error paths", flush=True)
    h = lbm.lbm_create(2, dims, 1.4, 0.7, 0.02)
    try:
        lbm.lbm_set_stream(h, torch.cuda.current_stream())
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_step(h, 1)
        assert e.value.code == lbm.LBM_ESTATE
        rho, u, T = I.uniform(2, dims[:2])
        T_bad = T.copy()
        T_bad[0, 3, 5] = 0.0
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_init_fields(h, rho, u, T_bad)
        assert e.value.code == lbm.LBM_EINVAL
        dev = [torch.from_numpy(a).cuda() for a in (rho, u, T_bad)]
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_init_fields(h, *dev)
        assert e.value.code == lbm.LBM_EINVAL
        u_nan = u.copy()
        u_nan[1, 0, 2, 2] = float("nan")
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_init_fields(h, rho, u_nan, T)
        assert e.value.code == lbm.LBM_EINVAL
        lbm.lbm_init_fields(h, rho, u, T)
        lbm.lbm_step(h, 3)
        d = lbm.lbm_diagnostics(h)
        assert d["nonfinite"] == 0
        # a non-finite population (set from the host) is found and blocks stepping
        st = np.zeros(lbm.lbm_state_bytes(h) // 8)
        lbm.lbm_get_state(h, st)
        st[5 * 128 + 17] = float("nan")
        lbm.lbm_set_state(h, st, step=3)
        d = lbm.lbm_diagnostics(h)
        assert d["nonfinite"] == 1
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_step(h, 1)
        assert e.value.code == lbm.LBM_EUNSTABLE
        with pytest.raises(lbm.LbmError):
            lbm.lbm_get_state(h, np.zeros(7))
    finally:
        lbm.lbm_destroy(h)


@pytest.mark.parametrize("D,dims", [(2, (1, 1)), (2, (3, 2)), (3, (1, 1, 1)), (3, (5, 1, 1)), (3, (2, 3, 4))])
def test_degenerate_small_grids(D, dims):
    f = I.smooth_random(D, dims, seed=3, u_amp=0.05) if np.prod(dims) > 1 else I.uniform(D, dims, u=(0.1, 0.05, 0.02))
    kw = dict(mu=0.02, Pr=0.7)
    for steps in (0, 1, 30):
        out, state, _ = run_gpu(D, dims, f, steps, **kw)
        s = run_oracle(D, dims, f, steps, **kw)
        check_fields(out, s, 1e-12)
        check_pops(state, s, 1e-12)


@pytest.mark.parametrize("fp32", [False, True])
def test_tile_shapes_give_the_same_result(fp32):
    """Every launch shape of a storage precision (FP64: 64 x 4 and 32 x 8;
    FP32 also 64 x 8) gives the same state up to rounding."""
    dims = (70, 20, 13)
    f = I.smooth_random(3, dims, seed=8, u_amp=0.1)
    f = (f[0], f[1] + (0.1 if fp32 else 0.0), f[2])  # FP32: keep the upwind sides unambiguous
    kw = dict(mu=0.02, Pr=0.7)
    tiles = [(64, 4, 32), (32, 8, 5), (32, 8, 1), (64, 4, 13)] + ([(64, 8, 5), (64, 8, 13)] if fp32 else [])
    ref = None
    for tile in tiles:
        _, state, _ = run_gpu(3, dims, f, 25, tile=tile, fp32=fp32, **kw)
        if ref is None:
            ref = state
        else:
            # FP64: rounding only; FP32: the 256-thread shapes keep the halo
            # node's populations in registers and the 512-thread one reloads
            # them, so the halo sums round differently (1.5e-6 after 25 steps)
            tol = 1e-5 if fp32 else 1e-13
            assert np.abs(state - ref).max() <= tol * np.abs(ref).max(), tile


def test_tile_query_and_default_chunk_for_a_given_shape():
    """lbm_get_tile reports the launch tile; a zero chunk with a given shape
    takes the default chunk for that shape (70 x 20 x 13 with 64 x 8 tiles:
    six tile columns, so the shortest chunk, 4 planes)."""
    lbm = _lbm()
    h = lbm.lbm_create(3, (70, 20, 13), 1.4, 0.7, 0.02, precision=lbm.LBM_FP32_DEV, tile=(64, 8, 0))
    try:
        assert lbm.lbm_get_tile(h) == (64, 8, 4)
    finally:
        lbm.lbm_destroy(h)
    h = lbm.lbm_create(3, (70, 20, 13), 1.4, 0.7, 0.02, tile=(32, 8, 9))
    try:
        assert lbm.lbm_get_tile(h) == (32, 8, 9)
    finally:
        lbm.lbm_destroy(h)


def test_fp32_turbulence_statistics_2000_steps_within_one_percent():
    """Decaying turbulence (256^3 D3Q27, Ma_t 0.5, Re_lambda 72): FP32 deviation storage
    against FP64 storage (the latter parity-checked against the oracle) over
    2000 steps (about 10 large-eddy turnovers): K, Ma_t, theta_rms, rho_rms
    and enstrophy every 250 steps within 1%."""
    lbm = _lbm()
    n, steps, every = 256, 2000, 250
    f = I.turbulence(3, n, seed=0, Ma_t=0.5, T0=0.15)
    mu = I.turbulence_viscosity(n, Ma_t=0.5, T0=0.15)
    dev = [torch.from_numpy(a).cuda() for a in f]
    stats = {}
    for prec in (lbm.LBM_FP64, lbm.LBM_FP32_DEV):
        print(f"[gpu case] 256^3 statistics precision={prec}", flush=True)
        h = lbm.lbm_create(3, (n, n, n), 1.4, 0.7, mu, precision=prec, visc_exponent=0.76, T_ref=0.15)
        try:
            lbm.lbm_set_stream(h, torch.cuda.current_stream())
            lbm.lbm_init_fields(h, *dev)
            rows = []
            for k in range(steps // every):
                lbm.lbm_step(h, every)
                d = lbm.lbm_diagnostics(h)
                N = d["nodes"]
                rows.append([d["kinetic_energy"] / N, math.sqrt(d["u2_sum"] / N) / (d["cs_sum"] / N),
                             math.sqrt(d["dilatation_sq_sum"] / N),
                             math.sqrt(max(d["rho2_sum"] / N - (d["mass"] / N) ** 2, 0.0)),
                             0.5 * d["vorticity_sq_sum"] / N])
                print(f"  step {(k + 1) * every}: K {rows[-1][0]:.6e} Ma_t {rows[-1][1]:.5f} "
                      f"theta {rows[-1][2]:.4e} rho_rms {rows[-1][3]:.4e} Omega {rows[-1][4]:.4e}", flush=True)
                assert d["nonfinite"] == 0
            stats[prec] = np.array(rows)
        finally:
            lbm.lbm_destroy(h)
    relerr = np.abs(stats[lbm.LBM_FP32_DEV] - stats[lbm.LBM_FP64]) / np.abs(stats[lbm.LBM_FP64])
    print("  max relative difference per statistic:", relerr.max(0), flush=True)
    assert relerr.max() < 0.01


@pytest.mark.parametrize("tile", [(64, 4, 7), (64, 8, 5), (32, 8, 9), (64, 8, 23), (64, 8, 64)])
def test_fp32_tiles_match_oracle(tile):
    """Every launch shape of the FP32 step kernel gives the result within 1e-5
    of the oracle (ragged tiles, several march chunks, a chunk longer than the
    march axis, periodic and zero-gradient axes)."""
    lbm = _lbm()
    dims = (70, 21, 23)
    f = I.smooth_random(3, dims, seed=12, u_amp=0.05)
    f = (f[0], f[1] + 0.1, f[2])  # keep the upwind branches unambiguous
    kw = dict(mu=0.02, Pr=0.7, visc_exp=0.76, T_ref=0.15, bc=(0, 1, 0))
    print(f"[gpu case] fp32 tile={tile}", flush=True)
    h = lbm.lbm_create(3, dims, 1.4, 0.7, 0.02, precision=lbm.LBM_FP32_DEV, bc=kw["bc"], visc_exponent=0.76,
                       T_ref=0.15, tile=tile)
    try:
        lbm.lbm_init_fields(h, *f)
        lbm.lbm_step(h, 60)
        out = [np.zeros(a.shape) for a in f]
        lbm.lbm_moments(h, *out)
    finally:
        lbm.lbm_destroy(h)
    s = run_oracle(3, dims, f, 60, **kw)
    check_fields(out, s, 1e-5)


@pytest.mark.parametrize("tile", [(64, 1, 32), (128, 1, 5), (256, 1, 1)])
def test_fp32_d2q9_tiles(tile):
    """Each D2Q9 launch width on the FP32 shock-vortex case, within 1e-5 of the oracle."""
    rho, u, T, rh = I.shock_vortex(300, 70, r_v=12.0, x_s=150)
    kw = dict(mu=0.0198, Pr=0.75, bc=(1, 0, 0), T_ref=0.05)
    ur = (float(u[0, 0, 0, 0]), 0.0)  # deviations from the free stream
    out, _, _ = run_gpu(2, (300, 70), (rho, u, T), 80, fp32=True, want_state=False, tile=tile, u_ref=ur, **kw)
    s = run_oracle(2, (300, 70), (rho, u, T), 80, **kw)
    check_fp32_with_floor(2, (300, 70), (rho, u, T), 80, out, s, u_ref=ur, **kw)


# ---- general caloric law (Sec. II.A, Eq. (6)) --------------------------------

CV_LAW = (1.5, 5.0, 20.0)  # C_v(T) = 1.5 + 5 T + 20 T^2


@pytest.mark.parametrize("D,dims", [(2, (40, 33)), (3, (21, 18, 13))])
def test_fp64_general_caloric_law_100_steps(D, dims):
    """U(T) in g^eq and Newton's temperature recovery: FP64 within 1e-12 of
    the oracle after 100 steps, on fields with strong temperature contrast,
    with the power-law viscosity."""
    f = I.smooth_random(D, dims, seed=21, u_amp=0.12, T_amp=0.06)
    kw = dict(mu=0.02, Pr=0.7, visc_exp=0.76, T_ref=0.15, cv=CV_LAW)
    out, state, diag = run_gpu(D, dims, f, 100, want_diag=True, **kw)
    s = run_oracle(D, dims, f, 100, **kw)
    check_fields(out, s, 1e-12)
    check_pops(state, s, 1e-12)
    ref = s.diagnostics()
    assert diag["cs_sum"] == pytest.approx(ref["cs"], rel=1e-12)
    assert diag["energy"] == pytest.approx(ref["energy"], rel=1e-12)


def test_fp32_general_caloric_law_turbulence():
    """FP32 deviation storage with the general law: fields within 1e-5 of the
    FP64 oracle after 100 steps (or twice the case's FP32 conditioning floor)."""
    D, dims = 3, (24, 24, 24)
    f = I.turbulence(3, 24, seed=5, Ma_t=0.3)
    kw = dict(mu=0.02, Pr=0.7, visc_exp=0.76, T_ref=0.15, cv=CV_LAW)
    out, _, _ = run_gpu(D, dims, f, 100, fp32=True, want_state=False, **kw)
    s = run_oracle(D, dims, f, 100, **kw)
    check_fp32_with_floor(D, dims, f, 100, out, s, **kw)


def test_filter_with_general_caloric_law():
    """The box filter recovers T from the filtered energy with the same law:
    the library's filter of its state after 3 steps against the filter
    written out here (block means of rho, rho u and rho E, T from U(T)) of the
    oracle's moments after the same 3 steps."""
    lbm = _lbm()
    dims = (16, 12, 8)
    rho, u, T = I.smooth_random(3, dims, seed=22, u_amp=0.1, T_amp=0.05)
    h = lbm.lbm_create(3, dims, 1.4, 0.7, 0.02, cv_poly=CV_LAW)
    try:
        lbm.lbm_init_fields(h, rho, u, T)
        lbm.lbm_step(h, 3)
        cs = (2, 3, 4)
        out = (np.zeros(cs), np.zeros((3,) + cs), np.zeros(cs))
        lbm.lbm_filter_moments(h, 4, *out)
    finally:
        lbm.lbm_destroy(h)
    s = run_oracle(3, dims, (rho, u, T), 3, mu=0.02, Pr=0.7, cv=CV_LAW)
    r, m, TT = s.moments()
    U = lambda t: CV_LAW[0] * t + CV_LAW[1] * t ** 2 / 2 + CV_LAW[2] * t ** 3 / 3
    E = U(TT) + 0.5 * (m ** 2).sum(0)

    def blocks(a):
        return a.reshape(2, 4, 3, 4, 4, 4).mean(axis=(1, 3, 5))

    rc = blocks(r)
    uc = np.stack([blocks(r * m[a]) / rc for a in range(3)])
    e = blocks(r * E) / rc - 0.5 * (uc ** 2).sum(0)
    assert np.abs(out[0] - rc).max() <= 1e-13
    assert np.abs(out[1] - uc).max() <= 1e-13
    assert np.abs(U(out[2]) - e).max() <= 1e-13 * np.abs(e).max()


def test_batch_refuses_a_general_caloric_law():
    lbm = _lbm()
    dims = (16, 8, 8)
    hs = [lbm.lbm_create(3, dims, 1.4, 0.7, 0.02, precision=lbm.LBM_FP32_DEV, T_ref=0.15, cv_poly=cv)
          for cv in (None, CV_LAW)]
    try:
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_batch_create(hs)
        assert "caloric" in str(e.value)
    finally:
        for h in hs:
            lbm.lbm_destroy(h)


def test_fp32_general_caloric_law_d2q9():
    """The caloric variant of the D2Q9 kernel with FP32 deviation storage."""
    D, dims = 2, (64, 48)
    f = I.smooth_random(D, dims, seed=23, u_amp=0.1, T_amp=0.04)
    kw = dict(mu=0.02, Pr=0.7, visc_exp=0.76, T_ref=0.15, cv=CV_LAW)
    out, _, _ = run_gpu(D, dims, f, 100, fp32=True, want_state=False, **kw)
    s = run_oracle(D, dims, f, 100, **kw)
    check_fp32_with_floor(D, dims, f, 100, out, s, **kw)


def test_fp64_general_caloric_law_zero_gradient():
    """The caloric law with zero-gradient ends along x and periodic y, z."""
    D, dims = 3, (20, 12, 8)
    f = I.smooth_random(D, dims, seed=24, u_amp=0.1, T_amp=0.05)
    kw = dict(mu=0.02, Pr=0.7, visc_exp=0.76, T_ref=0.15, cv=CV_LAW, bc=(1, 0, 0))
    out, state, _ = run_gpu(D, dims, f, 100, **kw)
    s = run_oracle(D, dims, f, 100, **kw)
    check_fields(out, s, 1e-12)
    check_pops(state, s, 1e-12)


@pytest.mark.parametrize("D,dims,fp32,tile", [
    (3, (40, 36, 20), True, (64, 8, 8)),
    (3, (40, 36, 20), True, (64, 4, 4)),
    (3, (37, 21, 18), False, (32, 8, 4)),
    (2, (300, 70, 1), True, (128, 1, 8)),
    (2, (130, 50, 1), False, (64, 1, 4)),
])
def test_block_layout_equals_slot_rows(D, dims, fp32, tile):
    """The two device layouts of lbm_options.layout run the same arithmetic on
    the same values: states (through the layout-independent ABI state),
    moments and diagnostics agree to the last bit after 20 steps, also when a
    batch steps a blocks-layout box."""
    lbm = _lbm()
    prec = lbm.LBM_FP32_DEV if fp32 else lbm.LBM_FP64
    d = dims[:D]
    f = I.smooth_random(D, d, seed=77, u_amp=0.05)
    print(f"[gpu case] layouts D={D} dims={d} fp32={fp32} tile={tile}", flush=True)
    hs = []
    for layout in (lbm.LBM_LAYOUT_SLOT_ROWS, lbm.LBM_LAYOUT_BLOCKS, lbm.LBM_LAYOUT_BLOCKS):
        h = lbm.lbm_create(D, d, 1.4, 0.7, 0.02, precision=prec, visc_exponent=0.76, T_ref=0.15, tile=tile,
                           layout=layout)
        lbm.lbm_init_fields(h, *f)
        hs.append(h)
    b = lbm.lbm_batch_create([hs[2]])
    try:
        lbm.lbm_batch_set_tile(b, tile)
        lbm.lbm_step(hs[0], 20)
        lbm.lbm_step(hs[1], 20)
        lbm.lbm_batch_step(b, 20)
        lbm.lbm_pattern_reference(hs[1], 2)  # runs on the blocks layout, leaves the state alone
        states = []
        for h in hs:
            t = torch.empty(lbm.lbm_state_bytes(h) // (4 if fp32 else 8),
                            dtype=torch.float32 if fp32 else torch.float64, device="cuda")
            lbm.lbm_get_state(h, t)
            torch.cuda.synchronize()
            states.append(t.cpu().numpy())
        assert np.isfinite(states[0]).all()
        for st in states[1:]:
            assert np.array_equal(states[0].view(np.uint32 if fp32 else np.uint64),
                                  st.view(np.uint32 if fp32 else np.uint64))
        d0, d1 = lbm.lbm_diagnostics(hs[0]), lbm.lbm_diagnostics(hs[1])
        for k in ("mass", "energy", "kinetic_energy", "vorticity_sq_sum", "dilatation_sq_sum"):
            assert d0[k] == d1[k], k
    finally:
        lbm.lbm_batch_destroy(b)
        for h in hs:
            lbm.lbm_destroy(h)
