"""The step kernel built with its LDS anomaly ring filled with NaN before
every use (liblbm_poison.so, LBM_POISON_LDS) must give the same populations,
to the last bit, as the normal build.  A value read from LDS that no thread
wrote for the current plane would be NaN in the debug build (and a stale
neighbour value in the normal one), so any such read shows up here.  The cases
cover every compiled tile family (one and two planes in flight), ragged tiles
in both in-plane axes, ragged march chunks, zero-gradient and periodic axes,
both derivative schemes and both storages."""
import ctypes as C

import numpy as np
import pytest

from paper_2102_09512_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lbm():
    from paper_2102_09512_amd import lbm

    return lbm


def _run(lbm, L, D, dims, fp32, tile, bc, deriv, fields, steps):
    o = lbm.lbm_default_options()
    o.precision = lbm.LBM_FP32_DEV if fp32 else lbm.LBM_FP64
    o.visc_exponent, o.T_ref = 0.76, 0.15
    o.deriv_scheme = deriv
    for a in range(3):
        o.bc[a] = bc[a]
        o.tile[a] = tile[a]
    h = C.c_void_p()
    d = (C.c_int64 * 3)(*(list(dims) + [1] * (3 - len(dims))))
    assert L.lbm_create(C.byref(h), D, d, 1.4, 0.7, 0.02, C.byref(o)) == lbm.LBM_OK, L.lbm_last_error(None)
    try:
        rho, u, T = fields
        assert L.lbm_init_fields(h, rho.data_ptr(), u.data_ptr(), T.data_ptr(), lbm.LBM_DEVICE) == lbm.LBM_OK
        assert L.lbm_step(h, steps) == lbm.LBM_OK
        nb = L.lbm_state_bytes(h)
        out = torch.empty(nb // (4 if fp32 else 8), dtype=torch.float32 if fp32 else torch.float64, device="cuda")
        assert L.lbm_get_state(h, out.data_ptr(), nb, lbm.LBM_DEVICE) == lbm.LBM_OK
        torch.cuda.synchronize()
        return out.cpu().numpy()
    finally:
        L.lbm_destroy(h)


@pytest.mark.parametrize("D,dims,fp32,tile,bc,central", [
    (3, (70, 45, 13), True, (64, 8, 4), (0, 0, 0), False),
    (3, (70, 45, 20), True, (64, 4, 8), (1, 0, 1), False),
    (3, (33, 17, 11), True, (32, 8, 5), (0, 1, 0), True),
    (3, (66, 9, 10), False, (64, 4, 4), (0, 0, 0), False),
    (3, (40, 20, 17), False, (32, 8, 8), (0, 1, 0), True),
    (2, (300, 70), True, (128, 1, 8), (0, 0, 0), False),
    (2, (130, 50), False, (64, 1, 4), (1, 0, 0), False),
])
def test_poisoned_lds_gives_the_same_populations(D, dims, fp32, tile, bc, central):
    lbm = _lbm()
    Lp = lbm.raw_poison()
    deriv = lbm.LBM_DERIV_CENTRAL if central else lbm.LBM_DERIV_UPWIND
    print(f"[gpu case] LDS poison D={D} dims={dims} fp32={fp32} tile={tile} bc={bc} central={central}", flush=True)
    fields = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in I.smooth_random(D, dims, seed=91, u_amp=0.05)]
    ref = _run(lbm, lbm.raw(), D, dims, fp32, tile, bc, deriv, fields, 12)
    got = _run(lbm, Lp, D, dims, fp32, tile, bc, deriv, fields, 12)
    assert np.isfinite(ref).all()
    assert np.isfinite(got).all(), "the debug build read an LDS value no thread wrote for that plane"
    assert np.array_equal(ref.view(np.uint32 if fp32 else np.uint64), got.view(np.uint32 if fp32 else np.uint64))
