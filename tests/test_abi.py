"""The C-ABI library loads and exports every entry point of include/*.h,
and its host-side argument checks answer before any device work (runs
without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if hdr.endswith(".h"):
            text = open(os.path.join(ROOT, "include", hdr)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lbm():
    from paper_2102_09512_amd import lbm as mod

    return mod


def test_every_declared_symbol_is_exported(lbm):
    names = _declared()
    assert "lbm_step" in names and "lbm_create" in names and len(names) >= 14
    lib = C.CDLL(lbm.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_default_options(lbm):
    o = lbm.lbm_default_options()
    assert o.precision == lbm.LBM_FP64
    assert list(o.bc) == [0, 0, 0]
    assert o.visc_exponent == 0.0 and o.rho_ref == 1.0 and abs(o.T_ref - 1 / 3) < 1e-15
    assert o.deriv_scheme == lbm.LBM_DERIV_UPWIND and list(o.tile) == [0, 0, 0]
    assert list(o.u_ref) == [0.0, 0.0, 0.0]
    assert o.layout == lbm.LBM_LAYOUT_SLOT_ROWS


@pytest.mark.parametrize("args,needle", [
    ((5, (4, 4, 1), 1.4, 0.7, 0.01), "lattice"),
    ((2, (4, 4, 2), 1.4, 0.7, 0.01), "D2Q9"),
    ((3, (0, 4, 4), 1.4, 0.7, 0.01), "dims"),
    ((3, (4, 4, 4), 1.0, 0.7, 0.01), "gamma"),
    ((3, (4, 4, 4), 1.4, 0.0, 0.01), "Pr"),
    ((3, (4, 4, 4), 1.4, 0.7, -1.0), "mu"),
    ((3, (4, 4, 4), 1.4, 0.7, float("nan")), "mu"),
    ((3, ((1 << 30) + 1, 1, 1), 1.4, 0.7, 0.01), "dims"),       # an axis beyond 2^30 nodes
    ((3, (2048, 2048, 1024), 1.4, 0.7, 0.01), "2^31 nodes"),    # 32-bit node indices
])
def test_create_rejects_bad_arguments(lbm, args, needle):
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(*args)
    assert e.value.code == lbm.LBM_EINVAL
    assert needle in str(e.value)


@pytest.mark.parametrize("kw,needle", [
    (dict(precision=7), "precision"),
    (dict(bc=(0, 2, 0)), "boundary"),
    (dict(deriv_scheme=3), "derivative"),
    (dict(T_ref=0.0), "T_ref"),
    (dict(rho_ref=-1.0), "rho_ref"),
    (dict(cv_poly=(0.0, 1.0, 0.0)), "cv_poly"),
    (dict(cv_poly=(1.5, -1.0, 0.0)), "cv_poly"),
    (dict(cv_poly=(1.5, 5.0, 20.0), tile=(64, 8, 16)), "default launch shape"),
    (dict(tile=(48, 4, 8)), "tile"),
    (dict(tile=(64, 4, -2)), "tile"),
    (dict(u_ref=(1.5, 0.0, 0.0)), "u_ref"),
    (dict(u_ref=(0.0, float("nan"), 0.0)), "u_ref"),
    (dict(layout=2), "layout"),
])
def test_create_rejects_bad_options(lbm, kw, needle):
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(3, (8, 8, 8), 1.4, 0.7, 0.01, **kw)
    assert e.value.code == lbm.LBM_EINVAL
    assert needle in str(e.value)


@pytest.mark.parametrize("dims,precision", [
    ((4096, 4096, 2), "LBM_FP64"),     # 16.8 M nodes per plane x 432 B
    ((8192, 4096, 2), "LBM_FP32_DEV"),  # 33.6 M nodes per plane x 216 B
])
def test_create_rejects_planes_beyond_4_gib(lbm, dims, precision):
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(3, dims, 1.4, 0.7, 0.01, precision=getattr(lbm, precision))
    assert e.value.code == lbm.LBM_EINVAL
    assert "4 GiB" in str(e.value)


def test_null_handle_calls_fail_cleanly(lbm):
    L = lbm.raw()
    assert L.lbm_destroy(None) == lbm.LBM_OK
    assert L.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert L.lbm_set_stream(None, None) == lbm.LBM_EINVAL
    assert L.lbm_step_count(None) == -1
    assert L.lbm_state_bytes(None) == 0
    assert L.lbm_device_copy(None, None, 16, None) == lbm.LBM_EINVAL


def test_batch_null_arguments_fail_cleanly(lbm):
    L = lbm.raw()
    import ctypes as C
    out = C.c_void_p()
    assert L.lbm_batch_create(C.byref(out), None, 0) == lbm.LBM_EINVAL
    assert out.value is None
    assert L.lbm_batch_destroy(None) == lbm.LBM_OK
    assert L.lbm_batch_step(None, 1, 0) == lbm.LBM_EINVAL
    assert L.lbm_batch_tune(None, 1, None) == lbm.LBM_EINVAL
    assert L.lbm_batch_set_stream(None, None) == lbm.LBM_EINVAL
    assert L.lbm_batch_set_persistent(None, 1) == lbm.LBM_EINVAL
    assert L.lbm_batch_get_persistent(None) == -1


@pytest.mark.parametrize("channels,dims,needle", [
    ([5, 32, 5], (16, 8, 8), "multiple of 32"),
    ([5, 32, 5], (32, 6, 8), "multiple of 32"),
    ([20, 32, 5], (32, 8, 8), "input channels"),
    ([5, 16, 5], (32, 8, 8), "hidden widths"),
    ([5, 32, 40], (32, 8, 8), "output channels"),
])
def test_nn_create_rejects_bad_shapes(lbm, channels, dims, needle):
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_nn_create(channels, dims)
    assert e.value.code == lbm.LBM_EINVAL and needle in str(e.value)


def test_coupling_null_arguments_fail_cleanly(lbm):
    L = lbm.raw()
    assert L.lbm_fields_add(None, None, None, None, 0) == lbm.LBM_EINVAL
    assert L.lbm_filter_moments(None, 2, None, None, None, 0) == lbm.LBM_EINVAL
    assert L.lbm_nn_destroy(None) == lbm.LBM_OK
    assert L.lbm_nn_correct(None, None) == lbm.LBM_EINVAL
    assert L.lbm_nn_param_count(None) == -1


def test_create_refuses_the_fp64_512_thread_tile(lbm):
    """64 x 8 tiles exist for FP32 storage only (FP64 would spill registers)."""
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(3, (64, 16, 8), 1.4, 0.7, 0.01, tile=(64, 8, 8))
    assert e.value.code == lbm.LBM_EINVAL and "tile" in str(e.value)


def test_get_dims_null_arguments(lbm):
    L = lbm.raw()
    assert L.lbm_get_dims(None, None, None) == lbm.LBM_EINVAL


# The binding checks array sizes against the handle's node count before a
# pointer reaches the library.  A handle the module has registered is enough
# to exercise that check without a GPU: no library call is made.
FAKE_H = 0x7FFF0001
FAKE_NET = 0x7FFF0002


@pytest.fixture
def fake_handles(lbm):
    lbm._HANDLES[FAKE_H] = (3, 4 * 3 * 2)
    lbm._NETS[FAKE_NET] = ((5, 32, 3), 32 * 4 * 4)
    yield
    lbm._HANDLES.pop(FAKE_H, None)
    lbm._NETS.pop(FAKE_NET, None)


@pytest.mark.parametrize("call", ["lbm_init_fields", "lbm_moments", "lbm_fields_add", "lbm_fields_set"])
@pytest.mark.parametrize("bad", ["rho", "u", "T"])
def test_field_arrays_of_the_wrong_size_are_refused(lbm, fake_handles, call, bad):
    import numpy as np

    N = 24
    arrays = {"rho": np.ones(N), "u": np.zeros(3 * N), "T": np.full(N, 0.15)}
    arrays[bad] = np.ones(arrays[bad].size - 1)
    with pytest.raises(ValueError) as e:
        getattr(lbm, call)(FAKE_H, arrays["rho"], arrays["u"], arrays["T"])
    assert bad in str(e.value)


def test_filter_outputs_of_the_wrong_size_are_refused(lbm, fake_handles):
    import numpy as np

    lbm._HANDLES[FAKE_H] = (3, 4 * 4 * 4)  # 4^3 -> 2^3 with factor 2
    with pytest.raises(ValueError) as e:
        lbm.lbm_filter_moments(FAKE_H, 2, np.zeros(8), np.zeros(3 * 8 - 1), np.zeros(8))
    assert "u" in str(e.value)
    with pytest.raises(ValueError):
        lbm.lbm_filter_moments(FAKE_H, 2, np.zeros(64), np.zeros(3 * 64), np.zeros(64))


def test_network_planes_of_the_wrong_size_are_refused(lbm, fake_handles):
    import numpy as np

    V = 32 * 4 * 4
    with pytest.raises(ValueError) as e:
        lbm.lbm_nn_forward(FAKE_NET, np.zeros(5 * V - 1, dtype=np.float32), np.zeros(3 * V, dtype=np.float32))
    assert "x" in str(e.value)
    with pytest.raises(ValueError) as e:
        lbm.lbm_nn_forward(FAKE_NET, np.zeros(5 * V, dtype=np.float32), np.zeros(5 * V, dtype=np.float32))
    assert "y" in str(e.value)
    with pytest.raises(ValueError) as e:
        lbm.lbm_nn_loss_backward(FAKE_NET, np.zeros(5 * V, dtype=np.float32), np.zeros(3 * V, dtype=np.float32))
    assert "target" in str(e.value)
