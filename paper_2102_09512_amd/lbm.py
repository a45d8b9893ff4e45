"""Python binding of liblbm.so (include/lbm.h): argument marshalling only.

Every function has the name of the C entry point it calls.  Arrays may be
numpy arrays (host memory) or torch tensors on the GPU (device memory); torch
is used for device memory and streams only.  A missing or unloadable library
raises at import of this module: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

try:
    # torch ships its own HIP runtime; loading it before liblbm.so lets the
    # library bind to that same runtime, so the process has one runtime and
    # torch's device memory and streams are valid in the library's calls.
    import torch  # noqa: F401
except ImportError:  # host-only use (symbol checks) needs no torch
    pass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")
# debug twin: the step kernel's LDS filled with NaN before use (tests only)
POISON_LIB_PATH = os.path.join(_HERE, "liblbm_poison.so")

LBM_D2Q9, LBM_D3Q27 = 2, 3
LBM_FP64, LBM_FP32_DEV = 0, 1
LBM_BC_PERIODIC, LBM_BC_ZERO_GRADIENT = 0, 1
LBM_HOST, LBM_DEVICE = 0, 1
LBM_DERIV_UPWIND, LBM_DERIV_CENTRAL = 0, 1
LBM_LAYOUT_SLOT_ROWS, LBM_LAYOUT_BLOCKS = 0, 1
LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5


class LbmError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{message} (code {code})")
        self.code = code


class lbm_options(C.Structure):
    _fields_ = [
        ("precision", C.c_int), ("bc", C.c_int * 3), ("visc_exponent", C.c_double),
        ("T_ref", C.c_double), ("rho_ref", C.c_double), ("deriv_scheme", C.c_int),
        ("tile", C.c_int * 3), ("u_ref", C.c_double * 3), ("cv_poly", C.c_double * 3), ("layout", C.c_int),
    ]


class lbm_diag(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("nodes", C.c_int64), ("mass", C.c_double), ("momentum", C.c_double * 3),
        ("energy", C.c_double), ("kinetic_energy", C.c_double), ("dilatation_sq_sum", C.c_double),
        ("u2_sum", C.c_double), ("cs_sum", C.c_double), ("rho2_sum", C.c_double),
        ("vorticity_sq_sum", C.c_double), ("dissipation_sum", C.c_double),
        ("u_axis_sq_sum", C.c_double * 3), ("du_axis_sq_sum", C.c_double * 3),
        ("nonfinite", C.c_int64), ("nonpositive", C.c_int64),
    ]


def _load(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
                          "(hipcc for gfx950)")
    L = C.CDLL(path)
    vp, i64, dp = C.c_void_p, C.c_int64, C.POINTER(C.c_double)
    L.lbm_default_options.argtypes = [C.POINTER(lbm_options)]
    L.lbm_default_options.restype = None
    L.lbm_create.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(i64), C.c_double, C.c_double, C.c_double,
                             C.POINTER(lbm_options)]
    L.lbm_destroy.argtypes = [vp]
    L.lbm_set_stream.argtypes = [vp, vp]
    L.lbm_init_fields.argtypes = [vp, vp, vp, vp, C.c_int]
    L.lbm_step.argtypes = [vp, i64]
    L.lbm_moments.argtypes = [vp, vp, vp, vp, C.c_int]
    L.lbm_diagnostics.argtypes = [vp, C.POINTER(lbm_diag)]
    L.lbm_diagnostics_noalloc.argtypes = [vp, C.POINTER(lbm_diag)]
    L.lbm_state_bytes.argtypes = [vp]
    L.lbm_state_bytes.restype = C.c_size_t
    L.lbm_get_state.argtypes = [vp, vp, C.c_size_t, C.c_int]
    L.lbm_set_state.argtypes = [vp, vp, C.c_size_t, C.c_int, i64]
    L.lbm_step_count.argtypes = [vp]
    L.lbm_step_count.restype = i64
    L.lbm_last_error.argtypes = [vp]
    L.lbm_last_error.restype = C.c_char_p
    L.lbm_device_copy.argtypes = [vp, vp, C.c_size_t, vp]
    L.lbm_fields_add.argtypes = [vp, vp, vp, vp, C.c_int]
    L.lbm_filter_moments.argtypes = [vp, C.c_int, vp, vp, vp, C.c_int]
    L.lbm_nn_create.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(C.c_int), C.POINTER(i64)]
    L.lbm_nn_destroy.argtypes = [vp]
    L.lbm_nn_set_stream.argtypes = [vp, vp]
    L.lbm_nn_param_count.argtypes = [vp]
    L.lbm_nn_param_count.restype = i64
    L.lbm_nn_set_params.argtypes = [vp, vp, C.c_int]
    L.lbm_nn_get_params.argtypes = [vp, vp, C.c_int]
    L.lbm_nn_get_grads.argtypes = [vp, vp, C.c_int]
    L.lbm_nn_zero_grad.argtypes = [vp]
    L.lbm_nn_set_scaling.argtypes = [vp, dp, dp, dp]
    L.lbm_nn_forward.argtypes = [vp, vp, vp]
    L.lbm_nn_loss_backward.argtypes = [vp, vp, vp, dp]
    L.lbm_nn_take_loss.argtypes = [vp, dp, C.POINTER(i64)]
    L.lbm_nn_adam_step.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, i64]
    L.lbm_nn_correct.argtypes = [vp, vp]
    L.lbm_nn_set_output_offset.argtypes = [vp, C.c_int]
    L.lbm_nn_set_correction_limit.argtypes = [vp, C.c_double]
    L.lbm_nn_fields_to_planes.argtypes = [C.c_int, i64, vp, vp, vp, vp, vp]
    L.lbm_fields_set.argtypes = [vp, vp, vp, vp, C.c_int]
    L.lbm_batch_create.argtypes = [C.POINTER(vp), C.POINTER(vp), C.c_int]
    L.lbm_batch_destroy.argtypes = [vp]
    L.lbm_batch_set_stream.argtypes = [vp, vp]
    L.lbm_batch_set_tile.argtypes = [vp, C.POINTER(C.c_int)]
    L.lbm_batch_get_tile.argtypes = [vp, C.POINTER(C.c_int)]
    L.lbm_get_tile.argtypes = [vp, C.POINTER(C.c_int)]
    L.lbm_get_dims.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(i64)]
    L.lbm_pattern_reference.argtypes = [vp, i64]
    L.lbm_batch_tune.argtypes = [vp, C.c_int, dp]
    L.lbm_batch_step.argtypes = [vp, i64, C.c_int]
    L.lbm_batch_set_persistent.argtypes = [vp, C.c_int]
    L.lbm_batch_get_persistent.argtypes = [vp]
    for name in ("lbm_create", "lbm_destroy", "lbm_set_stream", "lbm_init_fields", "lbm_step", "lbm_moments",
                 "lbm_diagnostics", "lbm_diagnostics_noalloc", "lbm_get_state", "lbm_set_state", "lbm_device_copy", "lbm_batch_create",
                 "lbm_batch_destroy", "lbm_batch_set_stream", "lbm_batch_set_tile", "lbm_batch_get_tile",
                 "lbm_get_tile", "lbm_get_dims", "lbm_pattern_reference", "lbm_batch_tune",
                 "lbm_batch_set_persistent", "lbm_batch_get_persistent", "lbm_batch_step", "lbm_fields_add", "lbm_filter_moments", "lbm_nn_create",
                 "lbm_nn_destroy", "lbm_nn_set_stream", "lbm_nn_set_params", "lbm_nn_get_params", "lbm_nn_get_grads",
                 "lbm_nn_zero_grad", "lbm_nn_set_scaling", "lbm_nn_forward", "lbm_nn_loss_backward",
                 "lbm_nn_adam_step", "lbm_nn_take_loss", "lbm_nn_correct", "lbm_nn_fields_to_planes", "lbm_fields_set",
                 "lbm_nn_set_output_offset", "lbm_nn_set_correction_limit"):
        getattr(L, name).restype = C.c_int
    return L


_L = _load()


def _check(rc: int) -> int:
    if rc != LBM_OK:
        raise LbmError(rc, lbm_last_error())
    return rc


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _arg(x, dtype=np.float64):
    """(pointer, memory kind, keep-alive) of a numpy array or a torch tensor;
    dtype None accepts any element type."""
    if x is None:
        return None, None, None
    if _is_torch(x):
        import torch

        if dtype is not None:
            want = torch.float64 if dtype == np.float64 else torch.float32
            if x.dtype != want:
                raise TypeError(f"expected a {want} tensor, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr(), (LBM_DEVICE if x.is_cuda else LBM_HOST), x
    if dtype is None:
        if not (isinstance(x, np.ndarray) and x.flags.c_contiguous):
            raise TypeError("expected a C-contiguous numpy array")
        return x.ctypes.data, LBM_HOST, x
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data, LBM_HOST, a


# Shapes of the handles and networks made through this module, so that array
# sizes are checked before a pointer reaches the library (the C ABI takes
# plain pointers and cannot).  Handles made elsewhere are asked for their dims.
_HANDLES: dict = {}
_NETS: dict = {}


def _numel(x) -> int:
    return int(x.numel()) if _is_torch(x) else int(np.asarray(x).size)


def _nodes(h):
    """(D, N) of a handle."""
    if h not in _HANDLES:
        lat, dims = lbm_get_dims(h)
        _HANDLES[h] = (lat, int(np.prod(dims)))
    return _HANDLES[h]


def _expect(call, name, x, n):
    if x is not None and _numel(x) != n:
        raise ValueError(f"{call}: {name} has {_numel(x)} values, expected {n}")


def _fields_sized(call, h, rho, u, T):
    D, N = _nodes(h)
    _expect(call, "rho", rho, N)
    _expect(call, "u", u, D * N)
    _expect(call, "T", T, N)


def _same_kind(*kinds):
    ks = {k for k in kinds if k is not None}
    if len(ks) > 1:
        raise ValueError("all arrays of one call must be in the same memory (host or device)")
    return ks.pop() if ks else LBM_HOST


# ---- entry points ----------------------------------------------------------

def lbm_default_options() -> lbm_options:
    o = lbm_options()
    _L.lbm_default_options(C.byref(o))
    return o


def lbm_create(lattice, dims, gamma, Pr, mu, options: lbm_options | None = None, *, precision=None, bc=None,
               visc_exponent=None, T_ref=None, rho_ref=None, deriv_scheme=None, tile=None, u_ref=None,
               cv_poly=None, layout=None) -> int:
    o = options if options is not None else lbm_default_options()
    if precision is not None:
        o.precision = precision
    if bc is not None:
        for a in range(3):
            o.bc[a] = int(bc[a])
    if visc_exponent is not None:
        o.visc_exponent = visc_exponent
    if T_ref is not None:
        o.T_ref = T_ref
    if rho_ref is not None:
        o.rho_ref = rho_ref
    if deriv_scheme is not None:
        o.deriv_scheme = deriv_scheme
    if tile is not None:
        for a in range(3):
            o.tile[a] = int(tile[a])
    if u_ref is not None:
        for a in range(len(u_ref)):
            o.u_ref[a] = float(u_ref[a])
    if cv_poly is not None:
        for k in range(3):
            o.cv_poly[k] = float(cv_poly[k])
    if layout is not None:
        o.layout = int(layout)
    d = (C.c_int64 * 3)(*[int(v) for v in (list(dims) + [1] * (3 - len(dims)))])
    h = C.c_void_p()
    _check(_L.lbm_create(C.byref(h), int(lattice), d, float(gamma), float(Pr), float(mu), C.byref(o)))
    _HANDLES[h.value] = (int(lattice), int(d[0]) * int(d[1]) * int(d[2]))
    return h.value


def lbm_destroy(h) -> int:
    _HANDLES.pop(h, None)
    return _check(_L.lbm_destroy(h))


def lbm_get_dims(h):
    """(lattice, (nx, ny, nz)) of a handle."""
    lat, d = C.c_int(), (C.c_int64 * 3)()
    _check(_L.lbm_get_dims(h, C.byref(lat), d))
    return lat.value, tuple(int(v) for v in d)


def lbm_set_stream(h, stream) -> int:
    """stream: a torch.cuda.Stream, a raw hipStream_t integer, or None (null stream)."""
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    return _check(_L.lbm_set_stream(h, stream))


def lbm_init_fields(h, rho, u, T) -> int:
    _fields_sized("lbm_init_fields", h, rho, u, T)
    pr, kr, _kr = _arg(rho)
    pu, ku, _ku = _arg(u)
    pt, kt, _kt = _arg(T)
    return _check(_L.lbm_init_fields(h, pr, pu, pt, _same_kind(kr, ku, kt)))


def lbm_step(h, n: int = 1) -> int:
    return _check(_L.lbm_step(h, int(n)))


def lbm_pattern_reference(h, launches: int = 1) -> int:
    return _check(_L.lbm_pattern_reference(h, int(launches)))


def lbm_moments(h, rho=None, u=None, T=None):
    """Writes into the given arrays (numpy or device tensors) and returns them."""
    _fields_sized("lbm_moments", h, rho, u, T)
    args = [_arg(x) for x in (rho, u, T)]
    kind = _same_kind(*[a[1] for a in args])
    if kind == LBM_HOST:
        for x in (rho, u, T):
            if x is not None and not _is_torch(x) and not (isinstance(x, np.ndarray) and x.dtype == np.float64
                                                           and x.flags.c_contiguous):
                raise TypeError("host outputs must be C-contiguous float64 numpy arrays")
    _check(_L.lbm_moments(h, args[0][0], args[1][0], args[2][0], kind))
    return rho, u, T


def _diag_dict(d) -> dict:
    out = {}
    for name, _ in lbm_diag._fields_:
        v = getattr(d, name)
        out[name] = list(v) if isinstance(v, C.Array) else v
    return out


def lbm_diagnostics(h) -> dict:
    d = lbm_diag()
    _check(_L.lbm_diagnostics(h, C.byref(d)))
    return _diag_dict(d)


def lbm_diagnostics_noalloc(h) -> dict:
    d = lbm_diag()
    _check(_L.lbm_diagnostics_noalloc(h, C.byref(d)))
    return _diag_dict(d)


def lbm_get_tile(h):
    t = (C.c_int * 3)()
    _check(_L.lbm_get_tile(h, t))
    return tuple(t)


def lbm_state_bytes(h) -> int:
    return int(_L.lbm_state_bytes(h))


def _nbytes(buf) -> int:
    return buf.numel() * buf.element_size() if _is_torch(buf) else buf.nbytes


def lbm_get_state(h, buf) -> int:
    p, k, _keep = _arg(buf, dtype=None)
    return _check(_L.lbm_get_state(h, p, _nbytes(buf), k))


def lbm_set_state(h, buf, step: int = 0) -> int:
    p, k, _keep = _arg(buf, dtype=None)
    return _check(_L.lbm_set_state(h, p, _nbytes(buf), k, int(step)))


def lbm_step_count(h) -> int:
    return int(_L.lbm_step_count(h))


def lbm_last_error(h=None) -> str:
    return _L.lbm_last_error(h).decode()


def lbm_device_copy(dst, src, nbytes: int, stream=None) -> int:
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    return _check(_L.lbm_device_copy(dst.data_ptr(), src.data_ptr(), int(nbytes), stream))


def raw():
    """The ctypes library object (for the ABI tests)."""
    return _L


def raw_poison():
    """The debug twin liblbm_poison.so as a ctypes library with the same
    argument types (its handles are used with its own functions only)."""
    return _load(POISON_LIB_PATH)


# ---- batches -----------------------------------------------------------------

def lbm_batch_create(handles) -> int:
    """A batch over the given handles (which must outlive it)."""
    arr = (C.c_void_p * len(handles))(*handles)
    b = C.c_void_p()
    _check(_L.lbm_batch_create(C.byref(b), arr, len(handles)))
    return b.value


def lbm_batch_destroy(b) -> int:
    return _check(_L.lbm_batch_destroy(b))


def lbm_batch_set_stream(b, stream) -> int:
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    return _check(_L.lbm_batch_set_stream(b, stream))


def lbm_batch_set_tile(b, tile) -> int:
    t = (C.c_int * 3)(*[int(v) for v in tile])
    return _check(_L.lbm_batch_set_tile(b, t))


def lbm_batch_get_tile(b):
    t = (C.c_int * 3)()
    _check(_L.lbm_batch_get_tile(b, t))
    return tuple(t)


def lbm_batch_tune(b, reps: int = 5) -> float:
    """Runs the autotuner; returns the best time per step in ms."""
    ms = C.c_double()
    _check(_L.lbm_batch_tune(b, int(reps), C.byref(ms)))
    return ms.value


def lbm_batch_set_persistent(b, on: bool) -> int:
    return _check(_L.lbm_batch_set_persistent(b, 1 if on else 0))


def lbm_batch_get_persistent(b) -> bool:
    return _L.lbm_batch_get_persistent(b) == 1


def lbm_batch_step(b, n: int = 1, graph_steps: int = 0) -> int:
    return _check(_L.lbm_batch_step(b, int(n), int(graph_steps)))


# ---- coupling of coarse runs and the learned corrector ---------------------------

def lbm_fields_add(h, drho, du, dT) -> int:
    _fields_sized("lbm_fields_add", h, drho, du, dT)
    pr, kr, _a = _arg(drho)
    pu, ku, _b = _arg(du)
    pt, kt, _c = _arg(dT)
    return _check(_L.lbm_fields_add(h, pr, pu, pt, _same_kind(kr, ku, kt)))


def lbm_fields_set(h, rho, u, T) -> int:
    _fields_sized("lbm_fields_set", h, rho, u, T)
    pr, kr, _a = _arg(rho)
    pu, ku, _b = _arg(u)
    pt, kt, _c = _arg(T)
    return _check(_L.lbm_fields_set(h, pr, pu, pt, _same_kind(kr, ku, kt)))


def lbm_filter_moments(h, factor, rho, u, T):
    """Writes the coarse moments into rho, u, T (numpy arrays or device tensors)."""
    D, N = _nodes(h)
    f = int(factor)
    if f < 1:
        raise ValueError("lbm_filter_moments: factor must be >= 1")
    Nc = N // (f ** D)
    for name, x, n in (("rho", rho, Nc), ("u", u, D * Nc), ("T", T, Nc)):
        if x is None:
            raise ValueError(f"lbm_filter_moments: {name} is required")
        _expect("lbm_filter_moments", name, x, n)
        if not _is_torch(x) and not (isinstance(x, np.ndarray) and x.dtype == np.float64 and x.flags.c_contiguous):
            raise TypeError("host outputs must be C-contiguous float64 numpy arrays")
    args = [_arg(x) for x in (rho, u, T)]
    kind = _same_kind(*[a[1] for a in args])
    _check(_L.lbm_filter_moments(h, int(factor), args[0][0], args[1][0], args[2][0], kind))
    return rho, u, T


def _f32(x):
    """(pointer, kind, keep-alive) of an FP32 numpy array or tensor."""
    if _is_torch(x):
        return _arg(x, dtype=np.float32)
    a = np.ascontiguousarray(x, dtype=np.float32)
    return a.ctypes.data, LBM_HOST, a


def lbm_nn_create(channels, dims) -> int:
    ch = (C.c_int * len(channels))(*[int(c) for c in channels])
    d = (C.c_int64 * 3)(*[int(v) for v in (list(dims) + [1] * (3 - len(dims)))])
    n = C.c_void_p()
    _check(_L.lbm_nn_create(C.byref(n), len(channels) - 1, ch, d))
    _NETS[n.value] = (tuple(int(c) for c in channels), int(d[0]) * int(d[1]) * int(d[2]))
    return n.value


def lbm_nn_destroy(n) -> int:
    _NETS.pop(n, None)
    return _check(_L.lbm_nn_destroy(n))


def _net_planes(call, n, **arrays):
    """Checks planar network tensors: name=(array, which) with which 'in'
    (c[0] planes) or 'out' (c[L] planes)."""
    if n not in _NETS:
        return
    ch, V = _NETS[n]
    for name, (x, which) in arrays.items():
        _expect(call, name, x, (ch[0] if which == "in" else ch[-1]) * V)


def lbm_nn_set_stream(n, stream) -> int:
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    return _check(_L.lbm_nn_set_stream(n, stream))


def lbm_nn_param_count(n) -> int:
    return int(_L.lbm_nn_param_count(n))


def lbm_nn_set_params(n, params) -> int:
    _expect("lbm_nn_set_params", "params", params, lbm_nn_param_count(n))
    p, k, _keep = _f32(params)
    return _check(_L.lbm_nn_set_params(n, p, k))


def lbm_nn_get_params(n) -> np.ndarray:
    out = np.zeros(lbm_nn_param_count(n), dtype=np.float32)
    _check(_L.lbm_nn_get_params(n, out.ctypes.data, LBM_HOST))
    return out


def lbm_nn_get_grads(n) -> np.ndarray:
    out = np.zeros(lbm_nn_param_count(n), dtype=np.float32)
    _check(_L.lbm_nn_get_grads(n, out.ctypes.data, LBM_HOST))
    return out


def lbm_nn_zero_grad(n) -> int:
    return _check(_L.lbm_nn_zero_grad(n))


def lbm_nn_set_scaling(n, mean, std, out_std=None) -> int:
    m = np.ascontiguousarray(mean, dtype=np.float64)
    s = np.ascontiguousarray(std, dtype=np.float64)
    o = None if out_std is None else np.ascontiguousarray(out_std, dtype=np.float64)
    dp = C.POINTER(C.c_double)
    return _check(_L.lbm_nn_set_scaling(n, m.ctypes.data_as(dp), s.ctypes.data_as(dp),
                                        None if o is None else o.ctypes.data_as(dp)))


def lbm_nn_set_output_offset(n, offset: int) -> int:
    return _check(_L.lbm_nn_set_output_offset(n, int(offset)))


def lbm_nn_set_correction_limit(n, limit: float) -> int:
    return _check(_L.lbm_nn_set_correction_limit(n, float(limit)))


def lbm_nn_forward(n, x, y) -> int:
    """x, y: contiguous float32 device tensors (planes)."""
    _net_planes("lbm_nn_forward", n, x=(x, "in"), y=(y, "out"))
    px, kx, _a = _arg(x, dtype=np.float32)
    py, ky, _b = _arg(y, dtype=np.float32)
    if kx != LBM_DEVICE or ky != LBM_DEVICE:
        raise ValueError("lbm_nn_forward takes device tensors")
    return _check(_L.lbm_nn_forward(n, px, py))


def lbm_nn_loss_backward(n, x, target, sync: bool = True):
    """The sample's loss (synchronous), or None with sync False: the loss is
    then added to the device-side sum that lbm_nn_take_loss returns."""
    _net_planes("lbm_nn_loss_backward", n, x=(x, "in"), target=(target, "in"))
    px, kx, _a = _arg(x, dtype=np.float32)
    pt, kt, _b = _arg(target, dtype=np.float32)
    if kx != LBM_DEVICE or kt != LBM_DEVICE:
        raise ValueError("lbm_nn_loss_backward takes device tensors")
    if not sync:
        _check(_L.lbm_nn_loss_backward(n, px, pt, None))
        return None
    loss = C.c_double()
    _check(_L.lbm_nn_loss_backward(n, px, pt, C.byref(loss)))
    return loss.value


def lbm_nn_take_loss(n):
    """(sum, count) of the asynchronous losses since the last call; resets them."""
    total, count = C.c_double(), C.c_int64()
    _check(_L.lbm_nn_take_loss(n, C.byref(total), C.byref(count)))
    return total.value, int(count.value)


def lbm_nn_adam_step(n, lr, beta1=0.9, beta2=0.999, eps=1e-8, grad_scale=1.0, t=1) -> int:
    return _check(_L.lbm_nn_adam_step(n, float(lr), float(beta1), float(beta2), float(eps), float(grad_scale), int(t)))


def lbm_nn_fields_to_planes(D, rho, u, T, x, stream=None) -> int:
    """Device FP64 fields -> the FP32 planes x (device tensor of D + 2 planes)."""
    args = [_arg(a) for a in (rho, u, T)]
    px, kx, _k = _arg(x, dtype=np.float32)
    if any(a[1] != LBM_DEVICE for a in args) or kx != LBM_DEVICE:
        raise ValueError("lbm_nn_fields_to_planes takes device tensors")
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    nodes = rho.numel()
    if x.numel() < (D + 2) * nodes or u.numel() < D * nodes or T.numel() < nodes:
        raise ValueError("lbm_nn_fields_to_planes: arrays too small")
    return _check(_L.lbm_nn_fields_to_planes(int(D), int(nodes), args[0][0], args[1][0], args[2][0], px, stream))


def lbm_nn_correct(n, h) -> int:
    return _check(_L.lbm_nn_correct(n, h))
