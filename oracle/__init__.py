"""CPU FP64 oracle of the two-population compressible LBM (arXiv:2102.09512).

TEST INFRASTRUCTURE.  This package wraps ``liboracle.so`` (plain C, built from
``oracle.c`` in this directory) with ctypes.  Only the test suite,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
it.  It shares no code with the GPU library ``paper_2102_09512_amd``; the GPU
library never imports it.

Field arrays are node-major FP64 numpy arrays of shape (nz, ny, nx) for rho and
T and (D, nz, ny, nx) for u; node = x + nx*(y + ny*z).  Populations are
returned as (Q, nz, ny, nx) with c_i = (i%3-1, (i/3)%3-1, (i/9)%3-1).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# A different build of oracle.c (the pin suite's planted-mistake check) can be
# loaded instead through this variable.
_LIB_OVERRIDE = os.environ.get("LBM_ORACLE_LIB")

PERIODIC, ZERO_GRADIENT = 0, 1
UPWIND, CENTRAL = 0, 1

DIAG_NAMES = [
    "mass", "mom_x", "mom_y", "mom_z", "energy", "kinetic", "dil2", "u2", "cs", "rho2",
    "vort2", "diss", "ux2", "uy2", "uz2", "dux2", "duy2", "duz2", "nonfinite",
    "nonpositive", "nodes",
]


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [
        ("D", C.c_int), ("n", C.c_long * 3), ("bc", C.c_int * 3), ("gamma", C.c_double),
        ("Pr", C.c_double), ("mu0", C.c_double), ("visc_exp", C.c_double),
        ("T_ref", C.c_double), ("deriv", C.c_int), ("cv", C.c_double * 3),
    ]


_lib = None
_dp = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = C.CDLL(_LIB_OVERRIDE)
        else:
            build()
            L = C.CDLL(_LIB)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(_Params)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_init.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_step.argtypes = [C.c_void_p, C.c_long]
        L.orc_step_sampled.argtypes = [C.c_void_p, C.POINTER(C.c_long), C.c_long, _dp, _dp]
        L.orc_step_sampled_branch.argtypes = [C.c_void_p, C.POINTER(C.c_long), C.c_long, C.POINTER(C.c_byte),
                                              _dp, _dp]
        L.orc_set_fp32_storage.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_set_upwind_band.argtypes = [C.c_void_p, C.c_double]
        L.orc_step_count.restype = C.c_long
        L.orc_step_count.argtypes = [C.c_void_p]
        L.orc_moments.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_diagnostics.argtypes = [C.c_void_p, _dp]
        L.orc_get_pops.argtypes = [C.c_void_p, _dp, _dp]
        L.orc_set_pops.argtypes = [C.c_void_p, _dp, _dp, C.c_long]
        L.orc_product_form.argtypes = [C.c_int, C.c_double, _dp, _dp, _dp]
        L.orc_feq.argtypes = [C.c_int, C.c_double, _dp, C.c_double, _dp]
        L.orc_fex.argtypes = [C.c_int, C.c_double, _dp, C.c_double, C.c_double, _dp, _dp]
        L.orc_geq.argtypes = [C.c_int, C.c_double, _dp, C.c_double, C.c_double, _dp]
        L.orc_geq_u.argtypes = [C.c_int, C.c_double, _dp, C.c_double, C.c_double, _dp]
        L.orc_caloric.argtypes = [C.POINTER(_Params), _dp]
        L.orc_internal_energy.argtypes = [_dp, C.c_double]
        L.orc_internal_energy.restype = C.c_double
        L.orc_temperature.argtypes = [_dp, C.c_double]
        L.orc_temperature.restype = C.c_double
        L.orc_dq.argtypes = [C.c_int, C.c_double, _dp, C.c_double, _dp, _dp, _dp]
        L.orc_gstar.argtypes = [C.c_int, C.c_double, _dp, C.c_double, C.c_double, _dp, _dp, _dp]
        for name in ("orc_anomaly",):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_omega.restype = C.c_double
        L.orc_omega.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_omega1.restype = C.c_double
        L.orc_omega1.argtypes = [C.c_double, C.c_double]
        L.orc_collide_node.argtypes = [C.POINTER(_Params), _dp, _dp, _dp, _dp, _dp]
        L.orc_derivative.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_set_num_threads.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _vec(x, n=3):
    a = np.zeros(n, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64).ravel()
    a[: x.size] = x
    return a


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (results do not depend on it)."""
    lib().orc_set_num_threads(int(n))


def Q(D: int) -> int:
    return 9 if D == 2 else 27


def velocities(D: int) -> np.ndarray:
    """(Q, 3) integer velocity table in the oracle's numbering."""
    i = np.arange(Q(D))
    c = np.stack([i % 3 - 1, (i // 3) % 3 - 1, (i // 9) % 3 - 1 if D == 3 else 0 * i], axis=1)
    return c


def make_params(D, dims, gamma=1.4, Pr=0.71, mu=0.01, visc_exp=0.0, T_ref=1.0,
                bc=(PERIODIC, PERIODIC, PERIODIC), deriv=UPWIND, cv=None) -> _Params:
    """cv: (c0, c1, c2) of C_v(T) = c0 + c1 T + c2 T^2, or None for 1/(gamma-1)."""
    p = _Params()
    p.D = D
    for a in range(3):
        p.n[a] = int(dims[a]) if a < len(dims) else 1
        p.bc[a] = int(bc[a])
    p.gamma, p.Pr, p.mu0, p.visc_exp, p.T_ref, p.deriv = gamma, Pr, mu, visc_exp, T_ref, deriv
    for k in range(3):
        p.cv[k] = float(cv[k]) if cv is not None else 0.0
    return p


def caloric(cv=None, gamma=1.4) -> np.ndarray:
    """The C_v(T) coefficients in effect (orc_caloric)."""
    p = make_params(3, (1, 1, 1), gamma=gamma, cv=cv)
    out = np.zeros(3)
    lib().orc_caloric(C.byref(p), _ptr(out))
    return out


def internal_energy(cv, T) -> float:
    return lib().orc_internal_energy(_ptr(np.ascontiguousarray(cv, dtype=np.float64)), float(T))


def temperature(cv, e) -> float:
    return lib().orc_temperature(_ptr(np.ascontiguousarray(cv, dtype=np.float64)), float(e))


# ---- nodal functions -------------------------------------------------------

def product_form(D, rho, xi, P):
    out = np.zeros(Q(D))
    lib().orc_product_form(D, rho, _ptr(_vec(xi)), _ptr(_vec(P)), _ptr(out))
    return out


def feq(D, rho, u, T):
    out = np.zeros(Q(D))
    lib().orc_feq(D, rho, _ptr(_vec(u)), T, _ptr(out))
    return out


def fex(D, rho, u, T, omega, d):
    out = np.zeros(Q(D))
    lib().orc_fex(D, rho, _ptr(_vec(u)), T, omega, _ptr(_vec(d)), _ptr(out))
    return out


def geq(D, rho, u, T, Cv):
    out = np.zeros(Q(D))
    lib().orc_geq(D, rho, _ptr(_vec(u)), T, Cv, _ptr(out))
    return out


def geq_u(D, rho, u, T, U):
    """g^eq with the internal energy U = U(T) of any caloric law."""
    out = np.zeros(Q(D))
    lib().orc_geq_u(D, rho, _ptr(_vec(u)), T, U, _ptr(out))
    return out


def dq(D, rho, u, T, P, d):
    out = np.zeros(3)
    Pm = np.ascontiguousarray(np.asarray(P, dtype=np.float64).reshape(D, D))
    lib().orc_dq(D, rho, _ptr(_vec(u)), T, _ptr(Pm), _ptr(_vec(d)), _ptr(out))
    return out[:D]


def gstar(D, rho, u, T, Cv, P, d):
    out = np.zeros(Q(D))
    Pm = np.ascontiguousarray(np.asarray(P, dtype=np.float64).reshape(D, D))
    lib().orc_gstar(D, rho, _ptr(_vec(u)), T, Cv, _ptr(Pm), _ptr(_vec(d)), _ptr(out))
    return out


def anomaly(rho, u, T):
    return lib().orc_anomaly(rho, u, T)


def omega(mu, rho, T):
    return lib().orc_omega(mu, rho, T)


def omega1(om, Pr):
    return lib().orc_omega1(om, Pr)


def collide_node(params: _Params, fh, gh, d):
    D = params.D
    fo, go = np.zeros(Q(D)), np.zeros(Q(D))
    fh = np.ascontiguousarray(fh, dtype=np.float64)
    gh = np.ascontiguousarray(gh, dtype=np.float64)
    lib().orc_collide_node(C.byref(params), _ptr(fh), _ptr(gh), _ptr(_vec(d)), _ptr(fo), _ptr(go))
    return fo, go


# ---- whole field -----------------------------------------------------------

class Sim:
    """Whole-field oracle simulation (see oracle.h)."""

    def __init__(self, D, dims, gamma=1.4, Pr=0.71, mu=0.01, visc_exp=0.0, T_ref=1.0,
                 bc=(PERIODIC, PERIODIC, PERIODIC), deriv=UPWIND, cv=None):
        dims = tuple(int(d) for d in dims) + (1,) * (3 - len(dims))
        self.D, self.dims = D, dims
        self.params = make_params(D, dims, gamma, Pr, mu, visc_exp, T_ref, bc, deriv, cv)
        self._h = lib().orc_create(C.byref(self.params))
        if not self._h:
            raise ValueError("oracle: invalid parameters")
        self.N = dims[0] * dims[1] * dims[2]
        self.shape = (dims[2], dims[1], dims[0])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def init(self, rho, u, T):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.shape)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(self.shape)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape((self.D,) + self.shape)
        if lib().orc_init(self._h, _ptr(rho), _ptr(u), _ptr(T)) != 0:
            raise ValueError("oracle: non-finite or non-positive rho/T in init")

    def step(self, n=1):
        if lib().orc_step(self._h, int(n)) != 0:
            raise ValueError("oracle: bad step count")

    @property
    def step_count(self):
        return lib().orc_step_count(self._h)

    def step_sampled(self, nodes):
        nodes = np.ascontiguousarray(nodes, dtype=np.int64)
        k = nodes.size
        f = np.zeros((Q(self.D), k))
        g = np.zeros((Q(self.D), k))
        rc = lib().orc_step_sampled(self._h, nodes.ctypes.data_as(C.POINTER(C.c_long)), k, _ptr(f), _ptr(g))
        if rc != 0:
            raise MemoryError("oracle: step_sampled failed")
        return f, g

    def step_sampled_branch(self, nodes, branch):
        """step_sampled with the upwind side forced per node and axis:
        branch (count, D) of -1 (sign of u), 0 (backward) or 1 (forward)."""
        nodes = np.ascontiguousarray(nodes, dtype=np.int64)
        k = nodes.size
        br = np.ascontiguousarray(branch, dtype=np.int8).reshape(k, self.D)
        f = np.zeros((Q(self.D), k))
        g = np.zeros((Q(self.D), k))
        rc = lib().orc_step_sampled_branch(self._h, nodes.ctypes.data_as(C.POINTER(C.c_long)), k,
                                           br.ctypes.data_as(C.POINTER(C.c_byte)), _ptr(f), _ptr(g))
        if rc != 0:
            raise ValueError("oracle: step_sampled_branch failed")
        return f, g

    def set_fp32_storage(self, f_ref=None, g_ref=None):
        """FP32 storage model (see oracle.h); None switches it off."""
        if f_ref is None:
            lib().orc_set_fp32_storage(self._h, None, None)
            return
        fr = np.ascontiguousarray(f_ref, dtype=np.float64)
        gr = np.ascontiguousarray(g_ref, dtype=np.float64)
        assert fr.size == Q(self.D) and gr.size == Q(self.D)
        if lib().orc_set_fp32_storage(self._h, _ptr(fr), _ptr(gr)) != 0:
            raise ValueError("oracle: non-finite storage reference")

    def set_upwind_band(self, band):
        """Upwind-side ambiguity model (see oracle.h); 0 switches it off."""
        if lib().orc_set_upwind_band(self._h, float(band)) != 0:
            raise ValueError("oracle: bad upwind band")

    def moments(self):
        rho = np.zeros(self.shape)
        T = np.zeros(self.shape)
        u = np.zeros((self.D,) + self.shape)
        lib().orc_moments(self._h, _ptr(rho), _ptr(u), _ptr(T))
        return rho, u, T

    def diagnostics(self) -> dict:
        out = np.zeros(len(DIAG_NAMES))
        if lib().orc_diagnostics(self._h, _ptr(out)) != 0:
            raise MemoryError("oracle: diagnostics failed")
        return dict(zip(DIAG_NAMES, out.tolist()))

    def get_pops(self):
        f = np.zeros((Q(self.D),) + self.shape)
        g = np.zeros((Q(self.D),) + self.shape)
        lib().orc_get_pops(self._h, _ptr(f), _ptr(g))
        return f, g

    def set_pops(self, f, g, step=0):
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        assert f.size == Q(self.D) * self.N and g.size == f.size
        lib().orc_set_pops(self._h, _ptr(f), _ptr(g), int(step))

    def derivative(self, axis, Qt, u):
        Qt = np.ascontiguousarray(Qt, dtype=np.float64).reshape(self.shape)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.shape)
        out = np.zeros(self.shape)
        lib().orc_derivative(self._h, int(axis), _ptr(Qt), _ptr(u), _ptr(out))
        return out
