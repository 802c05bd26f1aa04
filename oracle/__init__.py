"""Python access to the reference oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this
package.  It loads ``_build/liboracle.so`` (compiled from ``lbm_oracle.c`` by ``build.py``) with
ctypes and marshals numpy arrays; every piece of the method's arithmetic lives in the C file.

Problem descriptions are plain dicts (see ``paper_2012_14707_amd.geometry``):
``params`` (physical inputs), ``solid`` (uint8 [ny, nx], 1 = solid) and ``links`` (dict of
arrays x, y, dir, q, ubx, uby; ``dir`` is the direction from the fluid node toward the wall).
"""
import ctypes as C
import math
import os

import numpy as np

from . import build as _build

_L_MODES = {"paper": 0, "clamp_neg": 1, "zero": 2, "gamma": 3, "two_gamma": 4, "gamma2": 5,
            "gamma2_plus_gamma": 6, "fixed": 7, "wall_fit": 8}
_R_MODES = {"from_leff": 0, "paper": 1, "fixed": 2, "wall_fit": 3}
_DIFFUSE = {"node": 0, "wall": 1}
_BC = {"new": 0, "dbb": 1}


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
        ("kn", C.c_double), ("h", C.c_double),
        ("sigma", C.c_double), ("L1", C.c_double), ("L2", C.c_double), ("E", C.c_double),
        ("tau_rho", C.c_double), ("tau_e", C.c_double), ("tau_eps", C.c_double), ("tau_j", C.c_double),
        ("tau_s_override", C.c_double), ("tau_q_override", C.c_double),
        ("r_override", C.c_double), ("l_override", C.c_double),
        ("l_mode", C.c_int32), ("r_mode", C.c_int32), ("diffuse", C.c_int32), ("bc_kind", C.c_int32),
        ("ax", C.c_double), ("ay", C.c_double), ("rho0", C.c_double),
    ]


class _Globals(C.Structure):
    _fields_ = [("tau_s", C.c_double), ("tau_q", C.c_double), ("E", C.c_double), ("E_max", C.c_double),
                ("L1", C.c_double), ("L2", C.c_double), ("nu", C.c_double),
                ("n_clamped", C.c_int32), ("n_nonconvex", C.c_int32)]


_LIBS = {}

_DP = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_I32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_U8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def _lib(variant="ld"):
    if variant in _LIBS:
        return _LIBS[variant]
    path = _build.lib_path(variant)
    if not os.path.exists(path):
        _build.build(force=False)
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.ora_create.argtypes = [C.POINTER(_Params), _U8, C.c_int64, _I32, _I32, _I32, _DP, _DP, _DP,
                               C.POINTER(_Globals), C.POINTER(vp)]
    lib.ora_derive.argtypes = [C.POINTER(_Params), C.c_int64, _DP, C.POINTER(_Globals), _DP]
    lib.ora_destroy.argtypes = [vp]
    lib.ora_destroy.restype = None
    lib.ora_init_rest.argtypes = [vp]
    lib.ora_init_fields.argtypes = [vp, _DP, _DP, _DP]
    lib.ora_init_fields_neq.argtypes = [vp, _DP, _DP, _DP]
    lib.ora_step.argtypes = [vp, C.c_int64]
    lib.ora_moments.argtypes = [vp, _DP, _DP, _DP]
    lib.ora_residual.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.ora_last_link_flux.argtypes = [vp]
    lib.ora_last_link_flux.restype = C.c_double
    lib.ora_get_f.argtypes = [vp, _DP]
    lib.ora_set_f.argtypes = [vp, _DP]
    lib.ora_minv.argtypes = [_DP]
    lib.ora_steps.argtypes = [vp]
    lib.ora_steps.restype = C.c_int64
    for name, n in [("ora_l_of_gamma", 4), ("ora_r_of_l", 3), ("ora_r_of_gamma", 4), ("ora_tau_q_uniform", 4),
                    ("ora_e_max", 3), ("ora_tau_q_general", 5)]:
        fn = getattr(lib, name)
        fn.argtypes = [C.c_double] * n
        fn.restype = C.c_double
    if lib.ora_sizeof_params() != C.sizeof(_Params):
        raise RuntimeError("oracle parameter struct size mismatch")
    _LIBS[variant] = lib
    return lib


DEFAULTS = dict(nx=1, ny=1, periodic_x=0, periodic_y=0, kn=0.0, h=1.0, sigma=1.0, L1=math.nan, L2=math.nan, E=math.nan,
                tau_rho=1.0, tau_e=1.1, tau_eps=1.2, tau_j=1.0, tau_s_override=0.0, tau_q_override=0.0,
                r_override=0.0, l_override=0.0, l_mode="paper", r_mode="from_leff", diffuse="node", bc="new",
                ax=0.0, ay=0.0, rho0=1.0)


def _to_struct(params):
    p = dict(DEFAULTS)
    p.update(params)
    s = _Params()
    for name, _ in _Params._fields_:
        if name == "l_mode":
            s.l_mode = _L_MODES[p["l_mode"]]
        elif name == "r_mode":
            s.r_mode = _R_MODES[p["r_mode"]]
        elif name == "diffuse":
            s.diffuse = _DIFFUSE[p["diffuse"]]
        elif name == "bc_kind":
            s.bc_kind = _BC[p["bc"]]
        else:
            setattr(s, name, p[name])
    return s


def _globals_dict(g):
    return {name: getattr(g, name) for name, _ in _Globals._fields_}


class OracleError(RuntimeError):
    pass


def derive(params, q, variant="ld"):
    """Parameter prescription: returns (globals dict, array [n, 3] of l_raw, l_eff, r per link)."""
    lib = _lib(variant)
    q = np.ascontiguousarray(q, dtype=np.float64)
    out = np.zeros((max(len(q), 1), 3))
    g = _Globals()
    st = lib.ora_derive(C.byref(_to_struct(params)), len(q), q if len(q) else np.zeros(1), C.byref(g), out)
    if st != 0:
        raise OracleError(f"ora_derive failed with status {st}")
    return _globals_dict(g), out[: len(q)]


def formula(name, *args, variant="ld"):
    """Direct access to one closed form of the prescription (for identity checks)."""
    return getattr(_lib(variant), "ora_" + name)(*[float(a) for a in args])


def minv():
    out = np.zeros(81)
    if _lib().ora_minv(out) != 0:
        raise OracleError("ora_minv failed")
    return out.reshape(9, 9)


class Oracle:
    """One lattice problem held by the oracle."""

    def __init__(self, params, solid, links, variant="ld"):
        self._lib = _lib(variant)
        solid = np.ascontiguousarray(solid, dtype=np.uint8)
        ny, nx = solid.shape
        p = dict(params)
        p["nx"], p["ny"] = nx, ny
        self.shape = (ny, nx)
        self.solid = solid
        n = len(links["x"])
        arr = lambda k, dt: np.ascontiguousarray(links[k], dtype=dt) if n else np.zeros(1, dt)
        g = _Globals()
        h = C.c_void_p()
        st = self._lib.ora_create(C.byref(_to_struct(p)), solid.reshape(-1), n, arr("x", np.int32),
                                  arr("y", np.int32), arr("dir", np.int32), arr("q", np.float64),
                                  arr("ubx", np.float64), arr("uby", np.float64), C.byref(g), C.byref(h))
        self.globals = _globals_dict(g)
        if st != 0:
            raise OracleError(f"ora_create failed with status {st}")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.ora_destroy(h)
            self._h = None

    def init_rest(self):
        self._lib.ora_init_rest(self._h)

    def init_fields(self, rho, ux, uy, neq=False):
        """f^eq(rho, u - a/2); with neq, plus the first-order non-equilibrium stress of u's gradients."""
        c = lambda a: np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
        fn = self._lib.ora_init_fields_neq if neq else self._lib.ora_init_fields
        fn(self._h, c(rho), c(ux), c(uy))

    def step(self, n=1):
        self._lib.ora_step(self._h, int(n))

    @property
    def steps(self):
        return self._lib.ora_steps(self._h)

    def moments(self):
        ny, nx = self.shape
        rho, ux, uy = (np.zeros(nx * ny) for _ in range(3))
        self._lib.ora_moments(self._h, rho, ux, uy)
        return rho.reshape(ny, nx), ux.reshape(ny, nx), uy.reshape(ny, nx)

    def residual(self):
        r, m = C.c_double(), C.c_double()
        self._lib.ora_residual(self._h, C.byref(r), C.byref(m))
        return r.value, m.value

    def last_link_flux(self):
        return self._lib.ora_last_link_flux(self._h)

    def get_f(self):
        ny, nx = self.shape
        out = np.zeros(nx * ny * 9)
        self._lib.ora_get_f(self._h, out)
        return out.reshape(ny, nx, 9)

    def set_f(self, f):
        self._lib.ora_set_f(self._h, np.ascontiguousarray(f, dtype=np.float64).reshape(-1))

    def run_to_steady(self, tol, check_every=100, max_steps=2_000_000):
        """Steps in chunks until the residual is <= tol; returns (steps, residual)."""
        res = math.inf
        while self.steps < max_steps:
            self.step(check_every)
            res, _ = self.residual()
            if not math.isfinite(res):
                raise OracleError("oracle run went non-finite")
            if res <= tol:
                break
        return self.steps, res
