"""ctypes binding of liblbm (include/lbm.h): argument marshalling only.

Every step of the lattice path runs in the HIP kernels of ``lib/liblbm.so``; this module turns a
problem dict (``paper_2012_14707_amd.geometry``) into the C structs, passes torch device
pointers and the current torch stream, and raises ``LbmError`` on any non-zero status.  It
fails loudly when the library is missing: there is no CPU fallback.
"""
import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "liblbm.so")

L_MODES = {"paper": 0, "clamp_neg": 1, "zero": 2, "gamma": 3, "two_gamma": 4, "gamma2": 5,
           "gamma2_plus_gamma": 6, "fixed": 7, "wall_fit": 8}
R_MODES = {"from_leff": 0, "paper": 1, "fixed": 2, "wall_fit": 3}
DIFFUSE = {"node": 0, "wall": 1}
PRECISION = {"fp64": 0, "fp32": 1}

STATUS = {0: "LBM_OK", -1: "LBM_E_INVAL", -2: "LBM_E_NOMEM", -3: "LBM_E_HIP", -4: "LBM_E_GEOMETRY",
          -5: "LBM_E_PARAM", -6: "LBM_E_UNSTABLE", -7: "LBM_E_STATE"}


class LbmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Link(C.Structure):
    _fields_ = [("x", C.c_int32), ("y", C.c_int32), ("dir", C.c_int32), ("reserved", C.c_int32),
                ("q", C.c_double), ("ubx", C.c_double), ("uby", C.c_double)]


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
        ("kn", C.c_double), ("h", C.c_double), ("sigma", C.c_double), ("L1", C.c_double), ("L2", C.c_double),
        ("E", C.c_double), ("tau_rho", C.c_double), ("tau_e", C.c_double), ("tau_eps", C.c_double),
        ("tau_j", C.c_double), ("tau_s_override", C.c_double), ("tau_q_override", C.c_double),
        ("r_override", C.c_double), ("l_override", C.c_double),
        ("l_mode", C.c_int32), ("r_mode", C.c_int32), ("diffuse", C.c_int32), ("precision", C.c_int32),
        ("ax", C.c_double), ("ay", C.c_double), ("rho0", C.c_double),
    ]


class Info(C.Structure):
    _fields_ = [("tau_s", C.c_double), ("tau_q", C.c_double), ("E", C.c_double), ("E_max", C.c_double),
                ("L1", C.c_double), ("L2", C.c_double), ("nu", C.c_double),
                ("n_sites", C.c_int64), ("n_fluid", C.c_int64), ("n_links", C.c_int64),
                ("n_clamped", C.c_int32), ("n_nonconvex", C.c_int32), ("precision", C.c_int32),
                ("steps_per_launch", C.c_int32), ("bytes_per_step", C.c_int64), ("steps", C.c_int64)]


class BatchLaunch(C.Structure):
    _fields_ = [("block", C.c_int32), ("graph_steps", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("reserved", C.c_int32)]


class NnConfig(C.Structure):
    _fields_ = [("levels", C.c_int32), ("base_channels", C.c_int32), ("in_channels", C.c_int32),
                ("out_channels", C.c_int32), ("height", C.c_int32), ("width", C.c_int32),
                ("max_batch", C.c_int32), ("periodic", C.c_int32)]


BATCH_STATUS = {0: "running", 1: "converged", 2: "floor", 3: "capped", 4: "diverged"}

# Every entry point of include/lbm.h with its ctypes signature.
_VP = C.c_void_p
_DPTR = C.POINTER(C.c_double)
SIGNATURES = {
    "lbm_version": (C.c_int32, []),
    "lbm_last_error": (C.c_char_p, []),
    "lbm_params_default": (C.c_int32, [C.POINTER(Params)]),
    "lbm_params_comparison": (C.c_int32, [C.POINTER(Params), C.c_int32, C.c_double]),
    "lbm_create": (C.c_int32, [C.POINTER(Params), _VP, C.POINTER(Link), C.c_int64, _VP, C.POINTER(_VP)]),
    "lbm_destroy": (C.c_int32, [_VP]),
    "lbm_get_info": (C.c_int32, [_VP, C.POINTER(Info)]),
    "lbm_link_coeffs": (C.c_int32, [_VP, _VP]),
    "lbm_init_rest": (C.c_int32, [_VP]),
    "lbm_init_fields": (C.c_int32, [_VP, _VP, _VP, _VP, C.c_int32]),
    "lbm_init_fields_neq": (C.c_int32, [_VP, _VP, _VP, _VP, C.c_int32]),
    "lbm_step": (C.c_int32, [_VP, C.c_int64]),
    "lbm_moments": (C.c_int32, [_VP, _VP, _VP, _VP, C.c_int32]),
    "lbm_residual": (C.c_int32, [_VP, _DPTR, _DPTR]),
    "lbm_set_stream": (C.c_int32, [_VP, _VP]),
    "lbm_synchronize": (C.c_int32, [_VP]),
    "lbm_set_launch": (C.c_int32, [_VP, C.c_int32]),
    "lbm_stream_copy": (C.c_int32, [_VP, _VP, C.c_int64, _VP]),
    "lbm_set_timing": (C.c_int32, [_VP, C.c_int32]),
    "lbm_set_graphs": (C.c_int32, [_VP, C.c_int32]),
    "lbm_set_fusion": (C.c_int32, [_VP, C.c_int32, C.c_int32]),
    "lbm_last_step_ms": (C.c_int32, [_VP, _DPTR, C.POINTER(C.c_int64)]),
    "lbm_batch_create": (C.c_int32, [C.c_int32, C.POINTER(Params), C.POINTER(_VP), C.POINTER(_VP),
                                     C.POINTER(C.c_int64), _VP, C.POINTER(_VP)]),
    "lbm_batch_destroy": (C.c_int32, [_VP]),
    "lbm_batch_info": (C.c_int32, [_VP, C.c_int32, C.POINTER(Info)]),
    "lbm_batch_init_rest": (C.c_int32, [_VP]),
    "lbm_batch_step": (C.c_int32, [_VP, C.c_int64]),
    "lbm_batch_set_active": (C.c_int32, [_VP, _VP]),
    "lbm_batch_residuals": (C.c_int32, [_VP, _VP, _VP]),
    "lbm_batch_moments": (C.c_int32, [_VP, C.c_int32, _VP, _VP, _VP, C.c_int32]),
    "lbm_batch_solve": (C.c_int32, [_VP, C.c_double, C.c_int64, C.c_int64, _VP, _VP, _VP]),
    "lbm_batch_set_params": (C.c_int32, [_VP, C.c_int32, C.POINTER(Params)]),
    "lbm_batch_solve_fallback": (C.c_int32, [_VP, C.c_double, C.c_int64, C.c_int64, _VP, _VP, _VP, _VP]),
    "lbm_batch_set_launch": (C.c_int32, [_VP, C.POINTER(BatchLaunch)]),
    "lbm_batch_get_launch": (C.c_int32, [_VP, C.POINTER(BatchLaunch)]),
    "lbm_batch_tune": (C.c_int32, [_VP, C.c_char_p, C.c_int32, C.POINTER(BatchLaunch)]),
    "lbm_conv2d_forward": (C.c_int32, [_VP, _VP, _VP, _VP, _VP] + [C.c_int32] * 8 + [_VP]),
    "lbm_conv2d_dgrad": (C.c_int32, [_VP, _VP, _VP, _VP] + [C.c_int32] * 7 + [_VP]),
    "lbm_conv2d_wgrad_workspace": (C.c_int32, [C.c_int32] * 6 + [C.POINTER(C.c_int64)]),
    "lbm_conv2d_wgrad": (C.c_int32, [_VP, _VP, _VP, _VP, _VP, C.c_int64] + [C.c_int32] * 7 + [_VP]),
    "lbm_nn_create": (C.c_int32, [C.POINTER(NnConfig), C.c_uint64, _VP, C.POINTER(_VP)]),
    "lbm_nn_destroy": (C.c_int32, [_VP]),
    "lbm_nn_param_count": (C.c_int32, [_VP, C.POINTER(C.c_int64)]),
    "lbm_nn_set_params": (C.c_int32, [_VP, _VP]),
    "lbm_nn_get_params": (C.c_int32, [_VP, _VP]),
    "lbm_nn_get_grads": (C.c_int32, [_VP, _VP]),
    "lbm_nn_forward": (C.c_int32, [_VP, _VP, _VP, C.c_int32]),
    "lbm_nn_backward": (C.c_int32, [_VP, _VP, _VP, C.c_int32, _DPTR]),
    "lbm_nn_adam_step": (C.c_int32, [_VP, C.c_float, C.c_float, C.c_float, C.c_float]),
    "lbm_nn_features": (C.c_int32, [_VP, _VP, C.c_int64, C.c_int32, C.c_int32, C.c_float, C.c_float, C.c_float,
                                    _VP, C.c_int32, _VP]),
    "lbm_nn_fields": (C.c_int32, [_VP, C.c_int32, _VP, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                  C.c_double, C.c_double, _VP, _VP, _VP, C.POINTER(C.c_int64), _VP]),
    "lbm_nn_fields_noalloc": (C.c_int32, [_VP, C.c_int32, _VP, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                          C.c_double, C.c_double, C.c_double, _VP, _VP, _VP, C.POINTER(C.c_int64),
                                          _VP]),
}

_lib = None


def load():
    """Loads liblbm.so (after torch, so that both use one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2012_14707_amd/build.py "
                          "(or __graft_entry__.build()); there is no fallback")
    import torch  # noqa: F401  (loads torch's HIP runtime first; liblbm then binds to the same one)
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != 0:
        raise LbmError(status, _lib.lbm_last_error().decode())


def make_params(params, shape, precision="fp64"):
    """C parameter struct from a problem's physical inputs (names as in geometry.base_params)."""
    lib = load()
    p = Params()
    _check(lib.lbm_params_default(C.byref(p)))
    ny, nx = shape
    p.nx, p.ny = nx, ny
    for name, _ in Params._fields_:
        if name in ("nx", "ny", "precision"):
            continue
        if name in params:
            v = params[name]
            if name == "l_mode":
                v = L_MODES[v]
            elif name == "r_mode":
                v = R_MODES[v]
            elif name == "diffuse":
                v = DIFFUSE[v]
            setattr(p, name, v)
    p.precision = PRECISION[precision]
    return p


SCHEMES = {"present": 0, "previous": 1, "halfway_dbb": 2, "wall_reading": 3}
_L_NAMES = {v: k for k, v in L_MODES.items()}
_R_NAMES = {v: k for k, v in R_MODES.items()}
_DIFFUSE_NAMES = {v: k for k, v in DIFFUSE.items()}


def comparison_problem(problem, scheme, gamma_frozen=0.5):
    """A copy of a problem set up for one of the compared boundary schemes (lbm_params_comparison);
    for the halfway DBB scheme every link's q becomes 1/2."""
    lib = load()
    p = make_params(problem["params"], np.asarray(problem["solid"]).shape)
    _check(lib.lbm_params_comparison(C.byref(p), SCHEMES[scheme], float(gamma_frozen)))
    params = dict(problem["params"], l_mode=_L_NAMES[p.l_mode], r_mode=_R_NAMES[p.r_mode],
                  diffuse=_DIFFUSE_NAMES[p.diffuse], tau_q_override=p.tau_q_override)
    links = dict(problem["links"])
    if scheme == "halfway_dbb":
        links["q"] = np.full(len(links["q"]), 0.5)
    return dict(problem, params=params, links=links)


def make_links(links):
    n = len(links["x"])
    arr = (Link * max(n, 1))()
    if n:
        a = np.frombuffer(arr, dtype=np.dtype([("x", "<i4"), ("y", "<i4"), ("dir", "<i4"), ("reserved", "<i4"),
                                               ("q", "<f8"), ("ubx", "<f8"), ("uby", "<f8")]), count=n)
        a["x"] = links["x"]
        a["y"] = links["y"]
        a["dir"] = links["dir"]
        a["q"] = links["q"]
        a["ubx"] = links["ubx"]
        a["uby"] = links["uby"]
    return arr, n


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Lattice:
    """One lattice context of liblbm on the current torch device and stream."""

    def __init__(self, problem, precision="fp64", stream=None):
        lib = load()
        self._lib = lib
        solid = np.ascontiguousarray(problem["solid"], dtype=np.uint8)
        self.shape = solid.shape
        self.precision = precision
        p = make_params(problem["params"], solid.shape, precision)
        links, n = make_links(problem["links"])
        h = C.c_void_p()
        _check(lib.lbm_create(C.byref(p), solid.ctypes.data_as(C.c_void_p), links, n, _stream_handle(stream),
                              C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def info(self):
        i = Info()
        _check(self._lib.lbm_get_info(self._h, C.byref(i)))
        return {name: getattr(i, name) for name, _ in Info._fields_}

    def link_coeffs(self):
        """[n_links, 8]: l_raw, l_eff, r, alpha1, alpha2, alpha3, beta, kappa (caller's link order)."""
        n = self.info["n_links"]
        out = np.zeros((max(n, 1), 8))
        _check(self._lib.lbm_link_coeffs(self._h, out.ctypes.data_as(C.c_void_p)))
        return out[:n]

    def init_rest(self):
        _check(self._lib.lbm_init_rest(self._h))

    def init_fields(self, rho, ux, uy, neq=False):
        """rho, ux, uy: torch float64 CUDA tensors or numpy float64 arrays of the lattice shape;
        neq: add the first-order non-equilibrium stress (lbm_init_fields_neq)."""
        import torch
        fn = self._lib.lbm_init_fields_neq if neq else self._lib.lbm_init_fields
        if isinstance(rho, torch.Tensor):
            t = [x.contiguous() for x in (rho, ux, uy)]
            for x in t:
                if x.dtype != torch.float64 or not x.is_cuda or tuple(x.shape) != self.shape:
                    raise ValueError("fields must be float64 CUDA tensors of the lattice shape")
            _check(fn(self._h, *[C.c_void_p(x.data_ptr()) for x in t], 1))
        else:
            a = [np.ascontiguousarray(x, dtype=np.float64).reshape(self.shape) for x in (rho, ux, uy)]
            _check(fn(self._h, *[x.ctypes.data_as(C.c_void_p) for x in a], 0))

    def step(self, n=1):
        _check(self._lib.lbm_step(self._h, int(n)))

    def moments(self, out=None):
        """(rho, ux, uy) as float64 CUDA tensors (written on the current stream)."""
        import torch
        if out is None:
            out = [torch.empty(self.shape, dtype=torch.float64, device="cuda") for _ in range(3)]
        _check(self._lib.lbm_moments(self._h, *[C.c_void_p(x.data_ptr()) for x in out], 1))
        return out

    def moments_host(self):
        a = [np.zeros(self.shape) for _ in range(3)]
        _check(self._lib.lbm_moments(self._h, *[x.ctypes.data_as(C.c_void_p) for x in a], 0))
        return a

    def residual(self, raise_unstable=True):
        r, m = C.c_double(), C.c_double()
        st = self._lib.lbm_residual(self._h, C.byref(r), C.byref(m))
        if st != 0 and (raise_unstable or st != -6):
            _check(st)
        return r.value, m.value

    def synchronize(self):
        _check(self._lib.lbm_synchronize(self._h))

    def set_launch(self, block=256):
        _check(self._lib.lbm_set_launch(self._h, int(block)))

    def set_fusion(self, steps_per_launch=2, rows=0):
        """1: one step per kernel launch; 2: two steps per launch (temporal blocking)."""
        _check(self._lib.lbm_set_fusion(self._h, int(steps_per_launch), int(rows)))

    def set_timing(self, on=True):
        _check(self._lib.lbm_set_timing(self._h, int(bool(on))))

    def set_graphs(self, on=True):
        """lbm_step by graph replay (default) or by one launch after the other."""
        _check(self._lib.lbm_set_graphs(self._h, int(bool(on))))

    def last_step_ms(self):
        ms, n = C.c_double(), C.c_int64()
        _check(self._lib.lbm_last_step_ms(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def run_to_steady(self, tol, check_every=100, max_steps=2_000_000):
        res = math.inf
        steps = 0
        while steps < max_steps:
            self.step(check_every)
            steps += check_every
            res, _ = self.residual()
            if res <= tol:
                break
        return steps, res


class Batch:
    """Many lattices of uneven size advanced together (lbm_batch_* of include/lbm.h)."""

    def __init__(self, problems, precision="fp32", stream=None):
        lib = load()
        self._lib = lib
        n = len(problems)
        self.shapes = []
        params = (Params * n)()
        solids = (C.c_void_p * n)()
        links = (C.c_void_p * n)()
        counts = (C.c_int64 * n)()
        self._keep = []
        for i, pb in enumerate(problems):
            solid = np.ascontiguousarray(pb["solid"], dtype=np.uint8)
            self.shapes.append(solid.shape)
            params[i] = make_params(pb["params"], solid.shape, precision)
            arr, nl = make_links(pb["links"])
            self._keep += [solid, arr]
            solids[i] = solid.ctypes.data
            links[i] = C.cast(arr, C.c_void_p).value
            counts[i] = nl
        h = C.c_void_p()
        strm = None if stream is False else _stream_handle(stream)
        _check(lib.lbm_batch_create(n, params, solids, links, counts, strm, C.byref(h)))
        self._h = h
        self.n = n
        self.precision = precision
        self._keep = None

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self, i):
        inf = Info()
        _check(self._lib.lbm_batch_info(self._h, int(i), C.byref(inf)))
        return {name: getattr(inf, name) for name, _ in Info._fields_}

    def init_rest(self):
        _check(self._lib.lbm_batch_init_rest(self._h))

    def step(self, n=1):
        _check(self._lib.lbm_batch_step(self._h, int(n)))

    def set_active(self, active):
        a = np.ascontiguousarray(np.asarray(active, dtype=bool).astype(np.uint8))
        _check(self._lib.lbm_batch_set_active(self._h, a.ctypes.data_as(C.c_void_p)))

    def residuals(self, raise_unstable=True):
        r = np.zeros(self.n)
        m = np.zeros(self.n)
        st = self._lib.lbm_batch_residuals(self._h, r.ctypes.data_as(C.c_void_p), m.ctypes.data_as(C.c_void_p))
        if st != 0 and (raise_unstable or st != -6):
            _check(st)
        return r, m

    def moments_host(self, i):
        a = [np.zeros(self.shapes[i]) for _ in range(3)]
        _check(self._lib.lbm_batch_moments(self._h, int(i), *[x.ctypes.data_as(C.c_void_p) for x in a], 0))
        return a

    def solve(self, tol, check_every=100, max_steps=1_000_000):
        """Runs every instance until it retires; returns (status names, steps, residuals)."""
        st = np.zeros(self.n, np.int32)
        steps = np.zeros(self.n, np.int64)
        res = np.zeros(self.n)
        _check(self._lib.lbm_batch_solve(self._h, float(tol), int(check_every), int(max_steps),
                                         st.ctypes.data_as(C.c_void_p), steps.ctypes.data_as(C.c_void_p),
                                         res.ctypes.data_as(C.c_void_p)))
        return [BATCH_STATUS[int(x)] for x in st], steps, res

    def solve_fallback(self, tol, check_every=100, max_steps=1_000_000):
        """lbm_batch_solve_fallback: the solve, then instances that diverged under the paper's l rule
        re-run from rest with every negative l clamped to zero; returns (status names, steps,
        residuals, fell_back flags)."""
        st = np.zeros(self.n, np.int32)
        steps = np.zeros(self.n, np.int64)
        res = np.zeros(self.n)
        fb = np.zeros(self.n, np.uint8)
        _check(self._lib.lbm_batch_solve_fallback(self._h, float(tol), int(check_every), int(max_steps),
                                                  st.ctypes.data_as(C.c_void_p), steps.ctypes.data_as(C.c_void_p),
                                                  res.ctypes.data_as(C.c_void_p), fb.ctypes.data_as(C.c_void_p)))
        return [BATCH_STATUS[int(x)] for x in st], steps, res, fb.astype(bool)

    def set_params(self, i, params):
        """lbm_batch_set_params: new problem statement for instance i (same geometry); resets it to rest."""
        p = make_params(params, self.shapes[i], self.precision)
        _check(self._lib.lbm_batch_set_params(self._h, int(i), C.byref(p)))

    def set_launch(self, block=256, graph_steps=10, blocks_per_cu=4):
        lb = BatchLaunch(int(block), int(graph_steps), int(blocks_per_cu), 0)
        _check(self._lib.lbm_batch_set_launch(self._h, C.byref(lb)))

    def get_launch(self):
        lb = BatchLaunch()
        _check(self._lib.lbm_batch_get_launch(self._h, C.byref(lb)))
        return dict(block=lb.block, graph_steps=lb.graph_steps, blocks_per_cu=lb.blocks_per_cu)

    def tune(self, cache_path=None, trial_steps=100):
        lb = BatchLaunch()
        path = cache_path.encode() if cache_path else None
        _check(self._lib.lbm_batch_tune(self._h, path, int(trial_steps), C.byref(lb)))
        return dict(block=lb.block, graph_steps=lb.graph_steps, blocks_per_cu=lb.blocks_per_cu)


# ------------------------------------------------------------------------------ warm-start network

def _ptr(t):
    """Device pointer of a contiguous torch tensor (None -> NULL)."""
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous"
    return C.c_void_p(t.data_ptr())


def stream_copy(dst, src, stream=None):
    """lbm_stream_copy between two contiguous device tensors of the same size in bytes."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    _check(load().lbm_stream_copy(_ptr(dst), _ptr(src), nbytes, _stream_handle(stream)))


def conv2d_forward(x, w, bias=None, out=None, out32=None, relu=False, periodic=False, stream=None):
    """lbm_conv2d_forward on NHWC torch tensors: x bf16 [n,h,w,cin], w bf16 [k*k,cout,cin]."""
    import torch
    n, h, wd, cin = x.shape
    kk, cout, cin2 = w.shape
    assert cin2 == cin and x.dtype == w.dtype == torch.bfloat16
    assert out is None or (tuple(out.shape) == (n, h, wd, cout) and out.dtype == torch.bfloat16)
    assert out32 is None or (tuple(out32.shape) == (n, h, wd, cout) and out32.dtype == torch.float32)
    assert bias is None or (bias.numel() == cout and bias.dtype == torch.float32)
    _check(load().lbm_conv2d_forward(_ptr(x), _ptr(w), _ptr(bias), _ptr(out), _ptr(out32), n, h, wd, cin, cout,
                                     int(round(kk ** 0.5)), int(bool(relu)), int(bool(periodic)), _stream_handle(stream)))


def conv2d_dgrad(dout, w, din, periodic=False, stream=None):
    import torch
    n, h, wd, cout = dout.shape
    kk, cout2, cin = w.shape
    assert cout2 == cout and dout.dtype == w.dtype == din.dtype == torch.bfloat16
    assert tuple(din.shape) == (n, h, wd, cin)
    wt = torch.empty_like(w)
    _check(load().lbm_conv2d_dgrad(_ptr(dout), _ptr(w), _ptr(din), _ptr(wt), n, h, wd, cin, cout,
                                   int(round(kk ** 0.5)), int(bool(periodic)), _stream_handle(stream)))


def conv2d_wgrad(x, dout, dw, db=None, periodic=False, stream=None):
    import torch
    n, h, wd, cin = x.shape
    cout = dout.shape[-1]
    k = int(round(dw.shape[0] ** 0.5))
    assert tuple(dout.shape[:3]) == (n, h, wd) and tuple(dw.shape[1:]) == (cout, cin)
    assert x.dtype == dout.dtype == torch.bfloat16 and dw.dtype == torch.float32
    assert db is None or (db.numel() == cout and db.dtype == torch.float32)
    lib = load()
    need = C.c_int64()
    _check(lib.lbm_conv2d_wgrad_workspace(n, h, wd, cin, cout, k, C.byref(need)))
    work = torch.empty(max(int(need.value), 1), dtype=torch.float32, device=x.device)
    _check(lib.lbm_conv2d_wgrad(_ptr(x), _ptr(dout), _ptr(dw), _ptr(db), _ptr(work), int(need.value), n, h, wd, cin,
                                cout, k, int(bool(periodic)), _stream_handle(stream)))


def nn_features(solid, links, nx, ny, kn_feature, ax_feature, ay_feature, out, stream=None):
    """lbm_nn_features: solid uint8 [ny, nx] and links (structured uint8 bytes of lbm_link) on the device."""
    import torch
    n_links = links.numel() // C.sizeof(Link) if links is not None else 0
    assert tuple(solid.shape) == (ny, nx) and solid.dtype == torch.uint8
    assert tuple(out.shape[:2]) == (ny, nx) and out.dtype == torch.bfloat16
    assert links is None or (links.dtype == torch.uint8 and links.numel() == n_links * C.sizeof(Link))
    _check(load().lbm_nn_features(_ptr(solid), _ptr(links) if n_links else None, n_links, nx, ny, float(kn_feature),
                                  float(ax_feature), float(ay_feature), _ptr(out), out.shape[-1],
                                  _stream_handle(stream)))


def nn_fields(pred, solid, nx, ny, u_scale, rho_scale, rho0, rho, ux, uy, smooth_iters=0, periodic=False,
              stream=None, noalloc=False):
    """lbm_nn_fields (or lbm_nn_fields_noalloc, which uses the library's fixed scratch instead of
    allocating); returns the number of fluid sites with a non-finite prediction."""
    import torch
    assert pred.dtype == torch.float32 and pred.numel() == nx * ny * pred.shape[-1] and pred.shape[-1] >= 3
    assert solid.numel() == nx * ny and solid.dtype == torch.uint8
    assert all(t.numel() == nx * ny and t.dtype == torch.float64 for t in (rho, ux, uy))
    bad = C.c_int64()
    fn = load().lbm_nn_fields_noalloc if noalloc else load().lbm_nn_fields
    _check(fn(_ptr(pred), pred.shape[-1], _ptr(solid), nx, ny, int(smooth_iters), int(bool(periodic)),
              float(u_scale), float(rho_scale), float(rho0), _ptr(rho), _ptr(ux), _ptr(uy), C.byref(bad),
              _stream_handle(stream)))
    return int(bad.value)


class Net:
    """The warm-start encoder-decoder of liblbm (lbm_nn_* of include/lbm.h)."""

    def __init__(self, levels=5, base_channels=32, in_channels=12, out_channels=3, height=256, width=256,
                 max_batch=8, periodic=False, seed=0, stream=None):
        lib = load()
        self._lib = lib
        self.cfg = NnConfig(levels, base_channels, in_channels, out_channels, height, width, max_batch,
                            int(bool(periodic)))
        self.in_pad = (in_channels + 7) // 8 * 8
        h = C.c_void_p()
        _check(lib.lbm_nn_create(C.byref(self.cfg), int(seed), _stream_handle(stream), C.byref(h)))
        self._h = h
        cnt = C.c_int64()
        _check(lib.lbm_nn_param_count(h, C.byref(cnt)))
        self.n_params = int(cnt.value)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lbm_nn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        a = np.zeros(self.n_params, np.float32)
        _check(self._lib.lbm_nn_get_params(self._h, a.ctypes.data_as(C.c_void_p)))
        return a

    def set_params(self, a):
        a = np.ascontiguousarray(a, dtype=np.float32)
        assert a.size == self.n_params
        _check(self._lib.lbm_nn_set_params(self._h, a.ctypes.data_as(C.c_void_p)))

    def get_grads(self):
        a = np.zeros(self.n_params, np.float32)
        _check(self._lib.lbm_nn_get_grads(self._h, a.ctypes.data_as(C.c_void_p)))
        return a

    def forward(self, x, out=None):
        """x: bf16 device tensor [n, h, w, in_pad]; out: fp32 [n, h, w, out_channels] or None."""
        import torch
        n = int(x.shape[0])
        assert tuple(x.shape) == (n, self.cfg.height, self.cfg.width, self.in_pad) and x.dtype == torch.bfloat16
        assert out is None or (tuple(out.shape) == (n, self.cfg.height, self.cfg.width, self.cfg.out_channels)
                               and out.dtype == torch.float32)
        _check(self._lib.lbm_nn_forward(self._h, _ptr(x), _ptr(out), int(x.shape[0])))
        return out

    def backward(self, target, mask):
        import torch
        n = int(mask.shape[0])
        assert tuple(mask.shape) == (n, self.cfg.height, self.cfg.width) and mask.dtype == torch.uint8
        assert tuple(target.shape) == (n, self.cfg.height, self.cfg.width, self.cfg.out_channels)
        assert target.dtype == torch.float32
        loss = C.c_double()
        _check(self._lib.lbm_nn_backward(self._h, _ptr(target), _ptr(mask), int(mask.shape[0]), C.byref(loss)))
        return loss.value

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(self._lib.lbm_nn_adam_step(self._h, float(lr), float(beta1), float(beta2), float(eps)))
