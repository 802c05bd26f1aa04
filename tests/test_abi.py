"""C ABI of liblbm without a GPU: the library loads, exports every entry point include/lbm.h
declares, the binding's structs match the header, and every host-side validation path returns
its documented status before any device work (no compute calls here)."""
import ctypes as C
import math
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2012_14707_amd import geometry as G
from paper_2012_14707_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = lbm.load()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(lbm.SIGNATURES), set(names) ^ set(lbm.SIGNATURES)
    assert lib.lbm_version() >= 10000


def test_struct_layouts(tmp_path):
    """The ctypes mirrors have the size and field offsets the C compiler gives the header's structs."""
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbm.h"', "int main(void) {"]
    for cname, py in (("lbm_link", lbm.Link), ("lbm_params", lbm.Params), ("lbm_info", lbm.Info),
                      ("lbm_batch_launch", lbm.BatchLaunch), ("lbm_nn_config", lbm.NnConfig)):
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    for cname, py in (("lbm_link", lbm.Link), ("lbm_params", lbm.Params), ("lbm_info", lbm.Info),
                      ("lbm_batch_launch", lbm.BatchLaunch), ("lbm_nn_config", lbm.NnConfig)):
        assert int(out[cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_params_default_is_paper():
    lib = lbm.load()
    p = lbm.Params()
    assert lib.lbm_params_default(C.byref(p)) == 0
    assert (p.tau_rho, p.tau_e, p.tau_eps, p.tau_j) == (1.0, 1.1, 1.2, 1.0)
    assert math.isnan(p.L1) and math.isnan(p.L2) and math.isnan(p.E)
    assert p.sigma == 1.0 and p.rho0 == 1.0 and p.l_mode == 0 and p.r_mode == 0 and p.diffuse == 0


def _create(problem, **over):
    lib = lbm.load()
    pr = dict(problem["params"])
    pr.update(over)
    solid = np.ascontiguousarray(problem["solid"], np.uint8)
    p = lbm.make_params(pr, solid.shape)
    links, n = lbm.make_links(problem["links"])
    h = C.c_void_p()
    st = lib.lbm_create(C.byref(p), solid.ctypes.data_as(C.c_void_p), links, n, None, C.byref(h))
    return st, h, lib.lbm_last_error().decode()


def _mutate(problem, fn):
    pb = {"params": dict(problem["params"]), "solid": problem["solid"].copy(),
          "links": {k: v.copy() for k, v in problem["links"].items()}}
    fn(pb)
    return pb


BASE = G.couette_config2(0.05)


@pytest.mark.parametrize("name,fn,code", [
    ("missing link", lambda pb: [pb["links"].__setitem__(k, v[1:]) for k, v in list(pb["links"].items())], -4),
    ("duplicate link", lambda pb: [pb["links"].__setitem__(k, np.concatenate([v, v[:1]]))
                                   for k, v in list(pb["links"].items())], -4),
    ("q out of range", lambda pb: pb["links"]["q"].__setitem__(0, 1.5), -4),
    ("q zero", lambda pb: pb["links"]["q"].__setitem__(0, 0.0), -4),
    ("nan wall velocity", lambda pb: pb["links"]["ubx"].__setitem__(3, np.nan), -4),
    ("link from a solid node", lambda pb: pb["links"]["x"].__setitem__(0, 0), -4),
    ("link toward a fluid node", lambda pb: pb["links"]["dir"].__setitem__(
        0, {1: 3, 2: 4, 3: 1, 4: 2, 5: 7, 6: 8, 7: 5, 8: 6}[int(pb["links"]["dir"][0])]), -4),
    ("direction out of range", lambda pb: pb["links"]["dir"].__setitem__(0, 9), -4),
    ("unpadded edge", lambda pb: pb["solid"].__setitem__((0, 66), 0), -4),
])
def test_geometry_errors(name, fn, code):
    st, h, msg = _create(_mutate(BASE, fn))
    assert st == code, (name, st, msg)
    assert not h.value and msg


@pytest.mark.parametrize("over,code", [
    (dict(tau_s_override=0.5), -5),
    (dict(kn=0.0, tau_s_override=0.0), -5),          # tau_s = 1/2 exactly
    (dict(E=5.0), -5),                                # tau_q <= 1/2 by Eq. (EqECond)
    (dict(tau_e=0.4), -5),
    (dict(rho0=0.0), -5),
])
def test_parameter_errors(over, code):
    st, h, msg = _create(BASE, **over)
    assert st == code, (over, st, msg)
    assert not h.value


def test_isolated_fluid_node_rejected():
    s = np.ones((5, 5), np.uint8)
    s[2, 2] = 0
    xs, ys, ds = G.wall_candidates(s, 0, 0)
    pb = {"params": G.base_params(tau_s_override=0.8, tau_q_override=0.9), "solid": s,
          "links": dict(x=xs, y=ys, dir=ds, q=np.full(len(xs), 0.5), ubx=np.zeros(len(xs)), uby=np.zeros(len(xs)))}
    st, h, msg = _create(pb)
    assert st == -4 and "no fluid neighbour" in msg


def test_null_and_size_errors():
    lib = lbm.load()
    h = C.c_void_p()
    assert lib.lbm_create(None, None, None, 0, None, C.byref(h)) == -1
    p = lbm.Params()
    lib.lbm_params_default(C.byref(p))
    s = np.zeros(4, np.uint8)
    assert lib.lbm_create(C.byref(p), s.ctypes.data_as(C.c_void_p), None, 0, None, C.byref(h)) == -1  # 0 x 0
    p.nx, p.ny, p.l_mode = 2, 2, 42
    assert lib.lbm_create(C.byref(p), s.ctypes.data_as(C.c_void_p), None, 0, None, C.byref(h)) == -1
    assert lib.lbm_destroy(None) == 0
    assert lib.lbm_step(None, 1) == -1
    assert lib.lbm_get_info(None, None) == -1


def test_index_width_limits():
    """Lattices of 2^31 sites or more, and more than 2^31 - 1 wall links, are refused before any
    input is read (the kernels index sites and link offsets in 32 bits)."""
    lib = lbm.load()
    solid = np.ascontiguousarray(BASE["solid"], np.uint8)
    links, n = lbm.make_links(BASE["links"])
    h = C.c_void_p()
    p = lbm.make_params(dict(BASE["params"]), solid.shape)
    p.nx, p.ny = 1 << 16, 1 << 15  # 2^31 sites: refused on the size alone
    assert lib.lbm_create(C.byref(p), solid.ctypes.data_as(C.c_void_p), links, n, None, C.byref(h)) == -1
    assert "2^31" in lib.lbm_last_error().decode() and not h.value
    p = lbm.make_params(dict(BASE["params"]), solid.shape)  # valid, but a link count past int32 offsets
    assert lib.lbm_create(C.byref(p), solid.ctypes.data_as(C.c_void_p), links, 1 << 31, None, C.byref(h)) == -1
    assert "2^31 - 1" in lib.lbm_last_error().decode() and not h.value


def test_batch_validation_errors():
    """Batch creation validates every instance on the host and names the failing one."""
    lib = lbm.load()
    good = G.poiseuille_config1()
    bad = _mutate(G.poiseuille_config1(), lambda pb: pb["links"]["q"].__setitem__(0, 2.0))

    def create(problems, precisions):
        n = len(problems)
        params = (lbm.Params * n)()
        solids = (C.c_void_p * n)()
        links = (C.c_void_p * n)()
        counts = (C.c_int64 * n)()
        keep = []
        for i, (pb, prec) in enumerate(zip(problems, precisions)):
            s = np.ascontiguousarray(pb["solid"], np.uint8)
            params[i] = lbm.make_params(pb["params"], s.shape, prec)
            arr, nl = lbm.make_links(pb["links"])
            keep += [s, arr]
            solids[i] = s.ctypes.data
            links[i] = C.cast(arr, C.c_void_p).value
            counts[i] = nl
        h = C.c_void_p()
        st = lib.lbm_batch_create(n, params, solids, links, counts, None, C.byref(h))
        return st, h, lib.lbm_last_error().decode()

    st, h, msg = create([good, good], ["fp32", "fp64"])
    assert st == -1 and not h.value and "precision" in msg
    st, h, msg = create([good, bad], ["fp32", "fp32"])
    assert st == -4 and not h.value and msg.startswith("instance 1")
    assert lib.lbm_batch_destroy(None) == 0
    assert lib.lbm_batch_step(None, 1) == -1


def test_params_comparison_matches_the_paper_formulas():
    """lbm_params_comparison (host only) against the formulas typed from the paper in the tests."""
    from tests import paper_formulas as P
    lib = lbm.load()
    pb = G.inclined_channel(1.2)
    ts = P.tau_s_of_kn(pb["params"]["kn"], pb["params"]["h"])
    L1 = P.l1_poiseuille(1.0)
    L2 = P.l2_poiseuille(L1)
    for scheme, g, want in ((1, 0.3, P.tau_q_slicoeffrtstq(0.3, 0.0, ts, L1, L2)), (1, 0.5, P.tau_q_halfway(ts, L1, L2)),
                            (2, 0.0, P.tau_q_halfway(ts, L1, L2))):
        p = lbm.make_params(pb["params"], pb["solid"].shape)
        assert lib.lbm_params_comparison(C.byref(p), scheme, g) == 0
        assert p.l_mode == lbm.L_MODES["zero"] and p.r_mode == lbm.R_MODES["from_leff"]
        assert p.tau_q_override == pytest.approx(want, rel=1e-13)
    p = lbm.make_params(pb["params"], pb["solid"].shape)
    assert lib.lbm_params_comparison(C.byref(p), 0, 0.0) == 0
    assert p.l_mode == lbm.L_MODES["paper"] and p.tau_q_override == 0.0
    assert lib.lbm_params_comparison(C.byref(p), 3, 0.0) == 0
    assert (p.l_mode, p.r_mode, p.diffuse) == (lbm.L_MODES["wall_fit"], lbm.R_MODES["wall_fit"],
                                               lbm.DIFFUSE["wall"])
    assert p.tau_q_override == 0.0
    wb = lbm.comparison_problem(pb, "wall_reading")
    assert (wb["params"]["l_mode"], wb["params"]["r_mode"], wb["params"]["diffuse"]) == ("wall_fit",) * 2 + ("wall",)
    assert lib.lbm_params_comparison(C.byref(p), 1, 1.5) == -1
    assert lib.lbm_params_comparison(C.byref(p), 7, 0.5) == -1
    assert lib.lbm_params_comparison(None, 0, 0.5) == -1
    # the halfway problem copy puts every link at q = 1/2 and leaves the original alone
    q0 = pb["links"]["q"].copy()
    hb = lbm.comparison_problem(pb, "halfway_dbb")
    assert np.all(hb["links"]["q"] == 0.5) and np.array_equal(pb["links"]["q"], q0)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: asked for more it exits with status 2 and says so, before it
    touches a GPU."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_library_defines_every_kernel_it_launches():
    """Every kernel handle the host code references is defined in the library (a template kernel
    whose host-side instantiation was dropped shows up as an undefined symbol, and loading fails
    only at the first launch of that kernel)."""
    import subprocess
    from paper_2012_14707_amd import build as B
    out = subprocess.run(["nm", "-D", "--undefined-only", B.LIB], capture_output=True, text=True, check=True).stdout
    undefined = [line.split()[-1] for line in out.splitlines() if line.strip()]
    assert not [s for s in undefined if s.startswith("_ZN3lbm")], undefined
