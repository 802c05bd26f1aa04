"""Inclined channel (Sec. IV.A.2) and the paper's comparison schemes on the GPU.

The walls are flat but inclined to the lattice, so gamma varies from link to link.  Parity: the GPU
against the oracle for the present scheme, the previous l = 0 scheme with a frozen-gamma tau_q, and
halfway DBB (on the GPU: the same boundary rule with q = 1/2, l = 0 and the parameters of Eqs.
(SliCoeffHar), (SliCoeffHata), set by lbm_params_comparison; in the oracle: its separately coded
DBB rule).  Steady state: the present scheme follows the analytic slip profile within 4% of u_c and
beats both alternatives."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2012_14707_amd import geometry as G
from tests import paper_formulas as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _schemes(pb):
    """(name, GPU problem, oracle parameter overrides) for the three schemes; the oracle's
    parameters are computed from the formulas typed in the tests, not by the library."""
    from paper_2012_14707_amd import lbm
    p = pb["params"]
    ts = P.tau_s_of_kn(p["kn"], p["h"])
    L1 = P.l1_poiseuille(1.0)
    L2 = P.l2_poiseuille(L1)
    return [
        ("present", lbm.comparison_problem(pb, "present"), {}),
        ("previous", lbm.comparison_problem(pb, "previous", 0.5),
         dict(l_mode="zero", tau_q_override=P.tau_q_slicoeffrtstq(0.5, 0.0, ts, L1, L2))),
        ("halfway_dbb", lbm.comparison_problem(pb, "halfway_dbb"),
         dict(bc="dbb", l_mode="zero", tau_q_override=P.tau_q_halfway(ts, L1, L2))),
    ]


def _rel(g, o, solid):
    fl = solid == 0
    return np.max(np.hypot(g[1] - o[1], g[2] - o[2])[fl]) / np.max(np.hypot(o[1], o[2])[fl])


@pytest.mark.parametrize("tan_theta", [0.2, 1.2, 2.0])
def test_inclined_schemes_parity(tan_theta):
    from paper_2012_14707_amd import lbm
    pb = G.inclined_channel(tan_theta)
    for name, gpb, over in _schemes(pb):
        lat = lbm.Lattice(gpb, precision="fp64")
        ora = oracle.Oracle(dict(pb["params"], **over), pb["solid"], pb["links"])
        for lat_or_ora in (lat, ora):
            lat_or_ora.step(600)
        err = _rel(lat.moments_host(), ora.moments(), pb["solid"])
        _say(f"[schemes] tan {tan_theta} {name}: fp64 rel error vs oracle {err:.2e}")
        assert err <= 1e-12, (name, err)
        if name == "present":
            lat32 = lbm.Lattice(gpb, precision="fp32")
            lat32.step(600)
            err32 = _rel(lat32.moments_host(), ora.moments(), pb["solid"])
            assert err32 <= 1e-5, err32


@pytest.mark.parametrize("tan_theta", [0.2, 1.2, 2.0])
def test_inclined_steady_profile_and_ordering(tan_theta):
    from paper_2012_14707_amd import lbm
    pb = G.inclined_channel(tan_theta)
    p = pb["params"]
    ts = P.tau_s_of_kn(p["kn"], p["h"])
    L1 = P.l1_poiseuille(1.0)
    ana, uc = G.inclined_profile(pb, L1, P.l2_poiseuille(L1), (ts - 0.5) / 3)
    fl = pb["solid"] == 0
    c, s = 1 / math.sqrt(1 + tan_theta ** 2), tan_theta / math.sqrt(1 + tan_theta ** 2)
    err = {}
    for name, gpb, _ in _schemes(pb):
        lat = lbm.Lattice(gpb, precision="fp64")
        steps, res = lat.run_to_steady(1e-11, 100, 200_000)
        _, ux, uy = lat.moments_host()
        err[name] = float(np.max(np.abs(ux * c + uy * s - ana)[fl]) / uc)
        _say(f"[schemes] tan {tan_theta} {name}: steady after {steps} steps, max |u - u_analytic| / u_c = "
             f"{err[name]:.4f}")
    assert err["present"] < 0.04
    assert err["present"] < err["previous"] < err["halfway_dbb"]


# ------------------------------------------------- wall reading with re-derived parameters

def test_wall_reading_link_coefficients():
    """The wall-reading fit's per-link (l, r) (closed form, fp64 on the device) against the
    oracle's bisection on the two slip conditions, over the curved walls of the annulus at Kn = 0.05
    (every gamma admissible), and the rejection of inadmissible links at Kn = 0.0194."""
    from paper_2012_14707_amd import lbm
    pb = G.couette_config2(0.05)
    gpb = lbm.comparison_problem(pb, "wall_reading")
    lat = lbm.Lattice(gpb, precision="fp64")
    c = lat.link_coeffs()
    _, lk = oracle.derive(dict(pb["params"], l_mode="wall_fit", r_mode="wall_fit", diffuse="wall"), pb["links"]["q"])
    _say(f"[wall fit] {len(lk)} links, l in [{lk[:, 1].min():.3f}, {lk[:, 1].max():.3f}], "
         f"r in [{lk[:, 2].min():.3f}, {lk[:, 2].max():.3f}]")
    np.testing.assert_allclose(c[:, 0], lk[:, 0], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(c[:, 1], lk[:, 1], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(c[:, 2], lk[:, 2], rtol=1e-11, atol=1e-12)
    assert lat.info["n_clamped"] == 0
    lat.close()
    bad = lbm.comparison_problem(G.inclined_channel(0.2), "wall_reading")
    with pytest.raises(lbm.LbmError) as e:
        lbm.Lattice(bad, precision="fp64")
    assert e.value.status == -5 and "tau_s - L1 Kn H" in str(e.value)
    with pytest.raises(lbm.LbmError) as e:
        lbm.Lattice(dict(gpb, params=dict(gpb["params"], r_mode="from_leff")), precision="fp64")
    assert e.value.status == -1


def test_wall_reading_config1_parity_and_profile():
    """Config 1 under the wall reading with the re-derived parameters: fp64 and fp32 parity with the
    oracle after 300 steps, and the fp64 steady state on the analytic profile of Eq. (numvelo)."""
    from paper_2012_14707_amd import lbm
    pb = G.poiseuille_config1()
    gpb = lbm.comparison_problem(pb, "wall_reading")
    ora = oracle.Oracle(dict(pb["params"], l_mode="wall_fit", r_mode="wall_fit", diffuse="wall"),
                        pb["solid"], pb["links"])
    ora.step(300)
    for precision, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        lat = lbm.Lattice(gpb, precision=precision)
        lat.step(300)
        err = _rel(lat.moments_host(), ora.moments(), pb["solid"])
        _say(f"[wall fit] config 1 {precision}: rel error vs oracle {err:.2e}")
        assert err <= tol, (precision, err)
        lat.close()
    lat = lbm.Lattice(gpb, precision="fp64")
    steps, res = lat.run_to_steady(1e-13, 100, 50_000)
    _, ux, _ = lat.moments_host()
    g = lat.info
    h = pb["meta"]["H"]
    uc = 1e-6 * h * h / (8 * g["nu"])
    U = P.poiseuille_profile(pb["meta"]["y"], h, g["L1"], g["L2"], 0.1)
    e = np.max(np.abs(ux[1:-1, :] / uc - U[:, None])) / U.max()
    _say(f"[wall fit] config 1 steady after {steps} steps (residual {res:.1e}): max rel error vs Eq. (numvelo) {e:.2e}")
    assert e < 1e-9


def test_wall_reading_couette_parity():
    """Moving curved walls (annulus, Kn = 0.05) under the wall reading with the re-derived
    parameters: fp64 parity with the oracle after 200 steps."""
    from paper_2012_14707_amd import lbm
    pb = G.couette_config2(0.05)
    gpb = lbm.comparison_problem(pb, "wall_reading")
    ora = oracle.Oracle(dict(pb["params"], l_mode="wall_fit", r_mode="wall_fit", diffuse="wall"),
                        pb["solid"], pb["links"])
    ora.step(200)
    lat = lbm.Lattice(gpb, precision="fp64")
    lat.step(200)
    err = _rel(lat.moments_host(), ora.moments(), pb["solid"])
    _say(f"[wall fit] annulus Kn 0.05 fp64: rel error vs oracle {err:.2e}")
    assert err <= 1e-12
