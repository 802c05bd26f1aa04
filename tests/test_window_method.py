"""The windowed oracle used by the full-size parity test equals the oracle on the whole lattice.

A small periodic random-cylinder lattice is stepped by the oracle from seeded fields; sampled
sites are then stepped again inside windows of half-width N + 2 (tests/lattice_window.py). The
windows must reproduce the whole-lattice velocities to rounding: same arithmetic, same inputs."""
import numpy as np

import oracle
from paper_2012_14707_amd import geometry as G
from tests.lattice_window import samples, window


def test_window_reproduces_whole_lattice():
    n_steps, half = 5, 7
    pb = G.random_cylinders(n=96, porosity=0.7, rmin=6, rmax=12, seed=3, kn=0.05, h=20.0, ax=1e-6)
    ny, nx = pb["solid"].shape
    rng = np.random.default_rng(5)
    fluid = pb["solid"] == 0
    fields = (np.where(fluid, 1.0 + 2e-3 * rng.standard_normal((ny, nx)), 1.0),
              np.where(fluid, 1e-2 * rng.standard_normal((ny, nx)), 0.0),
              np.where(fluid, 1e-2 * rng.standard_normal((ny, nx)), 0.0))
    whole = oracle.Oracle(pb["params"], pb["solid"], pb["links"])
    whole.init_fields(*fields)
    whole.step(n_steps)
    rho_w, ux_w, uy_w = whole.moments()
    worst = 0.0
    pts = samples(pb, np.random.default_rng(9), n_bulk=12, n_wall=12)
    for cx, cy in pts:
        params, solid, links, init = window(pb, fields, cx, cy, half)
        o = oracle.Oracle(params, solid, links)
        o.init_fields(*init)
        o.step(n_steps)
        rho, ux, uy = o.moments()
        c = half + 1
        worst = max(worst, abs(ux[c, c] - ux_w[cy, cx]), abs(uy[c, c] - uy_w[cy, cx]), abs(rho[c, c] - rho_w[cy, cx]))
    assert worst < 1e-15, worst
    # a window one site too small is not exact: the frame's influence reaches the centre
    params, solid, links, init = window(pb, fields, *pts[0], n_steps - 1)
    o = oracle.Oracle(params, solid, links)
    o.init_fields(*init)
    o.step(n_steps)
    _, ux, _ = o.moments()
    assert abs(ux[n_steps, n_steps] - ux_w[pts[0][1], pts[0][0]]) > 1e-9
