"""Input generators: masks and wall-link tables (CPU only).

gamma is the distance ratio of Fig. 1 (Sec. III.A); the checks compare the closed-form circle
crossing with bisection on the inside/outside predicate, check that every fluid-to-solid
neighbour has exactly one link, and that the seeded cylinder arrays hit their porosity."""
import numpy as np
import pytest

from paper_2012_14707_amd import geometry as G


def _bisect(px, py, dx, dy, R, inside_is_solid=True, iters=200):
    """Bisection on the predicate 'point is solid' along the link (brute force)."""
    def solid(t):
        d2 = (px + t * dx) ** 2 + (py + t * dy) ** 2
        return d2 <= R * R if inside_is_solid else d2 >= R * R
    lo, hi = 0.0, 1.0
    assert not solid(lo) and solid(hi)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if solid(mid):
            hi = mid
        else:
            lo = mid
    return hi


def test_circle_crossing_matches_bisection():
    pb = G.couette_config2(0.05)
    L = pb["links"]
    cx, cy = pb["meta"]["center"]
    inner = pb["meta"]["inner"]
    rng = np.random.default_rng(0)
    idx = rng.choice(len(L["x"]), 300, replace=False)
    for k in idx:
        d = L["dir"][k]
        px, py = L["x"][k] - cx, L["y"][k] - cy
        R = 32.0 if inner[k] else 64.0
        t = _bisect(px, py, G.CX[d], G.CY[d], R, inside_is_solid=bool(inner[k]))
        # both sides round |p|^2 - R^2 with R^2 ~ 4e3, so agreement is limited to ~1e-14 .. 1e-13
        assert abs(t - L["q"][k]) < 1e-13


def test_annulus_links_complete_and_consistent():
    pb = G.couette_config2(0.01)
    s, L = pb["solid"], pb["links"]
    assert ((L["q"] > 0) & (L["q"] <= 1)).all()
    keys = set(zip(L["x"].tolist(), L["y"].tolist(), L["dir"].tolist()))
    assert len(keys) == len(L["x"])
    yy, xx = np.nonzero(s == 0)
    for d in range(1, 9):
        hit = s[yy + G.CY[d], xx + G.CX[d]] == 1
        for x, y in zip(xx[hit], yy[hit]):
            assert (x, y, d) in keys
    # wall speed: 0.01 on the inner cylinder (tangential), 0 on the outer one
    inner = pb["meta"]["inner"]
    sp = np.hypot(L["ubx"], L["uby"])
    assert np.allclose(sp[inner], 0.01, rtol=1e-12) and np.all(sp[~inner] == 0)
    # edges are solid: the mask is padded
    assert s[0].all() and s[-1].all() and s[:, 0].all() and s[:, -1].all()


def test_channel_config1_links():
    pb = G.poiseuille_config1()
    assert pb["solid"].shape == (22, 4)
    assert len(pb["links"]["x"]) == 24
    assert np.all(pb["links"]["q"] == 0.3)
    assert pb["meta"]["H"] == pytest.approx(19.6)
    bottom = pb["links"]["y"] == 1
    assert set(pb["links"]["dir"][bottom].tolist()) == {4, 7, 8}
    assert set(pb["links"]["dir"][~bottom].tolist()) == {2, 5, 6}


def test_random_cylinders_porosity_gap_and_crossing():
    pb = G.random_cylinders(n=512, porosity=0.7, rmin=8, rmax=24, seed=3)
    cyl = pb["meta"]["cylinders"]
    por = pb["meta"]["porosity"]
    assert 0.7 - np.pi * 24 ** 2 / 512 ** 2 <= por <= 0.7
    assert por == pytest.approx(1.0 - pb["solid"].mean(), abs=1e-12)
    n = 512
    for i in range(len(cyl)):
        dx = cyl[i, 0] - cyl[:, 0]
        dy = cyl[i, 1] - cyl[:, 1]
        dx -= n * np.round(dx / n)
        dy -= n * np.round(dy / n)
        gap = np.hypot(dx, dy) - cyl[i, 2] - cyl[:, 2]
        gap[i] = np.inf
        assert gap.min() >= 2.0
    L = pb["links"]
    assert ((L["q"] > 0) & (L["q"] <= 1)).all()
    lab = pb["meta"]["label"]
    rng = np.random.default_rng(1)
    for k in rng.choice(len(L["x"]), 200, replace=False):
        d = L["dir"][k]
        xn, yn = (L["x"][k] + G.CX[d]) % n, (L["y"][k] + G.CY[d]) % n
        c = cyl[lab[yn, xn]]
        px = L["x"][k] - c[0]
        py = L["y"][k] - c[1]
        px -= n * np.round(px / n)
        py -= n * np.round(py / n)
        assert abs(_bisect(px, py, G.CX[d], G.CY[d], c[2]) - L["q"][k]) < 1e-13
    # determinism of the seeded generator
    pb2 = G.random_cylinders(n=512, porosity=0.7, rmin=8, rmax=24, seed=3)
    assert np.array_equal(pb["solid"], pb2["solid"]) and np.array_equal(pb["links"]["q"], pb2["links"]["q"])


def test_unpadded_mask_rejected():
    s = np.zeros((5, 5), np.uint8)
    s[2, 2] = 1
    with pytest.raises(ValueError):
        G.wall_candidates(s, 0, 0)


@pytest.mark.parametrize("tan_theta", [0.2, 1.2, 2.0])
def test_inclined_channel_links_cross_the_walls(tan_theta):
    pb = G.inclined_channel(tan_theta)
    ny, nx = pb["solid"].shape
    assert (nx * tan_theta) % ny == pytest.approx(0.0, abs=1e-9) or (nx * tan_theta) % ny == pytest.approx(ny)
    L = pb["links"]
    t, off, nab = tan_theta, pb["meta"]["offset"], pb["meta"]["n_ab"]
    cx, cy = G.CX[L["dir"]], G.CY[L["dir"]]
    # the crossing point x_f + q c_d lies on a wall line (v = 0 or v = n_ab, v = y - x tan - offset)
    v = L["y"] + L["q"] * cy - (L["x"] + L["q"] * cx) * t - off
    vm = np.mod(v + 0.5, ny) - 0.5
    on_wall = np.minimum(np.abs(vm), np.abs(vm - nab))
    assert on_wall.max() < 1e-9
    assert np.all((L["q"] > 0) & (L["q"] <= 1))
    # x_f fluid, x_f + c_d solid (with the periodic wrap), every such pair exactly once
    s = pb["solid"]
    assert np.all(s[L["y"], L["x"]] == 0)
    assert np.all(s[(L["y"] + cy) % ny, (L["x"] + cx) % nx] == 1)
    xs, ys, ds = G.wall_candidates(s, 1, 1)
    assert len(xs) == len(L["x"])
    # the mask is periodic with the walls: shifting x by nx maps v onto itself modulo ny
    assert pb["meta"]["H"] == pytest.approx(nab / np.sqrt(1 + t * t))
    a = np.hypot(pb["params"]["ax"], pb["params"]["ay"])
    assert a == pytest.approx(pb["meta"]["a"]) and pb["params"]["ay"] / pb["params"]["ax"] == pytest.approx(t)
