"""Two time steps per launch (temporal blocking, lbm_set_fusion): bit-identical to one step per
launch on lattices that tile into 64 x rows blocks, for both storage precisions, every tile-row
option, odd step counts (pairs plus a single step) and moving walls; lattices that do not tile
keep one step per launch; both readings of the diffuse term, chunks with more link entries than a
wave holds, a lattice without walls and wholly solid tiles are covered."""
import sys

import numpy as np
import pytest

from paper_2012_14707_amd import geometry as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _problem(case):
    if case == "cylinders256":
        return G.random_cylinders(n=256, porosity=0.7, rmin=8, rmax=24, seed=11, kn=0.05, h=32.0, ax=1e-6)
    if case == "cylinders128x192":
        return G.random_cylinders(n=128, ny=192, porosity=0.75, rmin=5, rmax=14, seed=4, kn=0.02, h=20.0, ax=2e-6)
    if case == "cylinders2048x128":
        return G.random_cylinders(n=2048, ny=128, porosity=0.75, rmin=5, rmax=14, seed=5, kn=0.02, h=20.0, ax=2e-6)
    if case == "cylinders4096x256":
        # 64 x 64 tiles of 64 x 4 (64 x 32 of 64 x 8): fp32 launches walk them in the banded per-XCD
        # order, which remaps most tiles here (test_banded_tile_order_remaps_this_lattice)
        return G.random_cylinders(n=4096, ny=256, porosity=0.75, rmin=5, rmax=14, seed=6, kn=0.02, h=20.0, ax=2e-6)
    if case == "box128x16":
        # fully periodic, no walls: every tile's link range is empty
        return dict(params=G.base_params(periodic_x=1, periodic_y=1, tau_s_override=0.8, tau_q_override=1.1,
                                         ax=1e-5, ay=-2e-6),
                    solid=np.zeros((16, 128), np.uint8), links=G._empty_links(), meta=dict(kind="box"))
    if case == "slab128x32":
        # periodic channel whose wall is a 12-row solid slab with a ragged face: whole 64 x 4 and
        # 64 x 8 tiles are solid (no site of theirs is loaded, collided or stored)
        s = np.zeros((32, 128), np.uint8)
        s[8:20] = 1
        x = np.arange(128)
        s[7, (x % 5) == 0] = 1
        s[20, (x % 7) == 3] = 1
        xs, ys, ds = G.wall_candidates(s, 1, 1)
        q = np.random.default_rng(7).uniform(0.05, 1.0, len(xs))
        return dict(params=G.base_params(periodic_x=1, periodic_y=1, kn=0.05, h=18.0, ax=2e-6), solid=s,
                    links=dict(x=xs, y=ys, dir=ds, q=q, ubx=np.zeros(len(xs)), uby=np.zeros(len(xs))),
                    meta=dict(kind="slab"))
    if case == "channel64":
        return G.channel(30, nx=64, gamma=0.37, kn=0.05, ax=1e-6, u_top=0.01)
    if case == "annulus128":
        return G.annulus(128, 20.0, 50.0, (63.5, 63.5), u_inner=0.01, u_outer=-0.004, kn=0.05)
    raise KeyError(case)


def _fields(shape, seed):
    rng = np.random.default_rng(seed)
    ny, nx = shape
    y, x = np.mgrid[0:ny, 0:nx]
    ph = rng.random(3) * 2 * np.pi
    rho = 1.0 + 0.01 * np.sin(2 * np.pi * x / nx + ph[0])
    ux = 1e-3 * np.cos(2 * np.pi * 2 * y / ny + ph[1])
    uy = 5e-4 * np.sin(2 * np.pi * 3 * x / nx + ph[2])
    return rho, ux, uy


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a.moments_host(), b.moments_host()))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["cylinders256", "cylinders128x192", "cylinders2048x128", "cylinders4096x256",
                                  "channel64", "annulus128", "box128x16", "slab128x32"])
def test_two_step_launch_bitwise(case, precision):
    from paper_2012_14707_amd import lbm
    pb = _problem(case)
    fused = lbm.Lattice(pb, precision=precision)
    single = lbm.Lattice(pb, precision=precision)
    # default: two steps per launch where the lattice tiles
    assert fused.info["steps_per_launch"] == 2
    fused.set_fusion(2)
    assert fused.info["steps_per_launch"] == 2
    single.set_fusion(1)
    assert single.info["steps_per_launch"] == 1
    init = _fields(pb["solid"].shape, 3)
    for lat in (fused, single):
        lat.init_fields(*init)
    done = 0
    for rows in (8, 4):
        fused.set_fusion(2, rows)
        for n in (37, 2, 1, 60):
            fused.step(n)
            single.step(n)
            done += n
            assert _same(fused, single), (case, precision, rows, n)
            assert fused.residual() == single.residual()
    _say(f"[fused] {case} {precision}: {done} steps bitwise equal, residual {single.residual()[0]:.3e}")
    assert fused.info["steps"] == single.info["steps"] == done


def _xcd_tile(b, ntiles):
    return b if ntiles % 8 else (b % 8) * (ntiles // 8) + b // 8


def _band_tile(b, ntiles, tiles_x):
    """Tile of block b in the fp32 two-step launch: XCD b % 8 walks its contiguous run of tiles in
    bands of 4 tile rows x 32 tile columns, column-major within a band."""
    per = ntiles // 8
    if ntiles % 8 or tiles_x % 32 or per % (4 * tiles_x):
        return _xcd_tile(b, ntiles)
    xg, v = b % 8, b // 8
    band, w = v // (4 * tiles_x), v % (4 * tiles_x)
    grp, rem = w // 128, w % 128
    return xg * per + (band * 4 + rem // 32) * tiles_x + grp * 32 + rem % 32


@pytest.mark.parametrize("rows", [4, 8])
def test_banded_tile_order_remaps_this_lattice(rows):
    """The 4096 x 256 case takes the banded order (a permutation of the tiles that differs from the
    plain per-XCD runs for most blocks); the 2048 x 128 case does not remap any tile."""
    for (nx, ny), want_remapped in (((4096, 256), True), ((2048, 128), False)):
        tiles_x, ntiles = nx // 64, (nx // 64) * (ny // rows)
        band = [_band_tile(b, ntiles, tiles_x) for b in range(ntiles)]
        assert sorted(band) == list(range(ntiles))
        moved = sum(t != _xcd_tile(b, ntiles) for b, t in enumerate(band))
        assert (moved > ntiles // 2) == want_remapped, (nx, ny, rows, moved)


def test_lattices_that_do_not_tile_keep_single_steps():
    from paper_2012_14707_amd import lbm
    lat = lbm.Lattice(G.poiseuille_config1(), precision="fp64")
    assert lat.info["steps_per_launch"] == 1
    with pytest.raises(lbm.LbmError):
        lat.set_fusion(2)
    lat2 = lbm.Lattice(_problem("cylinders256"), precision="fp32")
    with pytest.raises(lbm.LbmError):
        lat2.set_fusion(2, 16)  # tiles have 4 or 8 rows
    with pytest.raises(lbm.LbmError):
        lat2.set_fusion(3)


def _slits():
    """One-site-wide periodic slits (even rows solid): every fluid site has six wall links, so each
    64-site chunk owns 384 link entries, far more than one wave holds per chunk row."""
    ny, nx = 16, 128
    solid = np.zeros((ny, nx), np.uint8)
    solid[0::2, :] = 1
    xs, ys, ds = G.wall_candidates(solid, 1, 1)
    q = np.array([0.3, 0.5, 0.7])[np.arange(len(xs)) % 3]
    links = dict(x=xs, y=ys, dir=ds, q=q, ubx=np.zeros(len(xs)), uby=np.zeros(len(xs)))
    params = G.base_params(periodic_x=1, periodic_y=1, kn=0.05, h=20.0, ax=1e-6)
    return dict(params=params, solid=solid, links=links, meta=dict(kind="slits"))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_two_step_launch_many_links_per_chunk(precision):
    from paper_2012_14707_amd import lbm
    pb = _slits()
    lk = pb["links"]
    per_chunk = np.bincount((lk["y"].astype(np.int64) * pb["solid"].shape[1] + lk["x"]) // 64)
    assert per_chunk.max() > 64
    fused = lbm.Lattice(pb, precision=precision)
    single = lbm.Lattice(pb, precision=precision)
    assert fused.info["steps_per_launch"] == 2
    single.set_fusion(1)
    init = _fields(pb["solid"].shape, 5)
    for lat in (fused, single):
        lat.init_fields(*init)
    for n in (37, 2, 1, 60):
        fused.step(n)
        single.step(n)
        assert _same(fused, single), (precision, n)
    assert np.isfinite(single.moments_host()[1]).all()
    _say(f"[fused] slits {precision}: {per_chunk.max()} links per chunk, 100 steps bitwise equal")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["cylinders256", "annulus128"])
def test_two_step_launch_wall_reading(case, precision):
    """The wall reading of the diffuse term (diffuse = wall; the annulus has moving walls): two steps
    per launch stay bit-identical to single steps, residual included."""
    from paper_2012_14707_amd import lbm
    pb = _problem(case)
    pb["params"] = dict(pb["params"], diffuse="wall")
    fused = lbm.Lattice(pb, precision=precision)
    single = lbm.Lattice(pb, precision=precision)
    assert fused.info["steps_per_launch"] == 2
    single.set_fusion(1)
    init = _fields(pb["solid"].shape, 9)
    for lat in (fused, single):
        lat.init_fields(*init)
    for n in (37, 2, 1, 60):
        fused.step(n)
        single.step(n)
        assert _same(fused, single), (case, precision, n)
        assert fused.residual() == single.residual()
    assert np.isfinite(single.moments_host()[1]).all()
    _say(f"[fused] {case} wall reading {precision}: 100 steps bitwise equal")
