"""Batched persistent launch (lbm_batch_*): every instance computes exactly what a single lattice
with the same inputs computes (bitwise), whatever the launch shape, graph chunking and retirement;
the solve loop retires instances with the right status and the autotuner picks a valid shape."""
import math
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


def _problems():
    from tests.test_gpu_fused import _problem
    ragged = np.zeros((23, 37), np.uint8)
    ragged[0], ragged[-1] = 1, 1
    yy, xx = np.mgrid[0:23, 0:37]
    ragged[(xx - 17.3) ** 2 + (yy - 11.6) ** 2 <= 4.2 ** 2] = 1
    xs, ys, ds = G.wall_candidates(ragged, 1, 0)
    q = np.random.default_rng(0).uniform(0.05, 1.0, len(xs))
    rag = dict(params=G.base_params(periodic_x=1, kn=0.05, h=21.0, ax=1e-5), solid=ragged,
               links=dict(x=xs, y=ys, dir=ds, q=q, ubx=np.zeros(len(xs)), uby=np.zeros(len(xs))),
               meta=dict(kind="ragged"))
    return [
        G.poiseuille_config1(),
        G.annulus(40, 8.0, 18.0, (19.5, 19.5), u_inner=0.02, u_outer=-0.01, kn=0.05),
        rag,
        G.random_cylinders(n=256, porosity=0.7, rmin=8, rmax=24, seed=11, kn=0.05, h=32.0, ax=1e-6),
        G.channel(300, nx=4, gamma=0.77, kn=0.02, ax=2e-7),
        # no wall link at all, and wholly solid tiles (rows 8-19 of the slab: 1536 sites)
        _problem("box128x16"),
        _problem("slab128x32"),
    ]


def _single(pb, precision, steps):
    from paper_2012_14707_amd import lbm
    lat = lbm.Lattice(pb, precision=precision)
    lat.step(steps)
    out = lat.moments_host()
    lat.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_matches_single_bitwise(precision):
    from paper_2012_14707_amd import lbm
    pbs = _problems()
    b = lbm.Batch(pbs, precision=precision)
    b.set_launch(block=256, graph_steps=10, blocks_per_cu=4)
    b.step(37)  # three graph replays and seven eager steps
    for i, pb in enumerate(pbs):
        _say(f"[batch] {precision} instance {i} {pb['meta']['kind']} {pb['solid'].shape}")
        ref = _single(pb, precision, 37)
        got = b.moments_host(i)
        for a, r in zip(got, ref):
            assert np.array_equal(a, r), (precision, i)
    b.close()


def test_batch_launch_shapes_and_retirement_bitwise():
    """Every launch shape gives identical bits; a retired instance keeps its state and resumes
    exactly where it stopped after re-activation."""
    from paper_2012_14707_amd import lbm
    pbs = _problems()
    refs = {(i, s): _single(pb, "fp32", s) for i, pb in enumerate(pbs) for s in (20, 44)}
    for block in (128, 256, 512):
        for gs in (2, 10):
            for bpc in (0, 2, 8):
                b = lbm.Batch(pbs, precision="fp32")
                b.set_launch(block=block, graph_steps=gs, blocks_per_cu=bpc)
                b.step(20)
                act = np.ones(len(pbs), bool)
                act[1] = act[3] = False
                b.set_active(act)
                b.step(24)
                for i in range(len(pbs)):
                    want = refs[(i, 20 if i in (1, 3) else 44)]
                    got = b.moments_host(i)
                    assert all(np.array_equal(x, y) for x, y in zip(got, want)), (block, gs, bpc, i)
                # re-activate: instances 1 and 3 continue from step 20 (odd buffer parity copied across)
                b.set_active(np.ones(len(pbs), bool))
                b.step(24)
                for i in (1, 3):
                    got = b.moments_host(i)
                    assert all(np.array_equal(x, y) for x, y in zip(got, refs[(i, 44)])), (block, gs, bpc, i)
                assert b.info(1)["steps"] == 44 and b.info(0)["steps"] == 68
                b.close()
        _say(f"[batch] launch shapes with block {block} identical")


def test_batch_residuals_and_solve_match_single():
    """Per-instance residual and mass agree with the single-lattice reductions; the solve loop
    stops each instance at the same step count as a single run to the same tolerance."""
    from paper_2012_14707_amd import lbm
    pbs = [G.poiseuille_config1(), G.couette_config2(0.1), G.channel(30, nx=4, gamma=0.6, kn=0.05, ax=1e-6)]
    b = lbm.Batch(pbs, precision="fp64")
    r, m = b.residuals()
    assert np.all(np.isinf(r))
    b.step(100)
    r, m = b.residuals()
    for i, pb in enumerate(pbs):
        lat = lbm.Lattice(pb, precision="fp64")
        lat.step(100)
        rs, ms = lat.residual()
        assert r[i] == pytest.approx(rs, rel=1e-10) and m[i] == pytest.approx(ms, rel=1e-14)
    b.init_rest()
    status, steps, res = b.solve(1e-10, check_every=100, max_steps=200_000)
    _say(f"[batch solve] {status} {steps} {res}")
    assert status == ["converged"] * 3
    for i, pb in enumerate(pbs):
        lat = lbm.Lattice(pb, precision="fp64")
        s, _ = lat.run_to_steady(1e-10, 100, 200_000)
        assert s == steps[i]
        assert all(np.array_equal(x, y) for x, y in zip(b.moments_host(i), lat.moments_host()))


def test_batch_solve_statuses():
    """Capped, floor and converged instances in one solve (fp32 cannot reach 1e-13)."""
    from paper_2012_14707_amd import lbm
    pbs = [G.poiseuille_config1(), G.couette_config2(0.05)]
    b = lbm.Batch(pbs, precision="fp32")
    status, steps, res = b.solve(1e-13, check_every=100, max_steps=3000)
    _say(f"[batch statuses] {status} {steps} {res}")
    assert set(status) <= {"floor", "capped"}
    assert all(s <= 3000 for s in steps)
    b = lbm.Batch(pbs, precision="fp32")
    status, steps, res = b.solve(1e-4, check_every=100, max_steps=100_000)
    assert status == ["converged", "converged"]


def test_batch_tune_and_cache(tmp_path):
    from paper_2012_14707_amd import lbm
    pbs = _problems()
    b = lbm.Batch(pbs, precision="fp32")
    cache = str(tmp_path / "tune.txt")
    chosen = b.tune(cache, trial_steps=40)
    _say(f"[batch tune] chosen {chosen}")
    assert chosen["block"] in (128, 256, 512) and chosen["graph_steps"] in (2, 10, 50)
    assert b.get_launch() == chosen
    text = open(cache).read()
    assert text.count("\n") == 1
    b2 = lbm.Batch(pbs, precision="fp32")
    assert b2.tune(cache, trial_steps=40) == chosen  # served from the cache
    assert open(cache).read() == text
    # tuning leaves the batch at rest: the results equal a fresh run
    b.step(20)
    for i, pb in enumerate(pbs):
        assert all(np.array_equal(x, y) for x, y in zip(b.moments_host(i), _single(pb, "fp32", 20)))


def test_batch_sweep_config4_runs():
    """The 256-instance uneven sweep (fp32): one persistent graph-captured launch per step over
    3.3 M sites; every instance ends with a status and none goes non-finite."""
    from paper_2012_14707_amd import lbm
    pbs = G.batched_sweep_config4()
    b = lbm.Batch(pbs, precision="fp32")
    b.set_launch(block=256, graph_steps=50, blocks_per_cu=4)
    status, steps, res = b.solve(1e-8, check_every=100, max_steps=5000)
    counts = {s: status.count(s) for s in set(status)}
    _say(f"[config4] statuses {counts}, steps min {steps.min()} max {steps.max()}")
    assert "diverged" not in counts and "running" not in counts
