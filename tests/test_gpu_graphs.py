"""lbm_step by graph replay against one launch after the other: the same launches, so the moments
and the residual must agree bit for bit.  Each context steps through counts that take every path
(fewer than four steps: plain launches; an odd count: a single step after the pairs; more than 256:
several graphs, only the last one recording u) with reads of the moments and residuals in between,
so that every graph is replayed several times with eager work and synchronisation around it."""
import sys

import numpy as np
import pytest

from paper_2012_14707_amd import geometry as G

pytestmark = pytest.mark.gpu

COUNTS = [100, 100, 7, 600, 1, 2, 100, 600]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield


def _problem(case):
    if case == "config1":
        return G.poiseuille_config1()
    return G.random_cylinders(n=256, porosity=0.7, rmin=8, rmax=24, seed=11, kn=0.05, h=32.0, ax=1e-6)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["config1", "cylinders256"])
def test_graph_replay_matches_launches(case, precision):
    from paper_2012_14707_amd import lbm
    pb = _problem(case)
    print(f"[graphs] {case} {precision}", flush=True)
    sys.stdout.flush()
    lat_g = lbm.Lattice(pb, precision=precision)
    lat_e = lbm.Lattice(pb, precision=precision)
    lat_e.set_graphs(False)
    for i, k in enumerate(COUNTS):
        lat_g.step(k)
        lat_e.step(k)
        rg, re = lat_g.residual(), lat_e.residual()
        assert rg == re, (i, k, rg, re)
        for a, b in zip(lat_g.moments_host(), lat_e.moments_host()):
            assert np.array_equal(a, b), (i, k)
    info = lat_g.info
    lat_g.close()
    lat_e.close()
    print(f"[graphs] {case} {precision}: {sum(COUNTS)} steps, {info['steps_per_launch']} per launch, identical",
          flush=True)
