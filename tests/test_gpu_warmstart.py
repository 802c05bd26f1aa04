"""Learned warm start end to end on the GPU: the committed network (trained on steady fields of
the solver, seeds 1000-2999) starts held-out 256^2 random-cylinder problems (seeds from 9000)
closer to steady state than rest, and the converged field is the lattice's own.  The rest start
is the yardstick and the fallback."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def model():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2012_14707_amd import warmstart as W
    return W.Model.load(W.DEFAULT_MODEL)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_warm_start_gains_over_rest(model):
    from paper_2012_14707_amd import warmstart as W
    rows = []
    for seed in range(9000, 9016):
        pb = W.instance(seed)
        r = W.compare(pb, model, tol=1e-8)
        _say(f"[warm] seed {seed} Kn {r['kn']:.4f}: rest {r['rest_steps']} steps {r['rest_wall'] * 1e3:.1f} ms, "
             f"warm {r['warm_steps']} steps {r['warm_wall'] * 1e3:.1f} ms, fallback {r['fallback']}, du {r['u_rel_diff']:.1e}")
        rows.append(r)
    s = W.summarize(rows)
    _say(f"[warm] {s}")
    assert s["all_converged"] and s["fallbacks"] == 0
    # fewer steps to residual 1e-8 than the rest start, in the median and in total
    assert s["step_ratio_median"] < 0.95
    assert sum(r["warm_steps"] for r in rows) < 0.95 * sum(r["rest_steps"] for r in rows)
    # both runs satisfy the same criterion; they differ by what the criterion leaves in the slow modes
    assert s["u_rel_diff_max"] < 1e-3


def test_non_finite_prediction_falls_back_to_rest(model):
    from paper_2012_14707_amd import warmstart as W
    pb = W.instance(9003)
    params = model.net.get_params()
    try:
        bad = params.copy()
        bad[-8] = np.nan  # bias of output row 0 (u_x; the vector ends with the 8 output biases)
        model.net.set_params(bad)
        warm, lat = W.solve(pb, model, tol=1e-8)
        rest, _ = W.solve(pb, None, tol=1e-8, lattice=lat)
        lat.close()
    finally:
        model.net.set_params(params)
    assert warm["fallback"] == "non-finite prediction" and warm["converged"]
    assert warm["steps"] == rest["steps"]
