"""The schedule autotuner: the chosen schedule gives the default schedule's
loss and gradient up to rounding, and the cache is written and taken."""
import json

import numpy as np
import pytest
import torch

from _designs import tiny
from _gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m", [[14, 14, 14], [15, 13, 12]])
def test_tune_keeps_results_and_caches(m, tmp_path, monkeypatch):
    from paper_2603_16014_amd import autotune, mtgp
    monkeypatch.setenv("MTGP_TUNE_CACHE", str(tmp_path / "schedules.json"))
    say("autotune", m)
    w = tiny("dseq", len(m), m, 3, seed=91, xi=1e-2, rank=2)
    rng = np.random.default_rng(5)
    y = torch.from_numpy(rng.normal(size=w.N)).cuda()
    plan = mtgp.Plan.from_workload(w, "fp64")
    plan.set_data(y)
    theta = plan.pack_theta(w.theta)
    o0, g0, _ = plan.nll_grad(theta)
    torch.cuda.synchronize()
    o0, g0 = o0.cpu().numpy(), g0.cpu().numpy()
    res = autotune.tune(plan, theta, reps=2)
    assert not res["cached"] and len(res["timings"]) >= len(autotune.CANDIDATES)
    assert plan.schedule == tuple(res["schedule"]) and plan.overlap == res["overlap"]
    o1, g1, _ = plan.nll_grad(theta)
    torch.cuda.synchronize()
    den = abs(o0[0]) + abs(o0[1])
    assert abs(float(o1[2]) - o0[2]) < 1e-12 * den
    assert np.abs(g1.cpu().numpy() - g0).max() < 1e-9 * np.abs(g0).max()
    table = json.loads((tmp_path / "schedules.json").read_text())
    assert len(table) == 1
    # a second plan of the same shape takes the cached choice without timing
    plan2 = mtgp.Plan.from_workload(w, "fp64")
    plan2.set_data(y)
    res2 = autotune.tune(plan2, theta)
    assert res2["cached"] and plan2.schedule == tuple(res["schedule"])


def test_tune_leaves_lattice_plans():
    from paper_2603_16014_amd import autotune, mtgp
    w = tiny("lat", 2, [8, 8], 2, seed=92)
    plan = mtgp.Plan.from_workload(w, "fp64")
    res = autotune.tune(plan, plan.pack_theta(w.theta), use_cache=False)
    assert res["schedule"] is None
