"""Edge cases of the C ABI against the dense oracle: the largest task and
dimension counts the library accepts (T = 16, d = 32), one point per task,
a nested design with 16 tasks down to n = 1, and empty inputs."""
import numpy as np
import pytest
import torch

from _designs import tiny
from _gpu_common import oracle_for, rel_err, say

pytestmark = pytest.mark.gpu


def _check_loss_grad(w, precision="fp64", elimination=None):
    from paper_2603_16014_amd import mtgp as mt
    ref = oracle_for(w, want_grad=True)
    plan = mt.Plan.from_workload(w, precision, elimination=elimination)
    theta = plan.pack_theta(w.theta)
    plan.set_data(torch.from_numpy(ref["y"]).cuda())
    out3, grad, tau = plan.nll_grad(theta)
    torch.cuda.synchronize()
    assert plan.status() == (0, -1)
    r = ref["res"]
    den = abs(r["quad"]) + abs(r["logdet"])
    tolL = 1e-10 if precision == "fp64" else 1e-5
    assert abs(float(out3[2]) - r["L"]) < tolL * den, (out3.cpu().numpy(), r["L"])
    np.testing.assert_allclose(tau.cpu().numpy(), r["tau_hat"], rtol=1e-8, atol=1e-11)
    g = plan.unpack(grad)
    scale = max(np.abs(np.concatenate([np.atleast_1d(v).ravel() for v in ref["grad"].values()])).max(),
                1e-300)
    tolg = 1e-7 if precision == "fp64" else 1e-4
    for k, v in ref["grad"].items():
        assert rel_err(g[k], v, scale) < tolg, k
    return plan, theta


@pytest.mark.parametrize("family", ["dseq", "lat"])
def test_sixteen_tasks(family):
    """T = 16 (the most tasks a plan accepts): 136 task pairs, 16 x 16 solves."""
    say("T=16", family)
    _check_loss_grad(tiny(family, 16, [4] * 16, 2, seed=81, rank=3))


@pytest.mark.parametrize("family", ["dseq", "lat"])
def test_thirty_two_dimensions(family):
    """d = 32 (the most dimensions a plan accepts)."""
    say("d=32", family)
    _check_loss_grad(tiny(family, 2, [6, 6], 32, seed=82, rank=2))


@pytest.mark.parametrize("family", ["dseq", "lat"])
def test_one_point_per_task(family):
    """n_t = 1: every transform is the identity, Lambda is R c(0) + diag(xi)."""
    say("n=1", family)
    _check_loss_grad(tiny(family, 3, [0, 0, 0], 2, seed=83, rank=2))


@pytest.mark.parametrize("family,elimination", [("dseq", "sparse"), ("lat", "sparse"),
                                                ("dseq", "alg1")])
def test_sixteen_nested_tasks_down_to_one_point(family, elimination):
    """Nested sizes over 16 tasks with pairs of equal lengths down to n = 1."""
    m = [6, 6, 5, 5, 4, 4, 3, 3, 2, 2, 1, 1, 0, 0, 0, 0]
    say("nested T=16", family, elimination)
    _check_loss_grad(tiny(family, 16, m, 2, seed=84, rank=2), elimination=elimination)


@pytest.mark.parametrize("family,elimination", [("dseq", "sparse"), ("dseq", "alg1"),
                                                ("lat", "sparse"), ("lat", "alg1")])
def test_sixteen_tasks_nine_distinct_sizes(family, elimination):
    """Sixteen tasks with nine distinct lengths: 9 diagonal columns + 120
    pair columns = 129, so column indices reach 128 (they must not wrap to
    negative values in the pair tables)."""
    from paper_2603_16014_amd import mtgp as mt
    m = [8, 7, 6, 5, 4, 3, 2, 1, 0, 0, 0, 0, 0, 0, 0, 0]
    say("nested T=16, 9 distinct sizes", family, elimination)
    plan, _ = _check_loss_grad(tiny(family, 16, m, 2, seed=87, rank=2), elimination=elimination)
    assert plan.ncol == 129
    assert max(plan.column_info(c)[0] for c in range(plan.ncol)) == 8


def test_empty_inputs():
    """Zero test points, zero transform rows: valid calls that do nothing."""
    from paper_2603_16014_amd import mtgp as mt
    w = tiny("dseq", 2, [5, 5], 2, seed=85)
    say("empty inputs")
    ref = oracle_for(w, want_grad=False)
    plan = mt.Plan.from_workload(w)
    theta = plan.pack_theta(w.theta)
    plan.set_data(torch.from_numpy(ref["y"]).cuda())
    mean = plan.predict(theta, torch.zeros((0, w.d), dtype=torch.int32, device="cuda"))
    assert mean.shape[0] == 0
    x = torch.zeros(0, dtype=torch.float64, device="cuda")
    mt.fwht(x, 4)
    X = mt.fft(x, 4)
    torch.cuda.synchronize()
    assert X.numel() == 0
    assert plan.status() == (0, -1)


@pytest.mark.parametrize("family,m,elimination", [("dseq", [6, 4], "sparse"), ("dseq", [6, 4], "alg1"),
                                                  ("lat", [6, 4], "sparse"), ("lat", [5, 5], None)])
def test_not_positive_definite_reported(family, m, elimination):
    """A non-finite Lambda is reported through the status word (code -2 and
    a frequency index) by every factorisation, and a valid call clears it."""
    from paper_2603_16014_amd import mtgp as mt
    w = tiny(family, len(m), m, 2, seed=86)
    say("not PD", family, m, elimination)
    ref = oracle_for(w, want_grad=False)
    plan = mt.Plan.from_workload(w, elimination=elimination)
    plan.set_data(torch.from_numpy(ref["y"]).cuda())
    th = dict(w.theta)
    th["eta"] = np.full(w.d, 1e300)
    plan.nll(plan.pack_theta(th))
    torch.cuda.synchronize()
    code, bad = plan.status()
    assert code == -2 and 0 <= bad < w.N
    plan.nll(plan.pack_theta(w.theta))
    torch.cuda.synchronize()
    assert plan.status() == (0, -1)

