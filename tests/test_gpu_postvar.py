"""Posterior variance at arbitrary inputs (mtgp_predict_var, through the C
ABI) against the dense oracle's posterior covariance diagonal.

Tolerances: the variance is R_tt Q(x,x) minus a quadratic form of the same
size, so its rounding is measured against the prior scale
s = max_t R_tt Q(x, x): FP64 1e-9 of s; mixed (FP32 spectrum storage,
relative rounding 6e-8 of each spectral entry, amplified by the condition
of Lambda in the quadratic form) 1e-4 of s, the mixed-path target for
predictions."""
import numpy as np
import pytest
import torch

import workloads
from oracle import dense
from _designs import tiny
from _gpu_common import oracle_for, say

pytestmark = pytest.mark.gpu

mt = pytest.importorskip("paper_2603_16014_amd.mtgp")


def _ref_var(w, ref, xs):
    X = ref["X"]
    return np.stack([np.diag(dense.posterior_cov(w, xs, xs, t, t, X=X, res=ref["res"]))
                     for t in range(w.T)], axis=1)


def _prior_scale(w, xs):
    R = dense.task_cov(w.theta)
    q0 = np.diag(dense.cross_q(w, w.theta, xs[:1], xs[:1]))[0]
    return float(np.max(np.diag(R)) * q0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("family,T,m,d,adaptive", [("dseq", 3, [7, 7, 7], 3, False),
                                                   ("dseq", 2, [8, 8], 5, True),
                                                   ("lat", 3, [7, 7, 7], 3, False),
                                                   ("dseq", 1, [9], 2, False),
                                                   ("dseq", 3, [8, 6, 4], 3, False),
                                                   ("lat", 3, [8, 6, 5], 2, False),
                                                   ("lat", 4, [6, 6, 4, 4], 2, False)])
def test_predict_var_against_oracle(precision, family, T, m, d, adaptive):
    w = tiny(family, T, m, d, adaptive=adaptive, seed=43)
    say("predict_var", family, T, m, d, adaptive, precision)
    ref = oracle_for(w, want_grad=False)
    xs = workloads.uniform_digits(np.random.default_rng(8), 40, w.d)
    want = _ref_var(w, ref, xs)
    plan = mt.Plan.from_workload(w, precision)
    theta = plan.pack_theta(w.theta)
    plan.set_data(torch.from_numpy(ref["y"]).cuda())
    # batches of 16: two full batches and a ragged one of 8
    got = plan.predict_var(theta, mt.digits_to_device(xs), batch=16).cpu().numpy()
    assert plan.status() == (0, -1)
    s = _prior_scale(w, xs)
    err = np.abs(got - want).max() / s
    say(f"predict_var err {err:.3g} of the prior scale")
    assert err < (1e-9 if precision == "fp64" else 1e-4), err
    # the same points in one batch give the same values
    got1 = plan.predict_var(theta, mt.digits_to_device(xs), batch=64).cpu().numpy()
    np.testing.assert_allclose(got1, got, rtol=0, atol=1e-13 * s)


@pytest.mark.parametrize("family,m", [("dseq", [6, 6]), ("lat", [6, 5])])
def test_predict_var_at_training_points(family, m):
    """At the training points of task t the latent variance lies in
    [0, xi_t] (up to rounding of the prior scale)."""
    w = tiny(family, 2, m, 2, seed=44, xi=1e-4)
    say("predict_var at training points", family, m)
    ref = oracle_for(w, want_grad=False)
    plan = mt.Plan.from_workload(w, "fp64")
    theta = plan.pack_theta(w.theta)
    plan.set_data(torch.from_numpy(ref["y"]).cuda())
    xi = np.asarray(w.theta["xi"])
    for t in range(2):
        xs = ref["X"][t]
        v = plan.predict_var(theta, mt.digits_to_device(xs), batch=32).cpu().numpy()[:, t]
        s = _prior_scale(w, xs)
        assert v.min() > -1e-9 * s and v.max() <= xi[t] + 1e-9 * s, (v.min(), v.max(), xi[t])


def test_predict_var_edges():
    """M = 0 does nothing; Algorithm 1 elimination is refused for nested
    sizes; a batch larger than M is fine."""
    w = tiny("dseq", 2, [6, 5], 2, seed=45)
    say("predict_var edges")
    ref = oracle_for(w, want_grad=False)
    plan = mt.Plan.from_workload(w, "fp64")
    theta = plan.pack_theta(w.theta)
    plan.set_data(torch.from_numpy(ref["y"]).cuda())
    empty = plan.predict_var(theta, torch.zeros((0, w.d), dtype=torch.int32, device="cuda"))
    assert empty.shape == (0, 2)
    xs = workloads.uniform_digits(np.random.default_rng(9), 3, w.d)
    v = plan.predict_var(theta, mt.digits_to_device(xs), batch=100).cpu().numpy()
    np.testing.assert_allclose(v, _ref_var(w, ref, xs), rtol=0, atol=1e-9 * _prior_scale(w, xs))
    a1 = mt.Plan.from_workload(w, "fp64", elimination="alg1")
    a1.set_data(torch.from_numpy(ref["y"]).cuda())
    with pytest.raises(Exception, match="not supported"):
        a1.predict_var(theta, mt.digits_to_device(xs))
