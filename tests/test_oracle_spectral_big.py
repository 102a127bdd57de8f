"""Pins of the C spectral oracle (oracle/spectral_big.c) against the dense
oracle and the point / target definitions, on designs small enough for a
dense Cholesky factorisation.  Each check below fails for a plausible
mistake in the C code:

* points: a wrong generating-column index or bit order;
* loss: a wrong DSI order formula, beta off by one, a wrong pair shift or
  pair-to-column map (T >= 3 with distinct shifts), a missing xi, the mean
  shift at a frequency other than 0 or without its sqrt(n), a wrong log-det
  factor (all against the dense Gram matrix);
* profiled means against the dense GLS means, fixed means passed through;
* alpha and the posterior mean against oracle.dense.posterior_mean;
* targets against workloads.target_values at the same points and noise.
"""
import numpy as np
import pytest

import workloads
from _designs import tiny
from oracle import dense, kernels as kn, points, spectral_big as sb


def test_points_against_definition():
    w = tiny("dseq", 2, [9, 9], 5, seed=301)
    np.testing.assert_array_equal(sb.points(w, 1 << 9), points.dseq_unshifted(w.gen, 1 << 9))


@pytest.mark.parametrize("order", [1, 2, 3, 4])
@pytest.mark.parametrize("T,m,profile", [(1, 6, True), (2, 6, True), (3, 5, False), (5, 4, True)])
def test_loss_against_dense(order, T, m, profile):
    w = tiny("dseq", T, [m] * T, 3, order=order, seed=310 + 7 * T + order, profile=profile)
    X = points.task_points(w)
    y = dense.targets(w, np.random.default_rng(5), X)
    ref = dense.nll(w, y, X=X)
    got = sb.mle(w, y)
    den = abs(ref["quad"]) + abs(ref["logdet"])
    for k in ("quad", "logdet", "L"):
        assert abs(got[k] - ref[k]) < 1e-11 * den, (k, got[k], ref[k])
    np.testing.assert_allclose(got["tau_hat"], ref["tau_hat"], rtol=1e-10, atol=1e-12)


def test_fixed_means_with_offset():
    """Fixed tau far from the data means: the shift enters only through
    frequency 0 with its sqrt(n), which the quadratic form then shows."""
    w = tiny("dseq", 3, [5, 5, 5], 2, seed=331, profile=False)
    w.theta["tau"] = np.array([3.0, -2.0, 0.5])
    X = points.task_points(w)
    y = dense.targets(w, np.random.default_rng(6), X)
    ref = dense.nll(w, y, X=X)
    got = sb.mle(w, y)
    den = abs(ref["quad"]) + abs(ref["logdet"])
    assert abs(got["L"] - ref["L"]) < 1e-11 * den
    np.testing.assert_array_equal(got["tau_hat"], w.theta["tau"])


@pytest.mark.parametrize("order", [2, 4])
def test_alpha_and_mean_against_dense(order):
    w = tiny("dseq", 3, [6, 6, 6], 4, order=order, seed=340 + order)
    X = points.task_points(w)
    y = dense.targets(w, np.random.default_rng(7), X)
    ref = dense.nll(w, y, X=X)
    got = sb.mle(w, y, want_alpha=True)
    a_ref = ref["alpha"].reshape(w.T, -1)
    assert np.abs(got["alpha"] - a_ref).max() < 1e-9 * np.abs(a_ref).max()
    xs = workloads.uniform_digits(np.random.default_rng(8), 17, w.d)
    mu_ref = dense.posterior_mean(w, y, xs, X=X, res=ref)
    mu = sb.posterior_mean(w, got, xs)
    assert np.abs(mu - mu_ref).max() < 1e-9 * np.abs(mu_ref).max()


def test_targets_against_workloads():
    w = tiny("dseq", 3, [7, 7, 7], 4, seed=350)
    X = points.task_points(w)
    ref = np.concatenate(workloads.target_values(w, [kn.to_unit(x) for x in X],
                                                 np.random.default_rng(9)))
    got = sb.targets(w, np.random.default_rng(9))
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


def test_rejects_other_designs():
    with pytest.raises(ValueError):
        sb.mle(tiny("lat", 2, [4, 4], 2, seed=360), np.zeros(32))
    with pytest.raises(ValueError):
        sb.mle(tiny("dseq", 2, [4, 3], 2, seed=361), np.zeros(24))
