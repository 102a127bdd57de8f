"""The extended-precision C twin against the float64 oracle and itself.

Two independent codings of the same dense definitions (numpy/LAPACK in
float64; plain C loops in long double and in __float128) must agree to the
accuracy the conditioning allows.  At the T=2, d=2, n=2^10 workload the
Gram matrix has condition number about 1e5, so float64 and long double
agree to ~1e-15 relative on L; this makes the long-double result a
reference accurate far below the 1e-10 tolerance used for the GPU FP64 path.
"""
import numpy as np
import pytest

import workloads
from oracle import dense, hp, points as pts
from _designs import tiny


@pytest.mark.parametrize("family,adaptive,profile,m,order", [
    ("dseq", False, True, [5, 5], 2), ("dseq", True, False, [5, 4, 3], 2),
    ("dseq", False, True, [4, 4, 4], 4), ("dseq", False, False, [5, 3], 1),
    ("lat", False, True, [5, 5, 5], 2), ("lat", False, False, [5, 3], 1),
    ("lat", False, True, [4, 2], 3)])
def test_twin_agrees_with_float64(family, adaptive, profile, m, order):
    w = tiny(family, len(m), m, 3, order=order, adaptive=adaptive, seed=12, profile=profile)
    X = pts.task_points(w)
    y = dense.targets(w, np.random.default_rng(5), X)
    Xs = workloads.uniform_digits(np.random.default_rng(6), 17, 3)
    ref = dense.nll(w, y, X=X)
    mu = dense.posterior_mean(w, y, Xs, X=X, res=ref)
    ld = hp.mtgp(w, y, X=X, Xs=Xs)
    qd = hp.mtgp(w, y, X=X, Xs=Xs, kind="quad")
    den = abs(ref["quad"]) + abs(ref["logdet"])
    assert abs(ld["L"] - ref["L"]) < 1e-12 * den
    assert abs(qd["L"] - ld["L"]) < 1e-15 * den
    np.testing.assert_allclose(ld["tau_hat"], ref["tau_hat"], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(ld["mean"], mu, rtol=1e-10, atol=1e-11 * np.abs(mu).max())
    np.testing.assert_allclose(qd["mean"], ld["mean"], rtol=1e-14, atol=1e-15 * np.abs(mu).max())


def test_config1_full_size():
    w = workloads.config1()
    X = pts.task_points(w)
    y = dense.targets(w, np.random.default_rng(w.seed), X)
    ref = dense.nll(w, y, X=X)
    ld = hp.mtgp(w, y, X=X)
    assert abs(ld["L"] - ref["L"]) < 1e-13 * (abs(ref["quad"]) + abs(ref["logdet"]))


@pytest.mark.parametrize("m,order,adaptive,profile", [
    ([5, 5], 2, False, True), ([6, 4, 3], 4, False, True), ([5, 5, 2], 2, True, False),
    ([6, 3, 3, 1], 1, False, True), ([4, 6, 5], 3, False, True)])
def test_spectral_nets_against_dense_twin(m, order, adaptive, profile):
    # the long-double spectral route (Walsh transforms, residue-class blocks)
    # against the long-double dense definitions and the float64 spectral
    # oracle: two codings of the loss in the same extended precision agree
    # to the roundoff that precision leaves at this conditioning
    from oracle import spectral
    w = tiny("dseq", len(m), m, 3, order=order, adaptive=adaptive, seed=41 + sum(m),
             profile=profile)
    X = pts.task_points(w)
    y = dense.targets(w, np.random.default_rng(7), X)
    ld = hp.mtgp(w, y, X=X)
    sp = hp.spectral_nets(w, y)
    f64 = spectral.mle(w, y)
    den = abs(ld["quad"]) + abs(ld["logdet"])
    assert abs(sp["L"] - ld["L"]) < 1e-15 * den, (sp["L"], ld["L"])
    assert abs(sp["quad"] - ld["quad"]) < 1e-15 * den
    np.testing.assert_allclose(sp["tau_hat"], ld["tau_hat"], rtol=1e-14, atol=1e-15)
    assert abs(f64["L"] - sp["L"]) < 1e-12 * den
