"""Pins of the spectral oracle (equal-size MLE loss through per-frequency
blocks) against the dense oracle, which factors the assembled Gram matrix:
both families, every kernel order, the adaptive DSI kernel, fixed and
profiled means.  A dropped transform normalisation, a wrong conjugate in
the off-diagonal lattice blocks, natural instead of radical-inverse order or a
wrong frequency-0 mean shift each breaks one of these cases.  Also the
Walsh routine against the Sylvester Hadamard matrix."""
import numpy as np
import pytest
import scipy.linalg as sla

from _designs import tiny
from oracle import dense, points, spectral

CASES = [
    ("dseq", 1, 5, 2, 2, False, True),
    ("dseq", 3, 5, 3, 1, False, False),
    ("dseq", 2, 6, 2, 3, False, True),
    ("dseq", 2, 5, 2, 4, False, True),
    ("dseq", 3, 5, 2, 2, True, True),
    ("lat", 1, 5, 2, 1, False, True),
    ("lat", 3, 5, 3, 2, False, False),
    ("lat", 2, 6, 2, 3, False, True),
    ("lat", 4, 4, 2, 2, False, True),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-T{c[1]}-m{c[2]}-o{c[4]}{'a' if c[5] else ''}"
                                            f"-{'prof' if c[6] else 'fixed'}" for c in CASES])
def test_spectral_loss_equals_dense(case):
    fam, T, m, d, order, adaptive, profile = case
    w = tiny(fam, T, [m] * T, d, order=order, adaptive=adaptive, seed=5 + T + m,
             profile=profile, rank=min(T, 2))
    X = points.task_points(w)
    y = dense.targets(w, np.random.default_rng(3), X)
    a = dense.nll(w, y, X=X)
    b = spectral.nll_equal(w, y)
    den = abs(a["quad"]) + abs(a["logdet"])
    assert abs(a["L"] - b["L"]) < 1e-12 * den
    assert abs(a["logdet"] - b["logdet"]) < 1e-12 * den
    np.testing.assert_allclose(b["tau_hat"], a["tau_hat"], rtol=1e-11, atol=1e-13)


def test_walsh_is_sylvester_hadamard():
    x = np.random.default_rng(2).normal(size=(3, 64))
    np.testing.assert_allclose(spectral.walsh(x), x @ sla.hadamard(64).T, rtol=0, atol=1e-12)


def test_unequal_sizes_refused():
    w = tiny("dseq", 2, [5, 4], 2, seed=1)
    with pytest.raises(ValueError):
        spectral.nll_equal(w, np.zeros(w.N))


NESTED = [
    # (family, m, d, order, adaptive, profile): descending, ascending and
    # mixed task orders, a one-point task, equal sizes through the same route
    ("dseq", [5, 3, 2], 2, 2, False, True),
    ("dseq", [3, 5, 4], 2, 1, False, False),
    ("dseq", [6, 0], 3, 4, False, True),
    ("dseq", [4, 4, 2, 3], 2, 2, True, True),
    ("lat", [5, 3, 2], 2, 2, False, True),
    ("lat", [4, 6, 6], 2, 3, False, False),
    ("lat", [2, 5, 3], 3, 1, False, True),
    ("lat", [5, 5], 2, 2, False, True),
]


def _nested_id(c):
    return f"{c[0]}-m{'_'.join(map(str, c[1]))}-o{c[3]}{'a' if c[4] else ''}-{'prof' if c[5] else 'fixed'}"


@pytest.mark.parametrize("case", NESTED, ids=[_nested_id(c) for c in NESTED])
def test_nested_spectral_mle_and_gcv_equal_dense(case):
    fam, m, d, order, adaptive, profile = case
    T = len(m)
    w = tiny(fam, T, m, d, order=order, adaptive=adaptive, seed=40 + sum(m), profile=profile,
             rank=min(T, 2))
    X = points.task_points(w)
    y = dense.targets(w, np.random.default_rng(4), X)
    a = dense.nll(w, y, X=X)
    b = spectral.mle(w, y)
    den = abs(a["quad"]) + abs(a["logdet"])
    assert abs(a["L"] - b["L"]) < 1e-11 * den, (a["L"], b["L"])
    assert abs(a["logdet"] - b["logdet"]) < 1e-11 * den
    np.testing.assert_allclose(b["tau_hat"], a["tau_hat"], rtol=1e-10, atol=1e-12)
    g = dense.gcv(w, y, X=X)
    h = spectral.gcv(w, y)
    assert abs(g["L"] - h["L"]) < 1e-10 * g["L"]
    assert abs(g["q"] - h["q"]) < 1e-10 * g["q"] and abs(g["s"] - h["s"]) < 1e-10 * g["s"]
    np.testing.assert_allclose(h["tau_hat"], g["tau_hat"], rtol=1e-9, atol=1e-12)


def test_class_route_equals_per_frequency_route_at_equal_sizes():
    w = tiny("lat", 3, [7, 7, 7], 2, seed=9, rank=2)
    y = np.random.default_rng(5).normal(size=w.N)
    a = spectral.nll_equal(w, y)
    b = spectral.mle(w, y)
    assert abs(a["L"] - b["L"]) < 1e-12 * abs(a["L"])
    np.testing.assert_allclose(b["tau_hat"], a["tau_hat"], rtol=1e-11)


GRAD_CASES = NESTED + [("dseq", [5, 5, 5], 2, 3, True, True), ("lat", [6, 6], 3, 2, False, False)]


@pytest.mark.parametrize("case", GRAD_CASES, ids=[_nested_id(c) for c in GRAD_CASES])
def test_spectral_gradient_equals_dense(case):
    fam, m, d, order, adaptive, profile = case
    T = len(m)
    w = tiny(fam, T, m, d, order=order, adaptive=adaptive, seed=40 + sum(m), profile=profile,
             rank=min(T, 2))
    X = points.task_points(w)
    y = dense.targets(w, np.random.default_rng(4), X)
    ga, _ = dense.grad(w, y, X=X)
    gb, res = spectral.mle_grad(w, y)
    scale = max(np.abs(np.atleast_1d(v)).max() for v in ga.values())
    assert set(ga) == set(gb)
    for k in ga:
        err = np.abs(np.atleast_1d(ga[k]) - np.atleast_1d(gb[k])).max() / scale
        assert err < 1e-10, (k, ga[k], gb[k])
    assert res["L"] == spectral.mle(w, y)["L"]


@pytest.mark.parametrize("case", NESTED, ids=[_nested_id(c) for c in NESTED])
def test_spectral_weights_cubature_and_mean_equal_dense(case):
    import workloads as wl
    fam, m, d, order, adaptive, profile = case
    T = len(m)
    w = wl.with_theta(tiny(fam, T, m, d, order=order, adaptive=adaptive, seed=40 + sum(m),
                           profile=profile, rank=min(T, 2)), tau=np.linspace(-0.3, 0.4, T))
    X = points.task_points(w)
    y = dense.targets(w, np.random.default_rng(4), X)
    res = dense.nll(w, y, X=X)
    sw = spectral.weights(w, y)
    scale = np.abs(res["alpha"]).max()
    assert np.abs(sw["alpha"] - res["alpha"]).max() < 1e-10 * scale
    cd = dense.bayesian_cubature(w, y, X=X, res=res)
    cs = spectral.cubature(w, y)
    np.testing.assert_allclose(cs["mu_hat"], cd["mu_hat"], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(cs["Sigma"], cd["Sigma"], rtol=0, atol=1e-10 * np.abs(cd["Sigma"]).max())
    xs = np.random.default_rng(9).integers(0, 2 ** 32, size=(8, w.d), dtype=np.uint64).astype(np.uint32)
    md = dense.posterior_mean(w, y, xs, X=X, res=res)
    ms = dense.posterior_mean(w, y, xs, X=X, res=dict(alpha=sw["alpha"], tau_hat=sw["tau_hat"]))
    assert np.abs(md - ms).max() < 1e-10 * np.abs(md).max()


@pytest.mark.parametrize("case", GRAD_CASES, ids=[_nested_id(c) for c in GRAD_CASES])
def test_spectral_gcv_gradient_equals_dense(case):
    import workloads as wl
    fam, m, d, order, adaptive, profile = case
    T = len(m)
    w = wl.with_theta(tiny(fam, T, m, d, order=order, adaptive=adaptive, seed=40 + sum(m),
                           profile=profile, rank=min(T, 2)), tau=np.linspace(-0.3, 0.4, T))
    X = points.task_points(w)
    y = dense.targets(w, np.random.default_rng(4), X)
    ga, _ = dense.gcv_grad(w, y, X=X)
    gb, res = spectral.gcv_grad(w, y)
    scale = max(np.abs(np.atleast_1d(v)).max() for v in ga.values())
    assert set(ga) == set(gb)
    for k in ga:
        # GCV weights carry Ktilde^-2: the squared conditioning of the MLE case
        err = np.abs(np.atleast_1d(ga[k]) - np.atleast_1d(gb[k])).max() / scale
        assert err < 1e-9, (k, ga[k], gb[k])
    assert res["L"] == spectral.gcv(w, y)["L"]
