"""Pins of the dense oracle (Gram, loss, optimal means, gradient, posterior mean).

* The loss against scipy's multivariate-normal log-density on the same Gram
  matrix (fixed means): L = -2 log p(y) - N log(2 pi).
* The block structure of Theorem "Fast MTGP computations": with V the
  normalised Walsh-Hadamard matrix (DSEQ) or bit-reversal followed by the DFT
  (LAT), V^dagger Ktilde V has tall blocks made of stacked diagonals, with
  Lambda_tt' 1 = sqrt(n_t') V_(m_t)^dagger (Ktilde_tt')_(:,0) and frequency f of
  the larger task coupled to f mod n_t' of the smaller; diagonal blocks'
  eigenvalues are that transform of the first column; Lambda is Hermitian.
* Equal sample sizes: the optimal means are the per-task sample means.
* Central finite differences of L for the gradient, fixed and profiled means.
* Posterior mean interpolates the data as xi -> 0, and with tau = tau_hat the
  Bayesian-cubature identity E alpha = 0 holds (last sentence of the
  multitask Bayesian cubature theorem).
"""
import math

import numpy as np
import pytest

import workloads
import scipy.linalg as sla
import scipy.stats

from oracle import dense, points as pts
from _designs import tiny


def _bitrev(j, m):
    return int(format(j, f"0{m}b")[::-1], 2) if m > 0 else 0


def _vdag(family, m):
    n = 1 << m
    if family == "dseq":
        return sla.hadamard(n).astype(np.float64) / math.sqrt(n)
    P = np.zeros((n, n))
    for j in range(n):
        P[j, _bitrev(j, m)] = 1.0
    F = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
    return F @ P / math.sqrt(n)


@pytest.mark.parametrize("family", ["dseq", "lat"])
@pytest.mark.parametrize("m", [[3, 3, 3], [3, 2, 1], [4, 4, 2]])
def test_block_structure(family, m):
    w = tiny(family, len(m), m, 2, seed=7)
    X = pts.task_points(w)
    K = dense.gram(w, X=X)
    n = [1 << v for v in m]
    off = np.concatenate([[0], np.cumsum(n)])
    Vd = [_vdag(family, v) for v in m]
    for t in range(len(m)):
        for s in range(len(m)):
            Kb = K[off[t]:off[t + 1], off[s]:off[s + 1]]
            Lam = Vd[t] @ Kb @ Vd[s].conj().T
            scale = np.abs(Kb).max()
            if n[t] >= n[s]:
                lam = math.sqrt(n[s]) * (Vd[t] @ Kb[:, 0])
                expect = np.zeros_like(Lam)
                for f in range(n[t]):
                    expect[f, f % n[s]] = lam[f]
            else:
                lam = math.sqrt(n[t]) * (Vd[s] @ Kb[0, :])
                expect = np.zeros_like(Lam)
                for g in range(n[s]):
                    expect[g % n[t], g] = np.conj(lam[g])
            np.testing.assert_allclose(Lam, expect, rtol=0, atol=1e-12 * scale * n[t])
            if t == s:
                ev = np.sort(np.linalg.eigvalsh(Kb))
                np.testing.assert_allclose(np.sort(lam.real), ev, rtol=0, atol=1e-12 * scale * n[t])
                assert np.abs(lam.imag).max() < 1e-12 * scale * n[t]


@pytest.mark.parametrize("family", ["dseq", "lat"])
def test_gram_symmetric_pd(family):
    w = tiny(family, 3, [5, 4, 4], 3, seed=2)
    K = dense.gram(w)
    assert np.array_equal(K, K.T)
    assert np.linalg.eigvalsh(K).min() > 0


@pytest.mark.parametrize("family", ["dseq", "lat"])
def test_loss_matches_mvn_logpdf(family):
    w = tiny(family, 2, [5, 4], 2, seed=3, profile=False)
    X = pts.task_points(w)
    y = dense.targets(w, np.random.default_rng(0), X)
    r = dense.nll(w, y, X=X)
    K = dense.gram(w, X=X)
    mean = dense.summing_matrix([32, 16]).T @ w.theta["tau"]
    lp = scipy.stats.multivariate_normal(mean=mean, cov=K).logpdf(y)
    N = K.shape[0]
    assert abs(r["L"] - (-2 * lp - N * math.log(2 * math.pi))) < 1e-9 * (abs(r["quad"]) + abs(r["logdet"]))
    assert abs(r["nll"] + lp) < 1e-9 * abs(lp)


@pytest.mark.parametrize("family", ["dseq", "lat"])
def test_equal_sizes_tau_hat_is_sample_mean(family):
    w = tiny(family, 3, [6, 6, 6], 2, seed=4)
    X = pts.task_points(w)
    y = dense.targets(w, np.random.default_rng(1), X)
    r = dense.nll(w, y, X=X)
    np.testing.assert_allclose(r["tau_hat"], y.reshape(3, -1).mean(axis=1), rtol=1e-10, atol=1e-12)


def _pack(theta, keys):
    return np.concatenate([np.atleast_1d(np.asarray(theta[k], dtype=np.float64)).ravel() for k in keys])


LOG_KEYS = {"gamma", "eta", "b", "xi", "zeta"}


def _unpack(vec, theta, keys):
    out = dict(theta)
    i = 0
    for k in keys:
        shape = np.shape(theta[k])
        size = int(np.prod(shape)) if shape else 1
        v = vec[i:i + size]
        out[k] = float(v[0]) if not shape else v.reshape(shape)
        i += size
    return out


@pytest.mark.parametrize("family,adaptive,profile,m", [
    ("dseq", False, True, [4, 4]), ("dseq", True, False, [4, 3, 2]),
    ("lat", False, False, [4, 4, 4]), ("lat", False, True, [4, 2])])
def test_gradient_central_differences(family, adaptive, profile, m):
    w = tiny(family, len(m), m, 2, adaptive=adaptive, seed=9, profile=profile, xi=1e-2)
    X = pts.task_points(w)
    y = dense.targets(w, np.random.default_rng(2), X)
    g, _ = dense.grad(w, y, X=X)
    keys = ["tau", "gamma", "eta"] + (["b"] if adaptive else []) + ["xi", "B", "zeta"]
    # FD in the parameterisation of the gradient: log for positive parameters
    base = {k: (np.log(w.theta[k]) if k in LOG_KEYS else np.asarray(w.theta[k], dtype=np.float64))
            for k in keys}
    vec = _pack(base, keys)
    gvec = _pack(g, keys)
    h = 1e-5

    def L_of(v):
        th = _unpack(v, base, keys)
        th = {k: (np.exp(th[k]) if k in LOG_KEYS else th[k]) for k in keys}
        return dense.nll(w, y, theta=th, X=X)["L"]

    for i in range(len(vec)):
        e = np.zeros_like(vec)
        e[i] = h
        fd = (L_of(vec + e) - L_of(vec - e)) / (2 * h)
        assert abs(fd - gvec[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gvec[i])


@pytest.mark.parametrize("family", ["dseq", "lat"])
def test_posterior_mean_interpolates(family):
    w = tiny(family, 2, [5, 4], 2, seed=5, xi=1e-10)
    X = pts.task_points(w)
    y = dense.targets(w, np.random.default_rng(3), X)
    for t in range(2):
        mu = dense.posterior_mean(w, y, X[t], X=X)[:, t]
        yt = y[:32] if t == 0 else y[32:]
        np.testing.assert_allclose(mu, yt, rtol=0, atol=1e-6 * np.abs(y).max())


@pytest.mark.parametrize("family", ["dseq", "lat"])
def test_bayesian_cubature_identity(family):
    w = tiny(family, 3, [5, 4, 3], 2, seed=6)
    X = pts.task_points(w)
    y = dense.targets(w, np.random.default_rng(4), X)
    r = dense.nll(w, y, X=X)
    Ea = dense.summing_matrix([32, 16, 8]) @ r["alpha"]
    assert np.abs(Ea).max() < 1e-8 * np.abs(r["alpha"]).sum()


def _fine_set(family, d, m, seed):
    """An independent good point set of 2^m points for quadrature.  Nets:
    the digitally shifted 2-D Hammersley net (generating matrices identity
    and reversed identity, a (0, m, 2)-net); random unit lower-triangular
    matrices share the leading digit in every coordinate and integrate the
    product kernel badly.  Lattices: a random rank-1 lattice."""
    rng = np.random.default_rng(seed)
    if family == "dseq":
        assert d == 2
        i = np.arange(1 << m, dtype=np.uint64)
        x1 = pts.van_der_corput_digits(1 << m)
        x2 = (i << np.uint64(32 - m)).astype(np.uint32)
        sh = workloads.random_shifts(rng, 1, d)[0]
        return np.stack([x1 ^ sh[0], x2 ^ sh[1]], axis=1).astype(np.uint32)
    gen = workloads.random_lattice_gen(rng, d)
    return pts.lattice_points(gen, 1 << m, workloads.random_shifts(rng, 1, d)[0])


@pytest.mark.parametrize("family", ["dseq", "lat"])
def test_cubature_covariance_is_double_integral_of_posterior_cov(family):
    """Sigma_tu = int int Cov[f(t,x), f(u,x') | data] dx dx', here by the
    average over a fine independent point set (quadrature, not the formula)."""
    w = tiny(family, 2, [5, 4], 2, seed=8)
    X = pts.task_points(w)
    y = dense.targets(w, np.random.default_rng(5), X)
    res = dense.nll(w, y, X=X)
    bc = dense.bayesian_cubature(w, y, X=X, res=res)
    Z = _fine_set(family, w.d, 12, 77)
    quad = np.zeros((2, 2))
    for a in range(2):
        for b in range(2):
            quad[a, b] = dense.posterior_cov(w, Z, Z, a, b, X=X, res=res).mean()
    scale = np.abs(bc["Sigma"]).max()
    # the net quadrature of these kernels converges like 2^-m (measured: the
    # kernel mean itself is off by 6e-3 at m = 12), the lattice one faster
    tol = 2e-2 if family == "dseq" else 2e-4
    assert np.abs(quad - bc["Sigma"]).max() < tol * scale, (quad, bc["Sigma"])
    assert np.allclose(bc["Sigma"], bc["Sigma"].T, rtol=0, atol=1e-14 * scale)
    assert np.linalg.eigvalsh(bc["Sigma"]).min() > -1e-12 * scale


@pytest.mark.parametrize("family", ["dseq", "lat"])
def test_cubature_mean_is_integral_of_posterior_mean(family):
    """With fixed means, mu_hat_t = int mu(t, x) dx (quadrature again); with
    profiled means, mu_hat = tau_hat (the theorem's last statement)."""
    w = workloads.with_theta(tiny(family, 3, [5, 5, 4], 2, seed=9), tau=np.array([0.3, -0.2, 0.1]))
    X = pts.task_points(w)
    y = dense.targets(w, np.random.default_rng(6), X)
    res = dense.nll(w, y, X=X, profile=False)
    bc = dense.bayesian_cubature(w, y, X=X, profile=False, res=res)
    Z = _fine_set(family, w.d, 12, 78)
    avg = dense.posterior_mean(w, y, Z, X=X, profile=False, res=res).mean(axis=0)
    tol = 2e-2 if family == "dseq" else 1e-4
    assert np.abs(avg - bc["mu_hat"]).max() < tol * np.abs(avg).max(), (avg, bc["mu_hat"])
    resp = dense.nll(w, y, X=X, profile=True)
    bcp = dense.bayesian_cubature(w, y, X=X, profile=True, res=resp)
    np.testing.assert_allclose(bcp["mu_hat"], resp["tau_hat"], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("family,profile", [("dseq", False), ("lat", False), ("dseq", True)])
def test_cubature_is_gaussian_conditioning_of_the_joint(family, profile):
    """The integrals and the data are jointly Gaussian with
    Cov(mu, mu) = gamma R, Cov(mu, y) = gamma R E, Cov(y, y) = Ktilde (the
    kernel means integrate to gamma).  Conditioning through the inverse of
    the full joint matrix (a different route from the Schur complement the
    oracle uses) gives the same mean and covariance."""
    w = workloads.with_theta(tiny(family, 3, [4, 4, 3], 2, seed=10), tau=np.array([0.2, 0.1, -0.3]))
    X = pts.task_points(w)
    y = dense.targets(w, np.random.default_rng(7), X)
    res = dense.nll(w, y, X=X, profile=profile)
    bc = dense.bayesian_cubature(w, y, X=X, profile=profile, res=res)
    n = [x.shape[0] for x in X]
    E = dense.summing_matrix(n)
    R = dense.task_cov(w.theta)
    g = w.theta["gamma"]
    K = dense.gram(w, w.theta, X)
    T = w.T
    J = np.block([[g * R, g * R @ E], [(g * R @ E).T, K]])
    Ji = np.linalg.inv(J)
    Sigma = np.linalg.inv(Ji[:T, :T])
    r = y - E.T @ res["tau_hat"]
    mu = res["tau_hat"] - Sigma @ Ji[:T, T:] @ r
    np.testing.assert_allclose(bc["Sigma"], Sigma, rtol=1e-8, atol=1e-10 * np.abs(Sigma).max())
    np.testing.assert_allclose(bc["mu_hat"], mu, rtol=1e-8, atol=1e-10 * np.abs(mu).max())


# ----------------------------------------------------------------- GCV
@pytest.mark.parametrize("family,m,profile", [("dseq", [5, 5], True), ("lat", [5, 4, 3], False),
                                              ("dseq", [5, 4, 3], True)])
def test_gcv_loss_by_eigendecomposition(family, m, profile):
    """q = sum_i (u_i^T r)^2 / lambda_i^2 and s = sum_i 1 / lambda_i from the
    eigenpairs of Ktilde (a different route from the Cholesky solves)."""
    w = tiny(family, len(m), m, 2, seed=12, profile=profile)
    X = pts.task_points(w)
    y = dense.targets(w, np.random.default_rng(8), X)
    res = dense.gcv(w, y, X=X)
    lam, U = np.linalg.eigh(res["K"])
    n = [x.shape[0] for x in X]
    r = y - dense.summing_matrix(n).T @ res["tau_hat"]
    c = U.T @ r
    q = float(np.sum(c * c / lam ** 2))
    s = float(np.sum(1.0 / lam))
    assert abs(q - res["q"]) < 1e-9 * q and abs(s - res["s"]) < 1e-11 * s
    assert abs(q / s ** 2 - res["L"]) < 1e-9 * res["L"]


@pytest.mark.parametrize("family", ["dseq", "lat"])
def test_gcv_tau_hat(family):
    """Equal sizes: tau_hat_GCV is the per-task sample mean (closed form, the
    constant vector is an eigenvector of every equal-size block structure
    here); nested sizes: it is a stationary point (fixed-tau gradient 0)."""
    w = tiny(family, 3, [5, 5, 5], 2, seed=13)
    X = pts.task_points(w)
    y = dense.targets(w, np.random.default_rng(9), X)
    res = dense.gcv(w, y, X=X, profile=True)
    np.testing.assert_allclose(res["tau_hat"], y.reshape(3, -1).mean(axis=1), rtol=1e-9,
                               atol=1e-9 * np.abs(y).max())
    w2 = tiny(family, 3, [5, 4, 3], 2, seed=14)
    X2 = pts.task_points(w2)
    y2 = dense.targets(w2, np.random.default_rng(10), X2)
    r2 = dense.gcv(w2, y2, X=X2, profile=True)
    wf = workloads.with_theta(w2, tau=r2["tau_hat"])
    g, _ = dense.gcv_grad(wf, y2, X=X2, profile=False)
    assert np.abs(g["tau"]).max() < 1e-8 * np.abs(g["eta"]).max()


@pytest.mark.parametrize("family,profile,adaptive", [("dseq", True, False), ("lat", False, False),
                                                     ("dseq", False, True)])
def test_gcv_gradient_central_differences(family, profile, adaptive):
    w = tiny(family, 2, [4, 3], 2, seed=15, profile=profile, adaptive=adaptive)
    X = pts.task_points(w)
    y = dense.targets(w, np.random.default_rng(11), X)
    g, res = dense.gcv_grad(w, y, X=X)
    keys = ["tau", "gamma", "eta"] + (["b"] if adaptive else []) + ["xi", "B", "zeta"]
    logk = {"gamma", "eta", "b", "xi", "zeta"}
    h = 1e-5
    for k in keys:
        base = np.atleast_1d(np.asarray(w.theta[k], dtype=np.float64)).astype(float)
        flat = base.ravel()
        gk = np.atleast_1d(np.asarray(g[k], dtype=np.float64)).ravel()
        for i in range(flat.size):
            vals = []
            for sgn in (1, -1):
                f2 = flat.copy()
                f2[i] = f2[i] * np.exp(sgn * h) if k in logk else f2[i] + sgn * h
                v = f2.reshape(base.shape)
                th = dict(w.theta)
                th[k] = float(v[0]) if k == "gamma" else v
                vals.append(dense.gcv(w, y, theta=th, X=X)["L"])
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - gk[i]) < 1e-5 * max(1.0, abs(gk[i])) + 1e-6 * res["L"], (k, i, fd, gk[i])


# ---------------------------------------------------- posterior covariance
def _joint_posterior_cov(w, X, Xs, t):
    """Cov[f(t, x*) | y] through the inverse of the full joint covariance of
    (f(t, x*), y): the noise-free Gram of a design whose task t also holds
    the test points, with the noise added on the training rows only."""
    Xa = [np.concatenate([X[u], Xs]) if u == t else X[u] for u in range(w.T)]
    Ka = dense.gram(w, w.theta, Xa, noise=False)
    n = [x.shape[0] for x in X]
    off = np.concatenate([[0], np.cumsum([x.shape[0] for x in Xa])])
    test = np.arange(off[t] + n[t], off[t + 1])
    train = np.setdiff1d(np.arange(off[-1]), test)
    xi = np.asarray(w.theta["xi"], dtype=np.float64)
    for u in range(w.T):
        idx = np.arange(off[u], off[u] + n[u])
        Ka[idx, idx] += xi[u]
    order = np.concatenate([test, train])
    J = Ka[np.ix_(order, order)]
    Ji = np.linalg.inv(J)
    M = test.size
    return np.linalg.inv(Ji[:M, :M])


@pytest.mark.parametrize("family,m", [("dseq", [4, 4, 3]), ("lat", [4, 3, 3])])
def test_posterior_cov_is_gaussian_conditioning_of_the_joint(family, m):
    """Cov[f(t,x), f(t,x') | y] equals the conditioning of the joint
    Gaussian of the latent values and the data, taken through the inverse of
    the full joint matrix (not the formula the oracle uses)."""
    w = tiny(family, 3, m, 2, seed=12)
    X = pts.task_points(w)
    Xs = workloads.uniform_digits(np.random.default_rng(3), 6, w.d)
    for t in range(w.T):
        ref = _joint_posterior_cov(w, X, Xs, t)
        got = dense.posterior_cov(w, Xs, Xs, t, t, X=X)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-9 * np.abs(ref).max())


@pytest.mark.parametrize("family", ["dseq", "lat"])
def test_posterior_variance_bounds(family):
    """At a training point of task t the latent variance lies in [0, xi_t]
    (one noisy observation alone already brings it below xi_t); anywhere it
    lies in [0, R_tt Q(x, x)]; with the noise taken to 1e8 times the prior
    scale the data carry no information and it returns to R_tt Q(x, x)."""
    w = tiny(family, 2, [4, 3], 2, seed=13, xi=1e-4)
    X = pts.task_points(w)
    R = dense.task_cov(w.theta)
    xi = np.asarray(w.theta["xi"])
    for t in range(2):
        v = np.diag(dense.posterior_cov(w, X[t], X[t], t, t, X=X))
        assert v.min() > -1e-12 and v.max() <= xi[t] * (1 + 1e-9), (v.min(), v.max(), xi[t])
    Xs = workloads.uniform_digits(np.random.default_rng(4), 20, w.d)
    q0 = np.diag(dense.cross_q(w, w.theta, Xs, Xs))
    for t in range(2):
        v = np.diag(dense.posterior_cov(w, Xs, Xs, t, t, X=X))
        assert v.min() > -1e-12 and (v <= R[t, t] * q0 * (1 + 1e-12)).all()
    loud = workloads.with_theta(w, xi=np.full(2, 1e8 * R.max() * q0.max()))
    for t in range(2):
        v = np.diag(dense.posterior_cov(loud, Xs, Xs, t, t, X=X))
        np.testing.assert_allclose(v, R[t, t] * q0, rtol=1e-6)
