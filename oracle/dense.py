"""Dense float64 multitask GP: Gram, MLE loss, optimal means, gradient, posterior mean.

Test infrastructure only.  Everything is the textbook dense computation with
the same kernel on the same points; it is exact up to rounding because the
fast method is exact (Theorem "Fast MTGP computations").

* Gram (Section "Multitask Setting"): blocks
  Ktilde_tt'[i, k] = R_tt' Q(x_ti, x_t'k) + delta_tt' delta_ik xi_t,
  R = B B^T + diag(zeta) (Eq. mtprod and the task-kernel parameterisation).
* MLE loss (Eq. MTGP_MLE_GCV_loss): L = r^T Ktilde^-1 r + log det Ktilde with
  r = y - E^T tau; E is the task-summing matrix.
* Optimal means (Eq. MTGP_optimal_tau): (E K^-1 E^T) tau_hat = E K^-1 y.
* Posterior mean (Eq. MTGP_post_mean_cov): tau_t + K(t, x)^T Ktilde^-1 (y - E^T tau).
* GCV loss (Eq. MTGP_MLE_GCV_loss) and its optimal means (Eq. MTGP_optimal_tau),
  with the exact gradient; Bayesian cubature of the task integrals.
* Gradient (the paper gives none; it is the exact derivative of L):
  dL/dtheta_k = -alpha^T (dK/dtheta_k) alpha + tr(K^-1 dK/dtheta_k) with
  alpha = K^-1 r, in the log-parameterisation of gamma, eta, b, xi, zeta and
  the plain parameterisation of tau and B.  With profiled means the tau
  components are zero (tau_hat is a stationary point of L in tau) and the
  rest is unchanged.

Pinned by: the multivariate-normal log-density (scipy), the eigenstructure of
Theorem "Fast MTGP computations" on tiny designs, central finite differences
of L, interpolation of the posterior mean as xi -> 0, the Bayesian-cubature
identity E alpha = 0 at tau_hat, the extended-precision twin; the cubature
mean and covariance by quadrature of the posterior mean and covariance over
fine independent point sets.
"""
import math

import numpy as np
import scipy.linalg as sla

from . import kernels as kn
from . import points as pts


def task_cov(theta):
    B = np.asarray(theta["B"], dtype=np.float64)
    return B @ B.T + np.diag(np.asarray(theta["zeta"], dtype=np.float64))


def _kernel_args(w):
    return (w.family, w.kernel_order, w.adaptive,
            None if w.theta.get("b") is None else np.asarray(w.theta["b"], dtype=np.float64))


def cross_q(w, theta, Xa, Xb):
    """Q(x_a, x_b) for all pairs: [len(Xa)][len(Xb)], dimension by dimension."""
    fam, order, adaptive, _ = _kernel_args(w)
    b = None if theta.get("b") is None else np.asarray(theta["b"], dtype=np.float64)
    eta = np.asarray(theta["eta"], dtype=np.float64)
    q = np.full((Xa.shape[0], Xb.shape[0]), float(theta["gamma"]))
    for j in range(w.d):
        u = kn.pair_arg(fam, Xa[:, j][:, None], Xb[:, j][None, :])
        q *= 1.0 + eta[j] * kn.univariate(fam, order, adaptive, b, u)
    return q


def gram(w, theta=None, X=None, noise=True):
    """Dense Ktilde (task-major blocks, radical-inverse order within a task)."""
    theta = w.theta if theta is None else theta
    X = pts.task_points(w) if X is None else X
    R = task_cov(theta)
    n = [x.shape[0] for x in X]
    off = np.concatenate([[0], np.cumsum(n)])
    K = np.empty((off[-1], off[-1]))
    for t in range(w.T):
        for s in range(t, w.T):
            blk = R[t, s] * cross_q(w, theta, X[t], X[s])
            K[off[t]:off[t + 1], off[s]:off[s + 1]] = blk
            K[off[s]:off[s + 1], off[t]:off[t + 1]] = blk.T
    if noise:
        xi = np.asarray(theta["xi"], dtype=np.float64)
        for t in range(w.T):
            idx = np.arange(off[t], off[t + 1])
            K[idx, idx] += xi[t]
    return K


def summing_matrix(n):
    E = np.zeros((len(n), int(sum(n))))
    off = 0
    for t, nt in enumerate(n):
        E[t, off:off + nt] = 1.0
        off += nt
    return E


def nll(w, y, theta=None, X=None, profile=None, K=None):
    """MLE loss pieces: quad, logdet, L = quad + logdet, NLL, tau_hat, alpha."""
    theta = w.theta if theta is None else theta
    profile = w.profile_tau if profile is None else profile
    X = pts.task_points(w) if X is None else X
    y = np.asarray(y, dtype=np.float64)
    n = [x.shape[0] for x in X]
    K = gram(w, theta, X) if K is None else K
    cf = sla.cho_factor(K, lower=True)
    logdet = 2.0 * float(np.sum(np.log(np.diag(cf[0]))))
    E = summing_matrix(n)
    if profile:
        Kinv_y = sla.cho_solve(cf, y)
        Kinv_Et = sla.cho_solve(cf, E.T)
        Pi = E @ Kinv_Et
        tau = np.linalg.solve(Pi, E @ Kinv_y)
    else:
        tau = np.asarray(theta["tau"], dtype=np.float64)
    r = y - E.T @ tau
    alpha = sla.cho_solve(cf, r)
    quad = float(r @ alpha)
    L = quad + logdet
    N = int(sum(n))
    return dict(quad=quad, logdet=logdet, L=L, nll=0.5 * L + 0.5 * N * math.log(2 * math.pi),
                tau_hat=tau, alpha=alpha, cf=cf, K=K)


def _param_grads(w, theta, X, Wd):
    """sum_ij Wd_ij dKtilde_ij / dtheta for every non-mean parameter, by
    assembling dKtilde densely from the analytic kernel derivatives."""
    fam, order, adaptive, _ = _kernel_args(w)
    b = None if theta.get("b") is None else np.asarray(theta["b"], dtype=np.float64)
    eta = np.asarray(theta["eta"], dtype=np.float64)
    R = task_cov(theta)
    n = [x.shape[0] for x in X]
    off = np.concatenate([[0], np.cumsum(n)])
    T, d = w.T, w.d
    g_eta = np.zeros(d)
    g_b = np.zeros(4) if adaptive else None
    G = np.zeros((T, T))                     # dL/dR_tt' (entries independent)
    for t in range(T):
        for s in range(T):
            Wb = Wd[off[t]:off[t + 1], off[s]:off[s + 1]]
            Xa, Xb = X[t], X[s]
            u = np.stack([kn.pair_arg(fam, Xa[:, j][:, None], Xb[:, j][None, :])
                          for j in range(d)], axis=-1)
            Q, dq_eta, dq_b = kn.product_kernel_grads(fam, order, adaptive, b,
                                                      theta["gamma"], eta, u)
            G[t, s] = float(np.sum(Wb * Q))
            for j in range(d):
                g_eta[j] += R[t, s] * float(np.sum(Wb * dq_eta[j]))
            if adaptive:
                for a in range(4):
                    g_b[a] += R[t, s] * float(np.sum(Wb * dq_b[a]))
    g_gamma = float(np.sum(R * G))           # Q is proportional to gamma
    xi = np.asarray(theta["xi"], dtype=np.float64)
    g_xi = np.array([xi[t] * float(np.trace(Wd[off[t]:off[t + 1], off[t]:off[t + 1]]))
                     for t in range(T)])
    B = np.asarray(theta["B"], dtype=np.float64)
    g_B = (G + G.T) @ B                      # R = B B^T + diag(zeta)
    zeta = np.asarray(theta["zeta"], dtype=np.float64)
    g_zeta = zeta * np.diag(G)
    out = dict(gamma=g_gamma, eta=g_eta, xi=g_xi, B=g_B, zeta=g_zeta)
    if adaptive:
        out["b"] = g_b
    return out


def grad(w, y, theta=None, X=None, profile=None):
    """Exact gradient of L in the packed parameterisation (dict keyed like theta)."""
    theta = w.theta if theta is None else theta
    profile = w.profile_tau if profile is None else profile
    X = pts.task_points(w) if X is None else X
    res = nll(w, y, theta, X, profile)
    alpha = res["alpha"]
    Kinv = sla.cho_solve(res["cf"], np.eye(res["K"].shape[0]))
    Wd = Kinv - np.outer(alpha, alpha)       # dL/dK_ij summed against dK_ij
    out = _param_grads(w, theta, X, Wd)
    n = [x.shape[0] for x in X]
    out["tau"] = np.zeros(w.T) if profile else -2.0 * (summing_matrix(n) @ alpha)
    return out, res


def gcv(w, y, theta=None, X=None, profile=None, K=None):
    """GCV loss (Eq. MTGP_MLE_GCV_loss) L_GCV = r^T Ktilde^-2 r / tr^2(Ktilde^-1),
    r = y - E^T tau, with tau = tau_hat_GCV solving
    (E Ktilde^-2 E^T) tau = E Ktilde^-2 y (Eq. MTGP_optimal_tau) when profiled.
    Returns dict(q = r^T Ktilde^-2 r, s = tr Ktilde^-1, L, tau_hat, a = Ktilde^-1 r,
    bvec = Ktilde^-2 r, cf, K)."""
    theta = w.theta if theta is None else theta
    profile = w.profile_tau if profile is None else profile
    X = pts.task_points(w) if X is None else X
    y = np.asarray(y, dtype=np.float64)
    n = [x.shape[0] for x in X]
    K = gram(w, theta, X) if K is None else K
    cf = sla.cho_factor(K, lower=True)
    Kinv = sla.cho_solve(cf, np.eye(K.shape[0]))
    E = summing_matrix(n)
    if profile:
        K2Et = Kinv @ (Kinv @ E.T)
        tau = np.linalg.solve(E @ K2Et, K2Et.T @ y)
    else:
        tau = np.asarray(theta["tau"], dtype=np.float64)
    r = y - E.T @ tau
    a = Kinv @ r
    bvec = Kinv @ a
    q = float(a @ a)
    s = float(np.trace(Kinv))
    return dict(q=q, s=s, L=q / (s * s), tau_hat=tau, a=a, bvec=bvec, cf=cf, K=K, Kinv=Kinv)


def gcv_grad(w, y, theta=None, X=None, profile=None):
    """Exact gradient of L_GCV: with a = Ktilde^-1 r, b = Ktilde^-2 r,
    q = a^T a, s = tr Ktilde^-1,
      dL = sum_ij W_ij dKtilde_ij,  W = -(a b^T + b a^T) / s^2 + (2 q / s^3) Ktilde^-2,
    profiled tau: dL/dtau = 0 (tau_hat_GCV is stationary); fixed tau:
    dL/dtau = -2 E b / s^2."""
    theta = w.theta if theta is None else theta
    profile = w.profile_tau if profile is None else profile
    X = pts.task_points(w) if X is None else X
    res = gcv(w, y, theta, X, profile)
    a, bv, q, s, Kinv = res["a"], res["bvec"], res["q"], res["s"], res["Kinv"]
    Wd = -(np.outer(a, bv) + np.outer(bv, a)) / s ** 2 + (2.0 * q / s ** 3) * (Kinv @ Kinv)
    out = _param_grads(w, theta, X, Wd)
    n = [x.shape[0] for x in X]
    out["tau"] = np.zeros(w.T) if profile else -2.0 * (summing_matrix(n) @ bv) / s ** 2
    return out, res


def posterior_mean(w, y, Xs, theta=None, X=None, profile=None, res=None):
    """mu[m, t] = tau_t + sum_t' R_tt' sum_k Q(x*_m, x_t'k) alpha_t'k."""
    theta = w.theta if theta is None else theta
    X = pts.task_points(w) if X is None else X
    res = nll(w, y, theta, X, profile) if res is None else res
    R = task_cov(theta)
    n = [x.shape[0] for x in X]
    off = np.concatenate([[0], np.cumsum(n)])
    alpha = res["alpha"]
    Xs = np.asarray(Xs, dtype=np.uint32)
    kv = np.zeros((Xs.shape[0], w.T))        # kv[:, t'] = sum_k Q(x*, x_t'k) alpha_t'k
    for s in range(w.T):
        kv[:, s] = cross_q(w, theta, Xs, X[s]) @ alpha[off[s]:off[s + 1]]
    return res["tau_hat"][None, :] + kv @ R.T


def posterior_cov(w, Xa, Xb, ta, tb, theta=None, X=None, res=None):
    """Cov[f(ta, x_a), f(tb, x_b) | data] for all pairs of the two point sets:
    R_{ta,tb} Q(x_a, x_b) - k_ta(x_a)^T Ktilde^-1 k_tb(x_b) with
    k_t(x)[(u, k)] = R_tu Q(x, x_uk) (the noise-free latent function)."""
    theta = w.theta if theta is None else theta
    X = pts.task_points(w) if X is None else X
    cf = sla.cho_factor(gram(w, theta, X), lower=True) if res is None else res["cf"]
    R = task_cov(theta)
    ka = np.concatenate([R[ta, u] * cross_q(w, theta, Xa, X[u]) for u in range(w.T)], axis=1)
    kb = np.concatenate([R[tb, u] * cross_q(w, theta, Xb, X[u]) for u in range(w.T)], axis=1)
    return R[ta, tb] * cross_q(w, theta, Xa, Xb) - ka @ sla.cho_solve(cf, kb.T)


def bayesian_cubature(w, y, theta=None, X=None, profile=None, res=None):
    """Posterior of the task integrals mu_t = int f(t, x) dx (Section
    "Extensions for Bayesian Cubature", multitask theorem): with
    gamma = int Q(x, x') dx' (the DSI and SI kernels here have zero-mean
    univariate parts, so gamma is the kernel's gamma),
      mu_hat = tau + gamma R E Ktilde^-1 (y - E^T tau),
      Sigma  = gamma R - gamma^2 R Pi R,   Pi = E Ktilde^-1 E^T.
    Returns dict(mu_hat[T], Sigma[T][T], Pi[T][T])."""
    theta = w.theta if theta is None else theta
    X = pts.task_points(w) if X is None else X
    res = nll(w, y, theta, X, profile) if res is None else res
    n = [x.shape[0] for x in X]
    E = summing_matrix(n)
    R = task_cov(theta)
    g = float(theta["gamma"])
    Pi = E @ sla.cho_solve(res["cf"], E.T)
    mu = res["tau_hat"] + g * R @ (E @ res["alpha"])
    Sigma = g * R - g * g * R @ Pi @ R
    return dict(mu_hat=mu, Sigma=Sigma, Pi=Pi)


def sample_prior(w, rng, theta=None, X=None):
    """y = E^T tau + chol(Ktilde) z, z ~ N(0, I): a draw from the MTGP prior."""
    theta = w.theta if theta is None else theta
    X = pts.task_points(w) if X is None else X
    K = gram(w, theta, X)
    Lc = np.linalg.cholesky(K)
    n = [x.shape[0] for x in X]
    z = rng.normal(size=K.shape[0])
    return summing_matrix(n).T @ np.asarray(theta["tau"], dtype=np.float64) + Lc @ z


def targets(w, rng, X=None):
    """Seeded targets of a workload on the oracle's points (task-major vector)."""
    import workloads
    X = pts.task_points(w) if X is None else X
    if w.target == "prior":
        return sample_prior(w, rng, X=X)
    ys = workloads.target_values(w, [kn.to_unit(x) for x in X], rng)
    return np.concatenate(ys)
