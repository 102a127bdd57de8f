"""Equal-size MLE loss through the eigenstructure of the Gram matrix (CPU,
float64).  Test infrastructure only: it lets loss parity reach sizes the
dense oracle cannot factor.

Theorem "Fast MTGP computations": with every task of size n, each block of
Ktilde is diagonalised by the same unitary V, so Ktilde = (I_T kron V)
Lambda (I_T kron V^dagger) with Lambda block-diagonal over frequencies f:

  Lambda(f)_tu = R_tu lambda_tu(f) + delta_tu xi_t,

and the MLE loss (Eq. MTGP_MLE_GCV_loss) is

  L = sum_f [ rhat(f)^H Lambda(f)^-1 rhat(f) + log det Lambda(f) ],
  rhat_t = V^dagger (y_t - tau_t 1).

* Digital nets, points in radical-inverse order: z_i XOR z_k = z_(i XOR k)
  (XOR-linearity), so block (t, u) is the dyadic convolution
  C[i, k] = c_tu[i XOR k] with c_tu[j] = Q(z_j XOR Delta_t XOR Delta_u).
  V = H / sqrt(n) (Sylvester-ordered Walsh-Hadamard) and lambda_tu = H c_tu.
* Rank-1 lattices: point i is (bitrev(i) g / n + Delta) mod 1, so in the
  natural order j = bitrev(i) block (t, u) is circulant,
  C[j, l] = c_tu[(j - l) mod n] with c_tu[j] = Q(j g / n + Delta_t - Delta_u);
  V = F^-1 sqrt(n) (F the DFT with e^{-2 pi i j f / n}) and lambda_tu = F c_tu.

Both V^dagger 1 = sqrt(n) e_0, so the normal equations of the optimal means
(Eq. MTGP_optimal_tau) involve frequency 0 only:
  n Lambda(0)^-1 tau_hat = sqrt(n) Lambda(0)^-1 yhat(0).

Pinned by: the dense oracle (tests/test_oracle_spectral.py) on small
designs of both families, every kernel order, fixed and profiled means.
"""
import numpy as np

from . import kernels as kn
from . import points as pts
from .dense import task_cov


def walsh(x):
    """Unnormalised Sylvester-ordered Walsh-Hadamard transform over the last
    axis (length a power of two): butterflies a + b, a - b per index bit."""
    x = np.array(x, dtype=np.float64, copy=True)
    n = x.shape[-1]
    lead = x.shape[:-1]
    h = 1
    while h < n:
        v = x.reshape(lead + (n // (2 * h), 2, h))
        a = v[..., 0, :].copy()
        b = v[..., 1, :]
        v[..., 0, :] = a + b
        v[..., 1, :] = a - b
        h *= 2
    return x


def _bitrev(n):
    m = n.bit_length() - 1
    i = np.arange(n, dtype=np.int64)
    r = np.zeros(n, dtype=np.int64)
    for b in range(m):
        r |= ((i >> b) & 1) << (m - 1 - b)
    return r


def _column(w, theta, t, u):
    """c_tu[j] in the order in which block (t, u) is a convolution."""
    n = 1 << w.m[t]
    b = None if theta.get("b") is None else np.asarray(theta["b"], dtype=np.float64)
    eta = np.asarray(theta["eta"], dtype=np.float64)
    if w.family == "dseq":
        z = pts.dseq_unshifted(w.gen, n)
        dig = z ^ (np.asarray(w.shift[t], dtype=np.uint32) ^ np.asarray(w.shift[u], dtype=np.uint32))[None, :]
    else:
        # natural order j: digit (j g 2^(32-m) + Delta_t - Delta_u) mod 2^32
        g = np.asarray(w.gen, dtype=np.uint64).reshape(-1)
        j = np.arange(n, dtype=np.uint64)
        base = ((j[:, None] * g[None, :]) << np.uint64(32 - w.m[t])) & np.uint64(0xFFFFFFFF)
        ds = (np.asarray(w.shift[t], dtype=np.int64) - np.asarray(w.shift[u], dtype=np.int64)) & 0xFFFFFFFF
        dig = ((base + ds.astype(np.uint64)[None, :]) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    q = np.full(n, float(theta["gamma"]))
    for k in range(w.d):
        q *= 1.0 + eta[k] * kn.univariate(w.family, w.kernel_order, w.adaptive, b, dig[:, k])
    return q


def nll_equal(w, y, theta=None, profile=None):
    """quad, logdet, L = quad + logdet and tau_hat for equal task sizes; y in
    the dense oracle's point order (task-major, radical-inverse order)."""
    theta = w.theta if theta is None else theta
    profile = w.profile_tau if profile is None else profile
    if len(set(w.m)) != 1:
        raise ValueError("equal task sizes only")
    T, n = w.T, 1 << w.m[0]
    Y = np.asarray(y, dtype=np.float64).reshape(T, n)
    R = task_cov(theta)
    xi = np.asarray(theta["xi"], dtype=np.float64)
    if w.family == "dseq":
        spec = lambda v: walsh(v).astype(np.complex128)
        yhat = spec(Y) / np.sqrt(n)
    else:
        nat = np.empty_like(Y)
        nat[:, _bitrev(n)] = Y  # point i sits at natural position bitrev(i)
        spec = lambda v: np.fft.fft(v, axis=-1)
        yhat = spec(nat) / np.sqrt(n)
    Lam = np.zeros((n, T, T), dtype=np.complex128)
    for t in range(T):
        for u in range(t, T):
            lam = spec(_column(w, theta, t, u))
            Lam[:, t, u] = R[t, u] * lam
            if u != t:
                Lam[:, u, t] = R[t, u] * np.conj(lam)
        Lam[:, t, t] += xi[t]
    Lc = np.linalg.cholesky(Lam)
    logdet = float(2.0 * np.sum(np.log(np.real(np.diagonal(Lc, axis1=1, axis2=2)))))
    if profile:
        inv0 = np.linalg.inv(Lam[0])
        tau = np.real(np.linalg.solve(n * inv0, np.sqrt(n) * (inv0 @ yhat[:, 0])))
    else:
        tau = np.asarray(theta["tau"], dtype=np.float64)
    rhat = yhat.T.copy()  # [n][T]
    rhat[0] -= np.sqrt(n) * tau
    a = np.linalg.solve(Lam, rhat[..., None])[..., 0]
    quad = float(np.real(np.sum(np.conj(rhat) * a)))
    return dict(quad=quad, logdet=logdet, L=quad + logdet, tau_hat=tau)
