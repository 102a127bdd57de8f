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

Nested sizes (any task order).  With n_t >= n_u the points of task u are
the first n_u points of the same sequence as task t, so block (t, u) is the
first n_u columns of the n_t x n_t convolution with c_tu of length n_t, and
in the spectral bases of the two tasks it is

  [V_t^dagger K_tu V_u](f, g) = sqrt(n_u / n_t) R_tu lambda_tu(f) [f = g mod n_u]

(for nets H_t[f, k] = H_u[f mod n_u, k] when k < n_u; for lattices the
points of u sit at every (n_t / n_u)-th natural position of t).  Frequencies
therefore fall into independent residue classes r mod n_min, each a dense
Hermitian matrix over the members (t, f = r + n_min k), k < n_t / n_min.
The MLE and GCV losses are sums over the classes; the means live in class 0
(V_t^dagger 1 = sqrt(n_t) e_0).  `mle` and `gcv` take this route for any
sizes, equal sizes included.

Pinned by: the dense oracle (tests/test_oracle_spectral.py) on small
designs of both families, every kernel order, fixed and profiled means,
equal and nested sizes in several task orders.
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


def _column_digits(w, t, u):
    """Kernel-argument digits [n_t][d] of c_tu in its convolution order."""
    n = 1 << w.m[t]
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
    return dig


def _column(w, theta, t, u):
    """c_tu[j] in the order in which block (t, u) is a convolution."""
    n = 1 << w.m[t]
    b = None if theta.get("b") is None else np.asarray(theta["b"], dtype=np.float64)
    eta = np.asarray(theta["eta"], dtype=np.float64)
    dig = _column_digits(w, t, u)
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


# ------------------------------------------------------------- nested sizes
def _task_spectrum(w, t, v):
    """V_t^dagger v for one task's vector v (oracle point order)."""
    n = 1 << w.m[t]
    v = np.asarray(v, dtype=np.float64)
    if w.family == "dseq":
        return walsh(v) / np.sqrt(n)
    nat = np.empty_like(v)
    nat[_bitrev(n)] = v
    return np.fft.fft(nat) / np.sqrt(n)


class _Classes:
    """Residue-class blocks of Ktilde in the tasks' spectral bases."""

    def __init__(self, w, theta):
        self.w, self.T = w, w.T
        self.n = [1 << m for m in w.m]
        self.nmin = min(self.n)
        self.size = [nt // self.nmin for nt in self.n]          # members per class
        self.off = np.concatenate([[0], np.cumsum(self.size)]).astype(np.int64)
        self.c = int(self.off[-1])
        self.real = w.family == "dseq"
        self.R = task_cov(theta)
        self.xi = np.asarray(theta["xi"], dtype=np.float64)
        self.lam = {}
        for t in range(self.T):
            for u in range(self.T):
                big = self.n[t] > self.n[u] or (self.n[t] == self.n[u] and t <= u)
                if big:
                    c = _column(self.w, theta, t, u)
                    self.lam[(t, u)] = walsh(c) if self.real else np.fft.fft(c)

    def matrices(self, r):
        """Dense class matrices for the classes in r, shape [len(r), c, c]."""
        r = np.asarray(r, dtype=np.int64)
        M = np.zeros((r.size, self.c, self.c), dtype=np.float64 if self.real else np.complex128)
        for (t, u), lam in self.lam.items():
            k = np.arange(self.size[t])
            l = k % self.size[u]
            vals = np.sqrt(self.n[u] / self.n[t]) * self.R[t, u] * lam[r[:, None] + self.nmin * k[None, :]]
            if self.real:
                vals = vals.real
            M[:, self.off[t] + k, self.off[u] + l] += vals
            if t != u:
                M[:, self.off[u] + l, self.off[t] + k] += np.conj(vals)
        for t in range(self.T):
            i = self.off[t] + np.arange(self.size[t])
            M[:, i, i] += self.xi[t]
        return M

    def data(self, y):
        """yhat[r, member] for every class r (shape [n_min, c])."""
        offs = np.concatenate([[0], np.cumsum(self.n)])
        out = np.zeros((self.nmin, self.c), dtype=np.float64 if self.real else np.complex128)
        for t in range(self.T):
            sp = _task_spectrum(self.w, t, y[offs[t]:offs[t + 1]])
            # frequency f = r + n_min k is member k of class r
            out[:, self.off[t]:self.off[t + 1]] = sp.reshape(self.size[t], self.nmin).T
        return out

    def mean_columns(self):
        """Class-0 image of E^T: column t is sqrt(n_t) at member (t, 0)."""
        A = np.zeros((self.c, self.T))
        for t in range(self.T):
            A[self.off[t], t] = np.sqrt(self.n[t])
        return A

    def chunks(self, budget=1 << 28):
        step = max(1, budget // (16 * self.c * self.c))
        for r0 in range(0, self.nmin, step):
            yield np.arange(r0, min(self.nmin, r0 + step))


def _profiled_tau(cl, yh0, power):
    """Normal equations in class 0: (A^H M0^-p A) tau = A^H M0^-p yhat(0).
    Also returns the 2-norm condition numbers of M0 and of A^H M0^-p A, whose
    product (times the unit roundoff) bounds the relative error of tau in
    FP64 arithmetic after p solves with M0."""
    A = cl.mean_columns()
    M0 = cl.matrices([0])[0]
    X = np.linalg.solve(M0, np.column_stack([A, yh0]))
    if power == 2:
        X = np.linalg.solve(M0, X)
    G = A.T @ X
    Gm = np.real(G[:, :cl.T])
    tau = np.linalg.solve(Gm, np.real(G[:, cl.T]))
    return tau, float(np.linalg.cond(M0)), float(np.linalg.cond(Gm))


def mle(w, y, theta=None, profile=None):
    """quad, logdet, L = quad + logdet and tau_hat for any nested sizes; y in
    the dense oracle's point order.  cond_M0 and cond_normal are the condition
    numbers of the class-0 block and of the normal equations of tau."""
    theta = w.theta if theta is None else theta
    profile = w.profile_tau if profile is None else profile
    cl = _Classes(w, theta)
    yh = cl.data(np.asarray(y, dtype=np.float64))
    tau, cond0, condn = _profiled_tau(cl, yh[0], 1)
    if not profile:
        tau = np.asarray(theta["tau"], dtype=np.float64)
    yh[0] -= cl.mean_columns() @ tau
    quad = logdet = 0.0
    for r in cl.chunks():
        Lc = np.linalg.cholesky(cl.matrices(r))
        logdet += float(2.0 * np.sum(np.log(np.real(np.diagonal(Lc, axis1=1, axis2=2)))))
        z = np.linalg.solve(Lc, yh[r][..., None])[..., 0]       # Lc z = rhat
        quad += float(np.sum(np.abs(z) ** 2))
    return dict(quad=quad, logdet=logdet, L=quad + logdet, tau_hat=tau, cond_M0=cond0,
                cond_normal=condn)


def gcv(w, y, theta=None, profile=None):
    """GCV pieces q = r^H Ktilde^-2 r, s = tr Ktilde^-1, L = q / s^2 and the
    GCV means (E Ktilde^-2 E^T) tau = E Ktilde^-2 y, for any nested sizes."""
    theta = w.theta if theta is None else theta
    profile = w.profile_tau if profile is None else profile
    cl = _Classes(w, theta)
    yh = cl.data(np.asarray(y, dtype=np.float64))
    tau, cond0, condn = _profiled_tau(cl, yh[0], 2)
    if not profile:
        tau = np.asarray(theta["tau"], dtype=np.float64)
    yh[0] -= cl.mean_columns() @ tau
    q = s = 0.0
    for r in cl.chunks():
        M = cl.matrices(r)
        a = np.linalg.solve(M, yh[r][..., None])[..., 0]
        q += float(np.sum(np.abs(a) ** 2))
        Minv = np.linalg.inv(M)
        s += float(np.sum(np.real(np.diagonal(Minv, axis1=1, axis2=2))))
    return dict(q=q, s=s, L=q / (s * s), tau_hat=tau, cond_M0=cond0, cond_normal=condn)


def _param_grad(w, theta, cl, chunk_w):
    """sum_r tr(W_r dM_r / dtheta) for every non-mean parameter, with W_r =
    chunk_w(r, M_r) Hermitian: dM_r takes the spectra of the derivative
    columns dc_tu / dtheta (log gamma, log eta_j, log b_alpha) and of c_tu
    (for R = B B^T + diag(zeta)), and xi_t on the diagonal."""
    T, d = w.T, w.d
    # Z[(t, u)][f] = W_(u, f mod n_u),(t, f) over the stored pairs; xi terms
    Z = {key: np.zeros(cl.n[key[0]], dtype=np.float64 if cl.real else np.complex128)
         for key in cl.lam}
    g_xi = np.zeros(T)
    xi = np.asarray(theta["xi"], dtype=np.float64)
    for r in cl.chunks():
        W = chunk_w(r, cl.matrices(r))
        for (t, u) in cl.lam:
            k = np.arange(cl.size[t])
            l = k % cl.size[u]
            Z[(t, u)][r[:, None] + cl.nmin * k[None, :]] = W[:, cl.off[u] + l, cl.off[t] + k]
        for t in range(T):
            i = cl.off[t] + np.arange(cl.size[t])
            g_xi[t] += xi[t] * float(np.sum(np.real(W[:, i, i])))
    b = None if theta.get("b") is None else np.asarray(theta["b"], dtype=np.float64)
    eta = np.asarray(theta["eta"], dtype=np.float64)
    R = cl.R
    spec = walsh if cl.real else (lambda v: np.fft.fft(v))
    G = np.zeros((T, T))
    g_eta = np.zeros(d)
    g_b = np.zeros(4) if w.adaptive else None
    for (t, u), lam in cl.lam.items():
        mult = 1.0 if t == u else 2.0
        sc = np.sqrt(cl.n[u] / cl.n[t])
        z = Z[(t, u)]
        G[t, u] = G[u, t] = float(np.real(np.sum(z * sc * lam)))
        _, dq_eta, dq_b = kn.product_kernel_grads(w.family, w.kernel_order, w.adaptive, b,
                                                  theta["gamma"], eta, _column_digits(w, t, u))
        for j in range(d):
            g_eta[j] += mult * sc * R[t, u] * float(np.real(np.sum(z * spec(dq_eta[j]))))
        if w.adaptive:
            for al in range(4):
                g_b[al] += mult * sc * R[t, u] * float(np.real(np.sum(z * spec(dq_b[al]))))
    # Q is proportional to gamma; R = B B^T + diag(zeta)
    B = np.asarray(theta["B"], dtype=np.float64)
    zeta = np.asarray(theta["zeta"], dtype=np.float64)
    out = dict(gamma=float(np.sum(R * G)), eta=g_eta, xi=g_xi, B=(G + G.T) @ B,
               zeta=zeta * np.diag(G))
    if w.adaptive:
        out["b"] = g_b
    return out


def mle_grad(w, y, theta=None, profile=None):
    """Exact gradient of the MLE loss in the packed parameterisation (dict
    keyed like theta), for any nested sizes:

      dL/dtheta = sum_r tr( (M_r^-1 - a_r a_r^H) dM_r/dtheta ),  a_r = M_r^-1 rhat_r.

    Profiled means contribute nothing (tau_hat is stationary); fixed means
    give -2 Re(A^T a_0).  Also returns the loss pieces of `mle`."""
    theta = w.theta if theta is None else theta
    profile = w.profile_tau if profile is None else profile
    res = mle(w, y, theta, profile)
    cl = _Classes(w, theta)
    yh = cl.data(np.asarray(y, dtype=np.float64))
    A = cl.mean_columns()
    yh[0] -= A @ res["tau_hat"]
    keep = {}

    def chunk_w(r, M):
        Minv = np.linalg.inv(M)
        a = np.einsum("rij,rj->ri", Minv, yh[r])
        if r[0] == 0:
            keep["a0"] = a[0]
        return Minv - a[:, :, None] * np.conj(a[:, None, :])

    out = _param_grad(w, theta, cl, chunk_w)
    out["tau"] = np.zeros(w.T) if profile else -2.0 * np.real(A.T @ keep["a0"])
    return out, res


def gcv_grad(w, y, theta=None, profile=None):
    """Exact gradient of L_GCV = q / s^2 (q = r^H Ktilde^-2 r, s = tr
    Ktilde^-1), for any nested sizes: with a_r = M_r^-1 rhat_r and
    b_r = M_r^-1 a_r,

      dL/dtheta = sum_r tr( W_r dM_r/dtheta ),
      W_r = -(a_r b_r^H + b_r a_r^H) / s^2 + (2 q / s^3) M_r^-2.

    Profiled GCV means contribute nothing; fixed means give
    -2 Re(A^T b_0) / s^2.  Also returns the loss pieces of `gcv`."""
    theta = w.theta if theta is None else theta
    profile = w.profile_tau if profile is None else profile
    res = gcv(w, y, theta, profile)
    q, s2 = res["q"], res["s"]
    cl = _Classes(w, theta)
    yh = cl.data(np.asarray(y, dtype=np.float64))
    A = cl.mean_columns()
    yh[0] -= A @ res["tau_hat"]
    keep = {}

    def chunk_w(r, M):
        Minv = np.linalg.inv(M)
        a = np.einsum("rij,rj->ri", Minv, yh[r])
        b = np.einsum("rij,rj->ri", Minv, a)
        if r[0] == 0:
            keep["b0"] = b[0]
        ab = a[:, :, None] * np.conj(b[:, None, :])
        return -(ab + np.conj(np.swapaxes(ab, 1, 2))) / s2 ** 2 + (2.0 * q / s2 ** 3) * (Minv @ Minv)

    out = _param_grad(w, theta, cl, chunk_w)
    out["tau"] = np.zeros(w.T) if profile else -2.0 * np.real(A.T @ keep["b0"]) / s2 ** 2
    return out, res


def weights(w, y, theta=None, profile=None):
    """alpha = Ktilde^-1 (y - E^T tau) in the dense oracle's point order,
    from a_r = M_r^-1 rhat_r mapped back per task (alpha_t = V_t ahat_t), with
    tau_hat, E alpha = A^T a_0 and Pi = E Ktilde^-1 E^T = A^T M0^-1 A."""
    theta = w.theta if theta is None else theta
    profile = w.profile_tau if profile is None else profile
    cl = _Classes(w, theta)
    yh = cl.data(np.asarray(y, dtype=np.float64))
    tau, _, _ = _profiled_tau(cl, yh[0], 1)
    if not profile:
        tau = np.asarray(theta["tau"], dtype=np.float64)
    A = cl.mean_columns()
    yh[0] -= A @ tau
    ahat = [np.zeros(nt, dtype=yh.dtype) for nt in cl.n]
    for r in cl.chunks():
        a = np.linalg.solve(cl.matrices(r), yh[r][..., None])[..., 0]
        for t in range(w.T):
            k = np.arange(cl.size[t])
            ahat[t][r[:, None] + cl.nmin * k[None, :]] = a[:, cl.off[t] + k]
        if r[0] == 0:
            Ea = np.real(A.T @ a[0])
    alpha = []
    for t in range(w.T):
        n = cl.n[t]
        if cl.real:
            alpha.append(walsh(ahat[t]) / np.sqrt(n))
        else:
            nat = np.fft.ifft(ahat[t]) * np.sqrt(n)     # V_t = F^H / sqrt(n)
            alpha.append(np.real(nat[_bitrev(n)]))      # point i at natural bitrev(i)
    M0 = cl.matrices([0])[0]
    Pi = np.real(A.T @ np.linalg.solve(M0, A))
    return dict(alpha=np.concatenate(alpha), tau_hat=tau, E_alpha=Ea, Pi=Pi)


def cubature(w, y, theta=None, profile=None):
    """Bayesian cubature of the task integrals (gamma = int Q(x, x') dx'):
    mu_hat = tau + gamma R E alpha, Sigma = gamma R - gamma^2 R Pi R."""
    theta = w.theta if theta is None else theta
    res = weights(w, y, theta, profile)
    R = task_cov(theta)
    g = float(theta["gamma"])
    return dict(mu_hat=res["tau_hat"] + g * R @ res["E_alpha"],
                Sigma=g * R - g * g * R @ res["Pi"] @ R, Pi=res["Pi"])
