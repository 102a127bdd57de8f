"""Kernels of the fast (multitask) GP, evaluated on 32-bit digits (test infrastructure only).

* SI kernel (Def. "Shift-invariant kernel", Eq. SI_kernel_1d_ex):
  K(x, x') = (-1)^(alpha+1) (2 pi)^(2 alpha) / (2 alpha)! * B_(2 alpha)((x - x') mod 1)
  with B_p the Bernoulli polynomial.
* DSI kernel (Def. "Digitally-shift-invariant kernel", Eq. DSI_kernel_1d_ex):
  K(x, x') = sum_alpha b_alpha Khat_alpha(x XOR x'), with
  beta(x) = -floor(log2 x), t_nu(x) = 2^(-nu beta(x)), beta(0) = t_nu(0) = 0.
  Reading of the order-1 term: the printed expression does not integrate to
  zero over [0,1), which the Bayesian-cubature section says these kernels do;
  the order-one Walsh-space kernel it refers to is 6 (1/6 - t_1/2) = 1 - 3 t_1,
  which does.  ``printed_order1=True`` returns the printed form instead.
  The order-4 digit series sum_(a>=1) (1 - 2 x_a) 8^-(a-1) is evaluated with
  the 32 available digits: digits beyond the 32nd are zero, so the tail adds
  sum_(a>32) 8^-(a-1) = (8/7) 8^-32.
* Product form (Eq. prod_kernel): Q(x, x') = gamma prod_j [1 + eta_j K(x_j, x'_j)].

Pinned by: zero mean of every univariate kernel (Bayesian-cubature section),
the values at zero, nonnegative Walsh / Fourier spectra on one-dimensional
nets, and the Fourier-series closed form of the SI kernel
(sum_(k != 0) e^(2 pi i k x) / |k|^(2 alpha)).
"""
import math

import numpy as np

TWO_M32 = 2.0 ** -32


def to_unit(u):
    """Digits -> float64 coordinate u 2^-32 (exact)."""
    return np.asarray(u, dtype=np.float64) * TWO_M32


def beta(u):
    """beta(x) = -floor(log2 x) for x = u 2^-32 > 0, and beta(0) = 0."""
    u = np.asarray(u, dtype=np.uint64)
    _, ex = np.frexp(u.astype(np.float64))       # u = mant 2^ex, 0.5 <= mant < 1
    b = (33 - ex).astype(np.float64)             # floor(log2 u) = ex - 1
    return np.where(u == 0, 0.0, b)


def t_nu(u, nu):
    """t_nu(x) = 2^(-nu beta(x)), t_nu(0) = 0."""
    u = np.asarray(u, dtype=np.uint64)
    b = beta(u)
    return np.where(u == 0, 0.0, np.exp2(-nu * b))


def _order4_digit_sum(u):
    """sum_(a>=1) (1 - 2 x_a) 8^-(a-1) over the binary digits x_a of x = u 2^-32."""
    u = np.asarray(u, dtype=np.uint64)
    s = np.zeros(u.shape, dtype=np.float64)
    for a in range(1, 33):
        xa = ((u >> np.uint64(32 - a)) & np.uint64(1)).astype(np.float64)
        s += (1.0 - 2.0 * xa) * 8.0 ** (-(a - 1))
    s += (8.0 / 7.0) * 8.0 ** (-32)
    return s


def dsi_khat(alpha: int, u, printed_order1: bool = False):
    """Khat_alpha(x), x = u 2^-32, for alpha in {1, 2, 3, 4}."""
    x = to_unit(u)
    b = beta(u)
    t1, t2, t3 = t_nu(u, 1), t_nu(u, 2), t_nu(u, 3)
    if alpha == 1:
        if printed_order1:
            return (1.0 / 6.0) * (1.0 - 0.5 * t1)
        return 6.0 * (1.0 / 6.0 - 0.5 * t1)
    if alpha == 2:
        return -1.0 - b * x + 2.5 * (1.0 - t1)
    if alpha == 3:
        return -1.0 + b * x * x - 5.0 * (1.0 - t1) * x + (43.0 / 18.0) * (1.0 - t2)
    if alpha == 4:
        return (-1.0 - (2.0 / 3.0) * b * x ** 3 + 5.0 * (1.0 - t1) * x * x
                - (43.0 / 9.0) * (1.0 - t2) * x + (701.0 / 294.0) * (1.0 - t3)
                + b * (_order4_digit_sum(u) / 48.0 - 1.0 / 42.0))
    raise ValueError("DSI order must be 1..4")


def bernoulli_poly(p: int, x):
    """Bernoulli polynomials B_2, B_4, B_6 (standard closed forms)."""
    x = np.asarray(x, dtype=np.float64)
    if p == 2:
        return x * x - x + 1.0 / 6.0
    if p == 4:
        return x ** 4 - 2.0 * x ** 3 + x * x - 1.0 / 30.0
    if p == 6:
        return x ** 6 - 3.0 * x ** 5 + 2.5 * x ** 4 - 0.5 * x * x + 1.0 / 42.0
    raise ValueError("Bernoulli degree must be 2, 4 or 6")


def si_kern(alpha: int, u):
    """(-1)^(alpha+1) (2 pi)^(2 alpha) / (2 alpha)! B_(2 alpha)(x), x = u 2^-32 in [0,1)."""
    c = (-1.0) ** (alpha + 1) * (2.0 * math.pi) ** (2 * alpha) / math.factorial(2 * alpha)
    return c * bernoulli_poly(2 * alpha, to_unit(u))


def pair_arg(family: str, xa, xb):
    """Kernel argument digits: x XOR x' (DSEQ) or (x - x') mod 1 (LAT)."""
    xa = np.asarray(xa, dtype=np.uint32)
    xb = np.asarray(xb, dtype=np.uint32)
    if family == "dseq":
        return xa ^ xb
    return ((xa.astype(np.int64) - xb.astype(np.int64)) & 0xFFFFFFFF).astype(np.uint32)


def univariate_terms(family: str, order: int, adaptive: bool, u):
    """List of (weight index, values) of the univariate terms at digits u.

    Non-adaptive kernels have a single term (weight index None).  The
    adaptive DSI kernel has the four terms Khat_1..Khat_4 weighted by b.
    """
    if family == "dseq":
        if adaptive:
            return [(a - 1, dsi_khat(a, u)) for a in (1, 2, 3, 4)]
        return [(None, dsi_khat(order, u))]
    if adaptive:
        raise ValueError("adaptive weights are defined for DSI kernels only")
    return [(None, si_kern(order, u))]


def univariate(family, order, adaptive, b, u):
    """The univariate kernel value K(u) = sum_alpha b_alpha Khat_alpha(u)."""
    s = 0.0
    for idx, v in univariate_terms(family, order, adaptive, u):
        s = s + (v if idx is None else b[idx] * v)
    return s


def product_kernel(family, order, adaptive, b, gamma, eta, u):
    """Q = gamma prod_j (1 + eta_j K(u_j)); u has trailing axis d."""
    u = np.asarray(u)
    d = u.shape[-1]
    q = np.full(u.shape[:-1], float(gamma))
    for j in range(d):
        q = q * (1.0 + eta[j] * univariate(family, order, adaptive, b, u[..., j]))
    return q


def product_kernel_grads(family, order, adaptive, b, gamma, eta, u):
    """(Q, dQ/dlog eta_j for each j, dQ/dlog b_alpha for each alpha or []).

    dQ/dlog eta_j = gamma eta_j K_j prod_(k != j)(1 + eta_k K_k); the product
    over k != j is formed directly (no division), as the definition reads.
    """
    u = np.asarray(u)
    d = u.shape[-1]
    Kj = [univariate(family, order, adaptive, b, u[..., j]) for j in range(d)]
    fac = [1.0 + eta[j] * Kj[j] for j in range(d)]
    Q = np.full(u.shape[:-1], float(gamma))
    for j in range(d):
        Q = Q * fac[j]
    dlog_eta = []
    for j in range(d):
        g = np.full(u.shape[:-1], float(gamma)) * eta[j] * Kj[j]
        for k in range(d):
            if k != j:
                g = g * fac[k]
        dlog_eta.append(g)
    dlog_b = []
    if adaptive:
        for a in range(4):
            tot = np.zeros(u.shape[:-1])
            for j in range(d):
                g = np.full(u.shape[:-1], float(gamma)) * eta[j] * b[a] * dsi_khat(a + 1, u[..., j])
                for k in range(d):
                    if k != j:
                        g = g * fac[k]
                tot = tot + g
            dlog_b.append(tot)
    return Q, dlog_eta, dlog_b
