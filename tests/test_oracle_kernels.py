"""Pins of the oracle's kernels.

* Zero mean of every univariate kernel: the Bayesian-cubature section states
  that the SI and DSI product kernels have constant integral gamma, i.e. each
  univariate kernel integrates to zero over [0,1).  The printed order-1 DSI
  expression does not (it integrates to 5/36), which is why the oracle reads
  it as 1 - 3 t_1; the printed form is checked to fail here.
* Values at zero of Eq. DSI_kernel_1d_ex (beta(0) = t_nu(0) = 0).
* Spectra: on a 1-D van der Corput set the Walsh transform of each DSI
  kernel column is nonnegative (PSD), and for order 1 equals the closed form
  lambda_f / n = 4^-floor(log2 f) / 2 [f >= 1] + 4^-m.  On the 1-D lattice
  with g = 1 the DFT of the SI column equals the Fourier-series closed form
  n^(-2 alpha) (zeta(2 alpha, f/n) + zeta(2 alpha, 1 - f/n)) (Hurwitz zeta),
  which fixes the Bernoulli constant and sign of Eq. SI_kernel_1d_ex.
"""
import mpmath
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import kernels as kn
from oracle import points as pts

GL_X, GL_W = np.polynomial.legendre.leggauss(4)


def _integrate_digits(f):
    """int_0^1 f(x) dx for f given on 32-bit digits: Gauss-Legendre on dyadic
    cells inside each [2^-k, 2^(1-k)), where beta and t_nu are constant."""
    total = 0.0
    for k in range(1, 33):
        S = min(1 << 12, 1 << (32 - k))
        a = 2.0 ** -k
        h = a / S
        left = a + h * np.arange(S)
        x = left[:, None] + h * (GL_X[None, :] + 1) / 2
        u = np.clip(np.floor(x * 2.0 ** 32), 1, 2 ** 32 - 1).astype(np.uint64).astype(np.uint32)
        total += float(np.sum(f(u) * (h / 2) * GL_W[None, :]))
    total += 2.0 ** -32 * float(f(np.zeros(1, dtype=np.uint32))[0])
    return total


@pytest.mark.parametrize("alpha", [1, 2, 3, 4])
def test_dsi_zero_mean(alpha):
    assert abs(_integrate_digits(lambda u: kn.dsi_khat(alpha, u))) < 1e-8


def test_printed_order1_is_not_zero_mean():
    got = _integrate_digits(lambda u: kn.dsi_khat(1, u, printed_order1=True))
    assert abs(got - 5.0 / 36.0) < 1e-8


@pytest.mark.parametrize("alpha", [1, 2, 3])
def test_si_zero_mean(alpha):
    x = (np.arange(1 << 16) + 0.5) / (1 << 16)
    u = np.floor(x * 2.0 ** 32).astype(np.uint64).astype(np.uint32)
    assert abs(np.mean(kn.si_kern(alpha, u))) < 1e-9


def test_dsi_values_at_zero():
    z = np.zeros(1, dtype=np.uint32)
    got = [kn.dsi_khat(a, z)[0] for a in (1, 2, 3, 4)]
    np.testing.assert_allclose(got, [1.0, 1.5, 25.0 / 18.0, 407.0 / 294.0], rtol=0, atol=1e-15)


@pytest.mark.parametrize("alpha", [1, 2, 3, 4])
def test_dsi_walsh_spectrum_nonnegative(alpha):
    m = 10
    n = 1 << m
    c = kn.dsi_khat(alpha, pts.van_der_corput_digits(n))
    lam = sla.hadamard(n) @ c
    assert lam.min() > 0


def test_dsi_order1_walsh_closed_form():
    m = 9
    n = 1 << m
    lam = sla.hadamard(n) @ kn.dsi_khat(1, pts.van_der_corput_digits(n)) / n
    f = np.arange(n)
    pred = np.where(f >= 1, 0.5 * 4.0 ** (-np.floor(np.log2(np.maximum(f, 1)))), 0.0) + 4.0 ** -m
    np.testing.assert_allclose(lam, pred, rtol=0, atol=1e-15)


@pytest.mark.parametrize("alpha", [1, 2, 3])
def test_si_fourier_closed_form(alpha):
    m = 7
    n = 1 << m
    j = np.arange(n, dtype=np.uint64)
    c = kn.si_kern(alpha, (j << np.uint64(32 - m)).astype(np.uint32))
    lam = np.fft.fft(c) / n
    pred = [2 * n ** (-2 * alpha) * float(mpmath.zeta(2 * alpha)) if f == 0 else
            n ** (-2 * alpha) * float(mpmath.zeta(2 * alpha, f / n) + mpmath.zeta(2 * alpha, 1 - f / n))
            for f in range(n)]
    np.testing.assert_allclose(lam.real, pred, rtol=0, atol=1e-14)
    assert np.abs(lam.imag).max() < 1e-14


def test_pair_args():
    a = np.array([5, 0xFFFFFFFF], dtype=np.uint32)
    b = np.array([3, 1], dtype=np.uint32)
    np.testing.assert_array_equal(kn.pair_arg("dseq", a, b), [6, 0xFFFFFFFE])
    np.testing.assert_array_equal(kn.pair_arg("lat", b, a), [0xFFFFFFFE, 2])


def test_product_kernel_grads_match_finite_differences():
    rng = np.random.default_rng(5)
    u = rng.integers(0, 2 ** 32, size=(50, 3), dtype=np.uint64).astype(np.uint32)
    eta = np.array([0.7, 1.3, 2.0])
    b = np.array([0.5, 1.0, 0.3, 0.8])
    for fam, adaptive in (("dseq", True), ("lat", False)):
        Q, de, db = kn.product_kernel_grads(fam, 2, adaptive, b, 1.7, eta, u)
        h = 1e-6
        for j in range(3):
            ep, em = eta.copy(), eta.copy()
            ep[j] *= np.exp(h)
            em[j] *= np.exp(-h)
            fd = (kn.product_kernel(fam, 2, adaptive, b, 1.7, ep, u)
                  - kn.product_kernel(fam, 2, adaptive, b, 1.7, em, u)) / (2 * h)
            np.testing.assert_allclose(de[j], fd, rtol=1e-7, atol=1e-9)
        for a in range(len(db)):
            bp, bm = b.copy(), b.copy()
            bp[a] *= np.exp(h)
            bm[a] *= np.exp(-h)
            fd = (kn.product_kernel(fam, 2, adaptive, bp, 1.7, eta, u)
                  - kn.product_kernel(fam, 2, adaptive, bm, 1.7, eta, u)) / (2 * h)
            np.testing.assert_allclose(db[a], fd, rtol=1e-7, atol=1e-9)
