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
