"""Pins of the oracle's point generators against the definitions and the
recursive identities of Section "Algorithm for Gram Matrix Calculations"."""
import numpy as np

import workloads
from oracle import points as pts


def test_van_der_corput_values():
    # v(i) = sum_p i_p 2^(-p-1): v(1) = 1/2, v(2) = 1/4, v(3) = 3/4, v(4) = 1/8, v(6) = 3/8
    v = pts.van_der_corput_digits(8).astype(np.float64) * 2.0 ** -32
    np.testing.assert_array_equal(v, [0, 0.5, 0.25, 0.75, 0.125, 0.625, 0.375, 0.875])


def test_identity_generating_matrix_is_van_der_corput():
    gen = np.array([[1 << (31 - p) for p in range(32)]], dtype=np.uint32)
    z = pts.dseq_unshifted(gen, 1 << 10)[:, 0]
    np.testing.assert_array_equal(z, pts.van_der_corput_digits(1 << 10))


def test_xor_linearity_and_recursion():
    rng = np.random.default_rng(0)
    gen = workloads.random_dseq_gen(rng, 3)
    n = 1 << 12
    z = pts.dseq_unshifted(gen, n)
    i = rng.integers(0, n, 500)
    k = rng.integers(0, n, 500)
    np.testing.assert_array_equal(z[i] ^ z[k], z[i ^ k])
    for p in range(1, 12):
        ii = np.arange(1 << p)
        np.testing.assert_array_equal(z[(1 << p) + ii], z[1 << p] ^ z[ii])


def test_lattice_recursion_and_grid():
    rng = np.random.default_rng(1)
    gen = workloads.random_lattice_gen(rng, 4)
    n = 1 << 10
    z = pts.lattice_unshifted(gen, n).astype(np.uint64)
    for p in range(1, 10):
        ii = np.arange(1 << p)
        np.testing.assert_array_equal(z[(1 << p) + ii], (z[1 << p] + z[ii]) & 0xFFFFFFFF)
    # first n points are the grid {k/n} in each coordinate with odd g
    for j in range(4):
        assert sorted((z[:, j] >> np.uint64(22)).tolist()) == list(range(n))
        assert np.all((z[:, j] & np.uint64((1 << 22) - 1)) == 0)


def test_digital_net_leading_digits():
    # unit lower-triangular generating matrices: the leading m digits of each
    # coordinate of the first 2^m points are a permutation of 0..2^m-1
    rng = np.random.default_rng(2)
    gen = workloads.random_dseq_gen(rng, 5)
    for m in (1, 4, 9):
        z = pts.dseq_unshifted(gen, 1 << m)
        for j in range(5):
            lead = (z[:, j] >> np.uint32(32 - m)).astype(np.int64)
            assert sorted(lead.tolist()) == list(range(1 << m))


def test_shifts():
    rng = np.random.default_rng(3)
    gen = workloads.random_dseq_gen(rng, 2)
    s = np.array([0xDEADBEEF, 0x12345678], dtype=np.uint32)
    np.testing.assert_array_equal(pts.dseq_points(gen, 64, s), pts.dseq_unshifted(gen, 64) ^ s)
    g = workloads.random_lattice_gen(rng, 2)
    x = pts.lattice_points(g, 64, s).astype(np.uint64)
    z = pts.lattice_unshifted(g, 64).astype(np.uint64)
    np.testing.assert_array_equal(x, (z + s.astype(np.uint64)) & 0xFFFFFFFF)
