"""Design points by their defining digit loops (test infrastructure only).

* Digital sequence (Def. "Base-2 digitally-shifted digital sequences"):
  z_i = XOR over the set bits p of i of the generating column g_p, and
  x_i = z_i XOR Delta.  Radical-inverse order: i = 0, 1, 2, ...
* Rank-1 lattice (Def. "Shifted rank-1 lattice"): z_i = v(i) g mod 1 with the
  van der Corput value v(i) = sum_p i_p 2^(-p-1), and x_i = (z_i + Delta) mod 1.

All coordinates are 32-bit digits u (x = u 2^-32).  For i < 2^32 the van der
Corput value is exactly V(i) 2^-32 with V(i) = sum_p i_p 2^(31-p), so the
lattice coordinate v(i) g mod 1 is exactly (V(i) g mod 2^32) 2^-32.

Pinned by: identity generating matrix gives the van der Corput sequence;
XOR-linearity z_i ^ z_k = z_(i^k); the recursive identities for 2^p > i
(Section "Algorithm for Gram Matrix Calculations"); the net property of the
leading digits.
"""
import numpy as np

MASK32 = (1 << 32) - 1


def van_der_corput_digits(n: int) -> np.ndarray:
    """V(i) = sum_p i_p 2^(31-p) for i < n, as uint32 (Def. of v(i))."""
    i = np.arange(n, dtype=np.uint64)
    v = np.zeros(n, dtype=np.uint64)
    for p in range(32):
        bit = (i >> np.uint64(p)) & np.uint64(1)
        v |= bit << np.uint64(31 - p)
    return v.astype(np.uint32)


def dseq_unshifted(gen: np.ndarray, n: int) -> np.ndarray:
    """z_i, i < n, for generating columns gen[j][p]; returns uint32 [n][d]."""
    gen = np.asarray(gen, dtype=np.uint32)
    d = gen.shape[0]
    i = np.arange(n, dtype=np.uint64)
    z = np.zeros((n, d), dtype=np.uint32)
    for p in range(64):
        if (n - 1) >> p == 0:
            break
        if p >= gen.shape[1]:
            raise ValueError("need more generating columns than given")
        sel = ((i >> np.uint64(p)) & np.uint64(1)).astype(bool)
        z[sel] ^= gen[:, p][None, :]
    return z


def dseq_points(gen: np.ndarray, n: int, shift: np.ndarray) -> np.ndarray:
    """x_i = z_i XOR Delta (digital shift)."""
    return dseq_unshifted(gen, n) ^ np.asarray(shift, dtype=np.uint32)[None, :]


def lattice_unshifted(gen: np.ndarray, n: int) -> np.ndarray:
    """z_i = v(i) g mod 1 as digits; gen[j][0] is g_j."""
    g = np.asarray(gen, dtype=np.uint64).reshape(-1)
    v = van_der_corput_digits(n).astype(np.uint64)
    return ((v[:, None] * g[None, :]) & np.uint64(MASK32)).astype(np.uint32)


def lattice_points(gen: np.ndarray, n: int, shift: np.ndarray) -> np.ndarray:
    """x_i = (z_i + Delta) mod 1 as digits."""
    z = lattice_unshifted(gen, n).astype(np.uint64)
    s = np.asarray(shift, dtype=np.uint64)[None, :]
    return ((z + s) & np.uint64(MASK32)).astype(np.uint32)


def task_points(w) -> list:
    """Per-task design points [n_t][d] (uint32) of a workload."""
    out = []
    for t in range(w.T):
        n = 1 << w.m[t]
        if w.family == "dseq":
            out.append(dseq_points(w.gen, n, w.shift[t]))
        else:
            out.append(lattice_points(w.gen, n, w.shift[t]))
    return out
