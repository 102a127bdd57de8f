"""Seeded synthetic workloads shared by the oracle-side tests and the GPU path.

This module only draws random numbers and fixes shapes: generating matrices,
shifts, hyperparameters, test-point digits and target functions of given
coordinates.  It contains none of the fast-MTGP arithmetic (no point
generation, no kernel evaluation, no transform, no solve), so the oracle and
the HIP library can both consume its outputs without sharing method code.

Conventions (stated once, used everywhere):

* Digits.  Every coordinate is a uint32 ``u`` standing for ``u * 2**-32``.
* Digital-net generating columns (DSEQ): ``gen[j][p]`` is column ``p`` of the
  generating matrix of dimension ``j``; bit ``31 - p`` is set (unit diagonal),
  lower bits are random, higher bits are zero (lower-triangular unit matrix
  with row = output digit, column = input digit).
* Lattice generating vector (LAT): ``gen[j][0]`` is the odd integer ``g_j``.
* Shifts: ``shift[t][j]`` is the digital shift (DSEQ) or the lattice shift
  times ``2**32`` (LAT) of task ``t``.
* Hyperparameters are held unpacked in a dict:
  ``tau[T], gamma, eta[d], b[4] (adaptive kernels only), xi[T], B[T][s],
  zeta[T]`` with task covariance ``R = B B^T + diag(zeta)``.

The five named workloads mirror the shapes of the paper's experiments
(digitally shifted nets, per-task shifts, nested power-of-two sizes; Section
4, Table of problem parameters) at the sizes of the benchmark configurations.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

DSEQ = "dseq"
LAT = "lat"


@dataclasses.dataclass
class Workload:
    name: str
    family: str               # DSEQ or LAT
    T: int
    d: int
    m: list                   # per-task log2 sizes, non-increasing
    kernel_order: int         # alpha
    adaptive: bool            # DSI only: K = sum_alpha b_alpha K_alpha
    gen: np.ndarray           # uint32 [d][32] (DSEQ) or [d][1] (LAT)
    shift: np.ndarray         # uint32 [T][d]
    theta: dict               # unpacked hyperparameters (see module doc)
    profile_tau: bool
    seed: int
    target: str               # "sincos", "corr_sines", "prior"
    target_params: dict
    noise_var: float
    n_test: int

    @property
    def n(self):
        return [1 << mt for mt in self.m]

    @property
    def N(self):
        return int(sum(self.n))

    @property
    def rank_s(self):
        return int(np.asarray(self.theta["B"]).shape[1])


# --------------------------------------------------------------------------
# generators of the design ingredients
# --------------------------------------------------------------------------
def random_dseq_gen(rng: np.random.Generator, d: int) -> np.ndarray:
    """Random lower-triangular unit generating matrices, 32 input digits."""
    gen = np.zeros((d, 32), dtype=np.uint32)
    for j in range(d):
        for p in range(32):
            top = 31 - p
            low = int(rng.integers(0, 1 << 32, dtype=np.uint64)) & ((1 << top) - 1)
            gen[j, p] = (1 << top) | low
    return gen


def random_lattice_gen(rng: np.random.Generator, d: int, bits: int = 16) -> np.ndarray:
    """Odd generating-vector entries below 2**bits."""
    g = rng.integers(0, 1 << (bits - 1), size=d, dtype=np.int64) * 2 + 1
    return g.astype(np.uint32).reshape(d, 1)


def random_shifts(rng: np.random.Generator, T: int, d: int) -> np.ndarray:
    return rng.integers(0, 1 << 32, size=(T, d), dtype=np.uint64).astype(np.uint32)


def uniform_digits(rng: np.random.Generator, M: int, d: int) -> np.ndarray:
    """Uniform test points as digits (floor(x * 2**32) of uniform x)."""
    return rng.integers(0, 1 << 32, size=(M, d), dtype=np.uint64).astype(np.uint32)


def digits_to_float(u: np.ndarray) -> np.ndarray:
    """x = u * 2**-32 (exact in float64)."""
    return np.asarray(u, dtype=np.float64) * (2.0 ** -32)


# --------------------------------------------------------------------------
# target functions of given coordinates x[..., d] in [0,1)
# --------------------------------------------------------------------------
def target_values(w: Workload, x_per_task: list, rng: np.random.Generator) -> list:
    """Targets y_t for each task's coordinates (list of float arrays [n_t][d])."""
    out = []
    p = w.target_params
    for t, x in enumerate(x_per_task):
        x = np.asarray(x, dtype=np.float64)
        if w.target == "sincos":
            # sum_j sin(2 pi (j+1) x_j) + 0.3 * t * prod_j x_j, tasks t = 1..T
            y = np.zeros(x.shape[0])
            for j in range(w.d):
                y += np.sin(2 * np.pi * (j + 1) * x[:, j])
            y += 0.3 * (t + 1) * np.prod(x, axis=1)
        elif w.target in ("corr_sines", "prior"):
            # rho_t g_0 + sqrt(1 - rho_t^2) g_t,
            # g_k(x) = sum_j j^-1 sin(2 pi k_kj x_j + phi_kj), j = 1..d
            def g(k):
                s = np.zeros(x.shape[0])
                for j in range(w.d):
                    s += np.sin(2 * np.pi * p["freq"][k][j] * x[:, j] + p["phase"][k][j]) / (j + 1)
                return s
            rho = p["rho"][t]
            y = rho * g(0) + math.sqrt(1 - rho * rho) * g(t + 1)
        else:
            raise ValueError(w.target)
        y = y + rng.normal(0.0, math.sqrt(w.noise_var), size=y.shape)
        out.append(y)
    return out


def _corr_sine_params(rng, T, d):
    return {
        "freq": rng.integers(1, 4, size=(T + 1, d)).tolist(),
        "phase": rng.uniform(0, 2 * np.pi, size=(T + 1, d)).tolist(),
        "rho": rng.uniform(0.5, 0.95, size=T).tolist(),
    }


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------
def config1() -> Workload:
    """T=2, d=2, n=2^10 digital net per task, order-2 DSI kernel, FP64."""
    rng = np.random.default_rng(1)
    T, d = 2, 2
    gen = random_dseq_gen(rng, d)
    shift = random_shifts(rng, T, d)
    theta = dict(tau=np.zeros(T), gamma=1.0, eta=np.ones(d), b=None,
                 xi=np.full(T, 1e-8), B=np.sqrt(0.8) * np.ones((T, 1)),
                 zeta=np.full(T, 0.2))
    return Workload("config1_dseq_T2_d2_n2^10", DSEQ, T, d, [10, 10], 2, False, gen,
                    shift, theta, True, 1, "sincos", {}, 1e-4, 1024)


def config2() -> Workload:
    """T=4, d=6, n=2^16 lattice per task, order-2 SI kernel, FFT path."""
    rng = np.random.default_rng(2)
    T, d = 4, 6
    gen = random_lattice_gen(rng, d)
    shift = random_shifts(rng, T, d)
    eta = np.exp(rng.uniform(np.log(0.1), np.log(10.0), size=d))
    B = rng.normal(0.0, 1.0, size=(T, 2))
    theta = dict(tau=np.zeros(T), gamma=1.0, eta=eta, b=None, xi=np.full(T, 1e-4),
                 B=B, zeta=np.full(T, 0.1))
    return Workload("config2_lat_T4_d6_n2^16", LAT, T, d, [16] * T, 2, False, gen, shift,
                    theta, True, 2, "prior", _corr_sine_params(rng, T, d), 1e-6, 1024)


def config3() -> Workload:
    """T=5, d=8, nested n = 2^20..2^12 digital nets, order-4 DSI kernel."""
    rng = np.random.default_rng(3)
    T, d = 5, 8
    gen = random_dseq_gen(rng, d)
    shift = random_shifts(rng, T, d)
    B = rng.normal(0.0, math.sqrt(1.0 / 3.0), size=(T, 3))
    theta = dict(tau=np.zeros(T), gamma=1.0, eta=np.ones(d), b=None, xi=np.full(T, 1e-4),
                 B=B, zeta=np.full(T, 0.1))
    return Workload("config3_dseq_T5_d8_nested2^20..2^12", DSEQ, T, d, [20, 18, 16, 14, 12],
                    4, False, gen, shift, theta, True, 3, "corr_sines",
                    _corr_sine_params(rng, T, d), 1e-6, 1024)


def config5() -> Workload:
    """T=8, d=10, n=2^24 digital net per task, order-2 DSI kernel."""
    rng = np.random.default_rng(5)
    T, d = 8, 10
    gen = random_dseq_gen(rng, d)
    shift = random_shifts(rng, T, d)
    B = rng.normal(0.0, math.sqrt(0.5), size=(T, 2))
    theta = dict(tau=np.zeros(T), gamma=1.0, eta=np.ones(d), b=None, xi=np.full(T, 1e-3),
                 B=B, zeta=np.full(T, 0.1))
    return Workload("config5_dseq_T8_d10_n2^24", DSEQ, T, d, [24] * T, 2, False, gen, shift,
                    theta, True, 5, "corr_sines", _corr_sine_params(rng, T, d), 1e-6, 1 << 20)


def config5_lat() -> Workload:
    """The config-5 shape on the lattice path: T=8, d=10, n=2^24 rank-1
    lattice per task, order-2 SI kernel (the paper names shift-invariant
    kernels on lattices as the untested variant of its method)."""
    rng = np.random.default_rng(6)
    T, d = 8, 10
    gen = random_lattice_gen(rng, d, bits=24)
    shift = random_shifts(rng, T, d)
    B = rng.normal(0.0, math.sqrt(0.5), size=(T, 2))
    theta = dict(tau=np.zeros(T), gamma=1.0, eta=np.full(d, 0.5), b=None, xi=np.full(T, 1e-3),
                 B=B, zeta=np.full(T, 0.1))
    return Workload("config5_lat_T8_d10_n2^24", LAT, T, d, [24] * T, 2, False, gen, shift,
                    theta, True, 6, "corr_sines", _corr_sine_params(rng, T, d), 1e-6, 1 << 20)


def config4_fits(nfits: int = 256, seed: int = 4, kmin: int = 8, kmax: int = 14) -> list:
    """Many independent fits: T in 2..8, d in 2..10, mixed families, n_t = 2^k."""
    rng = np.random.default_rng(seed)
    fits = []
    for f in range(nfits):
        T = int(rng.integers(2, 9))
        d = int(rng.integers(2, 11))
        fam = LAT if rng.random() < 0.5 else DSEQ
        m = sorted((int(k) for k in rng.integers(kmin, kmax + 1, size=T)), reverse=True)
        gen = random_lattice_gen(rng, d) if fam == LAT else random_dseq_gen(rng, d)
        shift = random_shifts(rng, T, d)
        B = rng.normal(0.0, math.sqrt(1.0 / 2.0), size=(T, 2))
        theta = dict(tau=np.zeros(T), gamma=1.0, eta=np.ones(d), b=None,
                     xi=np.full(T, 1e-3), B=B, zeta=np.full(T, 0.1))
        fits.append(Workload(f"fit{f}_{fam}_T{T}_d{d}", fam, T, d, m, 2, False, gen, shift,
                             theta, True, seed * 100000 + f, "corr_sines",
                             _corr_sine_params(rng, T, d), 1e-6, 0))
    return fits


CONFIGS = {1: config1, 2: config2, 3: config3, 5: config5}


def scaled(w: Workload, m: list, name_suffix: str = "") -> Workload:
    """Same family, T, d, kernel, seeds and hyperparameters; smaller sizes m."""
    m = [int(v) for v in m]
    if len(m) != w.T or any(m[i] < m[i + 1] for i in range(len(m) - 1)):
        raise ValueError("m must have T non-increasing entries")
    return dataclasses.replace(w, m=m, name=w.name + (name_suffix or f"_scaled{m}"))


def with_theta(w: Workload, **kw) -> Workload:
    th = dict(w.theta)
    th.update(kw)
    return dataclasses.replace(w, theta=th)


def adaptive_b(rng: np.random.Generator) -> np.ndarray:
    """Positive weights for the adaptive-smoothness DSI kernel."""
    return np.exp(rng.uniform(np.log(0.2), np.log(2.0), size=4))
