"""ctypes front-end of ``spectral_big.c`` (test infrastructure only).

The equal-size MLE loss of digital-net designs through the per-frequency
blocks of Theorem "Fast MTGP computations", the weights alpha = Ktilde^-1 r,
and the dense posterior-mean sum (Eq. MTGP_post_mean_cov), in plain C with
OpenMP threads, for sizes up to T = 8 tasks of 2^24 points.  See the C file
for the passages followed.

Pinned by tests/test_oracle_spectral_big.py against ``oracle.dense`` (loss,
means and posterior mean on small designs of every DSI order) and against
``oracle.points`` / ``workloads.target_values``.
"""
import ctypes
import os
import subprocess

import numpy as np

from .dense import task_cov

_HERE = os.path.dirname(os.path.abspath(__file__))
_BUILD = os.path.join(_HERE, "_build")
_SRC = os.path.join(_HERE, "spectral_big.c")
_LIB = None


def _lib_path():
    return os.path.join(_BUILD, "liboracle_spectral_big.so")


def build(force=False):
    """Compile the C oracle with gcc (-O2, OpenMP); returns the library path."""
    os.makedirs(_BUILD, exist_ok=True)
    path = _lib_path()
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", path + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(path + ".tmp", path)
    return path


def _load():
    global _LIB
    if _LIB is None:
        build()
        _LIB = ctypes.CDLL(_lib_path())
        for name in ("sb_points", "sb_mle_equal", "sb_mean", "sb_targets_corr_sines"):
            getattr(_LIB, name).restype = ctypes.c_int
    return _LIB


def _p(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def threads():
    """OpenMP threads the library will use (OMP_NUM_THREADS, else all cores)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env:
        return int(env)
    return len(os.sched_getaffinity(0))


def _check(w):
    if w.family != "dseq" or w.adaptive or len(set(w.m)) != 1:
        raise ValueError("spectral_big covers equal-size digital nets with a fixed-order DSI kernel")


def points(w, n):
    """Unshifted net points z_i, i < n, as uint32 [n][d]."""
    z = np.zeros((n, w.d), dtype=np.uint32)
    rc = _load().sb_points(_p(_u32(w.gen), ctypes.c_uint32), w.d, ctypes.c_int64(n),
                           _p(z, ctypes.c_uint32))
    assert rc == 0
    return z


def targets(w, rng):
    """Correlated-sine targets of the workload at its own points, with the
    noise drawn from rng per task as workloads.target_values draws it."""
    _check(w)
    if w.target not in ("corr_sines", "prior"):
        raise ValueError(w.target)
    n = 1 << w.m[0]
    noise = np.empty((w.T, n))
    for t in range(w.T):
        noise[t] = rng.normal(0.0, np.sqrt(w.noise_var), size=n)
    p = w.target_params
    y = np.empty((w.T, n))
    rc = _load().sb_targets_corr_sines(
        w.T, w.d, w.m[0], _p(_u32(w.gen), ctypes.c_uint32), _p(_u32(w.shift), ctypes.c_uint32),
        _p(_f64(p["freq"]), ctypes.c_double), _p(_f64(p["phase"]), ctypes.c_double),
        _p(_f64(p["rho"]), ctypes.c_double), _p(noise, ctypes.c_double), _p(y, ctypes.c_double))
    assert rc == 0
    return y.reshape(-1)


def mle(w, y, theta=None, profile=None, want_alpha=False):
    """quad, logdet, L, tau_hat (and alpha [T][n] if asked) for an equal-size
    digital-net workload; y task-major in radical-inverse order."""
    _check(w)
    theta = w.theta if theta is None else theta
    profile = w.profile_tau if profile is None else profile
    n = 1 << w.m[0]
    R = _f64(task_cov(theta))
    out3 = np.zeros(3)
    tau = np.zeros(w.T)
    alpha = np.zeros((w.T, n)) if want_alpha else None
    rc = _load().sb_mle_equal(
        w.T, w.d, w.m[0], _p(_u32(w.gen), ctypes.c_uint32), _p(_u32(w.shift), ctypes.c_uint32),
        w.kernel_order, ctypes.c_double(float(theta["gamma"])),
        _p(_f64(theta["eta"]), ctypes.c_double),
        _p(_f64(np.broadcast_to(theta["xi"], (w.T,))), ctypes.c_double), _p(R, ctypes.c_double),
        int(bool(profile)), _p(_f64(theta["tau"]), ctypes.c_double),
        _p(_f64(y), ctypes.c_double), _p(out3, ctypes.c_double), _p(tau, ctypes.c_double),
        _p(alpha, ctypes.c_double) if want_alpha else None)
    if rc != 0:
        raise RuntimeError(f"spectral_big.mle failed with code {rc}")
    res = dict(quad=out3[0], logdet=out3[1], L=out3[2], tau_hat=tau)
    if want_alpha:
        res["alpha"] = alpha
    return res


def posterior_mean(w, res, xs, theta=None):
    """mu(t, x) at test digits xs [M][d] from the weights of ``mle(...,
    want_alpha=True)``: the plain sum over every training point."""
    _check(w)
    theta = w.theta if theta is None else theta
    xs = _u32(xs)
    M = xs.shape[0]
    mean = np.zeros((M, w.T))
    rc = _load().sb_mean(
        w.T, w.d, w.m[0], _p(_u32(w.gen), ctypes.c_uint32), _p(_u32(w.shift), ctypes.c_uint32),
        w.kernel_order, ctypes.c_double(float(theta["gamma"])),
        _p(_f64(theta["eta"]), ctypes.c_double), _p(_f64(task_cov(theta)), ctypes.c_double),
        _p(_f64(res["tau_hat"]), ctypes.c_double), _p(_f64(res["alpha"]), ctypes.c_double),
        ctypes.c_int64(M), _p(xs, ctypes.c_uint32), _p(mean, ctypes.c_double))
    assert rc == 0
    return mean
