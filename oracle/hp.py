"""ctypes front-end of the extended-precision dense twin (test infrastructure only).

``build()`` compiles ``hp_dense.c`` twice with gcc: ``real = long double``
(64-bit significand) and ``real = __float128`` (113-bit significand, via
libquadmath).  ``mtgp(w, y, ...)`` returns quad, logdet, L, tau_hat and the
posterior mean at given test digits, computed by the dense definitions in
that precision (see the C file header for the passages followed).
``spectral_nets(w, y, ...)`` returns quad, logdet, L and tau_hat of a
digital-net design of nested sizes by the spectral route (Walsh transforms
and residue-class blocks) in long double, for sizes the dense twin cannot
factor.
"""
import ctypes
import os
import subprocess

import numpy as np

from . import points as pts

_HERE = os.path.dirname(os.path.abspath(__file__))
_BUILD = os.path.join(_HERE, "_build")
_SRC = os.path.join(_HERE, "hp_dense.c")
_LIBS = {}


def _lib_path(kind):
    return os.path.join(_BUILD, f"liboracle_hp_{kind}.so")


def build(force=False):
    """Compile both precisions; returns the two library paths."""
    os.makedirs(_BUILD, exist_ok=True)
    out = []
    for kind, extra in (("ld", []), ("quad", ["-DORACLE_QUAD", "-lquadmath"])):
        path = _lib_path(kind)
        if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", path + ".tmp", _SRC,
                   "-lm"] + extra
            subprocess.run(cmd, check=True)
            os.replace(path + ".tmp", path)
        out.append(path)
    return out


def _load(kind, name="hp_mtgp"):
    key = (kind, name)
    if key not in _LIBS:
        build()
        lib = ctypes.CDLL(_lib_path(kind))
        fn = getattr(lib, f"{name}_{kind}")
        fn.restype = ctypes.c_int
        _LIBS[key] = fn
    return _LIBS[key]


def _p(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def mtgp(w, y, theta=None, Xs=None, profile=None, kind="ld", X=None):
    """Dense MLE pieces and posterior mean in extended precision."""
    theta = w.theta if theta is None else theta
    profile = w.profile_tau if profile is None else profile
    X = pts.task_points(w) if X is None else X
    n = np.array([x.shape[0] for x in X], dtype=np.int32)
    Xall = np.ascontiguousarray(np.concatenate(X, axis=0), dtype=np.uint32)
    y = np.ascontiguousarray(y, dtype=np.float64)
    B = np.ascontiguousarray(theta["B"], dtype=np.float64)
    s = B.shape[1]
    b = np.ascontiguousarray(theta["b"] if theta.get("b") is not None else np.zeros(4),
                             dtype=np.float64)
    eta = np.ascontiguousarray(theta["eta"], dtype=np.float64)
    xi = np.ascontiguousarray(theta["xi"], dtype=np.float64)
    zeta = np.ascontiguousarray(theta["zeta"], dtype=np.float64)
    tau = np.ascontiguousarray(theta["tau"], dtype=np.float64)
    M = 0 if Xs is None else int(Xs.shape[0])
    Xs_c = np.ascontiguousarray(Xs if Xs is not None else np.zeros((1, w.d)), dtype=np.uint32)
    mean = np.zeros((max(M, 1), w.T))
    out = np.zeros(3)
    tau_hat = np.zeros(w.T)
    fam = 0 if w.family == "dseq" else 1
    rc = _load(kind)(fam, w.T, w.d, _p(n, ctypes.c_int), _p(Xall, ctypes.c_uint32),
                     w.kernel_order, int(bool(w.adaptive)), _p(b, ctypes.c_double),
                     ctypes.c_double(float(theta["gamma"])), _p(eta, ctypes.c_double),
                     _p(xi, ctypes.c_double), s, _p(B, ctypes.c_double),
                     _p(zeta, ctypes.c_double), int(bool(profile)), _p(tau, ctypes.c_double),
                     _p(y, ctypes.c_double), _p(out, ctypes.c_double),
                     _p(tau_hat, ctypes.c_double), M, _p(Xs_c, ctypes.c_uint32),
                     _p(mean, ctypes.c_double))
    if rc != 0:
        raise RuntimeError(f"extended-precision oracle failed with code {rc}")
    return dict(quad=out[0], logdet=out[1], L=out[2], tau_hat=tau_hat,
                mean=mean[:M] if M else None)


def spectral_nets(w, y, theta=None, profile=None, kind="ld"):
    """quad, logdet, L and tau_hat of a digital-net design (any nested sizes)
    by the spectral route in extended precision; y in the dense oracle's
    point order."""
    if w.family != "dseq":
        raise ValueError("the extended-precision spectral route covers digital nets")
    theta = w.theta if theta is None else theta
    profile = w.profile_tau if profile is None else profile
    nmax = 1 << max(w.m)
    z = np.ascontiguousarray(pts.dseq_unshifted(w.gen, nmax), dtype=np.uint32)
    shift = np.ascontiguousarray(np.asarray(w.shift, dtype=np.uint32).reshape(w.T, w.d))
    m = np.asarray(w.m, dtype=np.int32)
    y = np.ascontiguousarray(y, dtype=np.float64)
    B = np.ascontiguousarray(theta["B"], dtype=np.float64)
    b = np.ascontiguousarray(theta["b"] if theta.get("b") is not None else np.zeros(4),
                             dtype=np.float64)
    eta = np.ascontiguousarray(theta["eta"], dtype=np.float64)
    xi = np.ascontiguousarray(theta["xi"], dtype=np.float64)
    zeta = np.ascontiguousarray(theta["zeta"], dtype=np.float64)
    tau = np.ascontiguousarray(theta["tau"], dtype=np.float64)
    out = np.zeros(3)
    tau_hat = np.zeros(w.T)
    rc = _load(kind, "hp_spectral_nets")(
        w.T, w.d, _p(m, ctypes.c_int), _p(z, ctypes.c_uint32), _p(shift, ctypes.c_uint32),
        w.kernel_order, int(bool(w.adaptive)), _p(b, ctypes.c_double),
        ctypes.c_double(float(theta["gamma"])), _p(eta, ctypes.c_double), _p(xi, ctypes.c_double),
        B.shape[1], _p(B, ctypes.c_double), _p(zeta, ctypes.c_double), int(bool(profile)),
        _p(tau, ctypes.c_double), _p(y, ctypes.c_double), _p(out, ctypes.c_double),
        _p(tau_hat, ctypes.c_double))
    if rc != 0:
        raise RuntimeError(f"extended-precision spectral oracle failed with code {rc}")
    return dict(quad=out[0], logdet=out[1], L=out[2], tau_hat=tau_hat)
