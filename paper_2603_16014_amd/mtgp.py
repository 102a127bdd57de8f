"""Python front-end of the C ABI (include/mtgp.h): device memory and streams
come from PyTorch, every computation runs in the HIP library.

Only argument marshalling lives here: shapes, dtypes, packing of the
hyperparameter vector in the ABI's order, and the current torch stream.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib

DSEQ, LAT = 0, 1
FP64, MIXED, F32 = 0, 1, 2
FAMILIES = {"dseq": DSEQ, "lat": LAT, DSEQ: DSEQ, LAT: LAT}
PRECISIONS = {"fp64": FP64, "mixed": MIXED, "f32": F32, FP64: FP64, MIXED: MIXED, F32: F32}
ELIMINATIONS = {"sparse": 0, "alg1": 1, 0: 0, 1: 1}  # nested unequal sizes
DEFAULT_SCHEDULE = (12, 0, 73728)  # the library's default transform schedule
LOG_KEYS = ("gamma", "eta", "b", "xi", "zeta")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _need_cuda(t: torch.Tensor, dtype, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def theta_keys(adaptive: bool):
    return ["tau", "gamma", "eta"] + (["b"] if adaptive else []) + ["xi", "B", "zeta"]


class Plan:
    """A fast-MTGP design (points + kernel family) bound to the current device."""

    def __init__(self, family, m, gen, shift, kernel_order=2, adaptive=False, rank_s=1,
                 profile_tau=True, precision="fp64", schedule=None, elimination=None):
        self.lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the MTGP library has no CPU path")
        self.family = FAMILIES[family]
        self.m = [int(v) for v in m]
        self.T = len(self.m)
        gen = np.ascontiguousarray(gen, dtype=np.uint32)
        shift = np.ascontiguousarray(shift, dtype=np.uint32)
        self.d = int(gen.shape[0])
        self.adaptive = bool(adaptive)
        self.rank_s = int(rank_s)
        self.profile_tau = bool(profile_tau)
        self.precision = PRECISIONS[precision]
        self._m = np.ascontiguousarray(self.m, dtype=np.int32)
        self._gen = gen.reshape(-1)
        self._shift = shift.reshape(-1)
        des = _lib.Design(self.T, self.d, self.family,
                          self._m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          self._gen.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                          self._shift.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                          int(kernel_order), int(self.adaptive), self.rank_s,
                          int(self.profile_tau))
        h = ctypes.c_void_p()
        _lib.check(self.lib.mtgp_plan_create(ctypes.byref(des), self.precision, ctypes.byref(h)),
                   "mtgp_plan_create")
        self.h = h
        self.schedule = DEFAULT_SCHEDULE
        if schedule is not None:
            a, b, tile = schedule
            _lib.check(self.lib.mtgp_plan_set_schedule(h, int(a), int(b), int(tile)),
                       "mtgp_plan_set_schedule")
            self.schedule = (int(a), int(b), int(tile))
        self.overlap = 4
        if elimination is not None:
            _lib.check(self.lib.mtgp_plan_set_elimination(h, ELIMINATIONS[elimination]),
                       "mtgp_plan_set_elimination")
        self.theta_size = int(self.lib.mtgp_theta_size(h))
        self.N = int(self.lib.mtgp_num_points(h))
        self.ncol = int(self.lib.mtgp_num_columns(h))
        self.ws = torch.empty(int(self.lib.mtgp_workspace_bytes(h)), dtype=torch.uint8,
                              device="cuda")
        self.n = [1 << v for v in self.m]

    @classmethod
    def from_workload(cls, w, precision="fp64", profile_tau=None, schedule=None,
                      elimination=None):
        return cls(w.family, w.m, w.gen, w.shift, w.kernel_order, w.adaptive, w.rank_s,
                   w.profile_tau if profile_tau is None else profile_tau, precision, schedule,
                   elimination)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.mtgp_plan_destroy(h)
            self.h = None

    # ----------------------------------------------------------------- theta
    def pack_theta(self, theta: dict, device="cuda") -> torch.Tensor:
        parts = []
        for k in theta_keys(self.adaptive):
            v = np.atleast_1d(np.asarray(theta[k], dtype=np.float64)).ravel()
            parts.append(np.log(v) if k in LOG_KEYS else v)
        vec = np.concatenate(parts)
        if vec.size != self.theta_size:
            raise ValueError(f"theta has {vec.size} entries, plan expects {self.theta_size}")
        return torch.from_numpy(vec).to(device)

    def unpack(self, vec) -> dict:
        """Splits a packed vector (theta or gradient) into named numpy pieces."""
        v = vec.detach().cpu().numpy() if isinstance(vec, torch.Tensor) else np.asarray(vec)
        out, i = {}, 0
        sizes = {"tau": self.T, "gamma": 1, "eta": self.d, "b": 4, "xi": self.T,
                 "B": self.T * self.rank_s, "zeta": self.T}
        for k in theta_keys(self.adaptive):
            piece = v[i:i + sizes[k]]
            out[k] = float(piece[0]) if k == "gamma" else (
                piece.reshape(self.T, self.rank_s) if k == "B" else piece.copy())
            i += sizes[k]
        return out

    # ---------------------------------------------------------------- points
    def gen_points(self, task: int, first: int, count: int) -> torch.Tensor:
        out = torch.empty((count, self.d), dtype=torch.int32, device="cuda")
        _lib.check(self.lib.mtgp_gen_points(self.h, task, first, count, _ptr(out), _stream()),
                   "mtgp_gen_points")
        return out

    def column_info(self, c):
        m, off, t, u = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _lib.check(self.lib.mtgp_column_info(self.h, c, ctypes.byref(m), ctypes.byref(off),
                                             ctypes.byref(t), ctypes.byref(u)), "mtgp_column_info")
        return m.value, off.value, t.value, u.value

    def kernel_cols(self, theta: torch.Tensor) -> torch.Tensor:
        _need_cuda(theta, torch.float64, "theta")
        total = sum(1 << self.column_info(c)[0] for c in range(self.ncol))
        dt = torch.float32 if self.precision == F32 else torch.float64
        out = torch.empty(total, dtype=dt, device="cuda")
        _lib.check(self.lib.mtgp_kernel_cols(self.h, _ptr(theta), _ptr(out), _ptr(self.ws),
                                             _stream()), "mtgp_kernel_cols")
        return out

    # ------------------------------------------------------------------ loss
    def set_data(self, y: torch.Tensor):
        _need_cuda(y, torch.float64, "y")
        if y.numel() != self.N:
            raise ValueError(f"y has {y.numel()} entries, plan has N={self.N}")
        _lib.check(self.lib.mtgp_set_data(self.h, _ptr(y), _ptr(self.ws), _stream()),
                   "mtgp_set_data")
        self._y = y

    def nll(self, theta: torch.Tensor, out3=None, tau_hat=None):
        _need_cuda(theta, torch.float64, "theta")
        out3 = torch.empty(3, dtype=torch.float64, device="cuda") if out3 is None else out3
        tau_hat = torch.empty(self.T, dtype=torch.float64, device="cuda") if tau_hat is None else tau_hat
        _lib.check(self.lib.mtgp_nll(self.h, _ptr(theta), _ptr(out3), _ptr(tau_hat),
                                     _ptr(self.ws), _stream()), "mtgp_nll")
        return out3, tau_hat

    def nll_grad(self, theta: torch.Tensor, out3=None, grad=None, tau_hat=None):
        _need_cuda(theta, torch.float64, "theta")
        out3 = torch.empty(3, dtype=torch.float64, device="cuda") if out3 is None else out3
        grad = torch.empty(self.theta_size, dtype=torch.float64, device="cuda") if grad is None else grad
        tau_hat = torch.empty(self.T, dtype=torch.float64, device="cuda") if tau_hat is None else tau_hat
        _lib.check(self.lib.mtgp_nll_grad(self.h, _ptr(theta), _ptr(out3), _ptr(grad),
                                          _ptr(tau_hat), _ptr(self.ws), _stream()),
                   "mtgp_nll_grad")
        return out3, grad, tau_hat

    def negloglik(self, out3: torch.Tensor) -> torch.Tensor:
        """NLL = L/2 + N/2 log(2 pi) from out3 = (quad, logdet, L)."""
        return 0.5 * out3[2] + 0.5 * self.N * math.log(2 * math.pi)

    def predict(self, theta: torch.Tensor, xs: torch.Tensor) -> torch.Tensor:
        _need_cuda(theta, torch.float64, "theta")
        _need_cuda(xs, torch.int32, "xs (uint32 digits stored as int32)")
        M = xs.shape[0]
        mean = torch.empty((M, self.T), dtype=torch.float64, device="cuda")
        _lib.check(self.lib.mtgp_predict(self.h, _ptr(theta), _ptr(xs), M, _ptr(mean),
                                         _ptr(self.ws), _stream()), "mtgp_predict")
        return mean

    def predict_var(self, theta: torch.Tensor, xs: torch.Tensor, batch: int = 64) -> torch.Tensor:
        """Posterior variance var[M][T] of the latent f at M test digits."""
        _need_cuda(theta, torch.float64, "theta")
        _need_cuda(xs, torch.int32, "xs (uint32 digits stored as int32)")
        M = xs.shape[0]
        batch = max(1, min(int(batch), max(M, 1)))
        nbytes = int(self.lib.mtgp_predict_var_scratch_bytes(self.h, batch))
        scratch = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
        var = torch.empty((M, self.T), dtype=torch.float64, device="cuda")
        _lib.check(self.lib.mtgp_predict_var(self.h, _ptr(theta), _ptr(xs), M, batch, _ptr(var),
                                             _ptr(self.ws), _ptr(scratch), _stream()),
                   "mtgp_predict_var")
        return var

    def predict_net(self, theta: torch.Tensor, shift_star, m_star: int) -> torch.Tensor:
        _need_cuda(theta, torch.float64, "theta")
        sh = np.ascontiguousarray(shift_star, dtype=np.uint32)
        nbytes = int(self.lib.mtgp_predict_net_scratch_bytes(self.h, m_star))
        scratch = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
        mean = torch.empty(((1 << m_star), self.T), dtype=torch.float64, device="cuda")
        _lib.check(self.lib.mtgp_predict_net(
            self.h, _ptr(theta), sh.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), m_star,
            _ptr(mean), _ptr(self.ws), _ptr(scratch), _stream()), "mtgp_predict_net")
        return mean

    def set_fused_occupancy(self, blocks_per_cu: int):
        """Cap on workgroups per CU of the fused digital-net kernels (0 = none)."""
        _lib.check(self.lib.mtgp_plan_set_fused_occupancy(self.h, int(blocks_per_cu)),
                   "mtgp_plan_set_fused_occupancy")
        self.fused_occupancy = int(blocks_per_cu)

    def set_overlap(self, chunks: int):
        """Chunks of the overlapped digital-net passes (1 = no overlap)."""
        _lib.check(self.lib.mtgp_plan_set_overlap(self.h, int(chunks)), "mtgp_plan_set_overlap")
        self.overlap = int(chunks)

    def set_schedule(self, pass_a_bits: int, pass_b_bits: int, pass_b_tile_bytes: int):
        """Transform schedule of the digital-net passes (mtgp_plan_set_schedule).
        The workspace grows if the new schedule needs more; the data transform
        of set_data is then formed again."""
        _lib.check(self.lib.mtgp_plan_set_schedule(self.h, int(pass_a_bits), int(pass_b_bits),
                                                   int(pass_b_tile_bytes)),
                   "mtgp_plan_set_schedule")
        self.schedule = (int(pass_a_bits), int(pass_b_bits), int(pass_b_tile_bytes))
        need = int(self.lib.mtgp_workspace_bytes(self.h))
        if need > self.ws.numel():
            self.ws = torch.empty(need, dtype=torch.uint8, device="cuda")
            if getattr(self, "_y", None) is not None:
                self.set_data(self._y)

    def gcv(self, theta: torch.Tensor, grad=True):
        """GCV loss: (out3 = (q, s, L_GCV), gradient or None, tau_hat)."""
        _need_cuda(theta, torch.float64, "theta")
        out3 = torch.empty(3, dtype=torch.float64, device="cuda")
        g = torch.empty(self.theta_size, dtype=torch.float64, device="cuda") if grad else None
        tau = torch.empty(self.T, dtype=torch.float64, device="cuda")
        _lib.check(self.lib.mtgp_gcv(self.h, _ptr(theta), _ptr(out3),
                                     _ptr(g) if g is not None else None, _ptr(tau),
                                     _ptr(self.ws), _stream()), "mtgp_gcv")
        return out3, g, tau

    def cubature(self, theta: torch.Tensor):
        """Bayesian cubature: (mu_hat [T], Sigma [T][T]) of the task integrals."""
        _need_cuda(theta, torch.float64, "theta")
        mu = torch.empty(self.T, dtype=torch.float64, device="cuda")
        Sigma = torch.empty((self.T, self.T), dtype=torch.float64, device="cuda")
        _lib.check(self.lib.mtgp_cubature(self.h, _ptr(theta), _ptr(mu), _ptr(Sigma),
                                          _ptr(self.ws), _stream()), "mtgp_cubature")
        return mu, Sigma

    def enable_timing(self, on=True):
        _lib.check(self.lib.mtgp_plan_enable_timing(self.h, int(bool(on))), "mtgp_plan_enable_timing")

    def phase_times(self) -> dict:
        """Mean per-phase milliseconds over the evaluations recorded since the
        previous call (at most the 64 most recent; waits for the last one)."""
        buf = (ctypes.c_double * 16)()
        k = ctypes.c_int32()
        _lib.check(self.lib.mtgp_phase_times(self.h, buf, 16, ctypes.byref(k)), "mtgp_phase_times")
        return {self.lib.mtgp_phase_name(i).decode(): buf[i] for i in range(k.value)}

    def status(self):
        """(code, bad_index) of the last evaluation; synchronises the device."""
        torch.cuda.synchronize()
        bad = ctypes.c_int64()
        code = self.lib.mtgp_status(self.h, _ptr(self.ws), ctypes.byref(bad))
        return code, bad.value


def fwht(x: torch.Tensor, log2n: int) -> torch.Tensor:
    """In-place unnormalised Walsh-Hadamard transform of contiguous rows."""
    if x.dtype not in (torch.float64, torch.float32):
        raise TypeError("fwht needs float32 or float64")
    _need_cuda(x, x.dtype, "x")
    batch = x.numel() >> log2n
    dt = 0 if x.dtype == torch.float64 else 1
    _lib.check(_lib.load().mtgp_fwht(_ptr(x), batch, log2n, dt, _stream()), "mtgp_fwht")
    return x


def fft(x: torch.Tensor, log2n: int, bitrev_input=False) -> torch.Tensor:
    """Unnormalised forward DFT of real rows -> complex (interleaved) output."""
    if x.dtype not in (torch.float64, torch.float32):
        raise TypeError("fft needs float32 or float64")
    _need_cuda(x, x.dtype, "x")
    batch = x.numel() >> log2n
    X = torch.empty(2 * x.numel(), dtype=x.dtype, device="cuda")
    scratch = torch.empty(2 * x.numel() if log2n > 12 else 1, dtype=x.dtype, device="cuda")
    dt = 0 if x.dtype == torch.float64 else 1
    _lib.check(_lib.load().mtgp_fft(_ptr(x), _ptr(X), _ptr(scratch), batch, log2n, dt,
                                    int(bool(bitrev_input)), _stream()), "mtgp_fft")
    return torch.view_as_complex(X.view(-1, 2)).view(batch, 1 << log2n)


def digits_as_uint32(t: torch.Tensor) -> np.ndarray:
    """Device int32 digits -> host uint32 array (bit-exact reinterpretation)."""
    return t.cpu().numpy().view(np.uint32)


def digits_to_device(u: np.ndarray) -> torch.Tensor:
    """Host uint32 digits -> device int32 tensor holding the same bits."""
    return torch.from_numpy(np.ascontiguousarray(u, dtype=np.uint32).view(np.int32)).cuda()


def adam_step(theta: torch.Tensor, grad: torch.Tensor, m1: torch.Tensor, m2: torch.Tensor,
              step: torch.Tensor, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, frozen=None):
    """One on-device Adam update of theta in place (mtgp_adam_step)."""
    lib = _lib.load()
    for name, t in (("theta", theta), ("grad", grad), ("m1", m1), ("m2", m2)):
        _need_cuda(t, torch.float64, name)
    _need_cuda(step, torch.int64, "step")
    if frozen is not None:
        _need_cuda(frozen, torch.uint8, "frozen")
    _lib.check(lib.mtgp_adam_step(_ptr(theta), _ptr(grad), _ptr(m1), _ptr(m2), theta.numel(),
                                  float(lr), float(beta1), float(beta2), float(eps), _ptr(step),
                                  _ptr(frozen) if frozen is not None else None, _stream()),
               "mtgp_adam_step")


def nll_grad_batched(plans, thetas, out3s, grads):
    """mtgp_nll_grad for every fit, enqueued on the current stream in one call."""
    lib = _lib.load()
    k = len(plans)
    if not (len(thetas) == len(out3s) == len(grads) == k):
        raise ValueError("plans, thetas, out3s and grads must have the same length")
    arr = ctypes.c_void_p * max(k, 1)
    P = arr(*[p.h.value for p in plans])
    Th = arr(*[t.data_ptr() for t in thetas])
    O = arr(*[o.data_ptr() for o in out3s])
    G = arr(*[g.data_ptr() for g in grads])
    W = arr(*[p.ws.data_ptr() for p in plans])
    _lib.check(lib.mtgp_nll_grad_batched(k, P, Th, O, G, W, _stream()), "mtgp_nll_grad_batched")


class Batch:
    """Many independent fits with one launch per phase (mtgp_batch_*).

    Holds the plans, the per-fit buffers it was created with (theta, out3,
    grad and, with ``adam=True``, the Adam moments and step counters) and the
    batch workspace; ``nll_grad()`` evaluates loss + gradient of every fit,
    ``adam_step()`` updates every theta.  Both enqueue a fixed sequence of
    launches on the current stream, so they can be captured in a graph."""

    def __init__(self, plans, thetas, out3s=None, grads=None, adam=False, frozen=None):
        self.lib = _lib.load()
        k = len(plans)
        self.plans = list(plans)
        self.thetas = [t.contiguous() for t in thetas]
        for t in self.thetas:
            _need_cuda(t, torch.float64, "theta")
        self.out3s = out3s if out3s is not None else [
            torch.zeros(3, dtype=torch.float64, device="cuda") for _ in range(k)]
        self.grads = grads if grads is not None else [
            torch.zeros_like(t) for t in self.thetas]
        arr = ctypes.c_void_p * max(k, 1)
        P = arr(*[p.h.value for p in self.plans])
        nbytes = int(self.lib.mtgp_batch_workspace_bytes(k, P))
        if k > 0 and nbytes == 0:
            raise _lib.MTGPError(-5, "mtgp_batch_workspace_bytes")
        self.bws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")
        W = arr(*[p.ws.data_ptr() for p in self.plans])
        Th = arr(*[t.data_ptr() for t in self.thetas])
        O = arr(*[o.data_ptr() for o in self.out3s])
        G = arr(*[g.data_ptr() for g in self.grads])
        M1 = M2 = S = F = None
        if adam:
            self.m1 = [torch.zeros_like(t) for t in self.thetas]
            self.m2 = [torch.zeros_like(t) for t in self.thetas]
            self.steps = [torch.zeros(1, dtype=torch.int64, device="cuda") for _ in range(k)]
            M1 = arr(*[t.data_ptr() for t in self.m1])
            M2 = arr(*[t.data_ptr() for t in self.m2])
            S = arr(*[t.data_ptr() for t in self.steps])
            if frozen is not None:
                self.frozen = [torch.as_tensor(f, dtype=torch.uint8).cuda().contiguous()
                               for f in frozen]
                F = arr(*[f.data_ptr() for f in self.frozen])
        h = ctypes.c_void_p()
        _lib.check(self.lib.mtgp_batch_create(k, P, W, Th, O, G, M1, M2, S, F,
                                              ctypes.c_void_p(self.bws.data_ptr()),
                                              ctypes.byref(h)), "mtgp_batch_create")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.mtgp_batch_destroy(self.h)
            self.h = None

    def nll_grad(self):
        _lib.check(self.lib.mtgp_batch_nll_grad(self.h, _stream()), "mtgp_batch_nll_grad")

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        _lib.check(self.lib.mtgp_batch_adam_step(self.h, float(lr), float(beta1), float(beta2),
                                                 float(eps), _stream()), "mtgp_batch_adam_step")

    def reset_adam(self):
        for t in self.m1 + self.m2 + self.steps:
            t.zero_()
