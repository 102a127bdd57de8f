"""Hyperparameter training on the device: autograd, Adam and HIP graphs.

* ``MTGPLoss`` is a ``torch.autograd.Function`` whose forward is one
  ``mtgp_nll_grad`` call (loss L = quad + log det of the paper's MLE loss,
  Section "Multitask Setting") and whose backward returns the exact adjoint
  gradient computed in that same call, so ``loss.backward()`` costs nothing
  extra and the gradient never leaves the GPU.
* ``DeviceAdam`` keeps the Adam moments and step counter in device memory and
  updates theta with one library kernel (``mtgp_adam_step``), so a training
  step is a fixed sequence of kernel launches.
* ``fit`` runs K steps of one fit; with ``graph=True`` a single step (loss +
  gradient + Adam) is captured once in a HIP graph and replayed.
* ``BatchedFits`` does the same for many independent fits at once: one step
  of every fit is captured into one graph, fits spread over several capture
  streams so that independent fits run concurrently on replay.

Nothing here computes on the host: the library kernels do all arithmetic.
"""
from __future__ import annotations

import time

import torch

from . import mtgp


class MTGPLoss(torch.autograd.Function):
    """L(theta) = quad + logdet with the exact adjoint gradient as backward."""

    @staticmethod
    def forward(ctx, theta, plan):
        out3 = torch.empty(3, dtype=torch.float64, device=theta.device)
        grad = torch.empty_like(theta)
        plan.nll_grad(theta.detach().contiguous(), out3, grad)
        ctx.save_for_backward(grad)
        return out3[2].clone()

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g * grad, None


def loss(plan, theta: torch.Tensor) -> torch.Tensor:
    """Differentiable MLE loss L = quad + logdet (0-dim FP64 tensor)."""
    return MTGPLoss.apply(theta, plan)


def negloglik(plan, theta: torch.Tensor) -> torch.Tensor:
    """Differentiable negative log marginal likelihood L/2 + N/2 log(2 pi)."""
    import math
    return 0.5 * loss(plan, theta) + 0.5 * plan.N * math.log(2 * math.pi)


class DeviceAdam:
    """Adam on a packed FP64 theta; state lives on the device."""

    def __init__(self, n: int, lr=0.05, betas=(0.9, 0.999), eps=1e-8, frozen=None,
                 device="cuda"):
        self.lr, self.betas, self.eps = float(lr), betas, float(eps)
        self.m1 = torch.zeros(n, dtype=torch.float64, device=device)
        self.m2 = torch.zeros(n, dtype=torch.float64, device=device)
        self.count = torch.zeros(1, dtype=torch.int64, device=device)
        self.frozen = None
        if frozen is not None:
            self.frozen = torch.as_tensor(frozen, dtype=torch.uint8).to(device).contiguous()

    def reset(self):
        self.m1.zero_()
        self.m2.zero_()
        self.count.zero_()

    def step(self, theta: torch.Tensor, grad: torch.Tensor):
        mtgp.adam_step(theta, grad, self.m1, self.m2, self.count, self.lr, self.betas[0],
                       self.betas[1], self.eps, self.frozen)


def frozen_mask(plan, tau=True):
    """Entries of theta Adam leaves unchanged: the means when they are
    profiled (their gradient is identically zero) or when fixed by choice."""
    mask = torch.zeros(plan.theta_size, dtype=torch.uint8)
    if tau:
        mask[:plan.T] = 1
    return mask


class Fit:
    """State of one fit: theta, gradient, loss, optimiser."""

    def __init__(self, plan, theta0: torch.Tensor, lr=0.05, frozen=None):
        self.plan = plan
        self.theta = theta0.detach().clone().contiguous()
        self.grad = torch.zeros_like(self.theta)
        self.out3 = torch.zeros(3, dtype=torch.float64, device=self.theta.device)
        self.opt = DeviceAdam(self.theta.numel(), lr=lr, frozen=frozen)

    def step(self):
        self.plan.nll_grad(self.theta, self.out3, self.grad)
        self.opt.step(self.theta, self.grad)


def _capture(steps_fn, streams):
    """Captures steps_fn(streams) into a HIP graph; side streams fork from and
    join back into the capture stream."""
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        main = torch.cuda.current_stream()
        for s in streams:
            s.wait_stream(main)
        steps_fn(streams)
        for s in streams:
            main.wait_stream(s)
    return g


def fit(plan, theta0: torch.Tensor, steps: int, lr=0.05, graph=True, frozen=None,
        record=True):
    """K Adam steps on L(theta); returns (theta, losses [K] on the device, Fit).

    The loss entry k is L at the theta the k-th step started from.  With
    graph=True one step is captured once and replayed K times."""
    f = Fit(plan, theta0, lr=lr, frozen=frozen)
    hist = torch.zeros(steps, dtype=torch.float64, device=f.theta.device)
    if graph and steps > 0:
        # warm the library and the allocator outside capture, then restore
        f.step()
        torch.cuda.synchronize()
        f.theta.copy_(theta0)
        f.opt.reset()
        g = _capture(lambda ss: f.step(), [])
        for k in range(steps):
            g.replay()
            if record:
                hist[k].copy_(f.out3[2])
    else:
        for k in range(steps):
            f.step()
            if record:
                hist[k].copy_(f.out3[2])
    return f.theta, hist, f


class BatchedFits:
    """Many independent fits advanced together, one captured graph per step.

    Fits are dealt round-robin to ``nstreams`` capture streams: within a
    stream they run in order, across streams concurrently."""

    def __init__(self, plans, thetas, lr=0.05, frozen=None, nstreams=8):
        self.fits = [Fit(p, t, lr=lr, frozen=(frozen[i] if frozen is not None else None))
                     for i, (p, t) in enumerate(zip(plans, thetas))]
        self.theta0 = [t.detach().clone() for t in thetas]
        self.nstreams = max(1, int(nstreams))
        self.streams = [torch.cuda.Stream() for _ in range(self.nstreams)]
        self.graph = None

    def _enqueue(self, streams):
        for i, f in enumerate(self.fits):
            with torch.cuda.stream(streams[i % len(streams)]):
                f.step()

    def capture(self):
        for f in self.fits:
            f.step()
        torch.cuda.synchronize()
        self.reset()
        self.graph = _capture(self._enqueue, self.streams)

    def reset(self):
        for f, t0 in zip(self.fits, self.theta0):
            f.theta.copy_(t0)
            f.opt.reset()

    def run(self, steps: int):
        """Replays the graph `steps` times; returns per-step milliseconds."""
        if self.graph is None:
            self.capture()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        st = torch.cuda.current_stream()
        ev[0].record(st)
        for k in range(steps):
            self.graph.replay()
            ev[k + 1].record(st)
        torch.cuda.synchronize()
        return [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]

    def run_eager(self, steps: int):
        """The same steps as a Python loop of single fits on one stream (no
        graph); returns per-step milliseconds (host clock, synchronised)."""
        out = []
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for f in self.fits:
                f.step()
            torch.cuda.synchronize()
            out.append((time.perf_counter() - t0) * 1e3)
        return out


class PersistentBatchedFits:
    """Many independent fits advanced by the library's many-fit launches
    (``mtgp.Batch``): one step of every fit is one launch per phase (loss
    and gradient of all fits, then Adam of all fits), captured once in a
    graph and replayed.  Plans need sizes <= 2^14 per task and FP64 or mixed
    precision."""

    def __init__(self, plans, thetas, lr=0.05, frozen=None):
        self.lr = float(lr)
        self.theta0 = [t.detach().clone().contiguous() for t in thetas]
        if frozen is None:
            frozen = [frozen_mask(p).numpy() for p in plans]
        self.batch = mtgp.Batch(plans, [t.clone() for t in self.theta0], adam=True, frozen=frozen)
        self.graph = None

    @property
    def thetas(self):
        return self.batch.thetas

    def step(self):
        self.batch.nll_grad()
        self.batch.adam_step(self.lr)

    def reset(self):
        for t, t0 in zip(self.batch.thetas, self.theta0):
            t.copy_(t0)
        self.batch.reset_adam()

    def capture(self):
        self.step()
        torch.cuda.synchronize()
        self.reset()
        torch.cuda.synchronize()
        self.graph = _capture(lambda ss: self.step(), [])

    def run(self, steps: int):
        """Replays the graph `steps` times; returns per-step milliseconds."""
        if self.graph is None:
            self.capture()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        st = torch.cuda.current_stream()
        ev[0].record(st)
        for k in range(steps):
            self.graph.replay()
            ev[k + 1].record(st)
        torch.cuda.synchronize()
        return [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
