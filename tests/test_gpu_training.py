"""GPU tests of the training layer: autograd wrapper, on-device Adam, HIP-graph
capture of training steps (single and batched fits) and the multi-fit entry
point.  Everything is checked against the library's eager calls or a plain
PyTorch CPU reference of the same optimiser."""
import numpy as np
import pytest
import torch

from _designs import tiny
from _gpu_common import say

pytestmark = pytest.mark.gpu


def _plan(w, precision="fp64"):
    from oracle import dense, points
    from paper_2603_16014_amd import mtgp
    plan = mtgp.Plan.from_workload(w, precision)
    X = points.task_points(w)
    y = dense.targets(w, np.random.default_rng(w.seed + 1000), X)
    plan.set_data(torch.from_numpy(np.ascontiguousarray(y)).cuda())
    return plan, plan.pack_theta(w.theta)


DESIGNS = [("dseq", 3, [6, 6, 6], 3), ("lat", 2, [6, 6], 2), ("dseq", 3, [7, 5, 4], 2),
           ("lat", 3, [6, 5, 5], 3)]


@pytest.mark.parametrize("fam,T,m,d", DESIGNS)
def test_autograd_forward_backward(fam, T, m, d):
    from paper_2603_16014_amd import training
    say("autograd", fam, T, m, d)
    w = tiny(fam, T, m, d, seed=3)
    plan, theta = _plan(w)
    out3, grad, _ = plan.nll_grad(theta)
    th = theta.clone().requires_grad_(True)
    L = training.loss(plan, th)
    L.backward()
    torch.cuda.synchronize()
    assert float(L.detach()) == float(out3[2])
    assert torch.equal(th.grad, grad)
    # chain rule through a torch expression: theta = a * phi
    phi = (theta / 2.0).clone().requires_grad_(True)
    L2 = training.negloglik(plan, 2.0 * phi)
    L2.backward()
    assert torch.allclose(phi.grad, grad, rtol=1e-14, atol=0)  # d(L/2)/dphi = grad


def test_device_adam_matches_torch_adam():
    from paper_2603_16014_amd import training
    say("adam vs torch.optim.Adam")
    rng = np.random.default_rng(0)
    n = 37
    theta0 = rng.normal(size=n)
    grads = [rng.normal(size=n) * 10.0 ** rng.uniform(-3, 2) for _ in range(25)]
    frozen = np.zeros(n, dtype=np.uint8)
    frozen[:3] = 1
    th = torch.tensor(theta0, dtype=torch.float64, device="cuda")
    opt = training.DeviceAdam(n, lr=0.05, frozen=frozen)
    ref = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    ropt = torch.optim.Adam([ref], lr=0.05, betas=(0.9, 0.999), eps=1e-8)
    for g in grads:
        gd = torch.tensor(g, dtype=torch.float64, device="cuda")
        opt.step(th, gd)
        gm = g.copy()
        gm[:3] = 0.0  # frozen entries: plain Adam with a zero gradient never moves them
        ref.grad = torch.tensor(gm, dtype=torch.float64)
        ropt.step()
    torch.cuda.synchronize()
    got = th.cpu().numpy()
    want = ref.detach().numpy()
    assert np.array_equal(got[:3], theta0[:3])
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-14)
    assert int(opt.count.item()) == len(grads)


@pytest.mark.parametrize("fam,T,m,d", DESIGNS[:3])
def test_graph_replays_match_eager(fam, T, m, d):
    """Every replay of a captured training step equals the eager step, with
    eager work and synchronisation between replays."""
    from paper_2603_16014_amd import training
    say("graph replay", fam, T, m, d)
    w = tiny(fam, T, m, d, seed=5)
    plan, theta = _plan(w)
    K = 6
    f = training.Fit(plan, theta, lr=0.05)
    eager = []
    for _ in range(K):
        f.step()
        eager.append((f.theta.clone(), f.out3.clone()))
    torch.cuda.synchronize()
    g_fit = training.Fit(plan, theta, lr=0.05)
    g_fit.step()  # warm-up outside capture, then restore the start
    torch.cuda.synchronize()
    g_fit.theta.copy_(theta)
    g_fit.opt.reset()
    g = training._capture(lambda ss: g_fit.step(), [])
    for k in range(K):
        g.replay()
        torch.cuda.synchronize()
        _ = (g_fit.theta * 2.0).sum().item()  # eager work between replays
        assert torch.equal(g_fit.out3, eager[k][1]), k
        assert torch.equal(g_fit.theta, eager[k][0]), k


def test_fit_graph_equals_eager_and_descends():
    from paper_2603_16014_amd import training
    say("fit graph vs eager")
    w = tiny("dseq", 3, [7, 7, 7], 3, seed=7)
    plan, theta = _plan(w, "mixed")
    th_e, h_e, _ = training.fit(plan, theta, 20, lr=0.05, graph=False)
    th_g, h_g, _ = training.fit(plan, theta, 20, lr=0.05, graph=True)
    torch.cuda.synchronize()
    assert torch.equal(th_e, th_g)
    assert torch.equal(h_e, h_g)
    h = h_g.cpu().numpy()
    assert h[-1] < h[0]


@pytest.mark.skip(reason="with the fork onto the plan's own stream enabled under capture, this "
                         "capture of several fits from side streams ended in a host segfault in "
                         "the runtime's capture end; the cause is not shown, the library now "
                         "runs captured calls in order (see test_batched_fits_in_order_capture)")
def test_batched_fits_match_single_fits():
    _batched_fits_match_single_fits(overlap=None)


def test_batched_fits_in_order_capture():
    """The same check with every plan set to in-order passes before capture."""
    _batched_fits_match_single_fits(overlap=1)


def _batched_fits_match_single_fits(overlap):
    from paper_2603_16014_amd import training
    say("batched graph vs single fits", overlap)
    designs = [tiny("dseq", 2, [6, 5], 2, seed=11), tiny("lat", 3, [6, 6, 6], 2, seed=12),
               tiny("dseq", 3, [6, 6, 6], 4, seed=13), tiny("lat", 2, [7, 5], 3, seed=14),
               tiny("dseq", 4, [6, 6, 5, 4], 2, seed=15)]
    plans, thetas = zip(*[_plan(w) for w in designs])
    if overlap is not None:
        for p in plans:
            p.set_overlap(overlap)
    K = 4
    bf = training.BatchedFits(list(plans), list(thetas), lr=0.05, nstreams=3)
    ms = bf.run(K)
    assert len(ms) == K and all(v > 0 for v in ms)
    for p, t0, f in zip(plans, thetas, bf.fits):
        th, _, _ = training.fit(p, t0, K, lr=0.05, graph=False)
        torch.cuda.synchronize()
        assert torch.equal(f.theta, th)
    # a second run continues from the reached state after an explicit reset
    bf.reset()
    bf.run(K)
    for p, t0, f in zip(plans, thetas, bf.fits):
        th, _, _ = training.fit(p, t0, K, lr=0.05, graph=False)
        assert torch.equal(f.theta, th)


def test_nll_grad_batched_entry_point():
    from paper_2603_16014_amd import mtgp
    say("mtgp_nll_grad_batched")
    designs = [tiny("dseq", 2, [6, 6], 2, seed=21), tiny("lat", 3, [6, 5, 4], 2, seed=22),
               tiny("dseq", 3, [7, 6, 6], 3, seed=23)]
    plans, thetas = zip(*[_plan(w) for w in designs])
    outs = [torch.zeros(3, dtype=torch.float64, device="cuda") for _ in plans]
    grads = [torch.zeros(p.theta_size, dtype=torch.float64, device="cuda") for p in plans]
    mtgp.nll_grad_batched(list(plans), list(thetas), outs, grads)
    for p, t, o, g in zip(plans, thetas, outs, grads):
        o1, g1, _ = p.nll_grad(t)
        torch.cuda.synchronize()
        assert torch.equal(o, o1)
        assert torch.equal(g, g1)
    mtgp.nll_grad_batched([], [], [], [])


@pytest.mark.parametrize("m,precision", [([8, 8, 8], "fp64"), ([14, 14, 14], "mixed"),
                                         ([13, 13, 12, 9], "fp64"), ([14, 12, 12], "mixed"),
                                         ([14] * 6, "mixed")])
def test_overlap_is_bitwise_identical(m, precision):
    """Chunked overlap of the digital-net passes changes only the schedule
    (six equal tasks: 16 kernel columns, so 16 and 32 chunks are exercised)."""
    from _designs import tiny
    say("overlap", m, precision)
    w = tiny("dseq", len(m), m, 3, seed=31)
    plan, theta = _plan(w, precision)
    ref = None
    for chunks in (1, 2, 3, 8, 4, 16, 32):
        plan.set_overlap(chunks)
        out3, grad, tau = plan.nll_grad(theta)
        torch.cuda.synchronize()
        got = (out3.clone(), grad.clone(), tau.clone())
        if ref is None:
            ref = got
        else:
            for a, b in zip(got, ref):
                assert torch.equal(a, b), chunks
