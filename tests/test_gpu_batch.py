"""Many fits with one launch per phase (mtgp_batch_*, through the C ABI).

Against the dense oracle per fit (small heterogeneous fits of both families,
equal and nested sizes, T = 1..4): FP64 loss to 1e-10 of |quad| + |log det|
and gradient to 1e-7 of max |grad|; mixed 1e-5 and 1e-4 (the stated
targets).  Against the per-plan path on the shapes of the many-fit workload
(T up to 8, d up to 10, nested sizes up to 2^14, mixed families): the two
compute the same quantities through different transform and elimination
orders, so they agree to the same tolerances.  Adam and a captured graph
of (loss + gradient, Adam) are checked against the per-fit path step by
step."""
import numpy as np
import pytest
import torch

import workloads
from _designs import tiny
from _gpu_common import oracle_for, rel_err, say

pytestmark = pytest.mark.gpu

mt = pytest.importorskip("paper_2603_16014_amd.mtgp")

SMALL = [("dseq", 2, [6, 6], 2), ("lat", 3, [6, 5, 5], 3), ("dseq", 4, [7, 5, 4, 4], 2),
         ("lat", 1, [7], 2), ("dseq", 3, [5, 5, 5], 4), ("lat", 2, [7, 3], 2),
         ("dseq", 1, [6], 3), ("lat", 4, [6, 6, 6, 6], 2)]


def _targets(p, w):
    x = [workloads.digits_to_float(mt.digits_as_uint32(p.gen_points(t, 0, 1 << w.m[t])))
         for t in range(w.T)]
    return np.concatenate(workloads.target_values(w, x, np.random.default_rng(w.seed)))


def _grad_scale(g):
    return max(np.abs(np.concatenate([np.atleast_1d(v).ravel() for v in g.values()])).max(), 1e-300)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_against_oracle(precision):
    ws, plans, thetas, refs = [], [], [], []
    for k, (fam, T, m, d) in enumerate(SMALL):
        w = tiny(fam, T, m, d, seed=200 + k, rank=min(T, 2))
        ref = oracle_for(w, want_grad=True)
        p = mt.Plan.from_workload(w, precision)
        p.set_data(torch.from_numpy(ref["y"]).cuda())
        ws.append(w)
        plans.append(p)
        thetas.append(p.pack_theta(w.theta))
        refs.append(ref)
    say("batch against oracle", precision, len(plans), "fits")
    b = mt.Batch(plans, thetas)
    b.nll_grad()
    torch.cuda.synchronize()
    tl, tg = (1e-10, 1e-7) if precision == "fp64" else (1e-5, 1e-4)
    for k, (w, p, ref) in enumerate(zip(ws, plans, refs)):
        assert p.status() == (0, -1), k
        r = ref["res"]
        o3 = b.out3s[k].cpu().numpy()
        den = abs(r["quad"]) + abs(r["logdet"])
        assert abs(o3[2] - r["L"]) < tl * den, (k, o3, r["L"])
        g = p.unpack(b.grads[k])
        sc = _grad_scale(ref["grad"])
        for key, v in ref["grad"].items():
            assert rel_err(g[key], v, sc) < tg, (k, key, rel_err(g[key], v, sc))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_against_per_plan_path_many_fit_shapes(precision):
    fits = workloads.config4_fits(12)
    say("batch vs per-plan path", precision, [(f.family, f.T, f.d, f.m) for f in fits])
    plans, thetas = [], []
    for w in fits:
        p = mt.Plan.from_workload(w, precision)
        p.set_data(torch.from_numpy(_targets(p, w)).cuda())
        plans.append(p)
        thetas.append(p.pack_theta(w.theta))
    ref = [p.nll_grad(t) for p, t in zip(plans, thetas)]
    ref = [(o.cpu().numpy(), g.cpu().numpy()) for o, g, _ in ref]
    b = mt.Batch(plans, thetas)
    b.nll_grad()
    torch.cuda.synchronize()
    tl, tg = (1e-10, 1e-7) if precision == "fp64" else (1e-5, 1e-4)
    for k, p in enumerate(plans):
        assert p.status() == (0, -1), k
        o3, g = b.out3s[k].cpu().numpy(), b.grads[k].cpu().numpy()
        ro, rg = ref[k]
        den = abs(ro[0]) + abs(ro[1])
        assert abs(o3[2] - ro[2]) < tl * den, (k, o3, ro)
        assert np.abs(g - rg).max() < tg * np.abs(rg).max(), (k, np.abs(g - rg).max())


def test_batch_adam_and_graph_replays():
    """Three steps of (loss + gradient, Adam) for every fit, eager and as
    replays of one captured graph with eager work in between, against the
    per-fit path (FP64)."""
    fits = workloads.config4_fits(6, kmax=11)
    say("batch adam + graph", [(f.family, f.T, f.m) for f in fits])
    plans, thetas, frozen = [], [], []
    for w in fits:
        p = mt.Plan.from_workload(w, "fp64")
        p.set_data(torch.from_numpy(_targets(p, w)).cuda())
        plans.append(p)
        thetas.append(p.pack_theta(w.theta))
        fm = np.zeros(p.theta_size, dtype=np.uint8)
        fm[:w.T] = 1
        frozen.append(fm)
    from paper_2603_16014_amd import training
    # per-fit path
    ref_fits = [training.Fit(p, t, lr=0.05, frozen=f) for p, t, f in zip(plans, thetas, frozen)]
    ref_hist = []
    for _ in range(3):
        for f in ref_fits:
            f.step()
        ref_hist.append([f.theta.cpu().numpy().copy() for f in ref_fits])
    # batch, eager
    b = mt.Batch(plans, [t.clone() for t in thetas], adam=True, frozen=frozen)
    for s in range(3):
        b.nll_grad()
        b.adam_step(0.05)
        torch.cuda.synchronize()
        for k in range(len(plans)):
            got = b.thetas[k].cpu().numpy()
            want = ref_hist[s][k]
            assert np.abs(got - want).max() < 1e-9 * max(np.abs(want).max(), 1.0), (s, k)
    # batch, captured once and replayed
    for k, t in enumerate(thetas):
        b.thetas[k].copy_(t)
    b.reset_adam()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.nll_grad()   # warm (outside the capture), then restore
        b.adam_step(0.05)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for k, t in enumerate(thetas):
        b.thetas[k].copy_(t)
    b.reset_adam()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        b.nll_grad()
        b.adam_step(0.05)
    for s in range(3):
        g.replay()
        junk = torch.randn(1 << 16, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        del junk
        for k in range(len(plans)):
            got = b.thetas[k].cpu().numpy()
            want = ref_hist[s][k]
            assert np.abs(got - want).max() < 1e-9 * max(np.abs(want).max(), 1.0), (s, k)


def test_batch_refusals():
    say("batch refusals")
    big = mt.Plan.from_workload(tiny("dseq", 2, [15, 3], 2, seed=9), "fp64")
    small = mt.Plan.from_workload(tiny("dseq", 2, [6, 3], 2, seed=9), "fp64")
    f32 = mt.Plan.from_workload(tiny("dseq", 2, [6, 3], 2, seed=9), "f32")
    th = [p.pack_theta(tiny("dseq", 2, [6, 3], 2, seed=9).theta) for p in (big, small, f32)]
    for plans, thetas in (([small, big], th[:2]), ([small, f32], [th[1], th[2]])):
        with pytest.raises(Exception, match="not supported"):
            mt.Batch(plans, thetas)
    empty = mt.Batch([], [])
    empty.nll_grad()
