"""Benchmark: MLE loss + gradient evaluations per second of the fast MTGP
hot path at T=8 tasks x n=2^24 digitally shifted digital-net points per task
(d=10, order-2 DSI product kernel, low-rank + diagonal task covariance),
on one MI355X.

One step = one mtgp_nll_grad call: kernel columns fused with the low-bit
forward transform pass, the high-bit pass, the per-frequency 8x8
factorisations, loss, the adjoint transform passes fused with the derivative
reduction, and the final reductions (the data transform yhat is computed once
per data set by mtgp_set_data, outside the timed region).  Inputs are seeded
and synthetic and resident in HBM before timing starts.

Prints one JSON line: evals/s of the primary (mixed) path, the FP64 path
beside it, the mixed-vs-FP64 differences, per-kernel durations from HIP
events recorded on the launch stream inside the timed region, a roofline
entry for the dominant kernel, and the dense CPU oracle timed on a bounded
sample.

``python bench.py --pmc-summary FETCH_DIR WRITE_DIR TRACE_DIR`` turns the CSV
output of three rocprofv3 runs of this script (``--pmc FETCH_SIZE``,
``--pmc WRITE_SIZE``, ``--kernel-trace --stats``) into the markdown summary
kept under profiles/, whose JSON block is read back for ``traffic``.
"""
import argparse
import csv
import glob
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane
# operations/s (one wave64 instruction per CU per clock); FP64 FMA and the
# integer / conversion instructions of the fused kernels issue at this rate
# (FP32 vector 157.3 TFLOP/s = 4 flops per lane-op with packed FMA; FP64
# vector 78.6 TFLOP/s = 2 flops per lane-op)
CU_COUNT, CLOCK_HZ = 256, 2.4e9
VALU_LANE_OPS_PEAK = CU_COUNT * 64 * CLOCK_HZ
# Algorithmic VALU lane ops per (column, element, dimension) of the two fused
# kernels, counted from their arithmetic: generation 7 per dimension (digit
# XOR, leading-zero count, table offset, u32 -> f64 conversion, kappa FMA,
# factor FMA, product) plus 12 per element (the Walsh-Hadamard adds of the
# low bits) spread over d = 10; the reduction 10 per dimension (the
# same four digit / table steps, kappa and factor FMA, prefix product,
# suffix combine, suffix product, accumulate) plus 14 per element (12 adds,
# weight scale, value accumulate).  Set-up, addressing and loop control are
# not counted.
GEN_OPS_PER_UNIT = 8.2
ADJ_OPS_PER_UNIT = 11.4
COPY_PROBE_BYTES = 1 << 30     # plain streaming kernel used to scale the HBM counters
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_loss_grad_T8_d10_n2e24_mixed.md")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_gen_adj_T8_d10_n2e24_mixed.md")

# phase -> (kernel-name pattern in rocprofv3 output, bound)
PHASE_KERNELS = {
    "gen_fwd_low": ("gen_fwd_kernel", "alu"),
    "fwd_high": ("fwht_hi12_kernel (1 pass)", "hbm"),
    "solve": ("solve_eq_kernel", "hbm"),
    "adj_high": ("fwht_hi12_kernel (1 pass)", "hbm"),
    "adj_low_reduce": ("adj_reduce_kernel", "alu"),
}


_T0 = time.perf_counter()


def progress(*a):
    """Progress of the run on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f}s]", *a, file=sys.stderr, flush=True)


# the sources of the kernels a loss + gradient evaluation of the digital-net
# workload runs, and of their launch sequence
HOT_PATH_SOURCES = ("api.hip", "common.h", "kernels.h", "colgen.h", "fused_eval.h",
                    "fused_gen_o2.hip", "fused_adj_o2.hip", "adjoint.hip", "transform.hip",
                    "solve.hip", "solve_dev.h")


def kernel_sources_digest():
    """Digest of the hot path's HIP sources; a counter summary is stale once
    it changes."""
    h = hashlib.sha256()
    for name in HOT_PATH_SOURCES:
        f = os.path.join(ROOT, "paper_2603_16014_amd", "csrc", name)
        h.update(name.encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def targets_on_device(plan, w):
    """Seeded targets of the workload, built on the GPU from the plan's points."""
    import torch
    rng = np.random.default_rng(w.seed + 1000)
    p = w.target_params
    ys = []
    for t in range(w.T):
        n = 1 << w.m[t]
        x = plan.gen_points(t, 0, n).view(torch.int32)
        xf = (x.to(torch.int64) & 0xFFFFFFFF).to(torch.float64) * (2.0 ** -32)
        del x

        def g(k):
            s = torch.zeros(n, dtype=torch.float64, device="cuda")
            for j in range(w.d):
                s += torch.sin(2 * math.pi * p["freq"][k][j] * xf[:, j] + p["phase"][k][j]) / (j + 1)
            return s
        rho = p["rho"][t]
        y = rho * g(0) + math.sqrt(1 - rho * rho) * g(t + 1)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(int(rng.integers(0, 2 ** 31)))
        y += math.sqrt(w.noise_var) * torch.randn(n, dtype=torch.float64, device="cuda", generator=gen)
        ys.append(y)
        del xf
    return torch.cat(ys)


def copy_probe():
    """One plain streaming kernel (read B bytes, write B bytes) of known size,
    so that HBM byte counters of the other kernels can be scaled by what the
    same counters read for it."""
    import torch
    src = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()


def time_evals(plan, theta, steps, warmup, timing=True):
    """K timed evaluations bracketed by device synchronisation; per-phase
    durations come from the library's HIP events recorded on the same stream
    in the same timed region (no host wait between steps)."""
    import torch
    out3 = torch.empty(3, dtype=torch.float64, device="cuda")
    grad = torch.empty(plan.theta_size, dtype=torch.float64, device="cuda")
    tau = torch.empty(plan.T, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        plan.nll_grad(theta, out3, grad, tau)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    plan.enable_timing(timing)
    e0.record(st)
    for i in range(steps):
        plan.nll_grad(theta, out3, grad, tau)
    e1.record(st)
    torch.cuda.synchronize()
    # the event ring holds the 64 most recent steps
    phases = plan.phase_times() if timing else {}
    done = min(steps, 64) if timing else 0
    plan.enable_timing(False)
    ms = e0.elapsed_time(e1) / steps
    code, bad = plan.status()
    if code != 0:
        raise RuntimeError(f"status {code} at frequency {bad}")
    return ms, out3.cpu().numpy(), grad.cpu().numpy(), tau.cpu().numpy(), phases, done


def default_high_passes(r):
    """HBM passes of the library's default schedule over r high index bits."""
    n = 0
    while r > 0:
        r -= r if r in (8, 10, 12) else min(r, 6)
        n += 1
    return n


def algo_units(w, precision, a_bits=12):
    """Algorithmic HBM bytes per launch of each phase at this workload (P
    distinct kernel columns of length n, forward working values of wb bytes,
    spectrum / adjoint weights of sb bytes), and for the two fused evaluation
    kernels their algorithmic VALU lane operations: 8.2 per (column, element,
    dimension) for the generation and 11.4 for the derivative reduction
    (5.5e10 per evaluation at T=8, d=10, n=2^24)."""
    T, d, n, P = w.T, w.d, 1 << w.m[0], 1 + w.T * (w.T - 1) // 2
    wb, sb = {"fp64": (8, 8), "mixed": (8, 4), "f32": (4, 4)}[precision]
    lb = min(a_bits, w.m[0])  # width of the low-bit (LDS) transform pass
    return {
        "gen_fwd_low": {"bytes": P * n * wb, "ops": GEN_OPS_PER_UNIT * P * n * d},
        "fwd_high": {"bytes": P * n * (wb + sb)},        # read work, write spectrum
        "solve": {"bytes": P * n * 2 * sb + T * n * 8},  # read spectrum + yhat, write weights
        "adj_high": {"bytes": P * n * (sb + wb)},        # read weights, write work
        "adj_low_reduce": {"bytes": P * n * (wb if w.m[0] > lb else sb),
                           "ops": ADJ_OPS_PER_UNIT * P * n * d},
    }


def eval_bytes_model(w, precision):
    """HBM bytes of one loss + gradient evaluation by the model
    (8 P b + 8 T) n: two HBM passes per transform direction with column
    generation fused into the first forward pass and the derivative
    reduction into the last adjoint pass, b bytes per stored spectrum /
    weight value, and the FP64 transformed data read once."""
    T, n, P = w.T, 1 << w.m[0], 1 + w.T * (w.T - 1) // 2
    b = {"fp64": 8, "mixed": 4, "f32": 4}[precision]
    return (8 * P * b + 8 * T) * n


def load_valu(precision):
    """VALU counters per launch of the fused evaluation kernels from the
    committed summary, or None when it is missing or stale."""
    if precision != "mixed" or not os.path.exists(VALU_FILE):
        return None
    txt = open(VALU_FILE).read()
    if "```json" not in txt:
        return None
    blob = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
    if blob.get("sources_digest") != kernel_sources_digest():
        return None
    return blob.get("kernels", {})


def load_traffic(precision):
    """HBM bytes per launch of each kernel from the committed counter summary,
    or None when it is missing, for another precision, or stale."""
    if precision != "mixed" or not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    if "```json" not in txt:
        return None
    blob = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
    if blob.get("sources_digest") != kernel_sources_digest():
        return None
    return {k: v["hbm_bytes"] for k, v in blob.get("phases", {}).items()}


def _timed(fn, min_s=1.0, max_reps=5):
    """Mean wall time of fn() over repeats until min_s has passed."""
    t0, reps = time.perf_counter(), 0
    while True:
        fn()
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_s or reps >= max_reps:
            return el / reps


def dense_baseline():
    """The dense FP64 oracle (Gram assembly, LAPACK Cholesky, solves) timed on
    the host: the small net workload at its full size (T=2, d=2, n=2^10,
    N=2048; loss, loss + gradient, posterior mean at 1024 points), with all
    BLAS threads and with one, and the large workload's shape (T=8, d=10)
    scaled to 2^9 points per task (N=4096; loss).  The O(N^3) extrapolation
    to N=2^27 is labelled as one."""
    import threadpoolctl
    import workloads
    from oracle import dense, points
    info = threadpoolctl.threadpool_info()
    blas = sorted({f"{i.get('internal_api')} {i.get('version')}" for i in info
                   if i.get("user_api") == "blas"})
    threads = max([i.get("num_threads", 1) for i in info] + [1])
    out = {"blas": blas, "blas_threads": threads, "os_cpu_count": os.cpu_count(),
           "affinity_cpus": len(os.sched_getaffinity(0))}
    w1 = workloads.config1()
    X = points.task_points(w1)
    y = dense.targets(w1, np.random.default_rng(w1.seed), X)
    xs = workloads.uniform_digits(np.random.default_rng(0), 1024, w1.d)
    small = {"workload": f"T={w1.T}, d={w1.d}, n=2^{w1.m[0]} digital nets, N={w1.N}"}
    for label, limit in (("all_threads", None), ("1_thread", 1)):
        progress(f"cpu baseline: dense oracle N={w1.N}, {label}")
        with threadpoolctl.threadpool_limits(limits=limit):
            small[label] = {
                "nll_s": _timed(lambda: dense.nll(w1, y, X=X)),
                "nll_grad_s": _timed(lambda: dense.grad(w1, y, X=X), max_reps=2),
                "predict_1024_s": _timed(lambda: dense.posterior_mean(w1, y, xs, X=X), max_reps=2),
            }
    out["small_net_full_size"] = small
    w5 = workloads.config5()
    ws = workloads.scaled(w5, [9] * w5.T)
    Xs = points.task_points(ws)
    ys = dense.targets(ws, np.random.default_rng(1), Xs)
    progress(f"cpu baseline: dense oracle N={ws.N} (large workload's shape)")
    t = _timed(lambda: dense.nll(ws, ys, X=Xs), min_s=0.0, max_reps=1)
    out["large_shape_scaled"] = {
        "workload": f"T={ws.T}, d={ws.d}, n=2^9 per task, N={ws.N}", "nll_s": t,
        "extrapolated_nll_s_at_full_size": t * (w5.N / ws.N) ** 3,
        "extrapolation": "O(N^3) from N=4096 to N=2^27; the Gram matrix alone would need "
                         f"{8 * w5.N ** 2 / 2 ** 50:.0f} PiB"}
    return out


def cpu_baseline(w, budget_s=25.0):
    """The spectral oracle (numpy, FP64: Walsh / DFT of the kernel columns and
    of their derivative columns, per-frequency T x T solves) computing the MLE
    loss and gradient on the workload's shape at 2^16 points per task; the
    rate is scaled to the full size by the n log n cost of its transforms.
    The dense oracle's own timings go beside it."""
    import workloads
    from oracle import dense, points, spectral
    import threadpoolctl
    info = threadpoolctl.threadpool_info()
    threads = max([i.get("num_threads", 1) for i in info] + [1])
    m = min(16, min(w.m))
    ws = workloads.scaled(w, [m] * w.T)
    y = dense.targets(ws, np.random.default_rng(1), points.task_points(ws))
    t0 = time.perf_counter()
    reps = 0
    while True:
        spectral.mle_grad(ws, y)
        reps += 1
        progress(f"cpu baseline: {reps} evals")
        el = time.perf_counter() - t0
        if el > budget_s / 2 or reps >= 8:
            break
    per = el / reps
    mf = max(w.m)
    scale = (2.0 ** mf * mf) / (2.0 ** m * m)
    per_full = per * scale
    return {"value": 1.0 / per_full, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"spectral FP64 oracle (numpy) loss+gradient at T={w.T}, d={w.d}, "
                      f"n=2^{m} per task (N={ws.N}): {reps} evals in {el:.1f} s = {per:.2f} "
                      f"s/eval; value = that rate scaled by n log n to n=2^{mf} (x{scale:.0f}), "
                      "an extrapolation",
            "sample_evals_per_s": 1.0 / per,
            "os_cpu_count": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "dense": dense_baseline()}


def train_leg(plan, theta, steps, lr=0.05):
    """`steps` Adam steps of loss+gradient captured as one HIP graph step and
    replayed; timed with events around the replays (capture excluded)."""
    import torch
    from paper_2603_16014_amd import training
    f = training.Fit(plan, theta, lr=lr)
    f.step()
    torch.cuda.synchronize()
    f.theta.copy_(theta)
    f.opt.reset()
    g = training._capture(lambda ss: f.step(), [])
    hist = torch.zeros(steps, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for k in range(steps):
        g.replay()
        hist[k].copy_(f.out3[2])
    e1.record(st)
    torch.cuda.synchronize()
    h = hist.cpu().numpy()
    code, bad = plan.status()
    return {"adam_steps": steps, "lr": lr, "ms_per_step": e0.elapsed_time(e1) / steps,
            "L_first": float(h[0]), "L_last": float(h[-1]), "status": code,
            "theta_last": f.theta}


def predict_leg(plan, w, theta, m_star=20, M_direct=1 << 10):
    """Posterior mean at a fresh shifted test net of 2^m_star points
    (structured cross-block path) and at M_direct uniform points (direct sum)."""
    import torch
    import workloads
    rng = np.random.default_rng(w.seed + 2000)
    shift_star = workloads.random_shifts(rng, 1, w.d)[0]
    xs = workloads.uniform_digits(rng, M_direct, w.d)
    from paper_2603_16014_amd import mtgp
    xs_dev = mtgp.digits_to_device(xs)
    out = {}
    for name, fn in (("net", lambda: plan.predict_net(theta, shift_star, m_star)),
                     ("direct", lambda: plan.predict(theta, xs_dev))):
        progress("posterior mean", name)
        fn()
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        reps = 3
        for _ in range(reps):
            mean = fn()
        e1.record(st)
        torch.cuda.synchronize()
        npts = (1 << m_star) if name == "net" else M_direct
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"points": npts, "ms": ms, "points_per_s": npts / (ms * 1e-3),
                     "finite": bool(torch.isfinite(mean).all().item())}
    return out


def batched_leg(nfits, steps, nstreams=16, eager_steps=3):
    """Config of many small fits: each an independent MTGP (T 2..8, d 2..10,
    mixed families, nested sizes 2^8..2^14), `steps` Adam steps of every fit
    per replay of one captured graph, against a Python loop of single fits."""
    import torch
    import workloads
    from paper_2603_16014_amd import mtgp, training
    fits = workloads.config4_fits(nfits)
    plans, thetas = [], []
    for i, w in enumerate(fits):
        p = mtgp.Plan.from_workload(w, "mixed")
        p.set_data(targets_on_device(p, w))
        plans.append(p)
        thetas.append(p.pack_theta(w.theta))
        if (i + 1) % 32 == 0:
            progress(f"batched leg: {i + 1} plans")
    torch.cuda.synchronize()
    progress("batched leg: capture")
    bf = training.BatchedFits(plans, thetas, lr=0.05, nstreams=nstreams)
    t0 = time.perf_counter()
    bf.capture()
    cap_s = time.perf_counter() - t0
    ms = np.array(bf.run(steps))
    progress("batched leg: graph replays done")
    bad = sum(1 for p in plans if p.status()[0] != 0)
    bf.reset()
    eager = np.array(bf.run_eager(eager_steps))
    progress("batched leg: eager loop done")
    # the library's many-fit launches: one launch per phase for all fits
    pb = training.PersistentBatchedFits(plans, thetas, lr=0.05)
    t0 = time.perf_counter()
    pb.capture()
    pcap_s = time.perf_counter() - t0
    pms = np.array(pb.run(steps))
    pbad = sum(1 for p in plans if p.status()[0] != 0)
    progress("batched leg: many-fit launches done")
    persistent = {"fits_steps_per_s": nfits * steps / (pms.sum() * 1e-3),
                  "step_ms_p50": float(np.percentile(pms, 50)),
                  "step_ms_p99": float(np.percentile(pms, 99)),
                  "graph_capture_s": pcap_s, "fits_not_pd": pbad,
                  "launches_per_step": "prep, forward columns (one per kernel type and "
                                       "dimension width), elimination, adjoint columns, "
                                       "chain rule, Adam"}
    return {"fits": nfits, "adam_steps": steps, "streams": nstreams,
            "many_fit_launches": persistent,
            "fits_steps_per_s": nfits * steps / (ms.sum() * 1e-3),
            "step_ms_p50": float(np.percentile(ms, 50)), "step_ms_p99": float(np.percentile(ms, 99)),
            "graph_capture_s": cap_s, "fits_not_pd": bad,
            "eager_loop_fits_steps_per_s": nfits * eager_steps / (eager.sum() * 1e-3),
            "eager_step_ms_p50": float(np.percentile(eager, 50)),
            "total_points": int(sum(w.N for w in fits))}


def transforms_leg(ncols=29, m=24, reps=5):
    """Standalone transforms on the kernel-column shape of the workload:
    mtgp_fwht and mtgp_fft (natural frequency order out) on [ncols][2^m] in
    FP32 and FP64.  Algorithmic bytes: read + write once (FWHT), real read +
    complex write (FFT)."""
    import torch
    from paper_2603_16014_amd import mtgp
    out = {}
    st = torch.cuda.current_stream()
    for name, dt, b in (("fwht_f32", torch.float32, 4), ("fwht_f64", torch.float64, 8),
                        ("fft_f32", torch.float32, 4), ("fft_f64", torch.float64, 8)):
        progress("transform", name)
        if name.startswith("fwht"):
            x = torch.randn(ncols << m, dtype=dt, device="cuda")
            fn = lambda: mtgp.fwht(x, m)  # noqa: E731
            nbytes = 2 * x.numel() * b
            shape = f"[{ncols}][2^{m}]"
        else:
            x = torch.randn(ncols << m, dtype=dt, device="cuda")
            fn = lambda: mtgp.fft(x, m)  # noqa: E731
            nbytes = 3 * x.numel() * b
            shape = f"[{ncols}][2^{m}]"
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"shape": shape, "ms": ms, "algorithmic_bytes": nbytes,
                     "GB_s": nbytes / (ms * 1e-3) / 1e9,
                     "hbm_frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        if name.startswith("fwht"):
            # the passes each read and write every element once: the LDS pass
            # over the low 12 bits, then by size one pass over a remainder of
            # 8, 10 or 12 bits, else register passes of at most 6 bits
            passes = 1 + default_high_passes(m - 12)
            pb = passes * nbytes
            out[name].update({"passes": passes, "pass_bytes": pb,
                              "pass_GB_s": pb / (ms * 1e-3) / 1e9,
                              "pass_hbm_frac": pb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS})
        elif m == 24:
            # three passes at 2^24 points: the generating tile over the top
            # 10 bits (real in, complex out), one 5-bit register pass and the
            # 9-bit wave pass writing natural order (complex in and out)
            n_el = ncols << m
            pb = n_el * (3 * b + 2 * 4 * b)
            out[name].update({"passes": 3, "pass_bytes": pb,
                              "pass_GB_s": pb / (ms * 1e-3) / 1e9,
                              "pass_hbm_frac": pb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS})
        del x
        torch.cuda.empty_cache()
    return out


def lattice_leg(steps=5, warmup=1):
    """Loss + gradient on the config-5 shape with shifted rank-1 lattices and
    the order-2 SI kernel (FFT path), FP64 and mixed, with their agreement."""
    import torch
    import workloads
    from paper_2603_16014_amd import mtgp
    w = workloads.config5_lat()
    res, y, keep = {}, None, {}
    for prec in ("fp64", "mixed"):
        progress("lattice leg", prec)
        plan = mtgp.Plan.from_workload(w, prec)
        if y is None:
            y = targets_on_device(plan, w)
        plan.set_data(y)
        theta = plan.pack_theta(w.theta)
        ms, out3, grad, _, _, _ = time_evals(plan, theta, steps, warmup, timing=False)
        _, _, _, _, phases, _ = time_evals(plan, theta, steps, 1, timing=True)
        progress(f"lattice {prec}: {ms:.3f} ms per loss+gradient")
        res[prec] = {"evals_per_s": 1000.0 / ms, "ms_per_step": ms,
                     "phases_ms": {k: round(v, 4) for k, v in phases.items()}}
        keep[prec] = (out3, grad)
        del plan
        torch.cuda.empty_cache()
    (a3, ag), (b3, bg) = keep["mixed"], keep["fp64"]
    den = abs(b3[0]) + abs(b3[1])
    res["mixed_vs_fp64"] = {"L_rel": float(abs(a3[2] - b3[2]) / den),
                            "grad_rel_maxnorm": float(np.abs(ag - bg).max() / np.abs(bg).max())}
    res["workload"] = (f"T={w.T}, d={w.d}, n=2^{w.m[0]} shifted rank-1 lattice points per task "
                       f"(N={w.N}), order-2 SI kernel, rank-2 + diagonal task covariance")
    return res


def run(args):
    import torch
    import workloads
    from paper_2603_16014_amd import mtgp

    w = workloads.config5()
    if args.m != 24:
        w = workloads.scaled(w, [args.m] * w.T)
    copy_probe()
    results = {}
    y = None
    for prec in args.precisions.split(","):
        sched = tuple(int(v) for v in args.sched.split(",")) if args.sched else None
        progress("plan", prec)
        plan = mtgp.Plan.from_workload(w, prec, schedule=sched)
        if y is None:
            y = targets_on_device(plan, w)
        plan.set_data(y)
        theta = plan.pack_theta(w.theta)
        tuned = None
        if args.tune and not sched:
            from paper_2603_16014_amd import autotune
            progress("autotune", prec)
            tuned = autotune.tune(plan, theta)
            progress(f"{prec}: schedule {tuned['schedule']}, overlap {tuned['overlap']}"
                     f"{' (cached)' if tuned['cached'] else ''}")
        progress("timing", prec)
        # the measured configuration: overlapped passes (library default or tuned)
        if args.no_overlap:
            plan.set_overlap(1)
        chunks = plan.overlap
        ms, out3, grad, tau, _, _ = time_evals(plan, theta, args.steps, args.warmup, timing=False)
        progress(f"{prec}: {ms:.3f} ms per loss+gradient")
        # per-kernel durations need the passes in sequence on one stream
        plan.set_overlap(1)
        ms_seq, _, _, _, phases, nph = time_evals(plan, theta, args.steps, 1, timing=True)
        plan.set_overlap(chunks)
        progress(f"{prec}: {ms_seq:.3f} ms per loss+gradient without overlap")
        results[prec] = dict(ms=ms, out3=out3, grad=grad, phases=phases, nph=nph, ms_seq=ms_seq,
                             schedule=plan.schedule, overlap=chunks,
                             fused_occupancy=getattr(plan, "fused_occupancy", 0),
                             tuned=None if tuned is None else
                             {"cached": tuned["cached"],
                              "timings_ms": {k: round(v, 3) for k, v in tuned["timings"].items()}})
        if prec == "mixed" and args.train_steps > 0:
            progress("training leg")
            tr = train_leg(plan, theta, args.train_steps)
            th_last = tr.pop("theta_last")
            tr["evals_per_s_at_last_theta"] = 1000.0 / time_evals(plan, th_last, 5, 1)[0]
            results["train"] = tr
            if args.predict:
                progress("posterior-mean leg")
                results["predict"] = predict_leg(plan, w, th_last)
        del plan
        torch.cuda.empty_cache()
    primary = "mixed" if "mixed" in results else args.precisions.split(",")[0]
    r = results[primary]
    T, n = w.T, 1 << w.m[0]
    extra = {}
    if "fp64" in results and "mixed" in results:
        a, b = results["mixed"], results["fp64"]
        den = abs(b["out3"][0]) + abs(b["out3"][1])
        extra["mixed_vs_fp64"] = {
            "L_rel": float(abs(a["out3"][2] - b["out3"][2]) / den),
            "grad_rel_maxnorm": float(np.abs(a["grad"] - b["grad"]).max() / np.abs(b["grad"]).max()),
        }
        extra["fp64_evals_per_s"] = 1000.0 / b["ms"]
        extra["fp64_ms_per_step"] = b["ms"]
        extra["fp64_sequential_ms_per_step"] = b["ms_seq"]
        extra["fp64_phases_ms"] = {k: round(v, 4) for k, v in b["phases"].items()}
        eb64 = eval_bytes_model(w, "fp64")
        extra["fp64_roofline_eval"] = {
            "bound": "hbm", "model_bytes": eb64, "achieved": eb64 / (b["ms"] * 1e-3) / 1e9,
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": eb64 / (b["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
    ph = r["phases"]
    units = algo_units(w, primary, r["schedule"][0])
    # the committed counter profile was taken with the default schedule
    from paper_2603_16014_amd import mtgp as _mt
    traffic = (load_traffic(primary)
               if args.m == 24 and tuple(r["schedule"]) == _mt.DEFAULT_SCHEDULE else None)
    valu = load_valu(primary) if args.m == 24 else None
    kernels = {}
    for k, (pat, bound) in PHASE_KERNELS.items():
        if k not in ph or ph[k] <= 0:
            continue
        u = units[k]
        e = {"kernel": pat, "ms": round(ph[k], 4), "bound": bound,
             "GB_s": u["bytes"] / (ph[k] * 1e-3) / 1e9}
        e["hbm_frac"] = e["GB_s"] / HBM_PEAK_GBS
        if "ops" in u:
            e["Tops_s"] = u["ops"] / (ph[k] * 1e-3) / 1e12
            e["valu_frac"] = e["Tops_s"] * 1e12 / VALU_LANE_OPS_PEAK
        if traffic and k in traffic:
            e["traffic"] = traffic[k]
        if valu and pat in valu:
            # issued VALU instructions (wave64) per launch from the counters,
            # against one instruction per CU per clock over this launch's time
            v = valu[pat]
            e["counters"] = v
            e["valu_issue_frac"] = v["SQ_INSTS_VALU"] / (ph[k] * 1e-3 * CU_COUNT * CLOCK_HZ)
        kernels[k] = e
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    kd = kernels[dom]
    if kd["bound"] == "hbm":
        roof = {"bound": "hbm", "kernel": kd["kernel"], "achieved": kd["GB_s"],
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": kd["hbm_frac"]}
    else:
        roof = {"bound": "alu", "kernel": kd["kernel"], "achieved": kd["Tops_s"],
                "peak": VALU_LANE_OPS_PEAK / 1e12, "unit": "T VALU lane-ops/s",
                "frac": kd["valu_frac"],
                "model": f"{ADJ_OPS_PER_UNIT if dom == 'adj_low_reduce' else GEN_OPS_PER_UNIT} "
                         "lane ops per (column, element, dimension)"}
        if "valu_issue_frac" in kd:
            roof["valu_issue_frac"] = kd["valu_issue_frac"]
    roof["traffic"] = kd.get("traffic")
    eb = eval_bytes_model(w, primary)
    roof_eval = {"bound": "hbm", "model_bytes": eb, "achieved": eb / (r["ms"] * 1e-3) / 1e9,
                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": eb / (r["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                 "model": "(8 P b + 8 T) n bytes per evaluation, b = stored spectrum bytes"}
    if traffic:
        roof_eval["traffic"] = sum(traffic.values())
    line = {
        "metric": "NLL+grad evals/sec at T=8,n=2^24",
        "value": 1000.0 / r["ms"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "f64 arithmetic, f32 spectrum storage", "fp64": "f64",
                  "f32": "f32"}[primary],
        "data": "synthetic",
        "config": {"workload": f"fast MTGP loss+gradient, digitally shifted digital nets, T={T}, "
                               f"d={w.d}, n=2^{w.m[0]} per task (N={w.N}), order-2 DSI kernel, "
                               f"rank-2 + diagonal task covariance, {primary} path",
                   "T": T, "d": w.d, "n_per_task": n, "N": w.N, "precision": primary},
        "sequential_ms_per_step": r["ms_seq"],
        "phases_ms": {k: round(v, 4) for k, v in ph.items()},
        "phase_steps_timed": r["nph"],
        "kernels": kernels,
        "roofline": roof,
        "roofline_eval": roof_eval,
    }
    line.update(extra)
    line["schedule"] = {"pass_a_bits": r["schedule"][0], "pass_b_bits": r["schedule"][1],
                        "pass_b_tile_bytes": r["schedule"][2], "overlap_chunks": r["overlap"],
                        "fused_occupancy": r["fused_occupancy"],
                        "autotune": r["tuned"]}
    if "train" in results:
        line["training"] = results["train"]
    if "predict" in results:
        line["posterior_mean"] = results["predict"]
    if args.transforms:
        line["transforms"] = transforms_leg()
    if args.lattice:
        line["lattice"] = lattice_leg()
    if args.fits > 0:
        progress("batched leg")
        line["batched_fits"] = batched_leg(args.fits, args.fit_steps)
    if not args.no_cpu_baseline:
        progress("cpu baseline (spectral oracle)")
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)


# --------------------------------------------------------------------------
# rocprofv3 CSV -> markdown summary
# --------------------------------------------------------------------------
def _csv_rows(d, suffix):
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)):
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _phase_of(name, cur):
    """Phase of a library kernel given the phase of the previous dispatch of
    the same evaluation (the order is fixed: prep, generation + low pass,
    high passes, solve, adjoint high passes, adjoint low pass + reduction,
    partial-sum reductions and chain rule)."""
    if "mtgp::prep_kernel" in name:
        return "prep"
    if "gen_fwd_kernel" in name:
        return "gen_fwd_low"
    if "fwht_strided_kernel" in name or "fwht_reg_" in name or "fwht_hi" in name:
        return "fwd_high" if cur in ("gen_fwd_low", "fwd_high") else "adj_high"
    if "solve_eq" in name or "alg1_" in name:
        return "solve"
    if "adj_reduce_kernel" in name:
        return "adj_low_reduce"
    if "colsum_kernel" in name or "finalize_kernel" in name:
        return "finalize"
    return None


def _per_eval(rows, value):
    """Mean over complete evaluations of the per-phase sum of value(row)."""
    evals, cur, acc = [], None, None
    for row in sorted(rows, key=lambda r: int(r["Dispatch_Id"])):
        name = row["Kernel_Name"]
        ph = _phase_of(name, cur)
        if ph == "prep":
            if acc is not None and "finalize" in acc:
                evals.append(acc)
            acc = {}
        if ph is None or acc is None:
            continue
        cur = ph
        v, k = value(row)
        a = acc.setdefault(ph, [0.0, 0, set()])
        a[0] += v
        a[1] += 1
        a[2].add(name.split("(")[0].replace("void ", ""))
    if acc is not None and "finalize" in acc:
        evals.append(acc)
    if not evals:
        return {}, 0
    out = {}
    for ph in evals[-1]:
        vals = [e[ph][0] for e in evals if ph in e]
        out[ph] = (sum(vals) / len(vals), evals[-1][ph][1], sorted(evals[-1][ph][2]))
    return out, len(evals)


def pmc_summary(fetch_dir, write_dir, trace_dir, cmdline):
    fetch_rows = [r for r in _csv_rows(fetch_dir, "counter_collection.csv")
                  if r.get("Counter_Name") == "FETCH_SIZE"]
    write_rows = [r for r in _csv_rows(write_dir, "counter_collection.csv")
                  if r.get("Counter_Name") == "WRITE_SIZE"]
    trace_rows = _csv_rows(trace_dir, "kernel_trace.csv")
    stats = _csv_rows(trace_dir, "kernel_stats.csv")

    def probe(rows):
        v = [float(r["Counter_Value"]) for r in rows if "neg_kernel" in r["Kernel_Name"]]
        if not v:
            raise SystemExit("copy probe kernel not found in the counter output")
        return v[0]
    kib = COPY_PROBE_BYTES / 1024.0
    pf, pw = probe(fetch_rows), probe(write_rows)
    sf, sw = kib / pf, kib / pw
    fetch, nf = _per_eval(fetch_rows, lambda r: (float(r["Counter_Value"]), 1))
    write, nw = _per_eval(write_rows, lambda r: (float(r["Counter_Value"]), 1))
    dur, nt = _per_eval(trace_rows, lambda r: ((int(r["End_Timestamp"]) -
                                                int(r["Start_Timestamp"])) * 1e-3, 1))
    out = ["# HBM traffic and kernel durations: loss + gradient, T=8, d=10, n=2^24, mixed path",
           "", "Commands (run from the repository root on one MI355X):", "", "```"]
    out += cmdline
    out += ["```", "",
            f"Copy probe (torch.neg over {COPY_PROBE_BYTES} B of float32: reads and writes "
            f"{COPY_PROBE_BYTES} B): FETCH_SIZE {pf:.0f} KiB, WRITE_SIZE {pw:.0f} KiB per "
            f"dispatch, so bytes = FETCH_SIZE x 1024 x {sf:.4f} and WRITE_SIZE x 1024 x {sw:.4f}.",
            "", f"Per evaluation (means over {nf} / {nw} / {nt} complete evaluations of the "
            "FETCH, WRITE and trace runs); a phase may hold several kernel launches:", "",
            "| phase | kernels | launches | us (trace) | FETCH KiB | WRITE KiB | HBM bytes (scaled) |",
            "|---|---|---|---|---|---|---|"]
    blob = {"sources_digest": kernel_sources_digest(), "scale_fetch": sf, "scale_write": sw,
            "phases": {}}
    for ph in ("prep", "gen_fwd_low", "fwd_high", "solve", "adj_high", "adj_low_reduce",
               "finalize"):
        if ph not in fetch or ph not in write:
            continue
        b = (fetch[ph][0] * sf + write[ph][0] * sw) * 1024.0
        us = dur[ph][0] if ph in dur else float("nan")
        names = ", ".join(f"`{n[:60]}`" for n in fetch[ph][2])
        out.append(f"| {ph} | {names} | {fetch[ph][1]} | {us:.1f} | {fetch[ph][0]:.0f} | "
                   f"{write[ph][0]:.0f} | {b:.4g} |")
        blob["phases"][ph] = {"hbm_bytes": b, "us": us, "launches": fetch[ph][1]}
    out += ["", "Library kernels in the trace run (rocprofv3 --stats):", "",
            "| kernel | calls | avg us | total ms |", "|---|---|---|---|"]
    for row in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        if "mtgp::" not in row["Name"]:
            continue
        out.append(f"| `{row['Name'].split('(')[0][:90]}` | {row['Calls']} | "
                   f"{float(row['AverageNs']) / 1e3:.1f} | {float(row['TotalDurationNs']) / 1e6:.2f} |")
    out += ["", "```json", json.dumps(blob, indent=1), "```", ""]
    return "\n".join(out)


VALU_KERNELS = ("gen_fwd_kernel", "adj_reduce_kernel")


def valu_summary(pmc_dirs, trace_dir, cmdline):
    """Per-launch means of the counters of several rocprofv3 --pmc runs and
    the launch durations of a trace run, for the two fused evaluation
    kernels, as markdown with a JSON block read back by the benchmark."""
    acc = {k: {} for k in VALU_KERNELS}
    for d in pmc_dirs:
        for r in _csv_rows(d, "counter_collection.csv"):
            k = next((k for k in VALU_KERNELS if k in r["Kernel_Name"]), None)
            if k is None:
                continue
            a = acc[k].setdefault(r["Counter_Name"], [0.0, 0])
            a[0] += float(r["Counter_Value"])
            a[1] += 1
    dur = {k: [] for k in VALU_KERNELS}
    for r in _csv_rows(trace_dir, "kernel_trace.csv"):
        k = next((k for k in VALU_KERNELS if k in r["Kernel_Name"]), None)
        if k is not None:
            dur[k].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    blob = {"sources_digest": kernel_sources_digest(), "kernels": {}}
    out = ["# VALU counters: fused generation and derivative-reduction kernels, "
           "T=8, d=10, n=2^24, mixed path", "",
           "Commands (run from the repository root on one MI355X):", "", "```"]
    out += cmdline
    out += ["```", "",
            "Means per launch (counters summed over the whole GPU by rocprofv3). The issue "
            f"fraction is SQ_INSTS_VALU / (duration x {CU_COUNT} CUs x {CLOCK_HZ / 1e9} GHz): "
            "one wave64 VALU instruction per CU per clock is the issue peak (4 SIMDs x 16 "
            "lanes, 4 clocks per wave64 instruction).", "",
            "| kernel | us (trace) | counter | per launch |", "|---|---|---|---|"]
    for k in VALU_KERNELS:
        if not acc[k]:
            continue
        us = sum(dur[k]) / len(dur[k]) if dur[k] else float("nan")
        e = {c: v[0] / v[1] for c, v in sorted(acc[k].items())}
        e["us"] = us
        if "SQ_INSTS_VALU" in e and dur[k]:
            e["valu_issue_frac"] = e["SQ_INSTS_VALU"] / (us * 1e-6 * CU_COUNT * CLOCK_HZ)
        blob["kernels"][k] = e
        for c, v in e.items():
            if c != "us":
                out.append(f"| `{k}` | {us:.1f} | {c} | {v:.6g} |")
    out += ["", "```json", json.dumps(blob, indent=1), "```", ""]
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--m", type=int, default=24, help="log2 points per task")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precisions", default="fp64,mixed")
    ap.add_argument("--sched", default=None,
                    help="transform schedule a_bits,b_bits,b_tile_bytes (default: library default)")
    ap.add_argument("--train-steps", type=int, default=100,
                    help="Adam steps of the captured training leg (0: skip)")
    ap.add_argument("--no-predict", dest="predict", action="store_false")
    ap.add_argument("--no-transforms", dest="transforms", action="store_false")
    ap.add_argument("--no-lattice", dest="lattice", action="store_false",
                    help="skip the loss+gradient leg on the lattice (FFT) path")
    ap.add_argument("--no-tune", dest="tune", action="store_false",
                    help="keep the library's default schedule instead of the autotuned one")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run every pass in order on one stream (for per-kernel profiles)")
    ap.add_argument("--fits", type=int, default=256, help="fits of the batched leg (0: skip)")
    ap.add_argument("--fit-steps", type=int, default=50)
    ap.add_argument("--pmc-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "TRACE_DIR"))
    ap.add_argument("--valu-summary", nargs="+", metavar="DIR",
                    help="rocprofv3 --pmc output dirs, then the kernel-trace dir")
    ap.add_argument("--pmc-command", action="append", default=[],
                    help="command line recorded in the summary (repeatable)")
    args = ap.parse_args()
    if args.pmc_summary:
        print(pmc_summary(*args.pmc_summary, args.pmc_command))
        return
    if args.valu_summary:
        print(valu_summary(args.valu_summary[:-1], args.valu_summary[-1], args.pmc_command))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the fast MTGP path here runs on a single "
              "MI355X (no multi-GPU sharding is built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    run(args)


if __name__ == "__main__":
    main()
