"""Measured schedule selection for the digital-net transform passes.

`tune(plan, theta)` times mtgp_nll_grad on the caller's plan and data under
candidate schedules (bits of the LDS pass, bits per high pass, LDS tile
size), overlap chunk counts and caps on the fused kernels' workgroups per
CU, keeps the fastest, applies it to the plan and caches the choice in a
JSON file keyed by the design's shape, precision and device, so a later plan
of the same shape takes it without timing.  Results
do not depend on the schedule beyond rounding order; lattice plans have no
schedule to choose and are left unchanged.
"""
import json
import os

import torch

from . import mtgp

# (pass_a_bits, pass_b_bits, pass_b_tile_bytes): pass_b_bits 0 picks the
# high passes by size; register-resident passes for pass_b_bits <= 6,
# one-pass or LDS-tiled ones above
CANDIDATES = [
    (12, 0, 73728), (12, 6, 36864), (13, 6, 36864), (12, 5, 36864), (12, 4, 36864),
    (11, 6, 36864), (10, 7, 36864), (12, 12, 36864),
]
OVERLAPS = (1, 2, 4, 8, 16)
FINALISTS = 3  # schedules also timed with each overlap setting
# caps on workgroups per CU of the fused generation / reduction kernels,
# tried with the best schedule and the overlapped settings (0: no cap)
FUSED_CAPS = (3,)


def cache_path():
    return os.environ.get("MTGP_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mtgp", "schedules.json"))


def cache_key(plan, device_name):
    return "|".join(str(v) for v in (plan.family, tuple(plan.m), plan.d, plan.precision,
                                     device_name))


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + f".{os.getpid()}.tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time(plan, theta, reps):
    out3 = torch.empty(3, dtype=torch.float64, device="cuda")
    grad = torch.empty(plan.theta_size, dtype=torch.float64, device="cuda")
    tau = torch.empty(plan.T, dtype=torch.float64, device="cuda")
    plan.nll_grad(theta, out3, grad, tau)  # warm-up (and first-touch of a grown workspace)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        plan.nll_grad(theta, out3, grad, tau)
    e1.record(st)
    torch.cuda.synchronize()
    code, bad = plan.status()
    if code != 0:
        raise RuntimeError(f"loss evaluation failed during tuning (status {code} at {bad})")
    return e0.elapsed_time(e1) / reps


def tune(plan, theta, reps=5, candidates=None, overlaps=OVERLAPS, use_cache=True):
    """Choose and apply the fastest schedule; returns dict(schedule, overlap,
    ms, cached, timings)."""
    if plan.family != mtgp.DSEQ:
        return {"schedule": None, "overlap": None, "ms": None, "cached": False, "timings": {}}
    dev = torch.cuda.get_device_name()
    key = cache_key(plan, dev)
    path = cache_path()
    if use_cache:
        hit = _load(path).get(key)
        if hit is not None:
            plan.set_schedule(*hit["schedule"])
            plan.set_overlap(hit["overlap"])
            plan.set_fused_occupancy(hit.get("fused_occupancy", 0))
            return {"schedule": tuple(hit["schedule"]), "overlap": hit["overlap"], "ms": hit["ms"],
                    "fused_occupancy": hit.get("fused_occupancy", 0), "cached": True,
                    "timings": {}}
    cands = list(candidates or CANDIDATES)
    timings = {}
    # every schedule with the passes in sequence, then every overlap setting
    # for the fastest few: a schedule that wins in sequence (one block per CU
    # in its widest pass, say) can lose once passes of several chunks share
    # the CUs
    plan.set_overlap(1)
    seq = []
    for c in cands:
        plan.set_schedule(*c)
        ms = _time(plan, theta, reps)
        timings[str(c)] = ms
        seq.append((ms, c))
    seq.sort(key=lambda x: x[0])
    best = (seq[0][1], 1, seq[0][0])
    for _, c in seq[:FINALISTS]:
        plan.set_schedule(*c)
        for ov in overlaps:
            if ov == 1:
                continue
            plan.set_overlap(ov)
            ms = _time(plan, theta, reps)
            timings[f"{c} overlap {ov}"] = ms
            if ms < best[2]:
                best = (c, ov, ms)
        plan.set_overlap(1)
    plan.set_schedule(*best[0])
    cap_best = 0
    for cap in FUSED_CAPS:
        plan.set_fused_occupancy(cap)
        for ov in sorted({best[1], 2, 8}):
            if ov == 1:
                continue
            plan.set_overlap(ov)
            ms = _time(plan, theta, reps)
            timings[f"{best[0]} overlap {ov} fused cap {cap}"] = ms
            if ms < best[2]:
                best = (best[0], ov, ms)
                cap_best = cap
    plan.set_fused_occupancy(cap_best)
    plan.set_overlap(best[1])
    if use_cache:
        table = _load(path)
        table[key] = {"schedule": list(best[0]), "overlap": best[1], "ms": best[2],
                      "fused_occupancy": cap_best}
        _store(path, table)
    return {"schedule": best[0], "overlap": best[1], "ms": best[2], "fused_occupancy": cap_best,
            "cached": False, "timings": timings}
