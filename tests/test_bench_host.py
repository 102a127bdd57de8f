"""Host logic of bench.py that runs without a GPU: the one-GPU refusal and the
reduction of rocprofv3 counter and trace CSVs to per-evaluation phase bytes."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

EVAL = [  # one loss + gradient evaluation, in dispatch order
    "mtgp::prep_kernel",
    "void mtgp::gen_fwd_kernel<double, double, 2, 10, 16>(double*, long)",
    "void mtgp::fwht_reg_buf_kernel<double, double, double, 6>(double const*, double*)",
    "void mtgp::fwht_reg_buf_kernel<double, double, float, 6>(double const*, float*)",
    "void mtgp::solve_eq_kernel<float, 8, true>(float*, long)",
    "void mtgp::fwht_reg_buf_kernel<double, float, double, 6>(float const*, double*)",
    "void mtgp::fwht_reg_buf_kernel<double, double, double, 6>(double const*, double*)",
    "void mtgp::adj_reduce_kernel<double, double, 2, 10>(double const*, long)",
    "mtgp::colsum_kernel",
    "mtgp::finalize_kernel",
]
PHASE = ["prep", "gen_fwd_low", "fwd_high", "fwd_high", "solve", "adj_high", "adj_high",
         "adj_low_reduce", "finalize", "finalize"]


def _write(path, fields, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        w.writerows(rows)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 2, r.stderr
    assert "one GPU" in r.stderr and r.stdout == ""


def test_counter_summary_per_evaluation(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    probe_kib = bench.COPY_PROBE_BYTES / 1024.0
    # the copy probe reads and writes COPY_PROBE_BYTES; its counters read half
    # (FETCH) and a quarter (WRITE) of that, so the scales are 2 and 4
    fetch, write, trace = [], [], []
    did = 0
    fetch.append(dict(Dispatch_Id=did, Kernel_Name="void at::native::neg_kernel(float)",
                      Counter_Name="FETCH_SIZE", Counter_Value=probe_kib / 2))
    write.append(dict(Dispatch_Id=did, Kernel_Name="void at::native::neg_kernel(float)",
                      Counter_Name="WRITE_SIZE", Counter_Value=probe_kib / 4))
    for e in range(3):  # the third evaluation is cut off before its finalize
        for k, name in enumerate(EVAL if e < 2 else EVAL[:5]):
            did += 1
            fetch.append(dict(Dispatch_Id=did, Kernel_Name=name, Counter_Name="FETCH_SIZE",
                              Counter_Value=100 * (k + 1) + e))
            write.append(dict(Dispatch_Id=did, Kernel_Name=name, Counter_Name="WRITE_SIZE",
                              Counter_Value=10 * (k + 1)))
            trace.append(dict(Dispatch_Id=did, Kernel_Name=name, Start_Timestamp=1000 * did,
                              End_Timestamp=1000 * did + 1000 * (k + 1)))
    cf = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    _write(str(tmp_path / "pf" / "run_counter_collection.csv"), cf, fetch)
    _write(str(tmp_path / "pw" / "run_counter_collection.csv"), cf, write)
    _write(str(tmp_path / "kt" / "run_kernel_trace.csv"),
           ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"], trace)
    _write(str(tmp_path / "kt" / "run_kernel_stats.csv"),
           ["Name", "Calls", "AverageNs", "TotalDurationNs"],
           [dict(Name=n, Calls=2, AverageNs=1000.0, TotalDurationNs=2000.0) for n in EVAL])
    md = bench.pmc_summary(str(tmp_path / "pf"), str(tmp_path / "pw"), str(tmp_path / "kt"),
                           ["cmd"])
    blob = json.loads(md.split("```json", 1)[1].split("```", 1)[0])
    assert abs(blob["scale_fetch"] - 2.0) < 1e-12 and abs(blob["scale_write"] - 4.0) < 1e-12
    assert blob["sources_digest"] == bench.kernel_sources_digest()
    for ph in set(PHASE):
        ks = [k for k, p in enumerate(PHASE) if p == ph]
        # mean over the two complete evaluations (e = 0, 1) of the phase sums
        f = sum(100 * (k + 1) for k in ks) + 0.5 * len(ks)
        w = sum(10 * (k + 1) for k in ks)
        got = blob["phases"][ph]
        assert abs(got["hbm_bytes"] - (2.0 * f + 4.0 * w) * 1024.0) < 1e-6, ph
        assert got["launches"] == len(ks)
        assert abs(got["us"] - sum(k + 1 for k in ks)) < 1e-9, ph


def test_valu_summary_per_launch(tmp_path):
    """Counter means per launch of the two fused kernels over several --pmc
    runs, durations from the trace run, and the issue fraction
    SQ_INSTS_VALU / (duration x CUs x clock)."""
    sys.path.insert(0, ROOT)
    import bench
    gen = "void mtgp::gen_fwd_kernel<double, double, 2, 10, 16>(double*, long)"
    adj = "void mtgp::adj_reduce_kernel<double, double, 2, 10>(double const*, long)"
    other = "void mtgp::solve_eq_kernel<float, 8, true>(float*, long)"
    cf = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    a = [dict(Dispatch_Id=i, Kernel_Name=n, Counter_Name="SQ_INSTS_VALU", Counter_Value=v)
         for i, (n, v) in enumerate([(gen, 100.0), (adj, 300.0), (other, 7.0), (gen, 200.0),
                                     (adj, 500.0)])]
    b = [dict(Dispatch_Id=i, Kernel_Name=n, Counter_Name="VALUBusy", Counter_Value=v)
         for i, (n, v) in enumerate([(gen, 40.0), (adj, 60.0)])]
    _write(str(tmp_path / "a" / "run_counter_collection.csv"), cf, a)
    _write(str(tmp_path / "b" / "run_counter_collection.csv"), cf, b)
    _write(str(tmp_path / "kt" / "run_kernel_trace.csv"),
           ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           [dict(Dispatch_Id=0, Kernel_Name=gen, Start_Timestamp=0, End_Timestamp=2000),
            dict(Dispatch_Id=1, Kernel_Name=adj, Start_Timestamp=0, End_Timestamp=3000),
            dict(Dispatch_Id=2, Kernel_Name=gen, Start_Timestamp=0, End_Timestamp=4000)])
    md = bench.valu_summary([str(tmp_path / "a"), str(tmp_path / "b")], str(tmp_path / "kt"),
                            ["cmd"])
    blob = json.loads(md.split("```json", 1)[1].split("```", 1)[0])
    g, r = blob["kernels"]["gen_fwd_kernel"], blob["kernels"]["adj_reduce_kernel"]
    assert g["SQ_INSTS_VALU"] == 150.0 and r["SQ_INSTS_VALU"] == 400.0
    assert g["VALUBusy"] == 40.0 and r["VALUBusy"] == 60.0
    assert abs(g["us"] - 3.0) < 1e-12 and abs(r["us"] - 3.0) < 1e-12
    assert abs(g["valu_issue_frac"] - 150.0 / (3e-6 * bench.CU_COUNT * bench.CLOCK_HZ)) < 1e-15
    assert bench.VALU_LANE_OPS_PEAK == 256 * 64 * 2.4e9
