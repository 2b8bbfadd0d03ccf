"""Host-side tooling: the benchmark's one-GPU guard and the rocprofv3 counter
summary behind the bench line's `traffic` field (CPU only)."""
import os
import subprocess
import sys

from paper_1811_08095_amd import profsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def _counter_csv(path, rows):
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (k, c, v) in enumerate(rows):
            f.write(f'{i},"{k}",{c},{v}\n')


def test_traffic_summary_calibration_and_hash_guard(tmp_path):
    hop = "void odwf::hop_kernel<odwf::SP32, 16, false, false>(odwf::HopArgs)"
    copy = "__amd_rocclr_copyBuffer"
    fd, wd = tmp_path / "f", tmp_path / "w"
    fd.mkdir()
    wd.mkdir()
    # the copy of 4 GiB reads as 2 GiB of FETCH_SIZE and 4 GiB of WRITE_SIZE (KiB)
    _counter_csv(fd / "run_counter_collection.csv",
                 [(copy, "FETCH_SIZE", 2 * 1024 * 1024), (hop, "FETCH_SIZE", 10.0e6),
                  (hop, "FETCH_SIZE", 30.0e6)])
    _counter_csv(wd / "run_counter_collection.csv",
                 [(copy, "WRITE_SIZE", 4 * 1024 * 1024), (hop, "WRITE_SIZE", 5.0e6),
                  (hop, "WRITE_SIZE", 5.0e6)])
    out = tmp_path / "traffic.md"
    profsum.main(["traffic", str(out), "--fetch", str(fd), "--write", str(wd), "--kernel", "hop_kernel",
                  "--copy-bytes", str(4 << 30), "--workload", "wk", "--cmd-fetch", "a", "--cmd-write", "b"])
    # per launch: fetch mean 20e6 KiB x 2, write 5e6 KiB x 1 (the summary keeps 4 decimals of a GB)
    expect = (20.0e6 * 1024 * 2 + 5.0e6 * 1024) / 1e9
    got = profsum.read_traffic(str(out), "wk")
    assert abs(got - expect) < 1e-4
    assert profsum.read_traffic(str(out), "other workload") is None
    stale = out.read_text().replace(profsum.hop_source_hash(), "0000000000000000")
    out.write_text(stale)
    assert profsum.read_traffic(str(out), "wk") is None


def test_launch_cycle_summary(tmp_path):
    # two warm-up-like cycles, then three regular ones; an unrelated kernel in between
    seq = ["k1", "k1", "k2", "k2", "xp"]
    rows, t = [], 0
    for c in range(5):
        for k, n in enumerate(seq):
            rows.append((f"hop<{n}>" if n != "xp" else "xpby", t, t + 1000 * (k + 1) * (3 if c == 0 else 1)))
            t += 10_000
        rows.append(("other", t, t + 50_000))
        t += 60_000
    with open(tmp_path / "run_kernel_trace.csv", "w") as f:
        f.write("Kernel_Name,Start_Timestamp,End_Timestamp\n")
        for n, a, b in reversed(rows):  # order must come from the timestamps
            f.write(f'"{n}",{a},{b}\n')
    out = profsum.cycle_lines(str(tmp_path), r"hop<|xpby", 5, 1)
    pos = [ln for ln in out if ln.startswith("position")]
    assert len(pos) == 5
    assert "hop<k1>" in pos[0] and "xpby" in pos[4]
    assert [float(ln.split("median_us=")[1].split()[0]) for ln in pos] == [1.0, 2.0, 3.0, 4.0, 5.0]
    assert out[-1].endswith("15.00 us")


def test_committed_bench_line_keeps_the_contract():
    """The recorded bench line carries every field of the benchmark contract,
    with the roofline and CPU-baseline objects complete and self-consistent."""
    import json
    d = json.load(open(os.path.join(ROOT, "profiles", "bench_64x64x64x64_Ns16_mixed_cg.json")))
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["unit"] == "GB/s" and d["higher_is_better"] is True
    assert "workload" in d["config"] and "model" not in d["config"]
    rf = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rf, k
    assert rf["bound"] == "hbm" and rf["peak"] == 8000.0 and rf["unit"] == "GB/s"
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    cb = d["cpu_baseline"]
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in cb, k
    assert cb["kind"] == "oracle" and cb["cores"] >= 1


def _bench_args(argv):
    """Parse bench.py's arguments without running it."""
    import argparse
    import bench
    ns = argparse.Namespace(steps=20, warmup=5, time_budget=480.0, no_mixed_solve=False, no_hop_micro=False,
                            no_cpu_baseline=False, no_fp64_compare=False, no_serving=False)
    it = iter(argv)
    for a in it:
        key = a.lstrip("-").replace("-", "_")
        if key in ("steps", "warmup"):
            setattr(ns, key, int(next(it)))
        elif key == "time_budget":
            ns.time_budget = float(next(it))
    return bench, ns


def test_bench_plan_fits_the_driver_limit():
    """The driver's command (--steps 20 --warmup 5, killed at 600 s) plans to
    finish inside 400 s with the committed per-leg estimates, even after a slow
    first import of torch (90 s), and every leg of the default run is planned."""
    bench, ns = _bench_args(["--steps", "20", "--warmup", "5"])
    legs = bench.plan(ns, elapsed0=0.0)
    assert all(run for _, _, _, run in legs), legs
    assert legs[-1][2] <= 400.0, legs
    slow = bench.plan(ns, elapsed0=90.0)
    assert max(end for _, _, end, run in slow if run) <= ns.time_budget < 600.0
    # required legs run even when nothing else fits
    tight = bench.plan(_bench_args(["--time-budget", "10"])[1])
    assert [leg for leg, _, _, run in tight if run] == ["setup", "steps"]


def test_bench_budget_skips_a_leg_that_would_overrun():
    """Optional legs whose estimate would end past the budget are not started."""
    bench, ns = _bench_args(["--time-budget", "200"])
    legs = {leg: run for leg, _, _, run in bench.plan(ns)}
    assert legs["mixed_solve"] and legs["hop_micro"]
    assert not legs["fp64_solve"]
