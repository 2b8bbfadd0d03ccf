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
