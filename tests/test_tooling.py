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
