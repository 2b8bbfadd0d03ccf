"""Summaries of rocprofv3 CSV output for the profiles/ folder.

  python -m paper_1811_08095_amd.profsum ktrace DIR OUT --cmd "..." [--cycle REGEX --cycle-len N]
      per-kernel call count, average and share from the kernel-trace
      statistics (run_kernel_stats.csv); with --cycle, the dispatches whose
      names match REGEX are taken in start order as a repeating sequence of N
      launches (one solver iteration) and the median duration of each
      position in it is listed (run_kernel_trace.csv)

  python -m paper_1811_08095_amd.profsum traffic --fetch DIR1 --write DIR2 \
      --kernel REGEX --copy-bytes N --workload KEY OUT --cmd-fetch "..." --cmd-write "..."
      HBM-side traffic per dispatch of the kernels matching REGEX from a
      FETCH_SIZE run and a WRITE_SIZE run (KiB per dispatch), each scaled by
      what the same counter reads for the plain device copy of N bytes that the
      profiled program ran (the largest dispatch of a copy kernel); the file
      records the hash of the hopping-kernel sources so that a reader can tell
      whether the numbers still describe the built kernel.

These counters count requests from the L2 caches to the memory fabric, so a
fetch that hits the memory-side cache (MALL) counts as traffic here.
"""
import argparse
import collections
import csv
import glob
import hashlib
import os
import re
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
# the sources that define the hopping kernel, its data layout and its launch shape
HOP_SOURCES = ["csrc/hop.hip", "csrc/dev_common.h", "csrc/odwf_types.h", "csrc/runtime.cpp"]
COPY_RE = re.compile(r"copyBuffer|direct_copy|CatArray|copy_kernel", re.I)


def hop_source_hash():
    h = hashlib.sha256()
    for f in HOP_SOURCES:
        with open(os.path.join(PKG, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _find(d, suffix):
    fs = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not fs:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return fs[0]


def kernel_stats(d):
    rows = list(csv.DictReader(open(_find(d, "kernel_stats.csv"))))
    return [(r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["Percentage"]))
            for r in rows]


def counter_values(d, counter):
    """{kernel name: [value per dispatch]} for one counter."""
    out = collections.defaultdict(list)
    for r in csv.DictReader(open(_find(d, "counter_collection.csv"))):
        if r["Counter_Name"] == counter:
            out[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return out


def cmd_ktrace(a):
    rows = kernel_stats(a.dir)
    lines = [f"# rocprofv3 kernel-trace statistics: {a.title}",
             f"# command: {a.cmd}",
             f"# hop-kernel source hash: {hop_source_hash()}",
             "# avg_us = AverageNs / 1000; top kernels by total time", ""]
    for name, calls, avg_us, pct in rows[:a.top]:
        lines.append(f"{name[:110]:110s} calls={calls:6d} avg_us={avg_us:10.2f} pct={pct:6.2f}")
    if a.cycle:
        lines += [""] + cycle_lines(a.dir, a.cycle, a.cycle_len, a.cycle_skip)
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cycle_lines(d, regex, n, skip):
    """Median duration per position of a repeating launch sequence."""
    rx = re.compile(regex)
    rows = [r for r in csv.DictReader(open(_find(d, "kernel_trace.csv"))) if rx.search(r["Kernel_Name"])]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    rows = rows[skip * n:]
    ncyc = len(rows) // n
    if ncyc == 0:
        raise RuntimeError(f"fewer than {n} dispatches matching {regex} after the skipped cycles")
    out = [f"# launch sequence: dispatches matching {regex!r} in start order, taken as {ncyc} cycles of "
           f"{n} (the first {skip} skipped); median duration per position", ""]
    total = 0.0
    for k in range(n):
        names = collections.Counter(rows[c * n + k]["Kernel_Name"] for c in range(ncyc))
        durs = sorted((int(rows[c * n + k]["End_Timestamp"]) - int(rows[c * n + k]["Start_Timestamp"])) / 1e3
                      for c in range(ncyc))
        med = durs[len(durs) // 2]
        total += med
        name, cnt = names.most_common(1)[0]
        tag = "" if cnt == ncyc else f" (position holds {len(names)} kernels; {cnt} of {ncyc} are this one)"
        out.append(f"position {k}: {name[:100]:100s} median_us={med:10.2f}{tag}")
    out.append(f"sum of the medians per cycle: {total:.2f} us")
    return out


def _copy_factor(vals, nbytes):
    cands = [max(v) for k, v in vals.items() if COPY_RE.search(k) and v]
    if not cands:
        raise RuntimeError("no copy kernel dispatch in the counter output")
    kib = max(cands)
    return nbytes / (kib * 1024.0), kib


def cmd_traffic(a):
    rx = re.compile(a.kernel)
    fv = counter_values(a.fetch, "FETCH_SIZE")
    wv = counter_values(a.write, "WRITE_SIZE")
    ff, fkib = _copy_factor(fv, a.copy_bytes)
    fw, wkib = _copy_factor(wv, a.copy_bytes)
    lines = [f"# HBM-side traffic of {a.kernel} ({a.workload})",
             f"# command (FETCH_SIZE): {a.cmd_fetch}",
             f"# command (WRITE_SIZE): {a.cmd_write}",
             f"# copy calibration: {a.copy_bytes} bytes copied; FETCH_SIZE read {fkib:.1f} KiB "
             f"(factor {ff:.4f}), WRITE_SIZE read {wkib:.1f} KiB (factor {fw:.4f})",
             "# counters: requests from L2 to the memory fabric (memory-side cache hits included)", "",
             "| kernel | dispatches | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | scaled GB/dispatch |",
             "|---|---|---|---|---|"]
    tot_gb, tot_n = 0.0, 0
    for k in sorted(set(fv) | set(wv)):
        if not rx.search(k):
            continue
        f, w = fv.get(k, []), wv.get(k, [])
        if not f or not w:
            continue
        fm, wm = sum(f) / len(f), sum(w) / len(w)
        gb = (fm * 1024 * ff + wm * 1024 * fw) / 1e9
        n = min(len(f), len(w))
        tot_gb += gb * n
        tot_n += n
        lines.append(f"| {k[:90]} | {n} | {fm:.1f} | {wm:.1f} | {gb:.3f} |")
    if not tot_n:
        raise RuntimeError(f"no dispatch of a kernel matching {a.kernel}")
    lines += ["", f"workload: {a.workload}",
              f"traffic_gb_per_launch: {tot_gb / tot_n:.4f}",
              f"launches: {tot_n}",
              f"source_sha256: {hop_source_hash()}"]
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def read_traffic(path, workload):
    """traffic_gb_per_launch from a traffic summary when it was taken for this
    workload on the current hopping-kernel sources, else None."""
    try:
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith(("#", "|")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if kv.get("workload") != workload or kv.get("source_sha256") != hop_source_hash():
            return None
        return float(kv["traffic_gb_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="what", required=True)
    k = sub.add_parser("ktrace")
    k.add_argument("dir")
    k.add_argument("out")
    k.add_argument("--cmd", required=True)
    k.add_argument("--title", default="")
    k.add_argument("--top", type=int, default=20)
    k.add_argument("--cycle", default="")
    k.add_argument("--cycle-len", type=int, default=5)
    k.add_argument("--cycle-skip", type=int, default=1)
    t = sub.add_parser("traffic")
    t.add_argument("out")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    a = ap.parse_args(argv)
    {"ktrace": cmd_ktrace, "traffic": cmd_traffic}[a.what](a)


if __name__ == "__main__":
    sys.exit(main())
