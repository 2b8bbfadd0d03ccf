#!/usr/bin/env python3
"""Benchmark of the even-odd optimal domain-wall CG solve on one MI355X.

Workload (default): the full-size single-GPU lattice 64^3 x 64 with Ns = 16,
synthetic SU(3) links exp(i eps H) with eps = 0.7, m0 = 1.3, omega_s the
optimal weights for lambda in [0.05, 6.2], one Gaussian right-hand side, and
the FULL solve D x = b by even-odd CG on S_e^dag S_e in FP32 with FP64 reliable
updates to a true relative residual of 1e-10.  A step is one complete solve
(source preparation, CG, reconstruction) with the source resident in HBM;
consecutive steps cycle through the masses given by --mq.

The JSON line reports the Dslash (hopping-kernel) HBM bandwidth measured live
with HIP events recorded by the library around every hopping-kernel launch on
its stream, over the timed steps: algorithmic bytes (spinor reads and writes
plus link reads per launch) divided by summed kernel time, against the 8 TB/s
HBM peak, with the copy-calibrated L2-to-fabric traffic per launch when a
counter summary of the same kernel sources is committed.  Beside it: solves/s,
iterations per mass, device memory footprint, the plain FP64 CG on the same
GPU, a plain-hop microbenchmark per precision, a short serving stream (p50/p99
latency), and the FP64 CPU oracle timed on the host cores (its hopping term on
a bounded sample lattice, and the small FP64 solve beside the GPU's).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse_dims(s):
    d = tuple(int(v) for v in s.split(","))
    assert len(d) == 4
    return d


def hop_bytes_plain(dims, Ns, prec_bytes, link_bytes_per_site):
    """Algorithmic bytes of one plain even-odd hop (read input half once, write
    output half once, read the links of both parities' directions once)."""
    V = dims[0] * dims[1] * dims[2] * dims[3]
    h = V // 2
    return 2 * h * Ns * 24 * prec_bytes + h * 8 * link_bytes_per_site


def cpu_baseline(sample_dims, Ns, target_s=12.0):
    """Time the FP64 CPU oracle's hopping term (one even-odd hop over all Ns
    slices) on a bounded sample lattice; GB/s with the same algorithmic byte
    count as the GPU FP64 hop."""
    import numpy as np
    from oracle import oracle
    from paper_1811_08095_amd import synth
    U = synth.make_gauge(sample_dims, 0.7, 0)
    psi = synth.make_source(sample_dims, Ns, 1, 1005)[0]
    w = np.ones(Ns)
    t0 = time.perf_counter()
    oracle.apply(oracle.OP_HOP_EO, U, psi, 1.3, w, 0.0)
    one = time.perf_counter() - t0
    reps = max(1, int(target_s / max(one, 1e-3)))
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.apply(oracle.OP_HOP_EO, U, psi, 1.3, w, 0.0)
    dt = (time.perf_counter() - t0) / reps
    by = hop_bytes_plain(sample_dims, Ns, 8, 144)
    threads = oracle.num_threads()
    return {"value": by / dt / 1e9, "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle even-odd hop W_eo on {'x'.join(map(str, sample_dims))} x Ns={Ns}, "
                      f"{reps} reps of {dt:.3f} s (whole job {one + reps * dt:.1f} s), "
                      f"same algorithmic byte count as the GPU FP64 hop"}


def small_solve_comparison():
    """The plain FP64 configuration (4^4 lattice, Ns = 8, eps = 0.3 links from
    seed 0, m_q = 0.05, one Gaussian source from seed 1000, tol 1e-10): the FP64
    oracle's even-odd CG FULL solve on the host cores beside the GPU's FP64 solve
    of the same system (after one warm-up solve)."""
    import torch
    from oracle import oracle
    from paper_1811_08095_amd import odwf, synth
    dims, Ns, mq = (4, 4, 4, 4), 8, 0.05
    U = synth.make_gauge(dims, 0.3, 0)
    b = synth.make_source(dims, Ns, 1, 1000)
    w = odwf.zolotarev_omega(Ns, 0.05, 6.2)
    t0 = time.perf_counter()
    _, it, _, _ = oracle.solve(U, b[0], 1.3, w, mq / 2.6, oracle.SOLVE_FULL, tol=1e-10)
    cpu_s = time.perf_counter() - t0
    lat = odwf.Lattice(dims, bc_t=-1)
    lat.load_gauge(U)
    sol = odwf.Solver(lat, Ns, 1.3, w)
    bd = torch.from_numpy(b).cuda()
    sol.solve(bd, [mq], [1e-10], inner=odwf.FP64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = sol.solve(bd, [mq], [1e-10], inner=odwf.FP64)
    gpu_s = time.perf_counter() - t0
    sol.close()
    lat.close()
    return {"config": "4x4x4x4, Ns=8, eps=0.3, m_q=0.05, tol 1e-10, FP64 even-odd CG (FULL)",
            "cpu_oracle_s": round(cpu_s, 4), "cpu_oracle_iters": it,
            "gpu_s": round(gpu_s, 4), "gpu_iters": st[0]["iters"]}


def hop_micro(lat, Ns, omega, b, o, mq, stream, warm=3, reps=20):
    """Plain even-odd hop W_eo on the bench lattice, per storage precision:
    3 warm-up launches, then 20 timed launches (HIP events of the library),
    median / min / max launch time and GB/s with the algorithmic byte count.
    `o` is an output buffer of the source's shape (overwritten)."""
    import numpy as np
    from paper_1811_08095_amd import odwf
    out = {}
    sol = odwf.Solver(lat, Ns, 1.3, omega)
    for name, prec in (("fp64", odwf.FP64), ("fp32", odwf.FP32), ("fp16s", odwf.FP16S)):
        for _ in range(warm):
            sol.apply(odwf.OP_HOP_EO, b, [mq], prec=prec, out=o, stream=stream)
        ts, gb = [], 0.0
        for _ in range(reps):
            odwf.profile_enable(True)
            sol.apply(odwf.OP_HOP_EO, b, [mq], prec=prec, out=o, stream=stream)
            n, ms, by = odwf.profile_read()
            odwf.profile_enable(False)
            ts.append(ms / max(n, 1))
            gb = by / max(n, 1) / 1e9
        ts = np.array(ts)
        out[name] = {"median_ms": round(float(np.median(ts)), 4), "min_ms": round(float(ts.min()), 4),
                     "max_ms": round(float(ts.max()), 4), "gb_per_launch": round(gb, 3),
                     "gbs_median": round(gb / (float(np.median(ts)) * 1e-3), 1)}
    sol.close()
    return out


def serving_leg(nreq, rate, inner="fp32"):
    """Serving stream: Poisson arrivals over resident 8^4, 16^4 and 24^4 (Ns = 16,
    eps = 0.5) gauge fields, m_q from {0.005, 0.04, 0.5}, 1-12 right-hand sides
    and tolerance 1e-8 or 1e-10 per request, continuous batching into 12-slot
    multi-RHS engines; latency = completion - arrival (queueing included)."""
    from paper_1811_08095_amd import serve
    lattices = {f"{L}^4": {"dims": (L, L, L, L), "Ns": 16, "eps": 0.5, "seed": 0} for L in (8, 16, 24)}
    srv = serve.Server(lattices, max_slots=12, inner=inner)
    reqs = serve.poisson_stream(nreq, rate, list(lattices))
    t0 = time.perf_counter()
    done = srv.run(reqs)
    out = serve.summarize(done, time.perf_counter() - t0)
    out.update({"arrival_rate": rate, "lattices": list(lattices), "max_slots": 12, "inner": inner})
    for e in srv.engines.values():
        e["batch"].close()
        e["sol"].close()
        e["lat"].close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lattice", default="64,64,64,64", help="Lx,Ly,Lz,Lt")
    ap.add_argument("--Ns", type=int, default=16)
    ap.add_argument("--eps", type=float, default=0.7)
    ap.add_argument("--mq", default="0.04", help="comma-separated masses cycled over steps")
    ap.add_argument("--inner", default="fp32", choices=["fp64", "fp32", "fp16s", "bf16s"])
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--maxiter", type=int, default=100000)
    ap.add_argument("--no-fp64-compare", action="store_true", help="skip the plain FP64 CG comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", default="16,16,16,16")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-stream leg")
    ap.add_argument("--no-hop-micro", action="store_true", help="skip the plain-hop microbenchmark")
    ap.add_argument("--serve-requests", type=int, default=16)
    ap.add_argument("--serve-rate", type=float, default=0.5, help="Poisson arrivals per second")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="run a plain device copy of this size first (the reference dispatch "
                         "for scaling FETCH_SIZE / WRITE_SIZE counters under rocprofv3)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(the multi-GPU halo-exchange path is not part of this build)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1811_08095_amd import odwf, synth

    dims = parse_dims(args.lattice)
    Ns = args.Ns
    masses = [float(m) for m in args.mq.split(",")]
    inner = {"fp64": odwf.FP64, "fp32": odwf.FP32, "fp16s": odwf.FP16S, "bf16s": odwf.BF16S}[args.inner]
    dev = torch.device("cuda:0")
    free0, total = torch.cuda.mem_get_info()
    print(f"# device memory: free {free0/1e9:.1f} GB of {total/1e9:.1f} GB", file=sys.stderr, flush=True)

    if args.copy_calibration_gib > 0:
        nb = int(args.copy_calibration_gib * (1 << 30))
        src = torch.ones(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy calibration: {nb} bytes device to device", file=sys.stderr, flush=True)
        del src, dst
        torch.cuda.empty_cache()

    t0 = time.time()
    U = synth.make_gauge_device(dims, args.eps, 0)
    lat = odwf.Lattice(dims, bc_t=-1)
    lat.load_gauge(U)
    torch.cuda.synchronize()
    del U
    torch.cuda.empty_cache()
    omega = odwf.zolotarev_omega(Ns, 0.05, 6.2)
    sol = odwf.Solver(lat, Ns, 1.3, omega)
    b = synth.make_source_device(dims, Ns, 1, 1005)
    x = torch.empty_like(b)
    torch.cuda.synchronize()
    print(f"# setup {time.time() - t0:.1f} s", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    stats_all = []
    for w in range(args.warmup):
        _, st = sol.solve(b, [masses[w % len(masses)]], [args.tol], inner=inner, maxiter=args.maxiter,
                          x=x, stream=stream)
        print(f"# warmup {w}: {st[0]}", file=sys.stderr, flush=True)
    free1, _ = torch.cuda.mem_get_info()

    odwf.profile_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        mq = masses[k % len(masses)]
        _, st = sol.solve(b, [mq], [args.tol], inner=inner, maxiter=args.maxiter, x=x, stream=stream)
        st[0]["mq"] = mq
        stats_all.append(st[0])
        print(f"# step {k}: mq={mq} iters={st[0]['iters']} ru={st[0]['reliable_updates']} "
              f"resid={st[0]['true_rel_resid']:.2e} full={st[0]['full_rel_resid']:.2e} "
              f"t={st[0]['seconds']:.2f}s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    launches, kms, kbytes = odwf.profile_read()
    inner_k = [odwf.profile_read_kernel(inner, d) for d in (0, 1)]
    odwf.profile_enable(False)
    # dominant kernel: the inner-precision hopping kernel (both instantiations)
    dk_n = sum(k[0] for k in inner_k)
    dk_ms = sum(k[1] for k in inner_k)
    dk_by = sum(k[2] for k in inner_k)
    dk_gbs = dk_by / (dk_ms * 1e-3) / 1e9 if dk_ms > 0 else 0.0

    gbs = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else 0.0
    avg_ms = kms / max(launches, 1)
    # HBM-side traffic per launch of the same kernel, from the committed counter
    # summary of this workload, when it was taken on the current kernel sources
    from paper_1811_08095_amd import profsum
    wkey = f"{'x'.join(map(str, dims))}_Ns{Ns}_{args.inner}_mq{masses[0]}"
    traffic = profsum.read_traffic(os.path.join(ROOT, "profiles", f"hop_kernel_{wkey}_traffic.md"), wkey)
    traffic = round(traffic, 4) if traffic is not None else None
    result = {
        "metric": "EO-ODWF Dslash HBM GB/s; solves/s at 1e-10 resid, mixed vs FP64; p99 latency",
        "value": round(gbs, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_total / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64", "fp16s": "f16+f32+f64", "bf16s": "bf16+f32+f64"}[args.inner],
        "data": "synthetic",
        "config": {"workload": f"EO-ODWF CG solve D x = b, lattice {'x'.join(map(str, dims))} (x,y,z,t), "
                               f"Ns={Ns}, eps={args.eps}, m0=1.3, omega_s Zolotarev [0.05,6.2], "
                               f"1 Gaussian RHS, inner {args.inner} + FP64 reliable updates, tol {args.tol}",
                   "lattice": list(dims), "Ns": Ns, "masses": masses, "inner": args.inner, "tol": args.tol},
        "solves_per_s": round(args.steps / t_total, 4),
        "iters": [s["iters"] for s in stats_all],
        "true_rel_resid": [s["true_rel_resid"] for s in stats_all],
        "full_rel_resid": [s["full_rel_resid"] for s in stats_all],
        "dslash": {"launches": launches, "avg_ms": round(avg_ms, 4), "gbytes": round(kbytes / 1e9, 2),
                   "time_share": round(kms * 1e-3 / t_total, 3)},
        "memory_gb": {"device_total": round(total / 1e9, 1),
                      "used_after_setup_and_warmup": round((total - free1) / 1e9, 1),
                      "gauge_resident": round(lat.nbytes() / 1e9, 2),
                      "solver_workspace_est": round(odwf.footprint(dims, Ns, 1, inner) / 1e9, 2)},
        "roofline": {"bound": "hbm", "achieved": round(dk_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(dk_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "algorithmic_gb_per_launch": round(dk_by / max(dk_n, 1) / 1e9, 4),
                     "kernel": f"hop_kernel<{args.inner}, Ns={Ns}> (W and W^dag instantiations, "
                               f"{dk_n} launches, avg {dk_ms / max(dk_n, 1):.3f} ms)"},
    }
    if not args.no_fp64_compare:
        # a fresh solver: the mixed-precision workspaces are released first, so
        # the FP64 CG's six FP64 half fields fit beside the source and solution
        sol.close()
        torch.cuda.synchronize()
        sol = odwf.Solver(lat, Ns, 1.3, omega)
        print("# plain FP64 CG comparison ...", file=sys.stderr, flush=True)
        odwf.profile_enable(True)
        t1 = time.perf_counter()
        _, st64 = sol.solve(b, [masses[0]], [args.tol], inner=odwf.FP64, maxiter=args.maxiter, x=x,
                            stream=stream)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        n64, ms64, by64 = odwf.profile_read()
        odwf.profile_enable(False)
        print(f"# FP64 CG: {st64[0]['iters']} iterations, {t64:.1f} s", file=sys.stderr, flush=True)
        t_mixed = [s["seconds"] for s in stats_all if s["mq"] == masses[0]]
        result["fp64_compare"] = {"mq": masses[0], "seconds": round(t64, 3), "iters": st64[0]["iters"],
                                  "true_rel_resid": st64[0]["true_rel_resid"],
                                  "speedup_mixed_over_fp64": round(t64 / (sum(t_mixed) / len(t_mixed)), 3)
                                  if t_mixed else None,
                                  "dslash_gbs_fp64": round(by64 / (ms64 * 1e-3) / 1e9, 1) if ms64 > 0 else None,
                                  "dslash_launches": n64}
    if not args.no_hop_micro:
        sol.close()  # the solve workspaces are not needed by the plain hop
        torch.cuda.empty_cache()
        print("# plain-hop microbenchmark ...", file=sys.stderr, flush=True)
        result["hop_micro"] = hop_micro(lat, Ns, omega, b, x, masses[0], stream)
        print(f"# hop: {json.dumps(result['hop_micro'])}", file=sys.stderr, flush=True)
    if not args.no_serving:
        # release the 64^4 fields first: the serving leg has its own resident lattices
        sol.close()
        lat.close()
        del b, x
        torch.cuda.empty_cache()
        print(f"# serving stream: {args.serve_requests} requests at {args.serve_rate}/s ...",
              file=sys.stderr, flush=True)
        result["serving"] = serving_leg(args.serve_requests, args.serve_rate,
                                        inner=args.inner if args.inner in ("fp32", "fp64") else "fp32")
        print(f"# serving: {json.dumps(result['serving'])}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("# CPU oracle baseline ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(parse_dims(args.cpu_sample), Ns)
        result["cpu_baseline"]["solve_small"] = small_solve_comparison()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
