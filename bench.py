#!/usr/bin/env python3
"""Benchmark of the even-odd optimal domain-wall Dslash and CG solves on one MI355X.

Workload (default): the full-size single-GPU lattice 64^3 x 64 with Ns = 16,
synthetic SU(3) links exp(i eps H) with eps = 0.7, m0 = 1.3, omega_s the
optimal weights for lambda in [0.05, 6.2], one Gaussian right-hand side (seed
1005), m_q = 0.04, FP32 inner CG with FP64 reliable updates, tolerance 1e-10.

A step is one iteration of that solve: the right-hand side is admitted into a
one-slot batch engine (source preparation in FP64), and every step runs one CG
iteration on S_e^dag S_e -- the four fused hopping launches (W_oe, W_eo, and
their adjoints with the fifth-dimension programs A^{-1}, A^{-dag}, A^dag), the
FP64 reductions and scalar updates, p = r + beta p, and the check for an FP64
reliable update.  --warmup iterations run untimed first; --steps iterations are
timed, bracketed by device synchronisations.

`value` is the Dslash bandwidth over the timed steps: the algorithmic bytes of
one even-odd hop (half 5D spinor in, half 5D spinor out, 12-real FP32 links
read once per site) times the number of FP32 hopping launches, divided by their
summed duration from HIP events the library records around every launch on
its stream.  `roofline` relates it to the 8 TB/s HBM peak; beside it, the
library's fused-stream byte model (the CG vectors the fused launches also move)
and, when a counter summary of the current kernel sources is committed, the
measured L2-to-fabric traffic per launch.

Fixed legs after the steps, each started only if its estimated time fits the
wall-clock budget (--time-budget, counted from process start; a skipped leg is
listed under "skipped"): one complete mixed-precision solve (solves/s,
iterations, residuals), one plain FP64 CG solve of the same system (speedup
and the mixed solution's error against the FP64 solution), the plain-hop
microbenchmark per precision with its error against the FP64 hop, the FP64
CPU oracle on the host cores (the cpu_baseline), and a short serving stream
(p50/p99 latency).
"""
import argparse
import json
import os
import sys
import time

T_PROCESS0 = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Time of each fixed leg on MI355X at 64^3 x 64 x 16 (seconds; measured, with
# margin), used to decide before a leg starts whether it fits in the budget.
# The FP64 solve is estimated from the mixed solve measured in the same run.
LEG_ESTIMATE_S = {
    "setup": 40.0,          # gauge field, resident copies, source
    "admit": 10.0,          # batch engine and source preparation
    "per_step": 0.09,       # one CG iteration
    "mixed_solve": 50.0,
    "hop_micro": 15.0,
    "cpu_baseline": 60.0,
    "fp64_over_mixed": 3.2,  # FP64 solve time / mixed solve time
    "serving": 60.0,
}


def parse_dims(s):
    d = tuple(int(v) for v in s.split(","))
    assert len(d) == 4
    return d


def hop_bytes_plain(dims, Ns, prec_bytes, link_bytes_per_site, nrhs=1, scale_bytes=0):
    """Algorithmic bytes of one even-odd hop: read the opposite-parity half 5D
    spinor once, write the output half once (k right-hand sides), read the 8
    links of every output site once (r_U reals of b_U bytes each), plus the
    per-5D-site scales of the scaled formats."""
    V = dims[0] * dims[1] * dims[2] * dims[3]
    h = V // 2
    return nrhs * 2 * h * Ns * (24 * prec_bytes + scale_bytes) + h * 8 * link_bytes_per_site


def plan(args, est=None, elapsed0=0.0):
    """The legs a run would start, given estimated leg times: list of
    (leg, estimated start s, estimated end s, runs).  Required legs (setup,
    steps) always run; an optional leg runs when it ends inside the budget."""
    e = dict(LEG_ESTIMATE_S if est is None else est)
    t = elapsed0
    out = []
    for leg, dt in (("setup", e["setup"]), ("steps", e["admit"] + e["per_step"] * (args.warmup + args.steps))):
        out.append((leg, t, t + dt, True))
        t += dt
    opt = [("mixed_solve", e["mixed_solve"], args.no_mixed_solve),
           ("fp64_solve", e["mixed_solve"] * e["fp64_over_mixed"], args.no_fp64_compare),
           ("hop_micro", e["hop_micro"], args.no_hop_micro),
           ("cpu_baseline", e["cpu_baseline"], args.no_cpu_baseline),
           ("serving", e["serving"], args.no_serving)]
    for leg, dt, off in opt:
        runs = (not off) and t + dt <= args.time_budget
        out.append((leg, t, t + dt, runs))
        if runs:
            t += dt
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _time_oracle_hop(dims, Ns, target_s, seed_u=0, seed_b=1005):
    """FP64 oracle hop W_eo over all Ns slices: seconds per application."""
    import numpy as np
    from oracle import oracle
    from paper_1811_08095_amd import synth
    U = synth.make_gauge(dims, 0.7, seed_u)
    psi = synth.make_source(dims, Ns, 1, seed_b)[0]
    w = np.ones(Ns)
    t0 = time.perf_counter()
    oracle.apply(oracle.OP_HOP_EO, U, psi, 1.3, w, 0.0)
    one = time.perf_counter() - t0
    reps = max(1, int(target_s / max(one, 1e-3)))
    if reps == 1:
        return one, 1
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.apply(oracle.OP_HOP_EO, U, psi, 1.3, w, 0.0)
    return (time.perf_counter() - t0) / reps, reps


def cpu_baseline(sample_dims, Ns, bench_dims, cg_iters_gpu=None):
    """The FP64 CPU oracle on the host cores (a baseline, not a target):
      - its even-odd hop on the sample lattice (the reported value, GB/s with
        the algorithmic byte count of the GPU FP64 hop) and on 32^4 x Ns;
      - the bench lattice's hop time extrapolated from the 32^4 per-site rate
        (the bench lattice does not fit the oracle's host arrays);
      - its CG on the 16^4 x 16 system (eps 0.5, m_q 0.04, source seed 1001):
        a bounded number of iterations timed, and the whole solve projected
        with the GPU's iteration count for the same system;
      - the plain FP64 configuration (4^4 x 8) solved completely."""
    import numpy as np
    from oracle import oracle
    from paper_1811_08095_amd import synth
    t_all = time.perf_counter()
    dt, reps = _time_oracle_hop(sample_dims, Ns, 8.0)
    by = hop_bytes_plain(sample_dims, Ns, 8, 144)
    threads = oracle.num_threads()
    out = {"value": round(by / dt / 1e9, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"FP64 oracle even-odd hop W_eo on {'x'.join(map(str, sample_dims))} x Ns={Ns}, "
                     f"{reps} reps of {dt:.3f} s, GB/s with the algorithmic byte count of the GPU FP64 "
                     f"hop (spinor in + out, 18-real links)"}
    d32 = (32, 32, 32, 32)
    dt32, _ = _time_oracle_hop(d32, Ns, 0.0)
    V32 = 32 ** 4
    n5_32 = V32 // 2 * Ns
    out["hop_32x32x32x32"] = {"seconds": round(dt32, 3),
                              "gbs": round(hop_bytes_plain(d32, Ns, 8, 144) / dt32 / 1e9, 3),
                              "ns_per_5d_site": round(dt32 / n5_32 * 1e9, 3)}
    Vb = bench_dims[0] * bench_dims[1] * bench_dims[2] * bench_dims[3]
    out["hop_bench_lattice_extrapolated"] = {
        "lattice": "x".join(map(str, bench_dims)), "seconds": round(dt32 * Vb / V32, 2),
        "note": "extrapolated from the 32^4 per-site rate, not run"}
    # 16^4 x 16 FP64 CG: timed iterations, projected whole solve
    d16 = (16, 16, 16, 16)
    U = synth.make_gauge(d16, 0.5, 0)
    b = synth.make_source(d16, 16, 1, 1001)[0]
    w = oracle_omega(16)
    # two bounded runs (source preparation, n iterations, residuals, reconstruction);
    # their difference is the time of the extra iterations
    # (the oracle returns -1 when it stops at maxiter before the tolerance)
    tm = {}
    for n_it in (2, 6):
        t0 = time.perf_counter()
        _, it, _, _ = oracle.solve(U, b, 1.3, w, 0.04 / 2.6, oracle.SOLVE_FULL, tol=1e-10, maxiter=n_it)
        tm[n_it] = time.perf_counter() - t0
        assert it == -1, "the bounded run must stop at maxiter"
    per_it = (tm[6] - tm[2]) / 4
    fixed = tm[2] - 2 * per_it
    cg = {"config": "16^4 x 16, eps 0.5, m_q 0.04, FP64 even-odd CG (FULL)",
          "seconds_per_iter": round(per_it, 4), "seconds_prep_and_reconstruction": round(fixed, 3)}
    if cg_iters_gpu:
        cg["projected_solve_s"] = round(fixed + per_it * cg_iters_gpu, 2)
        cg["projection"] = (f"measured per-iteration time x the GPU FP64 solve's {cg_iters_gpu} "
                            f"iterations of the same system + measured preparation")
    out["cg_16x16x16x16"] = cg
    out["solve_small"] = small_solve_comparison()
    out["job_seconds"] = round(time.perf_counter() - t_all, 1)
    return out


def oracle_omega(Ns):
    from oracle.zolotarev import omega_zolotarev
    return omega_zolotarev(0.05, 6.2, Ns)


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


def gpu_cg16_iters():
    """Iterations of the GPU FP64 solve of the 16^4 x 16 system the CPU
    baseline projects (eps 0.5, m_q 0.04, source seed 1001, tol 1e-10)."""
    import torch
    from paper_1811_08095_amd import odwf, synth
    d16 = (16, 16, 16, 16)
    U = synth.make_gauge(d16, 0.5, 0)
    b = torch.from_numpy(synth.make_source(d16, 16, 1, 1001)).cuda()
    lat = odwf.Lattice(d16, bc_t=-1)
    lat.load_gauge(U)
    sol = odwf.Solver(lat, 16, 1.3, odwf.zolotarev_omega(16, 0.05, 6.2))
    t0 = time.perf_counter()
    _, st = sol.solve(b, [0.04], [1e-10], inner=odwf.FP64)
    dt = time.perf_counter() - t0
    sol.close()
    lat.close()
    return st[0]["iters"], dt


def hop_micro(lat, Ns, omega, b, o, ref, mq, stream, warm=3, reps=20):
    """Plain even-odd hop W_eo on the bench lattice per storage precision: 3
    warm-up launches, 20 timed launches (HIP events of the library), median /
    min / max launch time, GB/s with the algorithmic bytes of one hop and its
    fraction of the HBM peak, and the relative error of the output against the
    FP64 hop (`ref`, a buffer of the source's shape, receives the FP64 output;
    `o` is overwritten)."""
    import numpy as np
    import torch
    from paper_1811_08095_amd import odwf
    out = {}
    sol = odwf.Solver(lat, Ns, 1.3, omega)
    spec = {"fp64": (odwf.FP64, 8, 144, 0), "fp32": (odwf.FP32, 4, 48, 0),
            "fp16s": (odwf.FP16S, 2, 48, 4), "bf16s": (odwf.BF16S, 2, 48, 4)}
    ref_norm = None
    for name, (prec, pb, lb, sb) in spec.items():
        dst = ref if name == "fp64" else o
        for _ in range(warm):
            sol.apply(odwf.OP_HOP_EO, b, [mq], prec=prec, out=dst, stream=stream)
        ts = []
        for _ in range(reps):
            odwf.profile_enable(True)
            sol.apply(odwf.OP_HOP_EO, b, [mq], prec=prec, out=dst, stream=stream)
            n, ms, _ = odwf.profile_read()
            odwf.profile_enable(False)
            ts.append(ms / max(n, 1))
        ts = np.array(ts)
        by = hop_bytes_plain(lat.dims, Ns, pb, lb, scale_bytes=sb)
        med = float(np.median(ts))
        rec = {"median_ms": round(med, 4), "min_ms": round(float(ts.min()), 4),
               "max_ms": round(float(ts.max()), 4), "algorithmic_gb": round(by / 1e9, 3),
               "gbs_median": round(by / (med * 1e-3) / 1e9, 1),
               "frac_of_hbm_peak": round(by / (med * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        torch.cuda.synchronize()
        if name == "fp64":
            ref_norm = float(torch.linalg.vector_norm(ref))
        else:
            o.sub_(ref)
            rec["rel_err_vs_fp64"] = float(torch.linalg.vector_norm(o)) / ref_norm
        out[name] = rec
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
    out = serve.summarize(done, time.perf_counter() - t0, srv.admission)
    out.update({"arrival_rate": rate, "lattices": list(lattices), "max_slots": 12, "inner": inner})
    srv.close()
    return out


def log(msg):
    print(f"# [{time.perf_counter() - T_PROCESS0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed CG iterations")
    ap.add_argument("--warmup", type=int, default=5, help="untimed CG iterations before the timed ones")
    ap.add_argument("--lattice", default="64,64,64,64", help="Lx,Ly,Lz,Lt")
    ap.add_argument("--Ns", type=int, default=16)
    ap.add_argument("--eps", type=float, default=0.7)
    ap.add_argument("--mq", type=float, default=0.04)
    ap.add_argument("--inner", default="fp32", choices=["fp64", "fp32"],
                    help="inner precision of the stepped solve and the mixed solve")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--maxiter", type=int, default=100000)
    ap.add_argument("--time-budget", type=float, default=480.0,
                    help="seconds from process start within which optional legs must end")
    ap.add_argument("--no-mixed-solve", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true", help="skip the plain FP64 CG solve")
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
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1811_08095_amd import odwf, synth

    dims = parse_dims(args.lattice)
    Ns = args.Ns
    inner = {"fp64": odwf.FP64, "fp32": odwf.FP32}[args.inner]
    link_b = 144 if inner == odwf.FP64 else 48
    prec_b = 8 if inner == odwf.FP64 else 4
    dev = torch.device("cuda:0")
    free0, total = torch.cuda.mem_get_info()
    log(f"device memory: free {free0/1e9:.1f} GB of {total/1e9:.1f} GB")
    skipped = {}

    def budget_ok(leg, est):
        left = args.time_budget - (time.perf_counter() - T_PROCESS0)
        if est > left:
            skipped[leg] = f"estimated {est:.0f} s, {max(left, 0):.0f} s of the {args.time_budget:.0f} s budget left"
            log(f"skip {leg}: {skipped[leg]}")
            return False
        return True

    if args.copy_calibration_gib > 0:
        nb = int(args.copy_calibration_gib * (1 << 30))
        src = torch.ones(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nb} bytes device to device")
        del src, dst
        torch.cuda.empty_cache()

    t0 = time.perf_counter()
    U = synth.make_gauge_device(dims, args.eps, 0)
    lat = odwf.Lattice(dims, bc_t=-1)
    lat.load_gauge(U)
    torch.cuda.synchronize()
    del U
    torch.cuda.empty_cache()
    omega = odwf.zolotarev_omega(Ns, 0.05, 6.2)
    sol = odwf.Solver(lat, Ns, 1.3, omega)
    b = synth.make_source_device(dims, Ns, 1, 1005)
    torch.cuda.synchronize()
    log(f"setup {time.perf_counter() - t0:.1f} s")
    stream = torch.cuda.current_stream()

    # ---- steps: CG iterations of the warmed-up solve -------------------------
    t0 = time.perf_counter()
    batch = odwf.Batch(sol, 1, inner=inner)
    slot = batch.admit(b[0], args.mq, args.tol, maxiter=args.maxiter, stream=stream)
    for _ in range(args.warmup):
        batch.step(1, stream=stream)
    torch.cuda.synchronize()
    log(f"batch engine, source preparation and {args.warmup} warm-up iterations: "
        f"{time.perf_counter() - t0:.1f} s")
    free1, _ = torch.cuda.mem_get_info()
    odwf.profile_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        batch.step(1, stream=stream)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    kr = [odwf.profile_read_kernel(inner, d) for d in (0, 1)]
    odwf.profile_enable(False)
    done, st_steps = batch.poll(slot, stream=stream)
    batch.close()
    if done:
        print(f"the solve converged within the {args.warmup + args.steps} iterations: lower --steps "
              f"(one step is one iteration of a solve that needs {st_steps['iters']})", file=sys.stderr)
        sys.exit(3)
    n_hop = sum(k[0] for k in kr)
    ms_hop = sum(k[1] for k in kr)
    by_fused = sum(k[2] for k in kr)
    by_plain = hop_bytes_plain(dims, Ns, prec_b, link_b)
    gbs = by_plain * n_hop / (ms_hop * 1e-3) / 1e9 if ms_hop > 0 else 0.0
    gbs_fused = by_fused / (ms_hop * 1e-3) / 1e9 if ms_hop > 0 else 0.0
    log(f"{args.steps} steps: {1e3 * t_total / args.steps:.2f} ms per CG iteration, {n_hop} hop launches "
        f"avg {ms_hop / max(n_hop, 1):.3f} ms, Dslash {gbs:.0f} GB/s")

    from paper_1811_08095_amd import profsum
    wkey = f"{'x'.join(map(str, dims))}_Ns{Ns}_{args.inner}_mq{args.mq}"
    traffic = profsum.read_traffic(os.path.join(ROOT, "profiles", f"hop_kernel_{wkey}_traffic.md"), wkey)
    traffic = round(traffic, 4) if traffic is not None else None
    pname = {odwf.FP64: "SP64", odwf.FP32: "SP32"}[inner]
    result = {
        "metric": "EO-ODWF Dslash HBM GB/s; solves/s at 1e-10 resid, mixed vs FP64; p99 latency",
        "value": round(gbs, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_total / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32+f64"}[args.inner],
        "data": "synthetic",
        "config": {"workload": f"EO-ODWF CG on S_e^dag S_e, lattice {'x'.join(map(str, dims))} (x,y,z,t), "
                               f"Ns={Ns}, eps={args.eps}, m0=1.3, omega_s Zolotarev [0.05,6.2], "
                               f"1 Gaussian RHS, m_q={args.mq}, inner {args.inner} + FP64 reliable "
                               f"updates, tol {args.tol}; one step = one CG iteration",
                   "lattice": list(dims), "Ns": Ns, "mq": args.mq, "inner": args.inner, "tol": args.tol},
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "algorithmic_gb_per_launch": round(by_plain / 1e9, 4),
                     "kernel": f"hop_kernel<{pname}, {Ns}, dag, false> (W and W^dag instantiations of the "
                               f"CG iteration)",
                     "launches": n_hop, "avg_ms": round(ms_hop / max(n_hop, 1), 4),
                     "fused_stream_model": {
                         "gb_per_launch": round(by_fused / max(n_hop, 1) / 1e9, 3),
                         "gbs": round(gbs_fused, 1), "frac": round(gbs_fused / HBM_PEAK_GBS, 4),
                         "note": "bytes of the hop plus the CG vectors the fused launches read and write"}},
        "step_state": {"iters": st_steps["iters"], "reliable_updates": st_steps["reliable_updates"],
                       "iterated_rel_resid": st_steps["true_rel_resid"]},
        "memory_gb": {"device_total": round(total / 1e9, 1),
                      "used_with_stepped_engine": round((total - free1) / 1e9, 1),
                      "gauge_resident": round(lat.nbytes() / 1e9, 2),
                      "solve_workspace": round(odwf.footprint(dims, Ns, 1, inner) / 1e9, 2)},
    }

    x = None
    t_mixed = None
    if not args.no_mixed_solve and budget_ok("mixed_solve", LEG_ESTIMATE_S["mixed_solve"]):
        x = torch.empty_like(b)
        # the solver's workspaces are allocated first, so the timed solve
        # measures the solve and not the device allocation
        sol.reserve(1, inner, stream=stream)
        torch.cuda.synchronize()
        log("mixed-precision solve ...")
        odwf.profile_enable(True)
        t1 = time.perf_counter()
        _, st = sol.solve(b, [args.mq], [args.tol], inner=inner, maxiter=args.maxiter, x=x, stream=stream)
        torch.cuda.synchronize()
        t_mixed = time.perf_counter() - t1
        n, ms, _ = odwf.profile_read()
        kr = [odwf.profile_read_kernel(inner, d) for d in (0, 1)]
        odwf.profile_enable(False)
        nk, msk = sum(k[0] for k in kr), sum(k[1] for k in kr)
        s0 = st[0]
        result["solve"] = {"inner": args.inner, "seconds": round(t_mixed, 3),
                           "solves_per_s": round(1.0 / t_mixed, 5), "iters": s0["iters"],
                           "reliable_updates": s0["reliable_updates"],
                           "true_rel_resid": s0["true_rel_resid"], "full_rel_resid": s0["full_rel_resid"],
                           "dslash_gbs": round(by_plain * nk / (msk * 1e-3) / 1e9, 1) if msk > 0 else None,
                           "hop_time_share": round(ms * 1e-3 / t_mixed, 3)}
        result["solves_per_s"] = result["solve"]["solves_per_s"]
        free2, _ = torch.cuda.mem_get_info()
        result["memory_gb"]["used_in_mixed_solve"] = round((total - free2) / 1e9, 1)
        log(f"mixed solve: {s0['iters']} iterations, {t_mixed:.1f} s, resid {s0['true_rel_resid']:.2e}")

    est64 = (t_mixed if t_mixed else LEG_ESTIMATE_S["mixed_solve"]) * LEG_ESTIMATE_S["fp64_over_mixed"]
    if not args.no_fp64_compare and budget_ok("fp64_solve", est64):
        # a fresh solver: the mixed-precision workspaces are released first; the
        # solution overwrites the source (the last leg that reads it), so the
        # mixed solution, the FP64 solution and the FP64 workspace fit together
        sol.close()
        torch.cuda.synchronize()
        sol = odwf.Solver(lat, Ns, 1.3, omega)
        x64 = b
        sol.reserve(1, odwf.FP64, stream=stream)  # workspaces first, as for the mixed solve
        torch.cuda.synchronize()
        log("plain FP64 CG solve ...")
        odwf.profile_enable(True)
        t1 = time.perf_counter()
        _, st64 = sol.solve(b, [args.mq], [args.tol], inner=odwf.FP64, maxiter=args.maxiter, x=x64,
                            stream=stream)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t1
        kr = [odwf.profile_read_kernel(odwf.FP64, d) for d in (0, 1)]
        odwf.profile_enable(False)
        nk, msk = sum(k[0] for k in kr), sum(k[1] for k in kr)
        rec = {"mq": args.mq, "seconds": round(t64, 3), "iters": st64[0]["iters"],
               "true_rel_resid": st64[0]["true_rel_resid"], "full_rel_resid": st64[0]["full_rel_resid"],
               "dslash_gbs_fp64": round(hop_bytes_plain(dims, Ns, 8, 144) * nk / (msk * 1e-3) / 1e9, 1)
               if msk > 0 else None}
        if t_mixed:
            rec["speedup_mixed_over_fp64"] = round(t64 / t_mixed, 3)
            x.sub_(x64)
            rec["mixed_solution_rel_err_vs_fp64"] = float(torch.linalg.vector_norm(x)) / float(
                torch.linalg.vector_norm(x64))
        result["fp64_compare"] = rec
        free3, _ = torch.cuda.mem_get_info()
        result["memory_gb"]["used_in_fp64_solve"] = round((total - free3) / 1e9, 1)
        del x64
        log(f"FP64 solve: {st64[0]['iters']} iterations, {t64:.1f} s")

    if not args.no_hop_micro and budget_ok("hop_micro", LEG_ESTIMATE_S["hop_micro"]):
        sol.close()  # the solve workspaces are not needed by the plain hop
        sol = odwf.Solver(lat, Ns, 1.3, omega)
        # input: the source field (after the FP64 leg, which solves in place,
        # its solution); the mixed solution's buffer is no longer needed
        o = x if x is not None else torch.empty_like(b)
        x = None
        ref = torch.empty_like(b)
        log("plain-hop microbenchmark ...")
        result["hop_micro"] = hop_micro(lat, Ns, omega, b, o, ref, args.mq, stream)
        del o, ref
        torch.cuda.empty_cache()
        log(f"hop: {json.dumps(result['hop_micro'])}")

    if not args.no_cpu_baseline and budget_ok("cpu_baseline", LEG_ESTIMATE_S["cpu_baseline"]):
        log("CPU oracle baseline ...")
        it16, s16 = gpu_cg16_iters()
        result["cpu_baseline"] = cpu_baseline(parse_dims(args.cpu_sample), Ns, dims, cg_iters_gpu=it16)
        result["cpu_baseline"]["cg_16x16x16x16"]["gpu_fp64_solve_s"] = round(s16, 3)
        log(f"cpu baseline: {json.dumps(result['cpu_baseline'])}")

    if not args.no_serving and budget_ok("serving", LEG_ESTIMATE_S["serving"]):
        sol.close()
        lat.close()
        del b, x
        torch.cuda.empty_cache()
        log(f"serving stream: {args.serve_requests} requests at {args.serve_rate}/s ...")
        result["serving"] = serving_leg(args.serve_requests, args.serve_rate, inner=args.inner)
        log(f"serving: {json.dumps(result['serving'])}")
    result["skipped"] = skipped
    result["wall_s"] = round(time.perf_counter() - T_PROCESS0, 1)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
