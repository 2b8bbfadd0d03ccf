"""Full solves of one system at several quark masses and inner precisions.

  python -m paper_1811_08095_amd.solvebench --lattice 64,64,64,64 --inner fp32,fp16s,bf16s --mq 0.04

Synthetic links (eps, seed 0) and one Gaussian source (seed 1005) are
generated in HBM, as in bench.py.  For every (inner precision, mass) pair one
FULL solve D x = b to the tolerance runs after the solver's workspaces have
been reserved, timed end to end (source preparation and reconstruction
included) between device synchronisations.  One JSON line per solve:
seconds, iterations, reliable updates or outer steps, the true residual of the
normal system and the full residual |b - D x| / |b|.  Legs whose estimated
time would pass --time-budget (seconds from process start) are skipped and
listed.
"""
import argparse
import json
import os
import sys
import time

T0 = time.perf_counter()
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--lattice", default="64,64,64,64", help="Lx,Ly,Lz,Lt")
    ap.add_argument("--Ns", type=int, default=16)
    ap.add_argument("--eps", type=float, default=0.7)
    ap.add_argument("--inner", default="fp32", help="comma list of fp64, fp32, fp16s, bf16s")
    ap.add_argument("--mq", default="0.04", help="comma list of quark masses")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--time-budget", type=float, default=540.0)
    ap.add_argument("--est-solve", type=float, default=60.0, help="estimated seconds per solve")
    args = ap.parse_args(argv)

    import torch

    from paper_1811_08095_amd import odwf, synth
    dims = tuple(int(v) for v in args.lattice.split(","))
    names = {"fp64": odwf.FP64, "fp32": odwf.FP32, "fp16s": odwf.FP16S, "bf16s": odwf.BF16S}
    U = synth.make_gauge_device(dims, args.eps, 0)
    lat = odwf.Lattice(dims, bc_t=-1)
    lat.load_gauge(U)
    del U
    torch.cuda.empty_cache()
    omega = odwf.zolotarev_omega(args.Ns, 0.05, 6.2)
    b = synth.make_source_device(dims, args.Ns, 1, 1005)
    x = torch.empty_like(b)
    stream = torch.cuda.current_stream()
    skipped = []
    for pname in args.inner.split(","):
        inner = names[pname]
        sol = odwf.Solver(lat, args.Ns, 1.3, omega)
        sol.reserve(1, inner, stream=stream)
        torch.cuda.synchronize()
        for mq in (float(v) for v in args.mq.split(",")):
            est = args.est_solve * (3.0 if inner == odwf.FP64 else 1.0)
            if time.perf_counter() - T0 + est > args.time_budget:
                skipped.append(f"{pname} m_q={mq}")
                continue
            t1 = time.perf_counter()
            _, st = sol.solve(b, [mq], [args.tol], inner=inner, x=x, stream=stream)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            s = st[0]
            print(json.dumps({"lattice": list(dims), "Ns": args.Ns, "inner": pname, "mq": mq, "tol": args.tol,
                              "seconds": round(dt, 3), "iters": s["iters"],
                              "reliable_updates": s["reliable_updates"], "outer_steps": s["outer_steps"],
                              "true_rel_resid": s["true_rel_resid"], "full_rel_resid": s["full_rel_resid"]}),
                  flush=True)
        sol.close()
        torch.cuda.synchronize()
    if skipped:
        print(json.dumps({"skipped_for_time_budget": skipped}), flush=True)


if __name__ == "__main__":
    main()
