"""Microbenchmark of the hopping kernels on one lattice.

  python -m paper_1811_08095_amd.hopbench --dims 64x64x64x64 --Ns 16 --precs fp32,fp16s

Synthetic links (eps = 0.7, seed 0) and Gaussian sources (--nrhs right-hand
sides per launch, one mass) are generated in HBM; for every storage precision
the plain even-odd hop W_eo and the normal operator S_e^dag S_e (four fused
hop launches) are applied after one warm-up,
and the library's own HIP-event timing reports the average launch time and the
algorithmic GB/s of the hop launches.  The block traversal follows the
ODWF_TRAVERSAL and ODWF_XCD environment variables, which are echoed in every
output line.
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--dims", default="64x64x64x64", help="LxxLyxLzxLt")
    ap.add_argument("--Ns", type=int, default=16)
    ap.add_argument("--precs", default="fp32", help="comma list of fp64, fp32, fp16s, bf16s")
    ap.add_argument("--hop-reps", type=int, default=10)
    ap.add_argument("--normal-reps", type=int, default=5)
    ap.add_argument("--nrhs", default="1", help="comma list of right-hand-side counts per launch")
    args = ap.parse_args(argv)

    import torch

    from paper_1811_08095_amd import odwf, synth
    dims = tuple(int(v) for v in args.dims.split("x"))
    U = synth.make_gauge_device(dims, 0.7, 0)
    lat = odwf.Lattice(dims)
    lat.load_gauge(U)
    del U
    sol = odwf.Solver(lat, args.Ns, 1.3, odwf.zolotarev_omega(args.Ns))
    names = {"fp64": odwf.FP64, "fp32": odwf.FP32, "fp16s": odwf.FP16S, "bf16s": odwf.BF16S}
    for nrhs in (int(v) for v in args.nrhs.split(",")):
        psi = synth.make_source_device(dims, args.Ns, nrhs, 5)
        out = torch.empty_like(psi)
        mq = [0.04] * nrhs
        for pname in args.precs.split(","):
            prec = names[pname]
            for op, oname, reps in ((odwf.OP_HOP_EO, "HOP", args.hop_reps),
                                    (odwf.OP_SCHUR_NORMAL, "NORMAL", args.normal_reps)):
                sol.apply(op, psi, mq, prec=prec, out=out)
                torch.cuda.synchronize()
                odwf.profile_enable(True)
                for _ in range(reps):
                    sol.apply(op, psi, mq, prec=prec, out=out)
                n, ms, by = odwf.profile_read()
                odwf.profile_enable(False)
                print(json.dumps({"dims": args.dims, "Ns": args.Ns, "nrhs": nrhs,
                                  "traversal": os.environ.get("ODWF_TRAVERSAL", "default"),
                                  "xcd": os.environ.get("ODWF_XCD", "default"),
                                  "prec": pname, "op": oname,
                                  "launches": n, "avg_ms": round(ms / n, 4),
                                  "GBs": round(by / (ms * 1e-3) / 1e9, 1)}), flush=True)
        del psi, out
        sol.close()
        sol = odwf.Solver(lat, args.Ns, 1.3, odwf.zolotarev_omega(args.Ns))
    sol.close()
    lat.close()


if __name__ == "__main__":
    main()
