"""Multi-mass solve against one solve per mass, on one GPU.

  python -m paper_1811_08095_amd.massbench --dims 64,64,64,8 --Ns 16 --inner fp32

One Gaussian source (seed 1006) on synthetic links (eps = 0.7, seed 0), the
masses of the HMC forces (Hasenbusch 0.01 and 0.1, m_ud, m_s, m_c and the
Pauli-Villars mass 2 m0 = 2.6): the even-odd normal systems
S_e(m)^dag S_e(m) y = b_e are solved for all of them in one
multi-right-hand-side CG (every link load serves every mass), then one
mass per launch (both through odwf_solve_masses, per_launch = nmass and 1).
Printed as one JSON line: wall time, hopping-kernel launches, their time and
algorithmic bytes (from the library's HIP-event profiler), the per-mass
iterations of both ways, and which of the two the library picks by itself
(per_launch = 0); the link bytes a shared launch saves are the link reads of
the per-mass launches it does not repeat.  The default lattice is the per-GPU share of the paper's eight-GPU
split of 64^3 x 64 (64^3 x 8 x 16).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MASSES = [0.01, 0.1, 0.0025, 0.04, 0.5, 2.6]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--dims", default="64,64,64,8", help="Lx,Ly,Lz,Lt")
    ap.add_argument("--Ns", type=int, default=16)
    ap.add_argument("--inner", default="fp32", choices=["fp64", "fp32", "fp16s", "bf16s"])
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--masses", default=",".join(str(m) for m in MASSES))
    args = ap.parse_args(argv)

    import torch

    from paper_1811_08095_amd import odwf, synth
    dims = tuple(int(v) for v in args.dims.split(","))
    masses = [float(m) for m in args.masses.split(",")]
    inner = {"fp64": odwf.FP64, "fp32": odwf.FP32, "fp16s": odwf.FP16S, "bf16s": odwf.BF16S}[args.inner]
    U = synth.make_gauge_device(dims, 0.7, 0)
    lat = odwf.Lattice(dims, bc_t=-1)
    lat.load_gauge(U)
    del U
    omega = odwf.zolotarev_omega(args.Ns, 0.05, 6.2)
    b = synth.make_source_device(dims, args.Ns, 1, 1006)
    out = {"workload": f"multi-mass EO_NORMAL solves, lattice {'x'.join(map(str, dims))} x Ns={args.Ns}, "
                       f"eps 0.7, inner {args.inner}, tol {args.tol}", "masses": masses}

    def run(fn):
        odwf.profile_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        n, ms, by = odwf.profile_read()
        odwf.profile_enable(False)
        return st, {"seconds": round(dt, 3), "hop_launches": n, "hop_ms": round(ms, 1),
                    "hop_gbytes": round(by / 1e9, 1)}

    nm = len(masses)
    for name, per in (("shared_launches", nm), ("one_mass_per_launch", 1)):
        sol = odwf.Solver(lat, args.Ns, 1.3, omega)
        sol.reserve(per, inner)
        y = torch.zeros(sol.packed_even_shape(nm), dtype=torch.complex128, device=b.device)
        st, rec = run(lambda: sol.solve_masses(b, masses, args.tol, inner=inner, y=y, per_launch=per)[1])
        rec["iters"] = [s["iters"] for s in st]
        rec["true_rel_resid"] = [s["true_rel_resid"] for s in st]
        out[name] = rec
        print(f"# {name}: {json.dumps(rec)}", file=sys.stderr, flush=True)
        sol.close()
        del y
    half32 = dims[0] * dims[1] * dims[2] * dims[3] // 2 * args.Ns * 96
    out["library_choice"] = "one_mass_per_launch" if half32 > (256 << 20) else "shared_launches"
    V = dims[0] * dims[1] * dims[2] * dims[3]
    lb = 48 if inner != odwf.FP64 else 144  # link bytes per site and direction
    out["link_gbytes_per_hop"] = round(V // 2 * 8 * lb / 1e9, 3)
    out["speedup_shared"] = round(out["one_mass_per_launch"]["seconds"] / out["shared_launches"]["seconds"], 3)
    lat.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
