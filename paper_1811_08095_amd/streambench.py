"""Streaming reference rates of the device, beside which the hopping kernel's
traffic is judged.

  python -m paper_1811_08095_amd.streambench --mib 64,128,256,4096

For each buffer size (MiB per FP32 tensor) it times, with CUDA events over
many repetitions after a warm-up, y.copy_(x) (one read and one write stream)
and torch.add(x, y, alpha=0.5, out=y) (two reads, one write).  Buffers of a
few hundred MiB stay in the memory-side cache between repetitions; buffers of
several GiB stream from HBM.  One JSON line per size with the rates in TB/s.
"""
import argparse
import json


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--mib", default="64,128,256,512,4096", help="comma list of MiB per tensor")
    args = ap.parse_args(argv)

    import torch

    dev = torch.device("cuda:0")

    def rate(nbytes, fn, reps):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e12

    for mib in (int(v) for v in args.mib.split(",")):
        n = mib * 2**20 // 4
        x = torch.ones(n, device=dev, dtype=torch.float32)
        y = torch.zeros_like(x)
        reps = max(10, min(2000, 20000 // mib))
        copy = rate(2 * n * 4, lambda: y.copy_(x), reps)
        add = rate(3 * n * 4, lambda: torch.add(x, y, alpha=0.5, out=y), reps)
        print(json.dumps({"mib_per_tensor": mib, "copy_TBs": round(copy, 2), "add_TBs": round(add, 2)}),
              flush=True)
        del x, y


if __name__ == "__main__":
    main()
