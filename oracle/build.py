"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

The oracle is plain C compiled with gcc; it is loaded only by the tests, the
smoke check and the CPU-baseline leg of the benchmark.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "odwf_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, out: str = LIB, plant: int = 0) -> str:
    """Compile the oracle; plant = k > 0 builds the mutation-test variant with
    planted mistake k (tests only, written to `out`)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-Wno-unused-function", SRC, "-o", out + ".tmp", "-lm"]
    if plant:
        cmd.insert(1, f"-DORACLE_PLANT={int(plant)}")
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


def ensure_built() -> str:
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
