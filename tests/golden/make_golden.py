"""Writes the stored expected values under tests/golden/ by calling only the
oracle (oracle/zolotarev.py).  Run from the repository root:
    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.zolotarev import omega_zolotarev, sign_approx  # noqa: E402


def omega_file():
    lines = [
        "# Optimal weights omega_s for lambda in [0.05, 6.2] (paper §2: lambda_max/lambda_min",
        "# = 6.20/0.05, R5-symmetric weights, Ns = 2n), written by tests/golden/make_golden.py",
        "# from the oracle's closed form.  Columns: Ns, s (1-based), omega_s, then one line per",
        "# Ns with the maximum of 1 - S(lambda) on a 2e6-point grid (the 2 d_Z/(1+d_Z) bound).",
    ]
    for Ns in (4, 8, 16):
        w = omega_zolotarev(0.05, 6.2, Ns)
        for s, v in enumerate(w, 1):
            lines.append(f"omega {Ns} {s} {v:.15e}")
        lam = np.linspace(0.05, 6.2, 2000001)
        lines.append(f"maxdev {Ns} {np.max(1 - sign_approx(lam, w)):.10e}")
    with open(os.path.join(HERE, "omega_zolotarev.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    omega_file()
