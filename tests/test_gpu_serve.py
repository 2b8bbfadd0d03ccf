"""The serving loop end to end on the GPU: a small Poisson stream over two
resident lattices; every request converges to its tolerance, finished
results are checked against the FP64 oracle, and the statistics are sane."""
import numpy as np
import pytest

from oracle import oracle
from paper_1811_08095_amd import synth
from paper_1811_08095_amd.serve import Server, poisson_stream, summarize

pytestmark = pytest.mark.gpu


def test_serving_stream_small():
    lattices = {"4^4": {"dims": (4, 4, 4, 4), "Ns": 8, "eps": 0.5, "seed": 0},
                "6x4x4x4": {"dims": (6, 4, 4, 4), "Ns": 8, "eps": 0.5, "seed": 1}}
    srv = Server(lattices, max_slots=6, inner="fp32", iters_per_step=3)
    reqs = poisson_stream(10, 50.0, list(lattices), nrhs_range=(1, 4), seed=11)
    done = srv.run(reqs, time_limit=120, keep_solutions=True)
    assert len(done) == 10
    s = summarize(done, max(r.finished for r in done))
    assert s["all_converged"] and s["p99_latency_s"] >= s["p50_latency_s"] > 0
    # spot-check two requests against the oracle: D x = b with the request's mass
    for r in done[:2]:
        spec = lattices[r.lattice]
        U = synth.make_gauge_device(spec["dims"], spec["eps"], spec["seed"]).cpu().numpy()
        b = synth.make_source_device(spec["dims"], spec["Ns"], r.nrhs, r.seed).cpu().numpy()
        x = r.x.cpu().numpy()
        w = srv.engines[r.lattice]["sol"].omega
        for i in range(r.nrhs):
            Dx = oracle.apply(oracle.OP_D, U, x[i], 1.3, w, r.mq / 2.6)
            assert np.linalg.norm(b[i] - Dx) / np.linalg.norm(b[i]) < 1e3 * r.tol
