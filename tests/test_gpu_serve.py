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


def test_memory_budget_defers_a_request_until_an_engine_is_evicted():
    """A budget that holds one engine but not two: a request for the second
    lattice waits while the first lattice's engine is busy, is admitted after
    that engine drains and is evicted, and its result equals the same solve
    done directly (and meets the oracle's residual)."""
    import torch
    from paper_1811_08095_amd import odwf
    from paper_1811_08095_amd.serve import Request
    lattices = {"A": {"dims": (4, 4, 4, 4), "Ns": 8, "eps": 0.5, "seed": 0},
                "B": {"dims": (4, 4, 2, 4), "Ns": 8, "eps": 0.5, "seed": 2}}
    fa = odwf.batch_footprint((4, 4, 4, 4), 8, 4, odwf.FP32)
    fb = odwf.batch_footprint((4, 4, 2, 4), 8, 4, odwf.FP32)
    srv = Server(lattices, max_slots=4, inner="fp32", iters_per_step=2, hbm_budget=max(fa, fb) * 1.2)
    reqs = [Request(0, "A", 0.05, 3, 1e-10, 0.0, seed=101), Request(1, "B", 0.5, 2, 1e-10, 0.0, seed=102),
            Request(2, "A", 0.04, 1, 1e-10, 0.0, seed=103)]
    done = srv.run(reqs, time_limit=120, keep_solutions=True)
    assert len(done) == 3
    adm = srv.admission
    print(f"deferred {adm.deferred_for_memory}, evictions {adm.evictions}, peak {adm.peak_bytes}, "
          f"budget {adm.budget:.0f}, measured engine bytes {srv.engine_bytes_measured}")
    assert adm.deferred_for_memory >= 1 and adm.evictions >= 1
    assert adm.peak_bytes <= adm.budget
    for name, nb in srv.engine_bytes_measured.items():
        assert nb == adm.engine_bytes[name]  # the footprint the admission used is what was allocated
    rb = next(r for r in done if r.lattice == "B")
    assert rb.deferred and rb.admitted > 0
    ra = [r for r in done if r.lattice == "A"]
    assert rb.admitted >= max(r.finished for r in ra if r.rid == 0) - 1e-9
    # the deferred request's result: the same system solved directly
    spec = lattices["B"]
    U = synth.make_gauge_device(spec["dims"], spec["eps"], spec["seed"])
    lat = odwf.Lattice(spec["dims"], bc_t=-1)
    lat.load_gauge(U)
    sol = odwf.Solver(lat, 8, 1.3, odwf.zolotarev_omega(8, 0.05, 6.2))
    b = synth.make_source_device(spec["dims"], 8, 2, rb.seed)
    x, st = sol.solve(b, [0.5, 0.5], [1e-10, 1e-10], inner=odwf.FP32)
    d = float(torch.linalg.vector_norm(x - rb.x) / torch.linalg.vector_norm(x))
    assert d < 1e-7, d
    w = sol.omega
    Uh, bh, xh = U.cpu().numpy(), b.cpu().numpy(), rb.x.cpu().numpy()
    for i in range(2):
        Dx = oracle.apply(oracle.OP_D, Uh, xh[i], 1.3, w, 0.5 / 2.6)
        assert np.linalg.norm(bh[i] - Dx) / np.linalg.norm(bh[i]) < 1e-7
    sol.close()
    lat.close()
    srv.close()


def test_serving_configuration_lattices_oracle_spot_check():
    """The serving configuration's resident lattices, 8^4, 16^4 and 24^4 x 16
    (eps 0.5, one gauge field each), 12-slot engines, FP32 inner: a short
    Poisson stream with the configuration's draws (masses from {0.005, 0.04,
    0.5}, 1-12 right-hand sides, tolerance 1e-8 or 1e-10); one finished
    request per lattice is checked against the FP64 oracle over the whole
    lattice (D x = b with the request's mass)."""
    lattices = {f"{L}^4": {"dims": (L, L, L, L), "Ns": 16, "eps": 0.5, "seed": 0} for L in (8, 16, 24)}
    srv = Server(lattices, max_slots=12, inner="fp32")
    reqs = poisson_stream(8, 4.0, list(lattices), seed=40)
    done = srv.run(reqs, time_limit=200, keep_solutions=True)
    assert len(done) == 8
    s = summarize(done, max(r.finished for r in done), srv.admission)
    print(f"serving 8^4/16^4/24^4 x 16: {s}")
    assert s["all_converged"]
    checked = set()
    for r in done:
        if r.lattice in checked:
            continue
        checked.add(r.lattice)
        spec = lattices[r.lattice]
        U = synth.make_gauge_device(spec["dims"], spec["eps"], spec["seed"]).cpu().numpy()
        b = synth.make_source_device(spec["dims"], spec["Ns"], r.nrhs, r.seed).cpu().numpy()
        x = r.x.cpu().numpy()
        w = srv.engines[r.lattice]["sol"].omega
        i = r.nrhs - 1
        Dx = oracle.apply(oracle.OP_D, U, x[i], 1.3, w, r.mq / 2.6)
        fr = np.linalg.norm(b[i] - Dx) / np.linalg.norm(b[i])
        print(f"  {r.lattice} m_q={r.mq} tol={r.tol:g} nrhs={r.nrhs}: oracle |b - D x|/|b| = {fr:.3e}, "
              f"latency {r.latency:.3f} s")
        assert fr < 1e3 * r.tol
    srv.close()
