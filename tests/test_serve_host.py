"""Host logic of the serving loop (CPU only): the arrival stream, the
admission bookkeeping and the latency statistics."""
import numpy as np
import pytest

from paper_1811_08095_amd.serve import Admission, Request, percentile, poisson_stream, summarize


def test_poisson_stream_is_seeded_and_well_formed():
    a = poisson_stream(400, 2.0, ["8^4", "16^4", "24^4"], seed=4)
    b = poisson_stream(400, 2.0, ["8^4", "16^4", "24^4"], seed=4)
    assert [(r.arrival, r.lattice, r.mq, r.nrhs, r.tol) for r in a] == \
        [(r.arrival, r.lattice, r.mq, r.nrhs, r.tol) for r in b]
    t = np.array([r.arrival for r in a])
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 0.5) < 0.1           # rate 2/s
    assert abs(gaps.std() / gaps.mean() - 1) < 0.2  # exponential: cv = 1
    assert {r.nrhs for r in a} == set(range(1, 13))
    assert {r.mq for r in a} == {0.005, 0.04, 0.5}
    assert {r.tol for r in a} == {1e-8, 1e-10}
    assert len({r.seed for r in a}) == 400


def test_admission_respects_slots_and_budget():
    adm = Admission({"a": 12, "b": 12}, {"a": 10, "b": 100}, budget_bytes=1000)
    r1 = Request(0, "a", 0.1, 12, 1e-8, 0.0)
    r2 = Request(1, "a", 0.1, 1, 1e-8, 0.0)
    r3 = Request(2, "b", 0.1, 9, 1e-8, 0.0)
    r4 = Request(3, "b", 0.1, 2, 1e-8, 0.0)
    assert adm.fits(r1)
    adm.take(r1)
    assert not adm.fits(r2)          # no free slot on engine a
    adm2 = Admission({"a": 12, "b": 12}, {"a": 10, "b": 100}, budget_bytes=1000)
    adm2.take(r1)
    assert not adm2.fits(r3)         # 120 + 900 > 1000: over the HBM budget
    assert adm2.fits(r4)
    adm2.release(r1)
    assert adm2.fits(r3) and adm2.in_flight == 0
    with pytest.raises(AssertionError):
        adm2.take(Request(4, "a", 0.1, 13, 1e-8, 0.0))


def test_percentiles_and_summary():
    assert percentile([1, 2, 3, 4], 50) == 2.5
    assert percentile(list(range(101)), 99) == 99.0
    done = []
    for i in range(10):
        r = Request(i, "a", 0.1, 2, 1e-8, arrival=float(i))
        r.finished = float(i) + 1.0 + 0.1 * i
        r.stats = [{"true_rel_resid": 1e-9, "status": 0}] * 2
        done.append(r)
    s = summarize(done, makespan=20.0)
    assert s["requests"] == 10 and s["rhs"] == 20 and s["rhs_solves_per_s"] == 1.0
    assert abs(s["p50_latency_s"] - 1.45) < 1e-9
    assert s["p99_latency_s"] <= 1.9 + 1e-9 and s["all_converged"]
