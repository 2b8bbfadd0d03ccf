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


def test_admission_creates_engines_within_the_budget_and_evicts_idle_ones():
    adm = Admission({"a": 400, "b": 700}, {"a": 12, "b": 12}, budget_bytes=1000)
    ra1 = Request(0, "a", 0.1, 12, 1e-8, 0.0)
    ra2 = Request(1, "a", 0.1, 1, 1e-8, 0.1)
    rb = Request(2, "b", 0.1, 3, 1e-8, 0.2)
    ra3 = Request(3, "a", 0.1, 1, 1e-8, 0.3)
    # first request of a lattice: its engine is created (400 <= 1000)
    assert adm.next_decision([ra1, ra2, rb, ra3]) == (ra1, "create", [])
    adm.created("a")
    adm.take(ra1)
    # a's engine is full: ra2 waits for slots and holds back ra3 (FIFO per
    # lattice); b's engine (700) does not fit beside a's (400) while a is busy
    assert adm.decide(ra2) == ("wait_slots", [])
    assert adm.decide(rb) == ("wait_memory", [])
    assert adm.next_decision([ra2, rb, ra3]) == (None, None, rb)
    # a finishes: ra2 goes into the live engine first (arrival order)
    adm.release(ra1)
    assert adm.next_decision([ra2, rb, ra3]) == (ra2, "admit", [])
    adm.take(ra2)
    # rb still does not fit, and holds back ra3 (so that a drains)
    assert adm.next_decision([rb, ra3]) == (None, None, rb)
    adm.release(ra2)
    # a is idle: rb evicts it and creates b
    assert adm.next_decision([rb, ra3]) == (rb, "create", ["a"])
    adm.evicted("a")
    adm.created("b")
    adm.take(rb)
    assert adm.live_bytes() == 700 and adm.evictions == 1 and adm.peak_bytes == 700
    assert adm.decide(ra3) == ("wait_memory", [])


def test_admission_rejects_what_can_never_fit():
    adm = Admission({"a": 2000}, {"a": 4}, budget_bytes=1000)
    with pytest.raises(ValueError):
        adm.decide(Request(0, "a", 0.1, 1, 1e-8, 0.0))
    adm2 = Admission({"a": 10}, {"a": 4}, budget_bytes=1000)
    with pytest.raises(ValueError):
        adm2.decide(Request(0, "a", 0.1, 5, 1e-8, 0.0))
    adm2.created("a")
    with pytest.raises(AssertionError):
        adm2.take(Request(1, "a", 0.1, 5, 1e-8, 0.0))


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
