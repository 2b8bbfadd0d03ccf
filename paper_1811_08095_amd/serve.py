"""Serving loop: continuous batching of domain-wall CG solves.

Requests (a lattice, a quark mass, 1-12 right-hand sides, a tolerance) arrive
as a Poisson stream.  Gauge fields and solvers stay resident for every
lattice; each lattice's batch engine (libodwf odwf_batch_*: a fixed number of
right-hand-side slots, its own HIP stream) holds the CG state of the admitted
requests and is created when its first request is admitted.  The loop

  1. queues arrived requests in arrival order,
  2. admits them by device-memory footprint (Admission): into the lattice's
     live engine when slots are free, or by creating the engine when its
     bytes (odwf_batch_footprint) fit the budget beside the live engines --
     evicting idle engines of other lattices if that makes room; a request
     held back for memory holds back the later ones, so busy engines drain,
  3. enqueues a few CG iterations on every engine that has work (the engines'
     streams overlap on the device); an engine over a smaller lattice takes
     proportionally more iterations per step (up to 16x), so that every step
     is a similar slice of device time and the host's per-step polling does
     not dominate small lattices,
  4. polls the slots, retires finished requests and records their latency
     (completion - arrival, queueing included).

New requests are admitted between iterations, while earlier ones are still
iterating: a slot freed by a converged right-hand side is reused at the next
iteration boundary.  The default budget is 90 % of the device memory left
free once the lattices and solvers are resident.  Statistics: p50 / p99
latency, right-hand-side solves per second, requests per second, requests
held back for memory, engine evictions.
"""
import collections
import dataclasses
import json
import time
from typing import Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    lattice: str
    mq: float
    nrhs: int
    tol: float
    arrival: float                    # seconds after the stream start
    seed: int = 0                     # seed of the request's Gaussian sources
    b: object = None                  # device tensor [nrhs][Ns][t][z][y][x][4][3]
    slots: List[int] = dataclasses.field(default_factory=list)
    admitted: Optional[float] = None
    finished: Optional[float] = None
    stats: List[dict] = dataclasses.field(default_factory=list)
    x: object = None
    deferred: bool = False            # held back at least once for device memory

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


def poisson_stream(n, rate, lattices, masses=(0.005, 0.04, 0.5), nrhs_range=(1, 12),
                   tols=(1e-8, 1e-10), seed=4):
    """Arrival times, lattice, mass, right-hand-side count and tolerance of n
    requests, drawn from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    reqs = []
    for i in range(n):
        reqs.append(Request(rid=i, lattice=str(lattices[rng.integers(len(lattices))]),
                            mq=float(masses[rng.integers(len(masses))]),
                            nrhs=int(rng.integers(nrhs_range[0], nrhs_range[1] + 1)),
                            tol=float(tols[rng.integers(len(tols))]), arrival=float(t[i]),
                            seed=int(seed * 100000 + i)))
    return reqs


def percentile(vals, q):
    """q-th percentile with linear interpolation (numpy's default)."""
    return float(np.percentile(np.asarray(vals, dtype=np.float64), q)) if len(vals) else float("nan")


class Admission:
    """Host bookkeeping of the device memory of the batch engines (no GPU
    calls).  Each lattice's engine holds engine_bytes[name] while it exists;
    a request is admitted
      - into its lattice's live engine when nrhs slots are free there, or
      - by creating that engine when its bytes fit the budget beside the live
        engines, evicting idle engines (no admitted request) of other lattices
        first if that makes room;
    otherwise it waits.  Requests are considered in arrival order: one that
    waits for slots holds back the later requests of its own lattice (FIFO per
    lattice), one that waits for memory holds back every later request, so
    that busy engines drain, become idle and can be evicted (no request
    starves)."""

    def __init__(self, engine_bytes: Dict[str, int], slots_per_engine: Dict[str, int],
                 budget_bytes: float):
        self.engine_bytes = dict(engine_bytes)
        self.slots = dict(slots_per_engine)
        self.budget = float(budget_bytes)
        self.free: Dict[str, int] = {}    # live engines: free slots
        self.busy: Dict[str, int] = {}    # live engines: admitted requests in flight
        self.deferred_for_memory = 0
        self.evictions = 0
        self.peak_bytes = 0

    def live_bytes(self) -> int:
        return sum(self.engine_bytes[n] for n in self.free)

    def decide(self, req: Request):
        """("admit", []) | ("create", [idle engines to evict first]) |
        ("wait_slots", []) | ("wait_memory", [])."""
        name = req.lattice
        if req.nrhs > self.slots[name]:
            raise ValueError(f"request of {req.nrhs} right-hand sides exceeds the {self.slots[name]} slots")
        if name in self.free:
            return ("admit", []) if self.free[name] >= req.nrhs else ("wait_slots", [])
        need = self.engine_bytes[name]
        if need > self.budget:
            raise ValueError(f"the engine of {name} ({need} bytes) exceeds the budget alone")
        used = self.live_bytes()
        if used + need <= self.budget:
            return ("create", [])
        evict = []
        for n in sorted(self.free, key=lambda m: -self.engine_bytes[m]):
            if self.busy[n] == 0:
                evict.append(n)
                used -= self.engine_bytes[n]
                if used + need <= self.budget:
                    return ("create", evict)
        return ("wait_memory", [])

    def created(self, name: str):
        self.free[name] = self.slots[name]
        self.busy[name] = 0
        self.peak_bytes = max(self.peak_bytes, self.live_bytes())

    def evicted(self, name: str):
        assert self.busy[name] == 0
        del self.free[name], self.busy[name]
        self.evictions += 1

    def take(self, req: Request):
        assert self.free[req.lattice] >= req.nrhs
        self.free[req.lattice] -= req.nrhs
        self.busy[req.lattice] += 1

    def release(self, req: Request, nslots: int = None):
        n = req.nrhs if nslots is None else nslots
        self.free[req.lattice] += n
        self.busy[req.lattice] -= 1

    def next_decision(self, queued: List[Request]):
        """The first queued request (arrival order) the policy above lets in
        now, as (request, action, engines to evict first), or (None, None, r)
        where r is the request held back for memory (None if nothing waits
        for memory).  Decisions are taken one at a time: each changes the
        state the next one sees."""
        blocked = set()
        for r in queued:
            if r.lattice in blocked:
                continue
            act, ev = self.decide(r)
            if act == "wait_memory":
                return None, None, r
            if act == "wait_slots":
                blocked.add(r.lattice)
                continue
            return r, act, ev
        return None, None, None


class Server:
    """Resident lattices and solvers; one batch engine per lattice, created
    when a request for it is admitted within the device-memory budget and
    evicted when idle and its memory is needed by another lattice."""

    def __init__(self, lattices: Dict[str, dict], max_slots=12, inner="fp32", hbm_budget=None,
                 iters_per_step=4, m0=1.3, lmin=0.05, lmax=6.2, scale_steps=True, serialize=False):
        import torch

        from . import odwf, synth
        self.odwf = odwf
        self.torch = torch
        self.iters_per_step = int(iters_per_step)
        self.serialize = bool(serialize)
        self.inner_p = {"fp32": odwf.FP32, "fp64": odwf.FP64}[inner]
        self.max_slots = int(max_slots)
        self.engines = {}
        engine_bytes = {}
        for name, spec in lattices.items():
            dims, Ns = tuple(spec["dims"]), int(spec["Ns"])
            U = synth.make_gauge_device(dims, spec.get("eps", 0.5), spec.get("seed", 0))
            lat = odwf.Lattice(dims, bc_t=-1)
            lat.load_gauge(U)
            del U
            sol = odwf.Solver(lat, Ns, m0, odwf.zolotarev_omega(Ns, lmin, lmax))
            stream = torch.cuda.Stream()
            self.engines[name] = {"lat": lat, "sol": sol, "batch": None, "stream": stream,
                                  "dims": dims, "Ns": Ns, "active": []}
            engine_bytes[name] = odwf.batch_footprint(dims, Ns, max_slots, self.inner_p)
        # iterations per step: iters_per_step on the largest lattice, more on smaller ones
        vmax = max(int(np.prod(e["dims"])) * e["Ns"] for e in self.engines.values())
        for e in self.engines.values():
            v = int(np.prod(e["dims"])) * e["Ns"]
            mult = min(16, max(1, vmax // v)) if scale_steps else 1
            e["iters"] = self.iters_per_step * mult
        torch.cuda.synchronize()
        if hbm_budget is None:  # the engines may use most of what the resident fields leave free
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = 0.9 * free
        self.admission = Admission(engine_bytes, {n: max_slots for n in lattices}, hbm_budget)
        self.engine_bytes_measured = {}

    def close(self):
        """Release every engine, solver and resident lattice."""
        for e in self.engines.values():
            if e["batch"] is not None:
                e["batch"].close()
            e["sol"].close()
            e["lat"].close()
        self.engines = {}

    def _create(self, name):
        e = self.engines[name]
        e["batch"] = self.odwf.Batch(e["sol"], self.max_slots, inner=self.inner_p)
        self.engine_bytes_measured[name] = e["batch"].nbytes()
        self.admission.created(name)

    def _evict(self, name):
        e = self.engines[name]
        assert not e["active"]
        e["batch"].close()
        e["batch"] = None
        self.admission.evicted(name)

    def _admit(self, req: Request, now: float):
        from . import synth
        e = self.engines[req.lattice]
        with self.torch.cuda.stream(e["stream"]):
            if req.b is None:  # the client's right-hand sides, drawn on arrival
                req.b = synth.make_source_device(e["dims"], e["Ns"], req.nrhs, req.seed)
            for r in range(req.nrhs):
                q = e["batch"].admit(req.b[r], req.mq, req.tol, stream=e["stream"])
                assert q is not None
                req.slots.append(q)
        self.admission.take(req)
        req.admitted = now
        e["active"].append(req)
    def run(self, requests: List[Request], time_limit=600.0, keep_solutions=False, progress=None):
        """Serve the stream in real time; returns the finished requests.  With
        `progress` (a text stream) one line is written per finished request."""
        torch = self.torch
        queued: List[Request] = []
        pending = sorted(requests, key=lambda r: r.arrival)
        done: List[Request] = []
        pi = 0
        t0 = time.perf_counter()
        while len(done) < len(requests):
            now = time.perf_counter() - t0
            if now > time_limit:
                break
            while pi < len(pending) and pending[pi].arrival <= now:
                queued.append(pending[pi])
                pi += 1
            while True:
                req, act, ev = self.admission.next_decision(queued)
                if req is None:
                    if ev is not None and not ev.deferred:  # held back for memory
                        ev.deferred = True
                        self.admission.deferred_for_memory += 1
                    break
                if act == "create":
                    for name in ev:
                        self._evict(name)
                    self._create(req.lattice)
                self._admit(req, now)
                queued.remove(req)
            busy = [e for e in self.engines.values() if e["active"]]
            if not busy:
                if pi < len(pending):
                    time.sleep(min(0.002, max(0.0, pending[pi].arrival - now)))
                continue
            for e in busy:
                e["batch"].step(e["iters"], stream=e["stream"])
                if self.serialize:  # engines one after another (for the overlap measurement)
                    e["stream"].synchronize()
            for e in busy:
                still = []
                for req in e["active"]:
                    fin = True
                    for q in req.slots:
                        d, _ = e["batch"].poll(q, stream=e["stream"])
                        fin &= d
                    if not fin:
                        still.append(req)
                        continue
                    out = torch.empty_like(req.b) if keep_solutions else torch.empty_like(req.b[0])
                    for i, q in enumerate(req.slots):
                        st = e["batch"].retire(q, out[i] if keep_solutions else out,
                                               stream=e["stream"])
                        req.stats.append(st)
                    req.x = out if keep_solutions else None
                    req.finished = time.perf_counter() - t0
                    self.admission.release(req)
                    req.b = None
                    done.append(req)
                    if progress is not None:
                        print(f"# {len(done)}/{len(requests)} {req.lattice} m_q={req.mq} "
                              f"nrhs={req.nrhs} tol={req.tol:g} latency {req.latency:.3f} s",
                              file=progress, flush=True)
                e["active"] = still
        return done


def summarize(done: List[Request], makespan: float, admission: Admission = None):
    lat = [r.latency for r in done]
    nrhs = sum(r.nrhs for r in done)
    resid_ok = all(s["true_rel_resid"] <= r.tol and s["status"] == 0 for r in done for s in r.stats)
    out = {"requests": len(done), "rhs": nrhs, "makespan_s": round(makespan, 3),
           "p50_latency_s": round(percentile(lat, 50), 4), "p99_latency_s": round(percentile(lat, 99), 4),
           "rhs_solves_per_s": round(nrhs / makespan, 3) if makespan > 0 else None,
           "requests_per_s": round(len(done) / makespan, 3) if makespan > 0 else None,
           "all_converged": bool(resid_ok)}
    if admission is not None:
        out.update({"hbm_budget_gb": round(admission.budget / 1e9, 2),
                    "peak_engine_gb": round(admission.peak_bytes / 1e9, 3),
                    "requests_deferred_for_memory": admission.deferred_for_memory,
                    "engine_evictions": admission.evictions})
    return out


def main():
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="serve a Poisson stream of ODWF solve requests")
    ap.add_argument("--requests", type=int, default=60)
    ap.add_argument("--rate", type=float, default=0.0, help="arrivals/s (0: a fraction of saturation)")
    ap.add_argument("--loads", default="0.8",
                    help="comma list of fractions of the measured saturation throughput")
    ap.add_argument("--sizes", default="8,16,24")
    ap.add_argument("--Ns", type=int, default=16)
    ap.add_argument("--max-slots", type=int, default=12)
    ap.add_argument("--inner", default="fp32")
    ap.add_argument("--time-limit", type=float, default=900.0)
    ap.add_argument("--hbm-budget-gb", type=float, default=0.0, help="engine memory budget (0: 90%% of free)")
    ap.add_argument("--serialize", action="store_true", help="run the engines one after another")
    ap.add_argument("--progress", action="store_true", help="one line per finished request on stderr")
    args = ap.parse_args()
    lattices = {f"{L}^4": {"dims": (L, L, L, L), "Ns": args.Ns, "eps": 0.5, "seed": 0}
                for L in (int(v) for v in args.sizes.split(","))}
    srv = Server(lattices, max_slots=args.max_slots, inner=args.inner,
                 hbm_budget=args.hbm_budget_gb * 1e9 if args.hbm_budget_gb > 0 else None,
                 serialize=args.serialize)
    prog = sys.stderr if args.progress else None
    rates = [(None, args.rate)]
    sat = None
    if args.rate <= 0:  # saturation: a warm-up stream that arrives all at once
        warm = poisson_stream(min(24, args.requests), 1e9, list(lattices), seed=3)
        t = time.perf_counter()
        d = srv.run(warm, time_limit=args.time_limit, progress=prog)
        sat = len(d) / (time.perf_counter() - t)
        rates = [(float(f), float(f) * sat) for f in args.loads.split(",")]
    for load, rate in rates:
        reqs = poisson_stream(args.requests, rate, list(lattices))
        t = time.perf_counter()
        done = srv.run(reqs, time_limit=args.time_limit, progress=prog)
        out = summarize(done, time.perf_counter() - t, srv.admission)
        out.update({"arrival_rate": round(rate, 4), "load": load,
                    "saturation_requests_per_s": round(sat, 4) if sat else None,
                    "submitted": len(reqs)})
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
