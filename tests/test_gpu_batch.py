"""Batch engine (continuous batching at CG-iteration granularity) on the GPU.

Each slot's solution is checked by the FP64 oracle (D x = b with the slot's
own mass), and the same request gives the same result alone and admitted in
the middle of a mix of other requests.
"""
import numpy as np
import pytest

from oracle import oracle
from paper_1811_08095_amd import odwf, synth

pytestmark = pytest.mark.gpu

M0 = 1.3


def _mk(dims, Ns, eps, seed):
    U = synth.make_gauge(dims, eps, seed)
    w = odwf.zolotarev_omega(Ns, 0.05, 6.2)
    lat = odwf.Lattice(dims, bc_t=-1)
    lat.load_gauge(U)
    return U, w, lat, odwf.Solver(lat, Ns, M0, w)


def _run_to_completion(bt, slots, max_steps=2000, chunk=5):
    done = {}
    for _ in range(max_steps):
        for q in slots:
            if q in done:
                continue
            d, st = bt.poll(q)
            if d:
                done[q] = st
        if len(done) == len(slots):
            return done
        bt.step(chunk)
    raise AssertionError("batch did not finish")


@pytest.mark.parametrize("inner", [odwf.FP32, odwf.FP64], ids=["fp32", "fp64"])
def test_batch_slots_solve_their_own_systems(inner):
    import torch
    dims, Ns = (4, 4, 4, 4), 8
    U, w, lat, sol = _mk(dims, Ns, 0.5, 1)
    bt = odwf.Batch(sol, 4, inner=inner)
    masses, tols = [0.01, 0.5, 0.04], [1e-10, 1e-8, 1e-9]
    srcs = synth.make_source(dims, Ns, 3, 77)
    slots = []
    for i in range(3):
        q = bt.admit(torch.from_numpy(srcs[i]).cuda().contiguous(), masses[i], tols[i])
        slots.append(q)
    assert bt.free_slots() == 1
    stats = _run_to_completion(bt, slots)
    for i, q in enumerate(slots):
        assert stats[q]["status"] == odwf.OK and stats[q]["true_rel_resid"] <= tols[i]
        x = torch.zeros(sol.spinor_shape(1)[1:], dtype=torch.complex128, device="cuda")
        st = bt.retire(q, x)
        xh = x.cpu().numpy()
        Dx = oracle.apply(oracle.OP_D, U, xh, M0, w, masses[i] / (2 * M0))
        fr = np.linalg.norm(srcs[i] - Dx) / np.linalg.norm(srcs[i])
        assert fr <= 1e3 * tols[i], (i, fr)
    assert bt.free_slots() == 4


def test_batch_full_and_busy():
    import torch
    dims, Ns = (2, 2, 2, 2), 4
    U, w, lat, sol = _mk(dims, Ns, 0.3, 2)
    bt = odwf.Batch(sol, 2, inner=odwf.FP32)
    b = torch.from_numpy(synth.make_source(dims, Ns, 1, 5)[0]).cuda().contiguous()
    assert bt.admit(b, 0.1, 1e-9) == 0
    assert bt.admit(b, 0.1, 1e-9) == 1
    assert bt.admit(b, 0.1, 1e-9) is None   # EBUSY: no free slot


def test_alone_equals_in_mix():
    """The request's arithmetic does not depend on the other slots: its
    solution is bitwise identical alone and when admitted mid-way into a mix
    of requests with other masses and tolerances."""
    import torch
    dims, Ns = (4, 4, 4, 4), 8
    U, w, lat, sol = _mk(dims, Ns, 0.5, 3)
    srcs = synth.make_source(dims, Ns, 4, 91)
    dev = [torch.from_numpy(srcs[i]).cuda().contiguous() for i in range(4)]
    # alone
    bt = odwf.Batch(sol, 4, inner=odwf.FP32)
    q = bt.admit(dev[0], 0.04, 1e-10)
    st_alone = _run_to_completion(bt, [q])[q]
    x_alone = torch.zeros_like(dev[0])
    bt.retire(q, x_alone)
    # in a mix: others first, the request admitted after some iterations, into slot 2
    bm = odwf.Batch(sol, 4, inner=odwf.FP32)
    a = bm.admit(dev[1], 0.5, 1e-8)
    b = bm.admit(dev[2], 0.01, 1e-10)
    bm.step(7)
    c = bm.admit(dev[3], 0.1, 1e-9)
    bm.step(3)
    bm.retire(a, torch.zeros_like(dev[0])) if bm.poll(a)[0] else None
    q2 = bm.admit(dev[0], 0.04, 1e-10)
    others = [s for s in (b, c) if s is not None]
    st_mix = _run_to_completion(bm, [q2] + others)[q2]
    x_mix = torch.zeros_like(dev[0])
    bm.retire(q2, x_mix)
    assert st_alone["iters"] == st_mix["iters"]
    assert st_alone["reliable_updates"] == st_mix["reliable_updates"]
    assert torch.equal(x_alone, x_mix)
    assert st_mix["true_rel_resid"] <= 1e-10
