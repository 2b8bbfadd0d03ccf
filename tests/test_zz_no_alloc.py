"""odwf_apply_noalloc, the operator application that allocates no device
memory, against odwf_apply (the same kernels on the solver's workspace).

Two calls in a row on one GPU, the second with a smaller input, each equal to
odwf_apply bit for bit (and the FP64 ones within 1e-12 of the FP64 CPU
oracle); a call that needs more than the scratch array is refused before any
work is queued; and the call leaves the device's free memory unchanged.
"""
import numpy as np
import pytest

from oracle import oracle
from paper_1811_08095_amd import odwf, synth

pytestmark = pytest.mark.gpu

M0 = 1.3


def _setup(dims, Ns, nrhs, seed, bc=-1):
    import torch
    U = synth.make_gauge(dims, 0.5, seed)
    w = odwf.zolotarev_omega(Ns, 0.05, 6.2)
    lat = odwf.Lattice(dims, bc_t=bc)
    lat.load_gauge(U)
    sol = odwf.Solver(lat, Ns, M0, w)
    psi = synth.make_source(dims, Ns, nrhs, 3000 + seed)
    return U, w, lat, sol, psi, torch.from_numpy(psi).cuda()


def _relerr(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_two_calls_in_a_row_match_apply():
    import torch
    # first call: 8^4 x 16, two right-hand sides with different masses, the
    # normal operator (four fused hops, four of the six half fields)
    U, w, lat, sol, psi, psid = _setup((8, 8, 8, 8), 16, 2, 1)
    mq = [0.04, 0.5]
    print("noalloc call 1: 8^4 x 16, nrhs 2, SCHUR_NORMAL, FP64", flush=True)
    a1 = sol.apply_noalloc(odwf.OP_SCHUR_NORMAL, psid, mq, prec=odwf.FP64)
    r1 = sol.apply(odwf.OP_SCHUR_NORMAL, psid, mq, prec=odwf.FP64)
    torch.cuda.synchronize()
    assert torch.equal(a1, r1)
    a1 = a1.cpu().numpy()
    for r in range(2):
        ref = oracle.apply(oracle.OP_SCHUR_NORMAL, U, psi[r], M0, w, mq[r] / (2 * M0), -1)
        assert _relerr(a1[r], ref) <= 1e-12
    # second call, smaller input: 4^4 x 8, one right-hand side, D
    U2, w2, lat2, sol2, psi2, psid2 = _setup((4, 4, 4, 4), 8, 1, 2, bc=1)
    print("noalloc call 2: 4^4 x 8, nrhs 1, D, FP64", flush=True)
    a2 = sol2.apply_noalloc(odwf.OP_D, psid2, [0.05], prec=odwf.FP64)
    r2 = sol2.apply(odwf.OP_D, psid2, [0.05], prec=odwf.FP64)
    torch.cuda.synchronize()
    assert torch.equal(a2, r2)
    ref2 = oracle.apply(oracle.OP_D, U2, psi2[0], M0, w2, 0.05 / (2 * M0), 1)
    assert _relerr(a2.cpu().numpy()[0], ref2) <= 1e-12
    # and the first solver again, fewer right-hand sides, a scaled format
    print("noalloc call 3: 8^4 x 16, nrhs 1, HOP_EO, FP16S", flush=True)
    a3 = sol.apply_noalloc(odwf.OP_HOP_EO, psid[:1].contiguous(), [0.04], prec=odwf.FP16S)
    r3 = sol.apply(odwf.OP_HOP_EO, psid[:1].contiguous(), [0.04], prec=odwf.FP16S)
    torch.cuda.synchronize()
    assert torch.equal(a3, r3)
    for s in (sol, sol2):
        s.close()
    for lt in (lat, lat2):
        lt.close()


def test_every_operator_matches_apply():
    import torch
    U, w, lat, sol, psi, psid = _setup((6, 2, 4, 4), 8, 3, 4)
    mq = [0.01, 0.1, 2.6]
    for op in range(9):
        for prec in (odwf.FP64, odwf.FP32, odwf.BF16S):
            a = sol.apply_noalloc(op, psid, mq, prec=prec)
            r = sol.apply(op, psid, mq, prec=prec)
            torch.cuda.synchronize()
            assert torch.equal(a, r), (op, prec)
    sol.close()
    lat.close()


def test_oversize_request_is_refused():
    import torch
    # Ns = 32, 8 right-hand sides per launch: D needs six half fields of
    # 1024 sites x 8 x 32 x 192 bytes = 302 MB > 256 MiB
    U, w, lat, sol, psi, psid = _setup((8, 8, 8, 4), 32, 8, 5)
    out = torch.full_like(psid, 7.0)
    with pytest.raises(odwf.OdwfError) as e:
        sol.apply_noalloc(odwf.OP_D, psid, [0.04] * 8, prec=odwf.FP64, out=out)
    assert e.value.status == odwf.ENOMEM and "maximum" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())  # nothing was queued
    # one right-hand side fits
    a = sol.apply_noalloc(odwf.OP_D, psid[:1].contiguous(), [0.04], prec=odwf.FP64)
    r = sol.apply(odwf.OP_D, psid[:1].contiguous(), [0.04], prec=odwf.FP64)
    torch.cuda.synchronize()
    assert torch.equal(a, r)
    sol.close()
    lat.close()


def test_call_leaves_free_device_memory_unchanged():
    import torch
    U, w, lat, sol, psi, psid = _setup((8, 8, 8, 8), 16, 1, 6)
    out = torch.empty_like(psid)
    # load the kernels' code on the device first (through another solver)
    warm = odwf.Solver(lat, 16, M0, w)
    warm.apply(odwf.OP_SCHUR_NORMAL, psid, [0.04], out=out)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        sol.apply_noalloc(odwf.OP_SCHUR_NORMAL, psid, [0.04], out=out)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    warm.close()
    sol.close()
    lat.close()
