"""Edge cases of the C ABI on the GPU: more right-hand sides than one launch
takes (the library splits them), the smallest lattice, and every documented
error path (empty batch of right-hand sides, aliased buffers, gauge field not
loaded, unsupported N_s, oversized batch engine)."""
import numpy as np
import pytest

from oracle import oracle
from paper_1811_08095_amd import odwf, synth

pytestmark = pytest.mark.gpu

M0 = 1.3


def _mk(dims, Ns, seed=0, eps=0.5, bc=-1):
    U = synth.make_gauge(dims, eps, seed)
    w = odwf.zolotarev_omega(Ns, 0.05, 6.2)
    lat = odwf.Lattice(dims, bc_t=bc)
    lat.load_gauge(U)
    return U, w, lat, odwf.Solver(lat, Ns, M0, w)


def test_apply_more_rhs_than_one_launch():
    """N_s = 4 takes at most 16 right-hand sides per launch; 20 are split into
    16 + 4 and every one matches the oracle with its own mass."""
    import torch
    dims, Ns, n = (2, 2, 2, 4), 4, 20
    U, w, lat, sol = _mk(dims, Ns, seed=3)
    psi = synth.make_source(dims, Ns, n, 3300)
    masses = list(np.linspace(0.01, 0.9, n))
    for op in (odwf.OP_D, odwf.OP_SCHUR_NORMAL):
        out = sol.apply(op, torch.from_numpy(psi).cuda(), masses, prec=odwf.FP64).cpu().numpy()
        for r in range(n):
            ref = oracle.apply(op, U, psi[r], M0, w, masses[r] / (2 * M0), -1)
            assert np.linalg.norm(out[r] - ref) / np.linalg.norm(ref) <= 1e-12, (op, r)


def test_solve_more_rhs_than_one_launch():
    import torch
    dims, Ns, n = (2, 2, 2, 4), 4, 18
    U, w, lat, sol = _mk(dims, Ns, seed=4)
    b = synth.make_source(dims, Ns, n, 3400)
    masses = [0.05 + 0.02 * r for r in range(n)]
    x, st = sol.solve(torch.from_numpy(b).cuda(), masses, [1e-10] * n, inner=odwf.FP32)
    xh = x.cpu().numpy()
    for r in range(n):
        assert st[r]["status"] == odwf.OK and st[r]["true_rel_resid"] <= 1e-10
        Dx = oracle.apply(oracle.OP_D, U, xh[r], M0, w, masses[r] / (2 * M0), -1)
        assert np.linalg.norm(b[r] - Dx) / np.linalg.norm(b[r]) <= 1e-7


def test_error_paths():
    import torch
    dims, Ns = (2, 2, 2, 2), 4
    U, w, lat, sol = _mk(dims, Ns)
    psi = torch.from_numpy(synth.make_source(dims, Ns, 1, 1)).cuda()
    # no right-hand sides
    empty = psi[:0]
    with pytest.raises(odwf.OdwfError) as e:
        sol.apply(odwf.OP_D, empty, [], out=torch.empty_like(empty))
    assert e.value.status == odwf.EINVAL
    # input and output alias
    with pytest.raises(odwf.OdwfError) as e:
        sol.apply(odwf.OP_D, psi, [0.1], out=psi)
    assert e.value.status == odwf.EINVAL
    # non-finite mass
    with pytest.raises(odwf.OdwfError):
        sol.apply(odwf.OP_D, psi, [float("nan")])
    # gauge field not loaded
    lat2 = odwf.Lattice(dims)
    sol2 = odwf.Solver(lat2, Ns, M0, w)
    with pytest.raises(odwf.OdwfError) as e:
        sol2.apply(odwf.OP_D, psi, [0.1])
    assert e.value.status == odwf.EINVAL
    # unsupported N_s
    with pytest.raises(odwf.OdwfError):
        odwf.Solver(lat, 6, M0, odwf.zolotarev_omega(6))
    # batch engine wider than one launch
    with pytest.raises(odwf.OdwfError):
        odwf.Batch(sol, 17)
    # the library still works after every error
    out = sol.apply(odwf.OP_D, psi, [0.1], prec=odwf.FP64).cpu().numpy()[0]
    ref = oracle.apply(oracle.OP_D, U, psi.cpu().numpy()[0], M0, w, 0.1 / (2 * M0), -1)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) <= 1e-12


@pytest.mark.parametrize("prec,bound", [(odwf.FP64, 1e-12), (odwf.FP32, 1e-5), (odwf.FP16S, 4e-3)],
                         ids=["fp64", "fp32", "fp16s"])
def test_apply_widest_launch_ns16(prec, bound):
    """N_s = 16 takes at most 16 right-hand sides per launch: a block is then
    one site with 16 x 16 lanes (the fifth-dimension lane programs run on 16
    DPP rows of one block).  17 right-hand sides with their own masses are
    split 16 + 1; each matches the oracle (FP64 to 1e-12, reduced precisions
    within their stated bounds)."""
    import torch
    dims, Ns, n = (4, 2, 2, 4), 16, 17
    U, w, lat, sol = _mk(dims, Ns, seed=5, eps=0.7)
    psi = synth.make_source(dims, Ns, n, 3500)
    masses = list(np.linspace(0.0025, 0.5, n))
    for op in (odwf.OP_HOP_EO, odwf.OP_D, odwf.OP_SCHUR_NORMAL):
        out = sol.apply(op, torch.from_numpy(psi).cuda(), masses, prec=prec).cpu().numpy()
        for r in range(n):
            ref = oracle.apply(op, U, psi[r], M0, w, masses[r] / (2 * M0), -1)
            err = np.linalg.norm(out[r] - ref) / np.linalg.norm(ref)
            assert err <= bound, (op, r, err)


@pytest.mark.parametrize("Ns", [8, 16])
def test_massless_limit(Ns):
    """m_q = 0 (mu = 0): the boundary term of L vanishes and the cyclic
    fifth-dimension solves become plain bidiagonal ones (the cycle's closing
    factor is zero); every operator still matches the oracle, in FP64 to 1e-12
    and in FP32 (lane programs at N_s = 16, LDS columns at N_s = 8) to 1e-5."""
    import torch
    dims = (4, 2, 2, 4)
    U, w, lat, sol = _mk(dims, Ns, seed=6, eps=0.7)
    psi = synth.make_source(dims, Ns, 1, 3600)
    pd = torch.from_numpy(psi).cuda()
    for op in (odwf.OP_M5INV, odwf.OP_D, odwf.OP_DDAG, odwf.OP_SCHUR, odwf.OP_SCHUR_NORMAL):
        ref = oracle.apply(op, U, psi[0], M0, w, 0.0, -1)
        for prec, bound in ((odwf.FP64, 1e-12), (odwf.FP32, 1e-5)):
            out = sol.apply(op, pd, [0.0], prec=prec).cpu().numpy()[0]
            err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
            assert err <= bound, (op, prec, err)
