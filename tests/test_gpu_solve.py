"""GPU solves checked by the FP64 CPU oracle.

Acceptance (the paper's solves are CG on the normal operator, §2): the
relative residual of the system CG iterates, recomputed by the oracle in FP64
on the GPU's solution, meets the tolerance; FULL-mode solutions also satisfy
D x = b as checked by the oracle's D, and agree with the oracle's own solve to
the accuracy the conditioning allows (stated per test).
"""
import numpy as np
import pytest

from oracle import oracle
from paper_1811_08095_amd import odwf, synth

pytestmark = pytest.mark.gpu

M0 = 1.3


def _mk(dims, Ns, eps, seed, bc=-1):
    U = synth.make_gauge(dims, eps, seed)
    w = odwf.zolotarev_omega(Ns, 0.05, 6.2)
    lat = odwf.Lattice(dims, bc_t=bc)
    lat.load_gauge(U)
    return U, w, lat, odwf.Solver(lat, Ns, M0, w)


def _full_resid(U, w, x, b, mq, bc=-1):
    Dx = oracle.apply(oracle.OP_D, U, x, M0, w, mq / (2 * M0), bc)
    return np.linalg.norm(b - Dx) / np.linalg.norm(b)


@pytest.mark.parametrize("inner", [odwf.FP64, odwf.FP32, odwf.FP16S, odwf.BF16S],
                         ids=["fp64", "fp32", "fp16s", "bf16s"])
def test_plain_config_full_solve(inner):
    """4^4 x 8, eps = 0.3, m_q = 0.05, one Gaussian source, tol 1e-10."""
    import torch
    dims, Ns, mq = (4, 4, 4, 4), 8, 0.05
    U, w, lat, sol = _mk(dims, Ns, 0.3, 0)
    b = synth.make_source(dims, Ns, 1, 1000)
    x, st = sol.solve(torch.from_numpy(b).cuda(), [mq], [1e-10], mode=odwf.SOLVE_FULL,
                      inner=inner, maxiter=20000)
    st = st[0]
    print(odwf.PREC_NAMES[inner], st)
    assert st["status"] == odwf.OK and st["true_rel_resid"] <= 1e-10
    xh = x.cpu().numpy()[0]
    fr = _full_resid(U, w, xh, b[0], mq)
    assert fr <= 1e-8 and abs(fr - st["full_rel_resid"]) <= 1e-9
    xo, it, rr, fro = oracle.solve(U, b[0], M0, w, mq / (2 * M0), oracle.SOLVE_FULL, tol=1e-12)
    assert np.linalg.norm(xh - xo) / np.linalg.norm(xo) <= 1e-7
    if inner == odwf.FP64:
        # same algorithm on the same system and tolerance: same iteration count
        # up to rounding-order effects
        _, it10, _, _ = oracle.solve(U, b[0], M0, w, mq / (2 * M0), oracle.SOLVE_FULL, tol=1e-10)
        assert abs(st["iters"] - it10) <= 2, (st["iters"], it10)


def test_eo_normal_solve_oracle_residual():
    import torch
    dims, Ns, mq = (4, 4, 2, 6), 8, 0.04
    U, w, lat, sol = _mk(dims, Ns, 0.5, 2)
    b = synth.make_source(dims, Ns, 2, 1001)
    x, st = sol.solve(torch.from_numpy(b).cuda(), [mq, 0.5], [1e-10, 1e-9],
                      mode=odwf.SOLVE_EO_NORMAL, inner=odwf.FP32)
    xh = x.cpu().numpy()
    for r, (m, tol) in enumerate(((mq, 1e-10), (0.5, 1e-9))):
        res = oracle.normal_residual(U, b[r], xh[r], M0, w, m / (2 * M0))
        assert res <= 1.05 * tol, (r, res, st[r])
        odd = ~oracle.parity_mask((6, 2, 4, 4))
        assert np.all(xh[r][:, odd] == 0)


def test_multi_rhs_masses_and_tolerances():
    import torch
    dims, Ns = (4, 4, 4, 4), 8
    U, w, lat, sol = _mk(dims, Ns, 0.5, 4)
    b = synth.make_source(dims, Ns, 3, 1004)
    masses, tols = [0.01, 0.04, 0.5], [1e-10, 1e-8, 1e-10]
    x, st = sol.solve(torch.from_numpy(b).cuda(), masses, tols, inner=odwf.FP32)
    xh = x.cpu().numpy()
    for r in range(3):
        assert st[r]["true_rel_resid"] <= tols[r]
        assert _full_resid(U, w, xh[r], b[r], masses[r]) <= 1e3 * tols[r]
    # lighter quarks need more iterations
    assert st[0]["iters"] > st[2]["iters"]


def test_warm_start_converges_immediately():
    import torch
    dims, Ns, mq = (4, 4, 4, 4), 8, 0.05
    U, w, lat, sol = _mk(dims, Ns, 0.3, 0)
    bd = torch.from_numpy(synth.make_source(dims, Ns, 1, 1000)).cuda()
    x, st = sol.solve(bd, [mq], [1e-10])
    x2, st2 = sol.solve(bd, [mq], [1e-8], x=x.clone(), use_x0=True)
    assert st2[0]["iters"] <= 2 and st2[0]["true_rel_resid"] <= 1e-8


def test_noconv_and_nan_reported():
    import torch
    dims, Ns, mq = (4, 4, 4, 4), 8, 0.05
    U, w, lat, sol = _mk(dims, Ns, 0.3, 0)
    b = synth.make_source(dims, Ns, 1, 1000)
    x, st = sol.solve(torch.from_numpy(b).cuda(), [mq], [1e-10], maxiter=3, raise_on_noconv=False)
    assert st[0]["status"] == odwf.ENOCONV and st[0]["iters"] == 3
    assert np.isfinite(x.cpu().numpy()).all()
    bn = b.copy()
    bn[0, 0, 0, 0, 0, 0, 0, 0] = np.nan
    x, st = sol.solve(torch.from_numpy(bn).cuda(), [mq], [1e-10], raise_on_noconv=False)
    assert st[0]["status"] == odwf.ENAN
    with pytest.raises(odwf.OdwfError):
        sol.solve(torch.from_numpy(bn).cuda(), [mq], [1e-10])


def test_zero_source():
    import torch
    dims, Ns = (2, 2, 2, 2), 4
    U, w, lat, sol = _mk(dims, Ns, 0.3, 0)
    b = torch.zeros(sol.spinor_shape(1), dtype=torch.complex128, device="cuda")
    x, st = sol.solve(b, [0.1], [1e-10])
    assert st[0]["status"] == odwf.OK and st[0]["iters"] == 0
    assert torch.count_nonzero(x).item() == 0
