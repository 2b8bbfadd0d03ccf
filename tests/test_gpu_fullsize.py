"""Parity at the full single-GPU size, in the launch configuration the
benchmark times: 64^3 x 64 lattice, N_s = 16, eps = 0.7 links (seed 0),
m0 = 1.3, omega_s Zolotarev on [0.05, 6.2], antiperiodic in t, one Gaussian
right-hand side, the same kernels, block shapes and traversal as the timed
solve.

The oracle cannot hold this lattice, so it is evaluated at sampled sites (the
lattice corners, both time boundaries, random sites) through the frame
evaluation of sampled.py, which is pinned to the whole-lattice oracle by
test_sampled_oracle.py.  Bars: FP64 <= 1e-12 relative over the sampled sites;
reduced precisions within the bounds stated for the small lattices; the
mixed-precision solve's residual b - D x, recomputed by the oracle at the
sampled sites, is bounded by the full residual the solve reports (the norm over
a subset cannot exceed the norm over the lattice).
"""
import numpy as np
import pytest

import sampled
from oracle import oracle
from paper_1811_08095_amd import odwf, synth

pytestmark = pytest.mark.gpu

DIMS, NS, EPS, M0 = (64, 64, 64, 64), 16, 0.7, 1.3
PREC_BOUND = {odwf.FP32: 1e-5, odwf.FP16S: 4e-3, odwf.BF16S: 3e-2}
LIB_OP = {oracle.OP_HOP_EO: odwf.OP_HOP_EO, oracle.OP_D: odwf.OP_D, oracle.OP_DDAG: odwf.OP_DDAG,
          oracle.OP_SCHUR: odwf.OP_SCHUR, oracle.OP_SCHUR_NORMAL: odwf.OP_SCHUR_NORMAL}
NAMES = {oracle.OP_HOP_EO: "HOP_EO", oracle.OP_D: "D", oracle.OP_DDAG: "DDAG",
         oracle.OP_SCHUR: "SCHUR", oracle.OP_SCHUR_NORMAL: "SCHUR_NORMAL"}


@pytest.fixture(scope="module")
def full():
    import torch
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < 280e9:
        pytest.skip(f"the 64^4 x 16 lattice needs ~280 GB of device memory ({free / 1e9:.0f} GB free)")
    print(f"full size: {DIMS} Ns={NS}", flush=True)
    st = {"U": synth.make_gauge_device(DIMS, EPS, 0)}
    st["lat"] = odwf.Lattice(DIMS, bc_t=-1)
    st["lat"].load_gauge(st["U"])
    st["w"] = odwf.zolotarev_omega(NS, 0.05, 6.2)
    yield st
    st.clear()
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def src(full):
    """Holder of the operator input (a dict, so that the solve test can drop it)."""
    import torch
    h = {"psi": synth.make_source_device(DIMS, NS, 1, 2024)}
    yield h
    h.clear()
    torch.cuda.empty_cache()


def _sampled_check(full, src, op, mq, prec, nsites):
    import torch
    psi = src["psi"]
    sol = odwf.Solver(full["lat"], NS, M0, full["w"])
    try:
        out = sol.apply(LIB_OP[op], psi, [mq], prec=prec)
        torch.cuda.synchronize()
    finally:
        sol.close()
    sites = sampled.pick_sites(DIMS, nsites, sampled.OUT_PARITY.get(op), seed=100 + op)
    gp, gu = sampled.torch_getters(psi[0], full["U"])
    ref = sampled.oracle_at_sites(op, sites, DIMS, -1, gp, gu, NS, M0, full["w"], mq / (2 * M0))
    got = sampled.at_sites(out[0], sites)
    del out
    torch.cuda.empty_cache()
    return np.linalg.norm(got - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("op,mq", [(oracle.OP_D, 0.0025), (oracle.OP_DDAG, 0.5),
                                   (oracle.OP_HOP_EO, 0.04), (oracle.OP_SCHUR_NORMAL, 0.04)],
                         ids=["D_light", "DDAG_charm", "HOP_EO", "SCHUR_NORMAL_strange"])
def test_fullsize_fp64_sampled(full, src, op, mq):
    print(f"full size FP64 {NAMES[op]} mq={mq}", flush=True)
    err = _sampled_check(full, src, op, mq, odwf.FP64, 6 if op == oracle.OP_SCHUR_NORMAL else 16)
    print(f"  rel err over sampled sites {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("prec", [odwf.FP32, odwf.FP16S, odwf.BF16S], ids=["fp32", "fp16s", "bf16s"])
@pytest.mark.parametrize("op", [oracle.OP_HOP_EO, oracle.OP_SCHUR_NORMAL], ids=["HOP_EO", "SCHUR_NORMAL"])
def test_fullsize_reduced_precision_sampled(full, src, op, prec):
    print(f"full size {odwf.PREC_NAMES[prec]} {NAMES[op]}", flush=True)
    err = _sampled_check(full, src, op, 0.04, prec, 6 if op == oracle.OP_SCHUR_NORMAL else 16)
    print(f"  rel err vs FP64 oracle over sampled sites {err:.3e}")
    assert 0 < err <= PREC_BOUND[prec]


@pytest.fixture(scope="module")
def solve_sites(full, src):
    """Sampled sites for the solves' residuals and the links around them, kept
    on the host: the canonical gauge field and the operator input leave the
    device before the solves need the memory."""
    import torch
    src.clear()
    sites = sampled.pick_sites(DIMS, 16, None, seed=7)
    coords = np.concatenate([sampled.frame(s, DIMS, 1, -1)[0] for s in sites])
    lin = ((coords[:, 3] * DIMS[2] + coords[:, 2]) * DIMS[1] + coords[:, 1]) * DIMS[0] + coords[:, 0]
    uniq, first = np.unique(lin, return_index=True)
    ix = [torch.as_tensor(coords[first, k], device="cuda", dtype=torch.long) for k in (3, 2, 1, 0)]
    U_host = full["U"][ix[0], ix[1], ix[2], ix[3]].cpu().numpy()
    del full["U"], ix
    torch.cuda.empty_cache()

    def gu(c):
        cl = ((c[:, 3] * DIMS[2] + c[:, 2]) * DIMS[1] + c[:, 1]) * DIMS[0] + c[:, 0]
        return U_host[np.searchsorted(uniq, cl)]
    return sites, gu


@pytest.mark.parametrize("mq", [0.0025, 0.04, 0.5], ids=["light", "strange", "charm"])
def test_fullsize_mixed_solve_sampled_residual(full, solve_sites, mq):
    """The benchmark's solve at the three masses of the full-size
    configuration: FP32 inner CG with FP64 reliable updates, tolerance 1e-10,
    source seed 1005; the oracle recomputes b - D x at the sampled sites."""
    import torch
    sites, gu = solve_sites
    sol = odwf.Solver(full["lat"], NS, M0, full["w"])
    b = synth.make_source_device(DIMS, NS, 1, 1005)
    print(f"full size mixed solve fp32 inner, mq={mq}, tol 1e-10", flush=True)
    x, st = sol.solve(b, [mq], [1e-10], inner=odwf.FP32)
    sol.close()
    del sol
    torch.cuda.empty_cache()
    st = st[0]
    print(f"  {st}", flush=True)
    assert st["status"] == odwf.OK and st["true_rel_resid"] <= 1e-10
    bnorm = torch.linalg.vector_norm(b).item()
    gp = sampled.torch_getters(x[0], None)[0]
    Dx = sampled.oracle_at_sites(oracle.OP_D, sites, DIMS, -1, gp, gu, NS, M0, full["w"], mq / (2 * M0))
    bS = sampled.at_sites(b[0], sites)
    rS = np.linalg.norm(bS - Dx)
    print(f"  sampled |b - D x| / |b_S| = {rS / np.linalg.norm(bS):.3e}, "
          f"reported full residual {st['full_rel_resid']:.3e}")
    assert st["full_rel_resid"] <= 2e-8
    assert rS <= 1.05 * st["full_rel_resid"] * bnorm
    assert rS / np.linalg.norm(bS) <= 1e-6
    del x, b
    torch.cuda.empty_cache()
