"""Whole-lattice GPU parity on lattices that take the hopping kernel's tiled
traversal: (x-row segment, y, z) tiles with t innermost, which the library
selects when Lx/2 is a multiple of the sites per block (256 / (nrhs Ns)) and
Ly, Lz are multiples of the tile sides (8 or 4 by 4 by default) -- the
traversal of the 64^3 x 64 x 16 benchmark lattice, where the eight XCDs also
walk groups of adjacent tiles in lockstep.  The other traversals (lockstep
groups of several shapes, t chunks, whole-row tiles, linear) are forced
through the library's tuning variables and must give bitwise the same
operator results: the traversal only changes which block computes a site.

Every operator is compared with the FP64 CPU oracle element by element:
normwise |out - ref| / |ref| and per site, max over 5D sites of
|out(x, s) - ref(x, s)| / max over 5D sites of |ref(x, s)|, so that a single
wrong site cannot hide in the norm of a large lattice.
"""
import numpy as np
import pytest

from oracle import oracle
from paper_1811_08095_amd import odwf, synth

pytestmark = pytest.mark.gpu

M0 = 1.3
OPS = [odwf.OP_HOP_EO, odwf.OP_HOP_OE, odwf.OP_M5INV, odwf.OP_D, odwf.OP_DDAG, odwf.OP_DDAGD,
       odwf.OP_SCHUR, odwf.OP_SCHUR_DAG, odwf.OP_SCHUR_NORMAL]
OP_NAMES = ["HOP_EO", "HOP_OE", "M5INV", "D", "DDAG", "DDAGD", "SCHUR", "SCHUR_DAG", "SCHUR_NORMAL"]
DIMS = (32, 8, 8, 8)
NS = 16
MASSES = [0.04, 0.5]
# stated bounds of the reduced-precision operators against FP64 (normwise, per site)
PREC_BOUND = {odwf.FP32: (1e-5, 1e-5), odwf.FP16S: (4e-3, 8e-3), odwf.BF16S: (3e-2, 6e-2)}

_cache = {}


def takes_tiled_traversal(dims, Ns, nrhs):
    spb = 256 // (nrhs * Ns)
    return (dims[0] // 2) % spb == 0 and dims[1] % 4 == 0 and dims[2] % 4 == 0


# (name, ODWF_TRAVERSAL, ODWF_XCD); on DIMS the 2 x 2 tiles give 4 x 4 tiles in
# (y, z), so lockstep groups of 4 x 2 and 2 x 4 tiles exist
TRAVERSALS = [
    ("default", None, None),
    ("lockstep 4x2 groups of 2x2 one-segment tiles", "2,2,0,1", "lockstep:4"),
    ("lockstep 2x4 groups, t chunks of 4", "2,2,4,1", "lockstep:2"),
    ("contiguous XCD ranges, 4x4 whole-row tiles", "4,4,0,0", "contiguous"),
    ("contiguous XCD ranges, no tiles", "xcd", None),
    ("linear", "linear", None),
]


def _setup(bc):
    if bc in _cache:
        return _cache[bc]
    import torch
    U = synth.make_gauge(DIMS, 0.7, 31)
    w = odwf.zolotarev_omega(NS, 0.05, 6.2)
    lat = odwf.Lattice(DIMS, bc_t=bc)
    lat.load_gauge(U)
    sol = odwf.Solver(lat, NS, M0, w)
    psi = synth.make_source(DIMS, NS, len(MASSES), 2031)
    refs = {}
    _cache[bc] = (U, w, lat, sol, psi, torch.from_numpy(psi).cuda(), refs)
    return _cache[bc]


def _ref(bc, opi, r):
    U, w, lat, sol, psi, psid, refs = _setup(bc)
    key = (opi, r)
    if key not in refs:
        refs[key] = oracle.apply(OPS[opi], U, psi[r], M0, w, MASSES[r] / (2 * M0), bc)
    return refs[key]


def errors(out, ref):
    """(normwise relative error, per-site max error relative to the largest site)."""
    d = np.linalg.norm((out - ref).reshape(-1, 12), axis=1)
    rs = np.linalg.norm(ref.reshape(-1, 12), axis=1)
    return np.linalg.norm(out - ref) / np.linalg.norm(ref), d.max() / rs.max()


def test_lattice_takes_the_tiled_traversal():
    assert takes_tiled_traversal(DIMS, NS, 1) and takes_tiled_traversal(DIMS, NS, 2)
    assert takes_tiled_traversal((64, 64, 64, 64), NS, 1)


@pytest.mark.parametrize("bc", [-1, 1], ids=["bc-1", "bc+1"])
@pytest.mark.parametrize("nrhs", [1, 2], ids=["nrhs1", "nrhs2"])
@pytest.mark.parametrize("opi", range(len(OPS)), ids=OP_NAMES)
def test_fp64_tiled_parity(opi, nrhs, bc):
    U, w, lat, sol, psi, psid, refs = _setup(bc)
    print(f"tiled {DIMS} Ns={NS} bc={bc} nrhs={nrhs} op {OP_NAMES[opi]}", flush=True)
    out = sol.apply(OPS[opi], psid[:nrhs].contiguous(), MASSES[:nrhs], prec=odwf.FP64).cpu().numpy()
    for r in range(nrhs):
        en, es = errors(out[r], _ref(bc, opi, r))
        print(f"  rhs {r} m_q={MASSES[r]}: normwise {en:.2e}, per-site max {es:.2e}")
        assert en <= 1e-12 and es <= 1e-12, (OP_NAMES[opi], r, en, es)


@pytest.mark.parametrize("prec", [odwf.FP32, odwf.FP16S, odwf.BF16S], ids=["fp32", "fp16s", "bf16s"])
@pytest.mark.parametrize("nrhs", [1, 2], ids=["nrhs1", "nrhs2"])
@pytest.mark.parametrize("opi", [0, 8], ids=["HOP_EO", "SCHUR_NORMAL"])
def test_reduced_precision_tiled(opi, nrhs, prec):
    bc = -1
    U, w, lat, sol, psi, psid, refs = _setup(bc)
    out = sol.apply(OPS[opi], psid[:nrhs].contiguous(), MASSES[:nrhs], prec=prec).cpu().numpy()
    bn, bs = PREC_BOUND[prec]
    for r in range(nrhs):
        en, es = errors(out[r], _ref(bc, opi, r))
        print(f"{odwf.PREC_NAMES[prec]} {OP_NAMES[opi]} nrhs={nrhs} rhs {r}: normwise {en:.3e}, "
              f"per-site max {es:.3e} (vs FP64 oracle)")
        assert 0 < en <= bn and es <= bs, (en, es)


@pytest.mark.parametrize("prec", [odwf.FP64, odwf.FP32], ids=["fp64", "fp32"])
@pytest.mark.parametrize("nrhs", [1, 2], ids=["nrhs1", "nrhs2"])
def test_traversals_bitwise_identical(monkeypatch, nrhs, prec):
    bc = -1
    U, w, lat, sol, psi, psid, refs = _setup(bc)
    first = {}
    for name, trav, xcd in TRAVERSALS:
        if trav is None:
            monkeypatch.delenv("ODWF_TRAVERSAL", raising=False)
        else:
            monkeypatch.setenv("ODWF_TRAVERSAL", trav)
        if xcd is None:
            monkeypatch.delenv("ODWF_XCD", raising=False)
        else:
            monkeypatch.setenv("ODWF_XCD", xcd)
        print(f"traversal {name}: {DIMS} Ns={NS} nrhs={nrhs} {odwf.PREC_NAMES[prec]}", flush=True)
        for opi in (0, 1, 8):
            out = sol.apply(OPS[opi], psid[:nrhs].contiguous(), MASSES[:nrhs], prec=prec)
            if opi not in first:
                first[opi] = out
                bound = 1e-12 if prec == odwf.FP64 else PREC_BOUND[prec][0]
                o = out.cpu().numpy()
                for r in range(nrhs):
                    en, es = errors(o[r], _ref(bc, opi, r))
                    assert en <= bound and es <= max(bound, PREC_BOUND.get(prec, (0, 1e-12))[1]), (en, es)
            else:
                assert torch_equal(out, first[opi]), (name, OP_NAMES[opi])
    monkeypatch.delenv("ODWF_TRAVERSAL", raising=False)
    monkeypatch.delenv("ODWF_XCD", raising=False)


def torch_equal(a, b):
    import torch
    return bool(torch.equal(a, b))
