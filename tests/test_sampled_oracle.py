"""The per-site oracle evaluation used at full lattice size, pinned to the
whole-lattice oracle: at every sampled site (lattice corners, both time
boundaries, random sites) the frame evaluation equals the full evaluation for
every operator, both time boundary conditions and a non-cubic lattice."""
import numpy as np
import pytest

from oracle import oracle
from paper_1811_08095_amd import synth

import sampled

M0 = 1.3
OPS = [oracle.OP_HOP_EO, oracle.OP_HOP_OE, oracle.OP_M5INV, oracle.OP_D, oracle.OP_DDAG,
       oracle.OP_DDAGD, oracle.OP_SCHUR, oracle.OP_SCHUR_DAG, oracle.OP_SCHUR_NORMAL]


@pytest.mark.parametrize("dims,bc", [((10, 10, 10, 10), -1), ((10, 12, 10, 14), 1)])
def test_frame_equals_full_lattice(dims, bc):
    Ns, mq = 4, 0.04
    U = synth.make_gauge(dims, 0.5, 11)
    psi = synth.make_source(dims, Ns, 1, 12)[0]
    w = np.linspace(0.4, 1.7, Ns)  # any positive weights: the identity is algebraic
    gp, gu = sampled.numpy_getters(psi, U)
    for op in OPS:
        full = oracle.apply(op, U, psi, M0, w, mq / (2 * M0), bc)
        sites = sampled.pick_sites(dims, 6, sampled.OUT_PARITY.get(op), seed=op)
        assert any(s[3] in (0, dims[3] - 1) for s in sites)
        got = sampled.oracle_at_sites(op, sites, dims, bc, gp, gu, Ns, M0, w, mq / (2 * M0))
        ref = sampled.at_sites(full, sites)
        scale = np.abs(ref).max()
        assert scale > 0
        assert np.abs(got - ref).max() <= 1e-13 * scale, op


def test_frame_sees_the_boundary_sign():
    """Flipping bc_t changes the value at a t = 0 site and the frame follows."""
    dims, Ns = (10, 10, 10, 10), 4
    U = synth.make_gauge(dims, 0.5, 13)
    psi = synth.make_source(dims, Ns, 1, 14)[0]
    w = np.linspace(0.4, 1.7, Ns)
    gp, gu = sampled.numpy_getters(psi, U)
    site = [(0, 0, 0, 0)]
    a = sampled.oracle_at_sites(oracle.OP_D, site, dims, -1, gp, gu, Ns, M0, w, 0.01)
    b = sampled.oracle_at_sites(oracle.OP_D, site, dims, 1, gp, gu, Ns, M0, w, 0.01)
    assert np.abs(a - b).max() > 1e-3 * np.abs(a).max()
