"""Pins of the oracle's fermion force (CPU only), independent of its formula.

The force of the bilinear S(U) = Re <chi, W[U] psi> (W the hopping term of the
4D Wilson operator, which the HMC's fermion forces differentiate; paper §2) is
pinned by
  - the derivative it claims to be: for U_mu(x) -> exp(i eps T) U_mu(x), T
    Hermitian and traceless, the central difference of S computed with the
    oracle's (separately pinned) Wilson operator equals i tr(T F_mu(x)) to
    O(eps^2), on links inside the lattice, across the t boundary (both bc_t)
    and in an extent-2 direction (x + mu = x - mu);
  - gauge covariance: with U^g_mu(x) = g(x) U_mu(x) g(x+mu)^dag and the fields
    rotated by g, F^g_mu(x) = g(x) F_mu(x) g(x)^dag;
  - its algebra: F is traceless and anti-Hermitian.
"""
import numpy as np
import pytest

from dense_helpers import random_su3
from oracle import oracle
from paper_1811_08095_amd import synth

M0 = 1.3


def _fields(dims, Ns, seed):
    X, Y, Z, T = dims
    rng = np.random.default_rng(seed)
    sh = (Ns, T, Z, Y, X, 4, 3)
    chi = rng.standard_normal(sh) + 1j * rng.standard_normal(sh)
    psi = rng.standard_normal(sh) + 1j * rng.standard_normal(sh)
    return chi, psi


def action(U, chi, psi, bc_t):
    """S = Re sum_s <chi_s, W psi_s>; the oracle's D_w with m0 = 4 is the hopping term alone."""
    return sum(np.vdot(chi[s], oracle.dw(U, psi[s], 4.0, bc_t)).real for s in range(chi.shape[0]))


def _hermitian_traceless(rng):
    h = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    h = h + h.conj().T
    return h - np.trace(h) / 3 * np.eye(3)


def _expi(eps, T):
    w, V = np.linalg.eigh(T)
    return (V * np.exp(1j * eps * w)) @ V.conj().T


@pytest.mark.parametrize("bc_t", [1, -1])
def test_force_is_the_derivative_of_the_bilinear(bc_t):
    dims = (4, 2, 2, 4)  # y, z of extent 2: x + mu = x - mu
    X, Y, Z, T = dims
    U = synth.make_gauge(dims, 0.6, 5)
    chi, psi = _fields(dims, 2, 77)
    F = oracle.force(U, chi, psi, bc_t)
    rng = np.random.default_rng(8)
    # (t, z, y, x, mu): interior, the t boundary, extent-2 directions
    links = [(1, 0, 1, 2, 0), (T - 1, 1, 0, 3, 3), (0, 1, 1, 0, 1), (2, 0, 0, 1, 2), (T - 1, 0, 1, 0, 0)]
    eps = 1e-4
    for (t, z, y, x, mu) in links:
        for _ in range(2):
            Th = _hermitian_traceless(rng)
            Up, Um = U.copy(), U.copy()
            Up[t, z, y, x, mu] = _expi(eps, Th) @ U[t, z, y, x, mu]
            Um[t, z, y, x, mu] = _expi(-eps, Th) @ U[t, z, y, x, mu]
            fd = (action(Up, chi, psi, bc_t) - action(Um, chi, psi, bc_t)) / (2 * eps)
            an = 1j * np.trace(Th @ F[t, z, y, x, mu])
            assert abs(an.imag) < 1e-12 * max(1.0, abs(an.real))
            assert abs(fd - an.real) <= 1e-6 * max(1.0, abs(fd)), ((t, z, y, x, mu), fd, an)


def test_force_gauge_covariance():
    dims = (4, 2, 4, 2)
    X, Y, Z, T = dims
    U = synth.make_gauge(dims, 0.5, 12)
    chi, psi = _fields(dims, 3, 13)
    rng = np.random.default_rng(14)
    g = random_su3(rng, T * Z * Y * X).reshape(T, Z, Y, X, 3, 3)
    Ug = np.empty_like(U)
    for mu, ax in enumerate((3, 2, 1, 0)):
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ np.swapaxes(np.roll(g, -1, axis=ax).conj(), -1, -2)
    rot = lambda f: np.einsum("tzyxab,stzyxpb->stzyxpa", g, f)
    for bc in (1, -1):
        F = oracle.force(U, chi, psi, bc)
        Fg = oracle.force(Ug, rot(chi), rot(psi), bc)
        expect = g[..., None, :, :] @ F @ np.swapaxes(g.conj(), -1, -2)[..., None, :, :]
        assert np.abs(Fg - expect).max() < 1e-12 * np.abs(F).max()


def test_force_is_traceless_antihermitian():
    dims = (2, 2, 2, 2)
    U = synth.make_gauge(dims, 0.7, 1)
    chi, psi = _fields(dims, 4, 2)
    F = oracle.force(U, chi, psi, -1)
    assert np.abs(F + np.swapaxes(F.conj(), -1, -2)).max() < 1e-14 * np.abs(F).max()
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() < 1e-13 * np.abs(F).max()
    assert np.abs(F).max() > 0
