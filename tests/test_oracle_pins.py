"""Pins of the FP64 CPU oracle against facts fixed by the paper and by the
mathematics, independent of the oracle's own formulas (CPU only).

Each test names the passage or theorem that fixes the expected result.
Paper: Chiu, LATTICE2018, arXiv:1811.08095.
"""
import numpy as np
import pytest

from dense_helpers import (dense_dw, dense_of, dense_op, gamma5_full, m5_full, random_su3)
from oracle import oracle
from oracle.zolotarev import omega_zolotarev, sign_approx, sign_approx_matrix
from paper_1811_08095_amd import synth

M0 = 1.3  # §2: m0 = 1.3
LMIN, LMAX = 0.05, 6.2  # §2: lambda_max / lambda_min = 6.20 / 0.05


def test_gamma_algebra():
    """Chiral basis: Hermitian, Clifford algebra {g_mu, g_nu} = 2 delta, and
    gamma5 = g1 g2 g3 g4 = diag(1, 1, -1, -1) (the spinor-layout convention)."""
    g = oracle.gammas()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T, atol=0)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2.0 * (mu == nu) * np.eye(4), atol=1e-15)
    assert np.allclose(g[4], np.diag([1, 1, -1, -1]), atol=1e-15)


@pytest.mark.parametrize("bc_t", [1, -1])
def test_dw_gamma5_hermiticity(bc_t):
    """gamma5 D_w gamma5 = D_w^dag exactly (Wilson fermions; H_w = gamma5 D_w is
    Hermitian, §2 'H = H_w')."""
    U = synth.make_gauge((2, 2, 2, 2), 0.7, 11)
    D = dense_dw(U, M0, bc_t)
    G5 = gamma5_full(16)
    assert np.abs(G5 @ D @ G5 - D.conj().T).max() < 1e-14
    Ddag = dense_dw(U, M0, bc_t, dag=True)
    assert np.abs(Ddag - D.conj().T).max() < 1e-14


def _free_dw_symbol(p, m0, g):
    """Fourier symbol of the free Wilson operator with negative mass -m0:
    D_w(p) = sum_mu (1 - cos p_mu) - m0 + i sum_mu gamma_mu sin p_mu."""
    return (np.sum(1 - np.cos(p)) - m0) * np.eye(4) + 1j * sum(
        np.sin(p[m]) * g[m] for m in range(4))


@pytest.mark.parametrize("bc_t", [1, -1])
def test_dw_free_field_plane_waves(bc_t):
    """Unit links: a plane wave exp(i p.x) chi is an eigenvector of the hopping
    structure with the closed-form symbol (pins hop direction, the sign of
    gamma_mu in each projector, the 1/2 and the t boundary phase)."""
    X, Y, Z, T = 4, 4, 2, 6
    U = synth.unit_gauge((X, Y, Z, T))
    g = oracle.gammas()
    rng = np.random.default_rng(3)
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X),
                             indexing="ij")
    for trial in range(6):
        n = [rng.integers(0, L) for L in (X, Y, Z, T)]
        shift_t = 0.5 if bc_t == -1 else 0.0
        p = np.array([2 * np.pi * n[0] / X, 2 * np.pi * n[1] / Y, 2 * np.pi * n[2] / Z,
                      2 * np.pi * (n[3] + shift_t) / T])
        phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
        chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi = phase[..., None, None] * chi
        out = oracle.dw(U, psi, M0, bc_t)
        expect = phase[..., None, None] * (_free_dw_symbol(p, M0, g) @ chi)
        assert np.abs(out - expect).max() < 1e-13


def test_dw_gauge_covariance():
    """D_w[U^g](g psi) = g D_w[U] psi with U^g_mu(x) = g(x) U_mu(x) g(x+mu)^dag
    (pins link orientation: U vs U^dag and x vs x+mu)."""
    X, Y, Z, T = 4, 2, 4, 4
    U = synth.make_gauge((X, Y, Z, T), 0.5, 5)
    rng = np.random.default_rng(9)
    g = random_su3(rng, T * Z * Y * X).reshape(T, Z, Y, X, 3, 3)
    Ug = np.empty_like(U)
    for mu, ax in enumerate((3, 2, 1, 0)):
        g_fwd = np.roll(g, -1, axis=ax)
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ np.swapaxes(g_fwd.conj(), -1, -2)
    psi = rng.standard_normal((T, Z, Y, X, 4, 3)) + 1j * rng.standard_normal((T, Z, Y, X, 4, 3))
    gpsi = np.einsum("tzyxab,tzyxsb->tzyxsa", g, psi)
    for bc in (1, -1):
        lhs = oracle.dw(Ug, gpsi, M0, bc)
        rhs = np.einsum("tzyxab,tzyxsb->tzyxsa", g, oracle.dw(U, psi, M0, bc))
        assert np.abs(lhs - rhs).max() < 1e-13


def _rand5(rng, Ns, dims):
    X, Y, Z, T = dims
    sh = (Ns, T, Z, Y, X, 4, 3)
    return rng.standard_normal(sh) + 1j * rng.standard_normal(sh)


@pytest.mark.parametrize("op,adj", [(oracle.OP_D, oracle.OP_DDAG),
                                    (oracle.OP_SCHUR, oracle.OP_SCHUR_DAG)])
def test_adjoint_consistency(op, adj):
    """<chi, O psi> = <O^dag chi, psi> for separately coded adjoints."""
    dims = (4, 4, 2, 4)
    Ns = 8
    U = synth.make_gauge(dims, 0.5, 2)
    w = omega_zolotarev(LMIN, LMAX, Ns)
    rng = np.random.default_rng(4)
    psi, chi = _rand5(rng, Ns, dims), _rand5(rng, Ns, dims)
    if op == oracle.OP_SCHUR:
        ev = oracle.parity_mask((dims[3], dims[2], dims[1], dims[0]))
        psi = psi * ev[None, ..., None, None]
        chi = chi * ev[None, ..., None, None]
    mu = 0.05 / (2 * M0)
    a = np.vdot(chi, oracle.apply(op, U, psi, M0, w, mu))
    b = np.vdot(oracle.apply(adj, U, chi, M0, w, mu), psi)
    assert abs(a - b) < 1e-12 * abs(a)


def test_normal_ops_compose():
    """D^dag D and S_e^dag S_e are the compositions of their factors."""
    dims = (2, 4, 2, 2)
    Ns = 4
    U = synth.make_gauge(dims, 0.5, 8)
    w = omega_zolotarev(LMIN, LMAX, Ns)
    rng = np.random.default_rng(1)
    psi = _rand5(rng, Ns, dims)
    mu = 0.3
    for full, a, b in ((oracle.OP_DDAGD, oracle.OP_D, oracle.OP_DDAG),
                       (oracle.OP_SCHUR_NORMAL, oracle.OP_SCHUR, oracle.OP_SCHUR_DAG)):
        ref = oracle.apply(b, U, oracle.apply(a, U, psi, M0, w, mu), M0, w, mu)
        assert np.abs(oracle.apply(full, U, psi, M0, w, mu) - ref).max() < 1e-12


def _tiny_setup(Ns=4, eps=0.5, seed=0, bc_t=-1):
    dims = (2, 2, 2, 2)
    U = synth.make_gauge(dims, eps, seed)
    w = omega_zolotarev(LMIN, LMAX, Ns)
    return dims, U, w


@pytest.mark.parametrize("palindrome", [True, False])
def test_gamma5R5_hermiticity(palindrome):
    """With R5-symmetric weights (§2), D~ = w^{-1/2} D (1+L)^{-1} w^{-1/2} is
    Hermitian under Gamma5 = gamma5 R5, R5: s -> Ns+1-s; with weights that are
    not palindromic it is not (the symmetry the paper requires)."""
    dims, U, w = _tiny_setup()
    if not palindrome:
        w = np.sort(w)[::-1].copy()
    Ns, V = len(w), 16
    mu = 0.05 / (2 * M0)
    D = dense_op(oracle.OP_D, U, Ns, M0, w, mu, -1)
    inv1pL = m5_full(oracle.m5_matrix(Ns, M0, w, mu, oracle.M5_ONE_PLUS_L_INV), V)
    wmh = np.repeat(w ** -0.5, V * 12)
    Dt = (wmh[:, None] * (D @ inv1pL)) * wmh[None, :]
    R5 = np.kron(np.fliplr(np.eye(Ns)), np.eye(V * 12))
    G5 = np.kron(np.eye(Ns), gamma5_full(V))
    err = np.abs(G5 @ R5 @ Dt @ R5 @ G5 - Dt.conj().T).max() / np.abs(Dt).max()
    if palindrome:
        assert err < 1e-13
    else:
        assert err > 1e-2


@pytest.mark.parametrize("mq", [0.05, 0.5])
def test_determinant_identity_shifted_zolotarev(mq):
    """§2 and Eq. (1)-(2): the effective 4D operator of D_odwf is exactly the
    shifted-Zolotarev overlap, normalised by the Pauli-Villars operator
    D(m_PV), m_PV = 2 m0:
        det D(m_q) / det D(m_PV) = det[ (1+mu)/2 + (1-mu)/2 gamma5 S(H_w) ],
    mu = m_q / m_PV, S from the same weights, H_w = gamma5 D_w."""
    dims, U, w = _tiny_setup(eps=0.6, seed=21)
    Ns, V = len(w), 16
    mu = mq / (2 * M0)
    s_q, ld_q = np.linalg.slogdet(dense_op(oracle.OP_D, U, Ns, M0, w, mu, -1))
    s_pv, ld_pv = np.linalg.slogdet(dense_op(oracle.OP_D, U, Ns, M0, w, 1.0, -1))
    G5 = gamma5_full(V)
    Hw = G5 @ dense_dw(U, M0, -1)
    S = sign_approx_matrix(Hw, w)
    Deff = 0.5 * (1 + mu) * np.eye(V * 12) + 0.5 * (1 - mu) * G5 @ S
    s_e, ld_e = np.linalg.slogdet(Deff)
    assert abs((ld_q - ld_pv) - ld_e) < 1e-10
    assert abs(s_q / s_pv - s_e) < 1e-10


def test_m5_inverse_and_structure():
    """A A^{-1} = 1 and D = omega (A + W)(1 + L) with W = D_w - (4 - m0): the
    site-local factorisation behind even-odd preconditioning."""
    dims, U, w = _tiny_setup(Ns=4, seed=3)
    Ns, V = len(w), 16
    mu = 0.07
    A = oracle.m5_matrix(Ns, M0, w, mu, oracle.M5_A)
    Ai = oracle.m5_matrix(Ns, M0, w, mu, oracle.M5_AINV)
    assert np.abs(A @ Ai - np.eye(4 * Ns)).max() < 1e-13
    L = oracle.m5_matrix(Ns, M0, w, mu, oracle.M5_L)
    D = dense_op(oracle.OP_D, U, Ns, M0, w, mu, -1)
    Dw = dense_dw(U, M0, -1)
    W = np.kron(np.eye(Ns), Dw - (4 - M0) * np.eye(V * 12))
    Om = np.diag(np.repeat(w, V * 12))
    rebuilt = Om @ (m5_full(A, V) + W) @ m5_full(np.eye(4 * Ns) + L, V)
    assert np.abs(rebuilt - D).max() < 1e-12


@pytest.mark.parametrize("bc_t", [1, -1])
def test_eo_solve_matches_dense_inverse(bc_t):
    """Even-odd Schur solve + reconstruction equals the dense solve of D x = b
    on 2^4 x Ns=4 (pins the Schur complement, source preparation and
    reconstruction)."""
    dims = (2, 2, 2, 2)
    U = synth.make_gauge(dims, 0.5, 7)
    w = omega_zolotarev(LMIN, LMAX, 4)
    mu = 0.05 / (2 * M0)
    b = synth.make_source(dims, 4, 1, 1000)[0]
    D = dense_op(oracle.OP_D, U, 4, M0, w, mu, bc_t)
    x_dense = np.linalg.solve(D, b.reshape(-1)).reshape(b.shape)
    x, it, rr, fr = oracle.solve(U, b, M0, w, mu, oracle.SOLVE_FULL, tol=1e-13, maxiter=5000,
                                 bc_t=bc_t)
    assert it > 0
    assert rr <= 1e-13
    assert np.linalg.norm(x - x_dense) / np.linalg.norm(x_dense) < 1e-9
    assert fr < 1e-9


def test_eo_normal_solve_matches_dense():
    """EO_NORMAL mode solves S_e^dag S_e y = b_e; compare with the dense normal
    matrix restricted to even sites."""
    dims = (2, 2, 2, 2)
    Ns = 4
    U = synth.make_gauge(dims, 0.5, 17)
    w = omega_zolotarev(LMIN, LMAX, Ns)
    mu = 0.3
    b = synth.make_source(dims, Ns, 1, 3)[0]
    ev = oracle.parity_mask((2, 2, 2, 2))
    N = dense_op(oracle.OP_SCHUR_NORMAL, U, Ns, M0, w, mu, -1)
    sel = np.broadcast_to(ev[None, ..., None, None], b.shape).reshape(-1)
    Ne = N[np.ix_(sel, sel)]
    assert np.abs(Ne - Ne.conj().T).max() < 1e-12          # Hermitian
    assert np.linalg.eigvalsh(Ne).min() > 0                  # positive definite
    y_dense = np.linalg.solve(Ne, b.reshape(-1)[sel])
    y, it, rr, _ = oracle.solve(U, b, M0, w, mu, oracle.SOLVE_EO_NORMAL, tol=1e-12)
    assert rr <= 1e-12
    assert np.linalg.norm(y.reshape(-1)[sel] - y_dense) / np.linalg.norm(y_dense) < 1e-9
    assert np.all(y.reshape(-1)[~sel] == 0)


def test_cg_iteration_count_bounded_by_dimension():
    """Exact-arithmetic CG terminates in at most dim steps; in FP64 on a small,
    well-conditioned system it must reach 1e-10 well within that."""
    dims = (2, 2, 2, 2)
    U = synth.make_gauge(dims, 0.3, 0)
    w = omega_zolotarev(LMIN, LMAX, 4)
    b = synth.make_source(dims, 4, 1, 1000)[0]
    _, it, rr, _ = oracle.solve(U, b, M0, w, 0.5 / (2 * M0), oracle.SOLVE_FULL, tol=1e-10)
    assert 0 < it <= 8 * 4 * 12 and rr <= 1e-10


def _parity_split(dims):
    """Boolean masks (even, odd) over the rows of a dense 4D operator, basis
    [t][z][y][x][spin][colour]."""
    X, Y, Z, T = dims
    ev = np.repeat(oracle.parity_mask((T, Z, Y, X)).reshape(-1), 12)
    return ev, ~ev


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 6)], ids=["2^4", "4x2x2x6"])
@pytest.mark.parametrize("bc_t", [1, -1])
def test_hop_entries_are_parity_blocks_of_dense_wilson(dims, bc_t):
    """The even-odd hop entries of the oracle equal, slice by slice, the
    parity blocks of the pinned 4D Wilson matrix with its diagonal removed,
    W = D_w - (4 - m0) (the hopping term of D_w, §2 with H = H_w):
    HOP_EO gives W_eo psi_o on even sites and zeros on odd ones, HOP_OE gives
    W_oe psi_e on odd sites.  The input's other parity must not contribute."""
    X, Y, Z, T = dims
    V = X * Y * Z * T
    Ns = 4
    U = synth.make_gauge(dims, 0.6, 23)
    W = dense_dw(U, M0, bc_t) - (4 - M0) * np.eye(V * 12)
    ev, od = _parity_split(dims)
    rng = np.random.default_rng(41)
    psi = _rand5(rng, Ns, dims)
    w = omega_zolotarev(LMIN, LMAX, Ns)
    for op, rows, cols in ((oracle.OP_HOP_EO, ev, od), (oracle.OP_HOP_OE, od, ev)):
        out = oracle.apply(op, U, psi, M0, w, 0.01, bc_t).reshape(Ns, V * 12)
        blk = np.zeros_like(W)
        blk[np.ix_(rows, cols)] = W[np.ix_(rows, cols)]
        expect = psi.reshape(Ns, V * 12) @ blk.T
        assert np.abs(out - expect).max() < 1e-13
        assert np.all(out[:, ~rows] == 0)
    # the off-parity blocks of W vanish: W couples only opposite parities
    assert np.abs(W[np.ix_(ev, ev)]).max() == 0 and np.abs(W[np.ix_(od, od)]).max() == 0


def test_m5inv_entry_is_the_site_local_inverse():
    """M5INV applies A^{-1} (A = (4 - m0) + omega^{-1}(1 - L)(1 + L)^{-1}) at
    every site: the (s, spin) matrix of the oracle's m5_matrix, which the
    factorisation D = omega (A + W)(1 + L) pins, acting on each site's
    Ns x 4 x 3 block, and its product with A is the identity."""
    dims = (2, 2, 2, 4)
    Ns = 8
    U = synth.make_gauge(dims, 0.5, 5)
    w = omega_zolotarev(LMIN, LMAX, Ns)
    mu = 0.04 / (2 * M0)
    rng = np.random.default_rng(6)
    psi = _rand5(rng, Ns, dims)
    Ai = oracle.m5_matrix(Ns, M0, w, mu, oracle.M5_AINV)
    A = oracle.m5_matrix(Ns, M0, w, mu, oracle.M5_A)
    out = oracle.apply(oracle.OP_M5INV, U, psi, M0, w, mu)
    # psi[s][site][spin][colour] -> per site a (s, spin) vector for each colour
    v = np.moveaxis(psi.reshape(Ns, -1, 4, 3), 0, 1).reshape(-1, Ns * 4, 3)
    expect = np.moveaxis((Ai @ v).reshape(-1, Ns, 4, 3), 1, 0).reshape(psi.shape)
    assert np.abs(out - expect).max() < 1e-13
    back = np.moveaxis((A @ np.moveaxis(out.reshape(Ns, -1, 4, 3), 0, 1).reshape(-1, Ns * 4, 3))
                       .reshape(-1, Ns, 4, 3), 1, 0).reshape(psi.shape)
    assert np.abs(back - psi).max() < 1e-12


@pytest.mark.parametrize("bc_t", [1, -1])
def test_normal_residual_against_dense_schur_from_pinned_blocks(bc_t):
    """oracle_normal_residual(f, y) = |f_e - S_e^dag S_e y_e| / |f_e| with the
    even-site Schur complement S_e = 1 - A^{-1} W_eo A^{-1} W_oe built here
    densely from the pinned pieces (parity blocks of the dense Wilson matrix,
    the site-local A^{-1}), not from the oracle's Schur entries."""
    dims = (2, 2, 2, 2)
    X, Y, Z, T = dims
    V = 16
    Ns = 4
    U = synth.make_gauge(dims, 0.5, 13)
    w = omega_zolotarev(LMIN, LMAX, Ns)
    mu = 0.05 / (2 * M0)
    W = np.kron(np.eye(Ns), dense_dw(U, M0, bc_t) - (4 - M0) * np.eye(V * 12))
    Ainv = m5_full(oracle.m5_matrix(Ns, M0, w, mu, oracle.M5_AINV), V)
    ev4, od4 = _parity_split(dims)
    ev, od = np.tile(ev4, Ns), np.tile(od4, Ns)
    Weo, Woe = W[np.ix_(ev, od)], W[np.ix_(od, ev)]
    Ae, Ao = Ainv[np.ix_(ev, ev)], Ainv[np.ix_(od, od)]
    Se = np.eye(ev.sum()) - Ae @ Weo @ Ao @ Woe
    N = Se.conj().T @ Se
    rng = np.random.default_rng(19)
    f, y = _rand5(rng, Ns, dims), _rand5(rng, Ns, dims)
    fe, ye = f.reshape(-1)[ev], y.reshape(-1)[ev]
    # a y close to the solution, so the residual is small and a sign error is large
    ysol = np.linalg.solve(N, fe)
    ynear = y.reshape(-1).copy()
    ynear[ev] = ysol + 1e-6 * ye
    for yy in (y.reshape(-1), ynear):
        expect = np.linalg.norm(fe - N @ yy[ev]) / np.linalg.norm(fe)
        got = oracle.normal_residual(U, f, yy.reshape(f.shape), M0, w, mu, bc_t)
        # rounding of N y (entries of order |f|) bounds the difference, not its size
        assert abs(got - expect) <= 1e-12, (got, expect)


@pytest.mark.parametrize("mq", [0.01, 0.5])
def test_5d_free_field_blocks_give_the_pauli_villars_ratio(mq):
    """Unit links: the 5D operator maps a plane wave exp(i p.x) chi(s, spin) to
    a plane wave of the same momentum, colour by colour, so it block-
    diagonalises into 4 N_s x 4 N_s blocks D(p; mu) read off the oracle.  Per
    momentum, §2 fixes det D(p; mu) / det D(p; 1) = det[(1 + mu)/2 + (1 - mu)/2
    gamma5 S(H_w(p))], with H_w(p) = gamma5 D_w(p) and, on free fields,
    H_w(p)^2 = lambda_p^2 (lambda_p^2 = (sum(1 - cos p) - m0)^2 + sum sin^2 p),
    so S(H_w(p)) = S(lambda_p) H_w(p) / lambda_p with the Zolotarev S of the
    weights (pinned separately by equioscillation).  Pins the 5D momentum-space
    form: the s couplings, the mass term's corners and its chirality pairing."""
    dims = (4, 2, 2, 4)
    X, Y, Z, T = dims
    U = synth.unit_gauge(dims)
    Ns = 8
    w = omega_zolotarev(LMIN, LMAX, Ns)
    mu = mq / (2 * M0)
    g = oracle.gammas()
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    rng = np.random.default_rng(5)
    for _ in range(4):
        n = [rng.integers(0, L) for L in dims]
        p = np.array([2 * np.pi * n[0] / X, 2 * np.pi * n[1] / Y, 2 * np.pi * n[2] / Z,
                      2 * np.pi * (n[3] + 0.5) / T])  # bc_t = -1
        phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))

        def block(m):
            B = np.zeros((4 * Ns, 4 * Ns), np.complex128)
            for col in range(4 * Ns):
                for c in range(3):
                    psi = np.zeros((Ns, T, Z, Y, X, 4, 3), np.complex128)
                    psi[col // 4, ..., col % 4, c] = phase
                    out = oracle.apply(oracle.OP_D, U, psi, M0, w, m, -1)
                    # the image is the same plane wave in the same colour
                    coef = (out * phase.conj()[None, ..., None, None]).mean(axis=(1, 2, 3, 4))
                    rebuilt = coef[:, None, None, None, None, :, :] * phase[None, ..., None, None]
                    assert np.abs(out - rebuilt).max() < 1e-12
                    assert np.abs(np.delete(coef, c, axis=2)).max() < 1e-12
                    B[:, col] = coef[:, :, c].reshape(4 * Ns)
            return B

        ratio = np.linalg.det(block(mu)) / np.linalg.det(block(1.0))
        b = np.sum(1 - np.cos(p)) - M0
        Dw = b * np.eye(4) + 1j * sum(np.sin(p[m]) * g[m] for m in range(4))
        H = g[4] @ Dw
        lam = np.sqrt(b * b + np.sum(np.sin(p) ** 2))
        S = sign_approx(lam, w) * H / lam
        expect = np.linalg.det(0.5 * (1 + mu) * np.eye(4) + 0.5 * (1 - mu) * g[4] @ S)
        assert abs(ratio - expect) <= 1e-10 * abs(expect)
