"""Effective 4D operator of the optimal domain-wall fermion (oracle side).

TEST INFRASTRUCTURE ONLY: used by the tests; never imported by the library.

Paper §2: with the R5-symmetric optimal weights the effective 4D operator of
the optimal domain-wall fermion is exactly the shifted Zolotarev optimal
rational approximation of the overlap operator.  With the normalisation of the
Pauli-Villars factors of Eq. (1)-(2) (mu = m_q / m_PV, m_PV = 2 m0) it reads
    D_eff(mu) = (1 + mu)/2 + (1 - mu)/2 gamma5 S(H_w),
    S(H) = (1 - prod_s T_s)(1 + prod_s T_s)^{-1},  T_s = (1 - w_s H)(1 + w_s H)^{-1},
    H_w = gamma5 D_w.
This module writes that definition out densely (small lattices): H_w from the
oracle's Wilson operator, S through the eigendecomposition of the Hermitian
H_w (numpy's eigh is the library primitive).  Basis of 4D fields:
[t][z][y][x][spin][colour].
"""
import numpy as np

from . import oracle
from .zolotarev import sign_approx_matrix


def dense_dw(U, m0, bc_t):
    """Matrix of the oracle's 4D Wilson operator (column by column)."""
    T, Z, Y, X = U.shape[:4]
    n = T * Z * Y * X * 12
    M = np.zeros((n, n), np.complex128)
    e = np.zeros(n, np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        M[:, j] = oracle.dw(U, e.reshape(T, Z, Y, X, 4, 3), m0, bc_t).reshape(n)
    return M


def gamma5(V):
    return np.kron(np.eye(V), np.kron(np.diag([1.0, 1.0, -1.0, -1.0]), np.eye(3)))


def deff_matrix(U, m0, omega, mu, bc_t=-1):
    """D_eff(mu) as a dense matrix."""
    T, Z, Y, X = U.shape[:4]
    V = T * Z * Y * X
    g5 = gamma5(V)
    Hw = g5 @ dense_dw(U, m0, bc_t)
    Hw = 0.5 * (Hw + Hw.conj().T)  # Hermitian up to rounding (gamma5-hermiticity of D_w)
    S = sign_approx_matrix(Hw, omega)
    return 0.5 * (1 + mu) * np.eye(V * 12) + 0.5 * (1 - mu) * (g5 @ S)


def deff_apply(U, q, m0, omega, mu, bc_t=-1, inverse=False):
    """D_eff(mu) q (or D_eff(mu)^{-1} q) for 4D fields q[rhs][t][z][y][x][4][3]."""
    M = deff_matrix(U, m0, omega, mu, bc_t)
    n = M.shape[0]
    Q = np.asarray(q, np.complex128).reshape(-1, n).T
    out = np.linalg.solve(M, Q) if inverse else M @ Q
    return out.T.reshape(np.shape(q))
