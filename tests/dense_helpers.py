"""Dense-matrix helpers for the oracle pins on tiny lattices (CPU only).

They build the matrix of an oracle operator column by column, so every
property checked on the dense matrix is a property of the oracle itself.
"""
import numpy as np

from oracle import oracle


def dense_of(fn, shape):
    """Matrix of the linear map fn acting on complex arrays of the given shape."""
    n = int(np.prod(shape))
    M = np.zeros((n, n), np.complex128)
    e = np.zeros(n, np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        M[:, j] = fn(e.reshape(shape)).reshape(n)
    return M


def dense_dw(U, m0, bc_t, dag=False):
    T, Z, Y, X = U.shape[:4]
    return dense_of(lambda v: oracle.dw(U, v, m0, bc_t, dag), (T, Z, Y, X, 4, 3))


def dense_op(op, U, Ns, m0, omega, mu, bc_t):
    T, Z, Y, X = U.shape[:4]
    return dense_of(lambda v: oracle.apply(op, U, v, m0, omega, mu, bc_t), (Ns, T, Z, Y, X, 4, 3))


def gamma5_full(V):
    """gamma5 on a 4D field with V sites, basis [site][spin][color]."""
    g5 = np.diag([1.0, 1.0, -1.0, -1.0])
    return np.kron(np.eye(V), np.kron(g5, np.eye(3)))


def m5_full(M5, V):
    """(s, spin) matrix M5 (index s*4+spin) acting on a 5D field, basis
    [s][site][spin][color]."""
    Ns = M5.shape[0] // 4
    M = M5.reshape(Ns, 4, Ns, 4)
    out = np.einsum("satb,xy,cd->sxactybd", M, np.eye(V), np.eye(3))
    n = Ns * V * 12
    return out.reshape(n, n)


def random_su3(rng, n):
    """n Haar-ish random SU(3) matrices from QR of complex Gaussians."""
    z = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    return q / (det ** (1.0 / 3.0))[:, None, None]
