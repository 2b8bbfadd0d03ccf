"""ctypes front end of the FP64 CPU oracle (oracle/odwf_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it to produce expected values.  It never touches the GPU
library and the GPU library never calls it.

All fields are numpy complex128 arrays in the canonical layouts:
  gauge   U[t][z][y][x][mu][3][3]
  spinor  psi[s][t][z][y][x][spin][color]   (one right-hand side)
"""
import contextlib
import ctypes
import os

import numpy as np

from . import build as _build

OP_HOP_EO, OP_HOP_OE, OP_M5INV, OP_D, OP_DDAG, OP_DDAGD, OP_SCHUR, OP_SCHUR_DAG, \
    OP_SCHUR_NORMAL = range(9)
SOLVE_EO_NORMAL, SOLVE_FULL = 0, 1
M5_L, M5_ONE_PLUS_L_INV, M5_A, M5_AINV, M5_OMEGA, M5_OMEGA_INV = range(6)

_lib = None
_c128p = np.ctypeslib.ndpointer(dtype=np.complex128, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        _lib = _open(_build.ensure_built())
    return _lib


@contextlib.contextmanager
def using_library(path):
    """Run the oracle from another build of it (the mutation tests' variants
    with a planted mistake) inside the with-block."""
    global _lib
    saved = _lib
    _lib = _open(path)
    try:
        yield
    finally:
        _lib = saved


def _open(path):
    L = ctypes.CDLL(path)
    L.oracle_gammas.argtypes = [_c128p]
    L.oracle_dw.argtypes = [_i32p, ctypes.c_int, _c128p, ctypes.c_double, ctypes.c_int,
                            _c128p, _c128p]
    L.oracle_m5_matrix.argtypes = [ctypes.c_int, ctypes.c_double, _f64p, ctypes.c_double,
                                   ctypes.c_int, _c128p]
    L.oracle_apply.argtypes = [_i32p, ctypes.c_int, _c128p, ctypes.c_int, ctypes.c_double,
                               _f64p, ctypes.c_double, ctypes.c_int, _c128p, _c128p]
    L.oracle_solve.argtypes = [_i32p, ctypes.c_int, _c128p, ctypes.c_int, ctypes.c_double,
                               _f64p, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                               ctypes.c_int, _c128p, _c128p,
                               ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double)]
    L.oracle_normal_residual.argtypes = [_i32p, ctypes.c_int, _c128p, ctypes.c_int,
                                         ctypes.c_double, _f64p, ctypes.c_double,
                                         _c128p, _c128p]
    L.oracle_normal_residual.restype = ctypes.c_double
    L.oracle_force.argtypes = [_i32p, ctypes.c_int, _c128p, ctypes.c_int, _c128p, _c128p, _c128p]
    L.oracle_num_threads.restype = ctypes.c_int
    return L


def _dims(U):
    T, Z, Y, X = U.shape[:4]
    return np.array([X, Y, Z, T], dtype=np.int32)


def num_threads():
    """Threads the oracle's OpenMP loops use."""
    return int(lib().oracle_num_threads())


def gammas():
    """(gamma_1, gamma_2, gamma_3, gamma_4, gamma5) as the oracle builds them."""
    out = np.zeros((5, 4, 4), np.complex128)
    lib().oracle_gammas(out)
    return out


def dw(U, psi4, m0, bc_t=-1, dag=False):
    """4D Wilson-Dirac operator on a 4D spinor psi4[t][z][y][x][4][3]."""
    U = np.ascontiguousarray(U, np.complex128)
    psi4 = np.ascontiguousarray(psi4, np.complex128)
    out = np.zeros_like(psi4)
    lib().oracle_dw(_dims(U), int(bc_t), U, float(m0), int(bool(dag)), psi4, out)
    return out


def m5_matrix(Ns, m0, omega, mu, which):
    """(s, spin) matrix of dimension 4 Ns, index s*4 + spin."""
    out = np.zeros((4 * Ns, 4 * Ns), np.complex128)
    rc = lib().oracle_m5_matrix(int(Ns), float(m0), np.ascontiguousarray(omega, np.float64),
                                float(mu), int(which), out)
    if rc:
        raise RuntimeError("oracle_m5_matrix failed")
    return out


def apply(op, U, psi, m0, omega, mu, bc_t=-1):
    """out = op(psi) for one right-hand side psi[s][t][z][y][x][4][3]."""
    U = np.ascontiguousarray(U, np.complex128)
    psi = np.ascontiguousarray(psi, np.complex128)
    out = np.zeros_like(psi)
    rc = lib().oracle_apply(_dims(U), int(bc_t), U, psi.shape[0], float(m0),
                            np.ascontiguousarray(omega, np.float64), float(mu), int(op), psi, out)
    if rc:
        raise RuntimeError("oracle_apply failed")
    return out


def solve(U, b, m0, omega, mu, mode=SOLVE_FULL, tol=1e-10, maxiter=10000, bc_t=-1, x0=None):
    """Returns (x, iterations, normal-system residual, full-system residual)."""
    U = np.ascontiguousarray(U, np.complex128)
    b = np.ascontiguousarray(b, np.complex128)
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.complex128, copy=True)
    rr = ctypes.c_double()
    fr = ctypes.c_double()
    it = lib().oracle_solve(_dims(U), int(bc_t), U, b.shape[0], float(m0),
                            np.ascontiguousarray(omega, np.float64), float(mu), int(mode),
                            float(tol), int(maxiter), b, x, ctypes.byref(rr), ctypes.byref(fr))
    return x, it, rr.value, fr.value


def normal_residual(U, f, y, m0, omega, mu, bc_t=-1):
    """|f - S_e^dag S_e y| / |f| on even sites."""
    U = np.ascontiguousarray(U, np.complex128)
    return lib().oracle_normal_residual(_dims(U), int(bc_t), U, f.shape[0], float(m0),
                                        np.ascontiguousarray(omega, np.float64), float(mu),
                                        np.ascontiguousarray(f, np.complex128),
                                        np.ascontiguousarray(y, np.complex128))


def force(U, chi, psi, bc_t=-1):
    """Fermion force F_mu(x) = TA(U_mu(x) M_mu(x)) of S = Re <chi, W psi> (see
    oracle_force); chi, psi [s][t][z][y][x][4][3]; returns F [t][z][y][x][4][3][3]."""
    U = np.ascontiguousarray(U, np.complex128)
    F = np.zeros(U.shape, np.complex128)
    rc = lib().oracle_force(_dims(U), int(bc_t), U, chi.shape[0], np.ascontiguousarray(chi, np.complex128),
                            np.ascontiguousarray(psi, np.complex128), F)
    if rc:
        raise RuntimeError("oracle_force failed")
    return F


def parity_mask(dims_tzyx):
    """Boolean [t][z][y][x] array, True on even sites."""
    T, Z, Y, X = dims_tzyx
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X),
                             indexing="ij")
    return ((t + z + y + x) % 2) == 0
