"""Optimal weights omega_s and the shifted Zolotarev sign function (oracle side).

TEST INFRASTRUCTURE ONLY: used by the tests and the CPU-baseline leg of the
benchmark; never imported by the library.

Paper §2: with R5-symmetric weights (omega_s = omega_{N_s+1-s}) the effective
4D operator of the optimal domain-wall fermion equals the "shifted" Zolotarev
optimal rational approximation of the overlap operator, whose approximate sign
function
    S(lambda) = (1 - prod_s T_s) / (1 + prod_s T_s),
    T_s = (1 - omega_s lambda) / (1 + omega_s lambda),
obeys 0 <= 1 - S(lambda) <= 2 d_Z on [lambda_min, lambda_max], with
N_s = 2n and Zolotarev degree (n-1, n).

The weights are the closed-form optimal points of Chiu's optimal domain-wall
construction (the reading adopted where the paper gives properties only):
    kappa'^2 = 1 - lambda_min^2 / lambda_max^2,   K' = K(kappa'),
    omega_k = dn((2k - 1) K' / N_s; kappa') / lambda_min,   k = 1 .. N_s/2,
taken in descending order for s = 1..N_s/2 and mirrored (R5 symmetry).
scipy's elliptic routines are the library primitive for K and dn.
"""
import numpy as np
from scipy.special import ellipj, ellipk


def omega_zolotarev(lmin: float, lmax: float, Ns: int) -> np.ndarray:
    """Palindromic optimal weights omega_1..omega_Ns (float64)."""
    if Ns < 2 or Ns % 2:
        raise ValueError("Ns must be even and >= 2")
    m = 1.0 - (lmin / lmax) ** 2          # parameter m = kappa'^2
    K = ellipk(m)
    k = np.arange(1, Ns // 2 + 1)
    _, _, dn, _ = ellipj((2 * k - 1) * K / Ns, m)
    half = np.sort(dn / lmin)[::-1]        # descending
    return np.concatenate([half, half[::-1]]).astype(np.float64)


def sign_approx(lam, omega) -> np.ndarray:
    """S(lambda) for lambda > 0 (paper §2)."""
    lam = np.asarray(lam, dtype=np.float64)
    prod = np.ones_like(lam)
    for w in omega:
        prod = prod * (1.0 - w * lam) / (1.0 + w * lam)
    return (1.0 - prod) / (1.0 + prod)


def sign_approx_matrix(H: np.ndarray, omega) -> np.ndarray:
    """S(H) = (1 - prod T_s)(1 + prod T_s)^{-1}, T_s = (1 - w H)(1 + w H)^{-1},
    for a Hermitian matrix H, through its eigendecomposition."""
    lam, V = np.linalg.eigh(H)
    prod = np.ones_like(lam)
    for w in omega:
        prod = prod * (1.0 - w * lam) / (1.0 + w * lam)
    s = (1.0 - prod) / (1.0 + prod)
    return (V * s) @ V.conj().T
