"""Pins of the oracle's optimal weights omega_s (CPU only).

Paper §2: R5-symmetric weights, and 0 <= 1 - S(lambda) <= 2 d_Z on
[lambda_min, lambda_max] with the Zolotarev optimal rational approximation of
degree (n-1, n), N_s = 2n.  Optimality is pinned by the Chebyshev alternation
theorem: the best uniform approximation is characterised by equal-height
alternating extrema, so equioscillation of 1 - S with n + 1 equal maxima
(both endpoints and the n - 1 interior peaks between the n double zeros
lambda = 1/omega_k) identifies the minimax weights without any reference code.
"""
import os

import numpy as np
import pytest

from oracle.zolotarev import omega_zolotarev, sign_approx

LMIN, LMAX = 0.05, 6.2
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("Ns", [4, 8, 16])
def test_palindrome_and_positive(Ns):
    w = omega_zolotarev(LMIN, LMAX, Ns)
    assert w.shape == (Ns,)
    assert np.all(w > 0)
    assert np.array_equal(w, w[::-1])                       # R5 symmetry (§2)
    assert np.all(np.diff(w[: Ns // 2]) < 0)                # descending first half


def _local_maxima(lam, e):
    idx = [0] + [i for i in range(1, len(e) - 1) if e[i] >= e[i - 1] and e[i] > e[i + 1]] \
        + [len(e) - 1]
    return np.array(idx)


@pytest.mark.parametrize("Ns", [4, 8, 16])
def test_equioscillation(Ns):
    """1 - S(lambda) >= 0, its zeros sit at lambda = 1/omega_k, and it has
    exactly n + 1 local maxima on [lambda_min, lambda_max], all equal."""
    w = omega_zolotarev(LMIN, LMAX, Ns)
    n = Ns // 2
    # log grid resolves the peaks near lambda_min
    lam = np.geomspace(LMIN, LMAX, 400001)
    e = 1.0 - sign_approx(lam, w)
    assert e.min() > -1e-14
    for wk in w[:n]:
        assert abs(1.0 - sign_approx(np.array([1.0 / wk]), w)[0]) < 1e-14
    peaks = _local_maxima(lam, e)
    assert len(peaks) == n + 1
    # refine interior peaks with a golden-section search
    heights = [e[0], e[-1]]
    for i in peaks[1:-1]:
        a, b = lam[i - 1], lam[i + 1]
        g = (np.sqrt(5) - 1) / 2
        for _ in range(80):
            c, d = b - g * (b - a), a + g * (b - a)
            if 1 - sign_approx(np.array([c]), w)[0] > 1 - sign_approx(np.array([d]), w)[0]:
                b = d
            else:
                a = c
        heights.append(1 - sign_approx(np.array([(a + b) / 2]), w)[0])
    heights = np.array(heights)
    assert (heights.max() - heights.min()) / heights.max() < 1e-8


@pytest.mark.parametrize("Ns", [4, 8, 16])
def test_perturbed_weights_are_worse(Ns):
    """Minimax optimality: moving any single pair of weights raises the max
    deviation."""
    w = omega_zolotarev(LMIN, LMAX, Ns)
    lam = np.geomspace(LMIN, LMAX, 200001)
    best = np.max(1 - sign_approx(lam, w))
    for k in range(Ns // 2):
        for f in (0.99, 1.01):
            v = w.copy()
            v[k] *= f
            v[Ns - 1 - k] *= f
            assert np.max(1 - sign_approx(lam, v)) > best


def test_golden_values():
    """Regression fixture written by tests/golden/make_golden.py (oracle only)."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "omega_zolotarev.txt"))
            if not l.startswith("#")]
    for Ns in (4, 8, 16):
        w = omega_zolotarev(LMIN, LMAX, Ns)
        ref = np.array([float(r[3]) for r in rows if r[0] == "omega" and int(r[1]) == Ns])
        assert np.allclose(w, ref, rtol=1e-13, atol=0)
        md = [float(r[2]) for r in rows if r[0] == "maxdev" and int(r[1]) == Ns][0]
        lam = np.linspace(LMIN, LMAX, 2000001)
        assert abs(np.max(1 - sign_approx(lam, w)) - md) < 1e-9 * md
