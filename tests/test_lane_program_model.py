"""Model of the lane-parallel fifth-dimension programs (CPU only).

At N_s = 16 the fused FP32 hopping kernels keep slice s of a (site, rhs) in
lane s of one 16-lane DPP row and run the cyclic bidiagonal products and
solves across the row.  This test emulates that row in numpy, lane by lane:
row shifts that hand lanes outside the row an identity value, row rotations,
and a broadcast of one lane to the row, and checks the resulting algorithm
(rotation for the products; a four-step scan over affine maps closed around
the cycle for the solves) against dense N_s x N_s matrices written from the
definition of the factors: diagonal d, off-diagonal e on the lower (L) or upper
(U) side, and the corner element kappa * e closing the cycle.  Chirality +
holds local index u in lane u, chirality - in lane N_s - 1 - u, so each
operation is checked with both lane orders.
"""
import numpy as np
import pytest

NS = 16


# ---- the row primitives ------------------------------------------------------
def shr(v, k, old):  # lane i reads lane i - k
    out = np.full_like(v, old)
    out[k:] = v[:-k]
    return out


def shl(v, k, old):  # lane i reads lane i + k
    out = np.full_like(v, old)
    out[:-k] = v[k:]
    return out


def ror(v, k):  # lane i reads lane (i - k) mod 16
    return np.roll(v, k)


def bcast(v, last):
    return np.full_like(v, v[NS - 1] if last else v[0])


# ---- the algorithm as the kernel runs it (values indexed by lane) ---------------
def lane_mul(y, d, e, rot):
    return d * y + e * ror(y, rot)


def lane_solve(b, a, down, last):
    for k in (1, 2, 4, 8):
        mv = shr if down else shl
        b = b + a * mv(b, k, 0.0)
        a = a * mv(a, k, 1.0)
    x_last = bcast(b / (1.0 - a), last)
    return b + a * x_last


# ---- dense factors from their definitions (local index u) ------------------------
def dense(d, e, kappa, upper):
    m = np.diag(d).astype(complex)
    for u in range(NS):
        if upper:
            if u < NS - 1:
                m[u, u + 1] = e[u]
            else:
                m[u, 0] = kappa * e[u]
        else:
            if u > 0:
                m[u, u - 1] = e[u]
            else:
                m[u, NS - 1] = kappa * e[u]
    return m


def to_lanes(v_local, chi):
    return v_local if chi == 0 else v_local[::-1]


def from_lanes(v_lane, chi):
    return v_lane if chi == 0 else v_lane[::-1]


CASES = [(chi, upper) for chi in (0, 1) for upper in (False, True)]
IDS = [f"chi{'+-'[c]}_{'UP' if u else 'LO'}" for c, u in CASES]


def _coeffs(seed):
    rng = np.random.default_rng(seed)
    d = 1.0 + rng.random(NS)
    e = rng.standard_normal(NS)
    kappa = -rng.random()  # -mu, mu in [0, 1)
    y = rng.standard_normal(NS) + 1j * rng.standard_normal(NS)
    return d, e, kappa, y


def _corner_lane(u_corner, chi):
    return u_corner if chi == 0 else NS - 1 - u_corner


@pytest.mark.parametrize("chi,upper", CASES, ids=IDS)
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_row_rotation_product_matches_dense(chi, upper, seed):
    d, e, kappa, y = _coeffs(seed)
    ref = dense(d, e, kappa, upper) @ y
    # the neighbour in local order: u - 1 (LO) or u + 1 (UP); in lanes it is one
    # rotation step, whose direction flips with the mirrored chirality
    rot = (1 if not upper else -1) * (1 if chi == 0 else -1)
    e_lane = to_lanes(e, chi).copy()
    e_lane[_corner_lane(NS - 1 if upper else 0, chi)] *= kappa
    got = from_lanes(lane_mul(to_lanes(y, chi), to_lanes(d, chi), e_lane, rot), chi)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("chi,upper", CASES, ids=IDS)
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_affine_scan_solve_matches_dense(chi, upper, seed):
    d, e, kappa, y = _coeffs(seed)
    ref = np.linalg.solve(dense(d, e, kappa, upper), y)
    dinv = to_lanes(1.0 / d, chi)
    e_lane = to_lanes(e, chi).copy()
    e_lane[_corner_lane(NS - 1 if upper else 0, chi)] *= kappa
    # x_u = dinv_u (y_u - e_u x_prev): the previous element in scan order is the
    # lower lane for (chi+, LO) and (chi-, UP), the higher lane otherwise; the
    # final element closes the cycle
    down = (chi == 0) != upper
    last = down
    got = from_lanes(lane_solve(dinv * to_lanes(y, chi), -dinv * e_lane, down, last), chi)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_scan_without_closure_is_the_open_recurrence():
    """With a zero corner (kappa = 0) the closure term vanishes and the scan is
    plain forward substitution."""
    d, e, _, y = _coeffs(7)
    ref = np.linalg.solve(dense(d, e, 0.0, False), y)
    e0 = e.copy()
    e0[0] = 0.0
    got = lane_solve(y / d, -e0 / d, True, True)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
