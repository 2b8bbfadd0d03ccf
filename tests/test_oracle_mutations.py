"""The oracle's pins have teeth: each plausible mistake, planted in a separate
build of the oracle (-DORACLE_PLANT=k), makes at least one pin of
test_oracle_pins.py fail (CPU only).

Planted mistakes:
  1 sign of gamma_mu in the hop projectors flipped
  2 backward hop uses U_mu(x - mu) instead of its adjoint
  3 time-boundary factor bc_t dropped
  4 sign of the m_q boundary term in L_+ / L_- flipped
  5 both chiralities shifted the same way (L_+ built like L_-)
  6 Wilson mass term 5 - m0 instead of 4 - m0 in D
  7 Schur complement 1 + A^-1 W_eo A^-1 W_oe instead of 1 - ...
  8 hop normalised by -1 instead of -1/2
  9 z hop taken in the opposite direction
 10 even-odd hop entries with output and input parities exchanged
 11 normal-system residual formed as f + N y
 12 site-local A^{-1} applied transposed
 13 fermion force without the backward-hop term
 14 fermion force with the projector signs exchanged

Exchanging the chiral projectors of L_+ and L_- is not among them: that gives
R5 D R5 (R5: s -> Ns + 1 - s), the same operator up to relabelling s when
omega is palindromic, which no physical pin distinguishes; the convention is
fixed by the reading of the operator and the GPU path is held to it by parity.
"""
import pytest

import test_oracle_force as fpins
import test_oracle_pins as pins
from oracle import build, oracle

PLANTS = {1: "projector sign", 2: "missing link adjoint", 3: "boundary factor dropped",
          4: "boundary-term sign", 5: "one shift direction for both chiralities", 6: "Wilson mass 5 - m0",
          7: "Schur sign", 8: "hop normalisation", 9: "z hop reversed", 10: "hop parities swapped",
          11: "normal residual sign", 12: "A^-1 transposed", 13: "force without backward term",
          14: "force projector sign"}

# every pin, with the arguments its parametrisation uses
PIN_CALLS = [
    (pins.test_gamma_algebra, {}),
    (pins.test_dw_gamma5_hermiticity, {"bc_t": -1}),
    (pins.test_dw_free_field_plane_waves, {"bc_t": 1}),
    (pins.test_dw_free_field_plane_waves, {"bc_t": -1}),
    (pins.test_dw_gauge_covariance, {}),
    (pins.test_adjoint_consistency, {"op": oracle.OP_D, "adj": oracle.OP_DDAG}),
    (pins.test_normal_ops_compose, {}),
    (pins.test_gamma5R5_hermiticity, {"palindrome": True}),
    (pins.test_determinant_identity_shifted_zolotarev, {"mq": 0.05}),
    (pins.test_m5_inverse_and_structure, {}),
    (pins.test_eo_solve_matches_dense_inverse, {"bc_t": -1}),
    (pins.test_eo_normal_solve_matches_dense, {}),
    (pins.test_hop_entries_are_parity_blocks_of_dense_wilson, {"dims": (4, 2, 2, 6), "bc_t": -1}),
    (pins.test_m5inv_entry_is_the_site_local_inverse, {}),
    (pins.test_normal_residual_against_dense_schur_from_pinned_blocks, {"bc_t": -1}),
    (pins.test_5d_free_field_blocks_give_the_pauli_villars_ratio, {"mq": 0.5}),
    (fpins.test_force_is_the_derivative_of_the_bilinear, {"bc_t": -1}),
    (fpins.test_force_gauge_covariance, {}),
]


@pytest.mark.parametrize("plant", sorted(PLANTS), ids=[PLANTS[k] for k in sorted(PLANTS)])
def test_planted_mistake_fails_a_pin(plant, tmp_path):
    path = build.build(out=str(tmp_path / f"liboracle_plant{plant}.so"), plant=plant)
    caught = []
    with oracle.using_library(path):
        for fn, kw in PIN_CALLS:
            try:
                fn(**kw)
            except Exception:  # an assertion, or a solve that breaks down
                caught.append(fn.__name__ + (str(kw) if kw else ""))
    print(f"plant {plant} ({PLANTS[plant]}) caught by: {caught}")
    assert caught, f"no pin rejects planted mistake {plant}: {PLANTS[plant]}"


def test_unplanted_build_passes_every_pin(tmp_path):
    path = build.build(out=str(tmp_path / "liboracle_clean.so"))
    with oracle.using_library(path):
        for fn, kw in PIN_CALLS:
            fn(**kw)
