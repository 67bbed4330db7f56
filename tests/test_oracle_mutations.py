"""The pins must catch plausible mistakes: each case plants one in the oracle
(on the CPU, through monkeypatch) and checks that a pin then fails."""
import numpy as np
import pytest

import oracle.contract as C
import oracle.mpo as MPO
from tests import test_oracle_pins as pins


def _swap_phys(W):
    return np.ascontiguousarray(W.transpose(0, 1, 3, 2))


def test_transposed_mpo_in_heff_is_caught(monkeypatch):
    good = C.apply_heff
    monkeypatch.setattr(C, "apply_heff", lambda L, W, R, psi: good(L, _swap_phys(W), R, psi))
    with pytest.raises(AssertionError):
        pins.test_apply_heff_equals_kronecker_matrix(3, 2, 4, 5, 5)


def test_swapped_environment_legs_are_caught(monkeypatch):
    good = C.apply_heff
    monkeypatch.setattr(C, "apply_heff",
                        lambda L, W, R, psi: good(L, W, np.ascontiguousarray(R.transpose(2, 1, 0)), psi))
    with pytest.raises(AssertionError):
        pins.test_apply_heff_equals_kronecker_matrix(3, 2, 4, 5, 5)


def test_bra_ket_mixup_in_env_update_is_caught(monkeypatch):
    good = C.update_left
    monkeypatch.setattr(C, "update_left",
                        lambda L, W, A: good(np.ascontiguousarray(L.transpose(2, 1, 0)), W, A))
    with pytest.raises(AssertionError):
        pins.test_env_updates_equal_bruteforce()


def test_wrong_expansion_term_is_caught(monkeypatch):
    good = C.expansion_term_l2r
    monkeypatch.setattr(C, "expansion_term_l2r",
                        lambda L, W, psi, alpha: good(L, _swap_phys(W), psi, alpha))
    with pytest.raises(AssertionError):
        pins.test_worked_example_sec4_3(0.6, 0.8)


def test_missing_jordan_wigner_string_is_caught(monkeypatch):
    ops = MPO.fermion_site()
    good = MPO._finite_state_mpo

    def no_string(l, d, starts, strings, finishers, coupling, onsite, R):
        if d == 4:
            strings = [ops["I"]] * len(strings)
        return good(l, d, starts, strings, finishers, coupling, onsite, R)
    monkeypatch.setattr(MPO, "_finite_state_mpo", no_string)
    with pytest.raises(AssertionError):
        pins.test_long_range_hopping_mpo_equals_fock_ed()


def test_missing_range4_string_is_caught(monkeypatch):
    """Identity in place of F only on the last string step of a range-4
    hop: the range-3 pin on the 4 x 1 ring cannot see it, the 4 x 2 cylinder
    pin must."""
    ops = MPO.fermion_site()
    good = MPO._finite_state_mpo

    def bad(l, d, starts, strings, finishers, coupling, onsite, R):
        mpo = good(l, d, starts, strings, finishers, coupling, onsite, R)
        nk = len(starts)
        if d == 4 and R >= 4:
            for W in mpo:
                for k in range(nk):
                    a, b = 1 + 2 * nk + k, 1 + 3 * nk + k      # channels of ranges 3 and 4
                    if a < W.shape[0] and b < W.shape[1] and np.abs(W[a, b]).max() > 0:
                        W[a, b] = ops["I"]
        return mpo
    monkeypatch.setattr(MPO, "_finite_state_mpo", bad)
    pins.test_long_range_hopping_mpo_equals_fock_ed()
    bonds = MPO.cylinder_bonds(4, 2)
    hop = {b: 1.0 + 0.1 * k for k, b in enumerate(bonds)}
    H_unit = pins.ed.hubbard_hamiltonian(8, {b: 1.0 for b in bonds}, U=4.0)
    with pytest.raises(AssertionError):
        pins.test_cylinder_4x2_mpo_equals_fock_ed((bonds, hop, H_unit, H_unit))


def test_gram_floor_in_residual_truncation_is_caught(monkeypatch):
    """A residual truncation that drops values below the FP64 Gram
    resolution sqrt(n u) s_0 fails the dense-residual SVD pin."""
    good = C.truncation_size

    def floored(s, kmax, eps):
        return good(s, kmax, max(eps, np.sqrt(s.size * np.finfo(np.float64).eps)))
    monkeypatch.setattr(C, "truncation_size", floored)
    with pytest.raises(AssertionError):
        pins.test_residual_expanded_tensor_equals_dense_residual_svd("l2r", "heisenberg")


def test_residual_metric_without_square_root_is_caught(monkeypatch):
    good = C._metric_factor

    def bad(G):
        F = good(G)
        return F / np.sqrt(np.linalg.norm(F, axis=0))
    monkeypatch.setattr(C, "_metric_factor", bad)
    with pytest.raises(AssertionError):
        pins.test_residual_expanded_tensor_equals_dense_residual_svd("r2l", "hubbard")


def test_wrong_hopping_sign_is_caught(monkeypatch):
    ops = MPO.fermion_site()
    good = MPO._finite_state_mpo

    def bad_start(l, d, starts, strings, finishers, coupling, onsite, R):
        if d == 4:
            starts = [ops["cd_up"], ops["cd_dn"], ops["c_up"], ops["c_dn"]]   # F dropped
        return good(l, d, starts, strings, finishers, coupling, onsite, R)
    monkeypatch.setattr(MPO, "_finite_state_mpo", bad_start)
    with pytest.raises(AssertionError):
        pins.test_hubbard_mpo_equals_fock_ed(3, 4.0)


def test_wrong_neighbour_update_is_caught(monkeypatch):
    good = C.truncate_l2r

    def bad(Mt, psi, nbr, kmax, eps):
        A, B, s, disc = good(Mt, psi, nbr, kmax, eps)
        return A, B[::-1].copy(), s, disc        # rows of S V^T applied in the wrong order
    monkeypatch.setattr(C, "truncate_l2r", bad)
    with pytest.raises(AssertionError):
        pins.test_truncation_without_cut_keeps_state_and_discarded_weight("l2r")


def test_swapped_channel_pair_in_h2_environment_is_caught(monkeypatch):
    good = C.update_right_h2
    monkeypatch.setattr(C, "update_right_h2",
                        lambda G, W, B: np.ascontiguousarray(good(G, W, B).transpose(0, 2, 1, 3)))
    with pytest.raises(AssertionError):
        pins.test_h2_environments_equal_bruteforce("heisenberg")


@pytest.mark.parametrize("mistake", ["energy_sign", "no_cross_terms", "alpha_once"])
def test_wrong_residual_metric_is_caught(monkeypatch, mistake):
    good = C.residual_gram_l2r

    def bad(L, W, R, Gr, psi, E, alpha):
        if mistake == "energy_sign":
            return good(L, W, R, Gr, psi, -E, alpha)
        if mistake == "alpha_once":
            return good(L, W, R, Gr, psi, E, np.sqrt(alpha))
        return good(L, W, np.zeros_like(R), Gr, psi, E, alpha) + \
            (good(L, W, R, Gr, psi, E, 0.0) - good(L, W, np.zeros_like(R), Gr, psi, E, 0.0))
    monkeypatch.setattr(C, "residual_gram_l2r", bad)
    with pytest.raises(AssertionError):
        pins.test_residual_gram_equals_bruteforce("l2r", "heisenberg")
