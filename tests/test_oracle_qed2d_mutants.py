"""Planted mistakes in the 2d oracle (on the CPU): each must fail at least one
of the pins in test_oracle_qed2d.py, so that the pins, not the oracle's own
formulas, carry its correctness."""
import numpy as np
import pytest

from oracle import qed2d

import test_oracle_qed2d as pins


class _NumpyWithoutConj:
    """numpy with ``conj`` the identity: every backward link left unconjugated."""

    def __getattr__(self, name):
        return getattr(np, name)

    @staticmethod
    def conj(a):
        return a


def _fails(*checks):
    failed = 0
    for check in checks:
        try:
            check()
        except AssertionError:
            failed += 1
    return failed


def test_flipped_gamma_matrices_are_caught(monkeypatch):
    # (1 - gamma) and (1 + gamma) exchanged in both formulations
    monkeypatch.setattr(qed2d, "SIGMA", -qed2d.SIGMA)
    assert _fails(pins.test_plane_wave_in_a_constant_background_is_shifted) == 1


def test_unconjugated_backward_links_are_caught(monkeypatch):
    monkeypatch.setattr(qed2d, "np", _NumpyWithoutConj())
    assert _fails(pins.test_plane_wave_in_a_constant_background_is_shifted,
                  pins.test_gamma5_hermiticity_and_gauge_covariance) >= 1


def test_a_dropped_time_boundary_sign_is_caught(monkeypatch):
    apply_D, sparse_D = qed2d.apply_D, qed2d.sparse_D
    monkeypatch.setattr(qed2d, "apply_D", lambda u, psi, m, t_bc=-1.0: apply_D(u, psi, m, 1.0))
    monkeypatch.setattr(qed2d, "sparse_D", lambda u, m, t_bc=-1.0: sparse_D(u, m, 1.0))
    assert _fails(lambda: pins.test_free_field_spectrum_is_the_closed_form(-1.0)) == 1


def test_a_transposed_instead_of_adjoint_restriction_is_caught(monkeypatch):
    monkeypatch.setattr(qed2d, "galerkin", lambda A, P: (P.T @ A @ P).tocsr())
    assert _fails(pins.test_normal_galerkin_operator) == 1


def test_a_wrong_coarse_hop_block_is_caught(monkeypatch):
    # the coarse stencil read with the forward and backward offsets exchanged
    stencil_blocks = qed2d.stencil_blocks
    swapped = [qed2d.OFFSETS_DIRECT[i] for i in (0, 2, 1, 4, 3)]

    def mutant(M, dims2, n, offsets, groups=2):
        return stencil_blocks(M, dims2, n, swapped if offsets == qed2d.OFFSETS_DIRECT else offsets, groups)
    monkeypatch.setattr(qed2d, "stencil_blocks", mutant)
    assert _fails(lambda: pins.test_galerkin_of_the_free_field_with_constant_candidates((4, 4))) == 1


def test_an_inexact_coarsest_solve_is_caught(monkeypatch):
    # the coarsest level "solved" by one MR-like scaling instead of LU
    monkeypatch.setattr(qed2d.Hierarchy2d, "coarsest_solve", lambda self, rc: rc / 2.0)
    with pytest.raises(AssertionError):
        pins.test_solvers_reach_the_sparse_direct_solution()
