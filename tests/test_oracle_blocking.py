"""Negative control of the chirality-preserving blocking (Sec. 3 and its
footnote), through the oracle's two-level solver on dense 4^4 operators."""
import numpy as np
import pytest

import synthetic
from oracle import blocking, mg, wilson

DIMS = (4, 4, 4, 4)
SITES = (4, 4, 4, 4)
BLK = (2, 2, 2, 2)


@pytest.fixture(scope="module")
def free():
    """Free field (unit links), periodic time, m = 0.1: the constant spinor is an
    exact eigenvector of D with eigenvalue m."""
    u = synthetic.unit_gauge(DIMS)
    return u, blocking.dense_wilson(u, 0.1, 1.0)


@pytest.fixture(scope="module")
def rough():
    u = synthetic.gauge_field(DIMS, 0.3, 5)
    D = blocking.dense_wilson(u, -0.5, -1.0)
    v0 = synthetic.gaussian_vectors((2,) + SITES + (4, 3), 7)
    vecs = mg.relax_null_vectors(lambda f: wilson.apply_D(u, f, -0.5, -1.0), v0, 30)
    return u, D, vecs


def test_dense_wilson_is_the_oracle_operator(rough):
    u, D, _ = rough
    psi = synthetic.gaussian_spinor(DIMS, seed=11)
    assert np.allclose(D @ psi.reshape(-1), wilson.apply_D(u, psi, -0.5, -1.0).reshape(-1), atol=1e-13)


def test_prolongators_are_orthonormal_and_only_the_chiral_one_commutes_with_gamma5(rough):
    _, _, vecs = rough
    g5 = blocking.gamma5_matrix(SITES)
    for chiral, k in ((True, 1), (False, 2)):
        P = blocking.prolongator(vecs[:k], BLK, chiral=chiral)
        assert P.shape[1] == 16 * 2  # 16 aggregates, 2 coarse dof each in both cases
        assert np.allclose(P.conj().T @ P, np.eye(P.shape[1]), atol=1e-13)
        # [gamma5, P] = 0 means gamma5 P = P S with S = P^dagger gamma5 P (= diag(+-1))
        S = P.conj().T @ g5 @ P
        comm = np.linalg.norm(g5 @ P - P @ S)
        if chiral:
            assert comm < 1e-13 and np.allclose(np.abs(np.diagonal(S)), 1.0)
        else:
            assert comm > 0.1


def test_footnote_spin_blocking_of_the_constant_makes_the_gamma5_correction_ill_defined(free):
    u, D = free
    const = np.ones((1,) + SITES + (4, 3), dtype=np.complex128)
    b = synthetic.gaussian_spinor(DIMS, seed=12).reshape(-1)
    P = blocking.prolongator(const, BLK, chiral=False)
    g5 = blocking.gamma5_matrix(SITES)
    assert np.linalg.norm(P.conj().T @ g5 @ P) < 1e-14  # the footnote's P^dagger gamma5 P = 0
    tl = blocking.TwoLevel(D, SITES, P, gamma5_restriction=True)
    assert tl.coarse_singular_values()[0] < 1e-14 * np.linalg.norm(D)
    with pytest.raises(blocking.IllDefined):
        tl.cycle(b)
    # keeping chirality intact: the coarse operator keeps the exact eigenvalue m of
    # the constant mode (it lies in the range of P), and the solve converges
    Pc = blocking.prolongator(const, BLK, chiral=True)
    tc = blocking.TwoLevel(D, SITES, Pc, gamma5_restriction=True)
    assert np.allclose(tc.R @ Pc, np.diag(np.diagonal(tc.R @ Pc)), atol=1e-14)  # P^dagger gamma5 P = diag(+-1)
    ev = np.linalg.eigvals(Pc.conj().T @ D @ Pc)
    assert np.min(np.abs(ev - 0.1)) < 1e-12
    x, info = tc.solve(b)
    assert info["converged"] and np.linalg.norm(b - D @ x) <= 1e-10 * np.linalg.norm(b)


def test_with_chirality_intact_the_gamma5_factors_cancel(rough):
    _, D, vecs = rough
    P = blocking.prolongator(vecs[:1], BLK, chiral=True)
    a = blocking.TwoLevel(D, SITES, P, gamma5_restriction=True)
    g = blocking.TwoLevel(D, SITES, P, gamma5_restriction=False)
    r = synthetic.gaussian_spinor(DIMS, seed=13).reshape(-1)
    xa, xg = a.cycle(r), g.cycle(r)
    assert np.linalg.norm(xa - xg) <= 1e-12 * np.linalg.norm(xg)


def test_spin_blocking_with_gamma5_restriction_degrades_the_rough_field_solve(rough):
    """Same coarse dimension (2 per aggregate): chirality-split blocks of one
    relaxed candidate against spin blocks of two.  With the gamma5 restriction
    the spin-blocked coarse operator is nearly singular and the solve needs
    clearly more iterations."""
    _, D, vecs = rough
    b = synthetic.gaussian_spinor(DIMS, seed=14).reshape(-1)
    chi = blocking.TwoLevel(D, SITES, blocking.prolongator(vecs[:1], BLK, chiral=True), True)
    spin = blocking.TwoLevel(D, SITES, blocking.prolongator(vecs, BLK, chiral=False), True)
    s_chi, s_spin = chi.coarse_singular_values()[-1], spin.coarse_singular_values()[-1]
    assert s_spin < 0.1 * s_chi, (s_spin, s_chi)
    _, i_chi = chi.solve(b)
    _, i_spin = spin.solve(b)
    assert i_chi["converged"] and i_spin["converged"]
    assert i_spin["iters"] >= 1.3 * i_chi["iters"], (i_spin, i_chi)
