"""Pins of the 2d U(1) oracle (Sec. 4 workload) against closed forms,
invariants and library routines."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla
from scipy.special import iv

import synthetic
from oracle import qed2d, transfer

HERE = os.path.dirname(os.path.abspath(__file__))
# the gamma matrices of the 2d reading, written out here rather than taken
# from the oracle: gamma_0 = sigma_1, gamma_1 = sigma_2 (gamma5 = sigma_3)
PAULI = np.array([[[0, 1], [1, 0]], [[0, -1j], [1j, 0]]], dtype=np.complex128)


def _free(lx, lt):
    return np.ones((lt, lx, 2), dtype=np.complex128)


@pytest.mark.parametrize("t_bc", [1.0, -1.0])
def test_free_field_spectrum_is_the_closed_form(t_bc):
    # plane waves diagonalise the free operator: D(p) = m + sum_mu (1 - cos p_mu)
    # + i sum_mu gamma_mu sin p_mu, eigenvalues m + sum(1 - cos p) +- i |sin p|
    lx, lt, m = 6, 4, 0.3
    ev = np.linalg.eigvals(qed2d.sparse_D(_free(lx, lt), m, t_bc).toarray())
    px = 2 * np.pi * np.arange(lx) / lx
    pt = (2 * np.pi * np.arange(lt) + (np.pi if t_bc < 0 else 0.0)) / lt
    PX, PT = np.meshgrid(px, pt)
    re = m + (1 - np.cos(PX)) + (1 - np.cos(PT))
    im = np.sqrt(np.sin(PX) ** 2 + np.sin(PT) ** 2)
    want = np.concatenate([(re + 1j * im).ravel(), (re - 1j * im).ravel()])
    key = lambda z: (round(z.real, 9), round(z.imag, 9))  # noqa: E731
    np.testing.assert_allclose(np.array(sorted(ev, key=key)), np.array(sorted(want, key=key)), atol=1e-12)


def test_plane_wave_in_a_constant_background_is_shifted():
    # a constant U(1) link exp(i theta_mu) shifts the momentum by theta_mu
    lx, lt, m = 8, 6, 0.1
    th = (0.3, -0.7)
    u = np.ones((lt, lx, 2), dtype=np.complex128)
    u[..., 0], u[..., 1] = np.exp(1j * th[0]), np.exp(1j * th[1])
    p = (2 * np.pi * 3 / lx, 2 * np.pi * 1 / lt)
    t, x = np.meshgrid(np.arange(lt), np.arange(lx), indexing="ij")
    wave = np.exp(1j * (p[0] * x + p[1] * t))
    chi = np.array([0.6, -0.8j])
    psi = wave[..., None] * chi
    q = (p[0] + th[0], p[1] + th[1])
    Dp = (m + 2 - np.cos(q[0]) - np.cos(q[1])) * np.eye(2) + 1j * (
        PAULI[0] * np.sin(q[0]) + PAULI[1] * np.sin(q[1]))
    np.testing.assert_allclose(qed2d.apply_D(u, psi, m, 1.0), wave[..., None] * (Dp @ chi), atol=1e-13)


def test_two_formulations_agree():
    u = synthetic.u1_gauge_field((8, 6), 2.0, seed=3)
    psi = synthetic.gaussian_spinor_2d((8, 6), seed=4)
    A = qed2d.sparse_D(u, -0.2, -1.0)
    np.testing.assert_allclose((A @ psi.ravel()).reshape(psi.shape), qed2d.apply_D(u, psi, -0.2, -1.0), atol=1e-13)


def test_gamma5_hermiticity_and_gauge_covariance():
    lx, lt = 8, 6
    u = synthetic.u1_gauge_field((lx, lt), 1.0, seed=5)
    A = qed2d.sparse_D(u, -0.1, -1.0).toarray()
    g5 = qed2d.sparse_gamma5(lx * lt).toarray()
    np.testing.assert_allclose(g5 @ A @ g5, A.conj().T, atol=1e-14)
    # U'_mu(x) = g(x) U_mu(x) conj(g(x + mu))  =>  D' = G D G^dagger
    g = np.exp(1j * np.random.default_rng(6).uniform(-np.pi, np.pi, (lt, lx)))
    up = u.copy()
    up[..., 0] = g * u[..., 0] * np.conj(np.roll(g, -1, axis=1))
    up[..., 1] = g * u[..., 1] * np.conj(np.roll(g, -1, axis=0))
    G = np.diag(np.repeat(g.ravel(), 2))
    np.testing.assert_allclose(qed2d.sparse_D(up, -0.1, -1.0).toarray(), G @ A @ G.conj().T, atol=1e-13)


def test_u1_field_has_the_compact_u1_plaquette_distribution():
    # plaquette angles are von Mises(beta): <cos theta_P> = I1(beta) / I0(beta)
    u = synthetic.u1_gauge_field((128, 128), 6.0, seed=7000)
    P = u[..., 0] * np.roll(u[..., 1], -1, axis=1) * np.conj(np.roll(u[..., 0], -1, axis=0)) * np.conj(u[..., 1])
    assert abs(np.mean(P.real) - iv(1, 6.0) / iv(0, 6.0)) < 4 * 0.12 / 128
    np.testing.assert_allclose(np.abs(u), 1.0, atol=1e-15)


def _const_candidates(lx, lt):
    # one candidate, constant on both spins: the chirality split makes it one
    # constant column per chirality and aggregate (Nv = 1)
    return np.ones((1, lt, lx, 2, 1), dtype=np.complex128)


@pytest.mark.parametrize("block", [(4, 4), (2, 4)])
def test_galerkin_of_the_free_field_with_constant_candidates(block):
    # P of constant candidates (1/sqrt(b_x b_t) on an aggregate): D_c is the
    # coarse Wilson-like stencil diag = (2 + m) - sum_mu (b_mu - 1) / b_mu,
    # hop +-mu = -(1 / (2 b_mu)) (1 -+ gamma_mu) in chirality space
    lx, lt, m = 16, 12, 0.05
    q, _ = transfer.block_orthonormalize(qed2d.as_level(_const_candidates(lx, lt)), qed2d.block4(block))
    P = qed2d.prolongator_matrix(q, block)
    Dc = qed2d.galerkin(qed2d.sparse_D(_free(lx, lt), m, 1.0), P)
    cdims = (lx // block[0], lt // block[1])
    B = qed2d.stencil_blocks(Dc, cdims, 1, qed2d.OFFSETS_DIRECT)
    want = {(0, 0): (2 + m - sum((b - 1) / b for b in block)) * np.eye(2)}
    for mu in range(2):
        for s in (1, -1):
            d = (s, 0) if mu == 0 else (0, s)
            want[d] = -(np.eye(2) - s * PAULI[mu]) / (2 * block[mu])
    for o, d in enumerate(qed2d.OFFSETS_DIRECT):
        np.testing.assert_allclose(B[o], np.broadcast_to(want[d], B[o].shape), atol=1e-14)


def test_normal_galerkin_operator():
    lx, lt, block, nv = 12, 12, (2, 2), 2
    u = synthetic.u1_gauge_field((lx, lt), 3.0, seed=8)
    m = 0.1
    vecs = synthetic.gaussian_vectors((nv, lt, lx, 2, 1), seed=9)
    q, _ = transfer.block_orthonormalize(qed2d.as_level(vecs), qed2d.block4(block))
    P = qed2d.prolongator_matrix(q, block)
    D = qed2d.sparse_D(u, m, -1.0)
    A = qed2d.sparse_gamma5(lx * lt) @ D @ qed2d.sparse_gamma5(lx * lt) @ D
    Ac = qed2d.galerkin(A, P).toarray()
    # brute force: columns D P e_j through the shift-based operator and prolong
    nc = P.shape[1]
    cshape = (1, 1, lt // block[1], lx // block[0], 2, nv)
    cols = []
    for j in range(nc):
        e = np.zeros(nc, dtype=np.complex128)
        e[j] = 1.0
        f = transfer.prolong(q, e.reshape(cshape), qed2d.block4(block)).reshape(lt, lx, 2)
        cols.append(qed2d.apply_D(u, f, m, -1.0).ravel())
    DP = np.stack(cols, axis=1)
    np.testing.assert_allclose(Ac, DP.conj().T @ DP, atol=1e-12)
    assert np.linalg.eigvalsh((Ac + Ac.conj().T) / 2).min() > 0
    # two-step couplings of D^dagger D land on the 9-point coarse stencil
    B = qed2d.stencil_blocks(qed2d.galerkin(A, P), (lx // block[0], lt // block[1]), nv, qed2d.OFFSETS_NORMAL)
    assert np.abs(B[5:]).max() > 1e-3
    with pytest.raises(ValueError):
        qed2d.stencil_blocks(qed2d.galerkin(A, P), (lx // block[0], lt // block[1]), nv, qed2d.OFFSETS_DIRECT)


def test_solvers_reach_the_sparse_direct_solution():
    lx, lt = 16, 16
    u = synthetic.u1_gauge_field((lx, lt), 6.0, seed=10)
    m = 0.0
    b = synthetic.gaussian_spinor_2d((lx, lt), seed=11)
    exact = spla.spsolve(qed2d.sparse_D(u, m, -1.0).tocsc(), b.ravel()).reshape(b.shape)
    h = qed2d.build(u, m, -1.0, nvs=[4, 4], block=(2, 2), setup_iters=30, seeds=[12, 13])
    x, info = qed2d.mg_bicgstab(h, b, 1e-11)
    assert info["converged"]
    np.testing.assert_allclose(x, exact, atol=1e-9 * np.abs(exact).max())
    hn = qed2d.build(u, m, -1.0, nvs=[4, 4], block=(2, 2), setup_iters=30, seeds=[12, 13], normal=True)
    x, info = qed2d.mg_cg(hn, b, 1e-11)
    assert info["converged"]
    np.testing.assert_allclose(x, exact, atol=1e-9 * np.abs(exact).max())
    x, info = qed2d.cgnr(u, m, -1.0, b, 1e-11)
    assert info["converged"]
    np.testing.assert_allclose(x, exact, atol=1e-9 * np.abs(exact).max())
    # the coarsest level is solved to machine precision
    rc = synthetic.gaussian_vectors((1, 1, 4, 4, 2, 4), seed=14)
    ec = h.coarsest_solve(rc)
    assert np.linalg.norm(h.ops[-1].apply(ec) - rc) <= 1e-13 * np.linalg.norm(rc)


def test_mcrit_matches_dense_eigenvalues():
    u = synthetic.u1_gauge_field((8, 8), 6.0, seed=15)
    mc, _, res = qed2d.mcrit(u, ncv=30)
    ev = np.linalg.eigvals(qed2d.sparse_D(u, 0.0, -1.0).toarray())
    assert abs(mc + ev.real.min()) < 1e-10


def test_stored_mcrit_values_come_from_the_stored_recipe():
    with open(os.path.join(HERE, "golden", "mcrit_2d.json")) as fh:
        data = json.load(fh)
    e = data["32x32_beta6.0_seed7001"]
    u = synthetic.u1_gauge_field(tuple(e["dims"]), e["beta"], e["gauge_seed"])
    mc, _, _ = qed2d.mcrit(u, ncv=40)
    assert abs(mc - e["m_crit"]) < 1e-9


def test_spin_blocking_footnote_in_2d():
    # Sec. 3 footnote: blocking the spin makes P^dagger gamma5 P vanish for the
    # free-field constant, so the correction through gamma5 has no inverse;
    # keeping chirality (or restricting with P^dagger) keeps the mode's eigenvalue m
    lx, lt, m = 16, 12, 0.05
    D = qed2d.sparse_D(_free(lx, lt), m, 1.0)
    G = qed2d.sparse_gamma5(lx * lt)
    q, _ = transfer.block_orthonormalize(np.ones((1, 1, 1, lt, lx, 1, 2), dtype=np.complex128), (4, 4, 1, 1))
    P = qed2d.prolongator_matrix(q, (4, 4))
    assert abs((P.conj().T @ G @ P).toarray()).max() < 1e-15
    c = np.ones(P.shape[1])
    Dc_g5 = P.conj().T @ G @ D @ P
    assert np.linalg.norm(Dc_g5 @ c) < 1e-14 * np.linalg.norm(c) and abs(Dc_g5).max() > 0.1
    np.testing.assert_allclose((P.conj().T @ D @ P) @ c, m * c, atol=1e-14)
    # chirality kept: P^dagger gamma5 P is the coarse gamma5, and the constant keeps m
    qc, _ = transfer.block_orthonormalize(qed2d.as_level(_const_candidates(lx, lt)), (4, 4, 1, 1))
    Pc = qed2d.prolongator_matrix(qc, (4, 4))
    g5c = np.tile([1.0, -1.0], Pc.shape[1] // 2)
    np.testing.assert_allclose((Pc.conj().T @ G @ Pc).toarray(), np.diag(g5c), atol=1e-14)
    cc = np.ones(Pc.shape[1])
    np.testing.assert_allclose((Pc.conj().T @ G @ D @ Pc) @ cc, m * g5c, atol=1e-14)


def test_spin_blocked_hierarchies():
    # on a beta = 6 field the spin-blocked P with R = P^dagger is a well-defined
    # Galerkin method reaching the direct solution; with R = P^dagger gamma5 its
    # coarse operator is far worse conditioned and the solve needs more iterations
    lx = lt = 32
    u = synthetic.u1_gauge_field((lx, lt), 6.0, seed=10)
    b = synthetic.gaussian_spinor_2d((lx, lt), seed=11)
    exact = spla.spsolve(qed2d.sparse_D(u, 0.05, -1.0).tocsc(), b.ravel()).reshape(b.shape)
    its, conds = {}, {}
    for blk, nv in ((0, 4), (2, 8), (1, 8)):
        h = qed2d.build(u, 0.05, -1.0, nvs=[nv], block=(4, 4), setup_iters=50, seeds=[12], blocking=blk)
        sv = np.linalg.svd(h.mats[0].toarray(), compute_uv=False)
        conds[blk] = sv[0] / sv[-1]
        x, info = qed2d.mg_bicgstab(h, b, 1e-10, maxit=2000)
        assert info["converged"]
        np.testing.assert_allclose(x, exact, atol=1e-8 * np.abs(exact).max())
        its[blk] = info["iters"]
    assert conds[1] > 10 * conds[2] and its[1] > 2 * max(its[0], its[2]), (conds, its)
    with pytest.raises(ValueError):
        qed2d.build(u, 0.05, -1.0, nvs=[4, 4], block=(4, 4), setup_iters=5, seeds=[1, 2], blocking=1)
