"""Pins of the oracle's MR smoother, coarse-grid correction, V-cycle and solvers.

Sec. 2 (V-cycle, E_TG, adaptive setup), Sec. 3 (correction with step alpha,
MR smoother with omega = 0.8), Sec. 5 (GCR outer, BiCGstab comparator).
"""
import numpy as np
import pytest

import synthetic
from oracle import coarse, mg, transfer, wilson


def test_mr_one_step_closed_form():
    # A = diag(1, 2), b = (1, 1), x0 = 0: p = (1, 2), <p,r> = 3, <p,p> = 5,
    # alpha = 0.8 * 3 / 5 = 0.48 -> x = (0.48, 0.48), r = (0.52, 0.04).
    a = np.diag([1.0, 2.0]).astype(complex)
    b = np.array([1.0, 1.0], dtype=complex)
    x, r = mg.mr(lambda v: a @ v, np.zeros(2, complex), b, 1, omega=0.8)
    assert np.allclose(x, [0.48, 0.48], atol=1e-15)
    assert np.allclose(r, [0.52, 0.04], atol=1e-15)


def test_mr_residual_non_increasing_and_recursive_residual_true():
    dims = (4, 4, 4, 4)
    u = synthetic.gauge_field(dims, 0.3, seed=2)
    b = synthetic.gaussian_spinor(dims, seed=3)
    ap = lambda v: wilson.apply_D(u, v, -0.2)  # noqa: E731
    x = np.zeros_like(b)
    r = b.copy()
    prev = np.linalg.norm(r)
    for _ in range(6):
        x, r = mg.mr(ap, x, r, 1, omega=0.8)
        now = np.linalg.norm(r)
        assert now <= prev * (1 + 1e-15)
        prev = now
    assert np.linalg.norm(r - (b - ap(x))) < 1e-12 * np.linalg.norm(b)
    # zero residual: the step is zero, not 0/0
    x2, r2 = mg.mr(ap, x, np.zeros_like(b), 2)
    assert np.array_equal(x2, x) and not np.any(r2)


def _wilson_level(dims, eps=0.3, m=-0.2, seed=5):
    return coarse.WilsonLevel(synthetic.gauge_field(dims, eps, seed=seed), m, -1.0)


def test_unitary_prolongator_makes_one_vcycle_exact():
    """1^4 aggregates with Nv = 6: P is unitary, the coarse solve is the fine solve."""
    dims = (2, 2, 2, 4)
    lev = _wilson_level(dims)
    v = synthetic.gaussian_vectors((6, 4, 2, 2, 2, 2, 6), 8)
    q, _ = transfer.block_orthonormalize(v, (1, 1, 1, 1))
    st = coarse.build_stencil(lev, q, (1, 1, 1, 1))
    h = mg.Hierarchy([lev, st], [q], [(1, 1, 1, 1)], coarse_tol=1e-14, coarse_maxit=5000)
    r = transfer.as_chiral(synthetic.gaussian_spinor(dims, seed=9))
    x = h.vcycle(0, r)
    assert np.linalg.norm(lev.apply(x) - r) / np.linalg.norm(r) < 1e-11


def _dense_coarse(st, cs):
    return coarse.dense_from_apply(st.apply, cs)


def test_coarse_correction_exact_on_range_of_DP_and_projector():
    dims, blk, nv = (4, 4, 4, 4), (2, 2, 2, 2), 2
    lev = _wilson_level(dims, seed=11)
    v = synthetic.gaussian_vectors((nv, 4, 4, 4, 4, 2, 6), 12)
    q, _ = transfer.block_orthonormalize(v, blk)
    st = coarse.build_stencil(lev, q, blk)
    cs = (2, 2, 2, 2, 2, nv)
    dc = _dense_coarse(st, cs)
    h = mg.Hierarchy([lev, st], [q], [blk], coarse_tol=1e-14, coarse_maxit=2000)
    w = synthetic.gaussian_vectors(cs, 13)
    r = lev.apply(transfer.prolong(q, w, blk))
    y = h.correction(0, r)
    dy = lev.apply(y)
    alpha = mg.dot(dy, r) / mg.dot(dy, dy)
    assert abs(alpha - 1) < 1e-12
    assert np.linalg.norm(y - transfer.prolong(q, w, blk)) / np.linalg.norm(y) < 1e-11

    # pi_A = P D_c^{-1} P^dagger D (the E_TG projector): pi^2 = pi and pi P = P
    def pi(f):
        rc = transfer.restrict(q, lev.apply(f), blk).reshape(-1)
        return transfer.prolong(q, np.linalg.solve(dc, rc).reshape(cs), blk)
    f = transfer.as_chiral(synthetic.gaussian_spinor(dims, seed=14))
    p1 = pi(f)
    assert np.linalg.norm(pi(p1) - p1) / np.linalg.norm(p1) < 1e-12
    pw = transfer.prolong(q, w, blk)
    assert np.linalg.norm(pi(pw) - pw) / np.linalg.norm(pw) < 1e-12


def test_krylov_solvers_match_dense_solve():
    dims = (4, 4, 4, 4)
    u = synthetic.gauge_field(dims, 0.3, seed=15)
    m = -0.1
    b = synthetic.gaussian_spinor(dims, seed=16)
    ap = lambda v: wilson.apply_D(u, v, m)  # noqa: E731
    xs = np.linalg.solve(wilson.dense_D(u, m), b.reshape(-1)).reshape(b.shape)
    x1, i1 = mg.gcr(ap, b, 1e-10, restart=50)
    x2, i2 = mg.bicgstab(ap, b, 1e-10)
    for x, info in ((x1, i1), (x2, i2)):
        assert info["converged"] and info["true_res"] <= 1e-10
        assert np.linalg.norm(b - ap(x)) / np.linalg.norm(b) <= 1e-10
        assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-8


@pytest.mark.slow
def test_mg_fgcr_converges_with_fewer_iterations():
    dims = (8, 8, 8, 8)
    u = synthetic.gauge_field(dims, 0.3, seed=17)
    m = -0.55
    b = transfer.as_chiral(synthetic.gaussian_spinor(dims, seed=18))
    h = mg.build_hierarchy(u, m, -1.0, [(4, 4, 4, 4)], [6], seeds=[19], setup_iters=20,
                           coarse_tol=1e-2)
    x, info = h.solve(b, tol=1e-10, restart=50)
    assert info["converged"]
    lev = h.ops[0]
    assert np.linalg.norm(b - lev.apply(x)) / np.linalg.norm(b) <= 1e-10
    _, plain = mg.gcr(lev.apply, b, 1e-10, restart=50)
    assert info["iters"] < plain["iters"]


def test_three_level_cycle_runs_and_reduces_residual():
    dims = (8, 8, 8, 8)
    u = synthetic.gauge_field(dims, 0.3, seed=21)
    h = mg.build_hierarchy(u, -0.3, -1.0, [(2, 2, 2, 2), (2, 2, 2, 2)], [3, 4],
                           seeds=[22, 23], setup_iters=10, coarse_tol=1e-3)
    assert h.coarse_cycles == [4, 1]
    b = transfer.as_chiral(synthetic.gaussian_spinor(dims, seed=24))
    x = h.vcycle(0, b)
    assert np.linalg.norm(b - h.ops[0].apply(x)) < 0.9 * np.linalg.norm(b)


def _wilson_op(dims, eps, seed, m):
    u = synthetic.gauge_field(dims, eps, seed)
    return coarse.WilsonLevel(u, m, -1.0)


def test_adaptive_step_is_the_complementary_galerkin_projection():
    """With no smoothing, alpha = 1 and an (essentially) exact coarsest solve,
    one refinement step maps x to x - P D_c^{-1} P^dagger A x; since
    D_c = P^dagger A P this leaves P^dagger A x_new = 0 (Sec. 2)."""
    dims, blk = (4, 4, 4, 4), (2, 2, 2, 2)
    op = _wilson_op(dims, 0.3, 41, -0.3)
    v0 = transfer.as_chiral(synthetic.gaussian_vectors((3,) + dims + (4, 3), 42))
    kw = dict(nu_pre=0, nu_post=0, use_alpha=False, coarse_tol=1e-13, coarse_maxit=4000)
    vecs = mg.adaptive_null_vectors(op, v0, blk, iters=2, adapt_iters=1, **kw)
    relaxed = mg.relax_null_vectors(op.apply, v0, 2)
    for k in (1, 2):
        q, _ = transfer.block_orthonormalize(vecs[:k], blk)
        before = np.linalg.norm(transfer.restrict(q, op.apply(relaxed[k]), blk))
        after = np.linalg.norm(transfer.restrict(q, op.apply(vecs[k]), blk))
        assert after <= 1e-9 * before, (k, after, before)
        # the first k candidates are those of the previous steps, unchanged
        assert np.array_equal(vecs[:1], relaxed[:1])


def test_adaptive_candidates_are_smoother_and_span_p():
    """Refined candidates have a smaller residual ||A v|| / ||v|| than their
    relaxed starting points (the two-level iteration damps the smooth error
    slower than the rough), adapt_iters = 0 is plain relaxation, and the block
    QR of the candidates satisfies P^dagger P = I and P P^dagger v_k = v_k."""
    dims, blk, nv = (4, 4, 4, 4), (2, 2, 2, 2), 4
    op = _wilson_op(dims, 0.3, 43, -0.3)
    v0 = transfer.as_chiral(synthetic.gaussian_vectors((nv,) + dims + (4, 3), 44))
    relaxed = mg.relax_null_vectors(op.apply, v0, 3)
    assert np.array_equal(mg.adaptive_null_vectors(op, v0, blk, 3, 0), relaxed)
    vecs = mg.adaptive_null_vectors(op, v0, blk, 3, 3, coarse_tol=1e-12, coarse_maxit=4000)
    for k in range(1, nv):
        ratio_before = np.linalg.norm(op.apply(relaxed[k]))
        ratio_after = np.linalg.norm(op.apply(vecs[k]))
        assert ratio_after < ratio_before, (k, ratio_after, ratio_before)
        assert abs(np.linalg.norm(vecs[k]) - 1.0) < 1e-13
    q, _ = transfer.block_orthonormalize(vecs, blk)
    c = synthetic.gaussian_vectors((2, 2, 2, 2, 2, nv), 45)
    assert np.allclose(transfer.restrict(q, transfer.prolong(q, c, blk), blk), c, atol=1e-13)
    for k in range(nv):
        back = transfer.prolong(q, transfer.restrict(q, vecs[k], blk), blk)
        assert np.allclose(back, vecs[k], atol=1e-12)


def test_right_preconditioned_bicgstab():
    """With M = A^{-1} the first step is exact (alpha = 1, s = 0): one
    iteration; with the multigrid V-cycle as M the solution equals the dense
    solve and needs fewer iterations than without."""
    dims, blk = (4, 4, 4, 4), (2, 2, 2, 2)
    u = synthetic.gauge_field(dims, 0.3, seed=51)
    m = -0.2
    b = synthetic.gaussian_spinor(dims, seed=52)
    ap = lambda v: wilson.apply_D(u, v, m)  # noqa: E731
    dense = wilson.dense_D(u, m)
    xs = np.linalg.solve(dense, b.reshape(-1)).reshape(b.shape)
    inv = lambda f: np.linalg.solve(dense, f.reshape(-1)).reshape(f.shape)  # noqa: E731
    x, info = mg.bicgstab(ap, b, 1e-12, precond=inv)
    assert info["iters"] == 1 and np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-12
    op = coarse.WilsonLevel(u, m, -1.0)
    v0 = transfer.as_chiral(synthetic.gaussian_vectors((4,) + dims + (4, 3), 53))
    q, _ = transfer.block_orthonormalize(mg.relax_null_vectors(op.apply, v0, 10), blk)
    h = mg.Hierarchy([op, coarse.build_stencil(op, q, blk)], [q], [blk], coarse_tol=1e-12, coarse_maxit=4000)
    pre = lambda f: transfer.as_spinor(h.vcycle(0, transfer.as_chiral(f)))  # noqa: E731
    xm, im = mg.bicgstab(ap, b, 1e-10, precond=pre)
    _, i0 = mg.bicgstab(ap, b, 1e-10)
    assert im["converged"] and np.linalg.norm(xm - xs) / np.linalg.norm(xs) < 1e-8
    assert im["iters"] < i0["iters"], (im["iters"], i0["iters"])
