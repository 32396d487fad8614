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


# --- The modified 3-level cycle of Sec. 5 ------------------------------------
# Between the fine restriction and prolongation the correction runs 4 cycles of
# the next level as the stationary iteration e <- e + M_1 (r_c - D_1 e) from
# e = 0.  The three pins below fix it against exact results that do not reuse
# the oracle's loop: a level-1 operator c I (every step of the cycle becomes a
# scalar map, so the residual after k cycles has a closed form), a unitary
# second prolongator (M_1 = D_1^{-1}, so the correction is the exact level-1
# solve), and a cycle without smoothing or step size (M_1 D_1 is then a
# projector and the correction is M_1 r_c, independent of the count).

def _scaled_identity_level(site_shape, nv, c):
    n2 = 2 * nv
    x = np.broadcast_to(c * np.eye(n2, dtype=np.complex128), tuple(site_shape) + (n2, n2)).copy()
    y = np.zeros((4, 2) + tuple(site_shape) + (n2, n2), dtype=np.complex128)
    return coarse.StencilLevel(x, y, nv)


@pytest.mark.parametrize("cycles,omega", [(4, 0.5), (3, 0.5), (4, 0.8), (2, 0.3)])
def test_three_level_correction_closed_form_on_scaled_identity(cycles, omega):
    """Level-1 operator D_1 = c I (complex c), exact coarsest solve, alpha on.

    An MR step on c I maps r to (1 - omega) r with x += omega r / c.  The
    level-2 correction is y = Pi res / c with Pi = P_2 P_2^dagger, so
    D_1 y = Pi res and alpha = 1; the post-smoother then scales (1 - Pi) res.
    One level-1 V(2,2) cycle therefore has residual map
    T = (1 - omega)^4 (1 - Pi), and after k stationary cycles the residual is
    T^k r_c = (1 - omega)^(4k) (1 - Pi) r_c, i.e.
    e_k = [r_c - (1 - omega)^(4k) (1 - Pi) r_c] / c.  A cycle that never
    updates its residual, a wrong cycle count or an exact level-1 solve in
    place of the cycles all miss this by far more than rounding."""
    dims, blk1, blk2, nv1, nv2 = (4, 4, 4, 8), (2, 2, 2, 2), (2, 2, 2, 2), 2, 3
    c = 1.7 + 0.4j
    lev0 = _wilson_level(dims, seed=71)
    v1 = transfer.as_chiral(synthetic.gaussian_vectors((nv1,) + (8, 4, 4, 4) + (4, 3), 72))
    q1, _ = transfer.block_orthonormalize(v1, blk1)
    lev1 = _scaled_identity_level((4, 2, 2, 2), nv1, c)
    v2 = synthetic.gaussian_vectors((nv2, 4, 2, 2, 2, 2, nv1), 73)
    q2, _ = transfer.block_orthonormalize(v2, blk2)
    lev2 = coarse.build_stencil(lev1, q2, blk2)
    h = mg.Hierarchy([lev0, lev1, lev2], [q1, q2], [blk1, blk2], omega=omega,
                     coarse_cycles=[cycles, 1], coarse_tol=1e-15, coarse_maxit=50)
    r = transfer.as_chiral(synthetic.gaussian_spinor(dims, seed=74))
    rc = transfer.restrict(q1, r, blk1)
    pi_rc = transfer.prolong(q2, transfer.restrict(q2, rc, blk2), blk2)
    ek = (rc - (1 - omega) ** (4 * cycles) * (rc - pi_rc)) / c
    got = h.correction(0, r)
    want = transfer.prolong(q1, ek, blk1)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-13


def test_three_level_correction_is_exact_with_unitary_second_prolongator():
    """1^4 second-level aggregates with Nv_2 = Nv_1 make P_2 unitary; with an
    exact coarsest solve the level-1 V-cycle is then D_1^{-1} (the Galerkin
    D_2 = P_2^dagger D_1 P_2 is D_1 in another basis), every further cycle
    adds nothing, and the correction equals P_1 D_1^{-1} P_1^dagger r with D_1
    the dense Galerkin operator on a 3^4 level-1 grid (distinct +-mu
    neighbours)."""
    dims, blk1, blk2, nv1 = (6, 6, 6, 6), (2, 2, 2, 2), (1, 1, 1, 1), 3
    lev0 = _wilson_level(dims, eps=0.3, m=-0.3, seed=75)
    v1 = transfer.as_chiral(synthetic.gaussian_vectors((nv1,) + dims + (4, 3), 76))
    q1, _ = transfer.block_orthonormalize(v1, blk1)
    lev1 = coarse.build_stencil(lev0, q1, blk1)
    cs = (3, 3, 3, 3, 2, nv1)
    v2 = synthetic.gaussian_vectors((nv1,) + cs, 77)
    q2, _ = transfer.block_orthonormalize(v2, blk2)
    lev2 = coarse.build_stencil(lev1, q2, blk2)
    h = mg.Hierarchy([lev0, lev1, lev2], [q1, q2], [blk1, blk2], coarse_tol=1e-14,
                     coarse_maxit=5000)
    assert h.coarse_cycles == [4, 1]
    r = transfer.as_chiral(synthetic.gaussian_spinor(dims, seed=78))
    d1 = coarse.dense_from_apply(lambda f: coarse.apply_galerkin(lev0, q1, blk1, f), cs)
    rc = transfer.restrict(q1, r, blk1)
    want = transfer.prolong(q1, np.linalg.solve(d1, rc.reshape(-1)).reshape(cs), blk1)
    got = h.correction(0, r)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-10


def test_three_level_correction_without_smoothing_is_one_galerkin_solve():
    """With no smoothing, no step size and an exact coarsest solve,
    M_1 = P_2 D_2^{-1} P_2^dagger and (I - M_1 D_1) M_1 = 0, so the 4-cycle
    correction is P_1 M_1 P_1^dagger r whatever the count; a cycle that does
    not update its residual returns 4 times that."""
    dims, blk1, blk2, nv1, nv2 = (8, 8, 8, 8), (2, 2, 2, 2), (2, 2, 2, 2), 2, 3
    lev0 = _wilson_level(dims, eps=0.3, m=-0.3, seed=79)
    v1 = transfer.as_chiral(synthetic.gaussian_vectors((nv1,) + dims + (4, 3), 80))
    q1, _ = transfer.block_orthonormalize(v1, blk1)
    lev1 = coarse.build_stencil(lev0, q1, blk1)
    v2 = synthetic.gaussian_vectors((nv2, 4, 4, 4, 4, 2, nv1), 81)
    q2, _ = transfer.block_orthonormalize(v2, blk2)
    lev2 = coarse.build_stencil(lev1, q2, blk2)
    h = mg.Hierarchy([lev0, lev1, lev2], [q1, q2], [blk1, blk2], nu_pre=0, nu_post=0,
                     use_alpha=False, coarse_tol=1e-14, coarse_maxit=5000)
    cs2 = (2, 2, 2, 2, 2, nv2)
    d2 = coarse.dense_from_apply(lambda f: coarse.apply_galerkin(lev1, q2, blk2, f), cs2)
    r = transfer.as_chiral(synthetic.gaussian_spinor(dims, seed=82))
    rc2 = transfer.restrict(q2, transfer.restrict(q1, r, blk1), blk2)
    e2 = np.linalg.solve(d2, rc2.reshape(-1)).reshape(cs2)
    want = transfer.prolong(q1, transfer.prolong(q2, e2, blk2), blk1)
    got = h.correction(0, r)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-10


def test_alpha_step_leaves_a_residual_orthogonal_to_the_correction_image():
    # Sec. 3 step size: alpha = <D y, r> / <D y, D y> minimises ||r - alpha D y||,
    # so the new residual is orthogonal to D y (no smoothing around it here)
    dims, blk, nv = (4, 4, 4, 4), (2, 2, 2, 2), 3
    lev = _wilson_level(dims, seed=21)
    v = synthetic.gaussian_vectors((nv, 4, 4, 4, 4, 2, 6), 22)
    q, _ = transfer.block_orthonormalize(v, blk)
    st = coarse.build_stencil(lev, q, blk)
    h = mg.Hierarchy([lev, st], [q], [blk], nu_pre=0, nu_post=0, coarse_tol=1e-14, coarse_maxit=2000)
    r = transfer.as_chiral(synthetic.gaussian_spinor(dims, seed=23))
    x = h.vcycle(0, r)
    dy = lev.apply(h.correction(0, r))
    rn = r - lev.apply(x)
    assert abs(mg.dot(dy, rn)) <= 1e-12 * np.linalg.norm(dy) * np.linalg.norm(r)
    a = mg.dot(dy, r) / mg.dot(dy, dy)
    assert abs(a.imag) > 1e-3  # a complex step: a conjugated formula would not pass
