"""Pins of the oracle's normal-equation multigrid (Sec. 3 normal equations,
Sec. 4 MG-CG and CG): the 33-block Galerkin stencil against the literal map,
Hermiticity and positivity, the closed-form mass
dependence through D_c, flexible CG against dense solves, CGNR and MG-CG to
the true residual."""
import numpy as np
import pytest

import synthetic
from oracle import coarse, mg, normal, transfer, wilson


def _setup(dims, block, nv, eps=0.3, m=-0.3, seed=301):
    u = synthetic.gauge_field(dims, eps, seed=seed)
    op = normal.NormalLevel(u, m, -1.0)
    v = transfer.as_chiral(synthetic.gaussian_vectors((nv,) + op.site_shape + (4, 3), seed + 1))
    q, _ = transfer.block_orthonormalize(v, block)
    return u, op, q


def test_offsets_are_the_two_step_couplings():
    assert len(normal.OFFSETS) == 33 and normal.OFFSETS[0] == (0, 0, 0, 0)
    assert all(sum(1 for v in d if v) <= 2 for d in normal.OFFSETS)
    assert len(set(normal.OFFSETS)) == 33


@pytest.mark.parametrize("dims,block,nv", [((6, 6, 6, 6), (2, 2, 2, 2), 1), ((12, 6, 6, 8), (4, 2, 2, 2), 2)])
def test_stencil_equals_the_literal_galerkin_map(dims, block, nv):
    u, op, q = _setup(dims, block, nv)
    st = normal.build_normal_stencil(op, q, block)
    c = synthetic.gaussian_vectors(st.site_shape + (2, nv), 302)
    lit = transfer.restrict(q, op.apply(transfer.prolong(q, c, block)), block)
    got = st.apply(c)
    assert np.abs(got - lit).max() <= 1e-12 * np.abs(lit).max()


def test_stencil_is_hermitian_positive_and_two_step_local():
    """The dense matrix of the literal map P^dagger (D^dagger D) P on a 3^4
    coarse lattice is Hermitian positive definite, equals the stencil's dense
    matrix, and couples only sites within one coarse step in at most two
    directions (the 33 offsets)."""
    dims, block, nv, m = (6, 6, 6, 6), (2, 2, 2, 2), 1, -0.3
    u, op, q = _setup(dims, block, nv, m=m)
    st = normal.build_normal_stencil(op, q, block)
    cs = st.site_shape + (2, nv)
    ac = coarse.dense_from_apply(lambda f: transfer.restrict(q, op.apply(transfer.prolong(q, f, block)), block), cs)
    assert np.abs(ac - ac.conj().T).max() < 1e-12 * np.abs(ac).max()
    assert np.linalg.eigvalsh(ac).min() > 0
    dense_st = coarse.dense_from_apply(st.apply, cs)
    assert np.abs(dense_st - ac).max() < 1e-12 * np.abs(ac).max()
    n2 = 2 * nv
    ext = st.site_shape
    nsite = int(np.prod(ext))
    for i in range(nsite):
        ci = np.unravel_index(i, ext)
        for j in range(nsite):
            cj = np.unravel_index(j, ext)
            d = [((cj[k] - ci[k] + 1) % ext[k]) - 1 for k in range(4)]
            if any(abs(v) > 1 for v in d) or sum(1 for v in d if v) > 2:
                assert np.abs(ac[i * n2:(i + 1) * n2, j * n2:(j + 1) * n2]).max() < 1e-13


def test_mass_dependence_through_the_direct_coarse_operator():
    """(D + dm)^dagger (D + dm) = D^dagger D + dm (D + D^dagger) + dm^2, and
    P^dagger P = I: A_c(m + dm) = A_c(m) + dm (D_c + D_c^dagger) + dm^2 I."""
    dims, block, nv, m, dm = (6, 6, 6, 6), (2, 2, 2, 2), 1, -0.3, 0.17
    u, op, q = _setup(dims, block, nv, m=m)
    st0 = normal.build_normal_stencil(op, q, block)
    st1 = normal.build_normal_stencil(normal.NormalLevel(u, m + dm, -1.0), q, block)
    dc = coarse.build_stencil(coarse.WilsonLevel(u, m, -1.0), q, block)
    cs = st0.site_shape + (2, nv)
    a0 = coarse.dense_from_apply(st0.apply, cs)
    a1 = coarse.dense_from_apply(st1.apply, cs)
    d = coarse.dense_from_apply(dc.apply, cs)
    want = a0 + dm * (d + d.conj().T) + dm * dm * np.eye(a0.shape[0])
    assert np.abs(a1 - want).max() < 1e-12 * np.abs(want).max()


def test_coarse_extent_two_is_refused():
    u, op, q = _setup((4, 4, 4, 4), (2, 2, 2, 2), 1)
    with pytest.raises(ValueError):
        normal.build_normal_stencil(op, q, (2, 2, 2, 2))


def test_fcg_is_cg_and_exact_with_the_inverse():
    rng = np.random.default_rng(5)
    n = 60
    z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    a = z.conj().T @ z + 0.5 * np.eye(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    xs = np.linalg.solve(a, b)
    x, info = normal.fcg(lambda v: a @ v, b, 1e-12)
    assert info["converged"] and np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-9
    # CG in exact arithmetic needs at most n steps
    assert info["iters"] <= 3 * n
    inv = np.linalg.inv(a)
    x1, i1 = normal.fcg(lambda v: a @ v, b, 1e-12, precond=lambda r: inv @ r)
    assert i1["iters"] == 1 and np.linalg.norm(x1 - xs) / np.linalg.norm(xs) < 1e-10


def test_cgnr_matches_the_dense_solve():
    dims, m = (4, 4, 4, 4), -0.1
    u = synthetic.gauge_field(dims, 0.3, seed=311)
    op = normal.NormalLevel(u, m, -1.0)
    b = transfer.as_chiral(synthetic.gaussian_spinor(dims, seed=312))
    x, info = normal.cgnr(op, b, 1e-10)
    assert info["converged"] and info["true_res"] <= 1e-10
    xs = np.linalg.solve(wilson.dense_D(u, m), transfer.as_spinor(b).reshape(-1)).reshape(transfer.as_spinor(b).shape)
    assert np.linalg.norm(transfer.as_spinor(x) - xs) / np.linalg.norm(xs) < 1e-8


def test_mg_cg_reaches_the_true_residual_in_fewer_iterations_than_cg():
    dims, m = (6, 6, 6, 6), -0.6
    u = synthetic.gauge_field(dims, 0.3, seed=321)
    h = normal.build_normal_hierarchy(u, m, -1.0, (2, 2, 2, 2), 3, seed=322, setup_iters=20, coarse_tol=1e-2)
    b = transfer.as_chiral(synthetic.gaussian_spinor(dims, seed=323))
    x, info = normal.mg_cg(h, b, 1e-10)
    assert info["converged"] and info["true_res"] <= 1e-10
    _, plain = normal.cgnr(h.ops[0], b, 1e-10)
    assert plain["converged"] and info["iters"] < plain["iters"]
