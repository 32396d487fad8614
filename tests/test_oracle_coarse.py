"""Pins of the oracle's coarse stencil D_c = P^dagger D P (Sec. 2, Sec. 3)."""
import numpy as np
import pytest

import synthetic
from oracle import coarse, transfer, wilson


def _setup(dims, blk, nv, eps=0.4, m=-0.3, seed=1):
    u = synthetic.gauge_field(dims, eps, seed=seed)
    lx, ly, lz, lt = dims
    v = synthetic.gaussian_vectors((nv, lt, lz, ly, lx, 2, 6), seed + 100)
    q, _ = transfer.block_orthonormalize(v, blk)
    lev = coarse.WilsonLevel(u, m, -1.0)
    return u, lev, q


def _cshape(dims, blk, nv):
    cd = transfer.coarse_dims(dims, blk)
    return (cd[3], cd[2], cd[1], cd[0], 2, nv)


@pytest.mark.parametrize("dims,blk", [
    ((8, 8, 8, 8), (4, 4, 4, 4)),   # coarse extent 2: +mu and -mu neighbours coincide
    ((8, 8, 4, 8), (2, 2, 2, 2)),   # 4 x 4 x 2 x 4 coarse
    ((6, 6, 6, 6), (2, 2, 2, 2)),   # 3^4 coarse: all nine blocks distinct
    ((4, 4, 4, 4), (4, 4, 4, 4)),   # one aggregate: everything folds into X + Y at one site
])
def test_stencil_matches_galerkin_definition(dims, blk):
    nv = 3
    _, lev, q = _setup(dims, blk, nv)
    st = coarse.build_stencil(lev, q, blk)
    fc = synthetic.gaussian_vectors(_cshape(dims, blk, nv), 5)
    ref = coarse.apply_galerkin(lev, q, blk, fc)
    out = st.apply(fc)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-14


def test_dense_galerkin_is_nearest_neighbour_and_matches_blocks():
    dims, blk, nv = (6, 6, 6, 6), (2, 2, 2, 2), 2
    _, lev, q = _setup(dims, blk, nv, seed=3)
    cs = _cshape(dims, blk, nv)
    dense = coarse.dense_from_apply(lambda f: coarse.apply_galerkin(lev, q, blk, f), cs)
    st = coarse.build_stencil(lev, q, blk)
    n2 = 2 * nv
    c = 3
    blocks = dense.reshape(c, c, c, c, n2, c, c, c, c, n2)
    for t in range(c):
        for z in range(c):
            for y in range(c):
                for x in range(c):
                    here = np.array([x, y, z, t])
                    for t2 in range(c):
                        for z2 in range(c):
                            for y2 in range(c):
                                for x2 in range(c):
                                    d = (np.array([x2, y2, z2, t2]) - here) % c
                                    blk_ = blocks[t, z, y, x, :, t2, z2, y2, x2, :]
                                    nz = np.count_nonzero(d)
                                    if nz == 0:
                                        assert np.abs(blk_ - st.x[t, z, y, x]).max() < 1e-14
                                    elif nz == 1:
                                        mu = int(np.nonzero(d)[0][0])
                                        si = 0 if d[mu] == 1 else 1
                                        assert np.abs(blk_ - st.y[mu, si, t, z, y, x]).max() < 1e-14
                                    else:
                                        assert np.abs(blk_).max() == 0.0


def test_coarse_gamma5_hermiticity_and_mass_shift():
    dims, blk, nv = (8, 4, 4, 8), (2, 2, 2, 4), 3
    u, lev, q = _setup(dims, blk, nv, seed=7)
    st = coarse.build_stencil(lev, q, blk)
    cs = _cshape(dims, blk, nv)
    a = synthetic.gaussian_vectors(cs, 1)
    b = synthetic.gaussian_vectors(cs, 2)
    g5 = np.array([1.0, -1.0])[:, None]
    lhs = np.vdot(a, g5 * st.apply(b))
    rhs = np.vdot(g5 * st.apply(a), b)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    # D_c(m + dm) = D_c(m) + dm I, because P^dagger P = I
    lev2 = coarse.WilsonLevel(u, lev.m + 0.25, -1.0)
    st2 = coarse.build_stencil(lev2, q, blk)
    assert np.abs(st2.apply(a) - st.shifted(0.25).apply(a)).max() < 1e-13


@pytest.mark.parametrize("b,t_bc", [(2, -1.0), (4, -1.0), (2, 1.0)])
def test_free_field_coarse_operator_closed_form(b, t_bc):
    """Unit links with the 6 constant vectors e_{s,c} + e_{s+2,c}: the Galerkin
    operator is (1/b) times the Wilson operator on the coarse lattice at mass b*m."""
    dims = (8, 8, 8, 8)
    m = 0.21
    u = synthetic.unit_gauge(dims)
    v = np.zeros((6, 8, 8, 8, 8, 4, 3), dtype=complex)
    for s in range(2):
        for c in range(3):
            v[3 * s + c, ..., s, c] = 1.0
            v[3 * s + c, ..., s + 2, c] = 1.0
    blk = (b, b, b, b)
    q, _ = transfer.block_orthonormalize(transfer.as_chiral(v), blk)
    st = coarse.build_stencil(coarse.WilsonLevel(u, m, t_bc), q, blk)
    nc = 8 // b
    fc = synthetic.gaussian_vectors((nc, nc, nc, nc, 2, 6), 4)
    uc = synthetic.unit_gauge((nc, nc, nc, nc))
    ref = transfer.as_chiral(wilson.apply_D(uc, transfer.as_spinor(fc), b * m, t_bc)) / b
    assert np.abs(st.apply(fc) - ref).max() < 1e-13


def test_spin_blocking_footnote_gives_zero_gamma5_projection():
    """Sec. 3 footnote: blocking the full spin dimension of the free-field null
    vector (the constant) gives P^dagger gamma5 P = 0 on every aggregate."""
    b = 2
    v = np.zeros((b, b, b, b, 4, 3), dtype=complex)
    v[..., 0, 0] = v[..., 2, 0] = 1.0
    col = v.reshape(-1) / np.linalg.norm(v)
    g5col = wilson.apply_gamma5(col.reshape(v.shape)).reshape(-1)
    assert abs(np.vdot(col, g5col)) < 1e-15
    # whereas each chirality-split column has <p, gamma5 p> = +-1
    plus = v.copy()
    plus[..., 2:, :] = 0
    plus = plus.reshape(-1) / np.linalg.norm(plus)
    assert abs(np.vdot(plus, wilson.apply_gamma5(plus.reshape(v.shape)).reshape(-1)) - 1) < 1e-15


def test_second_level_stencil_matches_galerkin():
    dims = (8, 8, 8, 8)
    blk1, nv1 = (2, 2, 2, 2), 2
    blk2, nv2 = (2, 2, 2, 2), 3
    _, lev, q1 = _setup(dims, blk1, nv1, seed=9)
    st1 = coarse.build_stencil(lev, q1, blk1)
    v2 = synthetic.gaussian_vectors((nv2, 4, 4, 4, 4, 2, nv1), 77)
    q2, _ = transfer.block_orthonormalize(v2, blk2)
    st2 = coarse.build_stencil(st1, q2, blk2)
    fc = synthetic.gaussian_vectors((2, 2, 2, 2, 2, nv2), 78)
    ref = coarse.apply_galerkin(st1, q2, blk2, fc)
    assert np.linalg.norm(st2.apply(fc) - ref) / np.linalg.norm(ref) < 1e-14
    # and the two-level composition equals P2^dagger P1^dagger D P1 P2
    f1 = transfer.prolong(q2, fc, blk2)
    f0 = transfer.prolong(q1, f1, blk1)
    ref0 = transfer.restrict(q2, transfer.restrict(q1, lev.apply(f0), blk1), blk2)
    assert np.linalg.norm(st2.apply(fc) - ref0) / np.linalg.norm(ref0) < 1e-13
