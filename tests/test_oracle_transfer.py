"""Pins of the synthetic links and of the oracle's block QR, P and P^dagger.

Sec. 2: P V_c = V and P^dagger P = I through a QR of the aggregated
candidates; Sec. 3: chirality kept intact so R = P^dagger.
"""
import numpy as np
import pytest

import synthetic
from oracle import transfer


def test_links_are_su3_and_reproducible():
    dims = (4, 4, 2, 4)
    for eps in (0.2, 0.45):
        u = synthetic.gauge_field(dims, eps, seed=5)
        m = u.reshape(-1, 3, 3)
        eye = np.einsum("nba,nbc->nac", np.conj(m), m)
        assert np.abs(eye - np.eye(3)).max() < 1e-14
        assert np.abs(np.linalg.det(m) - 1).max() < 1e-14
        assert np.array_equal(u, synthetic.gauge_field(dims, eps, seed=5))
    assert np.abs(synthetic.gauge_field(dims, 0.0, seed=5) - synthetic.unit_gauge(dims)).max() < 1e-14


def _mgs_block(a):
    """Independent brute force: textbook modified Gram-Schmidt with a loop per column."""
    n, k = a.shape
    q = a.astype(complex).copy()
    r = np.zeros((k, k), dtype=complex)
    for j in range(k):
        for i in range(j):
            r[i, j] = np.vdot(q[:, i], q[:, j])
            q[:, j] -= r[i, j] * q[:, i]
        for i in range(j):  # second pass
            c = np.vdot(q[:, i], q[:, j])
            r[i, j] += c
            q[:, j] -= c * q[:, i]
        r[j, j] = np.linalg.norm(q[:, j])
        q[:, j] /= r[j, j]
    return q, r


def _vectors(dims, nv, seed):
    lx, ly, lz, lt = dims
    return synthetic.gaussian_vectors((nv, lt, lz, ly, lx, 2, 6), seed)


def test_block_qr_orthonormal_and_reproduces_candidates():
    dims, blk, nv = (4, 4, 4, 8), (2, 2, 2, 4), 5
    v = _vectors(dims, nv, 1)
    q, r = transfer.block_orthonormalize(v, blk)
    # P^dagger P = I  (restriction of every prolonged unit coarse vector)
    cd = transfer.coarse_dims(dims, blk)
    cshape = (cd[3], cd[2], cd[1], cd[0], 2, nv)
    ec = synthetic.gaussian_vectors(cshape, 2)
    assert np.abs(transfer.restrict(q, transfer.prolong(q, ec, blk), blk) - ec).max() < 1e-14
    # P V_c = V: every candidate is reproduced by P P^dagger
    for k in range(nv):
        back = transfer.prolong(q, transfer.restrict(q, v[k], blk), blk)
        assert np.linalg.norm(back - v[k]) / np.linalg.norm(v[k]) < 1e-14
    # R is upper triangular with real positive diagonal and P R = V blockwise
    d = np.diagonal(r, axis1=-2, axis2=-1)
    assert np.all(np.abs(d.imag) < 1e-14) and np.all(d.real > 0)
    assert np.abs(np.tril(r, -1)).max() == 0
    rc = np.swapaxes(r, -1, -2)  # [..., chi, k(col of V), j(row)] -> coefficients of V_k
    for k in range(nv):
        coeff = np.zeros(cshape, dtype=complex)
        coeff[..., :, :] = rc[..., k, :]
        assert np.linalg.norm(transfer.prolong(q, coeff, blk) - v[k]) / np.linalg.norm(v[k]) < 1e-13


def test_block_qr_matches_textbook_gram_schmidt():
    dims, blk, nv = (4, 2, 2, 4), (2, 2, 2, 2), 4
    v = _vectors(dims, nv, 7)
    q, _ = transfer.block_orthonormalize(v, blk)
    lx, ly, lz, lt = dims
    # aggregate (xhat,yhat,zhat,that) = (1,0,0,1), chirality -
    xh, yh, zh, th, chi = 1, 0, 0, 1, 1
    rows_v, rows_q = [], []
    for t in range(2):
        for z in range(2):
            for y in range(2):
                for x in range(2):
                    site = (2 * th + t, 2 * zh + z, 2 * yh + y, 2 * xh + x)
                    rows_v.append(v[(slice(None),) + site + (chi,)].T)
                    rows_q.append(q[(slice(None),) + site + (chi,)].T)
    a = np.concatenate(rows_v, axis=0)
    qq = np.concatenate(rows_q, axis=0)
    qref, _ = _mgs_block(a)
    assert np.abs(qq - qref).max() < 1e-13


def test_chirality_preserved_and_adjoint():
    dims, blk, nv = (4, 4, 4, 4), (2, 2, 2, 2), 3
    v = _vectors(dims, nv, 9)
    q, _ = transfer.block_orthonormalize(v, blk)
    cshape = (2, 2, 2, 2, 2, nv)
    ec = synthetic.gaussian_vectors(cshape, 10)
    ec[..., 1, :] = 0  # only chirality +
    f = transfer.as_spinor(transfer.prolong(q, ec, blk))
    assert np.abs(f[..., 2:, :]).max() == 0  # [gamma5, P] = 0: lower spins untouched
    # <P^dagger u, w> = <u, P w>
    uf = synthetic.gaussian_vectors((4, 4, 4, 4, 2, 6), 11)
    w = synthetic.gaussian_vectors(cshape, 12)
    lhs = np.vdot(transfer.restrict(q, uf, blk), w)
    rhs = np.vdot(uf, transfer.prolong(q, w, blk))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_rank_deficient_candidates_are_rejected():
    dims, blk = (2, 2, 2, 2), (2, 2, 2, 2)
    v = _vectors(dims, 3, 13)
    v[2] = 2.0 * v[0] - 1j * v[1]
    with pytest.raises(transfer.RankDeficient):
        transfer.block_orthonormalize(v, blk)


def test_indivisible_block_rejected():
    with pytest.raises(ValueError):
        transfer.coarse_dims((6, 4, 4, 4), (4, 4, 4, 4))
