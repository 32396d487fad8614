"""Chirality-split aggregation, block QR, restriction and prolongation (oracle).

Sec. 2 (last paragraph) defines the prolongator by ``P V_c = V`` and
``P^dagger P = I`` through a QR decomposition of the candidate vectors cut
into aggregates; Sec. 3 fixes the aggregates as regular geometric blocks and
keeps chirality intact (``[gamma5, P] = 0``), so ``R = P^dagger``.

Fields at any level are ``[..., T, Z, Y, X, 2, n]`` (chirality first, see the
package header).  A fine spinor ``[..., 4, 3]`` is passed as its reshape
``[..., 2, 6]``.  Blocks are ``(bx, by, bz, bt)``.

Readings: the QR algorithm and phase are not stated; a thin QR with real
positive ``diag(R)`` is taken, which makes ``Q`` unique for full-rank input.
Rows of an aggregate are ordered site-lexicographically inside the block
(x fastest), then by the dof inside the chirality.  A column whose ``R_jj``
falls below ``1e-12`` of its norm is reported as rank deficient.
"""
from __future__ import annotations

import numpy as np


class RankDeficient(ValueError):
    pass


def coarse_dims(dims, block):
    out = []
    for d, b in zip(dims, block):
        if d % b:
            raise ValueError(f"extent {d} not divisible by block {b}")
        out.append(d // b)
    return tuple(out)


def _split(f: np.ndarray, block) -> np.ndarray:
    """``[..., T,Z,Y,X,2,n] -> [..., Tc,bt,Zc,bz,Yc,by,Xc,bx,2,n]``."""
    bx, by, bz, bt = block
    lead = f.shape[:-6]
    lt, lz, ly, lx, two, n = f.shape[-6:]
    return f.reshape(lead + (lt // bt, bt, lz // bz, bz, ly // by, by, lx // bx, bx, two, n))


def block_orthonormalize(vecs: np.ndarray, block):
    """Block QR of the candidate vectors (Sec. 2, ``P V_c = V``, ``P^dagger P = I``).

    ``vecs``: ``[Nv, T, Z, Y, X, 2, n]``.  Returns ``(Q, R)``: ``Q`` has the shape
    of ``vecs`` and holds the orthonormal columns of ``P`` (column
    ``(xhat, chi, k)`` is ``Q[k]`` restricted to aggregate ``xhat`` and
    chirality ``chi``); ``R`` is ``[Tc, Zc, Yc, Xc, 2, Nv, Nv]``, the coarse
    representation ``V_c``, upper triangular with real positive diagonal.
    """
    nv = vecs.shape[0]
    vb = _split(vecs, block)  # [Nv, Tc,bt,Zc,bz,Yc,by,Xc,bx,2,n]
    tc, bt, zc, bz, yc, by, xc, bx, two, n = vb.shape[1:]
    # -> [Tc,Zc,Yc,Xc, chi, (bt,bz,by,bx,n), Nv]
    a = vb.transpose(1, 3, 5, 7, 9, 2, 4, 6, 8, 10, 0)
    a = a.reshape(tc, zc, yc, xc, two, bt * bz * by * bx * n, nv)
    q, r = np.linalg.qr(a, mode="reduced")
    d = np.diagonal(r, axis1=-2, axis2=-1)
    colnorm = np.linalg.norm(a, axis=-2)
    if np.any(np.abs(d) <= 1e-12 * np.maximum(colnorm, 1e-300)):
        raise RankDeficient("candidate vectors are rank deficient on some aggregate")
    ph = d / np.abs(d)
    q = q * ph[..., None, :]
    r = np.conj(ph)[..., :, None] * r
    # back to [Nv, T, Z, Y, X, 2, n]
    q = q.reshape(tc, zc, yc, xc, two, bt, bz, by, bx, n, nv)
    q = q.transpose(10, 0, 5, 1, 6, 2, 7, 3, 8, 4, 9)
    q = q.reshape(vecs.shape)
    return np.ascontiguousarray(q), r


def restrict(q: np.ndarray, f: np.ndarray, block) -> np.ndarray:
    """``P^dagger f`` (Sec. 2, ``R = P^dagger``; Sec. 3, chirality kept intact).

    ``r_c(xhat, chi, k) = sum_{x in B(xhat)} sum_{dof in chi} conj(Q_k(x)) f(x)``.
    ``f``: ``[..., T, Z, Y, X, 2, n]``; result ``[..., Tc, Zc, Yc, Xc, 2, Nv]``.
    """
    qb = _split(q, block)
    fb = _split(f, block)
    return np.einsum("kTtZzYyXxhn,...TtZzYyXxhn->...TZYXhk", np.conj(qb), fb, optimize=True)


def prolong(q: np.ndarray, fc: np.ndarray, block) -> np.ndarray:
    """``P f_c`` (Sec. 2): ``f(x)_{chi, i} = sum_k Q_k(x)_{chi, i} f_c(xhat(x), chi, k)``."""
    qb = _split(q, block)
    out = np.einsum("kTtZzYyXxhn,...TZYXhk->...TtZzYyXxhn", qb, fc, optimize=True)
    lead = fc.shape[:-6]
    return out.reshape(lead + q.shape[1:])


def as_chiral(psi: np.ndarray) -> np.ndarray:
    """Fine spinor ``[..., 4, 3]`` viewed as ``[..., 2, 6]`` (chirality split)."""
    return psi.reshape(psi.shape[:-2] + (2, 6))


def as_spinor(f: np.ndarray) -> np.ndarray:
    return f.reshape(f.shape[:-2] + (4, 3))
