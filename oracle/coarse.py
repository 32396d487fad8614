"""Galerkin coarse operator ``D_c = P^dagger D P`` as a nearest-neighbour stencil (oracle).

Sec. 2 defines the coarse-grid operator as ``A_c = P^dagger A P``; Sec. 3
notes that working directly with ``D`` (rather than the normal equations)
keeps the coarse operator a product of nearest-neighbour couplings, and that
with a chirality-preserving ``P`` the restriction is ``P^dagger``.

Every level operator here is written as ``diag + sum of eight hops``:
``(A f)(x) = diag(f)(x) + sum_{mu, +-} hop_{mu,+-}(f)(x)``, where
``hop_{mu,+}`` brings ``f`` from ``x + mu`` and ``hop_{mu,-}`` from ``x - mu``.
The coarse stencil then follows from the definition of ``P^dagger A P`` split
by where each fine coupling lands: a hop that leaves the aggregate through
its ``+-mu`` face couples ``xhat`` to ``xhat +- mu`` and goes into ``Y_{mu,+-}``;
every other coupling stays in ``X``.  So

    Y_{mu,+-}(xhat) = P_B^dagger [mask_face(+-mu) hop_{mu,+-}] P,
    X(xhat)        = P_B^dagger [diag + sum mask_inner hop] P,

and ``D_c c (xhat) = X c(xhat) + sum_mu Y_{mu,+} c(xhat+mu) + Y_{mu,-} c(xhat-mu)``
with periodic coarse indices (any time-boundary sign sits inside the face
blocks).  ``apply_galerkin`` evaluates ``P^dagger (A (P c))`` literally and is
the definition the stencil is tested against.

Reading: when a coarse extent is 1 or 2 the ``+mu`` and ``-mu`` neighbours
coincide; the stencil keeps the blocks separate (defined by the face the hop
crosses), which still sums to ``P^dagger A P``.
"""
from __future__ import annotations

import numpy as np

from . import transfer, wilson

# numpy axis of direction mu for fields [..., T, Z, Y, X, 2, n]
_AXIS = {0: -3, 1: -4, 2: -5, 3: -6}


class WilsonLevel:
    """The fine operator ``D`` of Sec. 1 on chirality-split fields ``[..., 2, 6]``."""

    def __init__(self, u, m, t_bc=-1.0):
        self.u = u
        self.m = float(m)
        self.t_bc = float(t_bc)
        lt, lz, ly, lx = u.shape[:4]
        self.site_shape = (lt, lz, ly, lx)
        self.dof = (2, 6)

    def apply(self, f):
        return transfer.as_chiral(
            wilson.apply_D(self.u, transfer.as_spinor(f), self.m, self.t_bc))

    def diag(self, f):
        return (4.0 + self.m) * f

    def hop(self, f, mu, sign):
        return transfer.as_chiral(
            wilson.hop(self.u, transfer.as_spinor(f), mu, sign, self.t_bc))


class StencilLevel:
    """A coarse operator stored as ``X[T,Z,Y,X,N,N]`` and ``Y[mu][+-][T,Z,Y,X,N,N]``."""

    def __init__(self, x_blk, y_blk, nv):
        self.x = x_blk
        self.y = y_blk  # shape [4, 2, T, Z, Y, X, N, N]; index 0 = +mu, 1 = -mu
        self.nv = nv
        self.site_shape = x_blk.shape[:4]
        self.dof = (2, nv)

    def _mv(self, blk, f):
        lead = f.shape[:-2]
        ff = f.reshape(lead + (2 * self.nv,))
        out = np.einsum("...ij,...j->...i", blk, ff)
        return out.reshape(lead + (2, self.nv))

    def diag(self, f):
        return self._mv(self.x, f)

    def hop(self, f, mu, sign):
        if sign > 0:
            return self._mv(self.y[mu, 0], np.roll(f, -1, axis=_AXIS[mu]))
        return self._mv(self.y[mu, 1], np.roll(f, 1, axis=_AXIS[mu]))

    def apply(self, f):
        out = self.diag(f)
        for mu in range(4):
            out = out + self.hop(f, mu, +1) + self.hop(f, mu, -1)
        return out

    def shifted(self, dm):
        """The same stencil with ``dm`` added to the diagonal (``P^dagger P = I``)."""
        x = self.x + dm * np.eye(2 * self.nv)
        return StencilLevel(x, self.y, self.nv)


def face_mask(site_shape, block, mu, sign):
    """1 on sites whose ``mu``-neighbour in direction ``sign`` lies in another aggregate."""
    lt, lz, ly, lx = site_shape
    ext = {0: lx, 1: ly, 2: lz, 3: lt}[mu]
    b = block[mu]
    coord = np.arange(ext) % b
    on_face = (coord == b - 1) if sign > 0 else (coord == 0)
    shape = [1, 1, 1, 1]
    shape[{0: 3, 1: 2, 2: 1, 3: 0}[mu]] = ext
    return on_face.reshape(shape).astype(np.float64)


def build_stencil(level, q, block) -> StencilLevel:
    """``D_c = P^dagger A P`` as a 9-point stencil (Sec. 2 Galerkin operator).

    ``level``: a WilsonLevel or StencilLevel; ``q``: ``[Nv, T,Z,Y,X, 2, n]``
    orthonormal block columns from ``transfer.block_orthonormalize``.
    """
    nv = q.shape[0]
    cdims = transfer.coarse_dims(
        (level.site_shape[3], level.site_shape[2], level.site_shape[1], level.site_shape[0]), block)
    cshape = (cdims[3], cdims[2], cdims[1], cdims[0])
    n2 = 2 * nv
    x_blk = np.zeros(cshape + (n2, n2), dtype=np.complex128)
    y_blk = np.zeros((4, 2) + cshape + (n2, n2), dtype=np.complex128)
    masks = {(mu, s): face_mask(level.site_shape, block, mu, s)[..., None, None]
             for mu in range(4) for s in (+1, -1)}
    for chi in range(2):
        for k in range(nv):
            col = chi * nv + k
            f = np.zeros_like(q[k])
            f[..., chi, :] = q[k][..., chi, :]
            x_blk[..., :, col] += transfer.restrict(q, level.diag(f), block).reshape(cshape + (n2,))
            for mu in range(4):
                for si, s in enumerate((+1, -1)):
                    h = level.hop(f, mu, s)
                    face = masks[(mu, s)]
                    y_blk[mu, si, ..., :, col] = transfer.restrict(
                        q, face * h, block).reshape(cshape + (n2,))
                    x_blk[..., :, col] += transfer.restrict(
                        q, (1.0 - face) * h, block).reshape(cshape + (n2,))
    return StencilLevel(x_blk, y_blk, nv)


def apply_galerkin(level, q, block, fc):
    """``P^dagger (A (P fc))`` evaluated literally (the definition of ``D_c``)."""
    return transfer.restrict(q, level.apply(transfer.prolong(q, fc, block)), block)


def dense_from_apply(apply, shape):
    """Dense matrix of a linear map on arrays of ``shape`` (tiny cases only)."""
    n = int(np.prod(shape))
    mat = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        mat[:, j] = apply(e.reshape(shape)).reshape(n)
    return mat
