"""Chirality-preserving against spin-blocking prolongators (oracle; test infrastructure only).

Sec. 3 derives the coarse-grid correction from left null vectors obtained
through gamma5 (the left eigenvectors of D are gamma5 times right ones):
``x_c = P (P^dagger gamma5 D P)^-1 P^dagger gamma5 r``.  Its footnote
observes that a prolongator that blocks the spin dimension can make this
correction ill-defined: for the free field the null vector is the constant,
and then ``P^dagger gamma5 P = 0``.  Keeping chirality intact,
``[gamma5, P] = 0``, avoids it, and the gamma5 factors then cancel, leaving
the Galerkin correction with ``R = P^dagger``.

This module is the negative control of that statement, on lattices small
enough for dense matrices (plain definitions, no blocking of the
arithmetic):

* ``prolongator``: the dense P of a set of candidate vectors, block QR per
  aggregate either per chirality (two columns sets, spins 0-1 and 2-3: the
  prolongator of this method) or over all four spins together (spin
  blocking);
* ``TwoLevel``: the two-level cycle MR(nu) - coarse correction - MR(nu) on
  the dense D (``dense_wilson``) with restriction ``R = P^dagger`` or
  ``R = P^dagger gamma5`` and the coarse operator ``R D P`` solved densely;
  a numerically vanishing coarse operator is reported as
  :class:`IllDefined`;
* ``solve``: flexible GCR preconditioned by that cycle (``mg.gcr``).
"""
from __future__ import annotations

import numpy as np

from . import coarse, mg, wilson


class IllDefined(ArithmeticError):
    """The coarse operator R D P vanishes (relative to ||D||): no correction exists."""


def prolongator(vecs, block, chiral=True):
    """Dense P (``[n_fine, n_coarse]``) of candidates ``vecs`` ``[k, T, Z, Y, X, 4, 3]``
    on aggregates ``block`` = (bx, by, bz, bt): per aggregate, the candidates
    restricted to it (and, with ``chiral``, to one chirality) are
    orthonormalised by QR; coarse dof per aggregate: 2k (chiral) or k."""
    k = vecs.shape[0]
    lt, lz, ly, lx = vecs.shape[1:5]
    bx, by, bz, bt = block
    n = lt * lz * ly * lx * 12
    spin = np.arange(4)[:, None] * np.ones((1, 3), dtype=int)
    groups = [spin < 2, spin >= 2] if chiral else [np.ones((4, 3), dtype=bool)]
    cols = []
    for tc in range(lt // bt):
        for zc in range(lz // bz):
            for yc in range(ly // by):
                for xc in range(lx // bx):
                    site = np.zeros((lt, lz, ly, lx, 1, 1), dtype=bool)
                    site[tc * bt:(tc + 1) * bt, zc * bz:(zc + 1) * bz, yc * by:(yc + 1) * by,
                         xc * bx:(xc + 1) * bx] = True
                    for g in groups:
                        rows = np.nonzero((site & g).reshape(n))[0]
                        a = vecs.reshape(k, n)[:, rows].T
                        q, r = np.linalg.qr(a)
                        if np.min(np.abs(np.diagonal(r))) <= 1e-12 * np.linalg.norm(a):
                            raise ValueError("candidates are rank deficient on an aggregate")
                        col = np.zeros((n, k), dtype=np.complex128)
                        col[rows] = q
                        cols.append(col)
    return np.concatenate(cols, axis=1)


def dense_wilson(u, m, t_bc):
    """Dense Wilson operator (Sec. 1) of the oracle on a tiny lattice."""
    shape = tuple(u.shape[:4]) + (4, 3)
    return coarse.dense_from_apply(lambda f: wilson.apply_D(u, f, m, t_bc), shape)


def gamma5_matrix(site_shape):
    """Dense gamma5 (chiral basis: +1 on spins 0, 1 and -1 on spins 2, 3)."""
    g = np.ones(site_shape + (4, 3))
    g[..., 2:, :] = -1.0
    return np.diag(g.reshape(-1)).astype(np.complex128)


class TwoLevel:
    """Two-level cycle with the coarse correction ``P (R D P)^-1 R r`` (Sec. 3),
    R = P^dagger or P^dagger gamma5, MR(nu_pre) before and MR(nu_post) after
    (omega = 0.8); every operator dense."""

    def __init__(self, D, site_shape, P, gamma5_restriction, nu_pre=2, nu_post=2, omega=0.8):
        self.shape = tuple(site_shape) + (4, 3)
        self.D = D
        self.P = P
        self.R = P.conj().T @ gamma5_matrix(self.shape[:4]) if gamma5_restriction else P.conj().T
        self.Dc = self.R @ self.D @ P
        self.nu_pre, self.nu_post, self.omega = nu_pre, nu_post, omega

    def coarse_singular_values(self):
        return np.linalg.svd(self.Dc, compute_uv=False)

    def apply(self, f):
        return self.D @ f

    def cycle(self, r):
        """x = M r from x = 0."""
        if np.linalg.norm(self.Dc) <= 1e-12 * np.linalg.norm(self.D):
            raise IllDefined("R D P vanishes")
        x, rr = mg.mr(self.apply, np.zeros_like(r), r, self.nu_pre, self.omega)
        x = x + self.P @ np.linalg.solve(self.Dc, self.R @ rr)
        dx, _ = mg.mr(self.apply, np.zeros_like(r), r - self.D @ x, self.nu_post, self.omega)
        return x + dx

    def solve(self, b, tol=1e-10, restart=50, maxit=400):
        """Flexible GCR on D x = b preconditioned by the cycle."""
        return mg.gcr(self.apply, b.reshape(-1), tol, restart=restart, maxit=maxit, precond=self.cycle)
