"""Critical mass ``m_crit = -min Re lambda(D_0)`` (oracle).

Sec. 1: the eigenvalues of ``D`` satisfy ``Re lambda > 0`` and ``D`` becomes
singular as ``Re lambda_min -> 0`` with decreasing mass; Sec. 5 quotes the
critical mass of its ensemble.  ``D_0`` is ``D`` at ``m = 0``, so
``lambda(D_m) = lambda(D_0) + m`` and the critical mass is minus the smallest
real part of the spectrum of ``D_0``.

Reading: the method is not stated; ARPACK (implicitly restarted Arnoldi,
through ``scipy.sparse.linalg.eigs``, ``which='SR'``) is used and a Ritz pair
is accepted only when its residual is below ``accept``.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse.linalg import LinearOperator, eigs

from . import wilson


def mcrit(u, t_bc=-1.0, k=4, ncv=40, tol=1e-8, accept=1e-6, seed=0, apply=None):
    """Returns ``(m_crit, eigenvalues, residuals)`` for the leftmost Ritz values."""
    lt, lz, ly, lx = u.shape[:4]
    shape = (lt, lz, ly, lx, 4, 3)
    n = int(np.prod(shape))
    if apply is None:
        def apply(v):
            return wilson.apply_D(u, v.reshape(shape), 0.0, t_bc).reshape(n)
    op = LinearOperator((n, n), matvec=apply, dtype=np.complex128)
    rng = np.random.default_rng(seed)
    v0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    vals, vecs = eigs(op, k=k, which="SR", ncv=min(ncv, n - 2), tol=tol, v0=v0)
    res = np.array([np.linalg.norm(apply(vecs[:, i]) - vals[i] * vecs[:, i])
                    / np.linalg.norm(vecs[:, i]) for i in range(len(vals))])
    order = np.argsort(vals.real)
    vals, res = vals[order], res[order]
    if res[0] > accept:
        raise RuntimeError(f"leftmost Ritz pair not converged (residual {res[0]:.2e})")
    return -float(vals[0].real), vals, res
