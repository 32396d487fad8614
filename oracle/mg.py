"""Smoother, Krylov solvers, coarse-grid correction, V-cycle and adaptive setup (oracle).

Paper passages followed:

* MR smoother, under-relaxed with ``omega = 0.8``: Sec. 3 (last paragraph).
* coarse-grid correction ``x_c = alpha P (P^dagger D P)^{-1} P^dagger r`` with
  the minimal-residual step ``alpha = <D x_c, r> / <D x_c, D x_c>``: Sec. 3
  (the correction with chirality-preserving P, and the step-size equation).
* V(m, n) cycle recursing to an exact coarsest solve: Sec. 2; the modified
  3-level cycle with 4 next-coarser V-cycles between fine restriction and
  prolongation: Sec. 5.
* adaptive setup: relax ``A x = 0`` from random ``x_0`` for ``l`` iterations,
  then block QR: Sec. 2 (the alpha-SA procedure); the augmentation in which
  the current multigrid, applied to ``A x = 0``, refines each next candidate:
  Sec. 2 (the paragraph after the three steps).
* flexible GCR(k) outer solver: Sec. 5; BiCGstab as the unpreconditioned
  comparator: Sec. 5, and with the V-cycle as right preconditioner (the
  MG-BiCGstab of the 2d study): Sec. 4.

Readings (the paper is silent):

* omega scales the MR step; the residual is updated recursively.
* alpha is applied at every level; a zero ``<p, p>`` (exact residual) gives a
  zero step instead of 0/0.
* "4 applications of the next coarsest level V-cycle" is the stationary
  iteration ``e <- e + M_1 (r_c - D_1 e)`` from ``e = 0``.
* the coarsest solve is GCR (restart 32) to a relative tolerance.
* the outer FGCR orthogonalises with modified Gram-Schmidt, starts from
  ``x = 0`` and declares convergence only on the true residual.
* the augmentation relaxes every starting vector first and then refines
  candidates 2..Nv with a fixed number of stationary two-level iterations
  ``x <- x - M A x`` (the paper gives no count and no stopping test).
"""
from __future__ import annotations

import numpy as np

from . import coarse, transfer


def dot(a, b):
    return complex(np.vdot(a.reshape(-1), b.reshape(-1)))


def norm(a):
    return float(np.linalg.norm(a.reshape(-1)))


def mr(apply, x, r, iters, omega=0.8):
    """``iters`` under-relaxed MR steps on ``A x = b`` with residual ``r = b - A x``.

    Step: ``p = A r``; ``alpha = omega <p, r> / <p, p>``; ``x += alpha r``;
    ``r -= alpha p``.  Returns ``(x, r)`` (new arrays).
    """
    x = x.copy()
    r = r.copy()
    for _ in range(iters):
        p = apply(r)
        pp = dot(p, p).real
        if pp == 0.0:
            break
        a = omega * dot(p, r) / pp
        x += a * r
        r -= a * p
    return x, r


def gcr(apply, b, tol, restart=32, maxit=1000, precond=None, x0=None, true_apply=None):
    """(Flexible) GCR with MGS orthogonalisation and true-residual restarts.

    Returns ``(x, info)``; ``info`` holds ``iters``, ``restarts``,
    ``true_res`` (relative, recomputed with ``true_apply`` or ``apply``) and
    ``converged``.
    """
    true_apply = true_apply or apply
    bn = norm(b)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    info = {"iters": 0, "restarts": 0, "converged": False, "true_res": 1.0}
    if bn == 0.0:
        x[...] = 0
        info.update(converged=True, true_res=0.0)
        return x, info
    r = b - true_apply(x) if x0 is not None else b.copy()
    while True:
        zs, ws = [], []
        for _ in range(restart):
            z = precond(r) if precond is not None else r.copy()
            w = apply(z)
            for zi, wi in zip(zs, ws):
                beta = dot(wi, w)
                w = w - beta * wi
                z = z - beta * zi
            nw = norm(w)
            if nw == 0.0:
                break
            w = w / nw
            z = z / nw
            zs.append(z)
            ws.append(w)
            a = dot(w, r)
            x = x + a * z
            r = r - a * w
            info["iters"] += 1
            if norm(r) <= tol * bn or info["iters"] >= maxit:
                break
        r = b - true_apply(x)
        rel = norm(r) / bn
        info["true_res"] = rel
        if rel <= tol:
            info["converged"] = True
            return x, info
        if info["iters"] >= maxit:
            return x, info
        info["restarts"] += 1


def bicgstab(apply, b, tol, maxit=100000, precond=None):
    """BiCGstab (van der Vorst 1992), ``x_0 = 0``; with ``precond`` (a map M)
    preconditioned on the right: the directions p and s enter A and the
    solution update as ``M p`` and ``M s`` (the MG-preconditioned BiCGstab of
    Sec. 4).  Without it, unpreconditioned (the Sec. 5 comparator).

    A breakdown (``rho = 0``) restarts from the true residual.  Returns
    ``(x, info)`` with ``iters`` (each costs two applications of ``A``).
    """
    m = precond if precond is not None else (lambda f: f)
    bn = norm(b)
    x = np.zeros_like(b)
    info = {"iters": 0, "converged": False, "true_res": 1.0, "restarts": 0}
    if bn == 0.0:
        info.update(converged=True, true_res=0.0)
        return x, info
    r = b.copy()
    while info["iters"] < maxit:
        rhat = r.copy()
        rho = alpha = omega = 1.0 + 0j
        v = np.zeros_like(b)
        p = np.zeros_like(b)
        while info["iters"] < maxit:
            rho_new = dot(rhat, r)
            if rho_new == 0:
                break
            beta = (rho_new / rho) * (alpha / omega)
            p = r + beta * (p - omega * v)
            ph = m(p)
            v = apply(ph)
            alpha = rho_new / dot(rhat, v)
            s = r - alpha * v
            sh = m(s)
            t = apply(sh)
            tt = dot(t, t).real
            omega = dot(t, s) / tt if tt != 0 else 0.0
            x = x + alpha * ph + omega * sh
            r = s - omega * t
            rho = rho_new
            info["iters"] += 1
            if norm(r) <= tol * bn or omega == 0:
                break
        rt = b - apply(x)
        info["true_res"] = norm(rt) / bn
        if info["true_res"] <= tol:
            info["converged"] = True
            return x, info
        r = rt
        info["restarts"] += 1
    return x, info


class Hierarchy:
    """Multigrid levels: ``ops[l]`` is the operator at level ``l``; ``qs[l]``,
    ``blocks[l]`` define the prolongator from level ``l+1`` to ``l``."""

    def __init__(self, ops, qs, blocks, *, omega=0.8, nu_pre=2, nu_post=2,
                 coarse_cycles=None, coarse_tol=1e-2, coarse_restart=32,
                 coarse_maxit=1000, use_alpha=True):
        self.ops = ops
        self.qs = qs
        self.blocks = blocks
        self.omega = omega
        self.nu_pre = nu_pre
        self.nu_post = nu_post
        nl = len(ops)
        # Sec. 5: between fine restriction and prolongation, 4 cycles of the
        # next level when that level is not the coarsest.
        self.coarse_cycles = coarse_cycles or [4 if l + 2 < nl else 1 for l in range(nl - 1)]
        self.coarse_tol = coarse_tol
        self.coarse_restart = coarse_restart
        self.coarse_maxit = coarse_maxit
        self.use_alpha = use_alpha
        self.counts = [0] * nl  # operator applications per level

    def _apply(self, l, f):
        self.counts[l] += 1
        return self.ops[l].apply(f)

    def coarsest_solve(self, rc):
        l = len(self.ops) - 1
        x, _ = gcr(lambda f: self._apply(l, f), rc, self.coarse_tol,
                   restart=self.coarse_restart, maxit=self.coarse_maxit)
        return x

    def correction(self, l, r):
        """Coarse-grid correction at level ``l`` (Sec. 3): returns ``y = P e_c``."""
        q, blk = self.qs[l], self.blocks[l]
        rc = transfer.restrict(q, r, blk)
        if l + 1 == len(self.ops) - 1:
            ec = self.coarsest_solve(rc)
        else:
            ec = np.zeros_like(rc)
            for it in range(self.coarse_cycles[l]):
                res = rc if it == 0 else rc - self._apply(l + 1, ec)
                ec = ec + self.vcycle(l + 1, res)
        return transfer.prolong(q, ec, blk)

    def vcycle(self, l, r):
        """``x = M_l r``: V(nu_pre, nu_post) from ``x = 0`` (Sec. 2, Sec. 3, Sec. 5)."""
        apply = lambda f: self._apply(l, f)  # noqa: E731
        x = np.zeros_like(r)
        x, res = mr(apply, x, r, self.nu_pre, self.omega)
        y = self.correction(l, res)
        dy = apply(y)
        if self.use_alpha:
            dd = dot(dy, dy).real
            a = dot(dy, res) / dd if dd != 0.0 else 0.0
        else:
            a = 1.0
        x = x + a * y
        res = res - a * dy
        x, res = mr(apply, x, res, self.nu_post, self.omega)
        return x

    def solve(self, b, tol=1e-10, restart=50, maxit=1000):
        """MG-preconditioned flexible GCR on the finest level (Sec. 5)."""
        return gcr(lambda f: self._apply(0, f), b, tol, restart=restart, maxit=maxit,
                   precond=lambda r: self.vcycle(0, r))


def relax_null_vectors(apply, v0, iters, omega=0.8):
    """Sec. 2 setup step: relax ``A v = 0`` from random ``v0`` for ``iters`` MR steps.

    Each vector has its own step size.  Returns the relaxed vectors, each
    normalised to unit norm.  ``v0``: ``[Nv, ...]``.
    """
    out = np.empty_like(v0)
    for k in range(v0.shape[0]):
        x = v0[k].copy()
        r = -apply(x)
        x, _ = mr(apply, x, r, iters, omega)
        out[k] = x / norm(x)
    return out


def adaptive_null_vectors(op, v0, blk, iters, adapt_iters, omega=0.8, **hier_kw):
    """Sec. 2 adaptive augmentation (alpha-SA): the current multigrid solver is
    applied to ``A x = 0`` to produce each next candidate.

    Every starting vector is first relaxed (``iters`` MR steps, as in
    ``relax_null_vectors``).  Then, for k = 2, ..., Nv, the two-level
    multigrid built from candidates 1..k-1 (block QR, Galerkin operator) is
    applied ``adapt_iters`` times to candidate k as the stationary iteration
    ``x <- x - M A x``.  Candidates are returned with unit norm; the block QR of
    all of them defines P (``P V_c = V``, ``P^dagger P = I``).  ``hier_kw`` go to
    the ``Hierarchy`` of each step (smoothing, alpha, coarsest tolerance).
    """
    vecs = relax_null_vectors(op.apply, v0, iters, omega)
    for k in range(1, vecs.shape[0]):
        if adapt_iters == 0:
            break
        q, _ = transfer.block_orthonormalize(vecs[:k], blk)
        h = Hierarchy([op, coarse.build_stencil(op, q, blk)], [q], [blk], omega=omega, **hier_kw)
        x = vecs[k]
        for _ in range(adapt_iters):
            x = x - h.vcycle(0, op.apply(x))
        vecs[k] = x / norm(x)
    return vecs


def build_hierarchy(u, m, t_bc, blocks, nvs, *, seeds=None, setup_iters=100,
                    null_vectors=None, **kw) -> Hierarchy:
    """Adaptive setup (Sec. 2) followed by block QR and Galerkin operators.

    ``blocks[l]``, ``nvs[l]`` for each coarsening ``l``.  Either
    ``null_vectors[l]`` (``[Nv, T,Z,Y,X, 2, n]``, used as the relaxed vectors)
    or a ``seeds[l]`` for complex Gaussian starting vectors.
    """
    from synthetic import gaussian_vectors

    ops = [coarse.WilsonLevel(u, m, t_bc)]
    qs = []
    for l, (blk, nv) in enumerate(zip(blocks, nvs)):
        op = ops[-1]
        shape = (nv,) + tuple(op.site_shape) + tuple(op.dof)
        if null_vectors is not None and null_vectors[l] is not None:
            vecs = null_vectors[l]
        else:
            v0 = gaussian_vectors(shape, seeds[l])
            vecs = relax_null_vectors(op.apply, v0, setup_iters, kw.get("omega", 0.8))
        q, _ = transfer.block_orthonormalize(vecs, blk)
        qs.append(q)
        ops.append(coarse.build_stencil(op, q, blk))
    return Hierarchy(ops, qs, list(blocks), **kw)
