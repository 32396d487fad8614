"""The 2d U(1) Wilson-Dirac workload and its multigrid solvers (oracle; test infrastructure only).

Sec. 4 compares, for two-dimensional QED on a 128^2 lattice, CG on the
normal equations, CG preconditioned by multigrid on the normal equations
(MG-CG, Nv = 8) and BiCGstab preconditioned by multigrid on D itself
(MG-BiCGstab, Nv = 3): 3-level V(2,2) cycles, 4^2 geometric blocks and a
solve to machine precision on the coarsest 8^2 lattice.  Its metric is the
number of Wilson matrix-vector products (and the flops) to solution.

Operator (the 2d form of the Sec. 1 operator; readings listed below):

    (D psi)(x) = (2 + m) psi(x)
                 - 1/2 sum_{mu=0,1} [ (1 - gamma_mu) U_mu(x) psi(x + mu)
                                    + (1 + gamma_mu) conj(U_mu(x - mu)) psi(x - mu) ]

with U(1) links ``U_mu(x)``, two spin components, ``gamma_0 = sigma_1``,
``gamma_1 = sigma_2`` and ``gamma5 = sigma_3 = diag(1, -1)`` (chirality + is
spin 0).  ``mu`` = 0 is x (periodic) and 1 is t (a hop across the t boundary
carries ``t_bc``, -1 by default).

Fields: a spinor is ``[..., t, x, 2]``; a field of multigrid level ``l`` is
``[..., t, x, 2, n]`` (chirality, then ``n`` = 1 at the fine level and Nv on
coarse levels).  Inside the hierarchy a 2d field is carried as
``[..., 1, 1, t, x, 2, n]`` (two axes of extent one in front) so that the
chirality-split block QR, restriction and prolongation of ``oracle.transfer``
and the cycle of ``oracle.mg`` apply unchanged, with blocks ``(b_x, b_t, 1, 1)``.

* ``apply_D`` (whole-lattice shifts) and ``sparse_D`` (the matrix assembled
  from its entries) are two formulations of D, compared in the tests.
* ``galerkin``: the coarse operator ``P^dagger A P`` (Sec. 2, Sec. 3) as a
  sparse product, for ``A = D`` and for the normal operator ``A = D^dagger D``
  (Sec. 3, first approach), at every coarsening.
* ``Hierarchy2d``: the V(nu_pre, nu_post) cycle of ``oracle.mg`` with every
  coarse operator a sparse matrix and the coarsest level solved by an LU
  factorisation (the machine-precision coarsest solve of Sec. 4).
* ``build``: candidates relaxed on ``A v = 0`` by MR from Gaussian starts
  (Sec. 2), block QR per chirality, Galerkin operators; ``mg_bicgstab``,
  ``mg_cg`` and ``cgnr`` are the three solvers of the comparison.
* ``build(..., blocking=1 or 2)``: the negative control of the Sec. 3
  footnote on two levels: both spins in one block per aggregate, restricted
  with ``P^dagger gamma5`` (left null vectors through gamma5; ill-defined for
  the free-field constant) or with ``P^dagger``.

Readings (the paper is silent): the 2d operator, gamma matrices and boundary
conditions above; the number of relaxation steps of the setup and the
candidates of the second coarsening (relaxed on the level-1 operator from
their own Gaussian starts, Nv as at the first coarsening); the cycle is the
plain V-cycle (one coarse cycle per level) with the minimal-residual step of
Sec. 3 after each prolongation; the coarsest solve is an LU solve.  Wilson
matrix-vector products are counted as fine-level applications of D or
D^dagger (an application of D^dagger D counts two).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import mg, normal, transfer

SIGMA = np.array([[[0, 1], [1, 0]], [[0, -1j], [1j, 0]]], dtype=np.complex128)  # gamma_0, gamma_1
GAMMA5 = np.diag([1.0, -1.0]).astype(np.complex128)
ID2 = np.eye(2, dtype=np.complex128)

# coarse offsets (d_x, d_t): nearest neighbours of D_c, and the 9-point
# stencil of the normal-equation operator (D^dagger D reaches two steps).
OFFSETS_DIRECT = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)]
OFFSETS_NORMAL = OFFSETS_DIRECT + [(1, 1), (-1, 1), (1, -1), (-1, -1)]


# ---------------------------------------------------------------------------
# The operator
def _shift(f, mu, step, t_bc):
    """``g(x) = f(x + step * mu)`` on ``[..., t, x, 2]``; a hop across the t
    boundary carries ``t_bc``."""
    ax = -2 if mu == 0 else -3
    g = np.roll(f, -step, axis=ax)
    if mu == 1 and t_bc != 1:
        if step == 1:
            g[..., -1, :, :] *= t_bc
        else:
            g[..., 0, :, :] *= t_bc
    return g


def apply_D(u, psi, m, t_bc=-1.0):
    """``D psi`` for links ``u[t, x, mu]`` and spinors ``psi[..., t, x, 2]``."""
    out = (2.0 + m) * psi
    for mu in range(2):
        fwd = u[..., mu][..., None] * _shift(psi, mu, 1, t_bc)
        ub = np.conj(np.roll(u[..., mu], 1, axis=1 - mu))  # conj(U_mu(x - mu))
        bwd = ub[..., None] * _shift(psi, mu, -1, t_bc)
        out = out - 0.5 * (np.einsum("st,...t->...s", ID2 - SIGMA[mu], fwd)
                           + np.einsum("st,...t->...s", ID2 + SIGMA[mu], bwd))
    return out


def apply_gamma5(psi):
    return psi * np.array([1.0, -1.0])


def apply_Ddag(u, psi, m, t_bc=-1.0):
    """``D^dagger psi = gamma5 D gamma5 psi`` (gamma5-Hermiticity, Sec. 1)."""
    return apply_gamma5(apply_D(u, apply_gamma5(psi), m, t_bc))


def sparse_D(u, m, t_bc=-1.0):
    """D as a sparse matrix, row/column index ``(t * Lx + x) * 2 + s``, assembled
    entry by entry from the definition above."""
    lt, lx = u.shape[:2]
    n = lt * lx * 2
    rows, cols, vals = [], [], []
    for t in range(lt):
        for x in range(lx):
            s = (t * lx + x) * 2
            for a in range(2):
                rows.append(s + a)
                cols.append(s + a)
                vals.append(2.0 + m)
            for mu in range(2):
                # forward: -1/2 (1 - gamma_mu) U_mu(x) psi(x + mu)
                xf, tf = (x + 1) % lx if mu == 0 else x, (t + 1) % lt if mu == 1 else t
                bc = t_bc if (mu == 1 and t == lt - 1) else 1.0
                blk = -0.5 * (ID2 - SIGMA[mu]) * u[t, x, mu] * bc
                sf = (tf * lx + xf) * 2
                # backward: -1/2 (1 + gamma_mu) conj(U_mu(x - mu)) psi(x - mu)
                xb, tb = (x - 1) % lx if mu == 0 else x, (t - 1) % lt if mu == 1 else t
                bcb = t_bc if (mu == 1 and t == 0) else 1.0
                blkb = -0.5 * (ID2 + SIGMA[mu]) * np.conj(u[tb, xb, mu]) * bcb
                sb = (tb * lx + xb) * 2
                for a in range(2):
                    for b in range(2):
                        rows += [s + a, s + a]
                        cols += [sf + b, sb + b]
                        vals += [blk[a, b], blkb[a, b]]
    return sp.csr_matrix((np.array(vals), (rows, cols)), shape=(n, n))


def sparse_gamma5(vol):
    return sp.diags(np.tile([1.0, -1.0], vol).astype(np.complex128))


# ---------------------------------------------------------------------------
# Transfer and Galerkin operators
def as_level(f):
    """``[..., t, x, 2, n]`` -> ``[..., 1, 1, t, x, 2, n]`` (the 4d field form)."""
    return f.reshape(f.shape[:-4] + (1, 1) + f.shape[-4:])


def block4(block2):
    bx, bt = block2
    return (bx, bt, 1, 1)


def prolongator_matrix(q, block2):
    """P as a sparse matrix from the block-orthonormal columns ``q`` of
    ``transfer.block_orthonormalize`` (``[Nv, 1, 1, t, x, g, n]`` with g = 2
    chirality groups, or g = 1 when the spin is blocked): row index
    ``((t * Lx + x) * g + chi) * n + i``, column index
    ``((tc * Lxc + xc) * g + chi) * Nv + k``."""
    nv = q.shape[0]
    lt, lx, g, n = q.shape[-4:]
    bx, bt = block2
    lxc = lx // bx
    t, x, chi, i, k = np.meshgrid(np.arange(lt), np.arange(lx), np.arange(g), np.arange(n), np.arange(nv),
                                  indexing="ij")
    rows = ((t * lx + x) * g + chi) * n + i
    cols = (((t // bt) * lxc + x // bx) * g + chi) * nv + k
    vals = q.reshape(nv, lt, lx, g, n)[k, t, x, chi, i]
    ncoarse = (lt // bt) * lxc * g * nv
    return sp.csr_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=(lt * lx * g * n, ncoarse))


def galerkin(A, P):
    """``P^dagger A P`` (Sec. 2 and 3), sparse."""
    return (P.conj().T @ A @ P).tocsr()


class SparseLevel:
    """A level operator held as a sparse matrix over fields ``[..., 1, 1, t, x, g, n]``."""

    def __init__(self, M, site_shape, n, groups=2):
        self.M = M.tocsr()
        self.site_shape = tuple(site_shape)  # (1, 1, t, x)
        self.dof = (groups, n)

    def apply(self, f):
        lead = f.shape[:-6]
        flat = f.reshape((-1, self.M.shape[0]))
        out = (self.M @ flat.T).T
        return out.reshape(lead + self.site_shape + self.dof)


def stencil_blocks(M, dims2, n, offsets, groups=2):
    """The blocks ``B[o][t, x, g n, g n]`` (g = ``groups``) of a coarse operator
    with ``(M c)(xhat) = sum_o B[o](xhat) c(xhat + d_o)`` (periodic coarse
    indexing), read off the sparse matrix; every entry of M must lie on one
    of the offsets (checked)."""
    lx, lt = dims2
    nn = groups * n
    B = np.zeros((len(offsets), lt, lx, nn, nn), dtype=np.complex128)
    C = M.tocoo()
    rs, cs = C.row // nn, C.col // nn
    rt, rx, ct, cxx = rs // lx, rs % lx, cs // lx, cs % lx
    dx = (cxx - rx + 1) % lx - 1
    dt = (ct - rt + 1) % lt - 1
    seen = np.zeros(len(C.data), dtype=bool)
    for o, (ox, ot) in enumerate(offsets):
        sel = (dx == ox) & (dt == ot)
        B[o, rt[sel], rx[sel], C.row[sel] % nn, C.col[sel] % nn] += C.data[sel]
        seen |= sel
    stray = np.abs(C.data[~seen])
    if stray.size and stray.max() > 0.0:
        raise ValueError("coarse operator has entries off the stencil")
    return B


# ---------------------------------------------------------------------------
# Levels and hierarchy
class Wilson2d:
    """The fine operator D on level fields ``[..., 1, 1, t, x, 2, 1]`` (the two
    spins as two chirality groups), or ``[..., 1, 1, t, x, 1, 2]`` when the
    spin is blocked (one group of both spins)."""

    def __init__(self, u, m, t_bc=-1.0, dof=(2, 1)):
        self.u, self.m, self.t_bc = u, float(m), float(t_bc)
        lt, lx = u.shape[:2]
        self.site_shape = (1, 1, lt, lx)
        self.dof = tuple(dof)

    def _spinor(self, f):
        return f.reshape(f.shape[:-6] + self.site_shape[2:] + (2,))

    def apply_D(self, f):
        return apply_D(self.u, self._spinor(f), self.m, self.t_bc).reshape(f.shape)

    def apply_Ddag(self, f):
        return apply_Ddag(self.u, self._spinor(f), self.m, self.t_bc).reshape(f.shape)

    def apply(self, f):
        return self.apply_D(f)


class Normal2d(Wilson2d):
    """``A = D^dagger D`` (Sec. 3, normal equations) on fine level fields."""

    def apply(self, f):
        return self.apply_Ddag(self.apply_D(f))


class Hierarchy2d(mg.Hierarchy):
    """``oracle.mg.Hierarchy`` with the coarsest level solved by LU (Sec. 4:
    machine precision on the coarsest lattice) and plain V-cycles.  With
    ``gamma5_restriction`` the fine-level restriction is ``P^dagger gamma5``
    (Sec. 3: left null vectors from right ones through gamma5), as the
    footnote's spin-blocked variant uses it."""

    def __init__(self, ops, qs, blocks, gamma5_restriction=False, **kw):
        kw.setdefault("coarse_cycles", [1] * (len(ops) - 1))
        super().__init__(ops, qs, blocks, **kw)
        self.gamma5_restriction = gamma5_restriction
        self.lu = sla.lu_factor(ops[-1].M.toarray())

    def correction(self, l, r):
        if l == 0 and self.gamma5_restriction:
            r = apply_gamma5(r.reshape(r.shape[:-2] + (2,))).reshape(r.shape)
        return super().correction(l, r)

    def coarsest_solve(self, rc):
        self.counts[-1] += 1
        return sla.lu_solve(self.lu, rc.reshape(-1)).reshape(rc.shape)


def build(u, m, t_bc, *, nvs, block=(4, 4), setup_iters=100, seeds=None, null_vectors=None, normal=False,
          blocking=0, **kw):
    """Hierarchy for D (``normal=False``, MG-BiCGstab) or for ``D^dagger D``
    (``normal=True``, MG-CG): per coarsening, ``nvs[l]`` candidates relaxed
    with ``setup_iters`` MR steps on ``A_l v = 0`` from Gaussian starts
    (``seeds[l]``) or given (``null_vectors[l]``, level-field shaped
    ``[Nv, t, x, 2, n]``), block QR on ``block`` aggregates, Galerkin operator.

    ``blocking`` (two levels of D only): 0 keeps chirality intact (Sec. 3);
    1 blocks both spins into one block per aggregate and restricts with
    ``P^dagger gamma5`` (the variant of the Sec. 3 footnote, coarse operator
    ``P^dagger gamma5 D P``); 2 blocks the spins and restricts with ``P^dagger``."""
    from synthetic import gaussian_vectors

    if blocking and (normal or len(nvs) != 1):
        raise ValueError("spin blocking is built for two-level hierarchies of D")
    fine = Normal2d(u, m, t_bc) if normal else Wilson2d(u, m, t_bc, dof=(1, 2) if blocking else (2, 1))
    lt, lx = u.shape[:2]
    A = sparse_D(u, m, t_bc)
    if normal:
        A = (sparse_gamma5(lt * lx) @ A @ sparse_gamma5(lt * lx) @ A).tocsr()
    ops, qs, blocks, mats = [fine], [], [], []
    dims2, n = (lx, lt), 1
    groups = 1 if blocking else 2
    for l, nv in enumerate(nvs):
        op = ops[-1]
        shape = (nv, dims2[1], dims2[0], 2, n)
        lshape = (nv, 1, 1, dims2[1], dims2[0]) + op.dof
        if null_vectors is not None and null_vectors[l] is not None:
            vecs = null_vectors[l].reshape(lshape)
        else:
            v0 = gaussian_vectors(shape, seeds[l]).reshape(lshape)
            vecs = mg.relax_null_vectors(op.apply, v0, setup_iters, kw.get("omega", 0.8))
        q, _ = transfer.block_orthonormalize(vecs, block4(block))
        P = prolongator_matrix(q, block)
        if blocking == 1:
            A = (P.conj().T @ sparse_gamma5(lt * lx) @ A @ P).tocsr()
        else:
            A = galerkin(A, P)
        dims2 = (dims2[0] // block[0], dims2[1] // block[1])
        n = nv
        qs.append(q)
        blocks.append(block4(block))
        mats.append(A)
        ops.append(SparseLevel(A, (1, 1, dims2[1], dims2[0]), n, groups))
    h = Hierarchy2d(ops, qs, blocks, gamma5_restriction=blocking == 1, **kw)
    h.mats = mats
    return h


def wilson_products(h: mg.Hierarchy) -> int:
    """Fine-level Wilson matrix-vector products counted by ``h`` (D^dagger D
    counts two)."""
    return h.counts[0] * (2 if isinstance(h.ops[0], Normal2d) else 1)


def mg_bicgstab(h, b, tol, maxit=10000):
    """MG-BiCGstab (Sec. 4): BiCGstab on ``D x = b`` with the V-cycle of the
    direct hierarchy as right preconditioner.  ``b``: ``[t, x, 2]``."""
    bl = b.reshape((1, 1) + b.shape[-3:-1] + h.ops[0].dof)
    x, info = mg.bicgstab(lambda f: h._apply(0, f), bl, tol, maxit=maxit, precond=lambda r: h.vcycle(0, r))
    return x.reshape(b.shape), info


def mg_cg(h, b, tol, maxit=10000):
    """MG-CG (Sec. 4): flexible CG on ``D^dagger D x = D^dagger b`` with the
    V-cycle of the normal hierarchy, stopped on ``||b - D x|| / ||b||``."""
    bl = as_level(b.reshape(b.shape[-3:] + (1,)))
    x, info = normal.mg_cg(_Counted(h), bl, tol, maxit=maxit)
    return x.reshape(b.shape), info


def cgnr(u, m, t_bc, b, tol, maxit=100000):
    """CG on the normal equations (the CG of Sec. 4), stopped on the true
    residual of ``D x = b``; ``info['wilson']`` counts D and D^dagger products."""
    op = _CountedNormal(u, m, t_bc)
    bl = as_level(b.reshape(b.shape[-3:] + (1,)))
    x, info = normal.cgnr(op, bl, tol, maxit=maxit)
    info["wilson"] = op.products
    return x.reshape(b.shape), info


class _Counted:
    """Routes ``normal.mg_cg``'s applications of ``D^dagger D`` through the
    hierarchy's counter."""

    def __init__(self, h):
        self.h = h
        self.ops = [self]

    def apply(self, f):
        return self.h._apply(0, f)

    def apply_D(self, f):
        return self.h.ops[0].apply_D(f)

    def apply_Ddag(self, f):
        return self.h.ops[0].apply_Ddag(f)

    def vcycle(self, l, r):
        return self.h.vcycle(l, r)


class _CountedNormal(Normal2d):
    def __init__(self, u, m, t_bc):
        super().__init__(u, m, t_bc)
        self.products = 0

    def apply_D(self, f):
        self.products += 1
        return super().apply_D(f)

    def apply_Ddag(self, f):
        self.products += 1
        return super().apply_Ddag(f)


def mcrit(u, t_bc=-1.0, k=4, ncv=40, tol=1e-10, seed=0):
    """``m_crit = -min Re lambda(D at m = 0)`` (Sec. 1) by ARPACK on the sparse D."""
    from scipy.sparse.linalg import eigs

    A = sparse_D(u, 0.0, t_bc)
    rng = np.random.default_rng(seed)
    v0 = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    vals, vecs = eigs(A, k=k, which="SR", ncv=ncv, tol=tol, v0=v0)
    res = np.linalg.norm(A @ vecs - vecs * vals, axis=0)
    i = int(np.argmin(vals.real))
    return -float(vals[i].real), vals, res
