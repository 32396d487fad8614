"""Multigrid on the normal equations (oracle; test infrastructure only).

Sec. 3 weighs two approaches: adaptive multigrid applied to the normal
equations ``D^dagger D x = D^dagger b``, whose operator is Hermitian positive
definite so the Galerkin coarse operator ``(D^dagger D)_c = P^dagger D^dagger D P``
is the optimal one, at the price of a squared condition number and of a
coarse operator that is no longer a product of nearest-neighbour couplings;
and multigrid on ``D`` itself.  Sec. 4 runs the normal-equation hierarchy as
the preconditioner of CG (MG-CG) beside plain CG.

* ``NormalLevel``: ``A = D^dagger D`` on chirality-split fields, with
  ``D^dagger = gamma5 D gamma5`` (gamma5-Hermiticity, Sec. 1).
* ``build_normal_stencil``: ``A_c = P^dagger A P``.  ``D`` couples sites at
  most one step apart, so ``D^dagger D`` couples sites up to two steps apart
  (``0``, ``+-mu``, ``+-2 mu``, ``+-mu +-nu``); on aggregates of extent >= 2
  these land on coarse offsets with every component in {-1, 0, 1} and at
  most two of them non-zero: 1 + 8 + 24 = 33 blocks per coarse site.  The
  blocks are read off the literal map ``P^dagger (A (P c))`` by probing:
  coarse sites are coloured by ``xhat_mu mod K_mu`` (``K_mu >= 3`` dividing the
  coarse extent), so a probe vector that is one dof on every site of one
  colour reaches each coarse site from at most one of them.
* ``fcg``: flexible CG (Notay 2000): the new direction is the preconditioned
  residual A-orthogonalised against the previous direction only, which is
  CG when the preconditioner is a fixed HPD map and stays convergent for a
  varying one such as a V-cycle with MR smoothing.
* ``cgnr``: CG on ``D^dagger D x = D^dagger b`` (the CG comparator of Sec. 4 and 5).
* ``mg_cg``: ``fcg`` on the normal equations with the V-cycle of the normal
  hierarchy (the ``Hierarchy`` of ``mg`` on ``A`` and ``A_c``) as preconditioner.

Readings (the paper is silent): the candidate vectors of the normal hierarchy
are relaxed on ``A v = 0`` with the MR steps of the direct setup and blocked
by chirality like the direct ones; the coarse extents must be >= 3 (with
extent 2 the +mu and -mu neighbours coincide and the offsets cannot be
told apart); every solve stops on the true residual ``||b - D x|| / ||b||`` of
the original system.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import mg, transfer, wilson

# coarse offsets (d_x, d_y, d_z, d_t) of the normal-equation stencil
OFFSETS = [d for d in itertools.product((-1, 0, 1), repeat=4) if sum(1 for v in d if v) <= 2]
OFFSETS.sort(key=lambda d: (sum(1 for v in d if v), d))
assert len(OFFSETS) == 33
_AXIS = {0: -3, 1: -4, 2: -5, 3: -6}  # numpy axis of direction mu for [..., T, Z, Y, X, 2, n]


class NormalLevel:
    """``A = D^dagger D`` for the Wilson operator of Sec. 1, chirality-split fields."""

    def __init__(self, u, m, t_bc=-1.0):
        self.u = u
        self.m = float(m)
        self.t_bc = float(t_bc)
        lt, lz, ly, lx = u.shape[:4]
        self.site_shape = (lt, lz, ly, lx)
        self.dof = (2, 6)

    def apply_D(self, f):
        return transfer.as_chiral(wilson.apply_D(self.u, transfer.as_spinor(f), self.m, self.t_bc))

    def apply_Ddag(self, f):
        g5 = lambda v: transfer.as_chiral(wilson.apply_gamma5(transfer.as_spinor(v)))  # noqa: E731
        return g5(self.apply_D(g5(f)))

    def apply(self, f):
        return self.apply_Ddag(self.apply_D(f))


class NormalStencil:
    """``A_c`` as 33 blocks per coarse site: ``B[o][T,Z,Y,X,N,N]`` for the
    offsets ``OFFSETS[o]``; ``(A_c c)(xhat) = sum_o B[o](xhat) c(xhat + d_o)``."""

    def __init__(self, blocks, nv):
        self.b = blocks
        self.nv = nv
        self.site_shape = blocks.shape[1:5]
        self.dof = (2, nv)

    def apply(self, f):
        lead = f.shape[:-2]
        n2 = 2 * self.nv
        out = np.zeros(lead + (n2,), dtype=np.complex128)
        for o, d in enumerate(OFFSETS):
            g = f
            for mu in range(4):
                if d[mu]:
                    g = np.roll(g, -d[mu], axis=_AXIS[mu])
            out += np.einsum("...ij,...j->...i", self.b[o], g.reshape(lead + (n2,)))
        return out.reshape(lead + (2, self.nv))


def colouring(cdims):
    """``K_mu``: the smallest divisor >= 3 of each coarse extent (the extent
    itself when it has none below it); extents below 3 are refused."""
    ks = []
    for e in cdims:
        if e < 3:
            raise ValueError(f"coarse extent {e} < 3: the +mu and -mu neighbours coincide")
        ks.append(next(k for k in range(3, e + 1) if e % k == 0))
    return ks


def build_normal_stencil(level, q, block) -> NormalStencil:
    """``A_c = P^dagger A P`` (Sec. 3 normal-equation Galerkin operator) read off
    ``P^dagger (A (P c))`` with coloured probe vectors."""
    nv = q.shape[0]
    n2 = 2 * nv
    lt, lz, ly, lx = level.site_shape
    cdims = transfer.coarse_dims((lx, ly, lz, lt), block)  # (X, Y, Z, T)
    if min(block) < 2:
        raise ValueError("aggregates of extent >= 2 keep the two-step couplings within one coarse step")
    ks = colouring(cdims)
    cshape = (cdims[3], cdims[2], cdims[1], cdims[0])
    blocks = np.zeros((len(OFFSETS),) + cshape + (n2, n2), dtype=np.complex128)
    index = {d: o for o, d in enumerate(OFFSETS)}
    coords = np.stack(np.meshgrid(*[np.arange(c) for c in cdims], indexing="ij"), axis=-1)  # [X,Y,Z,T,4]
    coords = coords.transpose(3, 2, 1, 0, 4)  # [T,Z,Y,X,4] with entries (x, y, z, t)
    # offset code of a site: d_mu + 1 in base 3, -1 where out of reach
    lookup = -np.ones(81, dtype=np.int64)
    for d, o in index.items():
        lookup[sum((v + 1) * 3 ** mu for mu, v in enumerate(d))] = o
    for kappa in itertools.product(*[range(k) for k in ks]):
        on = np.all(coords % np.array(ks) == np.array(kappa), axis=-1)
        # for every coarse site, the offset d (components in -1..1) to the
        # probed site of colour kappa within reach, if any
        code = np.zeros(cshape, dtype=np.int64)
        reach = np.ones(cshape, dtype=bool)
        for mu in range(4):
            dmu = np.full(cshape, 9, dtype=np.int64)
            for v in (1, 0, -1):
                dmu = np.where((coords[..., mu] + v) % ks[mu] == kappa[mu], v, dmu)
            reach &= dmu != 9
            code += np.where(dmu != 9, dmu + 1, 0) * 3 ** mu
        off = np.where(reach, lookup[code], -1)
        sites = np.nonzero(off >= 0)
        for a in range(n2):
            c = np.zeros(cshape + (n2,), dtype=np.complex128)
            c[on, a] = 1.0
            y = transfer.restrict(q, level.apply(transfer.prolong(q, c.reshape(cshape + (2, nv)), block)), block)
            y = y.reshape(cshape + (n2,))
            blocks[(off[sites],) + sites + (slice(None), a)] = y[sites]
    return NormalStencil(blocks, nv)


def fcg(apply, b, tol, maxit=10000, precond=None, true_res=None, x0=None):
    """Flexible CG on the HPD system ``A x = b`` (Notay 2000, one earlier
    direction kept).  ``true_res(x)`` (optional) decides convergence, else
    ``||b - A x|| / ||b||``.  Returns ``(x, info)``."""
    m = precond if precond is not None else (lambda f: f.copy())
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply(x) if x0 is not None else b.copy()
    bn = mg.norm(b)
    check = true_res or (lambda xx: mg.norm(b - apply(xx)) / bn)
    info = {"iters": 0, "converged": False, "true_res": 1.0}
    if bn == 0.0:
        info.update(converged=True, true_res=0.0)
        return x, info
    p = q = None
    while info["iters"] < maxit:
        z = m(r)
        if p is None:
            p = z
        else:
            beta = -mg.dot(q, z) / mg.dot(p, q)
            p = z + beta * p
        q = apply(p)
        pq = mg.dot(p, q)
        alpha = mg.dot(p, r) / pq
        x = x + alpha * p
        r = r - alpha * q
        info["iters"] += 1
        if mg.norm(r) <= tol * bn:
            info["true_res"] = check(x)
            if info["true_res"] <= tol:
                info["converged"] = True
                return x, info
    info["true_res"] = check(x)
    info["converged"] = info["true_res"] <= tol
    return x, info


def cgnr(op: NormalLevel, b, tol, maxit=100000):
    """CG on ``D^dagger D x = D^dagger b``, stopped on ``||b - D x|| / ||b|| <= tol``.

    The normal residual is driven to ``tol * ||D^dagger b||`` scaled down by
    a safety factor of 1e-2 (``||b - D x||`` can exceed the normal residual by
    the condition number), and the true residual is checked at the end."""
    bn = mg.norm(b)
    rhs = op.apply_Ddag(b)
    tres = lambda x: mg.norm(b - op.apply_D(x)) / bn  # noqa: E731
    x, info = fcg(op.apply, rhs, 1e-2 * tol * bn / max(mg.norm(rhs), 1e-300), maxit=maxit, true_res=tres)
    info["true_res"] = tres(x)
    info["converged"] = info["true_res"] <= tol
    return x, info


def build_normal_hierarchy(u, m, t_bc, block, nv, *, seed=None, setup_iters=50, null_vectors=None, **kw):
    """Two-level normal-equation hierarchy: candidates relaxed on ``A v = 0``
    (or given), chirality-split block QR, ``A_c`` by ``build_normal_stencil``."""
    from synthetic import gaussian_vectors

    op = NormalLevel(u, m, t_bc)
    if null_vectors is None:
        v0 = gaussian_vectors((nv,) + op.site_shape + op.dof, seed)
        vecs = mg.relax_null_vectors(op.apply, v0, setup_iters, kw.get("omega", 0.8))
    else:
        vecs = null_vectors
    q, _ = transfer.block_orthonormalize(vecs, block)
    return mg.Hierarchy([op, build_normal_stencil(op, q, block)], [q], [block], **kw)


def mg_cg(h: mg.Hierarchy, b, tol, maxit=2000):
    """MG-CG (Sec. 4): flexible CG on ``D^dagger D x = D^dagger b`` with the
    normal hierarchy's V-cycle as preconditioner, stopped on the true
    residual of ``D x = b``."""
    op = h.ops[0]
    bn = mg.norm(b)
    rhs = op.apply_Ddag(b)
    tres = lambda x: mg.norm(b - op.apply_D(x)) / bn  # noqa: E731
    x, info = fcg(op.apply, rhs, 1e-2 * tol * bn / max(mg.norm(rhs), 1e-300), maxit=maxit,
                  precond=lambda r: h.vcycle(0, r), true_res=tres)
    info["true_res"] = tres(x)
    info["converged"] = info["true_res"] <= tol
    return x, info
