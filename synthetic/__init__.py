"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module draws random numbers and nothing else: it holds none of the
multigrid method's arithmetic.  Both sides (the oracle under ``oracle/`` and
the GPU library through its Python binding) receive these arrays as inputs.

Canonical layouts (host, numpy):

* gauge field  ``U[t, z, y, x, mu, a, b]`` complex128, ``mu`` = 0..3 = x,y,z,t;
  ``U_mu(x)[a, b]`` carries colour ``b`` at ``x + mu`` to colour ``a`` at ``x``.
* spinor field ``psi[t, z, y, x, s, c]`` complex128, spin ``s`` 0..3, colour
  ``c`` 0..2.  A batch of fields adds a leading axis.

The paper measures on Monte-Carlo gauge ensembles (Sec. 4 and 5) that are not
available; links ``U = exp(i eps H)`` with random traceless Hermitian ``H``
stand in for them, ``eps`` setting the roughness.  The 2d U(1) fields of
Sec. 4 are drawn from the compact U(1) plaquette weight itself
(``u1_gauge_field``): building links from independently drawn plaquette
angles is input generation, not part of the solver.
"""
from __future__ import annotations

import numpy as np


def _dims_shape(dims):
    lx, ly, lz, lt = (int(d) for d in dims)
    return (lt, lz, ly, lx)


def random_su3(n: int, eps: float, rng: np.random.Generator) -> np.ndarray:
    """``n`` matrices ``exp(i eps H)``.

    Recipe for ``H`` (one per matrix, drawn in this order as whole arrays):
    three real diagonal entries N(0,1); then the real parts of the upper
    off-diagonal entries (0,1), (0,2), (1,2), each N(0,1); then their imaginary
    parts, each N(0,1).  ``H`` is completed to a Hermitian matrix and made
    traceless by subtracting ``tr(H)/3``.  The exponential is taken through the
    eigen-decomposition ``H = W diag(w) W^dagger``.
    """
    diag = rng.standard_normal((n, 3))
    off_re = rng.standard_normal((n, 3))
    off_im = rng.standard_normal((n, 3))
    h = np.zeros((n, 3, 3), dtype=np.complex128)
    h[:, 0, 0], h[:, 1, 1], h[:, 2, 2] = diag[:, 0], diag[:, 1], diag[:, 2]
    off = off_re + 1j * off_im
    for k, (a, b) in enumerate(((0, 1), (0, 2), (1, 2))):
        h[:, a, b] = off[:, k]
        h[:, b, a] = np.conj(off[:, k])
    tr = (diag[:, 0] + diag[:, 1] + diag[:, 2]) / 3.0
    for a in range(3):
        h[:, a, a] -= tr
    w, vecs = np.linalg.eigh(h)
    phase = np.exp(1j * eps * w)
    return np.einsum("nab,nb,ncb->nac", vecs, phase, np.conj(vecs))


def gauge_field(dims, eps: float, seed: int) -> np.ndarray:
    """Canonical links ``U[t,z,y,x,mu,3,3]`` with ``U = exp(i eps H)`` per link.

    Links are drawn in canonical order (site-lexicographic, then ``mu``).
    ``eps = 0`` gives the free field (unit links).
    """
    shp = _dims_shape(dims)
    nsite = int(np.prod(shp))
    rng = np.random.default_rng(seed)
    u = random_su3(nsite * 4, eps, rng)
    return u.reshape(shp + (4, 3, 3))


def unit_gauge(dims) -> np.ndarray:
    shp = _dims_shape(dims)
    u = np.zeros(shp + (4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def site_su3(dims, eps: float, seed: int) -> np.ndarray:
    """One random SU(3) matrix per site, ``[t,z,y,x,3,3]`` (gauge transforms)."""
    shp = _dims_shape(dims)
    rng = np.random.default_rng(seed)
    return random_su3(int(np.prod(shp)), eps, rng).reshape(shp + (3, 3))


def gaussian_spinor(dims, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Complex Gaussian fermion field(s): real and imaginary parts i.i.d. N(0,1).

    Shape ``[t,z,y,x,4,3]`` or ``[nrhs,t,z,y,x,4,3]``.  All real parts are drawn
    first as one array, then all imaginary parts.
    """
    shp = _dims_shape(dims) + (4, 3)
    if nrhs is not None:
        shp = (int(nrhs),) + shp
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shp)
    im = rng.standard_normal(shp)
    return re + 1j * im


def gaussian_vectors(shape, seed: int) -> np.ndarray:
    """Complex Gaussian array of any shape (coarse vectors, null-vector seeds)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return re + 1j * im


# Seed conventions for the benchmark workloads: gauge 1000*cfg + 10*i_eps +
# replica, right-hand sides 2000*cfg + j, null-vector starts 3000*cfg + k.
def gauge_seed(cfg: int, i_eps: int = 0, replica: int = 0) -> int:
    return 1000 * cfg + 10 * i_eps + replica


def rhs_seed(cfg: int, j: int = 0) -> int:
    return 2000 * cfg + j


def null_seed(cfg: int, k: int = 0) -> int:
    return 3000 * cfg + k


def u1_gauge_field(dims2, beta: float, seed: int) -> np.ndarray:
    """2d compact U(1) links ``U[t, x, mu] = exp(i theta_mu(x))``, ``mu`` = 0 (x),
    1 (t), distributed with the plaquette weight ``exp(beta cos theta_P)``.

    In two dimensions the plaquette angles of that weight are independent,
    up to one global constraint on the torus, so a field is built from them:
    in an axial gauge (t links zero except on the last time slice) the
    x links of slice t + 1 follow from those of slice t and the plaquettes
    between them, and the t links of the last slice follow from the
    plaquettes of that slice; the one plaquette left closes the torus.  A
    random gauge transformation ``theta_mu(x) += g(x) - g(x + mu)`` is
    applied last.  Plaquette: ``theta_P(x) = theta_0(x) + theta_1(x + 0hat)
    - theta_0(x + 1hat) - theta_1(x)``.

    Draws, in this order: the x-link angles of slice 0 (``Lx`` values,
    uniform on [-pi, pi)); the free plaquette angles (slices 0 .. Lt-2 with x
    fastest, then x = 0 .. Lx-2 of slice Lt-1; von Mises with mean 0 and
    concentration ``beta``); the t-link angle at (x = 0, t = Lt-1) (uniform);
    one gauge angle per site (uniform, [t, x] order).  ``dims2 = (Lx, Lt)``.
    """
    lx, lt = (int(d) for d in dims2)
    rng = np.random.default_rng(seed)
    th0 = np.zeros((lt, lx))
    th1 = np.zeros((lt, lx))
    th0[0] = rng.uniform(-np.pi, np.pi, lx)
    plaq = rng.vonmises(0.0, beta, (lt - 1) * lx + lx - 1)
    rows, last = plaq[:(lt - 1) * lx].reshape(lt - 1, lx), plaq[(lt - 1) * lx:]
    for t in range(lt - 1):
        th0[t + 1] = th0[t] - rows[t]
    a = th0[lt - 1] - th0[0]
    th1[lt - 1, 0] = rng.uniform(-np.pi, np.pi)
    for x in range(lx - 1):
        th1[lt - 1, x + 1] = th1[lt - 1, x] + last[x] - a[x]
    g = rng.uniform(-np.pi, np.pi, (lt, lx))
    th0 = th0 + g - np.roll(g, -1, axis=1)
    th1 = th1 + g - np.roll(g, -1, axis=0)
    return np.exp(1j * np.stack([th0, th1], axis=-1))


def gaussian_spinor_2d(dims2, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Complex Gaussian 2d fermion field(s) ``[t, x, 2]`` (or ``[nrhs, t, x, 2]``):
    all real parts first, then all imaginary parts, each N(0,1)."""
    lx, lt = (int(d) for d in dims2)
    shp = (lt, lx, 2) if nrhs is None else (int(nrhs), lt, lx, 2)
    return gaussian_vectors(shp, seed)
