"""Wilson-Dirac operator, FP64 (oracle; test infrastructure only).

Follows Sec. 1 of the paper: ``D = Dslash + m`` built from central covariant
differences plus a second-order Wilson term, non-Hermitian, with
``gamma5``-Hermiticity ``D^dagger = gamma5 D gamma5``.  The paper fixes neither
the normalisation, the gamma basis nor the boundary conditions; the reading
taken (Wilson parameter r = 1, lattice spacing 1, chiral basis, antiperiodic
time) is

    (D psi)(x) = (4 + m) psi(x)
                 - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
                              + (1 + gamma_mu) U_mu(x - mu)^dagger psi(x - mu) ].

With ``m = 1/(2 kappa) - 4`` this is the usual hopping-parameter form, which
puts the paper's quoted critical mass for its 4d ensemble (Sec. 5) near the
familiar quenched critical kappa.

Two independent formulations are given: ``apply_D`` (whole-lattice shifts
with full 4x4 spin matrices) and ``dense_D`` (an explicit matrix assembled
site by site with Kronecker products).  They are compared in the tests.
"""
from __future__ import annotations

import numpy as np

# Chiral basis.  gamma_1..gamma_3 act on mu = 0..2 (x, y, z), gamma_4 on t.
_I = 1j
GAMMA = np.array(
    [
        [[0, 0, 0, -_I], [0, 0, -_I, 0], [0, _I, 0, 0], [_I, 0, 0, 0]],
        [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],
        [[0, 0, -_I, 0], [0, 0, 0, _I], [_I, 0, 0, 0], [0, -_I, 0, 0]],
        [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],
    ],
    dtype=np.complex128,
)
GAMMA5 = np.diag([1.0, 1.0, -1.0, -1.0]).astype(np.complex128)
ID4 = np.eye(4, dtype=np.complex128)

# numpy axis of direction mu in a field whose last axes are [t,z,y,x,4,3]
# (or a link field [t,z,y,x,3,3]).
_AXIS = {0: -3, 1: -4, 2: -5, 3: -6}


def dims_of(u: np.ndarray):
    lt, lz, ly, lx = u.shape[:4]
    return (lx, ly, lz, lt)


def shift_fwd(f: np.ndarray, mu: int, t_bc: float) -> np.ndarray:
    """``g(x) = f(x + mu)``; a hop across the t boundary carries ``t_bc``."""
    ax = _AXIS[mu]
    g = np.roll(f, -1, axis=ax)
    if mu == 3 and t_bc != 1:
        g[..., -1, :, :, :, :, :] *= t_bc
    return g


def shift_bwd(f: np.ndarray, mu: int, t_bc: float) -> np.ndarray:
    """``g(x) = f(x - mu)``; a hop across the t boundary carries ``t_bc``."""
    ax = _AXIS[mu]
    g = np.roll(f, 1, axis=ax)
    if mu == 3 and t_bc != 1:
        g[..., 0, :, :, :, :, :] *= t_bc
    return g


def _colour(u_mu: np.ndarray, f: np.ndarray) -> np.ndarray:
    # (U f)(x)_{s,a} = sum_b U(x)_{a,b} f(x)_{s,b}
    return np.einsum("...ab,...sb->...sa", u_mu, f)


def _spin(g: np.ndarray, f: np.ndarray) -> np.ndarray:
    return np.einsum("st,...tc->...sc", g, f)


def hop(u: np.ndarray, f: np.ndarray, mu: int, sign: int, t_bc: float) -> np.ndarray:
    """One of the eight hopping terms of ``D`` (Sec. 1 operator, reading above).

    ``sign = +1``: ``-1/2 (1 - gamma_mu) U_mu(x) f(x + mu)``;
    ``sign = -1``: ``-1/2 (1 + gamma_mu) U_mu(x - mu)^dagger f(x - mu)``.
    ``D f = (4 + m) f + sum of the eight hops``.
    """
    u_mu = u[..., mu, :, :]
    if sign > 0:
        return -0.5 * _spin(ID4 - GAMMA[mu], _colour(u_mu, shift_fwd(f, mu, t_bc)))
    u_back = np.conj(np.swapaxes(np.roll(u_mu, 1, axis=_AXIS[mu]), -1, -2))
    return -0.5 * _spin(ID4 + GAMMA[mu], _colour(u_back, shift_bwd(f, mu, t_bc)))


def apply_D(u: np.ndarray, psi: np.ndarray, m: float, t_bc: float = -1.0) -> np.ndarray:
    """``D psi`` for a canonical field ``psi[..., t, z, y, x, 4, 3]`` (Sec. 1)."""
    out = (4.0 + m) * psi
    for mu in range(4):
        u_mu = u[..., mu, :, :]
        fwd = _colour(u_mu, shift_fwd(psi, mu, t_bc))
        u_back = np.conj(np.swapaxes(np.roll(u_mu, 1, axis=_AXIS[mu]), -1, -2))
        bwd = _colour(u_back, shift_bwd(psi, mu, t_bc))
        out = out - 0.5 * (_spin(ID4 - GAMMA[mu], fwd) + _spin(ID4 + GAMMA[mu], bwd))
    return out


def apply_gamma5(psi: np.ndarray) -> np.ndarray:
    return _spin(GAMMA5, psi)


def dense_D(u: np.ndarray, m: float, t_bc: float = -1.0) -> np.ndarray:
    """Explicit ``12V x 12V`` matrix of ``D``, assembled site by site (Sec. 1).

    Row and column index ``12 * site + 3 * s + c`` with the canonical site
    index ``x + Lx (y + Ly (z + Lz t))``.  Meant for tiny lattices only.
    """
    lx, ly, lz, lt = dims_of(u)
    vol = lx * ly * lz * lt
    mat = np.zeros((12 * vol, 12 * vol), dtype=np.complex128)
    ext = (lx, ly, lz, lt)

    def index(c):
        return c[0] + lx * (c[1] + ly * (c[2] + lz * c[3]))

    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    here = (x, y, z, t)
                    i = index(here)
                    rows = slice(12 * i, 12 * i + 12)
                    mat[rows, rows] += (4.0 + m) * np.eye(12)
                    for mu in range(4):
                        up = list(here)
                        up[mu] = (up[mu] + 1) % ext[mu]
                        s_up = t_bc if (mu == 3 and here[3] == lt - 1) else 1.0
                        j = index(up)
                        link = u[t, z, y, x, mu]
                        mat[rows, 12 * j:12 * j + 12] += -0.5 * s_up * np.kron(ID4 - GAMMA[mu], link)
                        dn = list(here)
                        dn[mu] = (dn[mu] - 1) % ext[mu]
                        s_dn = t_bc if (mu == 3 and here[3] == 0) else 1.0
                        k = index(dn)
                        link_dn = u[dn[3], dn[2], dn[1], dn[0], mu]
                        mat[rows, 12 * k:12 * k + 12] += -0.5 * s_dn * np.kron(
                            ID4 + GAMMA[mu], np.conj(link_dn.T))
    return mat


def gauge_transform(u: np.ndarray, omega: np.ndarray) -> np.ndarray:
    """``U^Omega_mu(x) = Omega(x) U_mu(x) Omega(x + mu)^dagger`` (no boundary sign)."""
    out = np.empty_like(u)
    for mu in range(4):
        om_up = np.roll(omega, -1, axis=_AXIS[mu])
        out[..., mu, :, :] = np.einsum(
            "...ab,...bc,...dc->...ad", omega, u[..., mu, :, :], np.conj(om_up))
    return out


def colour_rotate(omega: np.ndarray, psi: np.ndarray) -> np.ndarray:
    return np.einsum("...ab,...sb->...sa", omega, psi)


def apply_D_at(u: np.ndarray, psi: np.ndarray, m: float, sites, t_bc: float = -1.0) -> np.ndarray:
    """``(D psi)(x)`` at the listed sites only, each from its nine terms (Sec. 1
    operator, reading above): ``sites`` is a sequence of ``(x, y, z, t)``;
    returns ``[len(sites), 4, 3]``.  For sampled checks on lattices too large
    for the whole-lattice form; written out term by term like ``dense_D``."""
    lx, ly, lz, lt = dims_of(u)
    ext = (lx, ly, lz, lt)
    out = np.zeros((len(sites), 4, 3), dtype=np.complex128)
    for n, here in enumerate(sites):
        x, y, z, t = here
        acc = (4.0 + m) * psi[t, z, y, x]
        for mu in range(4):
            up = list(here)
            up[mu] = (up[mu] + 1) % ext[mu]
            s_up = t_bc if (mu == 3 and t == lt - 1) else 1.0
            f_up = psi[up[3], up[2], up[1], up[0]]
            acc = acc - 0.5 * s_up * (ID4 - GAMMA[mu]) @ (f_up @ u[t, z, y, x, mu].T)
            dn = list(here)
            dn[mu] = (dn[mu] - 1) % ext[mu]
            s_dn = t_bc if (mu == 3 and t == 0) else 1.0
            f_dn = psi[dn[3], dn[2], dn[1], dn[0]]
            link_dn = u[dn[3], dn[2], dn[1], dn[0], mu]
            acc = acc - 0.5 * s_dn * (ID4 + GAMMA[mu]) @ (f_dn @ np.conj(link_dn))
        out[n] = acc
    return out
