"""Pins of the oracle Wilson operator against things other than itself.

Sec. 1 of the paper: D = Dslash + m, non-Hermitian, gamma5-Hermitian.
"""
import numpy as np
import pytest

import synthetic
from oracle import wilson

RTOL = 1e-13
# the chiral basis of the reading, written out here rather than taken from the
# oracle (gamma_1..gamma_3 on x, y, z; gamma_4 on t; gamma5 = diag(1, 1, -1, -1))
CHIRAL_GAMMAS = np.array([
    [[0, 0, 0, -1j], [0, 0, -1j, 0], [0, 1j, 0, 0], [1j, 0, 0, 0]],
    [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],
    [[0, 0, -1j, 0], [0, 0, 0, 1j], [1j, 0, 0, 0], [0, -1j, 0, 0]],
    [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],
], dtype=np.complex128)


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def test_gamma_clifford_and_gamma5():
    g = wilson.GAMMA
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)  # Hermitian
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(anti, 2 * (mu == nu) * np.eye(4))
    # gamma5 = gamma1 gamma2 gamma3 gamma4 = diag(1, 1, -1, -1) in the chiral basis
    assert np.allclose(g[0] @ g[1] @ g[2] @ g[3], np.diag([1, 1, -1, -1]))
    assert np.allclose(wilson.GAMMA5, np.diag([1, 1, -1, -1]))


@pytest.mark.parametrize("dims,t_bc,m", [((3, 3, 3, 3), -1.0, -0.3), ((2, 3, 4, 3), 1.0, 0.17)])
def test_apply_matches_bruteforce_dense(dims, t_bc, m):
    u = synthetic.gauge_field(dims, 0.4, seed=11)
    psi = synthetic.gaussian_spinor(dims, seed=12)
    mat = wilson.dense_D(u, m, t_bc)
    ref = (mat @ psi.reshape(-1)).reshape(psi.shape)
    out = wilson.apply_D(u, psi, m, t_bc)
    assert rel(out, ref) < RTOL


def test_gamma5_hermiticity():
    dims = (4, 4, 4, 4)
    u = synthetic.gauge_field(dims, 0.45, seed=3)
    a = synthetic.gaussian_spinor(dims, seed=4)
    b = synthetic.gaussian_spinor(dims, seed=5)
    m = -0.4
    lhs = np.vdot(a, wilson.apply_gamma5(wilson.apply_D(u, b, m)))
    rhs = np.vdot(wilson.apply_gamma5(wilson.apply_D(u, a, m)), b)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    # and D is not Hermitian (Sec. 1)
    assert abs(np.vdot(a, wilson.apply_D(u, b, m)) - np.vdot(wilson.apply_D(u, a, m), b)) > 1e-3


@pytest.mark.parametrize("t_bc", [-1.0, 1.0])
def test_free_field_plane_wave_spectrum(t_bc):
    """Unit links: plane waves are eigenvectors with
    lambda = m + sum_mu (1 - cos p_mu) +- i sqrt(sum_mu sin^2 p_mu), each sign 6-fold."""
    dims = (4, 4, 4, 6)
    lx, ly, lz, lt = dims
    m = 0.13
    u = synthetic.unit_gauge(dims)
    tt, zz, yy, xx = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                                 indexing="ij")
    shift_t = 0.5 if t_bc < 0 else 0.0
    for n in [(0, 0, 0, 0), (1, 0, 0, 0), (1, 2, 3, 1), (3, 1, 0, 5), (2, 2, 2, 2)]:
        p = [2 * np.pi * n[0] / lx, 2 * np.pi * n[1] / ly, 2 * np.pi * n[2] / lz,
             2 * np.pi * (n[3] + shift_t) / lt]
        phase = np.exp(1j * (p[0] * xx + p[1] * yy + p[2] * zz + p[3] * tt))
        # the 12x12 matrix of D on the plane-wave subspace, read off numerically
        mk = np.zeros((12, 12), dtype=complex)
        for j in range(12):
            uvec = np.zeros(12, dtype=complex)
            uvec[j] = 1
            psi = phase[..., None, None] * uvec.reshape(4, 3)
            out = wilson.apply_D(u, psi, m, t_bc)
            coeff = out / phase[..., None, None]
            # no leakage out of the plane wave: the same coefficients everywhere
            assert np.allclose(coeff, coeff[0, 0, 0, 0], atol=1e-13)
            mk[:, j] = coeff[0, 0, 0, 0].reshape(12)
        # the matrix itself: D(p) = (m + sum (1 - cos p)) + i sum gamma_mu sin p_mu, per colour;
        # this fixes D against D^dagger, which has the same spectrum
        dp = (m + sum(1 - np.cos(q) for q in p)) * np.eye(4) + 1j * sum(
            CHIRAL_GAMMAS[mu] * np.sin(p[mu]) for mu in range(4))
        assert np.allclose(mk, np.kron(dp, np.eye(3)), atol=1e-12)
        ev = np.linalg.eigvals(mk)
        ev = ev[np.lexsort((ev.real, np.round(ev.imag, 9)))]
        re = m + sum(1 - np.cos(q) for q in p)
        im = np.sqrt(sum(np.sin(q) ** 2 for q in p))
        expect = np.array([re - 1j * im] * 6 + [re + 1j * im] * 6)
        assert np.allclose(ev, expect, atol=1e-12)


def test_gauge_covariance():
    dims = (4, 4, 4, 4)
    u = synthetic.gauge_field(dims, 0.3, seed=21)
    om = synthetic.site_su3(dims, 2.0, seed=22)
    psi = synthetic.gaussian_spinor(dims, seed=23)
    m = 0.1
    lhs = wilson.apply_D(wilson.gauge_transform(u, om), wilson.colour_rotate(om, psi), m)
    rhs = wilson.colour_rotate(om, wilson.apply_D(u, psi, m))
    assert rel(lhs, rhs) < 1e-14


def test_unit_links_constant_field_gives_mass_term():
    dims = (4, 2, 2, 4)
    u = synthetic.unit_gauge(dims)
    rng = np.random.default_rng(0)
    spin = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi = np.broadcast_to(spin, (4, 2, 2, 4, 4, 3)).copy()
    m = 0.37
    out = wilson.apply_D(u, psi, m, t_bc=1.0)
    assert np.allclose(out, m * psi, atol=1e-14)


def test_hops_sum_to_operator():
    dims = (4, 4, 2, 4)
    u = synthetic.gauge_field(dims, 0.3, seed=31)
    psi = synthetic.gaussian_spinor(dims, seed=32)
    m = -0.2
    tot = (4 + m) * psi
    for mu in range(4):
        for s in (1, -1):
            tot = tot + wilson.hop(u, psi, mu, s, -1.0)
    assert rel(tot, wilson.apply_D(u, psi, m, -1.0)) < 1e-14


def test_batched_apply_matches_single():
    dims = (2, 2, 4, 4)
    u = synthetic.gauge_field(dims, 0.3, seed=41)
    psi = synthetic.gaussian_spinor(dims, seed=42, nrhs=3)
    out = wilson.apply_D(u, psi, 0.1)
    for j in range(3):
        assert rel(out[j], wilson.apply_D(u, psi[j], 0.1)) < 1e-15


def test_per_site_operator_matches_whole_lattice_forms():
    """apply_D_at (term by term at chosen sites) against apply_D and dense_D."""
    dims = (4, 6, 2, 8)
    u = synthetic.gauge_field(dims, 0.4, 5)
    psi = synthetic.gaussian_spinor(dims, 6)
    full = wilson.apply_D(u, psi, -0.3, -1.0)
    sites = [(0, 0, 0, 0), (3, 5, 1, 7), (2, 3, 0, 0), (1, 1, 1, 7), (3, 0, 1, 3)]
    pt = wilson.apply_D_at(u, psi, -0.3, sites, -1.0)
    for n, (x, y, z, t) in enumerate(sites):
        assert np.abs(pt[n] - full[t, z, y, x]).max() < 1e-14
    small = (2, 2, 2, 4)
    u2 = synthetic.gauge_field(small, 0.4, 7)
    p2 = synthetic.gaussian_spinor(small, 8)
    dense = wilson.dense_D(u2, 0.2, 1.0) @ p2.reshape(-1)
    sites2 = [(1, 0, 1, 3), (0, 1, 0, 0)]
    pt2 = wilson.apply_D_at(u2, p2, 0.2, sites2, 1.0)
    for n, (x, y, z, t) in enumerate(sites2):
        i = x + 2 * (y + 2 * (z + 2 * t))
        assert np.abs(pt2[n].reshape(-1) - dense[12 * i:12 * i + 12]).max() < 1e-14


def test_exchanged_projectors_fail_the_plane_wave_pin(monkeypatch):
    # a planted mistake: (1 - gamma) and (1 + gamma) exchanged, i.e. D^dagger
    # computed in place of D; gamma5-Hermiticity and the spectrum cannot tell
    monkeypatch.setattr(wilson, "GAMMA", -wilson.GAMMA)
    with pytest.raises(AssertionError):
        test_free_field_plane_wave_spectrum(-1.0)
