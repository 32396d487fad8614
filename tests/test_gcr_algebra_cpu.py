"""The deferred-direction identity used by the batched coarsest GCR and the
outer FGCR: with z_m = z~_m - sum_{i<m} h_{m,i} z_i (the orthogonalised search
directions), the cycle's update sum_m a_m z_m equals sum_m y_m z~_m for
y_m = a_m - sum_{i>m} y_i h_{i,m}, taken from the last direction down.  Checked
in exact-enough FP64 on random data, including frozen iterations (a = 0) and a
zero basis norm, independently of the GPU kernels that use it."""
import numpy as np
import pytest


def _backsolve(a, h):
    J = len(a)
    y = np.zeros(J, dtype=complex)
    for m in range(J - 1, -1, -1):
        y[m] = a[m] - sum(y[i] * h[i, m] for i in range(m + 1, J))
    return y


@pytest.mark.parametrize("J,n,seed", [(1, 5, 0), (4, 30, 1), (16, 200, 2), (32, 500, 3)])
def test_backsolve_reproduces_the_orthogonalised_update(J, n, seed):
    rng = np.random.default_rng(seed)
    zt = rng.standard_normal((J, n)) + 1j * rng.standard_normal((J, n))
    h = np.zeros((J, J), dtype=complex)
    z = np.zeros_like(zt)
    for m in range(J):
        v = zt[m].copy()
        for i in range(m):  # modified Gram-Schmidt against the earlier directions
            h[m, i] = np.vdot(z[i], v) / np.vdot(z[i], z[i])
            v = v - h[m, i] * z[i]
        z[m] = v
    a = rng.standard_normal(J) + 1j * rng.standard_normal(J)
    direct = (a[:, None] * z).sum(axis=0)
    y = _backsolve(a, h)
    deferred = (y[:, None] * zt).sum(axis=0)
    assert np.abs(deferred - direct).max() <= 1e-10 * np.abs(direct).max()


def test_frozen_iterations_contribute_nothing():
    """Once a right-hand side is frozen its step sizes are zero; whatever h the
    later iterations record (finite), y stays zero from the freeze on."""
    rng = np.random.default_rng(7)
    J, j0 = 10, 6
    h = rng.standard_normal((J, J)) + 1j * rng.standard_normal((J, J))
    h[:, 3] = 0.0  # a direction with zero norm gives h = 0, as the coefficient launch sets it
    a = rng.standard_normal(J) + 1j * rng.standard_normal(J)
    a[j0:] = 0.0
    y = _backsolve(a, h)
    assert np.all(y[j0:] == 0.0)
    # and the earlier y equal the back-solve of the truncated cycle
    assert np.allclose(y[:j0], _backsolve(a[:j0], h[:j0, :j0]), rtol=0, atol=1e-12)
