"""Pin of the oracle critical mass against the free-field closed form.

Sec. 1: D becomes singular as the smallest real part of its spectrum goes
to zero.  With unit links the spectrum is known in closed form, so
m_crit = 0 for periodic time and cos(pi / Lt) - 1 for antiperiodic time.
"""
import numpy as np
import pytest

import synthetic
from oracle import mcrit


@pytest.mark.parametrize("t_bc,expect", [(1.0, 0.0), (-1.0, np.cos(np.pi / 4) - 1)])
def test_free_field_mcrit(t_bc, expect):
    u = synthetic.unit_gauge((4, 4, 4, 4))
    mc, vals, res = mcrit.mcrit(u, t_bc=t_bc, k=4, ncv=40)
    assert abs(mc - expect) < 1e-8
    assert res[0] < 1e-6


def test_interacting_mcrit_is_consistent_with_eigen_equation():
    u = synthetic.gauge_field((4, 4, 4, 4), 0.45, seed=3)
    mc, vals, res = mcrit.mcrit(u)
    # roughness pushes the leftmost real part away from the free value toward zero
    assert mc < 0
    assert res[0] < 1e-6
