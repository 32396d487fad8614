"""Parity at the benchmark lattice sizes on sampled outputs.

The whole-lattice oracle is too slow for 32^4 and 24^3 x 48 inside a test, so
the oracle evaluates the Wilson operator term by term at sampled sites
(oracle.wilson.apply_D_at): corners, both time boundaries, tile and
aggregate faces, and random sites.  The GPU output at those sites must meet
the same bars as the small-lattice tests (FP64 1e-13 relative, FP32 1e-6,
16-bit within the storage bound).
"""
import numpy as np
import pytest
import torch

import synthetic
from oracle import precision, wilson
from paper_0811_4331_amd import wdmg

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def sample_sites(dims, n_random, seed):
    lx, ly, lz, lt = dims
    fixed = [(0, 0, 0, 0), (lx - 1, ly - 1, lz - 1, lt - 1), (0, 0, 0, lt - 1), (lx - 1, 0, 0, 0),
             (3, 4, 7, 8), (4, 3, 8, 7), (lx // 2, ly // 2, lz // 2, lt // 2)]
    rng = np.random.default_rng(seed)
    rnd = [tuple(int(rng.integers(0, e)) for e in dims) for _ in range(n_random)]
    return fixed + rnd


@pytest.mark.parametrize("dims,eps,seed", [((32, 32, 32, 32), 0.45, 3020), ((24, 24, 24, 48), 0.45, 4020)])
def test_wilson_operator_at_full_size(dims, eps, seed):
    m = -1.585
    u = synthetic.gauge_field(dims, eps, seed)
    ctx = wdmg.Context(dims, DEV)
    ctx.set_gauge(torch.from_numpy(u).to(DEV), t_bc=-1)
    ctx.set_mass(m)
    psi = synthetic.gaussian_spinor(dims, seed=seed + 1)
    sites = sample_sites(dims, 40, seed)
    idx = tuple(np.array(c) for c in zip(*[(t, z, y, x) for (x, y, z, t) in sites]))
    ref = wilson.apply_D_at(u, psi, m, sites, -1.0)
    out = ctx.apply_D(torch.from_numpy(psi).to(DEV)).cpu().numpy()[idx]
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-13
    out32 = ctx.apply_D(torch.from_numpy(psi.astype(np.complex64)).to(DEV), prec="f32").cpu().numpy()[idx]
    assert np.linalg.norm(out32 - ref) / np.linalg.norm(ref) < 1e-6
    for kind in ("f16", "bf16"):
        got = ctx.apply_D(torch.from_numpy(psi.astype(np.complex64)).to(DEV), prec=kind).cpu().numpy()[idx]
        xin = precision.store_fine(psi, kind).astype(np.complex128)
        uq = precision.store_su3_links(u, kind)
        refq = wilson.apply_D_at(uq, xin, m, sites, -1.0)
        d = got.astype(np.complex128) - refq
        err = np.maximum(np.abs(d.real), np.abs(d.imag)).max(axis=(-2, -1))
        smax = np.maximum(np.abs(refq.real), np.abs(refq.imag)).max(axis=(-2, -1))
        bound = precision.HALF_ULP[kind] * smax * 1.001 + 8e-5 * np.abs(xin).max()
        assert np.all(err <= bound), (kind, float((err / bound).max()))
    ctx.close()
