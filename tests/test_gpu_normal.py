"""GPU parity of the normal-equation path (Sec. 3 first approach, Sec. 4 MG-CG
and CG) against the oracle (oracle/normal.py): the 33-block coarse operator
(D^dagger D)_c element by element (FP64, 1e-12), the candidates relaxed on
D^dagger D, the operator after a mass change, CGNR and MG-CG to the true
residual 1e-10 measured with the oracle's D, and the error paths."""
import json
import os

import numpy as np
import pytest
import torch

import synthetic
from oracle import coarse, mg, normal, transfer, wilson
from paper_0811_4331_amd import wdmg

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
with open(os.path.join(os.path.dirname(__file__), "golden", "mcrit.json")) as _fh:
    MCRIT = json.load(_fh)


def rel(a, b):
    """Largest element error over the largest element (or the 2-norm ratio if larger)."""
    d, r = (a - b).ravel(), b.ravel()
    return float(max(np.abs(d).max() / np.abs(r).max(), np.linalg.norm(d) / np.linalg.norm(r)))


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def setup(dims, blk, nv, m, seed, setup_iters=0, eps=0.3):
    u = synthetic.gauge_field(dims, eps, seed)
    ctx = wdmg.Context(dims, DEV)
    ctx.set_gauge(gpu(u), t_bc=-1)
    ctx.set_mass(m)
    lx, ly, lz, lt = dims
    v = synthetic.gaussian_vectors((nv, lt, lz, ly, lx, 4, 3), seed + 1)
    ctx.mg_setup([{"block": blk, "nv": nv, "setup_iters": setup_iters, "vectors": gpu(v)}], normal=True,
                 coarse_tol=1e-2, coarse_maxit=500)
    return ctx, u, v


@pytest.mark.parametrize("dims,blk,nv", [((6, 6, 6, 6), (2, 2, 2, 2), 2), ((12, 6, 6, 8), (4, 2, 2, 2), 3)])
def test_normal_coarse_operator_matches_oracle(dims, blk, nv):
    m = -0.3
    ctx, u, v = setup(dims, blk, nv, m, 400 + sum(dims))
    op = normal.NormalLevel(u, m, -1.0)
    q, _ = transfer.block_orthonormalize(transfer.as_chiral(v), blk)
    st = normal.build_normal_stencil(op, q, blk)
    c = synthetic.gaussian_vectors((2,) + st.site_shape + (2, nv), 403)
    got = ctx.apply_Nc(1, gpu(c)).cpu().numpy()
    for j in range(2):
        assert rel(got[j], st.apply(c[j])) < 1e-12, j
    # the direct coarse operator is unchanged by the normal-equation setup
    dc = coarse.build_stencil(coarse.WilsonLevel(u, m, -1.0), q, blk)
    assert rel(ctx.apply_Dc(1, gpu(c[0])).cpu().numpy(), dc.apply(c[0])) < 1e-12
    # a mass change probes (D^dagger D)_c again
    ctx.set_mass(m + 0.2)
    st2 = normal.build_normal_stencil(normal.NormalLevel(u, m + 0.2, -1.0), q, blk)
    assert rel(ctx.apply_Nc(1, gpu(c[1])).cpu().numpy(), st2.apply(c[1])) < 1e-12
    ctx.close()


def test_candidates_relaxed_on_the_normal_operator():
    dims, blk, nv, m = (6, 6, 6, 6), (2, 2, 2, 2), 3, -0.3
    ctx, u, v = setup(dims, blk, nv, m, 411, setup_iters=4)
    op = normal.NormalLevel(u, m, -1.0)
    relaxed = mg.relax_null_vectors(op.apply, transfer.as_chiral(v), 4, 0.8)
    q, _ = transfer.block_orthonormalize(relaxed, blk)
    qg = ctx.get_prolongator(0).cpu().numpy().reshape(q.shape)
    assert rel(qg, q) < 1e-9
    ctx.close()


def test_cgnr_and_mg_cg_reach_the_true_residual():
    dims = (8, 8, 8, 8)
    seed = synthetic.gauge_seed(1, 1)
    m = MCRIT[f"8x8x8x8_eps0.3_seed{seed}"]["m_crit"] + 0.1
    ctx, u, _ = setup(dims, (2, 2, 2, 2), 4, m, seed, setup_iters=20)
    b = synthetic.gaussian_spinor(dims, seed=412)
    res = {}
    for outer in ("cgnr", "mgcg"):
        x, st = ctx.solve(gpu(b), tol=1e-10, maxit=20000, outer=outer)
        r = np.linalg.norm(b - wilson.apply_D(u, x.cpu().numpy(), m)) / np.linalg.norm(b)
        assert st[0]["converged"] and r <= 1e-10, (outer, r, st[0])
        res[outer] = st[0]["iters"]
    assert res["mgcg"] < res["cgnr"], res
    ctx.close()


def test_normal_error_paths():
    dims = (8, 8, 8, 8)
    u = synthetic.gauge_field(dims, 0.3, 421)
    ctx = wdmg.Context(dims, DEV)
    ctx.set_gauge(gpu(u), t_bc=-1)
    ctx.set_mass(-0.4)
    v = gpu(synthetic.gaussian_vectors((2, 8, 8, 8, 8, 4, 3), 422))
    with pytest.raises(wdmg.WdmgError) as e:  # coarse extent 2
        ctx.mg_setup([{"block": (4, 4, 4, 4), "nv": 2, "setup_iters": 0, "vectors": v}], normal=True)
    assert e.value.name == "WDMG_ERR_DIMS"
    ctx.mg_setup([{"block": (4, 4, 4, 4), "nv": 2, "setup_iters": 0, "vectors": v}])
    b = gpu(synthetic.gaussian_spinor(dims, seed=423))
    with pytest.raises(wdmg.WdmgError) as e:  # MG-CG without a normal-equation hierarchy
        ctx.solve(b, outer="mgcg")
    assert e.value.name == "WDMG_ERR_NOT_SETUP"
    with pytest.raises(wdmg.WdmgError) as e:
        ctx.apply_Nc(1, torch.zeros(ctx.coarse_shape(1), dtype=torch.complex128, device=DEV))
    assert e.value.name == "WDMG_ERR_NOT_SETUP"
    ctx.close()
