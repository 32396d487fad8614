"""GPU parity of the 16-bit storage paths (FP16 and BF16 storage, FP32 arithmetic).

* Conversion (store and read back a fine field) is compared bit for bit with
  the oracle's definition of the format (``oracle.precision``).
* Every 16-bit kernel is compared with the FP64 oracle applied to the values
  the kernel reads (the stored input, the stored links or P), within the
  error the format adds to its output: half a unit in the last place times
  the scale of each stored result, plus FP32 arithmetic.
* A solve with the V-cycle in 16-bit storage must still reach the FP64 true
  residual 1e-10: the outer FGCR is FP64 (spec tolerance).
"""
import json
import os

import numpy as np
import pytest
import torch

import synthetic
from oracle import coarse, precision, transfer, wilson
from paper_0811_4331_amd import wdmg

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
KINDS = ["f16", "bf16"]
with open(os.path.join(os.path.dirname(__file__), "golden", "mcrit.json")) as _fh:
    MCRIT = json.load(_fh)


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def site_max(f):
    """Largest |real component| of every site of fields [..., 4, 3] (or [..., N])."""
    return np.maximum(np.abs(f.real), np.abs(f.imag)).max(axis=(-2, -1))


def spread_field(dims, seed, nrhs=1):
    """Gaussian spinors with per-site magnitudes spread over 8 decades, a zero
    site, a subnormal-scale site and a site of exact rounding ties."""
    lx, ly, lz, lt = dims
    psi = synthetic.gaussian_spinor(dims, seed=seed, nrhs=nrhs)
    rng = np.random.default_rng(seed + 1)
    psi = psi * 10.0 ** rng.uniform(-4, 4, size=psi.shape[:-2])[..., None, None]
    psi[..., 0, 0, 0, 0, :, :] = 0.0
    psi[..., 0, 0, 0, 1, :, :] = 1e-39 * (1 + 1j)            # scale below the normal range
    tie = np.zeros((4, 3), dtype=np.complex128)
    tie[0, 0] = 1.0                                          # scale exactly 1
    tie[1, 1] = (0.5 + 2.0 ** -12) + 1j * (0.5 + 2.0 ** -9)  # fp16 and bf16 ties
    tie[2, 2] = -(1.0 - 2.0 ** -12) + 1j * (0.25 + 3 * 2.0 ** -11)
    psi[..., 0, 0, 0, 2, :, :] = tie
    return psi


@pytest.mark.parametrize("kind", KINDS + ["f32", "f64"])
def test_storage_roundtrip_is_bit_exact(kind):
    dims = (6, 4, 2, 10)  # ragged: last 64-site block partly padding
    ctx = wdmg.Context(dims, DEV)
    psi = spread_field(dims, 5, nrhs=2)
    if kind == "f64":
        out = ctx.roundtrip(gpu(psi), "f64").cpu().numpy()
        assert np.array_equal(out, psi)
        return
    p32 = psi.astype(np.complex64)
    out = ctx.roundtrip(gpu(p32), kind).cpu().numpy()
    want = p32 if kind == "f32" else precision.store_fine(psi, kind)
    assert out.dtype == np.complex64
    bad = np.argwhere(out.view(np.uint32) != want.view(np.uint32))
    detail = [(tuple(i), p32.view(np.float32)[tuple(i)], out.view(np.float32)[tuple(i)],
               want.view(np.float32)[tuple(i)]) for i in bad[:4]]
    assert len(bad) == 0, (len(bad), detail)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("dims,t_bc", [((8, 8, 8, 8), -1), ((6, 4, 2, 10), 1), ((2, 2, 2, 2), -1)])
def test_apply_D_16bit(kind, dims, t_bc):
    m = -0.4
    u = synthetic.gauge_field(dims, 0.35, 300 + sum(dims))
    ctx = wdmg.Context(dims, DEV)
    ctx.set_gauge(gpu(u), t_bc=t_bc)
    ctx.set_mass(m)
    psi = synthetic.gaussian_spinor(dims, seed=9, nrhs=3)
    out = ctx.apply_D(gpu(psi.astype(np.complex64)), prec=kind).cpu().numpy().astype(np.complex128)
    # oracle on the values the kernel reads
    xin = precision.store_fine(psi, kind).astype(np.complex128)
    uq = precision.store_su3_links(u, kind)
    ref = wilson.apply_D(uq, xin, m, float(t_bc))
    err = np.maximum(np.abs((out - ref).real), np.abs((out - ref).imag)).max(axis=(-2, -1))
    bound = precision.HALF_ULP[kind] * site_max(ref) * 1.001 + 1e-5 * 8 * np.abs(xin).max()
    assert np.all(err <= bound), float((err / bound).max())
    # and the format error against the unrounded FP64 operator is what the formats imply
    exact = wilson.apply_D(u, psi, m, float(t_bc))
    r = np.linalg.norm(out - exact) / np.linalg.norm(exact)
    assert r < {"f16": 2e-3, "bf16": 1.5e-2}[kind], r


def _setup(dims, blk, nv, m, seed):
    u = synthetic.gauge_field(dims, 0.3, seed)
    ctx = wdmg.Context(dims, DEV)
    ctx.set_gauge(gpu(u), t_bc=-1)
    ctx.set_mass(m)
    lx, ly, lz, lt = dims
    v = synthetic.gaussian_vectors((nv, lt, lz, ly, lx, 4, 3), seed + 50)
    ctx.mg_setup([{"block": blk, "nv": nv, "setup_iters": 0, "vectors": gpu(v)}], coarse_tol=1e-12,
                 coarse_maxit=500)
    q, _ = transfer.block_orthonormalize(transfer.as_chiral(v), blk)
    return ctx, u, q, coarse.WilsonLevel(u, m, -1.0)


@pytest.mark.parametrize("kind", KINDS)
def test_transfer_16bit(kind):
    dims, blk, nv = (8, 8, 8, 8), (4, 4, 4, 4), 12
    ctx, u, q, lev = _setup(dims, blk, nv, -0.5, 91)
    qs = precision.store_links(q, kind).astype(np.complex128)   # P stored unscaled
    f = synthetic.gaussian_spinor(dims, seed=92, nrhs=5)
    fin = precision.store_fine(f, kind).astype(np.complex128)
    rc = ctx.restrict(0, gpu(f.astype(np.complex64)), prec=kind).cpu().numpy()
    rc_ref = np.stack([transfer.restrict(qs, transfer.as_chiral(fin[j]), blk) for j in range(5)])
    # a batch runs on the matrix cores with FP32 accumulation over the K = 2 x 6 x 4^4
    # real terms of an aggregate: per output, |err| <= 4 sqrt(K) u sum_r |v_r| |f_r|
    # (u = 2^-24, the statistical bound of a recursive FP32 sum)
    absum = np.stack([transfer.restrict(np.abs(qs).astype(np.complex128),
                                        np.abs(transfer.as_chiral(fin[j])).astype(np.complex128), blk)
                      for j in range(5)]).real
    bound = 4 * np.sqrt(2 * 6 * 256) * 2.0 ** -24 * absum + 1e-7 * np.abs(rc_ref).max()
    assert np.all(np.abs(rc - rc_ref) <= bound), float((np.abs(rc - rc_ref) / bound).max())
    ec = synthetic.gaussian_vectors(rc_ref.shape, 93)
    pe = ctx.prolong(0, gpu(ec.astype(np.complex64)), prec=kind).cpu().numpy().astype(np.complex128)
    pe_ref = np.stack([transfer.as_spinor(transfer.prolong(qs, ec[j].astype(np.complex64).astype(np.complex128),
                                                           blk)) for j in range(5)])
    err = np.maximum(np.abs((pe - pe_ref).real), np.abs((pe - pe_ref).imag)).max(axis=(-2, -1))
    bound = precision.HALF_ULP[kind] * site_max(pe_ref) * 1.001 + 1e-5 * np.abs(pe_ref).max()
    assert np.all(err <= bound), float((err / bound).max())


def _coarse_bound(st, c, kind, mfma):
    """Error bound of the 16-bit coarse operator on FP32 vectors c [nrhs, T,Z,Y,X, 2, Nv]:
    per block d of site x, u s_A (||c_nb||_1 + [mfma] 2N s_c(nb)), summed over d."""
    u = precision.HALF_ULP[kind]
    n2 = 2 * st.nv
    axis = {0: 3, 1: 2, 2: 1, 3: 0}
    blocks = [(st.x, 0, 0)]
    for mu in range(4):
        blocks.append((st.y[mu, 0], mu, -1))  # couples to x + mu
        blocks.append((st.y[mu, 1], mu, +1))  # couples to x - mu
    cr = c.reshape(c.shape[:-2] + (n2,))
    bound = 0.0
    for blk, mu, shift in blocks:
        sa = np.maximum(np.abs(blk.real), np.abs(blk.imag)).max(axis=(-2, -1))
        cn = cr if shift == 0 else np.roll(cr, shift, axis=1 + axis[mu])
        l1 = (np.abs(cn.real) + np.abs(cn.imag)).sum(axis=-1)
        sc = np.maximum(np.abs(cn.real), np.abs(cn.imag)).max(axis=-1)
        bound = bound + u * sa * (l1 + (2 * n2 * sc if mfma else 0.0))
    return bound


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("nv,nrhs", [(12, 1), (12, 5), (20, 33), (7, 2)])
def test_coarse_operator_16bit(kind, nv, nrhs):
    """16-bit blocks with one scale per block: the vector units for one rhs,
    the 16-bit MFMA units (32x32x8, FP32 accumulation) for a batch."""
    dims, blk = (12, 8, 8, 8), (4, 4, 4, 4)
    ctx, u, q, lev = _setup(dims, blk, nv, -0.45, 95)
    st = coarse.build_stencil(lev, q, blk)
    c = synthetic.gaussian_vectors((nrhs, 2, 2, 2, 3, 2, nv), 96).astype(np.complex64)
    out = ctx.apply_Dc(1, gpu(c), prec=kind).cpu().numpy().astype(np.complex128)
    c64 = c.astype(np.complex128)
    ref = np.stack([st.apply(c64[j]) for j in range(nrhs)])
    err = np.abs(out - ref).reshape(nrhs, 2, 2, 2, 3, -1).max(axis=-1)
    bound = 1.01 * _coarse_bound(st, c64, kind, mfma=nrhs >= 2) + 1e-5 * np.abs(ref).max()
    assert np.all(err <= bound), float((err / bound).max())
    # a mass shift invalidates and rebuilds the 16-bit blocks
    ctx.set_mass(-0.45 + 0.2)
    out2 = ctx.apply_Dc(1, gpu(c), prec=kind).cpu().numpy().astype(np.complex128)
    st2 = st.shifted(0.2)
    ref2 = np.stack([st2.apply(c64[j]) for j in range(nrhs)])
    bound2 = 1.01 * _coarse_bound(st2, c64, kind, mfma=nrhs >= 2) + 1e-5 * np.abs(ref2).max()
    err2 = np.abs(out2 - ref2).reshape(nrhs, 2, 2, 2, 3, -1).max(axis=-1)
    assert np.all(err2 <= bound2), float((err2 / bound2).max())


@pytest.mark.parametrize("kind", KINDS)
def test_mr_16bit_reduces_residual_like_fp64(kind):
    """MR in 16-bit storage from the same start: the residual after the steps
    agrees with FP64 MR to the storage precision."""
    dims = (8, 8, 8, 8)
    u = synthetic.gauge_field(dims, 0.3, 97)
    ctx = wdmg.Context(dims, DEV)
    ctx.set_gauge(gpu(u))
    ctx.set_mass(-0.3)
    b = synthetic.gaussian_spinor(dims, seed=98, nrhs=2)
    x0 = np.zeros_like(b)
    x64 = gpu(x0)
    ctx.smooth(0, x64, gpu(b), 4)
    xh = gpu(x0.astype(np.complex64))
    ctx.smooth(0, xh, gpu(b.astype(np.complex64)), 4, prec=kind)
    for j in range(2):
        r64 = b[j] - wilson.apply_D(u, x64[j].cpu().numpy(), -0.3)
        rh = b[j] - wilson.apply_D(u, xh[j].cpu().numpy().astype(np.complex128), -0.3)
        n64, nh = np.linalg.norm(r64), np.linalg.norm(rh)
        assert nh < np.linalg.norm(b[j])
        assert abs(nh - n64) <= {"f16": 5e-3, "bf16": 4e-2}[kind] * np.linalg.norm(b[j]), (nh, n64)


@pytest.mark.parametrize("kind", KINDS)
def test_solve_with_16bit_vcycle_reaches_fp64_tolerance(kind):
    dims = (8, 8, 8, 8)
    seed = synthetic.gauge_seed(1, 1)
    m = MCRIT[f"8x8x8x8_eps0.3_seed{seed}"]["m_crit"] + 0.05
    u = synthetic.gauge_field(dims, 0.3, seed)
    ctx = wdmg.Context(dims, DEV)
    ctx.set_gauge(gpu(u))
    ctx.set_mass(m)
    nv = 12
    v0 = synthetic.gaussian_vectors((nv,) + ctx.fine_shape(), synthetic.null_seed(1))
    ctx.mg_setup([{"block": (4, 4, 4, 4), "nv": nv, "setup_iters": 50, "vectors": gpu(v0)}], coarse_tol=1e-2)
    b = synthetic.gaussian_spinor(dims, seed=synthetic.rhs_seed(1), nrhs=3)
    x32, s32 = ctx.solve(gpu(b), tol=1e-10, restart=50, maxit=300, mg_prec="f32")
    x, st = ctx.solve(gpu(b), tol=1e-10, restart=50, maxit=300, mg_prec=kind)
    for j in range(3):
        res = float(np.linalg.norm(b[j] - wilson.apply_D(u, x[j].cpu().numpy(), m)) / np.linalg.norm(b[j]))
        assert st[j]["converged"] and res <= 1e-10, (res, st[j])
        # the 16-bit V-cycle is a slightly weaker preconditioner, not a different one
        assert st[j]["iters"] <= 1.5 * s32[j]["iters"] + 3, (st[j]["iters"], s32[j]["iters"])


def test_three_level_solve_with_16bit_intermediate_level():
    dims = (8, 8, 8, 8)
    m = -0.5
    u = synthetic.gauge_field(dims, 0.3, 61)
    ctx = wdmg.Context(dims, DEV)
    ctx.set_gauge(gpu(u))
    ctx.set_mass(m)
    v1 = synthetic.gaussian_vectors((4, 8, 8, 8, 8, 4, 3), 62)
    v2 = synthetic.gaussian_vectors((6, 4, 4, 4, 4, 2, 4), 63)
    ctx.mg_setup([{"block": (2, 2, 2, 2), "nv": 4, "setup_iters": 0, "vectors": gpu(v1)},
                  {"block": (2, 2, 2, 2), "nv": 6, "setup_iters": 0, "vectors": gpu(v2)}],
                 coarse_tol=1e-3, coarse_cycles=4)
    bb = synthetic.gaussian_spinor(dims, seed=68, nrhs=3)
    for kind in KINDS:
        xb, sb = ctx.solve(gpu(bb), tol=1e-10, restart=30, maxit=300, mg_prec=kind)
        for j in range(3):
            assert sb[j]["converged"], (kind, sb[j])
            res = np.linalg.norm(bb[j] - wilson.apply_D(u, xb[j].cpu().numpy(), m)) / np.linalg.norm(bb[j])
            assert res <= 1e-10


def _aggregate_columns(q, blk):
    """``[Nv, T, Z, Y, X, 2, 6]`` -> ``[Tc, Zc, Yc, Xc, chi, rows, Nv]``: the
    orthonormal columns of P on each (aggregate, chirality)."""
    bx, by, bz, bt = blk
    nv, lt, lz, ly, lx, two, n = q.shape
    a = q.reshape(nv, lt // bt, bt, lz // bz, bz, ly // by, by, lx // bx, bx, two, n)
    a = a.transpose(1, 3, 5, 7, 9, 2, 4, 6, 8, 10, 0)
    return a.reshape(lt // bt, lz // bz, ly // by, lx // bx, two, bt * bz * by * bx * n, nv)


@pytest.mark.parametrize("setup_prec", ["f32", "f16", "bf16"])
def test_setup_relaxation_in_reduced_precision(setup_prec):
    """Sec. 2 setup relaxation with the candidates in FP32 or 16-bit storage.

    The block QR of nearly dependent candidates amplifies a perturbation of
    the candidates in its last columns (FP32 storage, 6e-8, moves the spans
    by about 4e-5 here), so P itself is compared with the FP64 oracle's only
    in FP32 (largest principal-angle sine over all aggregates and both
    chiralities; the 16-bit spans are only reported), and for every
    precision the FP64 MG solve built on the hierarchy must reach 1e-10 with
    at most two more outer iterations than the one built on the FP64 setup:
    the relaxation is judged by the coarse space it delivers."""
    dims, blk, nv = (8, 8, 8, 8), (4, 4, 4, 4), 12
    seed = synthetic.gauge_seed(1, 1)
    m = MCRIT[f"8x8x8x8_eps0.3_seed{seed}"]["m_crit"] + 0.05
    u = synthetic.gauge_field(dims, 0.3, seed)
    ctx = wdmg.Context(dims, DEV)
    ctx.set_gauge(gpu(u))
    ctx.set_mass(m)
    v0 = synthetic.gaussian_vectors((nv,) + ctx.fine_shape(), synthetic.null_seed(1))
    b = synthetic.gaussian_spinor(dims, seed=synthetic.rhs_seed(1))
    op = coarse.WilsonLevel(u, m, -1.0)
    from oracle import mg
    qref, _ = transfer.block_orthonormalize(mg.relax_null_vectors(op.apply, transfer.as_chiral(v0), 50), blk)
    a_ref = _aggregate_columns(qref, blk)
    iters = {}
    for prec in ("f64", setup_prec):
        ctx.mg_setup([{"block": blk, "nv": nv, "setup_iters": 50, "vectors": gpu(v0), "setup_prec": prec}],
                     coarse_tol=1e-2)
        qg = ctx.get_prolongator(0).cpu().numpy().reshape(qref.shape)
        a = _aggregate_columns(qg, blk)
        # sine of the largest principal angle between the two column spans
        resid = a - a_ref @ (np.conj(np.swapaxes(a_ref, -1, -2)) @ a)
        sin_max = float(np.linalg.norm(resid, ord=2, axis=(-2, -1)).max())
        print(f"setup {prec}: largest principal-angle sine {sin_max:.2e}")
        if prec in ("f64", "f32"):
            assert sin_max <= {"f64": 1e-9, "f32": 1e-3}[prec], (prec, sin_max)
        x, st = ctx.solve(gpu(b), tol=1e-10, restart=50, maxit=300)
        res = float(np.linalg.norm(b - wilson.apply_D(u, x.cpu().numpy(), m)) / np.linalg.norm(b))
        assert st[0]["converged"] and res <= 1e-10, (prec, res)
        iters[prec] = st[0]["iters"]
    print(f"outer iterations: {iters}")
    assert iters[setup_prec] <= iters["f64"] + 2, iters
    ctx.close()


def test_in_place_solve_equals_the_regular_solve():
    """An in-place FGCR solve (x from zero, written over b, b read from the
    caller's buffer at every restart) gives the regular solve's iterates: the
    same kernels on the same values."""
    dims = (8, 8, 8, 8)
    seed = synthetic.gauge_seed(1, 1)
    m = MCRIT[f"8x8x8x8_eps0.3_seed{seed}"]["m_crit"] + 0.05
    u = synthetic.gauge_field(dims, 0.3, seed)
    ctx = wdmg.Context(dims, DEV)
    ctx.set_gauge(gpu(u))
    ctx.set_mass(m)
    v0 = synthetic.gaussian_vectors((12,) + ctx.fine_shape(), synthetic.null_seed(1))
    ctx.mg_setup([{"block": (4, 4, 4, 4), "nv": 12, "setup_iters": 20, "vectors": gpu(v0)}], coarse_tol=1e-2)
    b = synthetic.gaussian_spinor(dims, seed=synthetic.rhs_seed(1, 3), nrhs=4)
    for kind in KINDS:
        x, st = ctx.solve(gpu(b), tol=1e-10, restart=6, maxit=300, mg_prec=kind)
        bg = gpu(b)
        xi, sti = ctx.solve(bg, tol=1e-10, restart=6, maxit=300, mg_prec=kind, in_place=True)
        assert xi.data_ptr() == bg.data_ptr()
        xh, xih = x.cpu().numpy(), xi.cpu().numpy()
        for j in range(4):
            assert sti[j]["converged"] and sti[j]["iters"] == st[j]["iters"], (kind, j, st[j], sti[j])
            assert np.abs(xih[j] - xh[j]).max() <= 1e-13 * np.abs(xh[j]).max(), (kind, j)
            res = np.linalg.norm(b[j] - wilson.apply_D(u, xih[j], m)) / np.linalg.norm(b[j])
            assert res <= 1e-10, (kind, j, res)
    bg = gpu(b)
    import ctypes
    params = wdmg.SolveParams(1e-10, 6, 300, 1, wdmg.PREC["bf16"], 0, 0, 0)
    with pytest.raises(wdmg.WdmgError) as e:  # the same buffer without in_place
        ctx._check(ctx.lib.wdmg_solve(ctx.h, bg.data_ptr(), bg.data_ptr(), 4, ctypes.byref(params), None))
    assert e.value.name == "WDMG_ERR_ARG" and "in_place" in str(e.value)
    with pytest.raises(wdmg.WdmgError) as e:  # an FP64 V-cycle has no FP32 basis to hold b
        ctx.solve(bg, tol=1e-10, restart=6, maxit=300, mg_prec="f64", in_place=True)
    assert e.value.name == "WDMG_ERR_ARG"
    ctx.close()
