#!/usr/bin/env python
"""Benchmark of the adaptive-multigrid Wilson-Dirac solve on one MI355X.

One step = one pass of the whole hot path over one batch of right-hand sides:
the adaptive setup (MR relaxation of the Nv starting vectors on D v = 0,
FP64 block orthonormalisation, Galerkin coarse operator) followed by the
MG-preconditioned flexible GCR(50) solve of every right-hand side to true
relative residual 1e-10 (FP64).  `value` is the step's wall time per
right-hand side, inputs resident in HBM before the timed region.

Default workload: the 16^4 lattice with links exp(i 0.3 H), antiperiodic
time, m = m_crit + 0.01 (m_crit from the oracle's Arnoldi, stored in
tests/golden/mcrit.json), 2-level MG with 4^4 aggregates and Nv = 20, FP64
throughout, one Gaussian right-hand side.  Unpreconditioned FP64 BiCGStab on
the same GPU is timed beside it, outside the K steps.

The JSON line also carries the roofline of the dominant kernel (timed with
HIP events on the library's stream during the timed steps), Dslash bandwidth
on a lattice larger than the 256 MB Infinity Cache, and the FP64 oracle timed
on the host as `cpu_baseline`.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MG time-to-solution @ rel.res 1e-10 (s/RHS); Dslash GB/s; D_c MFMA util"
HBM_PEAK_GBS = 8000.0
# Algorithmic (compulsory) bytes per work unit, per kernel.
DSLASH_BYTES = {"f64": 960, "f32": 480, "f16": 248, "bf16": 248}  # per fine site: psi in, 4 links, out


def dc_bytes(prec, nv):                            # per coarse site: 9 blocks + in + out
    b = 16 if prec == "f64" else 8
    n2 = 2 * nv
    return 9 * n2 * n2 * b + 2 * n2 * b


def coarse_gcr_bytes(nsite, n2, units):           # one coarsest GCR operator launch (FP64 D_c)
    """D_c read once per launch (9 blocks per coarse site), r read, w_j and z_j written."""
    return nsite * 9 * n2 * n2 * 16 + units * 3 * n2 * 16


# Dense matrix-core peaks of MI355X (TFLOP/s) by the dtype the contraction runs in.
MFMA_PEAK_TFS = {"f64": 78.6, "f32": 157.3, "h": 2500.0}


def dc_mfma_util(kinfo, nrhs, n2_mid, n2_coarsest):
    """Achieved FLOP/s of the coarse-operator launches that run on matrix cores,
    against the dense peak of their dtype.  A unit is one (coarse site, rhs);
    one unit costs 9 (2Nv)^2 complex multiply-adds = 72 (2Nv)^2 real flops.
    The intermediate-level kernels use Nv of the first coarsening; the
    coarsest GCR's operator launch (FP64 matrix cores once nrhs > 1) uses the
    coarsest level's Nv."""
    out = {}
    for name, dt, n2 in (("dc_mfma_f64", "f64", n2_mid), ("dc_mfma_f32", "f32", n2_mid),
                         ("dc_mfma_h", "h", n2_mid), ("coarse_gcr", "f64", n2_coarsest)):
        k = kinfo.get(name)
        if k is None or (name == "coarse_gcr" and nrhs < 2):
            continue
        flops = 72.0 * n2 * n2 * k["units"]
        tfs = flops / (k["ms_total"] / 1e3) / 1e12
        out[name] = {"dtype": dt, "achieved_tflops": tfs, "peak_tflops": MFMA_PEAK_TFS[dt],
                     "util": tfs / MFMA_PEAK_TFS[dt]}
    return out or None


def counter_traffic(kernel, dims, bytes_per_launch, tuning=None):
    """HBM bytes per launch from the committed PMC measurement of this kernel on
    this lattice (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's reading), or
    None when there is none, the kernel's sources changed since, or this run's
    Wilson forms and rhs groups differ from the ones the counters were taken with."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    h = hashlib.sha256()
    for f in t["source_files"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != t["source_hash"]:
        return None
    for e in t["entries"].get(kernel + "@" + "x".join(map(str, dims)), []):
        if e.get("wilson_tuning") == tuning:
            return e["measured_over_algorithmic"] * bytes_per_launch
    return None


def transfer_bytes(prec, nv):                      # per fine site: Nv columns (12 cplx) + fine + coarse share
    b = 16 if prec == "f64" else 8
    return 12 * nv * b + 12 * b


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--L", type=int, default=16, help="lattice extent (L^4)")
    ap.add_argument("--dims", type=int, nargs=4, default=None, metavar=("LX", "LY", "LZ", "LT"),
                    help="lattice extents (overrides --L)")
    ap.add_argument("--mcrit-dims", type=int, nargs=4, default=None, metavar=("LX", "LY", "LZ", "LT"),
                    help="take m_crit from the oracle's value for this lattice at the same eps "
                         "(for lattices too large for the host Arnoldi)")
    ap.add_argument("--eps", type=float, default=0.3)
    ap.add_argument("--delta", type=float, default=0.01, help="m - m_crit")
    ap.add_argument("--mass", type=float, default=None,
                    help="use this bare mass instead of m_crit + delta (no m_crit lookup)")
    ap.add_argument("--nv", type=int, default=20)
    ap.add_argument("--levels", type=int, default=2, choices=[2, 3],
                    help="3: a second coarsening with 2^4 aggregates (Sec. 5 three-level cycle)")
    ap.add_argument("--nv2", type=int, default=32, help="near-null vectors of the second coarsening")
    ap.add_argument("--setup-iters", type=int, default=None,
                    help="MR relaxation steps per near-null vector (default 50 for fewer than 8 rhs, "
                         "100 for larger batches, whose setup cost is shared)")
    ap.add_argument("--adapt-iters", type=int, default=0,
                    help="adaptive augmentation (Sec. 2): two-level iterations refining each candidate "
                         "after the first (0: relaxation only)")
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--nullvec-source", default="host", choices=["host", "device"],
                    help="first-level null-vector starts: numpy on the host, kept on the device (default), or "
                         "torch's seeded device generator inside each step, released after the setup (large lattices)")
    ap.add_argument("--wilson-tuning", default=None, metavar="F1,FB,GB",
                    help="force the Wilson form of one-rhs launches (F1), and the form (FB) and rhs group (GB) "
                         "of the setup's batched launches, instead of the autotuner (one-rhs solves only)")
    ap.add_argument("--release-unused", action="store_true",
                    help="after each setup, free the FP64/FP32 copies of P and D_c that the 16-bit V-cycle "
                         "does not read (room for larger batches)")
    ap.add_argument("--coarse-apply", type=int, default=None, choices=[0, 1],
                    help="force a form of the batched coarsest-level operator (default: library choice)")
    ap.add_argument("--setup-prec", default="f64", choices=["f64", "f32"],
                    help="arithmetic of the setup relaxation (the block QR is FP64 either way)")
    ap.add_argument("--mg-prec", default="f64", choices=["f64", "f32", "f16", "bf16"])
    ap.add_argument("--coarse-tol", type=float, default=0.1)
    ap.add_argument("--alpha", action="store_true",
                    help="take the minimal-residual step size after prolongation (off: alpha = 1, "
                         "which converges in far fewer outer iterations on these fields)")
    ap.add_argument("--restart", type=int, default=50, help="FGCR restart length (paper: 50)")
    ap.add_argument("--outer", default="fgcr", choices=["fgcr", "bicgstab"],
                    help="outer Krylov method: flexible GCR (Sec. 5) or BiCGStab with the V-cycle as right "
                         "preconditioner (Sec. 4)")
    ap.add_argument("--precision-report", action="store_true",
                    help="relative error of every reduced-precision operator against its FP64 form")
    ap.add_argument("--graph", action="store_true",
                    help="capture the V-cycle in a HIP graph after its first application and replay it")
    ap.add_argument("--big-L", type=int, default=32, help="lattice for the out-of-cache Dslash figure (0: skip)")
    ap.add_argument("--no-bicgstab", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--only-dslash", type=int, default=0, metavar="L",
                    help="only time Dslash (FP64, FP32) on L^4 plus a plain 1 GiB device copy "
                         "(the reference for hardware byte counters), then exit")
    a = ap.parse_args()
    if a.setup_iters is None:
        a.setup_iters = 50 if a.nrhs < 8 else 100
    return a


def load_mcrit(dims, eps, seed):
    path = os.path.join(ROOT, "tests", "golden", "mcrit.json")
    key = "x".join(str(d) for d in dims) + f"_eps{eps}_seed{seed}"
    with open(path) as fh:
        data = json.load(fh)
    if key not in data:
        raise SystemExit(f"no oracle m_crit for {key} in {path}; run tests/golden/make_mcrit.py")
    return float(data[key]["m_crit"])


def workload_number(dims):
    """Seed family of a lattice: 8^4 -> 1, 16^4 -> 2, 32^4 -> 3, 24^3x48 -> 4, 48^3x96 -> 5."""
    return {(8, 8, 8, 8): 1, (16, 16, 16, 16): 2, (32, 32, 32, 32): 3, (24, 24, 24, 48): 4,
            (48, 48, 48, 96): 5}.get(tuple(dims), 9)


def dslash_bandwidth(wdmg, synthetic, torch, dev, L, reps=20):
    """Dslash kernel time on an L^4 lattice (links exp(i 0.45 H)), FP64 and FP32."""
    dims = (L, L, L, L)
    u = synthetic.gauge_field(dims, 0.45, synthetic.gauge_seed(3, 2))
    ctx = wdmg.Context(dims, dev)
    ctx.set_gauge(torch.from_numpy(u).to(dev), t_bc=-1)
    del u
    ctx.set_mass(-1.0)
    psi = torch.from_numpy(synthetic.gaussian_spinor(dims, 5)).to(dev)
    out = {}
    precs = (("f64", "dslash_f64"), ("f32", "dslash_f32"), ("f16", "dslash_f16"), ("bf16", "dslash_bf16"))
    # both kernel forms forced, then the autotuner's pick
    forms = {}
    for form in (0, 1, 2):
        ctx.set_tuning("dslash", form)
        for prec, key in precs:
            x = psi if prec == "f64" else psi.to(torch.complex64)
            ctx.apply_D(x, prec=prec)
            torch.cuda.synchronize()
            ctx.profile(True)
            for _ in range(reps):
                ctx.apply_D(x, prec=prec)
            n, units, ms = ctx.profile_read()[key]
            ctx.profile(False)
            sec = ms / 1e3 / n
            forms[f"{prec}_form{form}"] = {"us_per_launch": sec * 1e6,
                                           "GB_s": DSLASH_BYTES[prec] * units / n / sec / 1e9}
    ctx.set_tuning("dslash", None)
    out["forms"] = {"lattice": f"{L}^4", "form0": "one thread per site", "form1": "one wave per direction",
                    "form2": "one wave per direction, registers capped for 4 waves per SIMD",
                    **forms}
    for prec, key in precs:
        x = psi if prec == "f64" else psi.to(torch.complex64)
        ctx.apply_D(x, prec=prec)
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(reps):
            ctx.apply_D(x, prec=prec)
        n, units, ms = ctx.profile_read()[key]
        ctx.profile(False)
        sec = ms / 1e3 / n
        out[prec] = {"lattice": f"{L}^4", "us_per_launch": sec * 1e6,
                     "GB_s": DSLASH_BYTES[prec] * units / n / sec / 1e9,
                     "frac_hbm_peak": DSLASH_BYTES[prec] * units / n / sec / 1e9 / HBM_PEAK_GBS,
                     "form": ctx.get_tuning("dslash", prec, 1)}
    # a batch of 8 right-hand sides (links read once per 2 (FP64) or 4 (FP32) rhs)
    xb = psi.unsqueeze(0).repeat(8, 1, 1, 1, 1, 1, 1)
    for prec, key in (("f64", "dslash_f64"), ("f32", "dslash_f32"), ("bf16", "dslash_bf16")):
        x = xb if prec == "f64" else xb.to(torch.complex64)
        ctx.apply_D(x, prec=prec)
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(max(2, reps // 4)):
            ctx.apply_D(x, prec=prec)
        n, units, ms = ctx.profile_read()[key]
        ctx.profile(False)
        sec = ms / 1e3 / n
        out[prec + "_8rhs"] = {"lattice": f"{L}^4 x 8 rhs", "us_per_launch": sec * 1e6,
                               "ns_per_site_rhs": sec / units * n * 1e9,
                               "GB_s_alg_single_rhs_bytes": DSLASH_BYTES[prec] * units / n / sec / 1e9,
                               "form": ctx.get_tuning("dslash", prec, 8),
                               "rhs_group": ctx.get_tuning("dslash_group", prec, 8)}
    ctx.close()
    return out


def only_dslash(L, reps=10):
    """Dslash on L^4 and a plain device copy of known size (counter calibration)."""
    import torch

    import synthetic
    from paper_0811_4331_amd import wdmg
    dev = torch.device("cuda:0")
    res = {"dslash": dslash_bandwidth(wdmg, synthetic, torch, dev, L, reps=reps)}
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)  # 1 GiB
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 3
    res["copy_1GiB"] = {"bytes_read": src.numel() * 8, "bytes_written": dst.numel() * 8,
                        "GB_s_read_plus_write": 2 * src.numel() * 8 / dt / 1e9}
    print(json.dumps(res), flush=True)


def precision_report(ctx, torch, synthetic, dims, nv):
    """||A_prec v - A_f64 v|| / ||A_f64 v|| for D (level 0), P^dagger, P and D_c
    (level 1) on Gaussian vectors, per reduced precision.  The FP64 forms are
    those the parity tests pin to the oracle."""
    def rel(a, b):
        return float(torch.linalg.vector_norm(a.to(torch.complex128) - b) / torch.linalg.vector_norm(b))
    dev = ctx.device
    f = torch.from_numpy(synthetic.gaussian_spinor(dims, 777)).to(dev)
    cshape = ctx.coarse_shape(1)
    c = torch.from_numpy(synthetic.gaussian_vectors(cshape, 778)).to(dev)
    ref = {"D": ctx.apply_D(f), "P_dagger": ctx.restrict(0, f), "P": ctx.prolong(0, c), "D_c": ctx.apply_Dc(1, c)}
    out = {}
    for prec in ("f32", "f16", "bf16"):
        f32, c32 = f.to(torch.complex64), c.to(torch.complex64)
        out[prec] = {"level0_D": rel(ctx.apply_D(f32, prec=prec), ref["D"]),
                     "level0_P_dagger": rel(ctx.restrict(0, f32, prec=prec), ref["P_dagger"]),
                     "level0_P": rel(ctx.prolong(0, c32, prec=prec), ref["P"]),
                     "level1_D_c": rel(ctx.apply_Dc(1, c32, prec=prec), ref["D_c"])}
    return out


def cpu_baseline(u, b, m, n_d_per_step, nrhs, seconds):
    """The FP64 oracle's Wilson operator timed on the host (bounded sample)."""
    from oracle import wilson
    reps = 0
    t0 = time.perf_counter()
    while True:
        wilson.apply_D(u, b, m, -1.0)
        reps += 1
        el = time.perf_counter() - t0
        if el > seconds or reps >= 200:
            break
    t_apply = el / reps
    return {
        "value": t_apply * n_d_per_step / nrhs, "unit": "s/RHS", "cores": 1, "kind": "oracle",
        "sample": (f"{reps} oracle FP64 Wilson applications on the same lattice ({t_apply:.3f} s each, "
                   f"numpy, one thread), scaled by the {n_d_per_step} fine-operator applications of one "
                   "GPU step; a lower bound for the oracle's MG step (coarse, QR and vector work "
                   "excluded)"),
        "host_cpus": os.cpu_count(),
    }


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    if a.only_dslash:
        only_dslash(a.only_dslash)
        return
    import torch

    import synthetic
    from paper_0811_4331_amd import wdmg

    dev = torch.device("cuda:0")
    L = a.L
    dims = tuple(a.dims) if a.dims else (L, L, L, L)
    i_eps = {0.2: 0, 0.3: 1, 0.45: 2}.get(a.eps, 9)
    cfg = workload_number(dims)
    gseed = synthetic.gauge_seed(cfg, i_eps)
    mcrit_src = "oracle Arnoldi on this field"
    if a.mass is not None:
        m = a.mass
        a.delta = float("nan")
    elif a.mcrit_dims:
        md = tuple(a.mcrit_dims)
        m = load_mcrit(md, a.eps, synthetic.gauge_seed(workload_number(md), i_eps)) + a.delta
        mcrit_src = "oracle Arnoldi on the {} field of the same eps".format("x".join(map(str, md)))
    else:
        m = load_mcrit(dims, a.eps, gseed) + a.delta
    u = synthetic.gauge_field(dims, a.eps, gseed)
    ctx = wdmg.Context(dims, dev)
    ctx.set_gauge(torch.from_numpy(u).to(dev), t_bc=-1)
    ctx.set_mass(m)
    ctx.set_tuning("coarse_apply", a.coarse_apply)
    v0_shape = (a.nv,) + ctx.fine_shape()
    if a.nullvec_source == "host":
        v0 = torch.from_numpy(synthetic.gaussian_vectors(v0_shape, synthetic.null_seed(cfg))).to(dev)
    else:
        v0 = None  # drawn on the device inside each step

    def device_v0():
        g = torch.Generator(device=dev)
        g.manual_seed(synthetic.null_seed(cfg))
        return torch.randn(v0_shape, dtype=torch.complex128, device=dev, generator=g)
    bh = np.stack([synthetic.gaussian_spinor(dims, synthetic.rhs_seed(cfg, j)) for j in range(a.nrhs)])
    b = torch.from_numpy(bh).to(dev)
    levels = [{"block": (4, 4, 4, 4), "nv": a.nv, "setup_iters": a.setup_iters, "adapt_iters": a.adapt_iters,
               "vectors": v0,
               "setup_prec": a.setup_prec}]
    if a.levels == 3:
        cdims = tuple(d // 4 for d in dims)
        v1 = torch.from_numpy(synthetic.gaussian_vectors(
            (a.nv2, cdims[3], cdims[2], cdims[1], cdims[0], 2, a.nv), synthetic.null_seed(cfg) + 500)).to(dev)
        levels.append({"block": (2, 2, 2, 2), "nv": a.nv2, "setup_iters": a.setup_iters, "vectors": v1,
                       "setup_prec": a.setup_prec})

    # the setup relaxes its vectors in batches of at most 64 that fit a 16 GiB work budget
    setup_field = int(np.prod(dims)) * 12 * (16 if a.setup_prec == "f64" else 8)
    setup_batch = max(1, min(a.nv, 64, (16 << 30) // (2 * setup_field)))
    forced = None
    if a.wilson_tuning:
        if a.nrhs != 1:
            raise SystemExit("--wilson-tuning is for one-rhs solves")
        forced = [int(v) for v in a.wilson_tuning.split(",")]

    def step():
        if forced:
            ctx.set_tuning("dslash", forced[1])
            ctx.set_tuning("dslash_group", forced[2])
        if v0 is None:
            levels[0]["vectors"] = device_v0()
            torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.mg_setup(levels, coarse_tol=a.coarse_tol, use_alpha=a.alpha)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if v0 is None:
            levels[0]["vectors"] = None  # the setup copied them; the solve gets the memory
        if a.release_unused:
            ctx.release_unused(a.mg_prec)
        if forced:
            ctx.set_tuning("dslash", forced[0])
            ctx.set_tuning("dslash_group", None)
        x, st = ctx.solve(b, tol=1e-10, restart=a.restart, maxit=2000, mg_prec=a.mg_prec, graph=a.graph,
                          outer=a.outer)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return x, st, t1 - t0, t2 - t1

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    t_start = time.perf_counter()
    setups, solves, stats = [], [], []
    for _ in range(a.steps):
        x, st, ts, tv = step()
        setups.append(ts)
        solves.append(tv)
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    # Wilson forms and rhs groups this run used: one-rhs launches (form),
    # the setup's batched launches (form, group)
    if forced:
        wilson_tuning = list(forced)
    else:
        one = "f64" if a.mg_prec == "f64" else "f32"
        wilson_tuning = [ctx.get_tuning("dslash", one, 1), ctx.get_tuning("dslash", a.setup_prec, setup_batch),
                         ctx.get_tuning("dslash_group", a.setup_prec, setup_batch)]
    prof = ctx.profile_read()
    ctx.profile(False)
    last = stats[-1]
    if not all(s["converged"] and s["true_res"] <= 1e-10 for st in stats for s in st):
        raise SystemExit(f"solve did not reach 1e-10: {last}")
    # independent check of the final residual with the library's FP64 D, one
    # rhs at a time (a batch-sized temporary may not fit beside the solver's memory)
    rr = 0.0
    for j in range(a.nrhs):
        rj = b[j] - ctx.apply_D(x[j])
        rr += float(torch.linalg.vector_norm(rj)) ** 2
        del rj
    true_res = rr ** 0.5 / float(torch.linalg.vector_norm(b))

    ms_per_step = elapsed / a.steps * 1e3
    value = elapsed / a.steps / a.nrhs

    # dominant kernel of the step and its roofline
    kinfo = {}
    for name, (n, units, ms) in prof.items():
        if n == 0:
            continue
        kinfo[name] = {"launches": n, "ms_total": ms, "us_per_launch": ms / n * 1e3, "units": units}
    dom = max(kinfo, key=lambda k: kinfo[k]["ms_total"])
    n, units, ms = prof[dom]
    per_launch_s = ms / 1e3 / n
    if dom.startswith("dslash"):
        bpl = DSLASH_BYTES[dom.split("_")[1]] * units / n
    elif dom.startswith("dc_f"):
        bpl = dc_bytes(dom[-3:], a.nv) * units / n
    elif dom.startswith(("restrict", "prolong")):
        bpl = transfer_bytes(dom[-3:], a.nv) * units / n
    elif dom == "coarse_gcr":
        vol = int(np.prod(dims))
        csite, n2 = (vol // 256, 2 * a.nv) if a.levels == 2 else (vol // 4096, 2 * a.nv2)
        bpl = coarse_gcr_bytes(csite, n2, units / n)
    else:
        bpl = None
    roofline = None
    if bpl is not None:
        ach = bpl / per_launch_s / 1e9
        traffic = counter_traffic(dom, dims, bpl, wilson_tuning)
        roofline = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
                    "bytes_per_launch": bpl, "us_per_launch": per_launch_s * 1e6}
    dc_mfma = dc_mfma_util(kinfo, a.nrhs, 2 * a.nv, 2 * a.nv2 if a.levels == 3 else 2 * a.nv)
    ds = prof["dslash_f64"]
    dslash_step = None
    if ds[0]:
        sec = ds[2] / 1e3 / ds[0]
        dslash_step = {"lattice": "x".join(map(str, dims)), "us_per_launch": sec * 1e6,
                       "GB_s": DSLASH_BYTES["f64"] * ds[1] / ds[0] / sec / 1e9}

    result = {
        "metric": METRIC, "value": value, "unit": "s/RHS", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_per_step, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if a.mg_prec == "f64" else f"f64 outer / {a.mg_prec} V-cycle",
        "data": "synthetic",
        "config": {"workload": f"{'x'.join(map(str, dims))} Wilson-Dirac, links exp(i {a.eps} H), "
                               f"m = m_crit + {a.delta}, "
                               + (f"2-level MG 4^4 aggregates Nv={a.nv}, " if a.levels == 2 else
                                  f"3-level MG 4^4 then 2^4 aggregates Nv={a.nv} then {a.nv2}, ")
                               + f"MR setup {a.setup_iters} iters, "
                               + (f"adaptive {a.adapt_iters} two-level iters per candidate, " if a.adapt_iters else "")
                               + (f"FGCR({a.restart})" if a.outer == "fgcr" else "MG-BiCGStab")
                               + f" to 1e-10, {a.nrhs} Gaussian RHS",
                   "lattice": list(dims), "eps": a.eps, "m": m, "m_crit": m - a.delta,
                   "m_crit_source": mcrit_src, "levels": a.levels, "nv": a.nv,
                   "nv2": a.nv2 if a.levels == 3 else None,
                   "nrhs": a.nrhs, "mg_prec": a.mg_prec, "setup_prec": a.setup_prec, "coarse_tol": a.coarse_tol,
                   "adapt_iters": a.adapt_iters, "outer": a.outer,
                   "alpha_step": a.alpha, "graph": a.graph, "nullvec_source": a.nullvec_source,
                   "release_unused": a.release_unused},
        "setup_s": float(np.median(setups)), "solve_s_per_rhs": float(np.median(solves)) / a.nrhs,
        "mg_iters": [s["iters"] for s in last], "mg_n_D": [s["n_D"] for s in last],
        "mg_n_Dc": [s["n_Dc"][1] for s in last], "true_res": true_res,
        "roofline": roofline, "kernels": kinfo, "dslash_in_step": dslash_step, "dc_mfma": dc_mfma,
        "wilson_tuning": wilson_tuning,
    }
    if a.precision_report:
        result["precision_error"] = precision_report(ctx, torch, synthetic, dims, a.nv)
    if not a.no_bicgstab:
        t0 = time.perf_counter()
        xb, sb = ctx.solve_bicgstab(b, tol=1e-10, maxit=100000)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        result["bicgstab"] = {"s_per_rhs": tb / a.nrhs, "iters": [s["iters"] for s in sb],
                              "n_D": [s["n_D"] for s in sb], "converged": all(s["converged"] for s in sb)}
    if a.big_L:
        result["dslash_out_of_cache"] = dslash_bandwidth(wdmg, synthetic, torch, dev, a.big_L)
    if not a.no_cpu_baseline:
        n_d = int(np.sum([s["n_D"] for s in last])) + a.nv * (a.setup_iters + 1)
        result["cpu_baseline"] = cpu_baseline(u, bh[0], m, n_d, a.nrhs, a.cpu_seconds)
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
