#!/usr/bin/env python
"""Benchmark of the adaptive-multigrid Wilson-Dirac solve on one MI355X.

One step = one pass of the whole hot path over one batch of right-hand sides:
the adaptive setup (MR relaxation of the Nv starting vectors on D v = 0,
FP64 block orthonormalisation, Galerkin coarse operator) followed by the
MG-preconditioned flexible GCR solve of every right-hand side to true
relative residual 1e-10 (FP64).  `value` is the step's wall time per
right-hand side, inputs resident in HBM before the timed region.

Default workload: the 24^3 x 48 lattice with links exp(i 0.45 H),
antiperiodic time, m = m_crit + 0.005 with m_crit of this very field,
32 Gaussian right-hand sides solved together: batched FP32 setup (Nv = 24,
200 MR steps, 4^4 aggregates; then Nv = 16 on 2^4 aggregates of the coarse
lattice, 25 steps), the Sec. 5 three-level cycle (four level-1 V-cycles per
fine cycle) with the fine level in BF16 storage and FP32 arithmetic
(coarse operators and P^dagger on matrix cores), FP64 coarsest GCR to 0.3
and FP64 outer flexible GCR(6) with an FP32 basis.

Beside the K timed steps, on the same GPU and field, the line carries the
two comparators of the target: FP64 single-rhs MG (FP64 setup and V-cycle,
FGCR(50)) and plain FP64 BiCGStab, each timed after a warm-up.  It also
carries the roofline of the step's dominant kernel (HIP events on the
library's stream during the timed steps), the Wilson operator's bandwidth
on a 32^4 lattice (larger than the 256 MB Infinity Cache), the coarse
operator's matrix-core utilisation, and the FP64 oracle's real MG solve of
the 8^4 workload timed on the host as `cpu_baseline`.
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
# Dense peaks of MI355X (TFLOP/s) by the dtype a kernel computes in.
PEAK_TFS = {"f64": 78.6, "f32": 157.3, "h": 2500.0}

# Algorithmic (compulsory) bytes of the Wilson operator per fine site with N
# right-hand sides per launch: the four links of a site (as 18 reals each) once
# per launch, psi in and out once per rhs.  One rhs: 960 / 480 / 248 B.
WILSON_LINK_BYTES = {"f64": 576, "f32": 288, "f16": 144, "bf16": 144}
WILSON_SPINOR_BYTES = {"f64": 384, "f32": 192, "f16": 104, "bf16": 104}
WILSON_FLOPS = 1368  # per fine site and rhs: 8 spin-projected hops and the mass term

# Wilson kernel form and rhs group pinned per (precision, rhs per launch) for
# the default workload, from the form sweep on this lattice (24^3 x 48: form 5
# fastest in FP32 at 24 and 32 rhs, form 2 in BF16 at 32 rhs); the FP32 setup
# runs 24-rhs launches and the outer solve 32-rhs ones.  Pinning keeps the
# step's kernels, and so the committed counter profile, the same from box to
# box; elsewhere (or with --autotune) the library's autotuner decides.
PINNED_TUNING = {((24, 24, 24, 48), 32): {("f32", 24): (5, 8), ("f32", 32): (5, 8), ("bf16", 32): (2, 2)}}
# Sources of each profiled kernel family (a committed counter profile is
# used only while these files are unchanged).
KERNEL_SOURCES = {
    "dslash": ["paper_0811_4331_amd/csrc/dslash.hip", "paper_0811_4331_amd/csrc/fine_field.h",
               "paper_0811_4331_amd/csrc/half_field.h", "paper_0811_4331_amd/csrc/wilson_spin.h",
               "paper_0811_4331_amd/csrc/common.h"],
}


def wilson_bytes(prec, vol, launches, units):
    """Algorithmic bytes of `launches` Wilson launches on `vol` sites that
    processed `units` (site, rhs) pairs in total: 576/N + 384 B per site and rhs
    in FP64 (288/N + 192 FP32, 144/N + 104 16-bit)."""
    return launches * vol * WILSON_LINK_BYTES[prec] + units * WILSON_SPINOR_BYTES[prec]


def coarse_bytes(store, n2, nsite, launches, units, vec_bytes):
    """Coarse operator: the 9 (2Nv)^2 blocks of every coarse site once per
    launch (`store` bytes per complex entry), the input and output vectors
    (`vec_bytes` per complex entry) once per (site, rhs)."""
    return launches * nsite * 9 * n2 * n2 * store + units * 2 * n2 * vec_bytes


def transfer_bytes(store, nv, vol, launches, units, fine_bytes, coarse_vec_bytes, n2):
    """P^dagger or P at the fine level: the Nv columns of P (12 complex per
    fine site each) once per launch, the fine vector once per (site, rhs) and
    the coarse vector's share (2Nv entries per 256 fine sites)."""
    return launches * vol * 12 * nv * store + units * (fine_bytes + n2 * coarse_vec_bytes / 256.0)


def kernel_model(name, launches, units, w):
    """(bytes, flops, dtype) of the profiled launches of one library kernel.
    `w` describes the workload: fine volume, Nv and 2Nv per level, coarse sites."""
    vol, nv, n2m, n2c = w["vol"], w["nv"], w["n2_mid"], w["n2_coarsest"]
    if name.startswith("dslash_"):
        p = name.split("_")[1]
        return wilson_bytes(p, vol, launches, units), WILSON_FLOPS * units, "f32" if p != "f64" else "f64"
    if name in ("restrict_f64", "prolong_f64"):
        return transfer_bytes(16, nv, vol, launches, units, 192, 16, 2 * nv), 96 * nv * units, "f64"
    if name in ("restrict_f32", "prolong_f32"):
        return transfer_bytes(8, nv, vol, launches, units, 96, 8, 2 * nv), 96 * nv * units, "f32"
    if name in ("restrict_h", "prolong_h"):
        return transfer_bytes(4, nv, vol, launches, units, 52, 8, 2 * nv), 96 * nv * units, "f32"
    fl_mid, fl_c = 72 * n2m * n2m * units, 72 * n2c * n2c * units
    if name in ("dc_f64", "dc_mfma_f64"):
        return coarse_bytes(16, n2m, w["nsite_mid"], launches, units, 16), fl_mid, "f64"
    if name in ("dc_f32", "dc_mfma_f32"):
        return coarse_bytes(8, n2m, w["nsite_mid"], launches, units, 8), fl_mid, "f32"
    if name == "dc_h":
        return coarse_bytes(4, n2m, w["nsite_mid"], launches, units, 8), fl_mid, "f32"
    if name == "dc_mfma_h":
        return coarse_bytes(4, n2m, w["nsite_mid"], launches, units, 8), fl_mid, "h"
    if name == "coarse_gcr":
        # the coarsest GCR's operator launch: FP64 D_c once, r read, w_j and z_j written
        return (launches * w["nsite_coarsest"] * 9 * n2c * n2c * 16 + units * 3 * n2c * 16), fl_c, "f64"
    return None


def roofline_of(name, k, w):
    """Roofline record of one profiled kernel: the bound follows from its
    arithmetic intensity against the ridge of its dtype."""
    m = kernel_model(name, k["launches"], k["units"], w)
    if m is None:
        return None
    nbytes, flops, dt = m
    sec = k["ms_total"] / 1e3
    ridge = PEAK_TFS[dt] * 1e12 / (HBM_PEAK_GBS * 1e9)
    per = k["launches"]
    rec = {"kernel": name, "us_per_launch": sec / per * 1e6, "launches": per,
           "bytes_per_launch": nbytes / per, "flops_per_launch": flops / per,
           "arithmetic_intensity": flops / nbytes, "dtype": dt}
    if flops / nbytes > ridge:
        ach = flops / sec / 1e12
        rec.update(bound="mfma", achieved=ach, peak=PEAK_TFS[dt], unit="TFLOP/s", frac=ach / PEAK_TFS[dt])
    else:
        ach = nbytes / sec / 1e9
        rec.update(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS)
    return rec


def dc_mfma_util(kinfo, w, nrhs):
    """Achieved FLOP/s of the coarse-operator launches that run on matrix cores,
    against the dense peak of their dtype (one (site, rhs) unit = 72 (2Nv)^2
    real flops).  The coarsest GCR's operator runs on FP64 matrix cores once
    nrhs > 1."""
    out = {}
    for name in ("dc_mfma_f64", "dc_mfma_f32", "dc_mfma_h", "coarse_gcr"):
        k = kinfo.get(name)
        if k is None or (name == "coarse_gcr" and nrhs < 2):
            continue
        _, flops, dt = kernel_model(name, k["launches"], k["units"], w)
        tfs = flops / (k["ms_total"] / 1e3) / 1e12
        out[name] = {"dtype": dt, "achieved_tflops": tfs, "peak_tflops": PEAK_TFS[dt], "util": tfs / PEAK_TFS[dt]}
    return out or None


def counter_traffic(kernel, workload, bytes_per_launch, tuning=None):
    """HBM bytes per launch from the committed PMC measurement of this kernel in
    this workload (FETCH_SIZE + WRITE_SIZE, scaled by what the same counters read
    for a plain copy), or None when there is none, the kernel's sources changed
    since, or this run's kernel forms (the entries of ``tuning`` the
    measurement names) differ from the ones the counters were taken with."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    for e in t["entries"].get(kernel + "@" + workload, []):
        h = hashlib.sha256()
        for f in e["source_files"]:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest()[:16] != e["source_hash"]:
            continue
        want = e.get("tuning")
        if isinstance(want, dict) and isinstance(tuning, dict):
            same = all(tuning.get(k) == v for k, v in want.items())
        else:
            same = want == tuning
        if same:
            return e["measured_over_algorithmic"] * bytes_per_launch
    return None


def parse(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dims", type=int, nargs=4, default=(24, 24, 24, 48), metavar=("LX", "LY", "LZ", "LT"))
    ap.add_argument("--eps", type=float, default=0.45)
    ap.add_argument("--delta", type=float, default=0.005, help="m - m_crit")
    ap.add_argument("--mcrit-estimate", action="store_true",
                    help="accept an unconverged m_crit estimate of tests/inputs/mcrit_gpu.json (labelled in the line)")
    ap.add_argument("--mass", type=float, default=None,
                    help="use this bare mass instead of m_crit + delta (no m_crit lookup)")
    ap.add_argument("--nv", type=int, default=24)
    ap.add_argument("--levels", type=int, default=None, choices=[2, 3],
                    help="3: a second coarsening with 2^4 aggregates (Sec. 5 three-level cycle); default 3 for "
                         "batches of 16 or more on lattices whose extents are multiples of 8, else 2")
    ap.add_argument("--nv2", type=int, default=16, help="near-null vectors of the second coarsening")
    ap.add_argument("--setup-iters2", type=int, default=25,
                    help="MR relaxation steps of the second coarsening's vectors")
    ap.add_argument("--setup-iters", type=int, default=None,
                    help="MR relaxation steps per near-null vector (default 50 for fewer than 8 rhs, "
                         "100 for 8 to 15 and 250 for 16 or more, whose setup cost is shared)")
    ap.add_argument("--adapt-iters", type=int, default=0,
                    help="adaptive augmentation (Sec. 2): two-level iterations refining each candidate "
                         "after the first (0: relaxation only)")
    ap.add_argument("--nrhs", type=int, default=32)
    ap.add_argument("--nullvec-source", default="host", choices=["host", "device"],
                    help="first-level null-vector starts: numpy on the host, kept on the device, or "
                         "torch's seeded device generator inside each step, released after the setup (large lattices)")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library's autotuner pick every Wilson form (default: the forms pinned for the "
                         "default workload)")
    ap.add_argument("--in-place", action="store_true",
                    help="solve in place (x written over b, no internal copy of b; the host copy of the rhs "
                         "refills b before every step, outside the timing): room for the largest batches")
    ap.add_argument("--release-unused", action="store_true",
                    help="after each setup, free the FP64/FP32 copies of P and D_c that the 16-bit V-cycle "
                         "does not read (room for larger batches)")
    ap.add_argument("--coarse-apply", type=int, default=None, choices=[0, 1],
                    help="force a form of the batched coarsest-level operator (default: library choice)")
    ap.add_argument("--setup-prec", default="f32", choices=["f64", "f32", "f16", "bf16"],
                    help="arithmetic (storage, for 16 bits) of the setup relaxation; the block QR is FP64 either way")
    ap.add_argument("--mg-prec", default="bf16", choices=["f64", "f32", "f16", "bf16"])
    ap.add_argument("--coarse-tol", type=float, default=None,
                    help="relative residual of the coarsest GCR (default 0.3 with 3 levels, 0.1 with 2)")
    ap.add_argument("--alpha", action="store_true",
                    help="take the minimal-residual step size after prolongation (off: alpha = 1, "
                         "which converges in far fewer outer iterations on these fields)")
    ap.add_argument("--restart", type=int, default=None,
                    help="FGCR restart length (paper: 50; default 50 for fewer than 8 rhs, 12 for 8 to 15 and "
                         "6 for 16 or more: with the FP32 basis a cycle ends at the reliable update anyway, and "
                         "a short basis saves Gram-Schmidt passes)")
    ap.add_argument("--outer", default="fgcr", choices=["fgcr", "bicgstab"],
                    help="outer Krylov method: flexible GCR (Sec. 5) or BiCGStab with the V-cycle as right "
                         "preconditioner (Sec. 4)")
    ap.add_argument("--precision-report", action="store_true",
                    help="relative error of every reduced-precision operator against its FP64 form")
    ap.add_argument("--graph", action="store_true",
                    help="capture the V-cycle in a HIP graph after its first application and replay it")
    ap.add_argument("--big-L", type=int, default=32, help="lattice for the out-of-cache Dslash figure (0: skip)")
    ap.add_argument("--no-bicgstab", action="store_true")
    ap.add_argument("--bicgstab-budget", type=float, default=60.0,
                    help="seconds the BiCGStab comparator may run; its iteration cap follows from the "
                         "measured time per iteration, and a capped run is reported as a lower bound")
    ap.add_argument("--no-fp64-mg", action="store_true", help="skip the FP64 single-rhs MG comparator")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="start with a plain 1 GiB device copy (the reference for hardware byte counters)")
    ap.add_argument("--only-dslash", type=int, default=0, metavar="L",
                    help="only time Dslash on L^4 plus a plain 1 GiB device copy, then exit")
    ap.add_argument("--qed2d", action="store_true",
                    help="the 2d U(1) comparison of Sec. 4 instead of the 4d step (128^2, beta 6)")
    ap.add_argument("--qed2d-deltas", type=float, nargs="+", default=[0.1, 0.03, 0.01, 0.003],
                    help="m - m_crit of the 2d masses")
    ap.add_argument("--qed2d-rhs", type=int, default=1, help="rhs per launch of the timed 2d Wilson launch")
    ap.add_argument("--qed2d-setup-iters", type=int, default=300, help="MR setup steps per coarsening (2d)")
    ap.add_argument("--traffic-entry", nargs=5, metavar=("FETCH_CSV", "WRITE_CSV", "BENCH_JSON", "KERNEL", "COMMAND"),
                    help="no GPU work: turn two rocprofv3 --pmc runs of this benchmark (FETCH_SIZE, then "
                         "WRITE_SIZE, each started with --copy-calibration) and the JSON line of the first into "
                         "KERNEL's entry of profiles/traffic.json (KERNEL: the headline run's dominant kernel)")
    a = ap.parse_args(argv)
    if a.levels is None:
        a.levels = 3 if a.nrhs >= 16 and all(d % 8 == 0 for d in a.dims) else 2
    if a.coarse_tol is None:
        a.coarse_tol = 0.3 if a.levels == 3 else 0.1
    if a.setup_iters is None:
        a.setup_iters = 50 if a.nrhs < 8 else (100 if a.nrhs < 16 else 200)
    if a.restart is None:
        a.restart = 50 if a.nrhs < 8 else (12 if a.nrhs < 16 else 6)
    return a


def load_mcrit(dims, eps, seed, allow_estimate=False):
    """m_crit of a field: the oracle's Arnoldi (tests/golden/mcrit.json) where the
    host could run it, else the GPU Krylov-Schur of tests/inputs/mcrit_gpu.json
    (library FP64 D validated against the oracle on that field); with
    ``allow_estimate`` an unconverged Krylov-Schur estimate too, labelled as
    such.  Returns (m_crit, source)."""
    e = None
    key = "x".join(str(d) for d in dims) + f"_eps{eps}_seed{seed}"
    gold = os.path.join(ROOT, "tests", "golden", "mcrit.json")
    with open(gold) as fh:
        data = json.load(fh)
    if key in data:
        return float(data[key]["m_crit"]), "oracle Arnoldi on this field"
    gpu = os.path.join(ROOT, "tests", "inputs", "mcrit_gpu.json")
    if os.path.exists(gpu):
        with open(gpu) as fh:
            data = json.load(fh)
        e = data.get(key)
        if e is not None and e.get("accepted"):
            return float(e["m_crit"]), (f"Krylov-Schur on this field with the library's FP64 D "
                                        f"(residual {e['leftmost_explicit_residual']:.1e})")
        if e is not None and allow_estimate:
            return float(e["m_crit"]), (f"ESTIMATE: leftmost Ritz value of an unconverged Krylov-Schur run on this "
                                        f"field (residual {e['leftmost_explicit_residual']:.1e}, still moving by "
                                        f"{e['leftmost_re_drift_last_10_cycles']:.0e} per 10 restarts)")
    raise SystemExit(f"no m_crit for {key}: run tests/golden/make_mcrit.py or tests/inputs/make_mcrit_gpu.py"
                     + (" (an unconverged estimate exists: --mcrit-estimate)" if e is not None else ""))


def workload_number(dims):
    """Seed family of a lattice: 8^4 -> 1, 16^4 -> 2, 32^4 -> 3, 24^3x48 -> 4, 48^3x96 -> 5."""
    return {(8, 8, 8, 8): 1, (16, 16, 16, 16): 2, (32, 32, 32, 32): 3, (24, 24, 24, 48): 4,
            (48, 48, 48, 96): 5}.get(tuple(dims), 9)


def timed_apply(ctx, x, prec, key, reps, sync):
    """(launches, units, ms) of `reps` library Wilson launches, HIP events."""
    ctx.apply_D(x, prec=prec)
    sync()
    ctx.profile(True)
    for _ in range(reps):
        ctx.apply_D(x, prec=prec)
    n, units, ms = ctx.profile_read()[key]
    ctx.profile(False)
    return n, units, ms


def dslash_bandwidth(wdmg, synthetic, torch, dev, L, reps=20):
    """Wilson operator on an L^4 lattice (links exp(i 0.45 H)): one rhs in every
    form and precision, and a batch of 8 rhs, by the N-rhs byte model."""
    dims = (L, L, L, L)
    vol = L ** 4
    u = synthetic.gauge_field(dims, 0.45, synthetic.gauge_seed(3, 2))
    ctx = wdmg.Context(dims, dev)
    ctx.set_gauge(torch.from_numpy(u).to(dev), t_bc=-1)
    del u
    ctx.set_mass(-1.0)
    psi = torch.from_numpy(synthetic.gaussian_spinor(dims, 5)).to(dev)
    sync = torch.cuda.synchronize
    out = {"lattice": f"{L}^4", "bytes_model": "576/N + 384 B per site and rhs (FP64), 288/N + 192 (FP32), "
                                                "144/N + 104 (16-bit + scale)"}
    precs = (("f64", "dslash_f64"), ("f32", "dslash_f32"), ("f16", "dslash_f16"), ("bf16", "dslash_bf16"))

    def rec(prec, n, units, ms, form, group=None):
        sec = ms / 1e3
        gbs = wilson_bytes(prec, vol, n, units) / sec / 1e9
        r = {"us_per_launch": sec / n * 1e6, "GB_s": gbs, "frac_hbm_peak": gbs / HBM_PEAK_GBS, "form": form}
        if group is not None:
            r["rhs_group"] = group
        return r

    forms = {}
    for form in (0, 1, 2):
        ctx.set_tuning("dslash", form)
        for prec, key in precs:
            x = psi if prec == "f64" else psi.to(torch.complex64)
            forms[f"{prec}_form{form}"] = rec(prec, *timed_apply(ctx, x, prec, key, reps, sync), form)
    ctx.set_tuning("dslash", None)
    out["forms"] = {"form0": "one thread per site", "form1": "one wave per direction",
                    "form2": "one wave per direction, registers capped for 4 waves per SIMD", **forms}
    for prec, key in precs:
        x = psi if prec == "f64" else psi.to(torch.complex64)
        out[prec] = rec(prec, *timed_apply(ctx, x, prec, key, reps, sync), ctx.get_tuning("dslash", prec, 1))
    xb = psi.unsqueeze(0).repeat(8, 1, 1, 1, 1, 1, 1)
    for prec, key in (("f64", "dslash_f64"), ("f32", "dslash_f32"), ("bf16", "dslash_bf16")):
        x = xb if prec == "f64" else xb.to(torch.complex64)
        n, units, ms = timed_apply(ctx, x, prec, key, max(2, reps // 4), sync)
        r = rec(prec, n, units, ms, ctx.get_tuning("dslash", prec, 8), ctx.get_tuning("dslash_group", prec, 8))
        r["ns_per_site_rhs"] = ms / 1e3 / units * 1e9
        out[prec + "_8rhs"] = r
    ctx.close()
    return out


def copy_calibration(torch, dev):
    """A plain 1 GiB device copy: the reference for FETCH_SIZE / WRITE_SIZE."""
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 3
    res = {"bytes_read": src.numel() * 8, "bytes_written": dst.numel() * 8,
           "GB_s_read_plus_write": 2 * src.numel() * 8 / dt / 1e9}
    del src, dst
    return res


def only_dslash(L, reps=10):
    import torch

    import synthetic
    from paper_0811_4331_amd import wdmg
    dev = torch.device("cuda:0")
    res = {"copy_1GiB": copy_calibration(torch, dev),
           "dslash": dslash_bandwidth(wdmg, synthetic, torch, dev, L, reps=reps)}
    print(json.dumps(res), flush=True)


# The 2d U(1) workload (Sec. 4): 128^2 lattice, compact U(1) links at beta = 6
# (seed 7000, the stored m_crit), right-hand side seed 7100, candidate seeds
# 7200 (fine) and 7201 (level 1).  Bytes of one FP64 2d Wilson application per
# site: spinor in and out (2 x 32 B) and the site's two links (32 B).
QED2D_BYTES_PER_SITE = 96
QED2D_FLOPS_PER_SITE = 8 * 18


def qed2d_bench(a):
    """Sec. 4 comparison on one GPU: for each mass m_crit + delta, CG, MG-CG and
    MG-BiCGstab to ||b - D x|| / ||b|| <= 1e-10; Wilson products, operator flops,
    setup and solve seconds; one JSON line."""
    import torch

    import synthetic
    from paper_0811_4331_amd import qed2d

    dev = torch.device("cuda:0")
    with open(os.path.join(ROOT, "tests", "golden", "mcrit_2d.json")) as fh:
        e = json.load(fh)["128x128_beta6.0_seed7000"]
    dims = tuple(e["dims"])
    lx, lt = dims
    u = torch.from_numpy(synthetic.u1_gauge_field(dims, e["beta"], e["gauge_seed"])).to(dev)
    b = torch.from_numpy(synthetic.gaussian_spinor_2d(dims, 7100)).to(dev)
    ctx = qed2d.Context2d(dims, dev)
    ctx.set_gauge(u, -1)
    configs = [  # (name, method, nvs, coarse cycles); the last one gives the line's value
        ("CG", "cg", None, 1),
        ("MG-CG Nv=8, V-cycle", "mg-cg", [8, 8], 1),
        ("MG-CG Nv=8, 4 level-1 cycles", "mg-cg", [8, 8], 4),
        ("MG-CG Nv=8/16, 4 level-1 cycles", "mg-cg", [8, 16], 4),
        ("MG-BiCGstab Nv=3, V-cycle", "mg-bicgstab", [3, 3], 1),
        ("MG-BiCGstab Nv=3, 4 level-1 cycles", "mg-bicgstab", [3, 3], 4),
        ("MG-BiCGstab Nv=8, V-cycle", "mg-bicgstab", [8, 8], 1),
        ("MG-BiCGstab Nv=8, 4 level-1 cycles", "mg-bicgstab", [8, 8], 4),
        ("MG-BiCGstab Nv=8/16, 4 level-1 cycles", "mg-bicgstab", [8, 16], 4),
    ]
    rows = []
    for delta in a.qed2d_deltas:
        m = e["m_crit"] + delta
        ctx.set_mass(m)
        for name, method, nvs, cyc in configs:
            setup_s = 0.0
            if nvs:
                vecs = [torch.from_numpy(synthetic.gaussian_vectors((nvs[0], lt, lx, 2, 1), 7200)).to(dev),
                        torch.from_numpy(synthetic.gaussian_vectors((nvs[1], lt // 4, lx // 4, 2, nvs[0]),
                                                                    7201)).to(dev)]
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.mg_setup(nvs, vecs, setup_iters=a.qed2d_setup_iters, normal=(method == "mg-cg"),
                             coarse_cycles=cyc)
                torch.cuda.synchronize()
                setup_s = time.perf_counter() - t0
            ctx.solve(b, method=method, tol=1e-10, maxit=50000)  # warm-up
            x, st = ctx.solve(b, method=method, tol=1e-10, maxit=50000)
            r = b - ctx.apply_D(x)
            res = float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b))
            rows.append({"delta": delta, "solver": name, "iters": st["iters"], "wilson": st["wilson"],
                         "operator_gflop": st["flops"] / 1e9, "setup_s": setup_s, "solve_s": st["seconds"],
                         "true_res": res, "converged": bool(st["converged"] and res <= 1e-10)})
            print(json.dumps({"progress": rows[-1]}), flush=True)
    # roofline of the level-1 stencil of the last hierarchy (MG-BiCGstab, 2Nv = 16, 5 offsets): it
    # reads its blocks once per application (HIP events on the context's stream)
    lt1, lx1, g1, n1 = ctx.levels[1]
    N1, S1 = g1 * n1, (9 if ctx.normal else 5)
    v1 = torch.from_numpy(synthetic.gaussian_vectors((lt1, lx1, g1, n1), 7300)).to(dev)
    ctx.apply_coarse(1, v1)
    st_reps = 500
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(st_reps):
        ctx.apply_coarse(1, v1)
    ev1.record()
    torch.cuda.synchronize()
    st_us = ev0.elapsed_time(ev1) * 1e3 / st_reps
    st_bytes = (S1 * N1 * N1 + 2 * N1) * lx1 * lt1 * 16
    st_gbs = st_bytes / (st_us * 1e-6) / 1e9
    # the 2d Wilson launch on its own (HIP events on the context's stream)
    reps = 2000
    bb = b.reshape(1, lt, lx, 2).repeat(a.qed2d_rhs, 1, 1, 1).contiguous()
    ctx.apply_D(bb)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        ctx.apply_D(bb)
    ev1.record()
    torch.cuda.synchronize()
    us = ev0.elapsed_time(ev1) * 1e3 / reps
    site_rhs = lx * lt * a.qed2d_rhs
    gbs = (lx * lt * 32 + site_rhs * 64) / (us * 1e-6) / 1e9
    ctx.close()
    best = next(r for r in rows if r["delta"] == min(a.qed2d_deltas) and r["solver"] == configs[-1][0])
    cg = next(r for r in rows if r["delta"] == best["delta"] and r["solver"] == "CG")
    line = {"metric": "2d U(1) time-to-solution @ rel.res 1e-10 (s/RHS, setup included); Wilson products",
            "value": best["setup_s"] + best["solve_s"], "unit": "s/RHS", "n_gpus": 1, "steps": 1, "warmup": 1,
            "ms_per_step": 1e3 * (best["setup_s"] + best["solve_s"]), "higher_is_better": False, "scaling": "strong",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"2d U(1) {lx}x{lt}, beta {e['beta']}, m = m_crit + {best['delta']}",
                       "solver": best["solver"], "m_crit": e["m_crit"], "setup_iters": a.qed2d_setup_iters},
            "wilson_products": {"mg": best["wilson"], "cg": cg["wilson"], "ratio": cg["wilson"] / best["wilson"]},
            "cg_s": cg["solve_s"],
            "wilson_launch": {"rhs": a.qed2d_rhs, "us": us, "GB_s": gbs, "frac_hbm_peak": gbs / HBM_PEAK_GBS,
                              "bytes_model": "links 32 B per site once, spinor in and out 64 B per site and rhs"},
            "roofline": {"kernel": f"k_stencil_w<{N1}> (level-1 stencil, {S1} offsets)", "bound": "hbm",
                         "achieved": st_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": st_gbs / HBM_PEAK_GBS,
                         "traffic": None, "us_per_launch": st_us, "bytes_per_launch": st_bytes,
                         "bytes_model": "S (2Nv)^2 block entries and two coarse vectors per coarse site, 16 B each"},
            "rows": rows}
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = qed2d_cpu_baseline(e, 0.01, a.qed2d_setup_iters)
    print(json.dumps(line), flush=True)


def qed2d_cpu_baseline(e, delta, setup_iters):
    """The oracle's MG-BiCGstab (Nv 8 then 16, four level-1 cycles, the
    benchmark's MR setup steps) on the same 128^2 field at m_crit + delta, setup
    and solve, timed on the host."""
    import torch

    import synthetic
    from oracle import qed2d as O
    dims = tuple(e["dims"])
    u = synthetic.u1_gauge_field(dims, e["beta"], e["gauge_seed"])
    b = synthetic.gaussian_spinor_2d(dims, 7100)
    m = e["m_crit"] + delta
    t0 = time.perf_counter()
    h = O.build(u, m, -1.0, nvs=[8, 16], block=(4, 4), setup_iters=setup_iters, seeds=[7200, 7201],
                coarse_cycles=[4, 1])
    t1 = time.perf_counter()
    _, info = O.mg_bicgstab(h, b, 1e-10)
    t2 = time.perf_counter()
    return {"value": t2 - t0, "unit": "s/RHS", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"one rhs at m_crit + {delta}, setup {t1 - t0:.1f} s and solve {t2 - t1:.1f} s, "
                      f"{info['iters']} iterations, {O.wilson_products(h)} Wilson products"}


def precision_report(ctx, torch, synthetic, dims):
    """||A_prec v - A_f64 v|| / ||A_f64 v|| for D (level 0), P^dagger, P and D_c
    (level 1) on Gaussian vectors, per reduced precision.  The FP64 forms are
    those the parity tests pin to the oracle."""
    def rel(a, b):
        return float(torch.linalg.vector_norm(a.to(torch.complex128) - b) / torch.linalg.vector_norm(b))
    dev = ctx.device
    f = torch.from_numpy(synthetic.gaussian_spinor(dims, 777)).to(dev)
    c = torch.from_numpy(synthetic.gaussian_vectors(ctx.coarse_shape(1), 778)).to(dev)
    ref = {"D": ctx.apply_D(f), "P_dagger": ctx.restrict(0, f), "P": ctx.prolong(0, c), "D_c": ctx.apply_Dc(1, c)}
    out = {}
    for prec in ("f32", "f16", "bf16"):
        f32, c32 = f.to(torch.complex64), c.to(torch.complex64)
        out[prec] = {"level0_D": rel(ctx.apply_D(f32, prec=prec), ref["D"]),
                     "level0_P_dagger": rel(ctx.restrict(0, f32, prec=prec), ref["P_dagger"]),
                     "level0_P": rel(ctx.prolong(0, c32, prec=prec), ref["P"]),
                     "level1_D_c": rel(ctx.apply_Dc(1, c32, prec=prec), ref["D_c"])}
    return out


def progress(msg):
    """Progress of the long comparator runs (stderr; stdout carries the one JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bicgstab_comparator(ctx, b1, budget_s, torch):
    """Plain FP64 BiCGStab on one rhs after a short warm-up (20 iterations); the
    iteration cap is the time budget over the warm-up's time per iteration.  A
    run stopped by the cap is a lower bound (converged false)."""
    t0 = time.perf_counter()
    ctx.solve_bicgstab(b1, tol=1e-10, maxit=20)
    torch.cuda.synchronize()
    t_it = (time.perf_counter() - t0) / 20
    maxit = max(50, int(budget_s / t_it))
    progress(f"BiCGStab comparator: {t_it * 1e3:.2f} ms per iteration, at most {maxit} iterations")
    t0 = time.perf_counter()
    _, sb = ctx.solve_bicgstab(b1, tol=1e-10, maxit=maxit)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    conv = all(s["converged"] for s in sb)
    return {"s_per_rhs": dt, "iters": [s["iters"] for s in sb], "n_D": [s["n_D"] for s in sb],
            "converged": conv, "true_res": [s["true_res"] for s in sb], "maxit": maxit,
            "lower_bound": not conv, "what": "unpreconditioned FP64 BiCGStab, one rhs, same field and mass"}


def fp64_mg_comparator(ctx, b1, a, v0, torch):
    """FP64 single-rhs MG on the same field: FP64 setup (l = 50 MR steps, the
    single-rhs default) and V-cycle, 2 levels (4^4 aggregates, coarsest GCR to
    0.1; faster for one rhs than the batch's 3-level shape: 1.43 against
    1.58 s on the default workload), FGCR(50); one untimed run, then one
    timed."""
    levels = [{"block": (4, 4, 4, 4), "nv": a.nv, "setup_iters": 50, "vectors": v0, "setup_prec": "f64"}]

    def once():
        t0 = time.perf_counter()
        ctx.mg_setup(levels, coarse_tol=0.1, use_alpha=a.alpha)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, st = ctx.solve(b1, tol=1e-10, restart=50, maxit=3000, mg_prec="f64")
        torch.cuda.synchronize()
        return t1 - t0, time.perf_counter() - t1, st
    progress("FP64 single-rhs MG comparator")
    once()
    ts, tv, st = once()
    return {"s_per_rhs": ts + tv, "setup_s": ts, "solve_s": tv, "iters": [s["iters"] for s in st],
            "n_D": [s["n_D"] for s in st], "converged": all(s["converged"] for s in st),
            "true_res": [s["true_res"] for s in st],
            "what": f"FP64 setup (l = 50) and V-cycle, 2 levels, Nv = {a.nv}, FGCR(50), one rhs"}


def cpu_baseline_oracle(torch, dev, wdmg, synthetic):
    """The FP64 oracle's real MG-FGCR solve of the 8^4 workload (eps 0.3,
    m = m_crit + 0.05, 4^4 aggregates, Nv = 12, 50 MR setup steps, FGCR(50) to
    1e-10), setup + solve, timed on the host; the GPU's time for the same
    problem and inputs is reported beside it."""
    from oracle import mg, transfer
    from threadpoolctl import threadpool_info
    dims = (8, 8, 8, 8)
    seed = synthetic.gauge_seed(1, 1)
    m = load_mcrit(dims, 0.3, seed)[0] + 0.05
    u = synthetic.gauge_field(dims, 0.3, seed)
    bh = synthetic.gaussian_spinor(dims, synthetic.rhs_seed(1))
    t0 = time.perf_counter()
    h = mg.build_hierarchy(u, m, -1.0, [(4, 4, 4, 4)], [12], seeds=[synthetic.null_seed(1)], setup_iters=50,
                           coarse_tol=0.1, use_alpha=False)
    _, info = h.solve(transfer.as_chiral(bh), tol=1e-10, restart=50)
    t_cpu = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    # the same problem on the GPU (warm-up, then timed)
    ctx = wdmg.Context(dims, dev)
    ctx.set_gauge(torch.from_numpy(u).to(dev), t_bc=-1)
    ctx.set_mass(m)
    v0 = torch.from_numpy(synthetic.gaussian_vectors((12,) + ctx.fine_shape(), synthetic.null_seed(1))).to(dev)
    b = torch.from_numpy(bh).to(dev)
    lv = [{"block": (4, 4, 4, 4), "nv": 12, "setup_iters": 50, "vectors": v0}]
    for _ in range(2):
        t0 = time.perf_counter()
        ctx.mg_setup(lv, coarse_tol=0.1, use_alpha=False)
        _, st = ctx.solve(b, tol=1e-10, restart=50, maxit=1000)
        torch.cuda.synchronize()
        t_gpu = time.perf_counter() - t0
    ctx.close()
    return {"value": t_cpu, "unit": "s/RHS", "cores": threads, "kind": "oracle",
            "sample": ("the oracle's full MG solve (numpy FP64: 50-step relaxation of 12 null vectors, block QR, "
                       "Galerkin stencil, FGCR(50) with V(2,2) cycles to true residual 1e-10) of the 8^4 "
                       "workload, one rhs, timed once; element-wise numpy runs on one core, BLAS calls "
                       f"on up to {threads} threads.  The headline lattice is beyond the oracle's reach "
                       "(one numpy Wilson apply there takes seconds); its oracle time is not extrapolated."),
            "oracle_iters": info["iters"], "oracle_true_res": info["true_res"],
            "gpu_same_sample_s_per_rhs": t_gpu, "gpu_same_sample_iters": st[0]["iters"],
            "host_cpus": os.cpu_count()}


def kernel_family_names(kernel):
    """Substrings of the HIP kernel names (demangled or mangled) of one profiled kernel id."""
    fam, prec = kernel.split("_", 1)
    io = {"f64": ["FullIO<double>", "FullIOIdE"], "f32": ["FullIO<float>", "FullIOIfE"],
          "f16": ["HalfIO<_Float16>", "HalfIOIDF16_E"], "bf16": ["HalfIO<__bf16>", "HalfIOIDF16bE"]}[prec]
    return ["k_dslash"], io


def traffic_entry(fetch_csv, write_csv, bench_json, kernel, command):
    """Entry of profiles/traffic.json for one profiled kernel of a bench run:
    its FETCH_SIZE and WRITE_SIZE per launch (KiB per dispatch in the CSVs,
    scaled by the counters' reading of the run's 1 GiB copy) over the
    algorithmic bytes per launch of the same run."""
    import csv
    import hashlib
    with open(bench_json) as fh:
        line = [json.loads(x) for x in fh if x.startswith("{")][-1]
    roof = line["rooflines"][kernel]
    if not kernel.startswith("dslash_"):
        raise SystemExit(f"no counter mapping for {kernel}")
    must, io = kernel_family_names(kernel)

    def per_dispatch(path, counter):
        vals, copy = {}, []
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                name, v = r["Kernel_Name"], float(r["Counter_Value"])
                if "copyBuffer" in name:
                    copy.append(v)
                elif all(m in name for m in must) and any(t in name for t in io):
                    vals[r["Dispatch_Id"]] = v  # repeated rows of one dispatch carry one value
        return list(vals.values()), max(copy)

    fetch, fcopy = per_dispatch(fetch_csv, "FETCH_SIZE")
    write, wcopy = per_dispatch(write_csv, "WRITE_SIZE")
    if len(fetch) != roof["launches"] or len(write) != roof["launches"]:
        raise SystemExit(f"{len(fetch)} / {len(write)} profiled dispatches, {roof['launches']} launches in the line")
    gib_kib = float(1 << 20)  # the 1 GiB copy read and written, in KiB
    f_scale, w_scale = gib_kib / fcopy, gib_kib / wcopy
    alg = roof["bytes_per_launch"]
    fb = np.mean(fetch) * 1024 * f_scale / alg
    wb = np.mean(write) * 1024 * w_scale / alg
    fam = kernel.split("_")[0]
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[fam]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    prec = kernel.split("_", 1)[1]
    tuning = {k: v for k, v in line["tuning"].items() if k.startswith(prec + "x")}
    wl = "x".join(map(str, line["config"]["lattice"])) + f"_{line['config']['nrhs']}rhs_{line['config']['mg_prec']}"
    entry = {"tuning": tuning, "measured_over_algorithmic": fb + wb, "fetch_bytes_over_alg": fb,
             "write_bytes_over_alg": wb, "launches": roof["launches"], "alg_bytes_per_launch": alg,
             "fetch_kib_per_dispatch": float(np.mean(fetch)), "write_kib_per_dispatch": float(np.mean(write)),
             "copy_scale": {"FETCH_SIZE": f_scale, "WRITE_SIZE": w_scale},
             "source_files": KERNEL_SOURCES[fam], "source_hash": h.hexdigest()[:16], "command": command}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path) as fh:
        t = json.load(fh)
    t["entries"][f"{kernel}@{wl}"] = [entry]
    with open(path, "w") as fh:
        json.dump(t, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(json.dumps({f"{kernel}@{wl}": entry}))


def main(argv=None):
    a = parse(argv)
    if a.traffic_entry:
        traffic_entry(*a.traffic_entry)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (every path here is single-GPU); "
                                   "--gpus must be 1", "n_gpus": a.gpus}), flush=True)
        sys.exit(2)
    if a.only_dslash:
        only_dslash(a.only_dslash)
        return
    if a.qed2d:
        qed2d_bench(a)
        return
    import torch

    import synthetic
    from paper_0811_4331_amd import wdmg

    dev = torch.device("cuda:0")
    calib = copy_calibration(torch, dev) if a.copy_calibration else None
    dims = tuple(a.dims)
    vol = int(np.prod(dims))
    i_eps = {0.2: 0, 0.3: 1, 0.45: 2}.get(a.eps, 9)
    cfg = workload_number(dims)
    gseed = synthetic.gauge_seed(cfg, i_eps)
    if a.mass is not None:
        m, mc, mcrit_src = a.mass, float("nan"), "bare mass given"
        a.delta = float("nan")
    else:
        mc, mcrit_src = load_mcrit(dims, a.eps, gseed, a.mcrit_estimate)
        m = mc + a.delta
    u = synthetic.gauge_field(dims, a.eps, gseed)
    ctx = wdmg.Context(dims, dev)
    ctx.set_gauge(torch.from_numpy(u).to(dev), t_bc=-1)
    del u
    ctx.set_mass(m)
    ctx.set_tuning("coarse_apply", a.coarse_apply)
    pinned = {} if a.autotune else PINNED_TUNING.get((dims, a.nrhs), {})
    for (prec, n), (form, group) in pinned.items():
        ctx.set_tuning_for("dslash", prec, n, form)
        ctx.set_tuning_for("dslash_group", prec, n, group)
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
    if not a.in_place:
        del bh  # with --in-place the host copy refills b before every step, outside the timing
    levels = [{"block": (4, 4, 4, 4), "nv": a.nv, "setup_iters": a.setup_iters, "adapt_iters": a.adapt_iters,
               "vectors": v0, "setup_prec": a.setup_prec}]
    if a.levels == 3:
        cdims = tuple(d // 4 for d in dims)
        v1 = torch.from_numpy(synthetic.gaussian_vectors(
            (a.nv2, cdims[3], cdims[2], cdims[1], cdims[0], 2, a.nv), synthetic.null_seed(cfg) + 500)).to(dev)
        levels.append({"block": (2, 2, 2, 2), "nv": a.nv2, "vectors": v1, "setup_iters": a.setup_iters2,
                       "setup_prec": a.setup_prec if a.setup_prec in ("f64", "f32") else "f32"})
    def step():
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
        x, st = ctx.solve(b, tol=1e-10, restart=a.restart, maxit=3000, mg_prec=a.mg_prec, graph=a.graph,
                          outer=a.outer, in_place=a.in_place)
        torch.cuda.synchronize()
        return x, st, t1 - t0, time.perf_counter() - t1

    def refill():
        """In place, the previous step left its solution in b: restore the rhs (untimed)."""
        if a.in_place:
            b.copy_(torch.from_numpy(bh))
            torch.cuda.synchronize()

    for i in range(a.warmup):
        refill()
        step()
        progress(f"warm-up step {i + 1}/{a.warmup} done")
    torch.cuda.synchronize()
    ctx.profile(True)
    elapsed = 0.0
    setups, solves, stats = [], [], []
    for _ in range(a.steps):
        refill()
        t_step = time.perf_counter()
        x, st, ts, tv = step()
        elapsed += time.perf_counter() - t_step
        setups.append(ts)
        solves.append(tv)
        stats.append(st)
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    progress(f"{a.steps} timed steps done in {elapsed:.1f} s")
    one = "f64" if a.mg_prec == "f64" else "f32"
    field_b = {"f64": 2 * 12 * 16, "f32": 2 * 12 * 8, "f16": 3 * 52, "bf16": 3 * 52}[a.setup_prec]
    setup_batch = max(1, min(a.nv, 64, (16 << 30) // (vol * field_b)))  # the library's 16 GB relaxation budget
    vprec = a.mg_prec if a.mg_prec in ("f16", "bf16") else one
    # Wilson form and rhs group of every (precision, rhs per launch) the step runs
    tuning = {f"{p}x{n}": [ctx.get_tuning("dslash", p, n), ctx.get_tuning("dslash_group", p, n)]
              for p, n in ((a.setup_prec, setup_batch), (one, a.nrhs), (vprec, a.nrhs), ("f64", a.nrhs))}
    tuning["coarse_apply"] = ctx.get_tuning("coarse_apply", "f64", a.nrhs)
    tuning["pinned"] = bool(pinned)
    last = stats[-1]
    if not all(s["converged"] and s["true_res"] <= 1e-10 for st in stats for s in st):
        raise SystemExit(f"solve did not reach 1e-10: {last}")
    # independent check of the final residual with the library's FP64 D, one
    # rhs at a time (a batch-sized temporary may not fit beside the solver's memory)
    rr = bb = 0.0
    for j in range(a.nrhs):
        bj = torch.from_numpy(bh[j]).to(dev) if a.in_place else b[j]
        rj = bj - ctx.apply_D(x[j])
        rr += float(torch.linalg.vector_norm(rj)) ** 2
        bb += float(torch.linalg.vector_norm(bj)) ** 2
        del rj, bj
    true_res = (rr / bb) ** 0.5
    del x

    ms_per_step = elapsed / a.steps * 1e3
    value = elapsed / a.steps / a.nrhs
    n2_mid = 2 * a.nv
    n2_c = 2 * a.nv2 if a.levels == 3 else 2 * a.nv
    w = {"vol": vol, "nv": a.nv, "n2_mid": n2_mid, "n2_coarsest": n2_c, "nsite_mid": vol // 256,
         "nsite_coarsest": vol // 256 if a.levels == 2 else vol // 4096}
    kinfo = {name: {"launches": n, "ms_total": ms, "us_per_launch": ms / n * 1e3, "units": units}
             for name, (n, units, ms) in prof.items() if n}
    roofs = {k: roofline_of(k, kinfo[k], w) for k in kinfo}
    roofs = {k: r for k, r in roofs.items() if r is not None}
    step_ms = sum(k["ms_total"] for k in kinfo.values())
    dom = max(roofs, key=lambda k: kinfo[k]["ms_total"]) if roofs else None
    roofline = None
    if dom is not None:
        r = roofs[dom]
        wl = "x".join(map(str, dims)) + f"_{a.nrhs}rhs_{a.mg_prec}"
        traffic = counter_traffic(dom, wl, r["bytes_per_launch"], tuning)
        roofline = {"kernel": dom, "bound": r["bound"], "achieved": r["achieved"], "peak": r["peak"],
                    "unit": r["unit"], "frac": r["frac"], "traffic": traffic,
                    "bytes_per_launch": r["bytes_per_launch"], "flops_per_launch": r["flops_per_launch"],
                    "us_per_launch": r["us_per_launch"], "launches": r["launches"],
                    "share_of_profiled_time": kinfo[dom]["ms_total"] / step_ms}
    result = {
        "metric": METRIC, "value": value, "unit": "s/RHS", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_per_step, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if a.mg_prec == "f64" else f"f64 outer / {a.mg_prec} V-cycle",
        "data": "synthetic",
        "config": {"workload": f"{'x'.join(map(str, dims))} Wilson-Dirac, links exp(i {a.eps} H), "
                               f"m = m_crit + {a.delta}, "
                               + (f"2-level MG 4^4 aggregates Nv={a.nv}, " if a.levels == 2 else
                                  f"3-level MG 4^4 then 2^4 aggregates Nv={a.nv} then {a.nv2} "
                                  f"({a.setup_iters2} MR setup iters), ")
                               + f"{a.setup_prec} MR setup {a.setup_iters} iters, {a.mg_prec} V-cycle, "
                               + (f"adaptive {a.adapt_iters} two-level iters per candidate, " if a.adapt_iters else "")
                               + (f"FGCR({a.restart})" if a.outer == "fgcr" else "MG-BiCGStab")
                               + f" to 1e-10, {a.nrhs} Gaussian RHS solved together",
                   "lattice": list(dims), "eps": a.eps, "m": m, "m_crit": mc,
                   "m_crit_source": mcrit_src, "levels": a.levels, "nv": a.nv,
                   "nv2": a.nv2 if a.levels == 3 else None,
                   "nrhs": a.nrhs, "mg_prec": a.mg_prec, "setup_prec": a.setup_prec, "coarse_tol": a.coarse_tol,
                   "setup_iters": a.setup_iters, "adapt_iters": a.adapt_iters, "outer": a.outer,
                   "restart": a.restart, "alpha_step": a.alpha, "graph": a.graph,
                   "nullvec_source": a.nullvec_source, "release_unused": a.release_unused,
                   "in_place": a.in_place},
        "setup_s": float(np.median(setups)), "solve_s_per_rhs": float(np.median(solves)) / a.nrhs,
        "mg_iters": [s["iters"] for s in last], "mg_n_D": [s["n_D"] for s in last],
        "mg_n_Dc": [s["n_Dc"][1] for s in last], "true_res": true_res,
        "device_memory_peak_gb": torch.cuda.max_memory_allocated() / 1e9,
        "roofline": roofline, "rooflines": roofs, "kernels": kinfo, "dc_mfma": dc_mfma_util(kinfo, w, a.nrhs),
        "tuning": tuning,
    }
    if calib is not None:
        result["copy_calibration"] = calib
    if a.precision_report:
        result["precision_error"] = precision_report(ctx, torch, synthetic, dims)
    comps = {}

    def b1():
        """The first right-hand side (in place, b now holds the solution)."""
        return torch.from_numpy(bh[0]).to(dev) if a.in_place else b[0].contiguous()
    if not a.no_fp64_mg:
        v64 = v0 if v0 is not None else device_v0()
        comps["fp64_single_rhs_mg"] = fp64_mg_comparator(ctx, b1(), a, v64, torch)
        del v64
    if not a.no_bicgstab:
        comps["bicgstab"] = bicgstab_comparator(ctx, b1(), a.bicgstab_budget, torch)
    if comps:
        for c in comps.values():
            c["ratio_to_value"] = c["s_per_rhs"] / value
        result["comparators"] = comps
    ctx.close()
    del ctx, b, v0
    torch.cuda.empty_cache()
    if a.big_L:
        progress(f"Wilson operator bandwidth on {a.big_L}^4")
        result["dslash_out_of_cache"] = dslash_bandwidth(wdmg, synthetic, torch, dev, a.big_L)
    if not a.no_cpu_baseline:
        progress("oracle MG solve of the 8^4 workload on the host")
        result["cpu_baseline"] = cpu_baseline_oracle(torch, dev, wdmg, synthetic)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
