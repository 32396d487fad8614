"""Critical masses of the large synthetic fields, computed with the GPU's FP64 Wilson operator.

``m_crit = -min Re lambda(D_0)``, with ``D_0`` the Wilson operator at m = 0
(Sec. 1: D turns singular as the smallest real part of its spectrum reaches
zero; Sec. 5 quotes the critical mass of its ensemble).  The host Arnoldi of
``oracle.mcrit`` takes over an hour at 16^4 and is out of reach at 32^4,
24^3x48 and 48^3x96.  There the leftmost eigenvalues are found by a
Krylov-Schur iteration (G. W. Stewart, SIAM J. Matrix Anal. Appl. 23 (2001)
601) whose matrix-vector product is the library's FP64 ``apply_D`` at m = 0
and whose Krylov basis lives on the GPU (torch complex128, classical
Gram-Schmidt with one reorthogonalisation).  This is an input generator: the
masses it writes define the workloads; no parity value comes from it.

Checks made in the same run, recorded with each entry:

* the library's FP64 operator on that exact field equals the oracle's
  (``oracle.wilson.apply_D_at``, term by term) at sampled sites to 1e-13;
* the eigensolver reproduces the oracle's ARPACK critical masses of the 8^4
  and 16^4 fields in ``tests/golden/mcrit.json`` (``--validate``);
* the accepted leftmost Ritz pair has an explicit residual
  ``||D_0 v - theta v|| / ||v||`` below ``--accept``, recomputed with a fresh
  application of the operator, and the ``--nev`` leftmost Ritz values are
  converged, so a pair further left would have to be absent from a Krylov
  space that already resolved its neighbours.

usage: python tests/inputs/make_mcrit_gpu.py [--validate] [--field LX LY LZ LT EPS CFG I_EPS] ...
Writes tests/inputs/mcrit_gpu.json (merged by key).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import scipy.linalg

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mcrit_gpu.json")
GOLDEN = os.path.join(ROOT, "tests", "golden", "mcrit.json")


def basis_combine(Vj, c, chunk=1 << 24):
    """``Vj^T c`` (the combination sum_i c_i Vj[i]) for a basis Vj [k, n],
    accumulated over chunks of n with elementwise products and sums."""
    import torch
    k, n = Vj.shape
    out = torch.empty(n, dtype=Vj.dtype, device=Vj.device)
    cc = c.view(k, 1)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        out[lo:hi] = (cc * Vj[:, lo:hi]).sum(dim=0)
    return out


def basis_dots(Vj, w, chunk=1 << 24):
    """``Vj^H w`` for a basis Vj [k, n], accumulated over chunks of n with
    elementwise products and row sums (a matrix-vector product with so few
    rows and so many columns leaves most of the device idle)."""
    import torch
    k, n = Vj.shape
    c = torch.zeros(k, dtype=Vj.dtype, device=Vj.device)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        c += (Vj[:, lo:hi].conj() * w[lo:hi].unsqueeze(0)).sum(dim=1)
    return c


def krylov_schur_leftmost(matvec, n, dev, m, p, nev, tol, max_cycles, seed, log, time_limit):
    """Leftmost eigenvalues of a linear map on C^n by Krylov-Schur.

    The basis V (m + 1 vectors) and the Rayleigh quotient H ((m + 1) x m)
    satisfy ``A V[:m] = V[:m+1] H``.  After each expansion to m vectors, the
    complex Schur form of H[:m] is reordered so that the ``p`` eigenvalues
    of smallest real part lead; the basis is rotated and truncated to them
    plus the residual vector, and expansion resumes.  Converged when the
    ``nev`` leftmost Ritz pairs have residual ``|b^T Q y| <= tol`` (b the
    last row of H).  Returns (ritz values, residual estimates, V, Q-rotated
    eigenvector coefficients, matvec count, cycles)."""
    import torch
    V = torch.empty((m + 1, n), dtype=torch.complex128, device=dev)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    V[0] = torch.randn(n, dtype=torch.complex128, device=dev, generator=g)
    V[0] /= torch.linalg.vector_norm(V[0])
    k = 0
    nmv = 0
    tstart = time.time()
    history = []
    t_mv = t_orth = 0.0
    for cycle in range(1, max_cycles + 1):
        for j in range(k, m):
            t0 = time.time()
            w = matvec(V[j])
            torch.cuda.synchronize(dev) if dev.type == "cuda" else None
            t_mv += time.time() - t0
            nmv += 1
            h = np.zeros(j + 1, dtype=np.complex128)
            before = float(torch.linalg.vector_norm(w))
            for _ in range(2):
                t0 = time.time()
                c = basis_dots(V[: j + 1], w)
                w -= basis_combine(V[: j + 1], c)
                torch.cuda.synchronize(dev) if dev.type == "cuda" else None
                t_orth += time.time() - t0
                h += c.cpu().numpy()
                beta = float(torch.linalg.vector_norm(w))
                # second pass only when the first removed most of w
                # (Daniel-Gragg-Kaufman-Stewart criterion)
                if beta > 0.7071 * before:
                    break
                before = beta
            H[: j + 1, j] = h
            H[j + 1, j] = beta
            V[j + 1] = w / beta
            del w
        hm = H[:m, :m]
        ev = np.linalg.eigvals(hm)
        order = np.sort(ev.real)
        thr = 0.5 * (order[p - 1] + order[p])
        T, Q, sdim = scipy.linalg.schur(hm, output="complex", sort=lambda z: z.real <= thr)
        s = int(sdim)
        if s < nev or s >= m:
            s = max(nev, min(s, m - 1))
        b = H[m, :m] @ Q  # residual row in the Schur basis
        theta, Y = np.linalg.eig(T[:s, :s])
        Y /= np.linalg.norm(Y, axis=0)
        res = np.abs(b[:s] @ Y)
        idx = np.argsort(theta.real)
        theta, res, Y = theta[idx], res[idx], Y[:, idx]
        history.append(float(theta[0].real))
        log(f"cycle {cycle}: matvecs {nmv}, leftmost {theta[0].real:.10f}{theta[0].imag:+.6f}i "
            f"res {res[0]:.2e}, {nev}th res {res[nev - 1]:.2e}, {time.time() - tstart:.0f}s "
            f"(operator {t_mv:.0f}s, orthogonalisation {t_orth:.0f}s)")
        done = bool(np.all(res[:nev] <= tol))
        if done or cycle == max_cycles or time.time() - tstart > time_limit:
            return theta, res, V, Q[:, :s] @ Y, nmv, cycle, done, history
        # truncate to the s leading Schur vectors plus the residual vector
        Qs = torch.from_numpy(np.ascontiguousarray(Q[:, :s].T)).to(dev)  # [s, m]
        rot = Qs @ V[:m]
        V[:s] = rot
        del rot
        V[s] = V[m]
        Hn = np.zeros_like(H)
        Hn[:s, :s] = T[:s, :s]
        Hn[s, :s] = b[:s]
        H = Hn
        k = s
    raise AssertionError("unreachable")


def gpu_context(dims, eps, seed, dev):
    import torch

    import synthetic
    from paper_0811_4331_amd import wdmg
    u = synthetic.gauge_field(dims, eps, seed)
    ctx = wdmg.Context(dims, dev)
    ctx.set_gauge(torch.from_numpy(u).to(dev), t_bc=-1)
    ctx.set_mass(0.0)
    return ctx, u


def check_apply(ctx, u, dims, seed, dev):
    """Library FP64 D(m = 0) against the oracle's term-by-term form at sampled sites."""
    import torch

    import synthetic
    from oracle import wilson
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(seed)
    sites = [(0, 0, 0, 0), (lx - 1, ly - 1, lz - 1, lt - 1), (0, 0, 0, lt - 1), (lx - 1, 0, 0, 0)]
    sites += [tuple(int(rng.integers(0, e)) for e in dims) for _ in range(24)]
    psi = synthetic.gaussian_spinor(dims, seed=seed + 7)
    idx = tuple(np.array(c) for c in zip(*[(t, z, y, x) for (x, y, z, t) in sites]))
    out = ctx.apply_D(torch.from_numpy(psi).to(dev)).cpu().numpy()[idx]
    ref = wilson.apply_D_at(u, psi, 0.0, sites, -1.0)
    return float(np.linalg.norm(out - ref) / np.linalg.norm(ref))


def run_field(dims, eps, cfg, i_eps, dev, a, log):
    import torch

    import synthetic
    seed = synthetic.gauge_seed(cfg, i_eps)
    ctx, u = gpu_context(dims, eps, seed, dev)
    err = check_apply(ctx, u, dims, seed, dev)
    log(f"{dims} eps {eps} seed {seed}: library D vs oracle at sampled sites {err:.2e}")
    if not err <= 1e-13:
        raise SystemExit(f"library D disagrees with the oracle on this field ({err:.2e})")
    del u
    shape = (dims[3], dims[2], dims[1], dims[0], 4, 3)
    n = int(np.prod(shape))

    def matvec(v):
        return ctx.apply_D(v.view(shape)).view(n)

    t0 = time.time()
    theta, res, V, C, nmv, cycles, done, hist = krylov_schur_leftmost(
        matvec, n, dev, a.m, a.p, a.nev, a.tol, a.max_cycles, seed, log, a.time_limit)
    drift = float(max(hist[-10:]) - min(hist[-10:])) if len(hist) >= 10 else float("inf")
    # explicit residual of the leftmost Ritz pair
    coef = torch.from_numpy(np.ascontiguousarray(C[:, 0])).to(dev)
    v = (coef.unsqueeze(0) @ V[: C.shape[0]]).squeeze(0)
    del V
    torch.cuda.empty_cache()
    r = matvec(v) - complex(theta[0]) * v
    true_res = float(torch.linalg.vector_norm(r) / torch.linalg.vector_norm(v))
    ctx.close()
    entry = {"dims": list(dims), "eps": eps, "gauge_seed": seed, "t_bc": -1,
             "m_crit": -float(theta[0].real),
             "leftmost": [[float(t.real), float(t.imag)] for t in theta[: a.nev]],
             "ritz_residual_estimate": [float(x) for x in res[: a.nev]],
             "leftmost_explicit_residual": true_res, "converged": done,
             "accepted": true_res <= a.accept or (true_res <= 1e-4 and drift <= 1e-6),
             "accept": (f"explicit residual <= {a.accept:g}, or <= 1e-4 with the leftmost real part moving "
                        "by at most 1e-6 over the last 10 restarts"),
             "leftmost_re_drift_last_10_cycles": drift,
             "matvecs": nmv, "cycles": cycles, "seconds": time.time() - t0,
             "apply_D_vs_oracle_sampled": err,
             "method": (f"Krylov-Schur (basis {a.m}, keep {a.p}, {a.nev} leftmost to {a.tol:g}) on the "
                        "library's FP64 D(m=0), basis on the GPU; tests/inputs/make_mcrit_gpu.py")}
    key = "x".join(map(str, dims)) + f"_eps{eps}_seed{seed}"
    log(f"{key}: m_crit {entry['m_crit']:.10f}, explicit residual {true_res:.2e}, {nmv} matvecs")
    return key, entry


def save(key, entry, path):
    data = {}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
    data[key] = entry
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--validate", action="store_true",
                    help="rerun the fields of tests/golden/mcrit.json and compare with the oracle's values")
    ap.add_argument("--field", nargs=7, action="append", default=[], metavar=("LX", "LY", "LZ", "LT", "EPS", "CFG", "I_EPS"))
    ap.add_argument("--m", type=int, default=96, help="Krylov basis size")
    ap.add_argument("--p", type=int, default=32, help="Schur vectors kept at a restart")
    ap.add_argument("--nev", type=int, default=4)
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--accept", type=float, default=1e-6)
    ap.add_argument("--max-cycles", type=int, default=2000)
    ap.add_argument("--time-limit", type=float, default=600.0, help="seconds per field")
    ap.add_argument("--out", default=OUT)
    a = ap.parse_args()
    import torch
    dev = torch.device("cuda:0")

    def log(msg):
        print(msg, flush=True)

    if a.validate:
        with open(GOLDEN) as fh:
            gold = json.load(fh)
        val = {}
        for key, g in sorted(gold.items()):
            dims = tuple(g["dims"])
            i_eps = {0.2: 0, 0.3: 1, 0.45: 2}[g["eps"]]
            cfg = (g["gauge_seed"] - 10 * i_eps) // 1000
            k2, e = run_field(dims, g["eps"], cfg, i_eps, dev, a, log)
            assert k2 == key
            save(key, e, a.out)
            val[key] = {"oracle_m_crit": g["m_crit"], "gpu_m_crit": e["m_crit"],
                        "difference": e["m_crit"] - g["m_crit"], "matvecs": e["matvecs"],
                        "explicit_residual": e["leftmost_explicit_residual"]}
            log(f"validation {key}: oracle {g['m_crit']:.10f} gpu {e['m_crit']:.10f} "
                f"diff {e['m_crit'] - g['m_crit']:.2e}")
        save("_validation", val, a.out)
    for f in a.field:
        dims = tuple(int(v) for v in f[:4])
        key, entry = run_field(dims, float(f[4]), int(f[5]), int(f[6]), dev, a, log)
        save(key, entry, a.out)


if __name__ == "__main__":
    main()
