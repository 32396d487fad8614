"""Writes tests/golden/mcrit.json: critical masses of the synthetic benchmark fields.

Calls only the oracle (``oracle.mcrit``, ARPACK on the numpy Wilson operator)
and the seeded link generator.  ``m_crit = -min Re lambda(D at m=0)`` for the
links ``U = exp(i eps H)`` of each workload (antiperiodic time).

usage: python tests/golden/make_mcrit.py LX LY LZ LT EPS CFG I_EPS [TOL [NCV]]

Accuracy: ARPACK stops at relative tolerance TOL (default 1e-8 for small
lattices); a Ritz pair is accepted when ||D v - lambda v|| <= max(1e-6, 10 TOL).
For the gamma5-Hermitian D this bounds the error of m_crit far below the
smallest mass offset used (0.003).
"""
import fcntl
import json
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

import synthetic  # noqa: E402
from oracle import mcrit  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mcrit.json")


def main():
    lx, ly, lz, lt = (int(a) for a in sys.argv[1:5])
    eps = float(sys.argv[5])
    cfg, i_eps = int(sys.argv[6]), int(sys.argv[7])
    tol = float(sys.argv[8]) if len(sys.argv) > 8 else 1e-8
    ncv = int(sys.argv[9]) if len(sys.argv) > 9 else 60
    seed = synthetic.gauge_seed(cfg, i_eps)
    u = synthetic.gauge_field((lx, ly, lz, lt), eps, seed)
    t0 = time.time()
    mc, vals, res = mcrit.mcrit(u, t_bc=-1.0, k=4, ncv=ncv, tol=tol, accept=max(1e-6, 10 * tol))
    key = f"{lx}x{ly}x{lz}x{lt}_eps{eps}_seed{seed}"
    entry = {"dims": [lx, ly, lz, lt], "eps": eps, "gauge_seed": seed, "t_bc": -1,
             "m_crit": mc, "leftmost": [[v.real, v.imag] for v in vals],
             "ritz_residual": [float(r) for r in res], "seconds": time.time() - t0,
             "method": f"oracle.mcrit: ARPACK eigs which=SR k=4 ncv={ncv} tol={tol:g} on oracle D(m=0)"}
    with open(OUT + ".lock", "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        data = {}
        if os.path.exists(OUT):
            with open(OUT) as fh:
                data = json.load(fh)
        data[key] = entry
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
    print(key, mc, time.time() - t0, flush=True)


if __name__ == "__main__":
    main()
