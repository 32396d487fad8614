"""Writes tests/golden/mcrit_2d.json: the critical mass of the synthetic 2d U(1) field.

Calls only the oracle (``oracle.qed2d.mcrit``: ARPACK on the sparse 2d Wilson
operator) and the seeded link generator.  ``m_crit = -min Re lambda(D at m=0)``
for the compact U(1) field of ``synthetic.u1_gauge_field`` (antiperiodic time).

usage: python tests/golden/make_mcrit_2d.py LX LT BETA SEED
"""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

import synthetic  # noqa: E402
from oracle import qed2d  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mcrit_2d.json")


def main():
    lx, lt = int(sys.argv[1]), int(sys.argv[2])
    beta, seed = float(sys.argv[3]), int(sys.argv[4])
    u = synthetic.u1_gauge_field((lx, lt), beta, seed)
    mc, vals, res = qed2d.mcrit(u, t_bc=-1.0, ncv=60)
    i = int(abs(vals.real + mc).argmin())
    if res[i] > 1e-8:
        raise SystemExit(f"leftmost Ritz pair not converged (residual {res[i]:.1e})")
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    data[f"{lx}x{lt}_beta{beta}_seed{seed}"] = {
        "dims": [lx, lt], "beta": beta, "gauge_seed": seed, "t_bc": -1, "m_crit": mc,
        "leftmost": [[v.real, v.imag] for v in sorted(vals, key=lambda z: z.real)],
        "residual": float(res[i])}
    with open(OUT, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    print(f"m_crit = {mc:.10f}")


if __name__ == "__main__":
    main()
