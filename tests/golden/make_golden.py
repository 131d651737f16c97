"""Writes the stored expected values under tests/golden/ (calls only oracle/ and fks_inputs).

sigma_form_hard_spheres.json
    Q(v) of eq. boltzmann (Section 2.2, sigma form) for hard spheres,
    B = C |v - v*| with C = 1/4 (so the Carleman kernel B~ = 4C = 1), evaluated
    by brute-force quadrature (oracle.sigma_form) for an analytic
    two-Maxwellian f at five grid points of the N = 32, L = 8 velocity grid.
oracle_snapshot_n8.json
    Sampled values of O-fast Q for a seeded mixture at N = 8 (regression guard
    for the oracle's own arithmetic; regenerate only with a commit that names
    the passage justifying the change).

Run:  python tests/golden/make_golden.py
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import make_plan, sigma_form  # noqa: E402
from oracle.collide import collide_fast  # noqa: E402
import fks_inputs  # noqa: E402

COMPONENTS = [(0.7, (0.3, -0.2, 0.1), 0.7), (0.4, (-0.5, 0.4, 0.2), 0.9)]
POINTS = [(16, 16, 16), (17, 15, 16), (14, 18, 17), (19, 16, 13), (16, 16, 20)]


def sigma_golden():
    n, L = 32, 8.0
    v1 = fks_inputs.velocity_axis(n, L)
    fun = sigma_form.mixture(COMPONENTS)
    rows = []
    for idx in POINTS:
        v = np.array([v1[i] for i in idx])
        rows.append({"index": list(idx), "v": v.tolist(),
                     "Q": sigma_form.collision_integral(fun, v, 0.25, 1.0)})
    return {"source": "eq. boltzmann (Section 2.2), hard spheres B = C|g|, C = 1/4",
            "n": n, "L": L, "components": [[c[0], list(c[1]), c[2]] for c in COMPONENTS],
            "quadrature": "r in [0,12] GL48, ghat and omega GL16 x trapezoid32",
            "points": rows}


def snapshot_golden():
    n, L, R = 8, 6.0, 4.0
    plan = make_plan(n, L, R, a1=4, a2=4, C=0.25)
    f = fks_inputs.maxwellian_mixture(n, L, 1, seed=3)[0]
    Q = collide_fast(f, plan)
    idx = [(0, 0, 0), (3, 4, 5), (4, 4, 4), (7, 1, 2), (5, 5, 3), (2, 6, 4)]
    return {"source": "O-fast (Appendix A), hard spheres, n=8, L=6, R=4, A1=A2=4, C=1/4, "
                      "fks_inputs.maxwellian_mixture seed 3",
            "n": n, "L": L, "R": R, "samples": [{"index": list(i), "Q": float(Q[i])} for i in idx],
            "norm": float(np.linalg.norm(Q))}


if __name__ == "__main__":
    with open(os.path.join(HERE, "sigma_form_hard_spheres.json"), "w") as fh:
        json.dump(sigma_golden(), fh, indent=1)
    with open(os.path.join(HERE, "oracle_snapshot_n8.json"), "w") as fh:
        json.dump(snapshot_golden(), fh, indent=1)
    print("written")
