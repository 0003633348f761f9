"""Writes tests/golden/c1_tiny.json from the FP64 oracle alone (no GPU code):
the tiny configuration -- 4^4 lattice, Haar-random SU(3) links (seed 1001),
one complex Gaussian source (seed 2001), kappa = 0.160, mu = 0.01, one flavour
twisted up, antiperiodic in time -- through the symmetric preconditioned
operator of Eq. (2.3), CG to 1e-13 on its normal equations and the odd
reconstruction of Eq. (2.4).  Run from the repository root:

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O            # noqa: E402
from paper_1311_4462_amd import inputs    # noqa: E402

DIMS = (4, 4, 4, 4)
SITES = [(0, 0, 0, 0), (1, 0, 0, 0), (3, 2, 1, 3), (2, 3, 3, 1)]   # (x, y, z, t)


def compute():
    p = O.Params(DIMS, 0.160, 0.01, 0.0, O.PLUS)
    U = inputs.gauge_field(DIMS, "haar", 1001)
    b = inputs.gaussian_spinor(DIMS, 1, 2001)
    be = O.project(b, DIMS, 0)
    y = O.mat_pc(p, U, be, "sym")
    rhs = O.prepare(p, U, b, "sym")
    xe, info = O.cg(p, U, rhs, "sym", tol=1e-13)
    psi = xe + O.reconstruct(p, U, xe, b)

    def comp(f):
        out = {}
        for (x, yy, z, t) in SITES:
            v = f[t, z, yy, x, 0].reshape(-1)
            out[f"{x},{yy},{z},{t}"] = [[float(c.real), float(c.imag)] for c in v]
        return out

    return {
        "config": "4^4, haar seed 1001, source seed 2001, kappa 0.160, mu 0.01, PLUS, antiperiodic t",
        "mat_pc_sym_norm2": float(np.vdot(y, y).real),
        "mat_pc_sym_sites": comp(y),
        "cg_iters": int(info["iters"]),
        "cg_true_rel_res_normal": float(info["true_rel_res_normal"]),
        "solution_norm2": float(np.vdot(psi, psi).real),
        "solution_sites": comp(psi),
        "full_residual": float(np.linalg.norm(O.full_M(p, U, psi) - b) / np.linalg.norm(b)),
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "c1_tiny.json"), "w") as f:
        json.dump(compute(), f, indent=1)
    print("wrote", os.path.join(HERE, "c1_tiny.json"))
