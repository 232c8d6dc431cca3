"""Writes config0_20cube.json: the oracle's steady state and leading
eigenvalues for the 20^3 uniform-grid cube, Pr 0.71, Gr 1e5, conducting
spanwise walls (Sec. 2 problem, Sec. 3.1 method).

Calls only the oracle (and the seeded input module).  The steady state is
reached by Newton with continuation in Gr from the conduction state (the
oracle's Newton from the conduction state diverges at Gr = 1e5), each Newton
correction solved exactly (sparse direct); the eigenvalues are ARPACK's on the
oracle operator with the complement of the constraint subspace shifted away.
Run from the repository root:  python tests/golden/make_config0.py
(about half an hour on 8 cores)."""
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ops  # noqa: E402
from oracle.grid import Grid, UNIFORM  # noqa: E402
from oracle.krylov import Oracle  # noqa: E402
from paper_1905_11601_amd import inputs  # noqa: E402

STAGES = (1e3, 3.3e3, 1.1e4, 3.6e4, 1e5)


def main():
    g = Grid(20, kind=UNIFORM)
    U = torch.as_tensor(inputs.conduction_state(tuple(a.c for a in g.ax), 0))
    its = []
    t0 = time.time()
    for Gr in STAGES:
        orc = Oracle(g, ops.Params(Gr, 0.71), 0)
        U, hist = orc.newton(U, tol=1e-11, max_it=15)
        its.append(len(hist))
        print(f"Gr {Gr:g}: {len(hist)} Newton iterations, max|P F| {hist[-1]:.2e}, "
              f"{time.time() - t0:.0f} s", flush=True)
    res = float(orc.residual(U, project=True).abs().max())
    x = orc.project(torch.as_tensor(inputs.random_fields(g.n, 5000)))
    x = x / torch.linalg.norm(x)
    lam, _ = orc.leading_eigs(U, k=8, ncv=40, v0=x, tol=1e-12)
    print("eigenvalues", lam, flush=True)
    out = {
        "workload": "20^3 uniform grid, Pr 0.71, Gr 1e5, CC walls, oracle steady state",
        "stages_Gr": list(STAGES),
        "newton_iterations": its,
        "residual_max": res,
        "max_abs": [float(U[f].abs().max()) for f in range(4)],
        "eigenvalues_re": [float(v.real) for v in lam],
        "eigenvalues_im": [float(v.imag) for v in lam],
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "config0_20cube.json"),
              "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
