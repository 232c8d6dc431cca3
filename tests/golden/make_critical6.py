"""Writes critical_6cube.json: the critical Grashof number of the 6^3
uniform-grid cube, Pr 0.71, conducting spanwise walls -- the Gr at which the
real part of the leading (oscillatory) eigenvalue pair of eq. (10) about the
steady state crosses zero (Sec. 3.1: Newton steady state, then the leading
eigenvalues, repeated in Gr) -- with the leading eigenvalue and its total
derivative along the branch of steady states at Gr0 = 1.5e6; and the
crossing of the eigenvalue problem with the coupling term W dT/dz switched off
(the mechanism experiment of Sec. 4.2), the steady states unchanged.

Calls only the oracle (and the seeded input module).  Steady states: the
oracle's Newton (exact sparse solves) with continuation in Gr from the
conduction state; eigenvalues: the dense generalized eigenproblem of the
saddle-point pencil (a library eigen-solver); the crossing: secant iteration
on Re lambda(Gr), each Gr with its own Newton steady state; the derivative: a
central difference of lambda along the branch, the steady state re-solved at
Gr0 (1 +- 1e-4).  On this grid the second oscillatory pair crosses later
(between Gr = 2e6 and 3e6), so the leading pair is well separated.
Run from the repository root:  python tests/golden/make_critical6.py
(a few minutes on 8 cores)."""
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ops  # noqa: E402
from oracle.dense import dense_pencil_eigs  # noqa: E402
from oracle.grid import Grid, UNIFORM  # noqa: E402
from oracle.krylov import Oracle  # noqa: E402
from paper_1905_11601_amd import inputs  # noqa: E402

N, BC, PR = 6, 0, 0.71
GR0 = 1.5e6


def steady(g, U, Gr):
    orc = Oracle(g, ops.Params(Gr, PR), BC)
    U, hist = orc.newton(U, tol=1e-12, max_it=20)
    if hist[-1] > 1e-12:
        raise RuntimeError(f"oracle Newton did not converge at Gr {Gr:g}: {hist[-3:]}")
    return U


# the same crossing with the term W dT/dz switched off in the eigenvalue
# problem (the mechanism experiment of Sec. 4.2; a real leading eigenvalue)
MASK_NO_W_DT_DZ = ops.ALL_TERMS & ~(1 << (ops.TERM_U_GRAD_T + 2))


def leading(g, U, Gr, terms=ops.ALL_TERMS):
    """Leading eigenvalue (largest real part; the member of a complex pair
    with positive imaginary part)."""
    lam = dense_pencil_eigs(g, ops.Params(Gr, PR), U, BC, terms)
    top = lam[np.abs(lam.real - lam[0].real) < 1e-9 * np.abs(lam).max()]
    return top[np.argmax(top.imag)]


def main():
    t0 = time.time()
    g = Grid(N, kind=UNIFORM)
    U = torch.as_tensor(inputs.conduction_state(tuple(a.c for a in g.ax), BC))
    Gr = 1e3
    while Gr < GR0:
        Gr = min(GR0, Gr * 1.5)
        U = steady(g, U, Gr)
    U0 = U.clone()
    lam0 = leading(g, U0, GR0)
    d = 1e-4 * GR0
    lp = leading(g, steady(g, U0, GR0 + d), GR0 + d)
    lm = leading(g, steady(g, U0, GR0 - d), GR0 - d)
    dlam = (lp - lm) / (2 * d)
    print(f"Gr0 {GR0:g}: lambda {lam0}, d lambda/d Gr (central difference) {dlam}  "
          f"[{time.time() - t0:.0f} s]", flush=True)
    U2 = steady(g, steady(g, U0, 1.75e6), 2e6)

    def crossing(terms):
        """secant on Re lambda(Gr) from Gr0 and 2e6 (opposite signs)"""
        ga, la = GR0, leading(g, U0, GR0, terms)
        gb, Ub = 2e6, U2
        lb = leading(g, Ub, gb, terms)
        assert la.real < 0 < lb.real
        for it in range(30):
            gc = gb - lb.real * (gb - ga) / (lb.real - la.real)
            Uc = steady(g, Ub, gc)
            lc = leading(g, Uc, gc, terms)
            print(f"secant {it}: Gr {gc:.12g} Re lambda {lc.real:.3e}  "
                  f"[{time.time() - t0:.0f} s]", flush=True)
            ga, la, gb, lb, Ub = gb, lb, gc, lc, Uc
            if abs(gb - ga) < 1e-11 * gb:
                break
        return gb, lb

    gb, lb = crossing(ops.ALL_TERMS)
    gm, lm = crossing(MASK_NO_W_DT_DZ)
    out = {
        "workload": "6^3 uniform grid, Pr 0.71, conducting walls, oracle steady states",
        "Gr0": GR0,
        "lambda0": [float(lam0.real), float(lam0.imag)],
        "dlam_dGr_total_central_difference": [float(dlam.real), float(dlam.imag)],
        "fd_step": d,
        "Gr_critical": float(gb),
        "lambda_critical": [float(lb.real), float(lb.imag)],
        "terms_mask_no_W_dT_dz": MASK_NO_W_DT_DZ,
        "Gr_critical_no_W_dT_dz": float(gm),
        "lambda_critical_no_W_dT_dz": [float(lm.real), float(lm.imag)],
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "critical_6cube.json"),
              "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
