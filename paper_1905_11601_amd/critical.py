"""Critical Grashof number and frequency of the oscillatory instability
(Sec. 4.1): a steady state at a starting Gr, then the Newton iteration on Gr
for Re lambda_lead = 0 with the adjoint eigenvalue sensitivity
(drivers.critical_gr), on the paper's sine-stretched grid of eq. (22) or any
other grid kind.  Also prints the extrema of the vector potentials Psi_x,
Psi_y, Psi_z (Sec. 3.2) of the starting steady state.

    python -m paper_1905_11601_amd.critical --n 64 --grid sine --s 0.12 --bc CC --gr0 3.4e6

One progress line per Newton stage and Gr iterate on stderr, one JSON line on
stdout.  The paper's values (its own schemes and grids, 240^3-256^3 and
extrapolated) are a sanity check, not a target: Gr_cr ~ 3.43e6, f_cr = 0.2825
(CC-CC), Gr_cr ~ 3.40e6, f_cr = 0.2637 (CC-AA), with f = Im(lambda) / (2 pi).
"""
import argparse
import json
import math
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=64, help="cells per axis")
    ap.add_argument("--grid", choices=("uniform", "sine", "tanh"), default="sine")
    ap.add_argument("--s", type=float, default=0.12, help="stretching parameter")
    ap.add_argument("--bc", choices=("CC", "AA"), default="CC")
    ap.add_argument("--pr", type=float, default=0.71)
    ap.add_argument("--gr0", type=float, default=3.4e6, help="starting Grashof number")
    ap.add_argument("--coarse", type=int, default=0,
                    help="start the steady state from this coarser grid (0: continuation here)")
    ap.add_argument("--newton-tol", type=float, default=1e-8,
                    help="steady-state residual tolerance (the FP64 floor of max |P F| on "
                         "strongly stretched grids is ~1e-9)")
    ap.add_argument("--k", type=int, default=8,
                    help="eigenvalues per solve (every pair near the crossing must fit)")
    ap.add_argument("--m", type=int, default=60)
    ap.add_argument("--tol", type=float, default=1e-9, help="Ritz residual tolerance")
    ap.add_argument("--gr-rtol", type=float, default=1e-6)
    ap.add_argument("--max-it", type=int, default=8)
    ap.add_argument("--max-restarts", type=int, default=800)
    ap.add_argument("--chebyshev", type=int, default=0, metavar="DEGREE")
    args = ap.parse_args(argv)

    import torch
    import paper_1905_11601_amd as fvk
    from paper_1905_11601_amd import inputs
    from paper_1905_11601_amd.drivers import critical_gr, steady_state, steady_state_refined

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    kind = {"uniform": fvk.UNIFORM, "sine": fvk.SINE, "tanh": fvk.TANH}[args.grid]
    bc = fvk.CC if args.bc == "CC" else fvk.AA
    ctx = fvk.Ctx(args.n, grid=kind, s=args.s, span_bc=bc, Gr=args.gr0, Pr=args.pr)
    _, c, _ = ctx.coords()
    t0 = time.perf_counter()
    nopts = dict(tol=args.newton_tol)
    if args.coarse:
        base, rep, _ = steady_state_refined(ctx, args.coarse, args.gr0, log=log,
                                            newton_opts=nopts, coarse_opts=nopts)
    else:
        base = torch.as_tensor(inputs.conduction_state(c, bc)).cuda()
        steady_state(ctx, base, args.gr0, newton_opts=nopts, log=log)
    t_base = time.perf_counter() - t0
    psi = {}
    for axis, name in enumerate(("x", "y", "z")):
        _, p = ctx.psi_projection(base, axis)
        ph = p.cpu().numpy()
        psi[name] = [float(ph.min()), float(ph.max())]
    log(f"steady state at Gr {args.gr0:g} in {t_base:.0f} s; Psi extrema {psi}")
    v0 = ctx.project(torch.as_tensor(inputs.random_fields(ctx.n, 5000)).cuda())
    seed = torch.as_tensor(inputs.random_fields(ctx.n, 5001)).cuda()
    t1 = time.perf_counter()
    hist = critical_gr(ctx, base, args.gr0, v0, seed, k=args.k, m=args.m, tol=args.tol,
                       gr_rtol=args.gr_rtol, max_it=args.max_it, log=log,
                       chebyshev=args.chebyshev, max_restarts=args.max_restarts,
                       newton_opts=nopts)
    t_crit = time.perf_counter() - t1
    conv = bool(hist[-1].get("converged"))
    last = [h for h in hist if "lam" in h][-1]
    lam = complex(last["lam"])
    out = {"grid": [args.n] * 3, "grid_kind": args.grid, "s": args.s, "span_bc": args.bc,
           "Pr": args.pr, "Gr0": args.gr0, "converged": conv, "Gr_critical": hist[-1]["Gr"],
           "lambda_at_last_iterate": [lam.real, lam.imag],
           "f_critical": abs(lam.imag) / (2 * math.pi),
           "history": [{"Gr": h["Gr"], "lam": [complex(h["lam"]).real, complex(h["lam"]).imag],
                        "dlam_dGr": [complex(h["dlam_dGr"]).real, complex(h["dlam_dGr"]).imag],
                        "slope": h["slope"], "step_from": h["step_from"],
                        "eigenvalues": [[v.real, v.imag] for v in h["eigenvalues"]],
                        "transposed_eigenvalues": [[v.real, v.imag]
                                                   for v in h["transposed_eigenvalues"]],
                        "missed_by_forward_solve": [[v.real, v.imag]
                                                    for v in h["missed_by_forward_solve"]],
                        "nvec": h["nvec"]} for h in hist if "lam" in h],
           "psi_extrema_at_Gr0": psi, "base_seconds": t_base, "critical_seconds": t_crit}
    print(json.dumps(out))
    return 0 if conv else 1


if __name__ == "__main__":
    sys.exit(main())
