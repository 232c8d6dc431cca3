#!/usr/bin/env python
"""Rightmost eigenvalues of eq. (10) on the GPU, certified by the oracle.

Runs the library's Krylov-Schur solve (FP64, mixed precision, or both) for
the k rightmost eigenvalues about a base flow, then applies the oracle's
Krylov operator A (plain CPU FP64, no code shared with the library) once to
the real and imaginary parts of every GPU eigenvector on the host:

    oracle Ritz residual = || A_oracle x - lambda x || / || x ||,

an independent certificate of each eigenpair (the oracle cannot itself run
the ~10^4 Arnoldi steps a large grid needs).  Mixed-precision eigenvalues are
also compared with the FP64 ones.  One JSON line on stdout (and in --out).

    python tests/certify_eigs.py --n 256 --bc CC --k 4 --m 100 --prec both \\
        --out cert_256_CC.json

Test infrastructure: it imports the oracle, so it lives under tests/.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def oracle_residuals(orc, U, lam, X):
    """|| A_oracle x - lam x || / || x || for the GPU eigenvectors X (complex
    CUDA tensor, one row per eigenvector)."""
    import torch
    out = []
    for q in range(len(lam)):
        x = X[q].cpu().numpy().reshape(-1)
        xr = torch.as_tensor(np.ascontiguousarray(x.real).reshape(orc.shape4))
        xi = torch.as_tensor(np.ascontiguousarray(x.imag).reshape(orc.shape4))
        Ax = orc.krylov_vec(U, xr).reshape(-1).numpy() + 1j * orc.krylov_vec(U, xi).reshape(-1).numpy()
        out.append(float(np.linalg.norm(Ax - lam[q] * x) / np.linalg.norm(x)))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=100)
    ap.add_argument("--bc", choices=("CC", "AA"), default="CC")
    ap.add_argument("--gr", type=float, default=1e6)
    ap.add_argument("--pr", type=float, default=0.71)
    ap.add_argument("--base", choices=("synthetic", "newton", "refined"), default="synthetic")
    ap.add_argument("--coarse", default="64",
                    help="coarse grid(s) of --base refined, coarsest first (e.g. 64,128)")
    ap.add_argument("--newton-tol", type=float, default=1e-9)
    ap.add_argument("--newton-max", type=int, default=10,
                    help="Newton iterations on the fine grid of --base refined")
    ap.add_argument("--gmres-m", type=int, default=100,
                    help="GMRES restart length of the Newton linear solves (<= 400)")
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--m", type=int, default=100)
    ap.add_argument("--keep", type=int, default=None)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--max-restarts", type=int, default=3000)
    ap.add_argument("--prec", choices=("fp64", "mixed", "both"), default="both")
    ap.add_argument("--chebyshev", type=int, default=0, metavar="DEGREE",
                    help="Krylov-Schur on the Chebyshev filter of this degree (0: plain)")
    ap.add_argument("--threads", type=int, default=16, help="oracle (torch CPU) threads")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    import torch
    import paper_1905_11601_amd as fvk
    from paper_1905_11601_amd import inputs
    from paper_1905_11601_amd.drivers import steady_state, steady_state_refined
    from paper_1905_11601_amd.eigs import krylov_schur, krylov_schur_chebyshev, ritz_residual
    from oracle import ops
    from oracle.grid import Grid, TANH
    from oracle.krylov import Oracle

    torch.set_num_threads(args.threads)
    bc = fvk.CC if args.bc == "CC" else fvk.AA
    n = args.n
    print(f"case certify n={n} bc={args.bc} base={args.base} prec={args.prec}", file=sys.stderr,
          flush=True)
    ctx = fvk.Ctx(n, grid=fvk.TANH, s=1.5, span_bc=bc, Gr=args.gr, Pr=args.pr)
    g = Grid(n, kind=TANH, s=1.5)
    orc = Oracle(g, ops.Params(args.gr, args.pr), bc)
    t0 = time.perf_counter()
    if args.base == "synthetic":
        f = tuple(a.f for a in g.ax)
        c = tuple(a.c for a in g.ax)
        h = tuple(a.h for a in g.ax)
        U = torch.as_tensor(inputs.synthetic_base(f, c, h, bc))
        Ud = U.cuda()
        base_info = {"base": "synthetic"}
    else:
        c = tuple(a.c for a in g.ax)
        if args.base == "newton":
            Ud = torch.as_tensor(inputs.conduction_state(c, bc)).cuda()
            stages = steady_state(ctx, Ud, args.gr,
                                  newton_opts=dict(tol=args.newton_tol, gmres_m=args.gmres_m),
                                  log=log)
            fine = None
        else:
            levels = [int(v) for v in args.coarse.split(",")]
            Ud, fine, stages = steady_state_refined(ctx, levels, args.gr, log=log,
                                                    newton_opts=dict(tol=args.newton_tol,
                                                                     max_newton=args.newton_max,
                                                                     gmres_m=args.gmres_m),
                                                    coarse_opts=dict(tol=args.newton_tol,
                                                                     gmres_m=args.gmres_m))
        U = Ud.cpu()
        res_ora = float(orc.residual(U, project=True).abs().max())
        base_info = {"base": args.base, "newton_stages": [[s_[0], s_[1]["newton_its"]]
                                                          for s_ in stages],
                     "newton_seconds": time.perf_counter() - t0,
                     "oracle_max_projected_residual": res_ora}
        if fine is not None:
            base_info["coarse_grids"] = levels
            base_info["fine_newton"] = {k: fine[k] for k in ("status", "newton_its",
                                                              "res_before", "res_after",
                                                              "gmres_cycles", "bicgstab_its",
                                                              "krylov_vecs")}
        log(f"steady state: oracle max|P F| = {res_ora:.3e}")
    v0 = ctx.project(torch.as_tensor(inputs.random_fields(ctx.n, 5000)).cuda())
    out = {"grid": [n] * 3, "grid_kind": "tanh", "s": 1.5, "span_bc": args.bc, "Gr": args.gr,
           "gmres_m": args.gmres_m,
           "Pr": args.pr, "k": args.k, "m": args.m, "keep": args.keep, "tol": args.tol,
           "chebyshev": args.chebyshev}
    out.update(base_info)
    lams = {}
    precs = ["fp64", "mixed"] if args.prec == "both" else [args.prec]
    for prec in precs:
        ctx.set_precision(fvk.MIXED if prec == "mixed" else fvk.FP64)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        every = max(1, args.max_restarts // 60)
        if args.chebyshev > 0:
            r = krylov_schur_chebyshev(ctx, Ud, k=args.k, m=args.m, v0=v0, tol=args.tol,
                                       degree=args.chebyshev, max_restarts=args.max_restarts,
                                       keep=args.keep,
                                       log=lambda s_: log(s_) if ("restart" not in s_ or
                                                                  "00:" in s_ or
                                                                  "extraction" in s_) else None)
        else:
            r = krylov_schur(ctx, Ud, k=args.k, m=args.m, v0=v0, tol=args.tol,
                             max_restarts=args.max_restarts, keep=args.keep,
                             log=lambda s_: log(s_) if int(s_.split()[1].rstrip(":")) % every == 0
                             else None)
        torch.cuda.synchronize()
        t_eig = time.perf_counter() - t1
        gpu_res = [ritz_residual(ctx, Ud, r.lam[q], r.X[q]) for q in range(len(r.lam))]
        ctx.set_precision(fvk.FP64)
        t2 = time.perf_counter()
        ora_res = oracle_residuals(orc, U, r.lam, r.X)
        log(f"{prec}: {r.lam} oracle residuals {ora_res} ({time.perf_counter() - t2:.1f} s)")
        lams[prec] = r.lam
        out[prec] = {"converged": r.converged, "restarts": r.restarts, "krylov_vectors": r.nvec,
                     "orthogonalisation_steps": getattr(r, "orth_steps", r.nvec),
                     "ellipse": getattr(r, "ellipse", None),
                     "shift": r.shift, "eigen_seconds": t_eig,
                     "eigenvalues": [[float(v.real), float(v.imag)] for v in r.lam],
                     "gpu_ritz_residuals": gpu_res, "oracle_ritz_residuals": ora_res}
        del r
    if len(precs) == 2:
        d = [float(np.min(np.abs(lams["fp64"] - l))) for l in lams["mixed"]]
        out["mixed_vs_fp64_abs"] = d
        out["mixed_vs_fp64_max_rel"] = max(d) / float(np.abs(lams["fp64"]).max())
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(line + "\n")
    ok = all(out[p]["converged"] and max(out[p]["oracle_ritz_residuals"]) < 10 * args.tol
             for p in precs)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
