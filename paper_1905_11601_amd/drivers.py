"""Host drivers over the C ABI: steady states by Newton with continuation in
the Grashof number, and the critical Grashof number (Re lambda = 0, Sec. 2 and
eq. (10)) by a Newton iteration on Gr with the adjoint eigenvalue
sensitivity.

All vector work runs in the library (newton_step, fvk_linear_solve,
simple_krylov_vec, arnoldi_step); these functions only sequence the calls.
"""
import numpy as np

from .adjoint import dA_dGr_apply, _cdot, left_eigvecs
from .eigs import krylov_schur, krylov_schur_chebyshev


def steady_state(ctx, base, Gr, Gr_start=1e3, factor=3.3, newton_opts=None, log=None):
    """Newton iteration (newton_step) for the steady state at ``Gr``, reached by
    continuation from ``Gr_start`` in geometric steps of at most ``factor``.
    A stage that needs more than ``max_newton`` (8) iterations is rejected and
    retried from the last converged state with a smaller step: a Newton
    iteration that wanders far from its start can land on a different
    (spurious, on coarse grids) branch of steady states.  ``base`` (device,
    in/out) is the starting state: the conduction state, or a steady state at
    Gr_start.  Returns the list of (Gr, newton report) of the stages."""
    opts = dict(tol=1e-10, gmres_m=100, lin_tol=1e-10, max_newton=8)
    opts.update(newton_opts or {})
    stages = []
    good = base.clone()
    g_done = None
    g_next = min(Gr, Gr_start)
    step = factor
    while True:
        ctx.set_params(g_next)
        rep = ctx.newton_step(base, **opts)
        stages.append((g_next, rep))
        if log:
            log(f"Gr {g_next:.4g}: status {rep['status']} newton {rep['newton_its']} "
                f"res {rep['res_after']:.2e}")
        if rep["status"] == 0:
            good.copy_(base)
            g_done = g_next
            if g_done >= Gr:
                return stages
            step = min(factor, step * 1.5)
            g_next = min(Gr, g_done * step)
        else:
            base.copy_(good)
            if g_done is None:
                raise RuntimeError(f"Newton failed at the first continuation stage Gr={g_next:g}")
            step = step ** 0.5
            if step < 1.01:
                raise RuntimeError(f"continuation stalled at Gr={g_done:g}")
            g_next = min(Gr, g_done * step)


def _interp_axis(a, dim, xc, xf):
    """Linear interpolation of array a along dimension dim from the increasing
    coordinates xc to xf (both inside the same interval [xc[0], xc[-1]])."""
    idx = np.clip(np.searchsorted(xc, xf, side="right") - 1, 0, len(xc) - 2)
    w = (xf - xc[idx]) / (xc[idx + 1] - xc[idx])
    shape = [1] * a.ndim
    shape[dim] = len(xf)
    w = w.reshape(shape)
    return np.take(a, idx, axis=dim) * (1.0 - w) + np.take(a, idx + 1, axis=dim) * w


def prolong_fields(coarse, fc, cc, ff, cf):
    """A 4-field state on a coarse staggered grid interpolated (trilinear,
    field by field at its own nodes) to a fine grid of the same kind.

    coarse: (4, nz+2, ny+2, nx+2) array; fc, cc / ff, cf: per-axis (x, y, z)
    face coordinates f[0..n] and centres c[0..n+1] (wall nodes included) of
    the coarse / fine grid.  Velocity component a lives on the a-faces along
    axis a (stored indices 0..n; index n+1 is padding and stays 0) and on the
    centres along the other axes; T on the centres."""
    nzf, nyf, nxf = (len(ff[a]) - 1 for a in (2, 1, 0))
    out = np.zeros((4, nzf + 2, nyf + 2, nxf + 2))
    for fld in range(4):
        a = np.asarray(coarse[fld])
        sl_c, sl_f = [], []
        for axis in (2, 1, 0):               # array dims (z, y, x)
            own = fld == axis
            nc, nf = len(fc[axis]) - 1, len(ff[axis]) - 1
            sl_c.append(slice(0, nc + 1) if own else slice(0, nc + 2))
            sl_f.append(slice(0, nf + 1) if own else slice(0, nf + 2))
        a = a[tuple(sl_c)]
        for dim, axis in enumerate((2, 1, 0)):
            own = fld == axis
            xc = np.asarray(fc[axis] if own else cc[axis])
            xf = np.asarray(ff[axis] if own else cf[axis])
            a = _interp_axis(a, dim, xc, xf)
        out[fld][tuple(sl_f)] = a
    return out


def prolong_base(ctx_coarse, base_coarse, ctx_fine):
    """A steady state of ctx_coarse as the start of the Newton iteration on
    the finer grid of ctx_fine: interpolated to the fine nodes, velocity
    projected onto the divergence-free no-slip subspace by the library (one
    SIMPLE pass), temperature wall nodes reset to the boundary values of
    eqs (4)-(7).  Returns a fine-grid CUDA tensor."""
    import torch
    from . import inputs
    fc, cc, _ = ctx_coarse.coords()
    ff, cf, _ = ctx_fine.coords()
    U = prolong_fields(base_coarse.cpu().numpy(), fc, cc, ff, cf)
    U[3] = inputs._theta_walls(U[3], np.asarray(cf[0]), ctx_fine.span_bc)
    Ud = torch.as_tensor(U).cuda()
    P = ctx_fine.project(Ud)
    Ud[:3] = P[:3]
    return Ud


def steady_state_refined(ctx, n_coarse, Gr, log=None, newton_opts=None, coarse_opts=None):
    """Newton steady state at Gr on ctx's grid, started from the steady state
    of the same problem on coarser grids: continuation in Gr on the coarsest
    (n_coarse: cells per axis, or a list of them from the coarsest up), then
    on each finer grid the state of the one below interpolated by
    ``prolong_base`` and a Newton iteration (coarse_opts there, newton_opts on
    ctx's grid): each grid needs only the last Newton iterations.  Returns
    (base, report of the fine Newton iteration, coarse stages)."""
    import torch
    from . import Ctx, inputs
    levels = [int(n_coarse)] if np.isscalar(n_coarse) else [int(v) for v in n_coarse]

    def make(n):
        return Ctx(n, grid=ctx.grid_kind, s=ctx.s, span_bc=ctx.span_bc, Gr=Gr, Pr=ctx.Pr,
                   device=ctx.device)

    cctx = make(levels[0])
    _, c, _ = cctx.coords()
    Uc = torch.as_tensor(inputs.conduction_state(c, ctx.span_bc)).cuda()
    stages = steady_state(cctx, Uc, Gr, newton_opts=coarse_opts, log=log)
    opts = dict(tol=1e-10, gmres_m=100, lin_tol=1e-10, max_newton=10)
    for n in levels[1:]:
        mctx = make(n)
        Um = prolong_base(cctx, Uc, mctx)
        del Uc
        cctx.close()
        mid = dict(opts)
        mid.update(coarse_opts or {})
        rep = mctx.newton_step(Um, **mid)
        stages.append((Gr, rep))
        if log:
            log(f"refined Newton on {mctx.n}: status {rep['status']} its {rep['newton_its']} "
                f"res {rep['res_before']:.2e} -> {rep['res_after']:.2e}")
        cctx, Uc = mctx, Um
    U = prolong_base(cctx, Uc, ctx)
    del Uc
    cctx.close()
    ctx.set_params(Gr)
    opts.update(newton_opts or {})
    rep = ctx.newton_step(U, **opts)
    if log:
        log(f"refined Newton on {ctx.n}: status {rep['status']} its {rep['newton_its']} "
            f"res {rep['res_before']:.2e} -> {rep['res_after']:.2e}")
    return U, rep, stages


def base_flow_sensitivity(ctx, base, lin_opts=None):
    """U' = dU/dGr at a steady state: A U' = -P dF/dGr, where dF/dGr is the
    residual's explicit Gr dependence (nu' Lap U, kappa' Lap Theta)."""
    Gr, Pr = ctx.Gr, ctx.Pr
    dnu = -0.5 * Gr ** -1.5
    try:
        ctx.set_coeffs(dnu, dnu / Pr, 0.0)
        F1 = ctx.fv_residual(base)
        ctx.set_coeffs(0.0, 0.0, 0.0)
        F0 = ctx.fv_residual(base)
    finally:
        ctx.set_params(Gr, Pr)
    ctx.axpby(F1, -1.0, F0, 1.0)              # dF/dGr
    rhs = ctx.project(F1)
    ctx.axpby(rhs, 0.0, rhs, -1.0)            # -P dF/dGr
    opts = dict(lin_tol=1e-10, gmres_m=100)
    opts.update(lin_opts or {})
    Up, rep = ctx.linear_solve(base, rhs, **opts)
    return Up, rep


def total_dlam_dGr(ctx, base, x, y, Up):
    """d lambda / d Gr along the branch of steady states:
    y^H [ dA/dGr x + (dA/dU . U') x ] / (y^H x), with
    (dA/dU . U') x = A(U') x - A(0) x (J is affine in the base flow)."""
    import torch
    parts = []
    zero = ctx.zeros()
    for comp in (x.real, x.imag):
        c = comp.contiguous().reshape(ctx.shape4)
        d1 = dA_dGr_apply(ctx, c)
        a1 = ctx.simple_krylov_vec(Up, c)
        a0 = ctx.simple_krylov_vec(zero, c)
        ctx.axpby(d1, 1.0, a1, 1.0)
        ctx.axpby(d1, -1.0, a0, 1.0)
        parts.append(d1.reshape(-1))
    dAx = torch.complex(parts[0], parts[1])
    return _cdot(ctx, y.reshape(-1), dAx) / _cdot(ctx, y.reshape(-1), x.reshape(-1))


def leading_index(lams):
    """Index of the leading eigenvalue: the largest real part, and of a
    complex-conjugate pair the member with Im >= 0."""
    lams = np.asarray(lams)
    return int(sorted(range(len(lams)), key=lambda q: (-round(lams[q].real, 12),
                                                        -lams[q].imag))[0])


def gr_slope(dl, Gr, lam, last):
    """d Re(lambda) / d Gr for the Newton step on Gr: the adjoint estimate
    Re(dl), unless the previous iterate ``last`` = (Gr, lambda) led with the
    same mode (|lambda - lambda_last| < 2% of |lambda|) and the secant slope
    through it differs in sign or by more than a factor of 3; then the
    secant.  Returns (slope, "adjoint" | "secant")."""
    slope = float(np.real(dl))
    if last is not None and abs(lam - last[1]) < 0.02 * abs(lam) and Gr != last[0]:
        sec = (lam.real - last[1].real) / (Gr - last[0])
        if sec * slope <= 0 or not (1 / 3 < slope / sec < 3):
            return sec, "secant"
    return slope, "adjoint"


def critical_gr(ctx, base, Gr0, v0, seed, k=8, m=60, tol=1e-10, gr_rtol=1e-7, max_it=12,
                log=None, terms=None, chebyshev=0, max_restarts=400, newton_opts=None):
    """Newton iteration on Gr for Re lambda_lead(Gr) = 0 (the paper's critical
    Grashof number).  ``base`` (in/out) must be a steady state at Gr0.  Each
    iteration: Newton steady state at the current Gr (from the previous one),
    the k rightmost eigenvalues (Krylov-Schur on A), the leading one (largest
    real part, Im >= 0 of a pair) with its left eigenvector (Krylov-Schur on
    A^T), U', and Gr <- Gr - Re lambda / Re(d lambda / d Gr).  Returns a
    history list (each entry also lists the k eigenvalues found).

    k must hold every pair near the crossing: with fewer, the solve can
    return a set that misses the rightmost one.  When two successive
    iterates lead with the same mode, the secant slope of Re lambda checks
    the adjoint derivative; if they differ in sign or by more than a factor
    of 3, the step uses the secant (the adjoint estimate divides by y^H x,
    which is small for the strongly non-normal operators near the onset).

    terms: coupling terms kept in the eigenvalue problem (fvk TERM_* mask, the
    mechanism experiment of Sec. 4.2); the steady states and U' always use
    the full equations.  chebyshev: degree of the Chebyshev-accelerated
    eigenvalue solves (0: plain Krylov-Schur); newton_opts: options of the
    steady-state Newton iterations.

    The eigenvalue solves run on the shifted operator A + sigma P
    (krylov_schur's default), so a real eigenvalue crossing zero stays clear
    of the complement of the constraint subspace (eigenvalue 0 of the stored-
    array operator, at -sigma relative to the physical spectrum)."""
    from . import TERMS_ALL
    full = TERMS_ALL
    terms = full if terms is None else terms
    hist = []
    Gr = Gr0
    prev = Gr0
    last = None          # (Gr, lambda) of the previous iterate
    try:
        for it in range(max_it):
            ctx.set_terms(full)
            if it > 0:
                # from the steady state at the previous Gr, in steps of at most 1.5x
                steady_state(ctx, base, Gr, Gr_start=prev, factor=1.5, log=log,
                             newton_opts=newton_opts)
                prev = Gr
            ctx.set_params(Gr)
            Up, _ = base_flow_sensitivity(ctx, base)
            ctx.set_terms(terms)
            if chebyshev > 0:
                r = krylov_schur_chebyshev(ctx, base, k, m, v0, degree=chebyshev, tol=tol,
                                           max_restarts=max_restarts)
            else:
                r = krylov_schur(ctx, base, k, m, v0, tol=tol, max_restarts=max_restarts)
            lead = leading_index(r.lam)
            lam, x = r.lam[lead], r.X[lead]
            rT, ys = left_eigvecs(ctx, base, [lam], k, m, seed, tol=tol,
                                  max_restarts=max_restarts)
            dl = total_dlam_dGr(ctx, base, x, ys[0], Up)
            slope, how = gr_slope(dl, Gr, lam, last)
            # the transposed solve sees the same spectrum: a pair it finds to
            # the right of the leading one was missed by the forward solve
            missed = [complex(np.conj(v)) for v in rT.lam
                      if v.real > lam.real + 1e-3 * abs(lam) and v.imag <= 0]
            hist.append({"Gr": Gr, "lam": lam, "dlam_dGr": dl, "slope": slope, "step_from": how,
                         "nvec": r.nvec, "eigenvalues": [complex(v) for v in r.lam],
                         "transposed_eigenvalues": [complex(np.conj(v)) for v in rT.lam],
                         "missed_by_forward_solve": missed})
            if missed and log:
                log(f"critical Gr it {it}: the transposed solve found {np.round(missed, 5)} to "
                    f"the right of the leading {lam:.5g}")
            if log:
                log(f"critical Gr it {it}: Gr {Gr:.8g} lambda {lam:.6g} dlam/dGr {dl:.4g} "
                    f"({how} slope {slope:.4g}); found {np.round(r.lam, 5)}")
            last = (Gr, lam)
            # the Newton step on Gr, kept within a factor of 2 of the current
            # Gr (far from the crossing the linear model can point below 0)
            step = -lam.real / slope
            step = min(max(step, -0.5 * Gr), Gr)
            Gr = Gr + step
            if abs(step) < gr_rtol * abs(Gr):
                hist.append({"Gr": Gr, "converged": True})
                break
    finally:
        ctx.set_terms(full)
    return hist
