"""Rightmost eigenvalues of the Krylov operator A (or A^T) by Krylov-Schur
restarted Arnoldi (Stewart, SIAM J. Matrix Anal. Appl. 23, 2001).

The paper computes the leading eigenpairs of eq. (10) with ARPACK / HSL EB13
in the "single run" mode that the SIMPLE-based Krylov vectors allow (Sec. 3.1);
this driver plays that role.  Each Arnoldi step is the library's arnoldi_step
(Krylov vector + CGS2 orthogonalisation in HIP kernels); restarts rotate the
device-resident basis with fvk_basis_rotate.  Only the small (m x m)
Rayleigh quotient is handled on the host (real Schur form, scipy).

Convergence: a Ritz pair (theta, V x) is accepted when the residual
|| A V x - theta V x || / || V x || = |b^T x| is below ``tol`` (the paper
monitors || J X - lambda X || / || X || < 1e-10 after convergence).

The complement of the constraint subspace: eq. (10) is posed on the subspace
S of divergence-free velocities and temperatures satisfying the homogeneous
boundary conditions; A = P J acts on whole stored arrays and maps them into
S, so it also has the eigenvalue 0 with the multiplicity of the complement
ker P.  A start vector in S keeps the Krylov space in S only up to rounding,
and at a stable steady state (every eigenvalue of eq. (10) left of 0) the
restarts would amplify those rounding components until the cluster at 0
looks rightmost.  The iteration therefore runs on the shifted operator
A + sigma P (fvk_set_shift; the stencils add sigma times the centre value,
at no extra memory traffic), whose Krylov spaces, Ritz vectors and residuals
are those of A - sigma (I - P): the spectrum of eq. (10) moved right by sigma
while ker P stays at 0, i.e. the complement sits sigma to the left of the
physical spectrum.  The reported eigenvalues are the Ritz values minus sigma.
The shift should separate the complement from the wanted (rightmost) part of
the spectrum, and no more: each Krylov vector passes (J + sigma I) x through
the projection P, whose rounding (relative ~1e-13 at 256^3) then enters the
Krylov relation at the scale sigma || x ||, while the physical residual
|| A x - lambda x || of a smooth eigenvector is much smaller -- with sigma =
|| A || ~ 1e4 at 256^3 this put a floor of ~2e-9 under the residuals.  The
default is sigma = min(100, spectral radius of A) (estimated from a short
unshifted Arnoldi run, at least 1): 100 is far to the left of the
eigenvalues the stability problem asks for (|Re lambda| < 1 here).
"""
import numpy as np
import scipy.linalg as sla


def _order(lam):
    """Indices by decreasing real part (rounded to 1e-9 of the spectral
    radius, so conjugate pairs tie), then decreasing imaginary part."""
    lam = np.asarray(lam)
    scale = max(float(np.max(np.abs(lam))), 1e-300) if lam.size else 1.0
    re = np.round(lam.real / (1e-9 * scale))
    return np.lexsort((-lam.imag, -re))


class EigResult:
    def __init__(self, lam, X, res, restarts, nvec, converged, shift=0.0):
        self.lam, self.X, self.res = lam, X, res
        self.restarts, self.nvec, self.converged = restarts, nvec, converged
        self.shift = shift


def _arnoldi_cycle(ctx, base, V, H, p, m, transpose, lagged):
    """Arnoldi steps p .. m-1 on the current operator (V, H in place)."""
    for j in range(p, m):
        if lagged:
            ctx.arnoldi_step_lagged(base, V, j, H, transpose=transpose)
        else:
            h, brk = ctx.arnoldi_step(base, V, j, transpose=transpose)
            H[:j + 2, j] = h
            if brk:
                raise RuntimeError("Arnoldi breakdown (invariant subspace)")
    if lagged:
        ctx.arnoldi_finish(V, m, H)


def spectral_radius(ctx, base, v0, steps=20, transpose=False, V=None):
    """max |theta| over the Ritz values of ``steps`` Arnoldi steps on the
    unshifted A (A^T) from v0: the extreme eigenvalues of the stiff
    diffusion part converge first, so this approximates || A ||'s spectral
    radius from below.  V: optional (>= steps + 1, N) work tensor."""
    import torch
    steps = int(steps)
    if V is None:
        V = torch.zeros((steps + 1, ctx.N), dtype=torch.float64, device=ctx.device)
    saved = ctx.shift
    ctx.set_shift(0.0)
    try:
        V[0] = v0.reshape(-1)
        ctx.normalize(V[0])
        H = np.zeros((steps + 1, steps))
        _arnoldi_cycle(ctx, base, V, H, 0, steps, transpose, True)
    finally:
        ctx.set_shift(saved)
    theta = np.linalg.eigvals(H[:steps, :steps])
    return float(np.max(np.abs(theta))) if theta.size else 0.0


def krylov_schur(ctx, base, k, m, v0, tol=1e-10, max_restarts=200, transpose=False,
                 vectors=True, log=None, lagged=True, keep=None, shift="auto"):
    """k rightmost eigenvalues (largest real part) of A (transpose: A^T) on the
    constraint subspace.

    shift: sigma of the shifted operator A + sigma P (see the module notes);
    "auto" (default) takes min(100, the spectral radius estimated by 20
    unshifted Arnoldi steps from v0), at least 1; 0 runs on A itself.
    lagged: Arnoldi steps with the re-orthogonalisation lagged by one step
    (arnoldi_step_lagged, two passes over the basis per step, completed by
    arnoldi_finish at the end of each cycle); False: arnoldi_step (CGS2, four
    passes).

    v0: (N,) or ctx.shape4 float64 CUDA tensor (start vector; for A it should
    lie in the constraint subspace, e.g. the output of ctx.project).
    keep: Ritz values kept at a restart (default (m + k) // 2, at least k + 2).
    Fewer make each step of the next cycle cheaper (a shorter basis to
    orthogonalise against): at 100^3 with k = 4, m = 100, 12-24 kept took
    4.3-4.4 s against 5.6 s with 52, for the same eigenvalues.  But a small
    keep can also lose a wanted eigenvalue: at 20^3 with k = 6, m = 40, 11 kept
    converged to the wrong set, hence the conservative default.
    Returns EigResult with lam sorted by (-Re, -Im) and the shift used; X (if
    vectors) is a (kk, N) complex128 CUDA tensor of unit Ritz vectors."""
    import torch
    if not (0 < k < m):
        raise ValueError("need 0 < k < m")
    N = ctx.N
    V = torch.zeros((m + 1, N), dtype=torch.float64, device=ctx.device)
    if shift == "auto":
        ns = min(20, m)
        sigma = max(1.0, min(100.0, spectral_radius(ctx, base, v0, ns, transpose, V[:ns + 1])))
    else:
        sigma = float(shift)
    saved = ctx.shift
    ctx.set_shift(sigma)
    try:
        return _krylov_schur(ctx, base, k, m, v0, V, sigma, tol, max_restarts, transpose,
                             vectors, log, lagged, keep)
    finally:
        ctx.set_shift(saved)


def _krylov_schur(ctx, base, k, m, v0, V, sigma, tol, max_restarts, transpose, vectors, log,
                  lagged, keep):
    import torch
    V[0] = v0.reshape(-1)
    ctx.normalize(V[0])
    H = np.zeros((m + 1, m))
    p = 0
    nvec = 0
    lam = res = None
    kept = min(m - 1, max(k + 2, (m + k) // 2 if keep is None else int(keep)))
    for restart in range(max_restarts + 1):
        _arnoldi_cycle(ctx, base, V, H, p, m, transpose, lagged)
        nvec += m - p
        Hm = H[:m, :m]
        b = H[m, :m].copy()
        # residuals of the Ritz pairs: |b^T x| for unit eigenvectors x
        w, Xh = np.linalg.eig(Hm)
        o2 = _order(w)
        w, Xh = w[o2], Xh[:, o2]
        Xh = Xh / np.linalg.norm(Xh, axis=0, keepdims=True)
        res = np.abs(b @ Xh)
        lam = w
        nconv = int(np.sum(res[:k] < tol))
        if log:
            log(f"restart {restart}: nvec {nvec}, lead {w[0] - sigma:.10g}, "
                f"res {res[:k].max():.2e}")
        if nconv >= k or restart == max_restarts:
            break
        # Krylov-Schur truncation: keep the `kept` rightmost Ritz values
        thr = w[kept - 1].real
        scale = 1e-12 * max(1.0, np.abs(w).max())
        S, Q, sdim = sla.schur(Hm, output='real', sort=lambda re, im: re >= thr - scale)
        p = int(sdim)
        if p >= m or p == 0:
            p = kept
        ctx.basis_rotate(V, Q[:, :p])
        V[p] = V[m]
        H[:] = 0.0
        H[:p, :p] = S[:p, :p]
        H[p, :p] = b @ Q[:, :p]
    converged = bool(np.all(res[:k] < tol))
    kk = k
    # keep both members of a conjugate pair cut at position k
    if kk < len(lam) and lam[kk - 1].imag != 0 and abs(lam[kk] - np.conj(lam[kk - 1])) <= \
            1e-8 * abs(lam[kk - 1]):
        kk += 1
    X = None
    if vectors:
        if 2 * kk > m:
            raise ValueError("need 2 * (number of Ritz vectors) <= m")
        # real and imaginary parts in one in-place rotation of the basis
        M = np.concatenate([Xh[:, :kk].real, Xh[:, :kk].imag], axis=1)
        ctx.basis_rotate(V, M)
        X = torch.complex(V[:kk].clone(), V[kk:2 * kk].clone())
    out = EigResult(lam[:kk] - sigma, X, res[:kk], restart, nvec, converged, sigma)
    out.ritz_all = np.asarray(lam) - sigma      # every Ritz value of the last cycle
    return out


def ritz_residual(ctx, base, lam, x, transpose=False):
    """|| A x - lam x || / || x || for a complex CUDA vector x (two real
    Krylov-vector applications of the unshifted operator)."""
    import torch
    XX = torch.stack([x.real.reshape(-1), x.imag.reshape(-1)]).contiguous()
    xr, xi = XX[0].reshape(ctx.shape4), XX[1].reshape(ctx.shape4)
    lr, li = float(np.real(lam)), float(np.imag(lam))
    saved = ctx.shift
    ctx.set_shift(0.0)
    try:
        rr = ctx.simple_krylov_vec(base, xr, transpose=transpose)
        ri = ctx.simple_krylov_vec(base, xi, transpose=transpose)
    finally:
        ctx.set_shift(saved)
    ctx.multiaxpy(rr, 1.0, XX, [-lr, li])          # A xr - (lr xr - li xi)
    ctx.multiaxpy(ri, 1.0, XX, [-li, -lr])         # A xi - (lr xi + li xr)
    num = ctx.dot(rr, rr) + ctx.dot(ri, ri)
    den = ctx.dot(xr, xr) + ctx.dot(xi, xi)
    return float(np.sqrt(num / den))


# ---------------------------------------------------------------------------
# Chebyshev acceleration (the polynomial preconditioning of the Arnoldi
# iteration that the paper's eigenvalue solvers use, Sec. 3.1)
#
# Krylov-Schur runs on M = p_d(A_s), p_d the scaled Chebyshev polynomial of an
# ellipse E that encloses the unwanted part of the spectrum of A_s = A + s P:
#     p_d(z) = T_d((z - c) / e) / T_d((g - c) / e),
# centre c and foci c -+ e (e real, or imaginary for an ellipse taller than
# wide), normalised at a real point g to the right of E.  |p_d| is at most
# (a + b)^d / |e|^d ... on E and grows geometrically outside it, so the wanted
# (rightmost) eigenvalues become the dominant ones of M, while each Arnoldi
# step on M costs d Krylov vectors but only one orthogonalisation against the
# basis -- the part of a step that dominates at large grids and Krylov
# dimensions.  E is fitted to the unwanted Ritz values of a short plain
# Krylov-Schur run (Saad, Math. Comp. 42, 1984: Chebyshev acceleration of
# Arnoldi's method); the eigenpairs of A are extracted by a Rayleigh-Ritz step
# with A_s on the invariant subspace that Krylov-Schur on M converges to.
# ---------------------------------------------------------------------------


def _cheb_growth(z, c, e):
    """|w + sqrt(w^2 - 1)| >= 1 for w = (z - c) / e: the geometric growth rate
    of T_d at z."""
    w = (np.asarray(z, dtype=complex) - c) / e
    s_ = np.sqrt(w * w - 1.0)
    return np.maximum(np.abs(w + s_), np.abs(w - s_))


def fit_ellipse(theta, nwant):
    """Ellipse enclosing the unwanted Ritz values theta[nwant:] (theta sorted
    by decreasing real part) that damps them fastest relative to the slowest
    wanted value: a search over the centre c (on the real axis) and the
    aspect ratio r = b / a, each candidate the smallest ellipse of that
    centre and shape containing the unwanted set.  Returns (c, e, a, b, rate)
    with e complex (real or imaginary foci) and rate = the per-degree damping
    factor of the worst-placed wanted value (< 1), or None if no ellipse
    separates the two sets."""
    theta = np.asarray(theta, dtype=complex)
    U, W = theta[nwant:], theta[:nwant]
    lo, hi = float(U.real.min()), float(U.real.max())
    best = None
    for c in np.linspace(lo, hi, 41)[1:-1] if hi > lo else [lo]:
        for r in np.concatenate([np.logspace(-5, -0.05, 40), np.logspace(0.05, 1.5, 15)]):
            a = float(np.max(np.sqrt((U.real - c) ** 2 + (U.imag / r) ** 2)))
            b = r * a
            e = np.sqrt(complex(a * a - b * b))
            if abs(e) == 0.0:
                continue
            edge = (a + b) / abs(e)           # growth rate on E itself
            gw = _cheb_growth(W, c, e)
            if np.any(gw <= edge):
                continue
            rate = float(np.max(edge / gw))
            if best is None or rate < best[4]:
                best = (c, e, a, b, rate)
    return best


def _cheb_coeffs(c, e, g, d):
    """Coefficients (alpha, beta, delta) of the scaled Chebyshev recurrence
    y_{j+1} = alpha (A y_j) + beta y_j + delta y_{j-1}, j = 0 .. d-1 (delta of
    the first step unused): y_d = T_d((A - c)/e) y_0 / T_d((g - c)/e).  With
    imaginary foci the individual sigma_j are imaginary but every coefficient
    is real."""
    s1 = e / (g - c)
    out = [(s1 / e, -s1 * c / e, 0.0)]
    sj = s1
    for _ in range(1, d):
        sn = 1.0 / (2.0 / s1 - sj)
        out.append((2.0 * sn / e, -2.0 * sn * c / e, -sj * sn))
        sj = sn
    return [(float(np.real(a)), float(np.real(b)), float(np.real(dl))) for a, b, dl in out]


class _ChebOp:
    """y = p_d(A_s) x with the library's Krylov vector and three-term
    combination kernel (three work vectors)."""

    def __init__(self, ctx, base, coeffs, transpose):
        import torch
        self.ctx, self.base, self.coeffs, self.tr = ctx, base, coeffs, transpose
        self.W = torch.empty((3, ctx.N), dtype=torch.float64, device=ctx.device)

    def apply(self, x, out):
        ctx, W = self.ctx, self.W
        prev, cur = None, x.reshape(-1)
        for j, (al, be, de) in enumerate(self.coeffs):
            nxt = W[j % 3]
            ctx.simple_krylov_vec(self.base, cur.reshape(ctx.shape4), out=nxt.reshape(ctx.shape4),
                                  transpose=self.tr)
            if prev is None:
                ctx.axpby(nxt, be, cur, al)            # alpha A y_0 + beta y_0
            else:
                ctx.lincomb3(nxt, be, cur, de, prev, al)
            prev, cur = cur, nxt
        ctx.axpby(out.reshape(-1), 1.0, cur, 0.0)


def krylov_schur_chebyshev(ctx, base, k, m, v0, degree=10, tol=1e-10, max_restarts=200,
                           transpose=False, warm_restarts=3, extra=None, log=None,
                           shift="auto", keep=None, refit_every=40):
    """k rightmost eigenvalues of A (A^T) by Krylov-Schur on the Chebyshev
    filter M = p_degree(A + s P) (see the notes above).

    The filter's ellipse is fitted to the unwanted Ritz values of
    ``warm_restarts`` plain Krylov-Schur cycles (Krylov dimension m) from v0;
    the k + extra (default max(2, k // 2)) rightmost Ritz values are the
    wanted set.  The
    filtered iteration starts from the sum of the warm-up Ritz vectors of the
    wanted set and targets the largest |p(theta)|.  When its wanted Ritz
    values converge (relative residual of M below tol_m), and every
    ``refit_every`` restarts in any case, the eigenpairs of A are extracted by
    Rayleigh-Ritz on the dominant invariant subspace of M (one Krylov vector
    per basis vector); it stops when the k rightmost have explicit residuals
    || A x - lam x || / || x || below tol.  Otherwise the extracted values
    outside the wanted set join the unwanted ones and the ellipse is refitted
    (adaptive Chebyshev acceleration): a short warm-up can miss unwanted
    eigenvalues with large imaginary parts near the right end of the
    spectrum, which a too-flat ellipse then amplifies; once seen they are
    enclosed, and the iteration restarts from the current Ritz vectors of the
    wanted set.  If the fit does not change, tol_m is tightened tenfold.  Returns an EigResult (res = the explicit
    residuals; nvec counts every Krylov vector, filter and extraction
    included; .orth_steps the Arnoldi orthogonalisation steps)."""
    import torch
    extra = max(2, k // 2) if extra is None else int(extra)
    nw = k + extra
    if not (0 < k and 2 * (nw + 1) <= m):
        raise ValueError("need 2 (k + extra + 1) <= m (the warm-up Ritz vectors of the wanted "
                         "set, a conjugate pair included, fill at most half the basis)")
    r0 = krylov_schur(ctx, base, nw, m, v0, tol=tol, max_restarts=warm_restarts,
                      transpose=transpose, vectors=True, shift=shift, keep=keep)
    sigma = r0.shift
    nvec = r0.nvec + 20 * (shift == "auto")
    theta = r0.ritz_all + sigma
    fit = fit_ellipse(theta, min(len(r0.lam), nw))
    saved = ctx.shift
    ctx.set_shift(sigma)
    try:
        if fit is None:
            if log:
                log("chebyshev: no separating ellipse; plain Krylov-Schur")
            ctx.set_shift(saved)
            r = krylov_schur(ctx, base, k, m, v0, tol=tol, max_restarts=max_restarts,
                             transpose=transpose, shift=shift, keep=keep)
            r.orth_steps = r.nvec
            r.nvec += nvec
            return r
        c, e, a, b, rate = fit
        g = float(theta[0].real)
        coeffs = _cheb_coeffs(c, e, g, degree)
        if log:
            log(f"chebyshev: ellipse centre {c - sigma:.6g} semi-axes {a:.4g} x {b:.4g}, "
                f"per-degree damping {rate:.6f}, degree {degree}")
        op = _ChebOp(ctx, base, coeffs, transpose)
        N = ctx.N
        V = torch.zeros((m + 1, N), dtype=torch.float64, device=ctx.device)
        # start: the sum of the real and imaginary parts of the warm-up Ritz
        # vectors of the wanted set
        XR0, XI0 = r0.X.real.contiguous(), r0.X.imag.contiguous()
        V[0].zero_()
        for i in range(XR0.shape[0]):
            ctx.lincomb3(V[0], 1.0, XR0[i], 1.0, XI0[i], 1.0)
        del r0, XR0, XI0
        ctx.normalize(V[0])
        H = np.zeros((m + 1, m))
        p = 0
        kept = min(m - 1, max(nw + 2, (m + nw) // 2 if keep is None else int(keep)))
        tol_m = tol
        orth = 0
        res_a = lam_a = Xa = None
        converged = False
        pool = np.asarray(theta[min(len(theta), nw):])      # unwanted Ritz values seen so far
        best = None                                         # (worst residual, lam, X, res)
        since = 0                                           # restarts since the last (re)start
        for restart in range(max_restarts + 1):
            since += 1
            for j in range(p, m):
                op.apply(V[j], V[j + 1])
                ctx.arnoldi_step_lagged_applied(V, j, H)
                nvec += degree
                orth += 1
            ctx.arnoldi_finish(V, m, H)
            Hm = H[:m, :m]
            bvec = H[m, :m].copy()
            mu, Z = np.linalg.eig(Hm)
            o = np.argsort(-np.abs(mu), kind="stable")
            mu, Z = mu[o], Z[:, o] / np.linalg.norm(Z[:, o], axis=0, keepdims=True)
            res_m = np.abs(bvec @ Z) / np.maximum(np.abs(mu), 1e-300)
            thr_w = np.abs(mu[nw - 1])
            if log and restart % 10 == 0:
                log(f"chebyshev restart {restart}: nvec {nvec}, |mu_1| {abs(mu[0]):.4g}, "
                    f"res_M {res_m[:nw].max():.2e}")
            m_conv = bool(np.all(res_m[:nw] < tol_m))
            if m_conv or restart == max_restarts or since % refit_every == 0:
                # Rayleigh-Ritz with A_s on the wanted invariant subspace of M
                S, Q, sdim = sla.schur(Hm, output="real",
                                       sort=lambda re, im: np.hypot(re, im) >= thr_w * (1 - 1e-12))
                sdim = int(sdim)
                lam_a, Xa, res_a, nmv = _rayleigh_ritz(ctx, base, V, Q[:, :sdim], sigma, m,
                                                      transpose)
                nvec += nmv
                good = len(lam_a) >= k and np.all(res_a[:k] < tol)
                worst = float(res_a[:k].max()) if len(lam_a) >= k else np.inf
                if log:
                    log(f"chebyshev extraction at restart {restart}: {lam_a[:k]} "
                        f"residuals {worst:.2e}")
                if best is None or worst < best[0]:
                    best = (worst, lam_a, Xa, res_a)
                if good or restart == max_restarts:
                    converged = bool(good)
                    if not good:    # the best extraction seen, not the last one
                        _, lam_a, Xa, res_a = best
                    break
                if worst < 1e-3:
                    # converging on the wanted set: keep the filter
                    if m_conv:
                        tol_m = tol_m / 10.0
                    continue_refit = False
                else:
                    continue_refit = True
                # refit the ellipse to every unwanted value seen so far
                th_x = np.asarray(lam_a) + sigma
                if not continue_refit:
                    th_x = th_x[:0]
                pool = np.concatenate([pool, th_x[nw:]])
                allv = np.concatenate([th_x[:nw], pool])
                allv = allv[_order(allv)]
                nfit = fit_ellipse(allv, min(nw, len(th_x))) if continue_refit else None
                if nfit is not None and (abs(nfit[3] - b) > 1e-3 * max(b, 1e-300)
                                         or abs(nfit[0] - c) > 1e-6 * abs(c)):
                    c, e, a, b, rate = nfit
                    op.coeffs = _cheb_coeffs(c, e, float(allv[0].real), degree)
                    if log:
                        log(f"chebyshev refit at restart {restart}: ellipse centre {c - sigma:.6g} "
                            f"semi-axes {a:.4g} x {b:.4g}, per-degree damping {rate:.6f}")
                    # restart from the current Ritz vectors of the wanted set
                    V[0].zero_()
                    XRa, XIa = Xa.real.contiguous(), Xa.imag.contiguous()
                    for i in range(min(nw, XRa.shape[0])):
                        ctx.lincomb3(V[0], 1.0, XRa[i], 1.0, XIa[i], 1.0)
                    del XRa, XIa
                    ctx.normalize(V[0])
                    H[:] = 0.0
                    p = 0
                    since = 0
                    continue
                if m_conv and continue_refit:
                    tol_m = tol_m / 10.0
            # Krylov-Schur truncation on M: keep the largest |mu|
            thr = np.abs(mu[kept - 1])
            S, Q, sdim = sla.schur(Hm, output="real",
                                   sort=lambda re, im: np.hypot(re, im) >= thr * (1 - 1e-12))
            p = int(sdim)
            if p >= m or p == 0:
                p = kept
            ctx.basis_rotate(V, Q[:, :p])
            V[p] = V[m]
            H[:] = 0.0
            H[:p, :p] = S[:p, :p]
            H[p, :p] = bvec @ Q[:, :p]
        kk = k
        if kk < len(lam_a) and lam_a[kk - 1].imag != 0 and \
                abs(lam_a[kk] - np.conj(lam_a[kk - 1])) <= 1e-8 * abs(lam_a[kk - 1]):
            kk += 1
        out = EigResult(lam_a[:kk], Xa[:kk], res_a[:kk], restart, nvec, converged, sigma)
        out.orth_steps = orth
        out.ellipse = {"centre": c - sigma, "a": a, "b": b, "rate": rate, "degree": degree}
        return out
    finally:
        ctx.set_shift(saved)


def _rayleigh_ritz(ctx, base, V, Qs, sigma, m, transpose):
    """Eigenpairs of A from the subspace V[:m] Qs (orthonormal columns): the
    basis B = V Qs, C = A_s B (one Krylov vector per column), the Rayleigh
    quotient G = B^T C, its eigenpairs (theta, y), x = B y and the explicit
    residuals || C y - theta B y || / || B y || (no further Krylov vectors),
    all vector work in library kernels.  Returns (lam = theta - sigma sorted
    by (-Re, -Im), unit X (complex rows), residuals, Krylov vectors used)."""
    import torch
    q = Qs.shape[1]
    # B = V[:m] Qs in its own buffer (one pass over the basis per column): the
    # basis itself must stay intact for the iteration to continue
    Bm = torch.zeros((q, V.shape[1]), dtype=V.dtype, device=V.device)
    for i in range(q):
        ctx.multiaxpy(Bm[i], 0.0, V[:m], np.ascontiguousarray(Qs[:, i]))
    C = torch.empty_like(Bm)
    for i in range(q):
        ctx.simple_krylov_vec(base, Bm[i].reshape(ctx.shape4), out=C[i].reshape(ctx.shape4),
                              transpose=transpose)
    G = np.stack([ctx.multidot(Bm, q, C[j]) for j in range(q)], axis=1)   # G[i, j] = B_i . C_j
    th, Y = np.linalg.eig(G)
    lam = th - sigma
    o = _order(lam)
    lam, th, Y = lam[o], th[o], Y[:, o]
    XR, XI, CR, CI = Bm.clone(), Bm, C.clone(), C
    ctx.basis_rotate(XR, np.ascontiguousarray(Y.real))
    ctx.basis_rotate(XI, np.ascontiguousarray(Y.imag))
    ctx.basis_rotate(CR, np.ascontiguousarray(Y.real))
    ctx.basis_rotate(CI, np.ascontiguousarray(Y.imag))
    res = np.zeros(q)
    for i in range(q):
        tr, ti = float(th[i].real), float(th[i].imag)
        ctx.lincomb3(CR[i], -tr, XR[i], ti, XI[i], 1.0)      # Re (C y - theta B y)
        ctx.lincomb3(CI[i], -tr, XI[i], -ti, XR[i], 1.0)     # Im (C y - theta B y)
        nx2 = ctx.dot(XR[i], XR[i]) + ctx.dot(XI[i], XI[i])
        res[i] = np.sqrt((ctx.dot(CR[i], CR[i]) + ctx.dot(CI[i], CI[i])) / nx2)
        ctx.axpby(XR[i], 1.0 / np.sqrt(nx2), XR[i], 0.0)
        ctx.axpby(XI[i], 1.0 / np.sqrt(nx2), XI[i], 0.0)
    return lam, torch.complex(XR, XI), res, q
