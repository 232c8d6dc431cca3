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
By default sigma is the spectral radius of A estimated from a short
unshifted Arnoldi run, which puts the complement at the left edge of the
spectrum, far from the rightmost eigenvalues, and costs at most a digit of
the eigenvalues' absolute accuracy relative to || A ||.
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
    "auto" (default) takes the spectral radius estimated by 20 unshifted
    Arnoldi steps from v0 (at least 1); 0 runs on A itself.
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
        sigma = max(1.0, spectral_radius(ctx, base, v0, ns, transpose, V[:ns + 1]))
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
    return EigResult(lam[:kk] - sigma, X, res[:kk], restart, nvec, converged, sigma)


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
